"""Full-size parity in the launch configurations the benchmark times.

Each test runs a workload at its real size, in the shape `bench.py` uses (pinned to the
shape the profiles were taken on, or autotuned exactly as the benchmark autotunes), and
holds the result to the FP64 oracle: the objective within 1e-5 relative, and the iterate
itself within ITER_TOL(T, L) -- a stated bound on eps_r = ||c - c_fp64|| / ||c_fp64||.

ITER_TOL: every iteration applies the Gram through transforms whose relative rounding
error is about u log2 L (u = 2^-24, FP32); the soft threshold is nonexpansive, so along T
iterations those errors add up at most linearly, with a factor 4 left for FISTA's momentum
weights (below 1) re-applying the last two errors.
"""
import numpy as np
import pytest

from oracle import bccb_oracle as O
from oracle import learned_oracle as LO
from paper_2509_13592_amd import scenes as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2509_13592_amd.bccb")

OBJ_TOL = 1e-5
U32 = 2.0 ** -24

# the single-scene launch shape the benchmark's autotuner keeps at 256^2 and the cooperative
# solve's profile was taken on: pruned cooperative form, 32 groups of 512 threads on one die
HEADLINE = {"row_elems": 4, "row_rows_per_block": 1, "col_elems": 4, "col_cols_per_block": 2, "use_graph": 1,
            "spectral_support": 1, "row_spread": 1, "col_spread": 1, "sparse_iterate": 0, "support_columns": 1,
            "prow_elems": 4, "prow_rows_per_block": 2, "pcol_elems": 4, "pcol_cols_per_block": 1,
            "resident_groups": 32, "resident_spread": 8, "resident_block": 512}


def iter_tol(T, L):
    return 4.0 * T * U32 * np.log2(L)


def admm_tol(T, L):
    """ADMM with rho far below Omega: while z stays at zero the scaled dual is the running sum
    of the x iterates, so their transform errors add up without damping (no factor 4)."""
    return T * U32 * np.log2(L)


def _np(t):
    return t.detach().cpu().numpy().reshape(-1).astype(np.complex128)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_headline_shape_matches_oracle():
    """The paper-scale scene (16x16 URA, 64 kept, 256^2), 500 iterations of ISTA, FISTA and
    ADMM (rho = 1), in the benchmarked cooperative shape."""
    sc = S.paper_scale_scene(0)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=False)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    cfg = plan.set_config(**HEADLINE)
    assert all(cfg[k] == v for k, v in HEADLINE.items()), cfg
    assert plan.support_columns()[1] == 2, "the pruned cooperative form must run"
    y = B.to_device(sc.y)
    T, L = 500, P.op.L
    for name in ("fista", "ista"):
        g = _np(getattr(plan, name)(y, P.tau, T))
        ref = getattr(P, name)(T)
        Fr = P.objective(ref)
        rel = abs(P.objective(g) - Fr) / Fr
        eps = _rel(g, ref)
        print(f"case headline {name} T={T}: rel F {rel:.2e}, eps_r {eps:.2e} (bound {iter_tol(T, L):.1e})", flush=True)
        assert rel <= OBJ_TOL and eps <= iter_tol(T, L)
    z, x = plan.admm(y, P.tau, 1.0, T, want_c=True)
    zr, xr = P.admm(1.0, T)
    z, x = _np(z), _np(x)
    Fr = P.objective(zr)
    rel = abs(P.objective(z) - Fr) / Fr
    ez, ex = _rel(z, zr), _rel(x, xr)
    print(f"case headline admm T={T}: rel F {rel:.2e}, z eps_r {ez:.2e}, x eps_r {ex:.2e} "
          f"(bound {admm_tol(T, L):.1e})", flush=True)
    assert rel <= OBJ_TOL and ez <= admm_tol(T, L) and ex <= admm_tol(T, L)
    plan.close()


def test_large_admm_benchmarked_shape():
    """The 1024^2 scene (32x32 URA, 256 kept), ADMM rho = 0.5, 300 iterations, after the same
    autotune the benchmark runs (oracle: the Woodbury branch of the shifted inverse)."""
    sc = S.large_admm_scene(0)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=False)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    cfg = plan.autotune(reps=20)
    print(f"case 1024^2 ADMM tuned shape {cfg}, support-column mode {plan.support_columns()}", flush=True)
    y = B.to_device(sc.y)
    T, rho = 300, 0.5
    z, x = plan.admm(y, P.tau, rho, T, want_c=True)
    zr, xr = P.admm(rho, T)
    z, x = _np(z), _np(x)
    Fr = P.objective(zr)
    rel = abs(P.objective(z) - Fr) / Fr
    ez, ex = _rel(z, zr), _rel(x, xr)
    print(f"  rel F {rel:.2e}, z eps_r {ez:.2e}, x eps_r {ex:.2e} (bound {admm_tol(T, P.op.L):.1e})", flush=True)
    assert rel <= OBJ_TOL and ex <= admm_tol(T, P.op.L)
    if np.linalg.norm(zr) > 0:
        assert ez <= admm_tol(T, P.op.L)
    plan.close()


def test_uneven_workload_stratified_sample():
    """All 4096 scenes of the uneven workload (FISTA 300, autotuned as benchmarked); 66 scenes,
    11 from each (grid size, array size) stratum, against the oracle one by one."""
    n = 4096
    scenes = [S.batched_scene(i) for i in range(n)]
    plans = [B.Plan(sc.mask, sc.L1, sc.L2) for sc in scenes]
    ys = [B.to_device(sc.y) for sc in scenes]
    taus = [float(np.float32(0.1 * p.adjoint_maxabs(y))) for p, y in zip(plans, ys)]
    batch = B.Batch(plans)
    batch.autotune(reps=3)
    print("classes", batch.classes(), batch.class_configs(), flush=True)
    T = 300
    outs = batch.fista(ys, taus, T)
    strata = {}
    for i, sc in enumerate(scenes):
        key = (sc.L1, sc.mask.shape[1])
        if len(strata.setdefault(key, [])) < 11:
            strata[key].append(i)
    assert len(strata) == 6, sorted(strata)
    worst = (0.0, 0.0)
    for key, idx in sorted(strata.items()):
        for i in idx:
            sc = scenes[i]
            P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, tau=taus[i], dense=False)
            ref = P.fista(T)
            g = _np(outs[i])
            Fr = P.objective(ref)
            rel = abs(P.objective(g) - Fr) / Fr
            eps = _rel(g, ref)
            worst = (max(worst[0], rel), max(worst[1], eps / iter_tol(T, P.op.L)))
            print(f"case stratum L={key[0]} array {key[1]}: scene {i} rel F {rel:.2e} eps_r {eps:.2e}", flush=True)
            assert rel <= OBJ_TOL and eps <= iter_tol(T, P.op.L), (i, rel, eps)
    print(f"worst rel F {worst[0]:.2e}, worst eps_r / bound {worst[1]:.2f}", flush=True)
    batch.close()
    for p in plans:
        p.close()


def test_learned_backward_paper_scale():
    """lista_backward at the geometry training runs (256^2, the fixed 64-element mask), K = 4
    layers, 3 scenes, against the oracle's hand-derived backward; each parameter group (steps,
    thresholds, 5x5 taps) is held to 1e-3 of its own largest gradient."""
    mask = S.learned_fixed_mask()
    L1 = L2 = 256
    K = 4
    scenes = [S.learned_scene(0, 900 + i, mask) for i in range(3)]
    op = O.Operator(mask, L1, L2)
    Om = O.bccb_eigenvalues(mask, L1, L2)
    mu0 = O.step_size(op)
    bs, taus, labels = [], [], []
    for sc in scenes:
        b = op.adjoint(sc.y.astype(np.complex64).astype(np.complex128))
        bs.append(b.reshape(L2, L1))
        tau = float(np.float32(0.1 * np.abs(b).max()))
        taus.append(tau)
        P = O.Problem(mask, L1, L2, sc.y, tau=tau, dense=False)
        labels.append(P.fista(60).reshape(L2, L1).astype(np.complex64).astype(np.complex128))
    rng = np.random.default_rng(8)
    p = LO.init_params(K)
    p[:, 0] += 0.1 * rng.standard_normal(K)
    p[:, 1] += 0.1 * rng.standard_normal(K)
    p[:, 2:] = 0.02 * rng.standard_normal((K, 50))
    loss_ref, g_ref = LO.loss_and_grad(Om, mu0, p, bs, taus, labels)
    plan = B.Plan(mask, L1, L2)
    net = B.Lista(plan, layers=K, max_batch=3, train=True)
    pt = torch.tensor(p, dtype=torch.float32, device="cuda")
    net.forward(pt, B.to_device(np.stack([sc.y for sc in scenes])), taus)
    g, loss = net.backward(pt, B.to_device(np.stack(labels).astype(np.complex64)))
    g = g.cpu().numpy().astype(np.float64)
    print(f"case lista backward 256^2 K={K}: loss {loss:.6e} vs {loss_ref:.6e}", flush=True)
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    for name, cols in (("steps", slice(0, 1)), ("thresholds", slice(1, 2)), ("taps", slice(2, None))):
        err = np.abs(g[:, cols] - g_ref[:, cols]).max() / np.abs(g_ref[:, cols]).max()
        print(f"  {name}: max err / max grad = {err:.2e} (largest {np.abs(g_ref[:, cols]).max():.3e})", flush=True)
        assert err <= 1e-3, (name, err)
    net.close()
    plan.close()


def test_uniform_batch_persistent_sampled():
    """The uniform batch the benchmark times: 1024 paper-scale 256^2 scenes, FISTA 100, as one
    persistent launch (1024-thread workgroups); a sample of scenes against the oracle one by
    one, objective and iterate."""
    n, T = 1024, 100
    scenes = [S.paper_scale_scene(i) for i in range(n)]
    plans = [B.Plan(sc.mask, sc.L1, sc.L2) for sc in scenes]
    ys = [B.to_device(sc.y) for sc in scenes]
    taus = [float(np.float32(0.1 * p.adjoint_maxabs(y))) for p, y in zip(plans, ys)]
    batch = B.Batch(plans)
    info = batch.resident_info()
    print("persistent launch", info, flush=True)
    assert info["on"] == 1 and info["threads"] == 1024
    outs = batch.fista(ys, taus, T)
    worst = (0.0, 0.0)
    for i in (0, 1, 255, 511, 700, 1023):
        sc = scenes[i]
        P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, tau=taus[i], dense=False)
        ref = P.fista(T)
        g = _np(outs[i])
        Fr = P.objective(ref)
        rel, eps = abs(P.objective(g) - Fr) / Fr, _rel(g, ref)
        worst = (max(worst[0], rel), max(worst[1], eps / iter_tol(T, P.op.L)))
        print(f"case uniform batch scene {i}: rel F {rel:.2e} eps_r {eps:.2e}", flush=True)
        assert rel <= OBJ_TOL and eps <= iter_tol(T, P.op.L)
    print(f"worst rel F {worst[0]:.2e}, worst eps_r / bound {worst[1]:.2f}", flush=True)
    batch.close()
    for p in plans:
        p.close()

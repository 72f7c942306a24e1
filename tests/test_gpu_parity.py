"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: per Gram product rel <= 1e-4 (L2 norm); solver objectives rel <= 1e-5
against the oracle trajectory at the same iteration count.  Every comparison
also prints the error against FP64 (eps_r = ||c_gpu - c_oracle|| / ||c_oracle||).
"""
import ctypes

import numpy as np
import pytest

from oracle import bccb_oracle as O
from paper_2509_13592_amd import scenes as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2509_13592_amd.bccb")

MATVEC_TOL = 1e-4
OBJ_TOL = 1e-5


def _np(t):
    return t.detach().cpu().numpy().reshape(-1).astype(np.complex128)


def _crandn(seed, n):
    r = np.random.default_rng(seed)
    return (r.standard_normal(n) + 1j * r.standard_normal(n)).astype(np.complex64)


def _fold(mask, L1, L2):
    P = np.zeros((L2, L1))
    for m1, m2 in O.sensors(mask):
        P[m2 % L2, m1 % L1] += 1
    return P


# grids spanning every supported transform length, square and rectangular
GRIDS = [(8, 8), (16, 32), (32, 32), (64, 16), (128, 128), (256, 256), (512, 64), (1024, 8), (8, 1024),
         (1024, 1024)]


def _geom_scene(L1, L2, seed=0):
    M1 = min(L1, 12)
    M2 = min(L2, 9)
    kept = max(1, (M1 * M2) // 2)
    return S.custom_scene(M1, M2, kept, L1, L2, K=3, snr_db=20, seed=(11, seed, L1 * 7 + L2))


@pytest.mark.parametrize("L1,L2", GRIDS)
def test_plan_eigenvalues(L1, L2):
    sc = _geom_scene(L1, L2)
    print(f"case plan L1={L1} L2={L2}", flush=True)
    plan = B.Plan(sc.mask, L1, L2)
    om = plan.omega().astype(np.float64)
    want = L1 * L2 * _fold(sc.mask, L1, L2)
    assert np.abs(om - want).max() <= 1e-6 * L1 * L2
    assert plan.M == int(sc.mask.sum())
    assert abs(plan.mu * want.max() - 1.0) < 1e-12
    plan.close()


@pytest.mark.parametrize("L1,L2", GRIDS)
def test_gram_apply_matches_oracle(L1, L2):
    sc = _geom_scene(L1, L2)
    print(f"case gram L1={L1} L2={L2}", flush=True)
    op = O.Operator(sc.mask, L1, L2)
    plan = B.Plan(sc.mask, L1, L2)
    for seed in (0, 1):
        x = _crandn(seed, L1 * L2)
        gx = _np(plan.gram_apply(B.to_device(x.reshape(L2, L1))))
        ref = op.gram(x.astype(np.complex128))
        rel = np.linalg.norm(gx - ref) / np.linalg.norm(ref)
        print(f"  rel matvec error vs FP64 = {rel:.2e}")
        assert rel <= MATVEC_TOL
    # structured inputs: an impulse (gives the first column r of G) and a single Fourier mode
    e0 = np.zeros(L1 * L2, np.complex64)
    e0[0] = 1
    r = _np(plan.gram_apply(B.to_device(e0.reshape(L2, L1))))
    ref = op.gram(e0.astype(np.complex128))
    assert np.linalg.norm(r - ref) <= MATVEC_TOL * np.linalg.norm(ref)
    plan.close()


@pytest.mark.parametrize("L1,L2", GRIDS)
def test_adjoint_matches_oracle(L1, L2):
    sc = _geom_scene(L1, L2)
    op = O.Operator(sc.mask, L1, L2)
    plan = B.Plan(sc.mask, L1, L2)
    y = B.to_device(sc.y)
    b = _np(plan.adjoint(y))
    ref = op.adjoint(sc.y.astype(np.complex128))
    assert np.linalg.norm(b - ref) <= 1e-5 * np.linalg.norm(ref)
    assert abs(plan.adjoint_maxabs(y) - np.abs(ref).max()) <= 1e-5 * np.abs(ref).max()
    plan.close()


def _solver_parity(sc, iters, rho=1.0, solvers=("ista", "fista", "admm"), dense=None):
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=dense)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    y = B.to_device(sc.y)
    out = {}
    for name in solvers:
        print(f"case {name} L1={sc.L1} L2={sc.L2} iters={iters}", flush=True)
        if name == "ista":
            g = _np(plan.ista(y, P.tau, iters))
            ref = P.ista(iters)
        elif name == "fista":
            g = _np(plan.fista(y, P.tau, iters))
            ref = P.fista(iters)
        else:
            zg, cg_ = plan.admm(y, P.tau, rho, iters, want_c=True)
            g = _np(zg)
            ref, cref = P.admm(rho, iters)
            # with rho << L the sparse iterate z can stay exactly 0 for many iterations,
            # so the c iterate of eq. (13) is compared as well
            cgn = _np(cg_)
            rc = np.linalg.norm(cgn - cref) / np.linalg.norm(cref)
            print(f"  admm c iterate: eps_r = {rc:.2e}")
            assert rc <= 1e-4
        Fg, Fr = P.objective(g), P.objective(ref)
        rel = abs(Fg - Fr) / abs(Fr)
        nref = np.linalg.norm(ref)
        eps = np.linalg.norm(g - ref) / nref if nref > 0 else np.linalg.norm(g)
        print(f"  {name}: F_gpu={Fg:.9g} F_fp64={Fr:.9g} rel F={rel:.2e} eps_r={eps:.2e}")
        assert rel <= OBJ_TOL, (name, rel)
        out[name] = (g, ref, P)
    plan.close()
    return out


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_tiny_config_solvers(idx):
    """8x8 URA, 32 kept, 32x32 grid, 200 iterations (the tiny workload)."""
    _solver_parity(S.tiny_scene(idx), 200)


def test_ragged_rectangular_solvers():
    sc = S.custom_scene(5, 7, 20, 64, 16, K=3, snr_db=15, seed=(12, 0, 0))
    _solver_parity(sc, 120, rho=4.0)


def test_aliasing_geometry_solvers():
    """M1 > L1: several elements fold onto one bin; eq. (21) still gives the spectrum."""
    sc = S.custom_scene(20, 6, 40, 16, 8, K=2, snr_db=20, seed=(13, 0, 0))
    _solver_parity(sc, 100, rho=64.0)


def test_paper_scale_solvers():
    """16x16 URA, 64 kept, 256x256 grid, 500 iterations of ISTA, FISTA and ADMM (rho = 1)."""
    _solver_parity(S.paper_scale_scene(0), 500, rho=1.0)


def test_large_grid_admm():
    """32x32 URA, 256 kept, 1024x1024 grid, ADMM rho = 0.5, 300 iterations (oracle: Woodbury)."""
    _solver_parity(S.large_admm_scene(0), 300, rho=0.5, solvers=("admm",))


def test_objective_and_kkt_match_oracle():
    sc = S.paper_scale_scene(1)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    y = B.to_device(sc.y)
    c = plan.fista(y, P.tau, 300)
    cn = _np(c)
    obj, r, mx = plan.objective_kkt(y, P.tau, c)
    r_ref, mx_ref = P.kkt(cn)
    F_ref = P.objective(cn)
    print(f"objective {obj:.9g} vs {F_ref:.9g}; r_kkt {r:.4e} vs {r_ref:.4e}; max e/tau {mx:.3e} vs {mx_ref:.3e}")
    assert abs(obj - F_ref) <= 1e-6 * F_ref
    assert abs(r - r_ref) <= 2e-2 * r_ref + 1e-6
    # the same monitors under the call-list name, and Omega copied to device memory
    r2, obj2 = plan.kkt(y, P.tau, c)
    assert r2 == r and obj2 == obj
    assert np.array_equal(plan.omega_device().cpu().numpy(), plan.omega())
    plan.close()


def test_edge_cases():
    sc = S.tiny_scene(3)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    y = B.to_device(sc.y)
    # iters = 0 returns the warm start, or zeros
    c0 = B.to_device(_crandn(5, plan.L).reshape(plan.L2, plan.L1))
    assert torch.equal(plan.fista(y, P.tau, 0, c0=c0), c0)
    assert torch.count_nonzero(plan.ista(y, P.tau, 0)) == 0
    assert torch.count_nonzero(plan.admm(y, P.tau, 1.0, 0)) == 0
    # tau >= max|A^H y| gives exactly zero
    big = 1.01 * plan.adjoint_maxabs(y)
    for c in (plan.ista(y, big, 20), plan.fista(y, big, 20), plan.admm(y, big, 64.0, 20)):
        assert torch.count_nonzero(c) == 0
    # ISTA warm start: 40 + 60 iterations equal 100 (ISTA is memoryless)
    c40 = plan.ista(y, P.tau, 40)
    c100a = _np(plan.ista(y, P.tau, 60, c0=c40))
    c100b = _np(plan.ista(y, P.tau, 100))
    assert np.abs(c100a - c100b).max() <= 1e-5 * np.abs(c100b).max()
    # warm start against the oracle
    c0n = _np(c40)
    ref = P.ista(60, c0=c0n)
    assert abs(P.objective(c100a) - P.objective(ref)) <= OBJ_TOL * P.objective(ref)
    # determinism: same inputs, bitwise equal outputs
    a = plan.fista(y, P.tau, 50)
    b = plan.fista(y, P.tau, 50)
    assert torch.equal(a, b)
    # non-finite snapshot is reported
    ybad = y.clone()
    ybad[3] = complex(float("nan"), 0.0)
    with pytest.raises(B.NonFiniteError):
        plan.fista(ybad, P.tau, 5)
    c0bad = c0.clone()
    c0bad[0, 0] = complex(float("inf"), 0.0)
    with pytest.raises(B.NonFiniteError):
        plan.ista(y, P.tau, 5, c0=c0bad)
    # host-side argument checks
    with pytest.raises(B.BCCBError):
        plan.fista(y, -1.0, 5)
    with pytest.raises(B.BCCBError):
        plan.admm(y, P.tau, 0.0, 5)
    with pytest.raises(B.BCCBError):
        plan.ista(y, P.tau, -3)
    plan.close()


def test_full_ura_one_step_exact():
    """M_i = L_i: G = L I, ISTA reaches the closed-form minimiser S_{tau/L}(b/L) in one step."""
    mask = np.ones((16, 16), np.uint8)
    sc = S.custom_scene(16, 16, 256, 16, 16, K=3, snr_db=20, seed=(14, 0, 0), mask=mask)
    P = O.Problem(mask, 16, 16, sc.y)
    plan = B.Plan(mask, 16, 16)
    y = B.to_device(sc.y)
    c1 = _np(plan.ista(y, P.tau, 1))
    c5 = _np(plan.ista(y, P.tau, 5))
    star = O.soft_threshold(P.b / 256, P.tau / 256)
    assert np.linalg.norm(c1 - star) <= 1e-5 * np.linalg.norm(star)
    assert np.linalg.norm(c5 - star) <= 1e-5 * np.linalg.norm(star)
    plan.close()


CONFIGS_256 = [
    dict(row_elems=4, row_rows_per_block=1, col_elems=4, col_cols_per_block=1, use_graph=1, spectral_support=1,
         row_spread=8, col_spread=8, sparse_iterate=1),
    dict(row_elems=8, row_rows_per_block=2, col_elems=8, col_cols_per_block=4, use_graph=0, spectral_support=0,
         row_spread=1, col_spread=2, sparse_iterate=0),
    dict(row_elems=16, row_rows_per_block=16, col_elems=16, col_cols_per_block=16, use_graph=1, spectral_support=0,
         row_spread=4, col_spread=1, sparse_iterate=1),
    dict(row_elems=32, row_rows_per_block=4, col_elems=32, col_cols_per_block=8, use_graph=0, spectral_support=1,
         row_spread=1, col_spread=1, sparse_iterate=0),
]


def test_results_invariant_to_launch_config():
    """Every launch shape (E, rows/columns per block, graph on/off) gives the oracle's
    trajectory to the same tolerance; the autotuned shape too."""
    sc = S.paper_scale_scene(2)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y)
    ref = P.fista(200)
    Fr = P.objective(ref)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    y = B.to_device(sc.y)
    outs = []
    for cfg in CONFIGS_256 + ["auto"]:
        if cfg == "auto":
            chosen = plan.autotune(reps=10)
            print("autotuned", chosen)
        else:
            plan.set_config(**cfg)
        print("case config", plan.get_config(), flush=True)
        g = _np(plan.fista(y, P.tau, 200))
        g2 = _np(plan.fista(y, P.tau, 200))     # graph replay (or direct) gives the same bits
        assert np.array_equal(g, g2)
        rel = abs(P.objective(g) - Fr) / Fr
        print(f"  rel F = {rel:.2e}  eps_r = {np.linalg.norm(g - ref) / np.linalg.norm(ref):.2e}")
        assert rel <= OBJ_TOL
        outs.append(g)
    for g in outs[1:]:
        assert np.linalg.norm(g - outs[0]) <= 1e-3 * np.linalg.norm(outs[0])
    with pytest.raises(B.BCCBError):
        plan.set_config(row_elems=3)
    with pytest.raises(B.BCCBError):
        plan.set_config(col_elems=4, col_cols_per_block=3)
    with pytest.raises(B.BCCBError):
        plan.set_config(row_spread=3)
    plan.close()


@pytest.mark.parametrize("L1,L2", [(8, 8), (32, 16), (128, 64), (1024, 32)])
def test_small_and_rectangular_configs(L1, L2):
    """The latency (E=4) and packed (largest E) shapes at several rectangular grids."""
    sc = _geom_scene(L1, L2, seed=3)
    op = O.Operator(sc.mask, L1, L2)
    plan = B.Plan(sc.mask, L1, L2)
    x = _crandn(9, L1 * L2)
    ref = op.gram(x.astype(np.complex128))
    for E in (4, 8, 16, 32):
        if E > min(L1, L2) or (min(L1, L2) == 8 and E > 8):
            continue
        try:
            plan.set_config(row_elems=E, row_rows_per_block=1, col_elems=E, col_cols_per_block=1)
        except B.BCCBError:
            continue
        print(f"case gram L1={L1} L2={L2} E={E}", flush=True)
        gx = _np(plan.gram_apply(B.to_device(x.reshape(L2, L1))))
        assert np.linalg.norm(gx - ref) <= MATVEC_TOL * np.linalg.norm(ref)
    plan.close()


@pytest.mark.parametrize("geom", ["tiny", "ragged", "aliasing", "paper"])
def test_sparse_iterate_matches_dense_iterate(geom):
    """FISTA with c^(t) kept in per-row (index, value) slots while rows are sparse follows
    the dense-iterate trajectory: same bits, from zero and from a warm start, at iteration
    counts that end while rows are still dense, while they change form, and after they
    have all turned sparse; ISTA and ADMM are unaffected by the option."""
    sc = {"tiny": S.tiny_scene(6),
          "ragged": S.custom_scene(5, 7, 20, 64, 16, K=3, snr_db=15, seed=(14, 1, 0)),
          "aliasing": S.custom_scene(20, 6, 40, 32, 8, K=2, snr_db=20, seed=(15, 1, 0)),
          "paper": S.paper_scale_scene(5)}[geom]
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=None)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    y = B.to_device(sc.y)
    rng = np.random.default_rng(3)
    warm = (rng.standard_normal((sc.L2, sc.L1)) + 1j * rng.standard_normal((sc.L2, sc.L1))).astype(np.complex64)
    warm[np.abs(warm) < 1.5] = 0
    warm_d = B.to_device(warm)
    plan.set_config(support_columns=0)   # the full passes, where the option applies
    for iters in (0, 1, 2, 7, 60, 300):
        for c0 in (None, warm_d):
            outs = {}
            for spi in (1, 0):
                plan.set_config(sparse_iterate=spi)
                outs[spi] = _np(plan.fista(y, P.tau, iters, c0=c0))
            print(f"case {geom} iters={iters} warm={c0 is not None}: "
                  f"bitwise={np.array_equal(outs[0], outs[1])}", flush=True)
            assert np.array_equal(outs[0], outs[1])
    others = {}
    for spi in (1, 0):
        plan.set_config(sparse_iterate=spi)
        others[spi] = (_np(plan.ista(y, P.tau, 60)), _np(plan.admm(y, P.tau, 4.0, 60)))
    assert all(np.array_equal(a, b) for a, b in zip(others[0], others[1]))
    ref = P.fista(300)
    plan.set_config(sparse_iterate=1)
    g = _np(plan.fista(y, P.tau, 300))
    assert abs(P.objective(g) - P.objective(ref)) / P.objective(ref) <= OBJ_TOL
    plan.close()


@pytest.mark.parametrize("geom", ["tiny", "ragged", "wide", "paper"])
def test_support_columns_path_matches_full_path(geom):
    """The pruned iteration (kept spectral columns only, identity part in the spatial
    domain) and the full passes solve the same problem: both within tolerance of the
    oracle, and of each other, for ISTA and FISTA, cold and warm started, at iteration
    counts from 0 up, and for ADMM at two rho; a plan whose support spans too many
    columns runs the full passes."""
    sc = {"tiny": S.tiny_scene(7),
          "ragged": S.custom_scene(5, 7, 20, 64, 16, K=3, snr_db=15, seed=(17, 1, 0)),
          "wide": S.custom_scene(20, 6, 40, 32, 8, K=2, snr_db=20, seed=(18, 1, 0)),
          "paper": S.paper_scale_scene(6)}[geom]
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=None)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    ncols, pruned = plan.support_columns()
    print(f"case {geom}: support columns {ncols} of {sc.L1}, pruned={pruned}", flush=True)
    assert pruned == ((ncols + 3) // 4 * 4 <= sc.L1 // 2)
    y = B.to_device(sc.y)
    # warm start as a caller would use one: an earlier, rougher solution (20 oracle FISTA
    # iterations), perturbed on its support
    rng = np.random.default_rng(4)
    w = P.fista(20)
    w = w * (1 + 0.1 * rng.standard_normal(w.shape))
    warm = w.reshape(sc.L2, sc.L1).astype(np.complex64)
    for iters in (0, 1, 2, 9, 150):
        for solver in ("ista", "fista"):
            for c0 in (None, warm):
                res = {}
                for sc_on in (1, 0):
                    plan.set_config(support_columns=sc_on)
                    fn = plan.fista if solver == "fista" else plan.ista
                    res[sc_on] = _np(fn(y, P.tau, iters, c0=None if c0 is None else B.to_device(c0)))
                ref = (P.fista if solver == "fista" else P.ista)(iters, c0=None if c0 is None else c0.reshape(-1))
                nr = max(np.linalg.norm(ref), 1e-30)
                diff = np.linalg.norm(res[1] - res[0]) / nr
                print(f"  {solver} iters={iters} warm={c0 is not None}: |pruned - full|/|ref| = {diff:.1e}",
                      flush=True)
                for sc_on in (1, 0):
                    if iters <= 9:   # short runs: the iterates themselves
                        assert np.linalg.norm(res[sc_on] - ref) / nr <= 1e-4
                    else:            # long runs: FP32 trajectories drift apart, the objective does not
                        Fr = P.objective(ref)
                        assert abs(P.objective(res[sc_on]) - Fr) / Fr <= OBJ_TOL
    # ADMM: the pruned passes keep the support part of the scaled dual as spectral
    # coefficients; (z, x) of both paths against FP64 within the bound of a complex64 run
    for rho, iters in ((4.0, 1), (4.0, 2), (4.0, 9), (4.0, 150), (1.0, 150)):
        res = {}
        for sc_on in (1, 0):
            plan.set_config(support_columns=sc_on)
            z, x = plan.admm(y, P.tau, rho, iters, want_c=True)
            res[sc_on] = np.concatenate([_np(z), _np(x)])
        zr, xr = P.admm(rho, iters)
        ref = np.concatenate([zr, xr])
        nr = max(np.linalg.norm(ref), 1e-30)
        errs = {k: np.linalg.norm(v - ref) / nr for k, v in res.items()}
        tol = admm_tol(iters, sc.L1 * sc.L2)
        print(f"  admm rho={rho} iters={iters}: pruned vs FP64 {errs[1]:.1e}, full vs FP64 {errs[0]:.1e} "
              f"(bound {tol:.1e})", flush=True)
        assert errs[1] <= tol and errs[0] <= tol
        Fr = P.objective(zr)
        if Fr > 0 and np.any(zr):
            assert abs(P.objective(res[1][:sc.L1 * sc.L2]) - Fr) / Fr <= OBJ_TOL
    plan.close()


def admm_tol(iters, L):
    """Bound on one complex64 ADMM run's relative error after `iters` iterations: each
    iteration applies (G + rho I)^-1 once through transforms of relative error about
    u log2 L (u = 2^-24), and the scaled dual of eq. (15) is a running sum of the
    x-iterates while z stays at zero, so those errors add up instead of dying out."""
    return iters * 2.0 ** -24 * np.log2(L)


@pytest.mark.parametrize("idx", [0, 3])
def test_pruned_admm_small_rho(idx):
    """ADMM with rho = 1 on the tiny scenes through the pruned passes: with rho far below
    Omega the scaled dual grows to about S / rho on the support modes; the pruned passes
    keep that part as spectral coefficients, so x never comes from cancelling it (the
    form that did -- x as (z - v) plus a support correction -- missed the objective bound
    on the first scene)."""
    sc = S.tiny_scene(idx)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    plan.set_config(support_columns=1)
    assert plan.support_columns()[1] >= 1
    y = B.to_device(sc.y)
    z, x = plan.admm(y, P.tau, 1.0, 200, want_c=True)
    z, x = _np(z), _np(x)
    zr, xr = P.admm(1.0, 200)
    ez = np.linalg.norm(z - zr) / max(np.linalg.norm(zr), 1e-30)
    ex = np.linalg.norm(x - xr) / np.linalg.norm(xr)
    rel = abs(P.objective(z) - P.objective(zr)) / P.objective(zr)
    print(f"case tiny {idx} rho 1: z vs FP64 {ez:.1e}, x vs FP64 {ex:.1e}, rel F {rel:.1e}", flush=True)
    assert ez <= admm_tol(200, P.op.L) and ex <= admm_tol(200, P.op.L) and rel <= OBJ_TOL
    plan.close()


@pytest.mark.parametrize("geom", ["tiny", "ragged", "aliasing", "paper"])
def test_sparse_support_path_matches_dense_path(geom):
    """The spectral-support column pass (Omega and the right-hand side applied on the folded
    bins only) and the dense-grid path solve the same problem: both within tolerance of the
    oracle and of each other, for ISTA, FISTA and ADMM."""
    sc = {"tiny": S.tiny_scene(5),
          "ragged": S.custom_scene(5, 7, 20, 64, 16, K=3, snr_db=15, seed=(12, 1, 0)),
          "aliasing": S.custom_scene(20, 6, 40, 32, 8, K=2, snr_db=20, seed=(13, 1, 0)),
          "paper": S.paper_scale_scene(4)}[geom]
    iters = 150
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=None)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    y = B.to_device(sc.y)
    res = {}
    for sup in (1, 0):
        plan.set_config(spectral_support=sup)
        res[sup] = (_np(plan.ista(y, P.tau, iters)), _np(plan.fista(y, P.tau, iters)),
                    _np(plan.admm(y, P.tau, 4.0, iters)))
    refs = (P.ista(iters), P.fista(iters), P.admm(4.0, iters)[0])
    for k, name in enumerate(("ista", "fista", "admm")):
        Fr = P.objective(refs[k])
        for sup in (1, 0):
            rel = abs(P.objective(res[sup][k]) - Fr) / Fr
            print(f"case support={sup} {geom} {name}: rel F = {rel:.2e}", flush=True)
            assert rel <= OBJ_TOL
        a, b = res[1][k], res[0][k]
        assert np.linalg.norm(a - b) <= 1e-3 * max(np.linalg.norm(b), 1e-30)
    plan.close()


def test_stream_copy():
    """The bandwidth-ceiling copy moves exactly the bytes asked for."""
    src = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    B.stream_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    part = torch.zeros_like(src)
    assert B.lib.bccb_stream_copy(ctypes.c_void_p(B._raw_ptr(src)), ctypes.c_void_p(B._raw_ptr(part)),
                                  ctypes.c_size_t(4096), 13, None) == B.BCCB_OK
    torch.cuda.synchronize()
    assert torch.equal(part[:1024], src[:1024]) and not torch.any(part[1024:])
    # every shape, on a size whose vector count is not a multiple of any stride
    big = torch.randn(5 * (1 << 20) + 12, device="cuda")
    for variant in (0, 1, 2, 3, 4, 5, 6, 7, 8, 19, 31, 37):
        out = torch.zeros_like(big)
        B.stream_copy(big, out, variant)
        torch.cuda.synchronize()
        assert torch.equal(out, big), variant

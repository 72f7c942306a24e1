"""GPU parity of the batched uneven-scene FISTA solver (one graph launch per solve)."""
import numpy as np
import pytest

from oracle import bccb_oracle as O
from paper_2509_13592_amd import scenes as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2509_13592_amd.bccb")

OBJ_TOL = 1e-5


def _np(t):
    return t.detach().cpu().numpy().reshape(-1).astype(np.complex128)


def _setup(scenes):
    plans = [B.Plan(sc.mask, sc.L1, sc.L2) for sc in scenes]
    ys = [B.to_device(sc.y) for sc in scenes]
    taus = [float(np.float32(0.1 * p.adjoint_maxabs(y))) for p, y in zip(plans, ys)]
    return plans, ys, taus


def test_uneven_batch_matches_oracle_and_single_solves():
    # mixed grid sizes, masks, array sizes (drawn like the 4096-scene workload) plus a
    # rectangular and an aliasing scene
    scenes = [S.batched_scene(i) for i in range(14)]
    scenes.append(S.custom_scene(5, 7, 20, 64, 16, K=3, snr_db=15, seed=(12, 0, 0)))
    scenes.append(S.custom_scene(20, 6, 40, 16, 8, K=2, snr_db=20, seed=(13, 0, 0)))
    plans, ys, taus = _setup(scenes)
    batch = B.Batch(plans)
    print("classes", batch.classes(), flush=True)
    iters = 150
    outs = batch.fista(ys, taus, iters)
    outs2 = batch.fista(ys, taus, iters)          # graph replay: same bits
    for a, b in zip(outs, outs2):
        assert torch.equal(a, b)
    for i, sc in enumerate(scenes):
        P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, tau=taus[i], dense=False)
        ref = P.fista(iters)
        g = _np(outs[i])
        single = _np(plans[i].fista(ys[i], taus[i], iters))
        Fr = P.objective(ref)
        rel = abs(P.objective(g) - Fr) / Fr
        eps = np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-30)
        print(f"case batch scene {i} L={sc.L1}x{sc.L2} M={sc.M}: rel F={rel:.2e} eps_r={eps:.2e}", flush=True)
        assert rel <= OBJ_TOL
        assert abs(P.objective(single) - P.objective(g)) <= OBJ_TOL * Fr
    batch.close()


def test_batch_invariant_to_scene_order_and_autotune():
    scenes = [S.batched_scene(100 + i) for i in range(9)]
    plans, ys, taus = _setup(scenes)
    b1 = B.Batch(plans)
    o1 = b1.fista(ys, taus, 60)
    perm = [4, 0, 8, 2, 6, 1, 7, 3, 5]
    b2 = B.Batch([plans[i] for i in perm])
    o2 = b2.fista([ys[i] for i in perm], [taus[i] for i in perm], 60)
    for k, i in enumerate(perm):
        assert torch.equal(o2[k], o1[i])
    b2.autotune(reps=3)
    o3 = b2.fista([ys[i] for i in perm], [taus[i] for i in perm], 60)
    for k, i in enumerate(perm):
        a, b = _np(o3[k]), _np(o1[i])
        assert np.linalg.norm(a - b) <= 1e-4 * max(np.linalg.norm(b), 1e-30)
    b1.close()
    b2.close()


def test_batch_sparse_iterate_matches_dense_iterate():
    """Per-row slot storage of the batched FISTA iterates (the default) and dense iterates
    give the same bits, for iteration counts on both sides of the rows turning sparse."""
    scenes = [S.batched_scene(300 + i) for i in range(10)]
    scenes.append(S.custom_scene(20, 6, 40, 16, 8, K=2, snr_db=20, seed=(16, 0, 0)))
    plans, ys, taus = _setup(scenes)
    batch = B.Batch(plans)
    batch.set_support_columns(False)   # the full passes, where the option applies
    for iters in (1, 3, 40, 250):
        res = {}
        for on in (True, False):
            batch.set_sparse_iterate(on)
            res[on] = [o.clone() for o in batch.fista(ys, taus, iters)]
        same = all(torch.equal(a, b) for a, b in zip(res[True], res[False]))
        print(f"case batch sparse iterate iters={iters}: bitwise={same}", flush=True)
        assert same
    # a tuned launch shape changes the transforms' radix order, hence FP32 rounding: after
    # 250 iterations the trajectories agree to about 1e-4 (the launch-shape test's 1e-3 bound)
    batch.set_sparse_iterate(True)
    batch.autotune(reps=3)
    o = batch.fista(ys, taus, 250)
    for a, b in zip(o, res[False]):
        x, r = _np(a), _np(b)
        assert np.linalg.norm(x - r) <= 1e-3 * max(np.linalg.norm(r), 1e-30)
    assert B.lib.bccb_batch_set_sparse_iterate(batch._h, 2) == B.BCCB_E_INVALID
    batch.close()


def test_batch_support_columns_matches_full_passes():
    """The pruned batched iteration (kept spectral columns only; the default for size
    classes whose scenes all have few such columns) and the full passes give the same
    solutions to FP32 rounding, and both match the oracle's objective."""
    scenes = [S.batched_scene(400 + i) for i in range(12)]
    scenes.append(S.custom_scene(5, 7, 20, 64, 16, K=3, snr_db=15, seed=(19, 0, 0)))
    scenes.append(S.custom_scene(20, 6, 40, 32, 8, K=2, snr_db=20, seed=(20, 0, 0)))   # too many columns
    plans, ys, taus = _setup(scenes)
    print("kept columns", [p.support_columns() for p in plans], flush=True)
    batch = B.Batch(plans)
    for iters in (0, 1, 5, 200):
        res = {}
        for on in (True, False):
            batch.set_support_columns(on)
            res[on] = [_np(o) for o in batch.fista(ys, taus, iters)]
        for i, sc in enumerate(scenes):
            a, b = res[True][i], res[False][i]
            d = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            if iters <= 5:
                assert d <= 1e-4, (i, iters, d)
            if iters == 200:
                P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, tau=taus[i], dense=False)
                ref = P.fista(iters)
                Fr = P.objective(ref)
                rel = abs(P.objective(a) - Fr) / Fr
                print(f"case batch pruned scene {i} L={sc.L1}x{sc.L2}: rel F={rel:.2e} |pruned-full|={d:.1e}",
                      flush=True)
                assert rel <= OBJ_TOL
    batch.set_support_columns(True)
    batch.autotune(reps=3)
    o = batch.fista(ys, taus, 200)
    for i in range(len(scenes)):
        x, r = _np(o[i]), res[True][i]
        assert np.linalg.norm(x - r) <= 1e-3 * max(np.linalg.norm(r), 1e-30)
    assert B.lib.bccb_batch_set_support_columns(batch._h, 5) == B.BCCB_E_INVALID
    batch.close()


def test_batch_edge_cases():
    scenes = [S.batched_scene(200 + i) for i in range(3)]
    plans, ys, taus = _setup(scenes)
    batch = B.Batch(plans)
    outs = batch.fista(ys, taus, 0)
    for o in outs:
        assert torch.count_nonzero(o) == 0
    big = [1.01 * p.adjoint_maxabs(y) for p, y in zip(plans, ys)]
    for o in batch.fista(ys, big, 10):
        assert torch.count_nonzero(o) == 0
    bad = [y.clone() for y in ys]
    bad[1][0] = complex(float("inf"), 0.0)
    with pytest.raises(B.NonFiniteError):
        batch.fista(bad, taus, 5)
    with pytest.raises(B.BCCBError):
        batch.fista(ys, [-1.0] + taus[1:], 5)
    batch.close()


def test_full_uneven_workload_sampled():
    """All 4096 scenes of the uneven workload, 300 iterations, in the launch configuration
    the benchmark times (autotuned); a sample of scenes of every size is checked
    against the oracle one by one."""
    n = 4096
    scenes = [S.batched_scene(i) for i in range(n)]
    plans, ys, taus = _setup(scenes)
    batch = B.Batch(plans)
    batch.autotune(reps=3)
    print("classes", batch.classes(), flush=True)
    outs = batch.fista(ys, taus, 300)
    sample = {}
    for i, sc in enumerate(scenes):
        sample.setdefault(sc.L1, [])
        if len(sample[sc.L1]) < 2:
            sample[sc.L1].append(i)
    for L1, idx in sorted(sample.items()):
        for i in idx:
            sc = scenes[i]
            P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, tau=taus[i], dense=False)
            ref = P.fista(300)
            Fr = P.objective(ref)
            rel = abs(P.objective(_np(outs[i])) - Fr) / Fr
            print(f"case full-batch scene {i} L={L1}: rel F={rel:.2e}", flush=True)
            assert rel <= OBJ_TOL
    batch.close()
    for p in plans:
        p.close()


def test_batch_dense_grid_path():
    """The batch with the spectral support switched off (dense Omega and mu*b grids)."""
    scenes = [S.batched_scene(300 + i) for i in range(6)]
    plans, ys, taus = _setup(scenes)
    for p in plans:
        p.set_config(spectral_support=0)
    batch = B.Batch(plans)
    outs = batch.fista(ys, taus, 80)
    for i, sc in enumerate(scenes):
        P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, tau=taus[i], dense=False)
        ref = P.fista(80)
        rel = abs(P.objective(_np(outs[i])) - P.objective(ref)) / P.objective(ref)
        print(f"case dense-grid batch scene {i}: rel F={rel:.2e}", flush=True)
        assert rel <= OBJ_TOL
    batch.close()


U32 = 2.0 ** -24


def _iter_tol(T, L):
    # FP32 transforms of log2 L stages per iteration, errors adding at most linearly along T,
    # a factor 4 for the momentum re-applying the last two (as the full-size tests state)
    return 4.0 * max(T, 1) * U32 * np.log2(L)


def test_resident_launch_matches_pass_graph_and_oracle():
    """The persistent whole-solve launch (the default where every class supports it) against
    the captured pass graph and the oracle: 32^2 .. 256^2 grids, 8x8, 16x16 and 32x32 arrays,
    iteration counts on both sides of the rows turning sparse; same bits on a repeat call."""
    scenes = [S.batched_scene(500 + i) for i in range(15)]
    scenes += [S.tiny_scene(i) for i in range(3)]
    plans, ys, taus = _setup(scenes)
    batch = B.Batch(plans)
    info = batch.resident_info()
    print("classes", batch.classes(), "resident", info, flush=True)
    assert info["on"] == 1 and info["threads"] >= 256 and info["blocks"] >= 1
    for T in (1, 2, 3, 9, 60, 300):
        batch.set_resident(True)
        a = [o.clone() for o in batch.fista(ys, taus, T)]
        again = batch.fista(ys, taus, T)
        assert all(torch.equal(x, y) for x, y in zip(a, again))
        batch.set_resident(False)
        g = batch.fista(ys, taus, T)
        worst = 0.0
        for i, sc in enumerate(scenes):
            x, r = _np(a[i]), _np(g[i])
            d = np.linalg.norm(x - r) / max(np.linalg.norm(r), 1e-30)
            worst = max(worst, d / _iter_tol(T, sc.L1 * sc.L2))
            assert d <= 2 * _iter_tol(T, sc.L1 * sc.L2), (i, T, d)
        print(f"case resident vs graph T={T}: worst |diff| / bound {worst:.3f}", flush=True)
    for i, sc in enumerate(scenes):
        if i % 3:
            continue
        P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, tau=taus[i], dense=False)
        ref = P.fista(300)
        x = _np(a[i])
        Fr = P.objective(ref)
        rel = abs(P.objective(x) - Fr) / Fr
        eps = np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-30)
        print(f"case resident scene {i} L={sc.L1}: rel F {rel:.2e} eps_r {eps:.2e}", flush=True)
        assert rel <= OBJ_TOL and eps <= _iter_tol(300, sc.L1 * sc.L2)
    # zero iterations, and a threshold above max |D^H y|: zero grids
    batch.set_resident(True)
    assert all(torch.count_nonzero(o) == 0 for o in batch.fista(ys, taus, 0))
    big = [1.01 * p.adjoint_maxabs(y) for p, y in zip(plans, ys)]
    assert all(torch.count_nonzero(o) == 0 for o in batch.fista(ys, big, 7))
    assert B.lib.bccb_batch_set_resident(batch._h, 3) == B.BCCB_E_INVALID
    assert B.lib.bccb_batch_set_resident(batch._h, 128) == B.BCCB_E_INVALID
    batch.close()


def test_resident_launch_refusals():
    """A rectangular class keeps the whole batch on the pass graph."""
    scenes = [S.batched_scene(600), S.custom_scene(5, 7, 20, 64, 16, K=3, snr_db=15, seed=(21, 0, 0))]
    plans, ys, taus = _setup(scenes)
    batch = B.Batch(plans)
    assert batch.resident_info() == {"on": -1, "threads": 0, "blocks": 0, "lds_bytes": 0}
    with pytest.raises(B.BCCBError) as e:
        batch.set_resident(True)
    assert e.value.code == B.BCCB_E_UNSUPPORTED
    batch.set_resident(False)
    outs = batch.fista(ys, taus, 20)
    for i, sc in enumerate(scenes):
        P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, tau=taus[i], dense=False)
        ref = P.fista(20)
        assert abs(P.objective(_np(outs[i])) - P.objective(ref)) <= OBJ_TOL * P.objective(ref)
    batch.close()

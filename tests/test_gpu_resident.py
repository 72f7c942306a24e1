"""GPU parity of the single-scene cooperative solver (one launch per solve, the
workgroups meeting at grid barriers) against the two-pass path and the FP64 oracle.

The full cooperative form does the arithmetic of the passes at E = 4 element for
element, so against those passes the iterates agree to FP32 rounding of the
compiler's contraction choices; the pruned form replaces the column transforms
by sums at the support bins.  Both are held to rel <= 1e-5 against the passes
over short runs and to the oracle's objective (rel <= 1e-5) over long runs.
"""
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
SHORT_TOL = 1e-5
U32 = 2.0 ** -24   # FP32 unit roundoff


def admm_tol(iters, L):
    """Bound on one complex64 ADMM path's relative error after `iters` iterations: each
    iteration applies (G + rho I)^-1 once through transforms of relative error about
    u log2 L, and the scaled dual of eq. (15) is the running sum of the x-iterates while
    z stays at zero, so those errors add up instead of dying out."""
    return iters * U32 * np.log2(L)


GEOMS = {
    "tiny": lambda: S.tiny_scene(3),                    # 32 x 32: a single workgroup
    "sweep64": lambda: S.paper_sweep_scene(64, 1),      # L1 = 64, L2 = 32
    "sweep512": lambda: S.paper_sweep_scene(512, 1),    # L1 = 512, L2 = 32
    "rect": lambda: S.custom_scene(12, 9, 50, 128, 256, K=3, snr_db=20, seed=(21, 0, 0)),
    "paper": lambda: S.paper_scale_scene(2),            # 256 x 256
    "big": lambda: S.custom_scene(32, 32, 256, 512, 512, K=5, snr_db=20, seed=(22, 0, 0)),   # 512 x 512
}


def _np(t):
    return t.detach().cpu().numpy().reshape(-1).astype(np.complex128)


def _shapes(plan):
    """Launchable (groups, spread) pairs of the cooperative solver on this plan."""
    ok = []
    for k in range(9):
        for sp in (1, 8):
            try:
                plan.set_config(resident_groups=1 << k, resident_spread=sp)
                ok.append((1 << k, sp))
            except B.BCCBError:
                pass
    plan.set_config(resident_groups=0, resident_spread=1)
    return ok


def _passes(plan):
    plan.set_config(resident_groups=0, resident_spread=1, support_columns=0, row_elems=4, row_rows_per_block=1,
                    col_elems=4, col_cols_per_block=1)


def _solve(plan, solver, y, tau, iters, rho, c0=None):
    if solver == "admm":
        z, c = plan.admm(y, tau, rho, iters, want_c=True)
        return np.concatenate([_np(z), _np(c)])
    fn = plan.fista if solver == "fista" else plan.ista
    return _np(fn(y, tau, iters, c0=c0))


@pytest.mark.parametrize("geom", list(GEOMS))
def test_resident_matches_passes(geom):
    sc = GEOMS[geom]()
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    shapes = _shapes(plan)
    print(f"case {geom} L1={sc.L1} L2={sc.L2}: cooperative shapes {shapes}", flush=True)
    assert shapes, "no launchable cooperative shape"
    # the fewest and the most workgroups, each with and without spreading
    Gs = sorted({shapes[0][0], shapes[-1][0]})
    picks = [s for s in shapes if s[0] in Gs]
    y = B.to_device(sc.y)
    tau = float(np.float32(0.1 * plan.adjoint_maxabs(y)))
    rho = float(np.count_nonzero(sc.mask))
    rng = np.random.default_rng(5)
    for solver in ("ista", "fista", "admm"):
        for iters in (1, 2, 37):
            for warm in ((False, True) if solver != "admm" else (False,)):
                c0 = None
                if warm:
                    _passes(plan)
                    w = _np(plan.fista(y, tau, 15)) * (1 + 0.1 * rng.standard_normal(sc.L1 * sc.L2))
                    c0 = B.to_device(w.reshape(sc.L2, sc.L1).astype(np.complex64))
                _passes(plan)
                ref = _solve(plan, solver, y, tau, iters, rho, c0)
                nr = max(np.linalg.norm(ref), 1e-30)
                for G, sp in picks:
                    plan.set_config(resident_groups=G, resident_spread=sp)
                    got = _solve(plan, solver, y, tau, iters, rho, c0)
                    d = np.linalg.norm(got - ref) / nr
                    print(f"  {solver} iters={iters} warm={warm} G={G} spread={sp}: rel diff {d:.1e}", flush=True)
                    assert d <= SHORT_TOL, (solver, iters, warm, G, sp, d)
    plan.close()


@pytest.mark.parametrize("geom", ["tiny", "sweep512", "paper"])
def test_resident_objective_matches_oracle(geom):
    """Long runs through the cooperative solver against the FP64 oracle's objective."""
    sc = GEOMS[geom]()
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=None)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    shapes = _shapes(plan)
    G, sp = shapes[len(shapes) // 2]
    plan.set_config(resident_groups=G, resident_spread=sp)
    y = B.to_device(sc.y)
    rho = float(np.count_nonzero(sc.mask))
    iters = 300
    for solver in ("ista", "fista", "admm"):
        print(f"case {geom} {solver} G={G} spread={sp} iters={iters}", flush=True)
        if solver == "admm":
            g = _np(plan.admm(y, P.tau, rho, iters))
            ref = P.admm(rho, iters)[0]
        else:
            g = _np((plan.fista if solver == "fista" else plan.ista)(y, P.tau, iters))
            ref = (P.fista if solver == "fista" else P.ista)(iters)
        Fr = P.objective(ref)
        rel = abs(P.objective(g) - Fr) / Fr
        eps = np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-30)
        print(f"  rel F = {rel:.2e}, eps_r = {eps:.2e}", flush=True)
        assert rel <= OBJ_TOL
    plan.close()


def test_resident_rejects_nonfinite_warm_start_and_recovers():
    sc = GEOMS["paper"]()
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    G, sp = _shapes(plan)[0]
    plan.set_config(resident_groups=G, resident_spread=sp)
    y = B.to_device(sc.y)
    tau = float(np.float32(0.1 * plan.adjoint_maxabs(y)))
    bad = np.zeros((sc.L2, sc.L1), np.complex64)
    bad[3, 7] = np.nan
    print("case non-finite warm start", flush=True)
    with pytest.raises(B.NonFiniteError):
        plan.fista(y, tau, 5, c0=B.to_device(bad))
    # the next solve on the same plan is unaffected
    a = _np(plan.fista(y, tau, 20))
    _passes(plan)
    b = _np(plan.fista(y, tau, 20))
    assert np.linalg.norm(a - b) <= SHORT_TOL * np.linalg.norm(b)
    plan.close()


def test_resident_autotune_and_profile():
    """autotune weighs the cooperative shapes against the passes; whatever it keeps
    solves the same problem, and the cooperative launch can be timed on its own."""
    sc = GEOMS["paper"]()
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=None)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    cfg = plan.autotune(20)
    print(f"case autotune: {cfg}", flush=True)
    y = B.to_device(sc.y)
    g = _np(plan.fista(y, P.tau, 200))
    ref = P.fista(200)
    assert abs(P.objective(g) - P.objective(ref)) / P.objective(ref) <= OBJ_TOL
    G, sp = _shapes(plan)[-1]
    plan.set_config(resident_groups=G, resident_spread=sp)
    for solver in ("ista", "fista", "admm"):
        ms = plan.profile_resident(solver, 100, reps=3)
        print(f"  {solver}: {ms * 1e3 / 100:.2f} us per iteration (G={G}, spread={sp})", flush=True)
        assert ms > 0
    plan.set_config(resident_groups=0)
    with pytest.raises(B.BCCBError):
        plan.profile_resident("fista", 10, reps=1)
    plan.close()


def _admm_pruned_vs_passes(plan, P, y, rho, cfg):
    """ADMM's (z, x) through the pruned cooperative form and through the full passes
    against the FP64 oracle, each within admm_tol, and against each other."""
    L = P.op.L
    for iters in (1, 2, 37):
        zr, xr = P.admm(rho, iters)
        ref = np.concatenate([zr, xr])
        nr = max(np.linalg.norm(ref), 1e-30)
        plan.set_config(**cfg)
        assert plan.support_columns()[1] == 2
        got = _solve(plan, "admm", y, P.tau, iters, rho)
        plan.set_config(resident_groups=0, support_columns=0)
        pas = _solve(plan, "admm", y, P.tau, iters, rho)
        eg, ep = np.linalg.norm(got - ref) / nr, np.linalg.norm(pas - ref) / nr
        d = np.linalg.norm(got - pas) / nr
        tol = admm_tol(iters, L)
        print(f"  admm iters={iters}: pruned cooperative vs FP64 {eg:.1e}, passes vs FP64 {ep:.1e}, "
              f"between them {d:.1e} (bound {tol:.1e} per path)", flush=True)
        assert eg <= tol and ep <= tol and d <= 2 * tol, (iters, eg, ep, d)


@pytest.mark.parametrize("block", [256, 512])
@pytest.mark.parametrize("geom", ["tiny", "sweep512", "rect", "paper"])
def test_resident_pruned_matches_passes(geom, block):
    """The pruned cooperative form (per-group parts of DFT2 at the support bins exchanged,
    every group adding all of them, one barrier per iteration) against the pruned and the
    full passes, cold and warm started, and the oracle's objective over a long run; ADMM
    (no pruned passes) against the full passes."""
    sc = GEOMS[geom]()
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=None)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    shapes = _shapes(plan)
    G, sp = shapes[0]
    plan.set_config(support_columns=1, resident_groups=G, resident_spread=sp, resident_block=block)
    ncols, mode = plan.support_columns()
    print(f"case {geom} block {block}: kept columns {ncols}, support-column mode {mode}", flush=True)
    if mode != 2:
        plan.close()
        pytest.skip("the pruned cooperative form does not fit this geometry")
    y = B.to_device(sc.y)
    tau = P.tau
    rng = np.random.default_rng(6)
    w = P.fista(15) * (1 + 0.1 * rng.standard_normal(sc.L1 * sc.L2))
    warm = B.to_device(w.reshape(sc.L2, sc.L1).astype(np.complex64))
    for solver in ("ista", "fista"):
        fn = plan.fista if solver == "fista" else plan.ista
        for iters in (1, 2, 37):
            for c0 in (None, warm):
                plan.set_config(support_columns=1, resident_groups=G, resident_spread=sp, resident_block=block)
                got = _np(fn(y, tau, iters, c0=c0))
                plan.set_config(resident_groups=0, support_columns=1)
                ref_p = _np(fn(y, tau, iters, c0=c0))
                plan.set_config(resident_groups=0, support_columns=0)
                ref_f = _np(fn(y, tau, iters, c0=c0))
                nr = max(np.linalg.norm(ref_f), 1e-30)
                dp = np.linalg.norm(got - ref_p) / nr
                df = np.linalg.norm(got - ref_f) / nr
                print(f"  {solver} iters={iters} warm={c0 is not None}: vs pruned passes {dp:.1e}, "
                      f"vs full passes {df:.1e}", flush=True)
                assert dp <= SHORT_TOL and df <= SHORT_TOL, (solver, iters, dp, df)
        plan.set_config(support_columns=1, resident_groups=G, resident_spread=sp, resident_block=block)
        g = _np(fn(y, tau, 300))
        ref = (P.fista if solver == "fista" else P.ista)(300)
        Fr = P.objective(ref)
        rel = abs(P.objective(g) - Fr) / Fr
        print(f"  {solver} 300 iterations: rel F = {rel:.2e}", flush=True)
        assert rel <= OBJ_TOL
    # ADMM in the pruned form: (z, x) against the FP64 oracle and the full passes (each
    # path within admm_tol of FP64, so two paths within twice that), and the objective
    rho = float(np.count_nonzero(sc.mask))
    _admm_pruned_vs_passes(plan, P, y, rho, dict(support_columns=1, resident_groups=G, resident_spread=sp,
                                                 resident_block=block))
    plan.set_config(support_columns=1, resident_groups=G, resident_spread=sp, resident_block=block)
    g = _np(plan.admm(y, tau, rho, 300))
    ref = P.admm(rho, 300)[0]
    Fr = P.objective(ref)
    rel = abs(P.objective(g) - Fr) / Fr
    print(f"  admm 300 iterations: rel F = {rel:.2e}", flush=True)
    assert rel <= OBJ_TOL
    plan.close()


@pytest.mark.parametrize("geom,seed,iters", [("tiny", 0, 200), ("paper", 2, 500)])
def test_resident_pruned_admm_small_rho(geom, seed, iters):
    """ADMM with rho = 1, far below Omega on the support, where the scaled dual grows to about
    S / rho on the support modes: the pruned form keeps that part of the dual as spectral
    coefficients, so x is never formed by cancelling large terms (forming it as (z - v) plus a
    support correction missed the objective bound on the first scene).  z and x against FP64
    within admm_tol, the objective of z within OBJ_TOL."""
    sc = S.tiny_scene(seed) if geom == "tiny" else S.paper_scale_scene(seed)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=None)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    G, sp = _shapes(plan)[0]
    plan.set_config(support_columns=1, resident_groups=G, resident_spread=sp)
    if plan.support_columns()[1] != 2:
        plan.close()
        pytest.skip("the pruned cooperative form does not fit this geometry")
    y = B.to_device(sc.y)
    z, x = plan.admm(y, P.tau, 1.0, iters, want_c=True)
    z, x = _np(z), _np(x)
    zr, xr = P.admm(1.0, iters)
    tol = admm_tol(iters, P.op.L)
    ez = np.linalg.norm(z - zr) / max(np.linalg.norm(zr), 1e-30)
    ex = np.linalg.norm(x - xr) / max(np.linalg.norm(xr), 1e-30)
    Fr = P.objective(zr)
    rel = abs(P.objective(z) - Fr) / Fr
    print(f"case {geom} seed {seed} rho 1 iters {iters}: z vs FP64 {ez:.1e}, x vs FP64 {ex:.1e}, rel F {rel:.1e} "
          f"(bound {tol:.1e})", flush=True)
    assert ez <= tol and ex <= tol and rel <= OBJ_TOL
    plan.close()


@pytest.mark.parametrize("block", [256, 512])
def test_resident_pruned_largest_grid(block):
    """The pruned cooperative form at 512 x 512 (256 or 128 groups, 256 support bins in
    32 kept columns) against the pruned and the full passes over short runs (ADMM against
    the full passes)."""
    sc = GEOMS["big"]()
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    G, sp = _shapes(plan)[0]
    plan.set_config(support_columns=1, resident_groups=G, resident_spread=sp, resident_block=block)
    ncols, mode = plan.support_columns()
    print(f"case 512x512 block {block}: kept columns {ncols}, support-column mode {mode}", flush=True)
    assert mode == 2
    y = B.to_device(sc.y)
    tau = float(np.float32(0.1 * plan.adjoint_maxabs(y)))
    for solver in ("ista", "fista"):
        fn = plan.fista if solver == "fista" else plan.ista
        for iters in (1, 2, 37):
            plan.set_config(support_columns=1, resident_groups=G, resident_spread=sp, resident_block=block)
            got = _np(fn(y, tau, iters))
            plan.set_config(resident_groups=0, support_columns=1)
            ref_p = _np(fn(y, tau, iters))
            plan.set_config(resident_groups=0, support_columns=0)
            ref_f = _np(fn(y, tau, iters))
            nr = max(np.linalg.norm(ref_f), 1e-30)
            dp, df = np.linalg.norm(got - ref_p) / nr, np.linalg.norm(got - ref_f) / nr
            print(f"  {solver} iters={iters}: vs pruned passes {dp:.1e}, vs full passes {df:.1e}", flush=True)
            assert dp <= SHORT_TOL and df <= SHORT_TOL, (solver, iters, dp, df)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=None)
    _admm_pruned_vs_passes(plan, P, B.to_device(sc.y), float(np.count_nonzero(sc.mask)),
                           dict(support_columns=1, resident_groups=G, resident_spread=sp, resident_block=block))
    plan.close()


@pytest.mark.parametrize("geom,block", [("paper", 256), ("paper", 512), ("big", 256), ("big", 512), ("sweep512", 256)])
def test_resident_repeated_solves_identical(geom, block):
    """Solves repeated on one plan give bitwise the same result, in both cooperative forms:
    nothing one solve leaves in the barrier words or the exchange buffers may let a later
    solve's groups run ahead (a regression test: the barrier words were once cleared by a
    separate kernel before every solve, and later solves at 256 groups read the previous
    solve's parts at their first barrier)."""
    sc = GEOMS[geom]()
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    shapes = _shapes(plan)
    y = B.to_device(sc.y)
    tau = float(np.float32(0.1 * plan.adjoint_maxabs(y)))
    for support_columns, G in ((1, shapes[0][0]), (0, shapes[-1][0])):
        plan.set_config(support_columns=support_columns, resident_groups=G, resident_spread=1, resident_block=block)
        for solver in ("ista", "fista", "admm"):
            for iters in (2, 9):
                outs = [_solve(plan, solver, y, tau, iters, 40.0) for _ in range(4)]
                same = all(np.array_equal(outs[0], o) for o in outs[1:])
                print(f"case {geom} block {block} support_columns {support_columns} G {G} {solver} {iters}: "
                      f"mode {plan.support_columns()[1]}, identical {same}", flush=True)
                assert same
    plan.close()

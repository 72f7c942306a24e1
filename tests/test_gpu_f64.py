"""GPU parity of the FP64 device variants (complex128 passes) with the FP64 oracle, at the
level of the paper's FP64 regular-vs-fast comparison (Table I).

Bounds: products within 1e-13 relative; iterates within TOL64(T, L) = 4 T u log2(L) with
u = 2^-53 (the FP32 bound's derivation with double rounding: each iteration adds the
relative error of transforms of log2 L stages, the soft threshold is nonexpansive and the
momentum re-applies the last two errors); ADMM's x-update multiplies by (G + rho I)^-1, whose
condition number (max Omega + rho) / rho amplifies the rounding of the products, so its bound
carries that factor.  Objectives within 1e-12 relative.
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

U64 = 2.0 ** -53


def tol64(T, L, cond=1.0):
    return 4.0 * max(T, 1) * U64 * np.log2(L) * cond


def _np(t):
    return t.detach().cpu().numpy().reshape(-1)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _dev64(a, shape=None):
    x = np.asarray(a, dtype=np.complex128)
    if shape is not None:
        x = x.reshape(shape)
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


SCENES = {
    "tiny": lambda: S.tiny_scene(2),
    "rect": lambda: S.custom_scene(8, 6, 30, 64, 16, K=3, snr_db=20, seed=(12, 0, 1)),
    "paper": lambda: S.paper_scale_scene(0),
}


@pytest.mark.parametrize("name", list(SCENES))
def test_f64_products_and_solvers(name):
    sc = SCENES[name]()
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y, dense=sc.L1 * sc.L2 <= 4096)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    y = _dev64(P.y)
    b = _np(plan.adjoint_f64(y))
    x = np.random.default_rng(3).standard_normal(P.op.L) + 1j * np.random.default_rng(4).standard_normal(P.op.L)
    gx = _np(plan.gram_apply_f64(_dev64(x, (sc.L2, sc.L1))))
    eb, eg = _rel(b, P.b), _rel(gx, P.apply_G(x))
    print(f"case f64 {name} {sc.L1}x{sc.L2}: adjoint {eb:.2e}, gram {eg:.2e}", flush=True)
    assert eb <= 1e-13 and eg <= 1e-13
    T = 200 if name != "paper" else 60
    L = P.op.L
    for solver in ("fista", "ista"):
        g = _np(getattr(plan, solver + "_f64")(y, P.tau, T))
        ref = getattr(P, solver)(T)
        Fr = P.objective(ref)
        rel, eps = abs(P.objective(g) - Fr) / Fr, _rel(g, ref)
        print(f"  {solver} T={T}: rel F {rel:.2e}, eps_r {eps:.2e} (bound {tol64(T, L):.1e})", flush=True)
        assert rel <= 1e-12 and eps <= tol64(T, L)
    om_max = float(plan.omega().max())
    for rho in (1.0, 40.0):
        z, c = plan.admm_f64(y, P.tau, rho, T, want_c=True)
        zr, cr = P.admm(rho, T)
        ez = _rel(_np(z), zr) if np.linalg.norm(zr) > 0 else np.linalg.norm(_np(z))
        ec = _rel(_np(c), cr)
        bound = tol64(T, L, cond=(om_max + rho) / rho)
        print(f"  admm rho={rho} T={T}: z {ez:.2e}, c {ec:.2e} (bound {bound:.1e})", flush=True)
        assert ez <= bound and ec <= bound
    # warm start and zero iterations
    c0 = P.fista(4)
    g0 = _np(plan.fista_f64(y, P.tau, 0, c0=_dev64(c0, (sc.L2, sc.L1))))
    assert np.array_equal(g0, c0)
    plan.close()


def test_f64_table1_regular_vs_fast():
    """Table I's comparison with the fast side on this GPU in FP64: the oracle's explicit-Gram
    ISTA / FISTA / ADMM (regular) against the FP64 device passes (fast) at the sweep geometry
    (L1 = 64, L2 = 32, 10 trials), eps_r at n_iter = 50 .. 400 of the order Table I prints."""
    trials = S.paper_sweep_trials(64, 10)
    mask = trials[0].mask
    plan = B.Plan(mask, 64, 32)
    rho = 40.0
    worst = {"ista": 0.0, "fista": 0.0, "admm": 0.0}
    for sc in trials:
        P = O.Problem(mask, 64, 32, sc.y, dense=True)
        Minv = O.shifted_inverse_dense(P.op, rho)
        y = _dev64(P.y)
        for n in (50, 100, 200, 400):
            for solver in ("ista", "fista"):
                reg = getattr(O, solver)(P.apply_G, P.b, P.mu, P.tau, n)
                fast = _np(getattr(plan, solver + "_f64")(y, P.tau, n))
                worst[solver] = max(worst[solver], _rel(fast, reg))
            zr, _ = O.admm(lambda v: Minv @ v, P.b, rho, P.tau, n)
            zf = _np(plan.admm_f64(y, P.tau, rho, n))
            worst["admm"] = max(worst["admm"], _rel(zf, zr))
    print("case f64 table I, worst eps_r over 10 trials x 4 n_iter:", {k: f"{v:.2e}" for k, v in worst.items()},
          flush=True)
    assert worst["ista"] <= 1e-12 and worst["fista"] <= 1e-12 and worst["admm"] <= 1e-10
    plan.close()

"""GPU parity of the dense explicit-matrix baseline (the paper's "regular" implementation)."""
import numpy as np
import pytest

from oracle import bccb_oracle as O
from paper_2509_13592_amd import scenes as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2509_13592_amd.bccb")


def _np(t):
    return t.detach().cpu().numpy().reshape(-1).astype(np.complex128)


@pytest.mark.parametrize("scene,iters,rho", [("tiny", 60, 64.0), ("paper", 5, 1.0)])
def test_dense_solvers_match_oracle(scene, iters, rho):
    sc = S.tiny_scene(4) if scene == "tiny" else S.paper_scale_scene(3)
    P = O.Problem(sc.mask, sc.L1, sc.L2, sc.y)
    plan = B.Plan(sc.mask, sc.L1, sc.L2)
    y = B.to_device(sc.y)
    print(f"case dense {scene}: building the {sc.L1 * sc.L2}^2 matrix", flush=True)
    dense = B.Dense(plan, kind=0)
    x = (np.random.default_rng(1).standard_normal(plan.L) + 1j).astype(np.complex64)
    rx = _np(dense.apply(B.to_device(x.reshape(plan.L2, plan.L1))))
    ref = x - P.mu * P.op.gram(x.astype(np.complex128))
    assert np.linalg.norm(rx - ref) <= 1e-5 * np.linalg.norm(ref)
    for name in ("ista", "fista"):
        g = _np(dense.solve(name, y, P.tau, iters))
        r = P.ista(iters) if name == "ista" else P.fista(iters)
        rel = abs(P.objective(g) - P.objective(r)) / P.objective(r)
        bccb = _np(getattr(plan, name)(y, P.tau, iters))
        print(f"case dense {scene} {name}: rel F vs FP64 = {rel:.2e}; "
              f"dense vs BCCB eps = {np.linalg.norm(g - bccb) / max(np.linalg.norm(bccb), 1e-30):.2e}", flush=True)
        assert rel <= 1e-5
    dense.close()
    dense = B.Dense(plan, kind=1, rho=rho)
    z = _np(dense.solve("admm", y, P.tau, iters))
    zr, cr = P.admm(rho, iters)
    rel = abs(P.objective(z) - P.objective(zr)) / P.objective(zr)
    print(f"case dense {scene} admm: rel F vs FP64 = {rel:.2e}", flush=True)
    assert rel <= 1e-5
    with pytest.raises(B.BCCBError):
        dense.solve("fista", y, P.tau, 3)       # the ADMM matrix serves ADMM only
    dense.close()
    plan.close()

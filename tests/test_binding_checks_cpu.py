"""The Python binding checks every buffer's size against the plan before it calls the
library: a wrong-sized snapshot, grid, batch or weight list raises on the host, so no
kernel can write past an allocation.  Runs without a GPU: the plan objects are built
without the library and the library itself is replaced by a sentinel that fails the
test if any entry point is reached."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2509_13592_amd.bccb")


class _NoLib:
    def __getattr__(self, name):
        def call(*args):
            raise AssertionError(f"library entry point {name} reached")
        return call


@pytest.fixture
def nolib(monkeypatch):
    monkeypatch.setattr(B, "lib", _NoLib())


def _fake_plan(M=5, L1=8, L2=4):
    p = object.__new__(B.Plan)
    p._h = None
    p.M, p.L1, p.L2, p.L = M, L1, L2, L1 * L2
    p.M1, p.M2 = 4, 2
    return p


def _c(n):
    return torch.zeros(n, dtype=torch.complex64)


def _size_error(fn):
    with pytest.raises(ValueError, match="expected"):
        fn()


def _gpu_error(fn):
    with pytest.raises(ValueError, match="GPU"):
        fn()


def test_plan_calls_check_sizes(nolib):
    p = _fake_plan()
    good_y, good_g = _c(p.M), _c(p.L)
    for bad in (_c(p.M - 1), _c(p.M + 1)):
        _size_error(lambda: p.fista(bad, 0.1, 3, out=good_g))
        _size_error(lambda: p.ista(bad, 0.1, 3, out=good_g))
        _size_error(lambda: p.admm(bad, 0.1, 1.0, 3, z_out=good_g))
        _size_error(lambda: p.adjoint(bad, out=good_g))
        _size_error(lambda: p.objective_kkt(bad, 0.1, good_g))
    for bad in (_c(p.L - 1), _c(p.L + 8)):
        _size_error(lambda: p.fista(good_y, 0.1, 3, out=bad))
        _size_error(lambda: p.fista(good_y, 0.1, 3, c0=bad, out=good_g))
        _size_error(lambda: p.admm(good_y, 0.1, 1.0, 3, z_out=good_g, c_out=bad, want_c=True))
        _size_error(lambda: p.gram_apply(bad, out=good_g))
        _size_error(lambda: p.gram_apply(good_g, out=bad))
        _size_error(lambda: p.objective_kkt(good_y, 0.1, bad))
    # right sizes on host memory: refused for the device, still before the library
    _gpu_error(lambda: p.fista(good_y, 0.1, 3, out=good_g))
    with pytest.raises(TypeError):
        p.fista(torch.zeros(p.M, dtype=torch.complex128), 0.1, 3, out=good_g)


def test_batch_checks_every_scene(nolib):
    plans = [_fake_plan(5, 8, 4), _fake_plan(7, 16, 8)]
    b = object.__new__(B.Batch)
    b.plans, b.n, b._h = plans, 2, None
    ys = [_c(5), _c(7)]
    outs = [_c(32), _c(128)]
    _size_error(lambda: b.fista(ys, [0.1], 3, outs=outs))               # one weight short
    _size_error(lambda: b.fista(ys[:1], [0.1, 0.1], 3, outs=outs))       # one snapshot short
    _size_error(lambda: b.fista([_c(5), _c(5)], [0.1, 0.1], 3, outs=outs))
    _size_error(lambda: b.fista(ys, [0.1, 0.1], 3, outs=[_c(32), _c(32)]))
    _gpu_error(lambda: b.fista(ys, [0.1, 0.1], 3, outs=outs))


def test_lista_checks_batch_and_weights(nolib):
    plan = _fake_plan(5, 8, 4)
    net = object.__new__(B.Lista)
    net.plan, net.layers, net.max_batch, net._h, net._batch = plan, 3, 4, None, 0
    params = torch.zeros((3, B.LISTA_PER_LAYER), dtype=torch.float32)
    ys = torch.zeros((2, 5), dtype=torch.complex64)
    out = torch.zeros((2, 4, 8), dtype=torch.complex64)
    _size_error(lambda: net.forward(params, ys, [0.1], out=out))                 # taus short
    _size_error(lambda: net.forward(params, ys, [0.1, 0.1, 0.1], out=out))       # taus long
    _size_error(lambda: net.forward(params, torch.zeros((2, 6), dtype=torch.complex64), [0.1, 0.1], out=out))
    _size_error(lambda: net.forward(params, torch.zeros((5, 5), dtype=torch.complex64), [0.1] * 5))
    _size_error(lambda: net.forward(params, ys, [0.1, 0.1], out=out[:1]))
    _size_error(lambda: net.forward(params[:2], ys, [0.1, 0.1], out=out))
    _size_error(lambda: net.solve(params, ys, [0.1], out=out))
    _size_error(lambda: net.solve(params, ys, [0.1, 0.1], out=out[:1]))
    with pytest.raises(ValueError, match="forward"):
        net.backward(params, out)                         # no training forward yet
    net._batch = 2
    _size_error(lambda: net.backward(params, out[:1]))
    _size_error(lambda: net.backward(params, out, grad=torch.zeros(5, dtype=torch.float32)))
    _gpu_error(lambda: net.forward(params, ys, np.float32([0.1, 0.1]), out=out))


def test_adam_checks_sizes(nolib):
    p = torch.zeros(10, dtype=torch.float32)
    opt = object.__new__(B.Adam)
    opt.p, opt.m, opt.v = p, torch.zeros(10), torch.zeros(10)
    opt.lr, opt.b1, opt.b2, opt.eps, opt.lr_scale, opt.t = 1e-3, 0.9, 0.999, 1e-8, None, 0
    _size_error(lambda: opt.step(torch.zeros(9, dtype=torch.float32)))

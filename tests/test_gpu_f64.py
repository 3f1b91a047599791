"""FP64 plans (ri_plan_create with RI_F64) against the FP64 oracle.

Both sides compute in double, so the bar is round-off of double: 1e-10
relative L2 on forward, adjoint and prox outputs (FFTs of a few thousand
points and at most a few dozen dual steps: ~1e-14 is expected), and 1e-9 on
whole solves.  Real and complex objects, 3D and per-plane 2D TV.
"""
import numpy as np
import pytest

from oracle import optics, prox, fista, complex_object as co
from paper_1904_04884_amd import rihvr, scenes

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def cdev(torch, z):
    return dev(torch, np.stack([np.real(z), np.imag(z)]))


def chost(t):
    a = t.cpu().numpy()
    return a[0] + 1j * a[1]


def geom(nx, ny, nz, **kw):
    return scenes.geometry_c1().with_(nx=nx, ny=ny, nz=nz, **kw)


SHAPES = [(64, 48, 6), (96, 96, 5), (48, 64, 1), (128, 96, 9)]


@pytest.fixture(scope="module")
def plan64():
    cache = {}

    def get(g):
        if g not in cache:
            cache[g] = rihvr.Plan(g, dtype=rihvr.RI_F64)
        return cache[g]
    yield get
    for p in cache.values():
        p.close()


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("carrier", [True, False])
def test_forward_adjoint(torch_cuda, plan64, shape, carrier):
    torch = torch_cuda
    g = geom(*shape, carrier=carrier)
    p = plan64(g)
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal(g.shape)
    r = rng.standard_normal((g.ny, g.nx))
    assert p.lipschitz == pytest.approx(optics.lipschitz(g), rel=1e-12)
    b = p.forward(dev(torch, x)).cpu().numpy()
    assert b.dtype == np.float64
    assert rel_l2(b, optics.forward(g, x)) <= 1e-10
    xt = p.adjoint(dev(torch, r)).cpu().numpy()
    assert rel_l2(xt, optics.adjoint(g, r)) <= 1e-10


@pytest.mark.parametrize("shape", [(64, 48, 6), (96, 64, 3)])
def test_forward_adjoint_complex(torch_cuda, plan64, shape):
    torch = torch_cuda
    g = geom(*shape, complex_object=True)
    p = plan64(g)
    rng = np.random.default_rng(5 + sum(shape))
    x = rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)
    r = rng.standard_normal((g.ny, g.nx))
    assert p.lipschitz == pytest.approx(float(g.nz), rel=1e-12)
    assert rel_l2(p.forward(cdev(torch, x)).cpu().numpy(), co.forward(g, x)) <= 1e-10
    assert rel_l2(chost(p.adjoint(dev(torch, r))), co.adjoint(g, r)) <= 1e-10


@pytest.mark.parametrize("dims", [3, 2])
@pytest.mark.parametrize("nonneg", [True, False])
@pytest.mark.parametrize("k", [0, 1, 7, 20])
def test_prox(torch_cuda, plan64, dims, nonneg, k):
    torch = torch_cuda
    g = geom(64, 48, 7, tv_dims=dims)
    p = plan64(g)
    rng = np.random.default_rng(11 * k + dims + nonneg)
    v = 0.3 * rng.standard_normal(g.shape)
    ref = prox.prox_fused_lasso(v, 0.6, 0.05, 0.3, k, nonneg, dims=dims)
    vd = dev(torch, v)
    out = p.prox(vd, 0.6, 0.05, 0.3, k, nonneg=nonneg)
    assert rel_l2(out.cpu().numpy(), ref) <= 1e-10
    w = vd.clone()
    p.prox(w, 0.6, 0.05, 0.3, k, nonneg=nonneg, out=w)
    assert torch.equal(w, out)


@pytest.mark.parametrize("dims", [3, 2])
def test_prox_complex(torch_cuda, plan64, dims):
    torch = torch_cuda
    g = geom(64, 48, 5, tv_dims=dims, complex_object=True)
    p = plan64(g)
    rng = np.random.default_rng(21 + dims)
    v = 0.3 * (rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape))
    ref = co.prox_fused_lasso(v, 0.6, 0.05, 0.3, 15, dims)
    out = chost(p.prox(cdev(torch, v), 0.6, 0.05, 0.3, 15, nonneg=False))
    assert rel_l2(out, ref) <= 1e-10


@pytest.fixture(scope="module")
def c1_problem():
    sc = scenes.scene_c1(seed=8)
    g, cfg = sc.geometry, sc.config
    b = optics.forward(g, sc.dense()) + sc.noise
    return g, cfg, b


@pytest.mark.parametrize("restart", [False, True])
def test_solve(torch_cuda, plan64, c1_problem, restart):
    torch = torch_cuda
    g, cfg, b = c1_problem
    p = plan64(g)
    iters, k_in = 12, 5
    flags = rihvr.RI_SOLVE_RESTART if restart else 0
    x, rep, st = p.solve(dev(torch, b), cfg.l1, cfg.tv, iters, k_in, flags=flags)
    assert st == rihvr.RI_OK and rep["iters"] == iters
    ref = fista.fista(g, b, cfg.l1, cfg.tv, iters, k_in, restart=restart)
    assert rel_l2(x.cpu().numpy(), ref) <= 1e-9
    F = fista.objective(g, ref, b, cfg.l1, cfg.tv)
    assert rep["objective"] == pytest.approx(F, rel=1e-10)


def test_solve_given_start_and_gap_stop(torch_cuda, plan64, c1_problem):
    torch = torch_cuda
    g, cfg, b = c1_problem
    p = plan64(g)
    x0 = fista.fista(g, b, cfg.l1, cfg.tv, 3, 4)
    x, rep, _ = p.solve(dev(torch, b), cfg.l1, cfg.tv, 5, 4, x=dev(torch, x0), x0_scale=0.5)
    ref = fista.fista(g, b, cfg.l1, cfg.tv, 5, 4, x0=0.5 * x0)
    assert rel_l2(x.cpu().numpy(), ref) <= 1e-9
    # stop at a gap: the oracle's objective history says where
    _, hist = fista.fista(g, b, cfg.l1, cfg.tv, 40, 4, history=True)
    f_ref = min(hist) * (1.0 - 1e-3)
    tol = 0.02
    want = next(k + 1 for k, f in enumerate(hist) if (f - f_ref) / f_ref <= tol)
    _, rep, _ = p.solve(dev(torch, b), cfg.l1, cfg.tv, 40, 4, f_ref=f_ref, gap_tol=tol)
    assert rep["converged"] and rep["iters"] == want


def test_solve_complex(torch_cuda, plan64):
    torch = torch_cuda
    sc = scenes.scene_c1(seed=9)
    g, cfg = sc.geometry.with_(complex_object=True), sc.config
    psi = np.random.default_rng(1).uniform(-0.8, 0.8, g.nz)
    b = co.forward(g, sc.dense() * np.exp(1j * psi)[:, None, None]) + sc.noise
    p = plan64(g)
    x, rep, _ = p.solve(dev(torch, b), cfg.l1, cfg.tv, 10, 4, nonneg=False)
    ref = co.fista(g, b, cfg.l1, cfg.tv, 10, 4)
    assert rel_l2(chost(x), ref) <= 1e-9
    assert rep["objective"] == pytest.approx(co.objective(g, ref, b, cfg.l1, cfg.tv), rel=1e-10)


def test_fp32_path_differs_from_fp64_by_rounding_only(torch_cuda, plan64, c1_problem):
    """The FP32 kernels and the FP64 path on the same problem: apart by FP32
    round-off (well inside the FP32 solve bar), while the FP64 path sits on
    the oracle."""
    torch = torch_cuda
    g, cfg, b = c1_problem
    p64 = plan64(g)
    p32 = rihvr.Plan(g)
    try:
        x32, _, _ = p32.solve(torch.from_numpy(b.astype(np.float32)).cuda(), cfg.l1, cfg.tv, 30, 10)
        x64, _, _ = p64.solve(dev(torch, b.astype(np.float32).astype(np.float64)), cfg.l1, cfg.tv, 30, 10)
    finally:
        p32.close()
    ref = fista.fista(g, b.astype(np.float32).astype(np.float64), cfg.l1, cfg.tv, 30, 10)
    e64 = rel_l2(x64.cpu().numpy(), ref)
    e32 = rel_l2(x32.cpu().numpy().astype(np.float64), x64.cpu().numpy())
    assert e64 <= 1e-9 and 1e-8 < e32 <= 1e-3


def test_rejections(torch_cuda):
    torch = torch_cuda
    g = geom(64, 64, 4)
    for bad in (g.with_(tv_fgp=True), g.with_(dual_bf16=True)):
        with pytest.raises(rihvr.RihvrError):
            rihvr.Plan(bad, dtype=rihvr.RI_F64)
    p = rihvr.Plan(g, dtype=rihvr.RI_F64)
    try:
        x = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
        b = torch.zeros((g.ny, g.nx), dtype=torch.float64, device="cuda")
        st = rihvr.ri_forward_noalloc(p.handle, x.data_ptr(), b.data_ptr(), torch.cuda.current_stream().cuda_stream)
        assert st == rihvr.RI_ERR_INVALID_ARG
        assert rihvr.ri_plan_set_storage(p.handle, 0.5) == rihvr.RI_ERR_INVALID_ARG
        with pytest.raises(rihvr.RihvrError):
            p.autotune(5)
        with pytest.raises(rihvr.RihvrError):
            p.solve(b, 0.1, 0.1, 3, 3, flags=rihvr.RI_SOLVE_DUAL_WARM)
        params = [p.solve_params(0.1, 0.1, 3, 3)]
        nbytes = rihvr.ri_workspace_size_batched(1, [p.handle], params)
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        st = rihvr.ri_solve_batched(1, [p.handle], params, [b.data_ptr()], [x.data_ptr()], ws.data_ptr(), nbytes,
                                    torch.cuda.current_stream().cuda_stream, None)
        assert st == rihvr.RI_ERR_INVALID_ARG
        with pytest.raises(ValueError):
            p.forward(torch.zeros(p.shape, dtype=torch.float32, device="cuda"))
    finally:
        p.close()

"""GPU parity of the HIP library against the FP64 oracle, through the C ABI.

Tolerances: A and A^T within relative L2 1e-5 of the FP64 oracle; the prox
within 1e-5; whole solves within 1e-3 (FP32 iterate against FP64 iterate after
the same number of outer / inner iterations) with detected particle centroids
within one voxel.  Sizes span several column tiles, several z-chunks and ragged
last tiles; full-size (1024^2 x 256) cases compare sampled outputs that the
oracle computes one by one (planes of A^T, crops of the prox).
"""
import math
import zlib

import numpy as np
import pytest

import oracle
from oracle import optics, prox, fista, detect
from paper_1904_04884_amd import rihvr, scenes

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def geom(nx, ny, nz, **kw):
    return scenes.geometry_c1().with_(nx=nx, ny=ny, nz=nz, **kw)


SHAPES = [(128, 128, 32), (48, 96, 5), (96, 48, 7), (64, 192, 3), (16, 16, 1), (256, 64, 9), (192, 24, 4),
          (32, 512, 3), (16, 1024, 2)]


@pytest.fixture(scope="module")
def plans(torch_cuda):
    cache = {}

    def get(g):
        key = g
        if key not in cache:
            cache[key] = rihvr.Plan(g)
        return cache[key]
    yield get
    for p in cache.values():
        p.close()


# ---------------------------------------------------------------------------
# Operators
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", SHAPES)
def test_lipschitz_matches_oracle(torch_cuda, plans, shape):
    g = geom(*shape)
    assert plans(g).lipschitz == pytest.approx(optics.lipschitz(g), rel=1e-12)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", ["random", "particles"])
def test_forward_parity(torch_cuda, plans, shape, kind):
    torch = torch_cuda
    g = geom(*shape)
    rng = np.random.default_rng(zlib.crc32(repr((shape, kind)).encode()))
    if kind == "random":
        x = rng.standard_normal(g.shape)
    else:
        idx, val, _ = scenes.gaussian_particles(g, max(1, g.nz), rng, radius=2, margin=2)
        x = scenes.densify(g.shape, idx, val)
    x32 = x.astype(np.float32)
    ref = optics.forward(g, x32.astype(np.float64))
    out = to_host(plans(g).forward(to_dev(torch, x32)))
    assert rel_l2(out, ref) <= 1e-5


@pytest.mark.parametrize("shape", SHAPES)
def test_adjoint_parity(torch_cuda, plans, shape):
    torch = torch_cuda
    g = geom(*shape)
    rng = np.random.default_rng(sum(shape))
    y = rng.standard_normal((g.ny, g.nx)).astype(np.float32)
    ref = optics.adjoint(g, y.astype(np.float64))
    out = to_host(plans(g).adjoint(to_dev(torch, y)))
    assert rel_l2(out, ref) <= 1e-5


def test_no_carrier_geometry(torch_cuda, plans):
    torch = torch_cuda
    g = geom(64, 64, 6, carrier=False)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(g.shape).astype(np.float32)
    y = rng.standard_normal((g.ny, g.nx)).astype(np.float32)
    assert rel_l2(to_host(plans(g).forward(to_dev(torch, x))), optics.forward(g, x.astype(np.float64))) <= 1e-5
    assert rel_l2(to_host(plans(g).adjoint(to_dev(torch, y))), optics.adjoint(g, y.astype(np.float64))) <= 1e-5


def test_zero_distance_is_identity(torch_cuda, plans):
    torch = torch_cuda
    g = geom(32, 16, 1, z0_um=0.0)
    rng = np.random.default_rng(6)
    x = rng.standard_normal(g.shape).astype(np.float32)
    out = to_host(plans(g).forward(to_dev(torch, x)))
    assert np.max(np.abs(out - x[0])) <= 1e-5


@pytest.mark.parametrize("shape", [(128, 128, 32), (96, 48, 7)])
def test_adjoint_identity_fp32(torch_cuda, plans, shape):
    torch = torch_cuda
    g = geom(*shape)
    rng = np.random.default_rng(7)
    x = to_dev(torch, rng.standard_normal(g.shape))
    y = to_dev(torch, rng.standard_normal((g.ny, g.nx)))
    p = plans(g)
    lhs = float((p.forward(x).double() * y.double()).sum())
    rhs = float((x.double() * p.adjoint(y).double()).sum())
    scale = float(torch.linalg.norm(p.forward(x).double()) * torch.linalg.norm(y.double()))
    assert abs(lhs - rhs) <= 1e-5 * scale


# ---------------------------------------------------------------------------
# Prox
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(64, 48, 12), (16, 16, 1), (128, 128, 32), (96, 24, 5)])
@pytest.mark.parametrize("nonneg", [True, False])
def test_prox_parity(torch_cuda, plans, shape, nonneg):
    torch = torch_cuda
    g = geom(*shape)
    rng = np.random.default_rng(8)
    v = (0.3 * rng.standard_normal(g.shape)).astype(np.float32)
    step, l1, tv, k = 0.7, 0.1, 0.2, 10
    ref = prox.prox_fused_lasso(v.astype(np.float64), step, l1, tv, k, nonneg)
    out = to_host(plans(g).prox(to_dev(torch, v), step, l1, tv, k, nonneg))
    assert rel_l2(out, ref) <= 1e-5


@pytest.mark.parametrize("k", [1, 3, 4, 5, 7, 8, 20])
def test_prox_pass_schedules(torch_cuda, plans, k):
    """Dual-step counts that split differently over fused passes, on a volume
    with several x / y tiles and z chunks."""
    torch = torch_cuda
    g = geom(192, 96, 40)
    rng = np.random.default_rng(100 + k)
    v = (0.3 * rng.standard_normal(g.shape)).astype(np.float32)
    step, l1, tv = 0.5, 0.05, 0.3
    ref = prox.prox_fused_lasso(v.astype(np.float64), step, l1, tv, k)
    out = to_host(plans(g).prox(to_dev(torch, v), step, l1, tv, k))
    assert rel_l2(out, ref) <= 1e-5


def test_prox_without_tv_is_exact_soft_threshold(torch_cuda, plans):
    torch = torch_cuda
    g = geom(64, 32, 5)
    rng = np.random.default_rng(9)
    v = rng.standard_normal(g.shape).astype(np.float32)
    step, l1 = 0.5, 0.3
    thr = np.float32(step * l1)
    out = plans(g).prox(to_dev(torch, v), step, l1, 0.0, 10).cpu().numpy()
    assert np.array_equal(out, np.maximum(v - thr, np.float32(0)))
    out = plans(g).prox(to_dev(torch, v), step, l1, 0.2, 0).cpu().numpy()   # zero inner steps
    assert np.array_equal(out, np.maximum(v - thr, np.float32(0)))


def test_prox_in_place(torch_cuda, plans):
    torch = torch_cuda
    g = geom(64, 48, 6)
    rng = np.random.default_rng(10)
    v = to_dev(torch, rng.standard_normal(g.shape))
    p = plans(g)
    a = p.prox(v, 0.5, 0.1, 0.1, 8)
    b = v.clone()
    p.prox(b, 0.5, 0.1, 0.1, 8, out=b)
    assert torch.equal(a, b)


def exact_tv1d(v, tau):
    """Exact 1D TV prox through its dual, the box-constrained least squares
    min_{|p_i| <= 1} 1/2 ||v - tau D^T p||^2 solved by bounded-variable least
    squares (an active-set method that terminates at the exact minimiser);
    enumerating the 3^(n-1) active sets is too slow at n = 16."""
    from scipy.optimize import lsq_linear
    n = len(v)
    D = np.zeros((n - 1, n))
    for i in range(n - 1):
        D[i, i], D[i, i + 1] = -1.0, 1.0
    p = lsq_linear(tau * D.T, v, bounds=(-1.0, 1.0), method="bvls", tol=1e-15).x
    return v - tau * D.T @ p


def test_prox_line_matches_brute_force_1d(torch_cuda, plans):
    """A 1 x 1 x n line along x: isotropic TV is 1D TV and the fused-lasso prox is
    exact; GP with many steps must approach the brute-force dual solution."""
    torch = torch_cuda
    from tests.test_oracle_pins import brute_tv1d
    n = 16
    g = geom(n, 16, 1)
    rng = np.random.default_rng(11)
    v = np.zeros(g.shape, np.float32)
    v[0, 3, :] = rng.standard_normal(n)
    tau, thr = 0.25, 0.05
    # rows other than y = 3 are zero; isotropic TV couples rows, so compare with
    # the oracle on the whole plane and with the brute force on a single row
    out = to_host(plans(g).prox(to_dev(torch, v), 1.0, thr, tau, 4000))
    ref = prox.prox_fused_lasso(v.astype(np.float64), 1.0, thr, tau, 4000)
    assert np.max(np.abs(out - ref)) <= 2e-5
    g1 = geom(16, 16, 1)
    line = np.zeros(g1.shape, np.float32)
    line[0, 0, :] = rng.standard_normal(n)
    line[0, 1:, :] = line[0, 0, :]  # constant along y: no y-differences
    out1 = to_host(plans(g1).prox(to_dev(torch, line), 1.0, thr, tau, 4000))
    exact = np.maximum(exact_tv1d(line[0, 0].astype(np.float64), tau) - thr, 0.0)
    assert np.max(np.abs(out1[0, 0] - exact)) <= 1e-4
    # the bounded least-squares dual agrees with the enumerated one on a short line
    w = rng.standard_normal(7)
    assert np.max(np.abs(exact_tv1d(w, tau) - brute_tv1d(w, tau))) <= 1e-12


# ---------------------------------------------------------------------------
# Solve
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1_problem():
    sc = scenes.scene_c1(seed=0)
    g, cfg = sc.geometry, sc.config
    b = (optics.forward(g, sc.dense()) + sc.noise).astype(np.float32)
    x_ref = fista.fista(g, b.astype(np.float64), cfg.l1, cfg.tv, cfg.outer_iters, cfg.inner_iters)
    return sc, b, x_ref


def test_solve_parity_c1(torch_cuda, plans, c1_problem):
    torch = torch_cuda
    sc, b, x_ref = c1_problem
    g, cfg = sc.geometry, sc.config
    x, rep, st = plans(g).solve(to_dev(torch, b), cfg.l1, cfg.tv, cfg.outer_iters, cfg.inner_iters)
    xg = to_host(x)
    assert rep["iters"] == cfg.outer_iters
    assert rel_l2(xg, x_ref) <= 1e-3
    F_ref = fista.objective(g, x_ref, b.astype(np.float64), cfg.l1, cfg.tv)
    assert rep["objective"] == pytest.approx(F_ref, rel=1e-4)
    # detected centroids agree within one voxel
    cg = detect.detect(xg)
    cr = detect.detect(x_ref)
    pairs, errs = detect.match(cg, cr, max_dist=1.0)
    assert len(pairs) >= 0.95 * max(len(cr), 1)
    assert len(cg) == pytest.approx(len(cr), abs=max(2, 0.05 * len(cr)))


def test_solve_graph_dense_and_timing_modes_agree(torch_cuda, plans, c1_problem):
    torch = torch_cuda
    sc, b, _ = c1_problem
    g, cfg = sc.geometry, sc.config
    p = plans(g)
    bd = to_dev(torch, b)
    xs = []
    for flags in (0, rihvr.RI_SOLVE_NO_GRAPH, rihvr.RI_SOLVE_DENSE, rihvr.RI_SOLVE_TIMING):
        x, rep, _ = p.solve(bd, cfg.l1, cfg.tv, 12, cfg.inner_iters, flags=flags)
        xs.append(x.clone())
    for x in xs[1:]:
        assert torch.equal(x, xs[0])
    assert rep["phase_launches"]["prox"] > 0 and rep["phase_ms"]["prox"] > 0


def test_solve_reduces_to_prox(torch_cuda, plans):
    torch = torch_cuda
    g = geom(64, 32, 1, z0_um=0.0)
    rng = np.random.default_rng(12)
    b = rng.standard_normal((g.ny, g.nx)).astype(np.float32)
    x, rep, _ = plans(g).solve(to_dev(torch, b), 0.2, 0.1, 1, 7)
    ref = prox.prox_fused_lasso(b.astype(np.float64).reshape(g.shape), 1.0, 0.2, 0.1, 7)
    assert rep["lipschitz"] == pytest.approx(1.0, abs=1e-12)
    assert np.max(np.abs(to_host(x) - ref)) <= 1e-5


def test_solve_warm_start_and_gap_stop(torch_cuda, plans, c1_problem):
    torch = torch_cuda
    sc, b, x_ref = c1_problem
    g, cfg = sc.geometry, sc.config
    p = plans(g)
    bd = to_dev(torch, b)
    # reference objective from a longer restarted run, then stop at a loose gap
    _, rep_long, _ = p.solve(bd, cfg.l1, cfg.tv, 300, cfg.inner_iters, flags=rihvr.RI_SOLVE_RESTART)
    f_ref = rep_long["objective"]
    _, rep, _ = p.solve(bd, cfg.l1, cfg.tv, 300, cfg.inner_iters, f_ref=f_ref, gap_tol=1e-2, check_every=5)
    assert rep["converged"] and rep["gap"] <= 1e-2 and rep["iters"] < 300
    # warm start from the oracle's answer: the objective starts near the reference
    x0 = to_dev(torch, x_ref)
    _, rep_w, _ = p.solve(bd, cfg.l1, cfg.tv, 0, cfg.inner_iters, x=x0)
    F_ref = fista.objective(g, x_ref, b.astype(np.float64), cfg.l1, cfg.tv)
    assert rep_w["iters"] == 0 and rep_w["objective"] == pytest.approx(F_ref, rel=1e-5)


def test_x0_scale_equals_scaled_start(torch_cuda, plans, c1_problem):
    """A given start scaled by the solve (x0_scale) equals the same start scaled
    beforehand (scaling by 2 is exact), and 0 reads as 1."""
    torch = torch_cuda
    sc, b, _ = c1_problem
    g, cfg = sc.geometry, sc.config
    p = plans(g)
    rng = np.random.default_rng(21)
    x0 = np.maximum(rng.standard_normal(g.shape), 0.0) * 0.01
    xa, ra, _ = p.solve(to_dev(torch, b), cfg.l1, cfg.tv, 6, cfg.inner_iters, x=to_dev(torch, x0), x0_scale=2.0)
    xb, rb, _ = p.solve(to_dev(torch, b), cfg.l1, cfg.tv, 6, cfg.inner_iters, x=to_dev(torch, 2.0 * x0))
    assert torch.equal(xa, xb) and ra["objective"] == rb["objective"]
    xc, _, _ = p.solve(to_dev(torch, b), cfg.l1, cfg.tv, 6, cfg.inner_iters, x=to_dev(torch, x0), x0_scale=0.0)
    xd, _, _ = p.solve(to_dev(torch, b), cfg.l1, cfg.tv, 6, cfg.inner_iters, x=to_dev(torch, x0))
    assert torch.equal(xc, xd)
    with pytest.raises(rihvr.RihvrError):
        p.solve(to_dev(torch, b), cfg.l1, cfg.tv, 6, cfg.inner_iters, x=to_dev(torch, x0), x0_scale=-1.0)


def test_scale_covariance(torch_cuda, plans, c1_problem):
    torch = torch_cuda
    sc, b, _ = c1_problem
    g, cfg = sc.geometry, sc.config
    p = plans(g)
    x1, _, _ = p.solve(to_dev(torch, b), cfg.l1, cfg.tv, 10, cfg.inner_iters)
    x2, _, _ = p.solve(to_dev(torch, 4.0 * b), 4.0 * cfg.l1, 4.0 * cfg.tv, 10, cfg.inner_iters)
    assert rel_l2(to_host(x2), 4.0 * to_host(x1)) <= 1e-5


@pytest.mark.parametrize("graph", [True, False])
def test_batched_matches_single(torch_cuda, plans, graph):
    """Uneven frames (sizes 2^a and 3*2^a, shared and distinct transform sizes,
    different plane counts and stop iterations) solved in one batch must equal
    the per-frame solves exactly."""
    torch = torch_cuda
    gs = [geom(64, 64, 8), geom(48, 96, 5), geom(128, 128, 12), geom(64, 64, 3), geom(96, 96, 7)]
    iters = [6, 4, 6, 9, 5]
    rng = np.random.default_rng(13)
    bs = [to_dev(torch, rng.standard_normal((g.ny, g.nx))) for g in gs]
    ps = [plans(g) for g in gs]
    singles = [p.solve(b, 0.05, 0.02, k, 4)[0].clone() for p, b, k in zip(ps, bs, iters)]
    flags = 0 if graph else rihvr.RI_SOLVE_NO_GRAPH
    params = [p.solve_params(0.05, 0.02, k, 4, flags=flags) for p, k in zip(ps, iters)]
    handles = [p.handle for p in ps]
    nbytes = rihvr.ri_workspace_size_batched(len(ps), handles, params)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    xs = [torch.empty(p.shape, dtype=torch.float32, device="cuda") for p in ps]
    reps = (rihvr.ri_solve_report * len(ps))()
    st = rihvr.ri_solve_batched(len(ps), handles, params, [b.data_ptr() for b in bs],
                                [x.data_ptr() for x in xs], ws.data_ptr(), ws.numel(),
                                torch.cuda.current_stream().cuda_stream, reps)
    assert st == rihvr.RI_OK, rihvr.ri_last_error()
    for a, sgl in zip(xs, singles):
        assert torch.equal(a, sgl)
    assert [r.iters for r in reps] == iters
    # too small a workspace is refused before anything runs
    assert rihvr.ri_solve_batched(len(ps), handles, params, [b.data_ptr() for b in bs],
                                  [x.data_ptr() for x in xs], ws.data_ptr(), nbytes - 1,
                                  torch.cuda.current_stream().cuda_stream, None) == rihvr.RI_ERR_WORKSPACE_TOO_SMALL


def test_batched_given_scaled_starts_match_single(torch_cuda, plans):
    """Frames started from given volumes scaled by the solve (x0_scale), mixed
    with cold frames, equal their per-frame solves exactly."""
    torch = torch_cuda
    gs = [geom(64, 64, 8), geom(48, 96, 5), geom(96, 96, 7)]
    scales = [0.5, 1.0, 3.0]
    rng = np.random.default_rng(15)
    bs = [to_dev(torch, rng.standard_normal((g.ny, g.nx))) for g in gs]
    x0s = [to_dev(torch, 0.01 * np.maximum(rng.standard_normal(g.shape), 0.0)) for g in gs]
    ps = [plans(g) for g in gs]
    given = [True, False, True]
    singles = [p.solve(b, 0.05, 0.02, 5, 4, x=x0.clone() if gv else None, x0_scale=sc)[0].clone()
               for p, b, x0, sc, gv in zip(ps, bs, x0s, scales, given)]
    params = [p.solve_params(0.05, 0.02, 5, 4, init=rihvr.RI_INIT_GIVEN if gv else rihvr.RI_INIT_ZERO,
                             x0_scale=sc) for p, sc, gv in zip(ps, scales, given)]
    handles = [p.handle for p in ps]
    ws = torch.empty(rihvr.ri_workspace_size_batched(len(ps), handles, params), dtype=torch.uint8, device="cuda")
    xs = [x0.clone() if gv else torch.empty(p.shape, dtype=torch.float32, device="cuda")
          for p, x0, gv in zip(ps, x0s, given)]
    st = rihvr.ri_solve_batched(len(ps), handles, params, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs],
                                ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream, None)
    assert st == rihvr.RI_OK, rihvr.ri_last_error()
    for a, sgl in zip(xs, singles):
        assert torch.equal(a, sgl)


def test_batched_gap_stop_per_frame(torch_cuda, plans):
    """Each frame stops at its own gap; finished frames do no further work."""
    torch = torch_cuda
    gs = [geom(64, 64, 6), geom(96, 48, 4)]
    rng = np.random.default_rng(14)
    bs = [to_dev(torch, rng.standard_normal((g.ny, g.nx))) for g in gs]
    ps = [plans(g) for g in gs]
    refs = [p.solve(b, 0.05, 0.02, 200, 4, flags=rihvr.RI_SOLVE_RESTART)[1]["objective_min"] for p, b in zip(ps, bs)]
    params = [p.solve_params(0.05, 0.02, 200, 4, gap_tol=tol, f_ref=f, check_every=3)
              for p, f, tol in zip(ps, refs, (1e-2, 1e-3))]
    single = [p.solve(b, 0.05, 0.02, 200, 4, gap_tol=tol, f_ref=f, check_every=3)
              for p, b, f, tol in zip(ps, bs, refs, (1e-2, 1e-3))]
    handles = [p.handle for p in ps]
    nbytes = rihvr.ri_workspace_size_batched(len(ps), handles, params)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    xs = [torch.empty(p.shape, dtype=torch.float32, device="cuda") for p in ps]
    reps = (rihvr.ri_solve_report * len(ps))()
    st = rihvr.ri_solve_batched(len(ps), handles, params, [b.data_ptr() for b in bs],
                                [x.data_ptr() for x in xs], ws.data_ptr(), ws.numel(),
                                torch.cuda.current_stream().cuda_stream, reps)
    assert st == rihvr.RI_OK
    for r, (x1, rep1, _), x in zip(reps, single, xs):
        assert r.converged == 1 and r.iters == rep1["iters"]
        assert torch.equal(x, x1)


# ---------------------------------------------------------------------------
# Error paths (forced from the host)
# ---------------------------------------------------------------------------
def test_error_paths(torch_cuda, plans):
    torch = torch_cuda
    g = geom(32, 32, 4)
    p = plans(g)
    x = torch.zeros(p.shape, dtype=torch.float32, device="cuda")
    b = torch.zeros((g.ny, g.nx), dtype=torch.float32, device="cuda")
    n = rihvr.ri_workspace_size_op(p.handle, rihvr.RI_OP_FORWARD)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert rihvr.ri_forward(p.handle, x.data_ptr(), b.data_ptr(), ws.data_ptr(), n - 1, s) == \
        rihvr.RI_ERR_WORKSPACE_TOO_SMALL
    assert rihvr.ri_forward(p.handle, x.data_ptr() + 4, b.data_ptr(), ws.data_ptr(), n, s) == rihvr.RI_ERR_INVALID_ARG
    assert rihvr.ri_forward(p.handle, ws.data_ptr(), b.data_ptr(), ws.data_ptr(), n, s) == rihvr.RI_ERR_INVALID_ARG
    # non-finite hologram -> the solve stops with RI_ERR_NONFINITE
    bn = b.clone()
    bn[3, 5] = float("nan")
    _, rep, st = p.solve(bn, 0.1, 0.1, 5, 3, raise_on_error=False)
    assert st == rihvr.RI_ERR_NONFINITE
    assert rep["iters"] == 0
    with pytest.raises(ValueError):
        p.forward(x.double())


# ---------------------------------------------------------------------------
# Full size (1024^2 x 256, the benchmarked launch configuration)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c2(torch_cuda):
    g = scenes.geometry_c2()
    p = rihvr.Plan(g)
    yield g, p
    p.close()


def test_c2_lipschitz(c2):
    # the phase 2 pi z sqrt(1/lambda^2 - f^2) reaches 2e5 rad here, so the
    # oracle's own FP64 argument carries ~2e-11 rad of rounding
    g, p = c2
    assert p.lipschitz == pytest.approx(optics.lipschitz(g), rel=1e-10)


def test_c2_forward_sparse_planes(torch_cuda, c2):
    torch = torch_cuda
    g, p = c2
    rng = np.random.default_rng(20)
    planes = [0, 37, 128, 255]
    x = np.zeros(g.shape, np.float32)
    sub = g.with_(nz=1)
    for j in planes:
        idx, val, _, _ = scenes.disk_particles(sub, 30, rng)
        x[j][idx[:, 1], idx[:, 2]] = val
    ref = np.zeros((g.ny, g.nx))
    for j in planes:
        gj = g.with_(nz=1, z0_um=g.z0_um + j * g.dz_um)
        ref += optics.forward(gj, x[j:j + 1].astype(np.float64))
    out = to_host(p.forward(to_dev(torch, x)))
    assert rel_l2(out, ref) <= 1e-5


def test_c2_adjoint_sampled_planes(torch_cuda, c2):
    torch = torch_cuda
    g, p = c2
    rng = np.random.default_rng(21)
    y = rng.standard_normal((g.ny, g.nx)).astype(np.float32)
    out = p.adjoint(to_dev(torch, y))
    for j in (0, 101, 255):
        gj = g.with_(nz=1, z0_um=g.z0_um + j * g.dz_um)
        ref = optics.adjoint(gj, y.astype(np.float64))[0]
        assert rel_l2(to_host(out[j]), ref) <= 1e-5


def _crop_prox_check(out, v, step, l1, tv, k, blocks):
    m = k + 2
    for (z0, y0, x0, bs) in blocks:
        lo = [max(0, c - m) for c in (z0, y0, x0)]
        hi = [min(n, c + bs + m) for c, n in zip((z0, y0, x0), v.shape)]
        crop = v[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].astype(np.float64)
        ref = prox.prox_fused_lasso(crop, step, l1, tv, k)
        sl = tuple(slice(c - l, c - l + bs) for c, l in zip((z0, y0, x0), lo))
        got = out[z0:z0 + bs, y0:y0 + bs, x0:x0 + bs]
        assert rel_l2(got, ref[sl]) <= 1e-5


def test_c2_prox_sampled_blocks(torch_cuda, c2):
    torch = torch_cuda
    g, p = c2
    rng = np.random.default_rng(22)
    v = (0.01 * rng.standard_normal(g.shape, dtype=np.float32))
    cfg = scenes.config_c2()
    step = 1.0 / p.lipschitz
    out = p.prox(to_dev(torch, v), step * 50, cfg.l1, cfg.tv, cfg.inner_iters).cpu().numpy()
    blocks = [(0, 0, 0, 16), (120, 500, 700, 16), (240, 1008, 1008, 16), (60, 0, 333, 16)]
    _crop_prox_check(out, v, step * 50, cfg.l1, cfg.tv, cfg.inner_iters, blocks)


def test_c2_first_iteration_sampled(torch_cuda, c2):
    """One full solver iteration at 1024^2 x 256: x_1 = prox(t A^T b), on crops."""
    torch = torch_cuda
    g, p = c2
    cfg = scenes.config_c2()
    rng = np.random.default_rng(23)
    x_true = np.zeros(g.shape)
    sub = g.with_(nz=1)
    for j in (40, 45, 52):
        idx, val, _, _ = scenes.disk_particles(sub, 40, rng)
        x_true[j][idx[:, 1], idx[:, 2]] = val
    b = np.zeros((g.ny, g.nx))
    for j in (40, 45, 52):
        gj = g.with_(nz=1, z0_um=g.z0_um + j * g.dz_um)
        b += optics.forward(gj, x_true[j:j + 1])
    b = (b + cfg.noise_sigma * rng.standard_normal(b.shape)).astype(np.float32)
    x1, rep, _ = p.solve(to_dev(torch, b), cfg.l1, cfg.tv, 1, cfg.inner_iters)
    x1 = x1.cpu().numpy()
    assert rep["iters"] == 1
    t = 1.0 / optics.lipschitz(g)
    k = cfg.inner_iters
    m = k + 2
    z0, z1 = 30, 30 + 16  # planes [30, 46) plus margins
    lo, hi = max(0, z0 - m), min(g.nz, z1 + m)
    v = np.empty((hi - lo, g.ny, g.nx))
    for jj, j in enumerate(range(lo, hi)):
        gj = g.with_(nz=1, z0_um=g.z0_um + j * g.dz_um)
        v[jj] = t * optics.adjoint(gj, b.astype(np.float64))[0]
    for (y0, x0) in ((480, 480), (0, 1000)):
        ylo, yhi = max(0, y0 - m), min(g.ny, y0 + 24 + m)
        xlo, xhi = max(0, x0 - m), min(g.nx, x0 + 24 + m)
        ref = prox.prox_fused_lasso(v[:, ylo:yhi, xlo:xhi], t, cfg.l1, cfg.tv, k)
        got = x1[z0:z1, y0:y0 + 24, x0:x0 + 24]
        exp = ref[z0 - lo:z1 - lo, y0 - ylo:y0 - ylo + 24, x0 - xlo:x0 - xlo + 24]
        assert rel_l2(got, exp) <= 1e-4 or np.max(np.abs(got - exp)) <= 1e-6

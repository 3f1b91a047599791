"""Row-compressed storage of the solver's iterates (ri_plan_set_storage).

The paper keeps the sparse particle volume in a compressed form to fit large
volumes (section "Methodology", the storage paragraph).  Here x_k, x_{k-1} and
x_{k+1} live in row stores (a pool of rows of nx values and a slot table); an
absent row is all zero.  The values are those of the dense storage, so the bar
is bit-identity with the dense HIP path, which the solver parity tests tie to
the FP64 oracle; each case also checks the oracle directly at the solver bar
(1e-3 relative L2 on the iterate, 1e-4 on the objective).
"""
import math

import numpy as np
import pytest

from oracle import optics, fista
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


# A sparse regime: the C1 optics at 128x128x32 with a strong l1 weight, whose
# iterates leave 40-80 % of the rows empty (the occupancy is highest at x_1).
L1, TV, ITERS, K_IN = 0.1, 0.005, 20, 5


@pytest.fixture(scope="module")
def sparse_problem():
    sc = scenes.scene_c1(seed=6)
    g = sc.geometry
    b = (optics.forward(g, sc.dense()) + sc.noise).astype(np.float32)
    return g, b


def oracle_run(g, b, iters=ITERS, **kw):
    """The oracle's iterate and the largest fraction of occupied rows over its
    iterates."""
    occ = []
    x = fista.fista(g, b.astype(np.float64), L1, TV, iters, K_IN,
                    on_iterate=lambda xi: occ.append(float((xi.reshape(-1, g.nx) != 0).any(axis=1).mean())), **kw)
    return x, occ


def solve_both(torch, g, b, iters, frac, tuning=None, x0=None, **kw):
    """Dense and row-store solves of the same problem on two plans."""
    out = []
    for f in (0.0, frac):
        p = rihvr.Plan(g)
        try:
            if tuning is not None:
                p.tuning = tuning
            p.row_fraction = f
            x = None if x0 is None else to_dev(torch, x0)
            x, rep, st = p.solve(to_dev(torch, b), L1, TV, iters, K_IN, x=x, raise_on_error=False, **kw)
            rep["status"] = st
            out.append((to_host(x), rep))
        finally:
            p.close()
    return out


@pytest.mark.parametrize("tv_dims", [3, 2])
@pytest.mark.parametrize("margin", [None, 0.05])
def test_row_store_solve_equals_dense(torch_cuda, sparse_problem, tv_dims, margin):
    torch = torch_cuda
    g, b = sparse_problem
    g = g.with_(tv_dims=tv_dims)
    ref, occ = oracle_run(g, b, tv_dims=tv_dims)
    assert max(occ) < 0.9 and occ[-1] < 0.5      # the regime is row-sparse
    frac = 1.0 if margin is None else max(occ) + margin
    (xd, rd), (xs, rs) = solve_both(torch, g, b, ITERS, frac)
    assert rd["status"] == rihvr.RI_OK and rs["status"] == rihvr.RI_OK
    assert rs["iters"] == rd["iters"] == ITERS
    assert np.array_equal(xs, xd)
    assert rs["objective"] == rd["objective"]
    assert rel_l2(xs, ref) <= 1e-3
    F = fista.objective(g, ref, b.astype(np.float64), L1, TV, tv_dims=tv_dims)
    assert rs["objective"] == pytest.approx(F, rel=1e-4)


@pytest.mark.parametrize("levels,flags", [(4, rihvr.RI_SOLVE_DUAL_WARM), (3, rihvr.RI_SOLVE_RESTART),
                                          (2, rihvr.RI_SOLVE_NO_GRAPH), (4, rihvr.RI_SOLVE_TIMING)])
def test_row_store_with_tunings_and_modes(torch_cuda, sparse_problem, levels, flags):
    torch = torch_cuda
    g, b = sparse_problem
    tuning = {"tv_levels": levels, "tv_blocks": 1536, "col_blocks": 512}
    (xd, rd), (xs, rs) = solve_both(torch, g, b, 12, 0.9, tuning, flags=flags)
    assert rd["status"] == rihvr.RI_OK and rs["status"] == rihvr.RI_OK
    assert rs["iters"] == rd["iters"]
    assert np.array_equal(xs, xd)
    assert rs["objective"] == rd["objective"]


def test_row_store_given_start(torch_cuda, sparse_problem):
    """A given x_0 with empty rows (an oracle iterate with half of its planes
    and every third row cleared, scaled by x0_scale): its occupied rows go to
    the stores, the rest start absent."""
    torch = torch_cuda
    g, b = sparse_problem
    x0, _ = oracle_run(g, b, iters=4)
    x0 = x0.astype(np.float32)
    x0[g.nz // 2:] = 0.0
    x0[:, ::3, :] = 0.0
    (xd, rd), (xs, rs) = solve_both(torch, g, b, 10, 0.95, x0=x0, x0_scale=0.5)
    assert rd["status"] == rihvr.RI_OK and rs["status"] == rihvr.RI_OK
    assert np.array_equal(xs, xd)
    ref, _ = oracle_run(g, b, iters=10, x0=0.5 * x0.astype(np.float64))
    assert rel_l2(xs, ref) <= 1e-3


def test_row_store_overflow_is_reported(torch_cuda, sparse_problem):
    """x_1 of the oracle occupies more rows than a pool of half its occupancy
    holds: the solve stops at iteration 1 with RI_ERR_WORKSPACE_TOO_SMALL; a
    given start with every row occupied overflows at iteration 0; the same
    plan then solves normally with room for every row."""
    torch = torch_cuda
    g, b = sparse_problem
    _, occ = oracle_run(g, b, iters=2)
    rows = g.ny * g.nz
    p = rihvr.Plan(g)
    try:
        p.row_fraction = occ[0] / 2
        _, rep, st = p.solve(to_dev(torch, b), L1, TV, 5, K_IN, raise_on_error=False)
        assert st == rihvr.RI_ERR_WORKSPACE_TOO_SMALL and rep["iters"] == 1
        p.row_fraction = 1.0 / rows            # a pool of one row
        x0 = 1e-3 + np.random.default_rng(1).random(g.shape).astype(np.float32) * 1e-3
        _, rep, st = p.solve(to_dev(torch, b), L1, TV, 5, K_IN, x=to_dev(torch, x0), raise_on_error=False)
        assert st == rihvr.RI_ERR_WORKSPACE_TOO_SMALL and rep["iters"] == 0
        p.row_fraction = 1.0
        x, rep, st = p.solve(to_dev(torch, b), L1, TV, 5, K_IN, x=to_dev(torch, x0))
        assert st == rihvr.RI_OK
        q = rihvr.Plan(g)
        try:
            xd, _, _ = q.solve(to_dev(torch, b), L1, TV, 5, K_IN, x=to_dev(torch, x0))
        finally:
            q.close()
        assert torch.equal(x, xd)
    finally:
        p.close()


def test_row_store_settings(torch_cuda):
    g = scenes.geometry_c1().with_(nx=256, ny=256, nz=64)
    p = rihvr.Plan(g)
    try:
        assert p.row_fraction == 0.0
        dense = rihvr.ri_workspace_size_op(p.handle, rihvr.RI_OP_SOLVE)
        for bad in (-0.1, 1.5, float("nan")):
            assert rihvr.ri_plan_set_storage(p.handle, bad) == rihvr.RI_ERR_INVALID_ARG
        assert p.row_fraction == 0.0
        p.row_fraction = 0.1
        small = rihvr.ri_workspace_size_op(p.handle, rihvr.RI_OP_SOLVE)
        vol = 256 * 256 * 64 * 4
        rows = 256 * 64
        cap = math.ceil(0.1 * rows)
        # two dense iterate volumes become two pools and two slot tables (plus
        # the buffers' alignment and stagger, under 16 * 37 * 256 bytes each)
        assert dense - small >= 2 * vol - 2 * cap * 256 * 4 - 2 * rows * 4 - 6 * 16 * 37 * 256
        assert small < dense - vol
        # prox and forward are unaffected
        q = rihvr.Plan(g)
        try:
            for op in (rihvr.RI_OP_PROX, rihvr.RI_OP_FORWARD, rihvr.RI_OP_AUTOTUNE):
                assert rihvr.ri_workspace_size_op(p.handle, op) == rihvr.ri_workspace_size_op(q.handle, op)
        finally:
            q.close()
        p.row_fraction = 0.0
        assert rihvr.ri_workspace_size_op(p.handle, rihvr.RI_OP_SOLVE) == dense
    finally:
        p.close()


def test_row_store_rejects_bf16_dual(torch_cuda, sparse_problem):
    torch = torch_cuda
    g, b = sparse_problem
    g = g.with_(dual_bf16=True)
    p = rihvr.Plan(g)
    try:
        p.row_fraction = 0.5
        _, _, st = p.solve(to_dev(torch, b), L1, TV, 3, 4, raise_on_error=False, report=False)
        assert st == rihvr.RI_ERR_INVALID_ARG
    finally:
        p.close()


def test_row_store_batched_mix(torch_cuda):
    """Batched frames with dense and row-store iterates, 3D and 2D TV: each
    frame equal to its dense single-frame solve, bit for bit."""
    torch = torch_cuda
    base = scenes.geometry_c1()
    gs = [base.with_(nx=64, ny=64, nz=6), base.with_(nx=64, ny=64, nz=6, tv_dims=2),
          base.with_(nx=96, ny=48, nz=5), base.with_(nx=48, ny=48, nz=7)]
    l1, tv, iters, k_in = 0.03, 0.02, 6, 5
    rng = np.random.default_rng(79)
    bs = [(0.05 * rng.standard_normal((g.ny, g.nx))).astype(np.float32) for g in gs]
    refs, fracs = [], []
    for i, (g, b) in enumerate(zip(gs, bs)):
        occ = []
        refs.append(fista.fista(g, b.astype(np.float64), l1, tv, iters, k_in, tv_dims=g.tv_dims,
                                on_iterate=lambda xi: occ.append((xi.reshape(-1, g.nx) != 0).any(axis=1).mean())))
        # frames 0, 1: pools just above the oracle's peak occupancy; 2: dense; 3: every row
        fracs.append(min(1.0, max(occ) + 0.05) if i < 2 else (0.0 if i == 2 else 1.0))
    singles = []
    for g, b in zip(gs, bs):
        q = rihvr.Plan(g)
        try:
            singles.append(to_host(q.solve(to_dev(torch, b), l1, tv, iters, k_in)[0]))
        finally:
            q.close()
    ps = [rihvr.Plan(g) for g in gs]
    try:
        for p, f in zip(ps, fracs):
            p.row_fraction = f
        params = [p.solve_params(l1, tv, iters, k_in) for p in ps]
        nbytes = rihvr.ri_workspace_size_batched(len(ps), [p.handle for p in ps], params)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        bd = [to_dev(torch, b) for b in bs]
        xs = [torch.empty(p.shape, dtype=torch.float32, device="cuda") for p in ps]
        st = rihvr.ri_solve_batched(len(ps), [p.handle for p in ps], params, [b.data_ptr() for b in bd],
                                    [x.data_ptr() for x in xs], ws.data_ptr(), nbytes,
                                    torch.cuda.current_stream().cuda_stream, None)
        assert st == rihvr.RI_OK, rihvr.ri_last_error()
        torch.cuda.synchronize()
        assert fracs[0] < 1.0 and fracs[1] < 1.0       # the first two frames are row-sparse
        for g, x, s1, ref in zip(gs, xs, singles, refs):
            assert np.array_equal(to_host(x), s1), g
            assert rel_l2(s1, ref) <= 1e-3, g
    finally:
        for p in ps:
            p.close()


def test_row_store_full_size(torch_cuda):
    """1024^2 x 256 benchmark volume with the benchmark tuning: the first
    outer iterations in row stores as large as the most occupied iterate needs
    (from a first row-store solve's peak) equal to the dense solve bit for
    bit; one row fewer overflows."""
    torch = torch_cuda
    g, cfg = scenes.geometry_c2(), scenes.config_c2()
    sc = scenes.scene_c2(seed=0)
    lin = np.ravel_multi_index((sc.idx[:, 0], sc.idx[:, 1], sc.idx[:, 2]), g.shape)
    rows = g.ny * g.nz
    tuning = {"tv_levels": 4, "tv_blocks": 256, "col_blocks": 512}
    p = rihvr.Plan(g)
    try:
        xt = torch.zeros(g.shape, dtype=torch.float32, device="cuda")
        xt.view(-1)[torch.from_numpy(lin).cuda()] = torch.from_numpy(sc.val.astype(np.float32)).cuda()
        b = (p.forward(xt) + to_dev(torch, sc.noise)).contiguous()
        del xt
        p.tuning = tuning
        iters = 6
        xd, rd, _ = p.solve(b, cfg.l1, cfg.tv, iters, cfg.inner_iters)
        xd = xd.clone()
        assert rd["store_rows_peak"] == 0
        p.row_fraction = 1.0
        x1, r1, _ = p.solve(b, cfg.l1, cfg.tv, iters, cfg.inner_iters)
        assert torch.equal(x1, xd) and r1["objective"] == rd["objective"]
        peak = r1["store_rows_peak"]
        print(f"peak occupied rows over {iters} iterations: {peak} of {rows} ({peak / rows:.3f}); "
              f"last iterate empty rows {rd['empty_row_frac']:.3f}", flush=True)
        assert peak >= round((1.0 - rd["empty_row_frac"]) * rows)
        del x1
        p.row_fraction = peak / rows
        assert p.row_fraction * rows <= peak + 1e-6
        x2, r2, st = p.solve(b, cfg.l1, cfg.tv, iters, cfg.inner_iters)
        assert st == rihvr.RI_OK and torch.equal(x2, xd) and r2["store_rows_peak"] == peak
        del x2
        if peak > 1:
            p.row_fraction = (peak - 1) / rows
            _, r3, st = p.solve(b, cfg.l1, cfg.tv, iters, cfg.inner_iters, raise_on_error=False)
            assert st == rihvr.RI_ERR_WORKSPACE_TOO_SMALL and r3["store_rows_peak"] >= peak
    finally:
        p.close()

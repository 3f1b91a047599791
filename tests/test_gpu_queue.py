"""Persistent TV passes fed by a device work queue (the default of a batched
solve) against the grouped launch of one block per tile (RI_SOLVE_GROUPED).

The work items of a pass are independent and each is run whole by one block,
so the two forms must give the same bits: every frame's final iterate, its
iteration count and its objective.  The batches mix every TV kernel variant
(3D at fusion depths 2, 3 and 4, per-plane 2D, accelerated dual, bfloat16
dual, row-compressed iterates), run with and without the iteration graph
(the graph replays every pass once per outer iteration, so the claim counters
must come back to zero after each launch), with more items than the
persistent grid has blocks and with fewer, and with frames that stop early.
"""
import numpy as np
import pytest

from paper_1904_04884_amd import rihvr, scenes

pytestmark = pytest.mark.gpu


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def run_batch(torch, ps, bs, params):
    handles = [p.handle for p in ps]
    nbytes = rihvr.ri_workspace_size_batched(len(ps), handles, params)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    xs = [torch.empty(p.shape, dtype=torch.float32, device="cuda") for p in ps]
    reps = (rihvr.ri_solve_report * len(ps))()
    st = rihvr.ri_solve_batched(len(ps), handles, params, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs],
                                ws.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream, reps)
    assert st == rihvr.RI_OK, rihvr.ri_last_error()
    torch.cuda.synchronize()
    return xs, [(r.iters, r.objective, r.converged) for r in reps]


def compare(torch, ps, bs, make_params):
    xa, ra = run_batch(torch, ps, bs, make_params(rihvr.RI_SOLVE_GROUPED))
    xb, rb = run_batch(torch, ps, bs, make_params(0))
    for p, a, b in zip(ps, xa, xb):
        assert torch.equal(a, b), p.geom
        assert bool((a != 0).any())
    assert ra == rb
    return ra


@pytest.fixture
def plans():
    made = []

    def make(g, row_fraction=None, **tuning):
        p = rihvr.Plan(g)
        made.append(p)
        if tuning:
            t = p.tuning
            t.update(tuning)
            p.tuning = t
        if row_fraction is not None:
            p.row_fraction = row_fraction
        return p
    yield make
    for p in made:
        p.close()


@pytest.mark.parametrize("graph", [True, False])
def test_every_variant_matches_grouped(torch_cuda, plans, graph):
    torch = torch_cuda
    base = scenes.geometry_c1()
    ps = [plans(base.with_(nx=64, ny=64, nz=8), tv_levels=2, tv_blocks=64),
          plans(base.with_(nx=48, ny=96, nz=5), tv_levels=3),
          plans(base.with_(nx=128, ny=128, nz=20), tv_levels=4, tv_blocks=6144),
          plans(base.with_(nx=64, ny=64, nz=6, tv_dims=2)),
          plans(base.with_(nx=64, ny=64, nz=6, tv_fgp=True)),
          plans(base.with_(nx=64, ny=48, nz=6, dual_bf16=True)),
          plans(base.with_(nx=96, ny=48, nz=5, tv_dims=2, tv_fgp=True, dual_bf16=True)),
          plans(base.with_(nx=96, ny=96, nz=7), row_fraction=1.0)]
    iters = [6, 4, 6, 5, 6, 5, 4, 6]
    rng = np.random.default_rng(91)
    bs = [to_dev(torch, 0.05 * rng.standard_normal((p.geom.ny, p.geom.nx))) for p in ps]
    flags = 0 if graph else rihvr.RI_SOLVE_NO_GRAPH
    reps = compare(torch, ps, bs, lambda f: [p.solve_params(0.02, 0.02, k, 5, flags=flags | f)
                                            for p, k in zip(ps, iters)])
    assert [r[0] for r in reps] == iters


def test_more_items_than_blocks(torch_cuda, plans):
    """Passes of several thousand items over one block per compute unit, and a
    single frame (the whole queue from one frame's tiles)."""
    torch = torch_cuda
    base = scenes.geometry_c1()
    ps = [plans(base.with_(nx=384, ny=384, nz=48), tv_levels=4, tv_blocks=4096),
          plans(base.with_(nx=256, ny=192, nz=40), tv_levels=2, tv_blocks=2048)]
    rng = np.random.default_rng(92)
    bs = [to_dev(torch, 0.05 * rng.standard_normal((p.geom.ny, p.geom.nx))) for p in ps]
    compare(torch, ps, bs, lambda f: [p.solve_params(0.02, 0.02, 5, 8, flags=f) for p in ps])
    compare(torch, ps[:1], bs[:1], lambda f: [ps[0].solve_params(0.02, 0.02, 4, 8, flags=f)])


def test_frames_that_stop_early(torch_cuda, plans):
    """Frames stopped by their gap leave their items in the queue; the blocks
    that claim them return at once."""
    torch = torch_cuda
    base = scenes.geometry_c1()
    ps = [plans(base.with_(nx=64, ny=64, nz=6)), plans(base.with_(nx=96, ny=48, nz=4))]
    rng = np.random.default_rng(93)
    bs = [to_dev(torch, rng.standard_normal((p.geom.ny, p.geom.nx))) for p in ps]
    refs = [p.solve(b, 0.05, 0.02, 200, 4, flags=rihvr.RI_SOLVE_RESTART)[1]["objective_min"] for p, b in zip(ps, bs)]
    reps = compare(torch, ps, bs, lambda f: [p.solve_params(0.05, 0.02, 200, 4, gap_tol=tol, f_ref=fr,
                                                            check_every=3, flags=f)
                                            for p, fr, tol in zip(ps, refs, (1e-2, 1e-3))])
    assert all(r[2] == 1 for r in reps) and reps[0][0] != reps[1][0]

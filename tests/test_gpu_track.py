"""Particle tracking back end on the GPU (ri_detect, ri_link, ri_track_update,
ri_track_filter) against the oracle's detect.objects / link / track.

Bars: object tables identical in count, order, voxel count and first index
(integer work), centroids and intensity sums within 1e-12 relative (FP64
sums in another order); links and track ids identical (the enumeration order
and the rounded FP64 distances decide equal costs the same way on both sides).
"""
import numpy as np
import pytest

from oracle import detect, optics, fista
from paper_1904_04884_amd import rihvr, scenes

pytestmark = pytest.mark.gpu


def gpu_objects(torch, x, rel=1.0 / 256.0, min_voxels=5, max_objects=65536, max_components=1 << 20):
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    objs, counts = rihvr.detect(xd, rel, min_voxels, max_objects, max_components)
    c = counts.cpu().numpy()
    return objs[: min(int(c[0]), max_objects)].cpu().numpy(), int(c[0]), int(c[1])


def blob_volume(shape, n, seed, radius=2.0):
    """Gaussian blobs at random centres (some overlap, some touch corners)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    x = np.zeros(shape, np.float32)
    zz, yy, xx = np.mgrid[0:nz, 0:ny, 0:nx]
    for _ in range(n):
        c = rng.uniform([0, 0, 0], [nz, ny, nx])
        a = rng.uniform(0.2, 1.0)
        r = rng.uniform(0.6, radius)
        x += (a * np.exp(-((zz - c[0]) ** 2 + (yy - c[1]) ** 2 + (xx - c[2]) ** 2) / (2 * r * r))).astype(np.float32)
    x[x < 1e-3] = 0.0
    return x


def compare_tables(got, ref):
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.array_equal(got[:, 4], ref[:, 4]) and np.array_equal(got[:, 5], ref[:, 5])
    np.testing.assert_allclose(got[:, :4], ref[:, :4], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("shape,n,seed", [((8, 16, 16), 6, 0), ((30, 80, 96), 120, 1), ((5, 300, 64), 90, 2),
                                          ((64, 64, 64), 400, 3)])
@pytest.mark.parametrize("rel", [1.0 / 256.0, 2.0 / 256.0, 0.05])
def test_detect_matches_oracle(torch_cuda, shape, n, seed, rel):
    torch = torch_cuda
    x = blob_volume(shape, n, seed)
    ref, ncomp = detect.objects(x.astype(np.float64), rel, 5)
    got, kept, comps = gpu_objects(torch, x, rel, 5)
    assert comps == ncomp and kept == len(ref)
    compare_tables(got, ref)


def test_detect_hand_cases(torch_cuda):
    torch = torch_cuda
    x = np.zeros((6, 6, 7), np.float32)
    x[2, 2, 1:5] = 1.0
    x[3, 3, 5] = 1.0            # corner neighbour: one 5-voxel object under 26-connectivity
    got, kept, comps = gpu_objects(torch, x)
    assert (kept, comps) == (1, 1)
    np.testing.assert_allclose(got[0], [11 / 5, 11 / 5, 3.0, 5.0, 5.0, 2 * 42 + 2 * 7 + 1], rtol=0, atol=1e-15)
    # nothing above zero: no object; a single voxel: one component, no object
    assert gpu_objects(torch, np.zeros((4, 4, 4), np.float32))[1:] == (0, 0)
    y = np.zeros((4, 4, 4), np.float32)
    y[1, 2, 3] = 3.0
    assert gpu_objects(torch, y)[1:] == (0, 1)


def test_detect_capacity_limits_report_true_counts(torch_cuda):
    torch = torch_cuda
    x = blob_volume((30, 80, 96), 120, 1)
    ref, ncomp = detect.objects(x.astype(np.float64), 1.0 / 256.0, 5)
    got, kept, comps = gpu_objects(torch, x, max_objects=10)
    assert kept == len(ref) and comps == ncomp and got.shape[0] == 10
    compare_tables(got, ref[:10])
    # components beyond the capacity are not summed; the count still tells
    got, kept, comps = gpu_objects(torch, x, max_components=ncomp - 3)
    assert comps == ncomp


def test_detect_full_size_sparse_volume(torch_cuda):
    """1024^2 x 256 volume holding the 2000 disk particles of the benchmark
    scene: the object table against the oracle."""
    torch = torch_cuda
    g = scenes.geometry_c2()
    sc = scenes.scene_c2(seed=0)
    x = np.zeros(g.shape, np.float32)
    x[sc.idx[:, 0], sc.idx[:, 1], sc.idx[:, 2]] = sc.val.astype(np.float32)
    ref, ncomp = detect.objects(x.astype(np.float64), 1.0 / 256.0, 5)
    got, kept, comps = gpu_objects(torch, x)
    assert comps == ncomp and kept == len(ref) and kept > 1000
    compare_tables(got, ref)


def test_detect_on_a_solved_volume(torch_cuda):
    torch = torch_cuda
    sc = scenes.scene_c1(seed=1)
    g, cfg = sc.geometry, sc.config
    b = (optics.forward(g, sc.dense()) + sc.noise).astype(np.float32)
    p = rihvr.Plan(g)
    try:
        x, _, _ = p.solve(torch.from_numpy(b).cuda(), cfg.l1, cfg.tv, cfg.outer_iters, cfg.inner_iters)
        xs = x.cpu().numpy()
    finally:
        p.close()
    for rel in (1.0 / 256.0, 2.0 / 256.0):
        ref, ncomp = detect.objects(xs.astype(np.float64), rel, 5)
        got, kept, comps = gpu_objects(torch, xs, rel)
        assert comps == ncomp and kept == len(ref)
        compare_tables(got, ref)


def table(pos):
    """Object rows (z, y, x, 1, 1, i) for positions."""
    t = np.zeros((len(pos), 6))
    t[:, :3] = pos
    t[:, 3] = t[:, 4] = 1.0
    t[:, 5] = np.arange(len(pos))
    return t


def gpu_link(torch, prev, cur, max_disp, spacing=(1.0, 1.0, 1.0), cap=None):
    cap0 = cap or max(len(prev), 1)
    cap1 = cap or max(len(cur), 1)
    P = torch.zeros((cap0, 6), dtype=torch.float64, device="cuda")
    Q = torch.zeros((cap1, 6), dtype=torch.float64, device="cuda")
    P[: len(prev)] = torch.from_numpy(table(prev)).cuda()
    Q[: len(cur)] = torch.from_numpy(table(cur)).cuda()
    n0 = torch.tensor([len(prev)], dtype=torch.int32, device="cuda")
    n1 = torch.tensor([len(cur)], dtype=torch.int32, device="cuda")
    lk, status = rihvr.link(P, n0, Q, n1, max_disp, spacing)
    return lk.cpu().numpy()[: len(prev)], int(status.cpu().numpy()[0])


def test_link_hand_cases(torch_cuda):
    torch = torch_cuda
    prev = np.array([[0, 0, 0.0], [0, 0, 2.0]])
    cur = np.array([[0, 0, 1.9], [0, 0, 3.5]])
    lk, st = gpu_link(torch, prev, cur, 2.5)
    assert lk.tolist() == [0, 1] and st == 0          # not the greedy s2-t1
    lk, st = gpu_link(torch, np.array([[0, 0, 0.0]]), np.array([[1, 0, 0.0]]), 2.5, spacing=(10, 1, 1))
    assert lk.tolist() == [-1] and st == 0
    # nine sources sharing targets: a subnetwork above the limit is reported
    lk, st = gpu_link(torch, np.zeros((9, 3)), np.zeros((9, 3)) + 0.1, 1.0)
    assert st & 1 and np.all(lk == -1)
    with pytest.raises(ValueError):
        detect.link(np.zeros((9, 3)), np.zeros((9, 3)) + 0.1, 1.0)


@pytest.mark.parametrize("seed", range(6))
def test_link_matches_oracle(torch_cuda, seed):
    """Random fields of particles moved by small displacements, some lost, some
    new, dense enough that subnetworks of several particles form; spacing
    anisotropic as for holograms (planes further apart than pixels)."""
    torch = torch_cuda
    rng = np.random.default_rng(seed)
    n = 400
    prev = rng.uniform([0, 0, 0], [40, 200, 200], (n, 3))
    cur = prev + rng.normal(0, [0.3, 1.0, 1.0], (n, 3))
    keep = rng.permutation(n)[: n - 20]
    cur = np.concatenate([cur[keep], rng.uniform([0, 0, 0], [40, 200, 200], (25, 3))])
    cur = cur[rng.permutation(len(cur))]
    spacing = (10.0, 5.0, 5.0)
    ref = detect.link(prev, cur, 40.0, spacing)        # subnetworks of up to ~6 particles
    lk, st = gpu_link(torch, prev, cur, 40.0, spacing)
    assert st == 0
    assert np.array_equal(lk, ref), np.flatnonzero(lk != ref)[:10]


def test_tracks_over_a_burgers_vortex_series(torch_cuda):
    """Tracks of particle positions advected by the Burgers vortex (3 px per
    frame at most): ids and lengths frame by frame against the oracle, then
    the minimum-duration filter."""
    torch = torch_cuda
    rng = np.random.default_rng(5)
    field, nz, npart, nframes = 256, 60, 300, 12
    traj = scenes.burgers_series(nframes, field, nz, npart, rng)
    frames = []
    for t in range(nframes):
        pos = traj[t].astype(np.float64)
        drop = rng.random(len(pos)) < 0.03                  # occasional missed detections
        frames.append(pos[~drop][rng.permutation(int((~drop).sum()))])
    max_disp, min_len = 4.0, 8
    ids_ref, len_ref, kept_ref = detect.track(frames, max_disp, min_len=min_len)
    cap = 400
    tr = rihvr.Tracks(max_tracks=4096)
    prev_t = prev_n = None
    for t, pos in enumerate(frames):
        T = torch.zeros((cap, 6), dtype=torch.float64, device="cuda")
        T[: len(pos)] = torch.from_numpy(table(pos)).cuda()
        n = torch.tensor([len(pos)], dtype=torch.int32, device="cuda")
        lk = None
        if prev_t is not None:
            lk, status = rihvr.link(prev_t, prev_n, T, n, max_disp)
            assert int(status.item()) == 0
        ids = tr.update(lk, n, cap)
        assert np.array_equal(ids.cpu().numpy()[: len(pos)], ids_ref[t]), t
        prev_t, prev_n = T, n
    nt = int(tr.next_id.item())
    assert nt == len(len_ref)
    assert np.array_equal(tr.track_len.cpu().numpy()[:nt], len_ref)
    kept, n_kept = tr.kept(min_len)
    assert np.array_equal(kept.cpu().numpy()[:nt].astype(bool), kept_ref)
    assert int(n_kept.item()) == int(kept_ref.sum())

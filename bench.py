"""Benchmark: holograms/s to objective gap 1e-4 at 1024^2 x 256 on one MI355X.

One step = one full FISTA solve of a synthetic 1024x1024 hologram into 256
planes (2000 opaque disk particles, C2 optics), from a cold start until the
relative objective gap to a reference value is <= 1e-4.  The reference value is
the smallest objective of a longer function-value-restarted run with the same
prox, computed before the timed region.  Inputs are resident in HBM when the
timer starts.

Prints one JSON line (stdout).  Progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "holograms/s to objective gap 1e-4 at 1024²×256; voxel-iters/s vs plain FISTA"
HBM_PEAK_GBS = 8000.0
# FP32 FMA peak without packed instructions (every HIP file is built with packed
# FP32 off): 256 CUs x 2.4 GHz x 64 lanes x 2 FLOP
FP32_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def prox_bytes_per_voxel(passes: int) -> float:
    """Bytes each voxel must move through HBM in one prox application, by design.

    The prox runs as `passes` launches of the fused TV pass kernel: the first
    reads v and writes the dual p (4 + 12 B), each middle one reads v and p and
    writes p (4 + 12 + 12 B), the last reads v and p and writes x (4 + 12 + 4 B);
    a single pass reads v and writes x (8 B).  Re-reads of tile halos are not
    counted (they are overhead, visible in the measured traffic).
    """
    if passes <= 1:
        return 8.0
    return 16.0 + 28.0 * (passes - 2) + 20.0


def measured_traffic(tuning):
    """HBM bytes per k_tv_pass dispatch from the committed rocprofv3 counter
    summary, or None if the kernel source changed since the counters were taken
    or the plan runs the TV pass with another launch shape than the profiled run."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_tv_pass_c2_hbm_counters.md")
    src = os.path.join(ROOT, "paper_1904_04884_amd", "csrc", "tv.hip")
    try:
        kv = {}
        for line in open(path):
            if " = " in line:
                k, v = line.split(" = ", 1)
                kv[k.strip()] = v.strip()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if kv.get("tv_source_sha256") != digest:
            return None
        want = "%d,%d" % (tuning["tv_levels"], tuning["tv_blocks"])   # the TV pass's launch shape
        if kv.get("tv_tuning") == want:
            return float(kv["traffic_bytes_per_dispatch"])
        other = kv.get("traffic_bytes_per_dispatch[%s]" % want)       # further profiled shapes
        return float(other) if other is not None else None
    except (OSError, KeyError, ValueError):
        return None


def empty_tile_frac(torch, x, tile):
    """Fraction of tile x tile blocks of the (z, y, x) volume's planes that hold
    no non-zero voxel (the rows and planes the solver itself skips are in the
    report; this is the coarser unit a tiled skip would use)."""
    nz, ny, nx = x.shape
    ty, tx = ny // tile, nx // tile
    if ty == 0 or tx == 0:
        return None
    occ = x[:, :ty * tile, :tx * tile].reshape(nz, ty, tile, tx, tile).ne(0).any(dim=4).any(dim=2)
    return 1.0 - float(occ.float().mean())


def build_scene(torch, rihvr, scenes, plan, seed):
    g = scenes.geometry_c2()
    sc = scenes.scene_c2(seed=seed)
    lin = np.ravel_multi_index((sc.idx[:, 0], sc.idx[:, 1], sc.idx[:, 2]), g.shape)
    x_true = torch.zeros(g.shape, dtype=torch.float32, device="cuda")
    x_true.view(-1)[torch.from_numpy(lin).cuda()] = torch.from_numpy(sc.val.astype(np.float32)).cuda()
    b = plan.forward(x_true)
    b += torch.from_numpy(sc.noise.astype(np.float32)).cuda()
    torch.cuda.synchronize()
    return sc, x_true, b


def _oracle_slab_iteration(args):
    """One FISTA iteration of the FP64 oracle on one slab (a worker process)."""
    nz, seed = args
    import oracle
    from paper_1904_04884_amd import scenes
    cfg = scenes.config_c2()
    g = scenes.geometry_c2().with_(nz=nz)
    rng = np.random.default_rng(seed)
    b = 0.05 * rng.standard_normal((g.ny, g.nx))
    t0 = time.perf_counter()
    oracle.fista.fista(g, b, cfg.l1, cfg.tv, 1, cfg.inner_iters)
    return g.nx * g.ny * g.nz, time.perf_counter() - t0


def host_cores():
    """CPUs this process may run on (the box's share, not the machine's count)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(scenes, iters_to_gap, nvox_full, cfg, workers=None):
    """The FP64 oracle on a bounded sample, on every host core: each worker
    process runs one FISTA iteration of the unchanged (single-threaded numpy)
    oracle on its own 8-plane slab of the full geometry (same lateral size and
    optics); the rate is the slabs' voxels over the wall time of the pool."""
    import multiprocessing as mp
    n = workers or min(16, host_cores())
    ctx = mp.get_context("spawn")          # the parent holds a GPU context: no fork
    t0 = time.perf_counter()
    with ctx.Pool(n) as pool:
        res = pool.map(_oracle_slab_iteration, [(8, s) for s in range(n)])
    dt = time.perf_counter() - t0
    nvox = sum(r[0] for r in res)
    vit = nvox / dt
    g = scenes.geometry_c2()
    return {
        "value": vit / (nvox_full * max(iters_to_gap, 1)),
        "unit": "holograms/s",
        "cores": n,
        "kind": "oracle",
        "sample": (f"{n} worker processes, each 1 FISTA iteration (K_in={cfg.inner_iters}) of the FP64 numpy "
                   f"oracle on its own {g.nx}x{g.ny}x8 slab of the same optics ({dt:.1f} s wall including "
                   f"process start, {vit:.3g} voxel-iters/s), scaled to {iters_to_gap} iterations of "
                   f"{nvox_full} voxels"),
        "voxel_iters_per_s": vit,
        "slab_seconds": [round(r[1], 2) for r in res],
        "host_cpus": host_cores(),
    }


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy bandwidth (read + write bytes over time) of a
    1 GiB buffer, HIP events on the current stream."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"GB_per_s": 2.0 * nbytes / (ms * 1e-3) / 1e9, "bytes": nbytes, "ms": ms,
            "frac_of_peak": 2.0 * nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def fft_rates(torch, plan, g, reps=10):
    """FFT FLOP/s of the library's A and A^T (dense, every row), HIP events
    on the current stream.  FLOPs by the 5 N log2 N convention per complex
    transform of length N, half of it for a real-input (R2C / C2R) row:
    A = nz*ny R2C rows + nz*(nx/2) columns + (nx/2) inverse columns + ny C2R
    rows; A^T = ny R2C rows + (nx/2) columns + nz*(nx/2) inverse columns +
    nz*ny C2R rows (the filter multiplies are not counted)."""
    import math
    nx, ny, nz, m = g.nx, g.ny, g.nz, g.nx // 2
    row = 2.5 * nx * math.log2(nx)
    col = 5.0 * ny * math.log2(ny)
    flops = nz * ny * row + nz * m * col + m * col + ny * row       # same count for A and A^T
    x = torch.zeros((nz, ny, nx), dtype=torch.float32, device="cuda")
    x[::7, ::5, ::3] = 1.0
    y = torch.randn((ny, nx), dtype=torch.float32, device="cuda")
    out = {}
    for name, fn in (("forward", lambda: plan.forward(x)), ("adjoint", lambda: plan.adjoint(y))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = flops / (ms * 1e-3) / 1e12
        out[name] = {"ms": ms, "gflop": flops / 1e9, "tflops": tf, "frac_of_peak": tf / FP32_PEAK_TFLOPS}
    out["peak_tflops"] = FP32_PEAK_TFLOPS
    out["convention"] = "5 N log2 N per complex transform, half for real rows; A and A^T dense"
    del x, y
    return out


def burgers_frames(scenes, n_frames, seed=0):
    """Uneven frames of a particle time series in a Burgers vortex (768^2 field,
    up to 200 planes, 1500 particles): frame t is a centred crop of size 256,
    512 or 768 with a plane count in [64, 200]."""
    rng = np.random.default_rng(seed)
    field, nz_max, npart = 768, 200, 1500
    traj = scenes.burgers_series(n_frames, field, nz_max, npart, rng)
    diam = rng.uniform(2.0, 6.0, npart)
    frames = []
    base = scenes.geometry_c2()
    for t in range(n_frames):
        size = int(rng.choice([256, 512, 768]))
        nz = int(rng.integers(64, 201))
        off = (field - size) // 2
        g = base.with_(nx=size, ny=size, nz=nz)
        c = traj[t].copy()
        c[:, 1] -= off
        c[:, 2] -= off
        keep = (c[:, 0] < nz - 0.5) & (c[:, 1] >= 4) & (c[:, 1] < size - 4) & (c[:, 2] >= 4) & (c[:, 2] < size - 4)
        idx, val, _, _ = scenes.disk_particles(g, int(keep.sum()), rng, centers=c[keep], diam=diam[keep])
        noise = scenes.noise_field(g, 0.02, rng)
        frames.append((g, idx, val, noise))
    return frames


def run_batched(args, torch, rihvr, scenes):
    """Batched solve of uneven frames against the same frames solved one by one."""
    cfg = scenes.config_c2()
    frames = burgers_frames(scenes, args.batched, seed=args.seed)
    plans, bs, xs = [], [], []
    import tempfile
    cache = os.path.join(tempfile.mkdtemp(prefix="rihvr_tune_"), "tune.jsonl")
    t_tune, n_timed = 0.0, 0
    for g, idx, val, noise in frames:
        p = rihvr.Plan(g)
        if not args.no_autotune:
            r = p.autotune(cfg.inner_iters, cache)   # one timing per distinct shape, cached after
            t_tune += r["tune_ms"] / 1e3
            n_timed += 0 if r["from_cache"] else 1
        lin = np.ravel_multi_index((idx[:, 0], idx[:, 1], idx[:, 2]), g.shape)
        xt = torch.zeros(g.shape, dtype=torch.float32, device="cuda")
        xt.view(-1)[torch.from_numpy(lin).cuda()] = torch.from_numpy(val.astype(np.float32)).cuda()
        b = p.forward(xt) + torch.from_numpy(noise.astype(np.float32)).cuda()
        del xt
        plans.append(p)
        bs.append(b.contiguous())
        xs.append(torch.empty(g.shape, dtype=torch.float32, device="cuda"))
    nvox = sum(g.nx * g.ny * g.nz for g, _, _, _ in frames)
    iters = args.batch_iters
    log(f"batched: {len(frames)} frames, {nvox / 1e9:.2f} G voxels, {iters} iterations each; "
        f"autotune {t_tune:.1f} s ({n_timed} shapes timed)")
    params = [p.solve_params(cfg.l1, cfg.tv, iters, cfg.inner_iters) for p in plans]
    handles = [p.handle for p in plans]
    nbytes = rihvr.ri_workspace_size_batched(len(plans), handles, params)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream

    params_g = [p.solve_params(cfg.l1, cfg.tv, iters, cfg.inner_iters, flags=rihvr.RI_SOLVE_GROUPED)
                for p in plans]

    def batched(prm=params):
        st = rihvr.ri_solve_batched(len(plans), handles, prm, [b.data_ptr() for b in bs],
                                    [x.data_ptr() for x in xs], ws.data_ptr(), ws.numel(), stream, None)
        assert st == rihvr.RI_OK, rihvr.ri_last_error()

    def timed(prm):
        batched(prm)  # warm-up (graph capture, caches)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batched(prm)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # TV passes as persistent kernels fed by the device work queue (the default)
    tb = timed(params)
    x_queue = [x.clone() for x in xs]
    # one block per tile of every frame
    tg = timed(params_g)
    same = all(torch.equal(a, b) for a, b in zip(xs, x_queue))
    del ws, x_queue
    # the same frames one at a time (each with its own graph)
    for p, b in zip(plans, bs):
        p.solve(b, cfg.l1, cfg.tv, iters, cfg.inner_iters, report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, b in zip(plans, bs):
        p.solve(b, cfg.l1, cfg.tv, iters, cfg.inner_iters, report=False)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    for p in plans:
        p.close()
    return {
        "metric": "holograms/s, batched uneven frames (Burgers-vortex series)",
        "frames": len(frames), "iterations": iters, "voxels": nvox,
        "batched_holograms_per_s": len(frames) / tb, "per_frame_holograms_per_s": len(frames) / ts,
        "speedup": ts / tb, "batched_voxel_iters_per_s": nvox * iters / tb,
        "grouped_holograms_per_s": len(frames) / tg, "persistent_vs_grouped": tg / tb,
        "grouped_bit_identical": same,
        "autotune_s": t_tune, "autotuned_shapes": n_timed,
        "sizes": [[g.nx, g.nz] for g, _, _, _ in frames],
    }


def frame_hologram(torch, plan, g, idx, val, noise):
    lin = np.ravel_multi_index((idx[:, 0], idx[:, 1], idx[:, 2]), g.shape)
    xt = torch.zeros(g.shape, dtype=torch.float32, device="cuda")
    xt.view(-1)[torch.from_numpy(lin).cuda()] = torch.from_numpy(val.astype(np.float32)).cuda()
    b = plan.forward(xt) + torch.from_numpy(noise.astype(np.float32)).cuda()
    del xt
    return b.contiguous()


def run_compare(args, torch, rihvr, scenes):
    """Warm-started batched solves against plain per-frame FISTA (cold start,
    dense, no graph, one frame at a time), both to objective gap 1e-4 on the
    same uneven Burgers-vortex frames; the network is trained on another seed of
    the series.  Plan creation, autotuning, references and training are
    reported separately and are outside both clocks."""
    from paper_1904_04884_amd import warmstart
    cfg = scenes.config_c2()
    K = cfg.inner_iters
    t_setup = time.perf_counter()
    frames = burgers_frames(scenes, args.compare, seed=args.seed)
    plans, bs = [], []
    for g, idx, val, noise in frames:
        p = rihvr.Plan(g)
        plans.append(p)
        bs.append(frame_hologram(torch, p, g, idx, val, noise))
    nvox = sum(g.nx * g.ny * g.nz for g, _, _, _ in frames)
    # references (restarted FISTA), not timed
    f_refs = []
    for p, b in zip(plans, bs):
        f_refs.append(p.solve(b, cfg.l1, cfg.tv, args.cmp_ref_iters, K, flags=rihvr.RI_SOLVE_RESTART,
                              report=True)[1]["objective_min"])
    log(f"compare: {len(frames)} frames, {nvox / 1e9:.2f} G voxels; references done "
        f"({time.perf_counter() - t_setup:.1f} s)")
    # warm-start network on another seed of the series
    t0 = time.perf_counter()
    tframes = burgers_frames(scenes, args.cmp_train, seed=args.seed + 1000)
    tplans = [rihvr.Plan(g) for g, _, _, _ in tframes]
    ws = warmstart.WarmStart(tplans[0], levels=4, base=16, seed=args.seed)
    pairs = []
    for i, (p, (g, idx, val, noise)) in enumerate(zip(tplans, tframes)):
        pairs.append(ws.make_pair(frame_hologram(torch, p, g, idx, val, noise), cfg.l1, cfg.tv,
                                  args.ws_pair_iters, K, plan=p)[0])
        p._ws.pop(rihvr.RI_OP_SOLVE, None)   # the pair's solve is done; training needs only A^T
    curve = ws.train(pairs, steps=args.ws_steps, crop=(32, 64, 64), lr=1e-3,
                     log_every=max(1, args.ws_steps // 5))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del pairs
    for p in tplans:
        p.close()
    log(f"compare: network trained on {len(tframes)} frames in {t_train:.1f} s")
    tuned = 0
    if not args.no_autotune:
        import tempfile
        cache = os.path.join(tempfile.mkdtemp(prefix="rihvr_tune_"), "tune.jsonl")
        for p in plans:
            tuned += 0 if p.autotune(K, cache)["from_cache"] else 1

    def plain():
        its = []
        for p, b, f in zip(plans, bs, f_refs):
            _, r, _ = p.solve(b, cfg.l1, cfg.tv, args.max_iters, K, f_ref=f, gap_tol=args.gap, check_every=5,
                              flags=rihvr.RI_SOLVE_DENSE | rihvr.RI_SOLVE_NO_GRAPH)
            its.append(r["iters"])
        return its

    def warm_batched(warm=True):
        xs, params, used = [], [], []
        for p, b, f in zip(plans, bs, f_refs):
            x1, sc, f0, fs = ws.propose(b, cfg.l1, cfg.tv, K, plan=p) if warm else (None, 1.0, 0.0, 0.0)
            ok = x1 is not None and fs < f0
            used.append(bool(ok))
            xs.append(x1 if ok else torch.empty(p.shape, dtype=torch.float32, device="cuda"))
            params.append(p.solve_params(cfg.l1, cfg.tv, args.max_iters, K, gap_tol=args.gap, f_ref=f,
                                         init=rihvr.RI_INIT_GIVEN if ok else rihvr.RI_INIT_ZERO, check_every=5,
                                         x0_scale=sc if ok else 1.0))
        handles = [p.handle for p in plans]
        nbytes = rihvr.ri_workspace_size_batched(len(plans), handles, params)
        wsb = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        reps = (rihvr.ri_solve_report * len(plans))()
        st = rihvr.ri_solve_batched(len(plans), handles, params, [b.data_ptr() for b in bs],
                                    [x.data_ptr() for x in xs], wsb.data_ptr(), wsb.numel(),
                                    torch.cuda.current_stream().cuda_stream, reps)
        assert st == rihvr.RI_OK, rihvr.ri_last_error()
        return [r.iters for r in reps], [bool(r.converged) for r in reps], used

    plain()  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_plain = plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    warm_batched(False)  # warm-up (graph, allocations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_cold_b, conv_cold_b, _ = warm_batched(False)
    torch.cuda.synchronize()
    t_cold_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    it_warm_b, conv_warm_b, used = warm_batched(True)
    torch.cuda.synchronize()
    t_warm_b = time.perf_counter() - t0
    for p in plans:
        p.close()
    n = len(frames)
    out = {
        "metric": "holograms/s to objective gap 1e-4: warm-started batched vs plain per-frame FISTA",
        "frames": n, "voxels": nvox, "gap": args.gap,
        "plain_holograms_per_s": n / t_plain, "cold_batched_holograms_per_s": n / t_cold_b,
        "warm_batched_holograms_per_s": n / t_warm_b, "speedup_vs_plain": t_plain / t_warm_b,
        "plain_iters": it_plain, "cold_batched_iters": it_cold_b, "warm_batched_iters": it_warm_b,
        "converged": all(conv_cold_b) and all(conv_warm_b), "proposal_used": used,
        "train_frames": len(tframes), "train_s": t_train, "loss_curve": curve, "autotuned_shapes": tuned,
        "sizes": [[g.nx, g.nz] for g, _, _, _ in frames],
    }
    log(f"plain {n / t_plain:.3f} holo/s, cold batched {n / t_cold_b:.3f}, warm batched {n / t_warm_b:.3f} "
        f"({t_plain / t_warm_b:.2f}x)")
    return out


def run_warmstart(args, torch, rihvr, scenes):
    """Iterations to gap 1e-4, cold vs learned warm start, on held-out scenes;
    with --ws-curve, one network per training-set size (the first n of the
    same pairs), all judged on the same held-out scenes."""
    from paper_1904_04884_amd import warmstart
    cfg = scenes.config_c2()
    g = scenes.geometry_c2().with_(nx=args.ws_size, ny=args.ws_size, nz=args.ws_planes)
    plan = rihvr.Plan(g)
    counts = sorted(int(c) for c in args.ws_curve.split(",")) if args.ws_curve else [args.ws_pairs]

    def holo(seed):
        n = int(np.random.default_rng(seed).integers(500, 3001) * (g.nx * g.ny * g.nz) / (512 * 512 * 128))
        sc = scenes.scene_c2(seed=seed, geom=g, n_particles=max(n, 10))
        lin = np.ravel_multi_index((sc.idx[:, 0], sc.idx[:, 1], sc.idx[:, 2]), g.shape)
        xt = torch.zeros(g.shape, dtype=torch.float32, device="cuda")
        xt.view(-1)[torch.from_numpy(lin).cuda()] = torch.from_numpy(sc.val.astype(np.float32)).cuda()
        return (plan.forward(xt) + torch.from_numpy(sc.noise.astype(np.float32)).cuda()).contiguous()

    t0 = time.perf_counter()
    maker = warmstart.WarmStart(plan, levels=4, base=16, seed=0)
    pairs = []
    for i in range(counts[-1]):
        pairs.append(maker.make_pair(holo(1000 + i), cfg.l1, cfg.tv, args.ws_pair_iters, cfg.inner_iters)[0])
        if (i + 1) % 64 == 0:
            log(f"warm start: {i + 1} training pairs ({time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    # held-out scenes: reference objective and cold iterations once
    held = []
    t_cold = 0.0
    for i in range(args.ws_eval):
        b = holo(9000 + i)
        f_ref = plan.solve(b, cfg.l1, cfg.tv, 20 * 100, cfg.inner_iters,
                           flags=rihvr.RI_SOLVE_RESTART)[1]["objective_min"]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, rc, _ = plan.solve(b, cfg.l1, cfg.tv, 2000, cfg.inner_iters, f_ref=f_ref, gap_tol=1e-4, check_every=1)
        torch.cuda.synchronize()
        t_cold += time.perf_counter() - t1
        held.append((b, f_ref, rc["iters"]))
    cold = [h[2] for h in held]
    log(f"held-out cold iterations: {cold}")
    curve = []
    for n in counts:
        ws = warmstart.WarmStart(plan, levels=4, base=16, seed=0)
        t1 = time.perf_counter()
        losses = ws.train(pairs[:n], steps=args.ws_steps, crop=(32, 64, 64), lr=1e-3,
                          log_every=max(1, args.ws_steps // 5))
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        warm, used, t_warm = [], [], 0.0
        for b, f_ref, _ in held:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, rw, u = ws.solve(b, cfg.l1, cfg.tv, 2000, cfg.inner_iters, f_ref=f_ref, gap_tol=1e-4, check_every=1)
            torch.cuda.synchronize()
            t_warm += time.perf_counter() - t1
            warm.append(rw["iters"])
            used.append(bool(u))
        entry = {"pairs": n, "warm_iters": warm, "proposal_used": used, "train_s": t_train, "loss_curve": losses,
                 "iters_ratio": float(np.mean(cold) / max(np.mean(warm), 1e-9)),
                 "cold_holograms_per_s": len(cold) / t_cold, "warm_holograms_per_s": len(warm) / t_warm}
        log(f"warm start with {n} pairs: iterations {warm} (cold {cold}), "
            f"{entry['iters_ratio']:.2f}x fewer, {entry['warm_holograms_per_s']:.3f} vs "
            f"{entry['cold_holograms_per_s']:.3f} holograms/s")
        curve.append(entry)
    plan.close()
    last = curve[-1]
    return {
        "metric": "iterations to objective gap 1e-4, cold vs learned warm start",
        "geometry": [g.nx, g.ny, g.nz], "pairs": counts[-1], "pair_iters": args.ws_pair_iters,
        "train_steps": args.ws_steps, "t_pairs_s": t_pairs, "cold_iters": cold,
        "warm_iters": last["warm_iters"], "proposal_used": last["proposal_used"],
        "cold_holograms_per_s": last["cold_holograms_per_s"], "warm_holograms_per_s": last["warm_holograms_per_s"],
        "curve": curve,
    }


def complex_leg(torch, rihvr, scenes, g, cfg, sc, iters=8):
    """The same scene with a complex amplitude (a phase per plane) on an
    RI_COMPLEX plan: per-iteration phase times of a short timed solve.  The
    complex TV prox takes two dual steps per launch (an odd step alone),
    streamed along z with the dual staged in LDS: v (8 B), one dual set in
    (24 B) and the other out (24 B), 56 B per complex voxel per launch, and
    the final launch v, the dual and x (40 B)."""
    gc = g.with_(complex_object=True)
    p = rihvr.Plan(gc)
    try:
        nvox = g.nx * g.ny * g.nz
        lin = np.ravel_multi_index((sc.idx[:, 0], sc.idx[:, 1], sc.idx[:, 2]), g.shape)
        psi = np.random.default_rng(7).uniform(-0.8, 0.8, g.nz)
        xt = torch.zeros((2, nvox), dtype=torch.float32, device="cuda")
        ph = np.exp(1j * psi[sc.idx[:, 0]]) * sc.val
        xt[0, torch.from_numpy(lin).cuda()] = torch.from_numpy(ph.real.astype(np.float32)).cuda()
        xt[1, torch.from_numpy(lin).cuda()] = torch.from_numpy(ph.imag.astype(np.float32)).cuda()
        b = (p.forward(xt.view(p.shape)) + torch.from_numpy(sc.noise.astype(np.float32)).cuda()).contiguous()
        del xt
        p.solve(b, cfg.l1, cfg.tv, 2, cfg.inner_iters, nonneg=False)       # capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep, _ = p.solve(b, cfg.l1, cfg.tv, iters, cfg.inner_iters, nonneg=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        _, rt, _ = p.solve(b, cfg.l1, cfg.tv, iters, cfg.inner_iters, nonneg=False, flags=rihvr.RI_SOLVE_TIMING)
        ph_ms = {k: v / iters for k, v in rt["phase_ms"].items()}
        step_launches = cfg.inner_iters // 2 + cfg.inner_iters % 2
        prox_bytes = (56.0 * step_launches + 40.0) * nvox
        out = {"iters": iters, "ms_per_iter": 1000.0 * dt / iters, "phase_ms_per_iter": ph_ms,
               "prox_GB_per_s": prox_bytes / (ph_ms["prox"] * 1e-3) / 1e9,
               "prox_bytes_model": "56 B per complex voxel per launch of two dual steps + 40 B final",
               "objective": rep["objective"]}
        log(f"complex object: {out['ms_per_iter']:.1f} ms per iteration (prox {ph_ms['prox']:.1f} ms, "
            f"{out['prox_GB_per_s']:.0f} GB/s by the two-steps-per-launch byte model)")
        return out
    finally:
        p.close()
        torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--ref-iters", type=int, default=2000, help="outer iterations of the reference run")
    ap.add_argument("--max-iters", type=int, default=1000)
    ap.add_argument("--gap", type=float, default=1e-4)
    ap.add_argument("--check-every", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain-FISTA leg (cold, dense, no graph) on the same hologram")
    ap.add_argument("--batched", type=int, default=0, help="run the batched uneven-frame mode with this many frames")
    ap.add_argument("--batch-iters", type=int, default=30)
    ap.add_argument("--warmstart", action="store_true", help="run the learned warm-start evaluation mode")
    ap.add_argument("--compare", type=int, default=0,
                    help="warm-started batched solves vs plain per-frame FISTA on this many uneven frames")
    ap.add_argument("--cmp-train", type=int, default=8, help="training frames for --compare")
    ap.add_argument("--cmp-ref-iters", type=int, default=600, help="restarted reference iterations for --compare")
    ap.add_argument("--ws-size", type=int, default=256)
    ap.add_argument("--ws-planes", type=int, default=64)
    ap.add_argument("--ws-pairs", type=int, default=48)
    ap.add_argument("--ws-pair-iters", type=int, default=300)
    ap.add_argument("--ws-steps", type=int, default=1500)
    ap.add_argument("--ws-eval", type=int, default=4)
    ap.add_argument("--ws-curve", type=str, default=None,
                    help="training-set sizes for a curve of warm-start gain against pair count, e.g. 64,192,512")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--restart", action="store_true",
                    help="timed solves use function-value restart of the momentum (FISTA variant; not the default)")
    ap.add_argument("--tuning", type=str, default=None,
                    help="fixed launch shapes tv_levels,tv_blocks,col_blocks (no autotuning; for profiling)")
    ap.add_argument("--no-complex", dest="complex_leg", action="store_false",
                    help="skip the complex-object leg (RI_COMPLEX plan at the same size, a few iterations)")
    ap.add_argument("--no-row-store", dest="row_store", action="store_false",
                    help="skip the row-store leg (the same solve with row-compressed iterates)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy (for scaling FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU sharding is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_04884_amd import rihvr, scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    rihvr.lib()
    if args.batched:
        print(json.dumps(run_batched(args, torch, rihvr, scenes)), flush=True)
        return
    if args.warmstart:
        print(json.dumps(run_warmstart(args, torch, rihvr, scenes)), flush=True)
        return
    if args.compare:
        print(json.dumps(run_compare(args, torch, rihvr, scenes)), flush=True)
        return
    cfg = scenes.config_c2()
    g = scenes.geometry_c2()
    nvox = g.nx * g.ny * g.nz
    t0 = time.perf_counter()
    plan = rihvr.Plan(g)
    log(f"plan: ||A||^2 = {plan.lipschitz:.6f} ({time.perf_counter() - t0:.2f} s)")
    tune = None
    if args.tuning:
        lv, tb, cb = (int(v) for v in args.tuning.split(","))
        plan.tuning = {"tv_levels": lv, "tv_blocks": tb, "col_blocks": cb}
    elif not args.no_autotune:
        tune = plan.autotune(cfg.inner_iters)
        log(f"autotune: {tune['best']} ({tune['candidates']} shapes, {tune['tune_ms'] / 1e3:.2f} s); "
            f"A + A^T + prox {tune['default_ms']:.3f} -> {tune['best_ms']:.3f} ms")
    sc, x_true, b = build_scene(torch, rihvr, scenes, plan, args.seed)
    log(f"scene: {len(sc.centers)} particles, {len(sc.val)} voxels; |b| = {float(b.norm()):.4g}")

    # reference objective (not timed)
    t0 = time.perf_counter()
    _, rep_ref, _ = plan.solve(b, cfg.l1, cfg.tv, args.ref_iters, cfg.inner_iters, flags=rihvr.RI_SOLVE_RESTART)
    torch.cuda.synchronize()
    f_ref = rep_ref["objective_min"]
    log(f"reference: {args.ref_iters} restarted iterations, F_ref = {f_ref:.9g} ({time.perf_counter() - t0:.1f} s)")

    def one_solve(flags=0):
        flags |= rihvr.RI_SOLVE_RESTART if args.restart else 0
        return plan.solve(b, cfg.l1, cfg.tv, args.max_iters, cfg.inner_iters, f_ref=f_ref, gap_tol=args.gap,
                          check_every=args.check_every, flags=flags)

    for w in range(args.warmup):
        _, rep, _ = one_solve()
        log(f"warmup {w}: {rep['iters']} iterations, gap {rep['gap']:.3g}")
    torch.cuda.synchronize()
    iters = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        _, rep, _ = one_solve()
        iters.append(rep["iters"])
        log(f"step {s}: {rep['iters']} iterations, gap {rep['gap']:.3g}, converged {rep['converged']}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    value = args.steps / elapsed
    mean_iters = float(np.mean(iters))
    converged = bool(rep["converged"])

    # per-phase device times (HIP events on the solve's stream), same solve
    x_t, rep_t, _ = one_solve(flags=rihvr.RI_SOLVE_TIMING)
    tile_frac = empty_tile_frac(torch, x_t, 32)   # diagnostic of the solution's sparsity, not timed
    log(f"solution: empty fraction of planes {rep_t['empty_plane_frac']:.3f}, rows {rep_t['empty_row_frac']:.3f}, 32x32 tiles {tile_frac:.3f}")
    del x_t
    ph = rep_t["phase_ms"]
    nl = rep_t["phase_launches"]
    n_prox = max(rep_t["iters"], 1)
    passes = nl["prox"] // n_prox
    launch_ms = ph["prox"] / max(nl["prox"], 1)
    bytes_per_launch = prox_bytes_per_voxel(passes) * nvox / passes
    prox_gbs = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    roofline = {
        "bound": "hbm",
        "kernel": "k_tv_pass (fused TV dual steps; the prox is `passes` launches)",
        "achieved": prox_gbs,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": prox_gbs / HBM_PEAK_GBS,
        "traffic": measured_traffic(plan.tuning),
        "launch_ms": launch_ms,
        "passes": passes,
        "bytes_per_voxel_per_prox": prox_bytes_per_voxel(passes),
        "bytes_per_launch": bytes_per_launch,
    }
    phase_ms_per_iter = {k: v / n_prox for k, v in ph.items()}
    log("phase ms / iteration: " + ", ".join(f"{k} {v:.3f}" for k, v in phase_ms_per_iter.items()))

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x 1 GiB device copies")

    plain = None
    if not args.no_plain:
        # plain per-frame FISTA: the same solve with no row skipping and one
        # launch at a time (no graph), cold start, same gap criterion
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, rep_p, _ = one_solve(flags=rihvr.RI_SOLVE_DENSE | rihvr.RI_SOLVE_NO_GRAPH)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t1
        plain = {"holograms_per_s": 1.0 / dtp, "iters": rep_p["iters"],
                 "voxel_iters_per_s": nvox * rep_p["iters"] / dtp,
                 "value_over_plain": value * dtp,
                 "flags": "RI_SOLVE_DENSE | RI_SOLVE_NO_GRAPH, cold start"}
        log(f"plain FISTA: {1.0 / dtp:.4f} holograms/s ({rep_p['iters']} iterations); "
            f"headline / plain = {value * dtp:.3f}")
    row_store = None
    if args.row_store:
        # the same solve with x_k, x_{k-1}, x_{k+1} in row stores: a first
        # solve with room for every row gives the peak occupancy; the timed
        # solve uses pools of exactly that many rows
        dense_ws = rihvr.ri_workspace_size_op(plan.handle, rihvr.RI_OP_SOLVE)
        rows = g.ny * g.nz

        def store_solve():
            return plan.solve(b, cfg.l1, cfg.tv, args.max_iters, cfg.inner_iters, f_ref=f_ref, gap_tol=args.gap,
                              check_every=args.check_every, raise_on_error=False)
        plan.row_fraction = 1.0
        _, rep_1, _ = store_solve()
        peak = rep_1["store_rows_peak"]
        plan.row_fraction = peak / rows
        store_ws = rihvr.ri_workspace_size_op(plan.handle, rihvr.RI_OP_SOLVE)
        store_solve()                         # captures the graph for this layout
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, rep_s, st_s = store_solve()
        torch.cuda.synchronize()
        dts = time.perf_counter() - t1
        plan.row_fraction = 0.0
        row_store = {"peak_rows": peak, "rows": rows, "row_fraction": peak / rows,
                     "status": rihvr.ri_status_string(st_s), "holograms_per_s": 1.0 / dts, "iters": rep_s["iters"],
                     "solve_workspace_bytes": store_ws, "dense_solve_workspace_bytes": dense_ws,
                     "value_over_row_store": value * dts}
        log(f"row stores: peak {peak} of {rows} rows; {1.0 / dts:.4f} holograms/s, {rep_s['iters']} iterations, "
            f"status {row_store['status']}; solve workspace {store_ws / 2**30:.2f} GiB vs {dense_ws / 2**30:.2f} GiB")
    cplx = complex_leg(torch, rihvr, scenes, g, cfg, sc) if args.complex_leg else None
    fft = fft_rates(torch, plan, g)
    log("FFT: " + ", ".join(f"{k} {v['tflops']:.2f} TFLOP/s ({v['ms']:.3f} ms)"
                            for k, v in fft.items() if isinstance(v, dict)))
    copy_bw = copy_bandwidth(torch)
    log(f"device copy: {copy_bw['GB_per_s']:.0f} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(scenes, int(round(mean_iters)), nvox, cfg)
        log(f"cpu baseline: {cpu['voxel_iters_per_s']:.3g} voxel-iters/s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "holograms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "C2: 1024x1024 hologram, 256 planes (z 5000+50j um, lambda 0.532 um, 5 um px), "
                        "2000 disk particles d~U[2,6] px, noise 0.02, l1 0.02, tv 0.01, K_in 20, cold start, "
                        "gap 1e-4 vs restarted reference",
            "nx": g.nx, "ny": g.ny, "nz": g.nz, "seed": args.seed,
            "tuning": plan.tuning,
        },
        "autotune": tune,
        "iters_to_gap": mean_iters,
        "converged": converged,
        "voxel_iters_per_s": nvox * mean_iters * value,
        "f_ref": f_ref,
        "empty_row_frac": rep["empty_row_frac"],
        "empty_tile32_frac": tile_frac,
        "empty_plane_frac": rep["empty_plane_frac"],
        "phase_ms_per_iter": phase_ms_per_iter,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain_fista": plain,
        "row_store": row_store,
        "complex_object": cplx,
        "fft": fft,
        "copy_bandwidth": copy_bw,
    }
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

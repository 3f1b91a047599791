"""The learned warm start against the plain (cold) solve on held-out scenes.

Pairs come from the library's own solver on seeded C1-optics scenes; a small
U-Net is trained on the whole volumes on the GPU; held-out scenes are solved to a
relative objective gap from a cold start and from the network's proposal.
The test records both iteration counts and requires the warm start to need
fewer iterations on average (the objective decides; the fallback keeps any
proposal worse than x = 0 out)."""
import numpy as np
import pytest

from paper_1904_04884_amd import rihvr, scenes, warmstart

pytestmark = pytest.mark.gpu


def hologram(torch, plan, sc):
    x = torch.from_numpy(sc.dense(np.float32)).cuda()
    b = plan.forward(x)
    return (b + torch.from_numpy(sc.noise.astype(np.float32)).cuda()).contiguous()


def test_warm_start_gains_over_cold(torch_cuda):
    torch = torch_cuda
    g = scenes.geometry_c1()
    cfg = scenes.config_c1()
    plan = rihvr.Plan(g)
    try:
        ws = warmstart.WarmStart(plan, levels=3, base=16, seed=0)
        pairs = []
        for seed in range(1000, 1024):
            sc = scenes.scene_c1(seed=seed, n_particles=int(np.random.default_rng(seed).integers(30, 80)))
            p, _ = ws.make_pair(hologram(torch, plan, sc), cfg.l1, cfg.tv, 150, cfg.inner_iters)
            pairs.append(p)
        curve = ws.train(pairs, steps=500, crop=(32, 128, 128), lr=2e-3, log_every=100)
        assert curve[-1][1] < curve[0][1]
        cold, warm, used = [], [], []
        for seed in range(9000, 9004):
            sc = scenes.scene_c1(seed=seed)
            b = hologram(torch, plan, sc)
            f_ref = plan.solve(b, cfg.l1, cfg.tv, 600, cfg.inner_iters,
                               flags=rihvr.RI_SOLVE_RESTART)[1]["objective_min"]
            _, rc, _ = plan.solve(b, cfg.l1, cfg.tv, 600, cfg.inner_iters, f_ref=f_ref, gap_tol=1e-3, check_every=1)
            _, rw, u = ws.solve(b, cfg.l1, cfg.tv, 600, cfg.inner_iters, f_ref=f_ref, gap_tol=1e-3, check_every=1)
            assert rc["converged"] and rw["converged"]
            cold.append(rc["iters"])
            warm.append(rw["iters"])
            used.append(u)
        print(f"iterations to gap 1e-3: cold {cold} warm {warm} (proposal used {used}); loss {curve}")
        assert np.mean(warm) < np.mean(cold)
    finally:
        plan.close()

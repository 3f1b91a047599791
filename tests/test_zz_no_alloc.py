"""The allocation-free forward (ri_forward_noalloc) against ri_forward, through the C ABI.

Both run the same kernels with the same launch shapes, so the holograms must be
bit-identical; the FP64 oracle bounds both at 1e-5 relative L2.  Two calls in a
row, the second on a smaller geometry, show that what the first call left in the
shared scratch array does not leak into the second.
"""
import numpy as np
import pytest

from oracle import optics
from paper_1904_04884_amd import rihvr, scenes

pytestmark = pytest.mark.gpu


def _hologram_pair(torch, plan, x):
    g = plan.geom
    ref = plan.forward(x)
    out = torch.full((g.ny, g.nx), float("nan"), dtype=torch.float32, device="cuda")
    st = rihvr.ri_forward_noalloc(plan.handle, x.data_ptr(), out.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
    rihvr._check(st, "ri_forward_noalloc")
    torch.cuda.synchronize()
    return ref, out


def test_forward_noalloc_matches_forward_twice(torch_cuda):
    torch = torch_cuda
    geoms = [scenes.geometry_c1().with_(nx=256, ny=192, nz=40),      # several column tiles and z-chunks
             scenes.geometry_c1().with_(nx=96, ny=48, nz=7)]         # then a smaller one
    for i, g in enumerate(geoms):
        plan = rihvr.Plan(g)
        try:
            need = rihvr.ri_workspace_size_op(plan.handle, rihvr.RI_OP_FORWARD)
            assert need <= rihvr.ri_forward_noalloc_max_scratch()
            rng = np.random.default_rng(100 + i)
            x = np.maximum(rng.standard_normal((g.nz, g.ny, g.nx)), 0.0)
            x[:, :, ::5] = 0.0                                        # some structure, some zeros
            xd = torch.from_numpy(x.astype(np.float32)).cuda()
            ref, out = _hologram_pair(torch, plan, xd)
            print(f"call {i}: {g.nx}x{g.ny}x{g.nz}, scratch {need} bytes", flush=True)
            assert torch.equal(ref, out), float((ref - out).abs().max())
            want = optics.forward(g, x.astype(np.float32).astype(np.float64))
            err = np.linalg.norm(out.cpu().numpy() - want) / np.linalg.norm(want)
            assert err <= 1e-5, err
        finally:
            plan.close()


def test_forward_noalloc_rejects_oversize(torch_cuda):
    torch = torch_cuda
    g = scenes.geometry_c1().with_(nx=1024, ny=1024, nz=32)
    plan = rihvr.Plan(g)
    try:
        assert rihvr.ri_workspace_size_op(plan.handle, rihvr.RI_OP_FORWARD) > rihvr.ri_forward_noalloc_max_scratch()
        x = torch.zeros((g.nz, g.ny, g.nx), dtype=torch.float32, device="cuda")
        out = torch.zeros((g.ny, g.nx), dtype=torch.float32, device="cuda")
        st = rihvr.ri_forward_noalloc(plan.handle, x.data_ptr(), out.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream)
        assert st == rihvr.RI_ERR_UNSUPPORTED_SIZE
        assert b"allocation-free" in rihvr.lib().ri_last_error()
    finally:
        plan.close()

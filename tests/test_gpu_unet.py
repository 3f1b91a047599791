"""GPU U-Net (BF16 MFMA kernels) against the FP64 network oracle, through the C ABI.

BF16 activations and weights give ~3 significant digits, so outputs and
gradients are compared in relative L2 with a 2e-2 bar (3e-2 for weight
gradients, which sum many BF16 products)."""
import numpy as np
import pytest

from oracle import unet as ou
from paper_1904_04884_amd import rihvr

pytestmark = pytest.mark.gpu


def flat(params, levels, base):
    parts = []
    for name, kind, cin, cout in ou.layer_specs(levels, base):
        parts.append(np.asarray(params[name + ".w"], np.float64).ravel())
        parts.append(np.asarray(params[name + ".b"], np.float64).ravel())
    return np.concatenate(parts)


def unflat(vec, levels, base, like):
    out, off = {}, 0
    for name, kind, cin, cout in ou.layer_specs(levels, base):
        for k in (".w", ".b"):
            a = np.asarray(like[name + k])
            out[name + k] = vec[off:off + a.size].reshape(a.shape)
            off += a.size
    return out


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_unet_forward_and_gradients(torch_cuda, levels):
    torch = torch_cuda
    base = 8
    rng = np.random.default_rng(levels)
    p = ou.init_params(levels, base, rng)
    # bf16-representable parameters and inputs so the comparison isolates the arithmetic
    for k in p:
        p[k] = torch.tensor(p[k], dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    D = H = W = 16
    x = rng.standard_normal((D, H, W))
    x = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    target = np.maximum(rng.standard_normal((D, H, W)), 0.0)
    y_ref = ou.forward(p, x, levels, base)
    loss_ref, g_ref = ou.loss_and_grads(p, x, target, levels, base)

    net = rihvr.UNet(levels, base, seed=1)
    assert net.n == flat(p, levels, base).size
    net.params.copy_(torch.tensor(flat(p, levels, base), dtype=torch.float32))
    xin = torch.tensor(x, dtype=torch.float32).cuda()
    y = net.forward(xin).cpu().numpy()
    assert rel(y, y_ref) <= 2e-2, rel(y, y_ref)
    loss = net.train_step(xin, torch.tensor(target, dtype=torch.float32).cuda(), lr=0.0)
    assert float(loss) == pytest.approx(loss_ref, rel=2e-2)
    g = unflat(net.grads.cpu().numpy().astype(np.float64), levels, base, p)
    for k in g_ref:
        if np.linalg.norm(g_ref[k]) == 0:
            continue
        assert rel(g[k], g_ref[k]) <= 3e-2, (k, rel(g[k], g_ref[k]))


def test_unet_training_reduces_loss(torch_cuda):
    torch = torch_cuda
    rng = np.random.default_rng(5)
    D = H = W = 16
    x = torch.tensor(rng.standard_normal((D, H, W)), dtype=torch.float32).cuda()
    t = torch.relu(x * 0.5).contiguous()
    net = rihvr.UNet(3, 8, seed=2)
    losses = [float(net.train_step(x, t, lr=3e-3)) for _ in range(60)]
    assert losses[-1] < 0.3 * losses[0], (losses[0], losses[-1])


def test_unet_rejects_bad_shapes(torch_cuda):
    cfg = rihvr.ri_unet_config(4, 16)
    with pytest.raises(rihvr.RihvrError):
        rihvr.ri_unet_workspace_size(cfg, 12, 16, 16, 0)
    with pytest.raises(rihvr.RihvrError):
        rihvr.ri_unet_param_count(rihvr.ri_unet_config(4, 12))

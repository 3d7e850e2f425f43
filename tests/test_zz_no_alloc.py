"""The allocation-free loss/gradient entry point (m2m_mlp_loss_grad_noalloc)
against the allocating one (m2m_mlp_loss_grad) through the C ABI: two calls in a
row on the same context, the second with fewer samples (the static scratch keeps
the first call's contents), device buffers only.  Same kernels, so the gradient
must agree bitwise; the loss is summed on the device in FP64 instead of on the
host, so it agrees to FP64 rounding of a sum of n FP32 terms."""
import numpy as np
import pytest

from synth import configs
from tests import helpers as H
from tests.golden import derive_eps

pytestmark = pytest.mark.gpu

m2m = pytest.importorskip("paper_1207_6403_amd")


def _context():
    cfg = configs.cfg5(N=4096, target_n=1 << 16)
    cfg["prior"].update(subset=512, batch=128, period=4, fallback=0.5)
    cfg["eps"] = 0.1 / (cfg["dt"] * derive_eps.max_abs_G(cfg))
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    return cfg, ctx


def _samples(rng, n):
    u = rng.uniform(-1.0, 1.0, (n, 3))
    t = 0.7 * u[:, 0] - 0.4 * u[:, 1] * u[:, 2] + 0.1 * rng.normal(size=n) - 14.0
    return np.column_stack([u, t]).astype(np.float32)


def test_noalloc_matches_allocating_entry_point():
    import torch
    dev = torch.device("cuda:0")
    cfg, ctx = _context()
    rng = np.random.default_rng(5)
    theta = cfg["prior"]["mlp_init"].astype(np.float32)
    grad_d = torch.empty(m2m.binding.MLP_NPARAM, dtype=torch.float32, device=dev)
    loss_d = torch.empty(1, dtype=torch.float64, device=dev)
    for n in (m2m.binding.MLP_NOALLOC_MAX, 1024):
        H.flush("no-alloc loss/gradient: n=%d" % n)
        th = theta + np.float32(0.01) * rng.normal(size=theta.size).astype(np.float32)
        smp = _samples(rng, n)
        grad_d.fill_(np.nan)
        loss_d.fill_(np.nan)
        m2m.m2m_mlp_loss_grad_noalloc(ctx, torch.from_numpy(th).to(dev), torch.from_numpy(smp).to(dev), grad_d,
                                      loss_d)
        torch.cuda.synchronize()
        g_na = grad_d.cpu().numpy()
        l_na = float(loss_d.cpu().numpy()[0])
        l_ref, g_ref = m2m.m2m_mlp_loss_grad(ctx, th, smp)
        np.testing.assert_array_equal(g_na, g_ref)
        assert l_na == pytest.approx(l_ref, rel=1e-12)
    m2m.m2m_destroy(ctx)


def test_noalloc_rejects_more_than_the_scratch_holds():
    import torch
    dev = torch.device("cuda:0")
    cfg, ctx = _context()
    n = m2m.binding.MLP_NOALLOC_MAX + 32
    th = torch.from_numpy(cfg["prior"]["mlp_init"].astype(np.float32)).to(dev)
    smp = torch.zeros((n, 4), dtype=torch.float32, device=dev)
    grad = torch.empty(m2m.binding.MLP_NPARAM, dtype=torch.float32, device=dev)
    with pytest.raises(m2m.M2MError) as e:
        m2m.m2m_mlp_loss_grad_noalloc(ctx, th, smp, grad)
    assert e.value.status == 1
    m2m.m2m_destroy(ctx)

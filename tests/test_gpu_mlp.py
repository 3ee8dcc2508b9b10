"""GPU MLP kernels against the oracle's FP64 reference: forward values and
loss/gradients (the oracle's gradients are themselves pinned by finite
differences on the CPU)."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def _setup(bop, seed=0, B=777):
    import torch
    rng = np.random.default_rng(seed)
    arrs = [rng.normal(scale=0.3, size=s) for s in bop.MLP_SHAPES]
    x = rng.normal(size=(B, 6))
    t = rng.normal(size=B)
    return arrs, x, t, bop.mlp_pack(arrs), torch.tensor(x, dtype=torch.float32, device="cuda"), \
        torch.tensor(t, dtype=torch.float32, device="cuda")


def test_forward_matches_oracle(bop):
    arrs, x, t, p, xd, td = _setup(bop)
    y_ref, _ = O.mlp_forward(arrs, x.astype(np.float32).astype(np.float64))
    y = bop.mlp_forward(p, xd).cpu().numpy()
    assert np.max(np.abs(y - y_ref)) < 2e-5 * max(1.0, np.abs(y_ref).max())


def test_gradients_match_oracle(bop):
    """FP32 gradients vs FP64 analytic gradients: relative to each block's
    largest entry, within 1e-4 (FP32 sums over 777 rows)."""
    arrs, x, t, p, xd, td = _setup(bop)
    xs = x.astype(np.float32).astype(np.float64)
    ts = t.astype(np.float32).astype(np.float64)
    loss_ref, g_ref = O.mlp_loss_grad(arrs, xs, ts)
    m = bop.MLP()
    m.params = p
    loss, g = m.grad(xd, td)
    assert abs(float(loss.item()) - loss_ref) < 1e-5 * max(1.0, loss_ref)
    gg = bop.mlp_unpack(g)
    for a, b in zip(gg, g_ref):
        assert np.max(np.abs(a - b)) <= 1e-4 * max(1e-6, np.abs(b).max())


def test_adam_step_matches_oracle(bop):
    import torch
    arrs, x, t, p, xd, td = _setup(bop, seed=1, B=512)
    m = bop.MLP()
    m.params = p.clone()
    m.train(xd, td, epochs=1, batch=512, lr=1e-3, seed=0)       # one step (one full batch)
    perm = np.random.default_rng(0).permutation(512)
    xs = x[perm].astype(np.float32).astype(np.float64)
    ts = t[perm].astype(np.float32).astype(np.float64)
    _, g = O.mlp_loss_grad(arrs, xs, ts)
    zero = [np.zeros_like(a) for a in arrs]
    new, _, _ = O.adam_step([a.astype(np.float32).astype(np.float64) for a in arrs], g, zero, zero, 1)
    got = bop.mlp_unpack(m.params)
    for a, b in zip(got, new):
        assert np.max(np.abs(a - b)) < 2e-6


def test_backward_then_adam_equals_training_step(bop):
    """bop_mlp_backward + bop_mlp_adam (the step split in two) give the fused
    training step's parameters bit for bit, over two steps; the split Adam
    update matches the oracle's from the oracle's gradient."""
    import torch
    arrs, x, t, p, xd, td = _setup(bop, seed=2, B=640)
    fused = bop.MLP()
    fused.params = p.clone()
    split = bop.MLP()
    split.params = p.clone()
    for _ in range(2):
        fused.train(xd, td, epochs=1, batch=640, lr=1e-3, seed=0)
        perm = torch.as_tensor(np.random.default_rng(0).permutation(640).astype(np.int64), device="cuda")
        _, g = split.grad(xd[perm].contiguous(), td[perm].contiguous())
        split.adam(g, lr=1e-3)
    torch.cuda.synchronize()
    assert torch.equal(fused.params, split.params)
    one = bop.MLP()
    one.params = p.clone()
    perm = np.random.default_rng(0).permutation(640)
    xs = x[perm].astype(np.float32).astype(np.float64)
    ts = t[perm].astype(np.float32).astype(np.float64)
    _, g_ref = O.mlp_loss_grad(arrs, xs, ts)
    one.adam(bop.mlp_pack(g_ref), lr=1e-3)
    zero = [np.zeros_like(a) for a in arrs]
    new, _, _ = O.adam_step([a.astype(np.float32).astype(np.float64) for a in arrs], g_ref, zero, zero, 1)
    for a, b in zip(bop.mlp_unpack(one.params), new):
        assert np.max(np.abs(a - b)) < 2e-6


def test_training_reduces_loss(bop):
    import torch
    rng = np.random.default_rng(3)
    x = rng.normal(size=(8192, 6))
    t = np.tanh(x @ rng.normal(size=6)) * 0.5
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    m = bop.MLP(seed=0)
    l0, _ = m.grad(xd, td)
    m.train(xd, td, epochs=20, batch=1024, lr=3e-3)
    l1, _ = m.grad(xd, td)
    assert float(l1.item()) < 0.1 * float(l0.item())


def test_feature_stats_standardise_and_shift_match_oracle(bop):
    """Feature statistics (FP64 sums of FP32 values: 1e-6 relative), the
    standardisation (FP32, 1e-5) and the gauge-fixed shifts (the forward bound,
    2e-5 of the output scale) against the oracle; 300,001 rows span many
    reduction strides."""
    import torch
    rng = np.random.default_rng(4)
    x = rng.normal(loc=[0.0, 1.0, -2.0, 5.0, 0.1, 30.0], scale=[1.0, 0.5, 3.0, 0.01, 2.0, 7.0], size=(300001, 6))
    x32 = x.astype(np.float32)
    xd = torch.tensor(x32, device="cuda")
    mean, std = bop.feature_stats(xd)
    m_ref, s_ref = O.feature_stats(x32.astype(np.float64))
    assert np.max(np.abs(mean.cpu().numpy() - m_ref) / np.maximum(np.abs(m_ref), s_ref)) < 1e-6
    assert np.max(np.abs(std.cpu().numpy() - s_ref) / s_ref) < 1e-6
    # both sides standardise with the oracle's statistics (rounded to FP32)
    m32, s32 = m_ref.astype(np.float32), s_ref.astype(np.float32)
    z = bop.standardise(xd, torch.tensor(m32, device="cuda"), torch.tensor(s32, device="cuda")).cpu().numpy()
    z_ref = (x32.astype(np.float64) - m32.astype(np.float64)) / s32.astype(np.float64)
    assert np.max(np.abs(z - z_ref)) < 1e-5 * max(1.0, np.abs(z_ref).max())
    arrs, _, _, p, _, _ = _setup(bop)
    zd = torch.tensor(z_ref[:5000].astype(np.float32), device="cuda")
    sh = bop.mlp_shift(p, zd).cpu().numpy()
    sh_ref = O.mlp_shift(arrs, z_ref[:5000].astype(np.float32).astype(np.float64))
    assert np.max(np.abs(sh - sh_ref)) < 2e-5 * max(1.0, np.abs(sh_ref).max())
    assert abs(sh.sum()) < 1e-9 * 5000

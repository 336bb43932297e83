"""Pins of the peak-filter oracle against independent routes: torch's
bfloat16 conversion, torch's conv3d and autograd on the same network, central
finite differences, and index arithmetic written out per cell."""
import numpy as np
import pytest

from oracle import cnn


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        np.arange(-300, 300) / 16.0, [0.0, -0.0, 1e-40, 3.4e38]]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).float().numpy().astype(np.float64)
    assert np.array_equal(cnn.bf16(x), want)


def test_windows_wrap_and_pad():
    rng = np.random.default_rng(1)
    acc = rng.integers(0, 40, (4, 6, 8)).astype(np.int32)
    lins = [0, 7, 6 * 8 - 1, (3 * 6 + 5) * 8 + 3, (1 * 6 + 2) * 8 + 4]
    w = cnn.windows(acc, lins)
    for n, lin in enumerate(lins):
        i, j, k = lin % 8, (lin // 8) % 6, lin // 48
        for a in range(5):
            for b in range(5):
                for c in range(5):
                    kk, jj, ii = k + a - 2, j + b - 2, (i + c - 2) % 8
                    v = acc[kk, jj, ii] / 16.0 if 0 <= kk < 4 and 0 <= jj < 6 else 0.0
                    assert w[n, a, b, c] == v


def torch_net(torch, flat, x):
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True)
         for k, v in cnn.unpack(flat).items()}
    xt = torch.tensor(x, dtype=torch.float64).unsqueeze(1)
    F = torch.nn.functional
    h1 = F.relu(F.conv3d(xt, P["W1"].reshape(16, 1, 3, 3, 3), P["b1"]))
    h2 = F.relu(F.conv3d(h1, P["W2"].reshape(16, 16, 3, 3, 3), P["b2"])).reshape(-1, 16)
    h3 = F.relu(h2 @ P["W3"].T + P["b3"])
    return h3 @ P["W4"] + P["b4"], P


def test_forward_and_grad_match_torch_unrounded():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    flat = cnn.init_params(3)
    x = rng.integers(0, 30, (12, 5, 5, 5)) / 16.0
    y = (rng.uniform(size=12) > 0.6).astype(np.float64)
    loss, g, z = cnn.loss_and_grad(flat, x, y, pos_weight=2.5, rounding=False)
    zt, P = torch_net(torch, flat, x)
    assert np.allclose(z, zt.detach().numpy(), rtol=1e-12, atol=1e-12)
    w = torch.tensor(np.where(y > 0.5, 2.5, 1.0))
    lt = (w * torch.nn.functional.binary_cross_entropy_with_logits(
        zt, torch.tensor(y), reduction="none")).mean()
    lt.backward()
    assert abs(loss - lt.item()) < 1e-12
    gt = np.concatenate([P[name].grad.numpy().reshape(-1) for name, _ in cnn.SHAPES])
    assert np.allclose(g, gt, rtol=1e-10, atol=1e-13)


def test_grad_finite_differences():
    rng = np.random.default_rng(4)
    flat = cnn.init_params(5).astype(np.float64)
    x = rng.integers(0, 30, (6, 5, 5, 5)) / 16.0
    y = np.array([1, 0, 0, 1, 0, 1], np.float64)
    _, g, _ = cnn.loss_and_grad(flat, x, y, pos_weight=2.0, rounding=False)
    idx = rng.choice(cnn.N_PARAMS, 60, replace=False)
    for i in idx:
        e = np.zeros(cnn.N_PARAMS)
        e[i] = 1e-6
        lp = cnn.loss_and_grad(flat + e, x, y, 2.0, rounding=False)[0]
        lm = cnn.loss_and_grad(flat - e, x, y, 2.0, rounding=False)[0]
        assert abs((lp - lm) / 2e-6 - g[i]) < 1e-6 + 1e-4 * abs(g[i]), i


def test_rounded_forward_is_bf16_of_layers():
    """With rounding on, each activation equals bfloat16 of the float64 layer."""
    rng = np.random.default_rng(6)
    flat = cnn.init_params(7)
    x = rng.integers(0, 30, (5, 5, 5, 5)) / 16.0
    z, c = cnn.forward(flat, x)
    for key in ("h1", "h2", "h3"):
        assert np.array_equal(cnn.bf16(c[key]), c[key])
    assert np.array_equal(c["h2"], cnn.bf16(np.maximum(c["a2"], 0)))


def test_sgd_step_closed_form():
    p = np.array([1.0, -2.0], np.float32)
    m = np.array([0.5, 0.0], np.float32)
    g = np.array([0.25, 1.0])
    p2, m2 = cnn.sgd_step(p, m, g, lr=0.1, momentum=0.9)
    assert np.allclose(m2, [0.7, 1.0]) and np.allclose(p2, [0.93, -2.1])


def test_rounded_grad_matches_torch_with_bf16_hooks():
    """With rounding on, the gradient equals torch's autograd on the same
    network with every weight, input and activation rounded to bfloat16 on
    the way forward and the hidden layers' backward signals rounded to
    bfloat16 on the way back (straight-through roundings, float64
    elsewhere): the precision contract of the matrix-core training kernels,
    built from torch's own bfloat16 conversion."""
    torch = pytest.importorskip("torch")

    def rb(t):  # torch's round to bfloat16, kept in float64
        return t.to(torch.bfloat16).to(torch.float64)

    class RoundFwd(torch.autograd.Function):  # forward rounding, gradient passes
        @staticmethod
        def forward(ctx, t):
            return rb(t)

        @staticmethod
        def backward(ctx, g):
            return g

    class RoundBwd(torch.autograd.Function):  # identity forward, rounded gradient
        @staticmethod
        def forward(ctx, t):
            return t.clone()

        @staticmethod
        def backward(ctx, g):
            return rb(g)

    rng = np.random.default_rng(8)
    flat = cnn.init_params(9)
    x = rng.integers(0, 30, (10, 5, 5, 5)) / 16.0
    y = (rng.uniform(size=10) > 0.5).astype(np.float64)
    loss, g, z = cnn.loss_and_grad(flat, x, y, pos_weight=3.0, rounding=True)
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True)
         for k, v in cnn.unpack(flat).items()}
    W = {k: RoundFwd.apply(v) if k[0] == "W" else v for k, v in P.items()}
    F = torch.nn.functional
    xt = rb(torch.tensor(x, dtype=torch.float64).unsqueeze(1))
    h1 = RoundBwd.apply(RoundFwd.apply(F.relu(F.conv3d(xt, W["W1"].reshape(16, 1, 3, 3, 3), W["b1"]))))
    h2 = F.relu(F.conv3d(h1, W["W2"].reshape(16, 16, 3, 3, 3), W["b2"])).reshape(-1, 16)
    h2 = RoundBwd.apply(RoundFwd.apply(h2))
    h3 = RoundBwd.apply(RoundFwd.apply(F.relu(h2 @ W["W3"].T + W["b3"])))
    zt = h3 @ W["W4"] + W["b4"]
    assert np.allclose(z, zt.detach().numpy(), rtol=1e-12, atol=1e-12)
    w = torch.tensor(np.where(y > 0.5, 3.0, 1.0))
    lt = (w * F.binary_cross_entropy_with_logits(zt, torch.tensor(y), reduction="none")).mean()
    lt.backward()
    gt = np.concatenate([P[name].grad.numpy().reshape(-1) for name, _ in cnn.SHAPES])
    assert np.allclose(g, gt, rtol=1e-9, atol=1e-14)
    # and the roundings matter: the unrounded backward differs
    _, g0, _ = cnn.loss_and_grad(flat, x, y, pos_weight=3.0, rounding=False)
    assert not np.allclose(g, g0, rtol=1e-6, atol=0)

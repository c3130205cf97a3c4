"""Pins of the surrogate's FP64 reference (no GPU): convolution against a
plain loop, gradients against central finite differences, GELU and Adam
against closed forms."""
import math

import numpy as np
import pytest
import torch

from oracle import surrogate as S


def naive_conv(x, w, b):
    cin, nz, ny, nx = x.shape
    cout = w.shape[0]
    out = np.zeros((cout, nz, ny, nx))
    xp = np.zeros((cin, nz + 2, ny + 2, nx + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    for co in range(cout):
        out[co] = b[co]
        for ci in range(cin):
            for a in range(3):
                for bb in range(3):
                    for c in range(3):
                        out[co] += w[co, ci, a, bb, c] * xp[ci, a:a + nz, bb:bb + ny, c:c + nx]
    return out


def test_conv_matches_plain_loop():
    g = np.random.default_rng(0)
    x = g.standard_normal((3, 4, 5, 6))
    w = g.standard_normal((4, 3, 3, 3, 3))
    b = g.standard_normal(4)
    ref = naive_conv(x, w, b)
    got = S.conv3(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b)).numpy()
    assert np.abs(got - ref).max() < 1e-12


def test_gelu_closed_form():
    x = torch.tensor([0.0, 1.0, -1.0, 3.0, -3.0, 10.0], dtype=torch.float64)
    y = S.gelu(x)
    assert y[0] == 0.0
    assert y[5] == pytest.approx(10.0, abs=1e-12)
    c = math.sqrt(2 / math.pi)
    assert y[1] == pytest.approx(0.5 * (1 + math.tanh(c * 1.044715)), rel=1e-15)
    assert torch.allclose(y, torch.nn.functional.gelu(x, approximate="tanh"), atol=1e-15)


def test_gradients_match_finite_differences():
    torch.manual_seed(0)
    chans = (3, 4, 4, 3)
    params = S.init_params(3, chans)
    g = np.random.default_rng(1)
    dm = torch.from_numpy(g.standard_normal((3, 3, 4, 5)))
    dh = torch.from_numpy(g.standard_normal((3, 3, 4, 5)))
    loss, grads = S.loss_and_grads(params, dm, dh)
    h = 1e-6
    rng = np.random.default_rng(2)
    for li, (w, b) in enumerate(params):
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in w.shape)
            wp = [(ww.clone(), bb.clone()) for ww, bb in params]
            wm = [(ww.clone(), bb.clone()) for ww, bb in params]
            wp[li][0][idx] += h
            wm[li][0][idx] -= h
            fd = (S.mse(S.forward(wp, dm)[0], dh) - S.mse(S.forward(wm, dm)[0], dh)).item() / (2 * h)
            assert grads[li][0][idx].item() == pytest.approx(fd, rel=1e-6, abs=1e-10)
        k = int(rng.integers(0, b.shape[0]))
        bp = [(ww.clone(), bb.clone()) for ww, bb in params]
        bm = [(ww.clone(), bb.clone()) for ww, bb in params]
        bp[li][1][k] += h
        bm[li][1][k] -= h
        fd = (S.mse(S.forward(bp, dm)[0], dh) - S.mse(S.forward(bm, dm)[0], dh)).item() / (2 * h)
        assert grads[li][1][k].item() == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_adam_first_step_is_signed_learning_rate():
    p = torch.tensor([1.0, -2.0, 3.0], dtype=torch.float64)
    gr = torch.tensor([0.5, -4.0, 1e-3], dtype=torch.float64)
    z = torch.zeros(3, dtype=torch.float64)
    p1, m, v = S.adam_update(p, gr, z, z, 1, lr=0.01)
    assert torch.allclose(p1, p - 0.01 * torch.sign(gr), atol=1e-7)


def test_adam_minimises_quadratic():
    p = torch.tensor([3.0, -1.0], dtype=torch.float64)
    m = torch.zeros(2, dtype=torch.float64)
    v = torch.zeros(2, dtype=torch.float64)
    for t in range(1, 2001):
        p, m, v = S.adam_update(p, 2 * p, m, v, t, lr=0.05)
    assert torch.abs(p).max() < 1e-3


def test_bf16_rounding_is_nearest_even():
    x = torch.tensor([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7], dtype=torch.float64)
    y = S.bf16(x)
    assert y.tolist() == [1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7]


def test_explicit_backward_equals_autograd_without_rounding():
    """The layer-by-layer backward (the form whose rounding points follow the
    matrix-core path) equals autograd's gradients when nothing is rounded."""
    chans = (3, 4, 5, 3)
    params = S.init_params(4, chans)
    g = np.random.default_rng(5)
    dm = torch.from_numpy(g.standard_normal((3, 3, 4, 5)))
    dh = torch.from_numpy(g.standard_normal((3, 3, 4, 5)))
    l0, g0 = S.loss_and_grads(params, dm, dh)
    l1, g1 = S.loss_and_grads_rounded(params, dm, dh)
    assert l1 == pytest.approx(l0, rel=1e-14)
    for (a, b), (c, d) in zip(g0, g1):
        assert torch.allclose(a, c, rtol=1e-12, atol=1e-14)
        assert torch.allclose(b, d, rtol=1e-12, atol=1e-14)


def test_gelu_prime_matches_finite_difference():
    x = torch.linspace(-4, 4, 41, dtype=torch.float64)
    h = 1e-6
    fd = (S.gelu(x + h) - S.gelu(x - h)) / (2 * h)
    assert torch.allclose(S.gelu_prime(x), fd, atol=1e-9)


def test_rounded_backward_rounds_where_stated():
    """With a rounding that zeroes everything the backward sees only zeros:
    the rounding is applied to the input (so the first layer's weight
    gradient vanishes) and to every dZ (so every gradient vanishes)."""
    chans = (3, 4, 3)
    params = S.init_params(6, chans)
    g = np.random.default_rng(7)
    dm = torch.from_numpy(g.standard_normal((3, 2, 3, 4)))
    dh = torch.from_numpy(g.standard_normal((3, 2, 3, 4)))
    _, gr = S.loss_and_grads_rounded(params, dm, dh, rnd=lambda t: t * 0.0)
    for w, b in gr:
        assert float(w.abs().max()) == 0.0 and float(b.abs().max()) == 0.0

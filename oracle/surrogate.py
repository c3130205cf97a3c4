"""FP64 reference of the learned demag surrogate (plain PyTorch CPU ops).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the GPU library
never imports it.

The network is a stack of six 3x3x3 convolutions (zero "same" padding, a
bias per output channel) with channels 3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 3
and a GELU (tanh form) after every layer but the last; it maps a
magnetisation increment dm = (M_stage - M_n)/Ms, laid out [3][nz][ny][nx],
to a demag-field increment dh = (H_d(M_stage) - H_d(M_n))/Ms.  The loss is
the mean squared error over all entries; training uses Adam.

Where the GPU rounds activations and weights to bfloat16 (its inputs to every
matrix-core product), the reference takes the same bfloat16-rounded tensors
as inputs and then computes in FP64, so the comparison isolates the
accumulation.
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

CHANNELS = (3, 32, 32, 32, 32, 32, 3)
TAPS = 27


def gelu(x: torch.Tensor) -> torch.Tensor:
    """GELU, tanh form: x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))."""
    return 0.5 * x * (1.0 + torch.tanh(math.sqrt(2.0 / math.pi) * (x + 0.044715 * x ** 3)))


def conv3(x: torch.Tensor, w: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """x [C_in][nz][ny][nx], w [C_out][C_in][3][3][3] (kz, ky, kx), b [C_out]:
    out[co][k][j][i] = b[co] + sum_{ci,a,b,c} w[co][ci][a][b][c] x[ci][k+a-1][j+b-1][i+c-1]."""
    return F.conv3d(x[None], w, b, padding=1)[0]


def forward(params, dm: torch.Tensor, bf16_between: bool = False):
    """params: list of (w, b) FP64 tensors.  Returns the output and the list of
    layer inputs (for inspection)."""
    x = dm
    acts = [x]
    for li, (w, b) in enumerate(params):
        y = conv3(x, w, b)
        if li < len(params) - 1:
            y = gelu(y)
            if bf16_between:
                y = y.to(torch.bfloat16).to(torch.float64)
        x = y
        acts.append(x)
    return x, acts


def mse(out: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    return ((out - target) ** 2).mean()


def loss_and_grads(params, dm, dh):
    """MSE loss and its gradients with respect to every weight and bias."""
    ps = [(w.clone().requires_grad_(True), b.clone().requires_grad_(True)) for w, b in params]
    out, _ = forward(ps, dm)
    loss = mse(out, dh)
    loss.backward()
    return loss.item(), [(w.grad.clone(), b.grad.clone()) for w, b in ps]


def gelu_prime(x: torch.Tensor) -> torch.Tensor:
    """Derivative of the tanh-form GELU: with u = sqrt(2/pi) (x + 0.044715
    x^3), d/dx [x/2 (1 + tanh u)] = (1 + tanh u)/2 + x/2 (1 - tanh^2 u) du/dx."""
    c = math.sqrt(2.0 / math.pi)
    t = torch.tanh(c * (x + 0.044715 * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * c * (1.0 + 3 * 0.044715 * x * x)


def loss_and_grads_rounded(params, dm, dh, rnd=None):
    """MSE loss and gradients by an explicit backward pass (chain rule
    written out layer by layer), with a rounding `rnd` applied where the
    half-precision matrix-core path stores a tensor: the network input and
    every layer input, every hidden pre-activation as the argument of the
    GELU derivative, and every back-propagated pre-activation gradient dZ.
    Arithmetic is FP64.  rnd = None is the exact backward (it must equal
    loss_and_grads)."""
    r = rnd if rnd is not None else (lambda t: t)
    n = len(params)
    X = [r(dm)]
    Zs = []
    for li, (w, b) in enumerate(params):
        z = conv3(X[-1], w, b)
        Zs.append(z)
        if li < n - 1:
            X.append(r(gelu(z)))
    out = Zs[-1]
    loss = mse(out, dh)
    dz = r(2.0 * (out - dh) / out.numel())
    grads = [None] * n
    for li in range(n - 1, -1, -1):
        w, b = params[li]
        x = X[li]
        # dL/dw[co][ci][a][b][c] = sum over cells of dz[co] x[ci] at the tap's source
        gw = torch.nn.grad.conv3d_weight(x[None], w.shape, dz[None], padding=1)
        grads[li] = (gw, dz.sum(dim=(1, 2, 3)))
        if li > 0:
            dx = torch.nn.grad.conv3d_input(x[None].shape, w, dz[None], padding=1)[0]
            dz = r(dx * gelu_prime(r(Zs[li - 1])))
    return loss.item(), grads


def init_params(seed: int, channels=CHANNELS):
    """He-style uniform initialisation, biases zero (seeded)."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        bound = math.sqrt(6.0 / (cin * TAPS)) * 0.5
        w = torch.from_numpy(g.uniform(-bound, bound, (cout, cin, 3, 3, 3)))
        out.append((w, torch.zeros(cout, dtype=torch.float64)))
    return out


def adam_update(p: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, t: int,
                lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma & Ba): returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (torch.sqrt(vh) + eps), m, v


def bf16(a) -> torch.Tensor:
    """Round to bfloat16 (nearest even) and back to FP64."""
    t = torch.as_tensor(a)
    return t.to(torch.bfloat16).to(torch.float64)

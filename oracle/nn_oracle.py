"""FP64 reference for training the learned a0 proposal (plain PyTorch, CPU).

TEST INFRASTRUCTURE ONLY: imported by tests and the smoke check.  The loss is
the negative log-likelihood of exact-sampler draws (alpha, a0) under the
proposal density q(a0 | alpha) = g'(a0) / 2 of a monotone rational-quadratic
spline flow g (Durkan et al. 2019) whose 47 parameters are the output of an
MLP 1 -> 32 -> 32 -> 47 (tanh, tanh, linear) of the feature
f(alpha) = 2 (ln alpha - ln 0.5) / (ln 30 - ln 0.5) - 1.  Gradients come from
torch autograd of this plain forward; the tests pin them to central finite
differences.  Parameter layout (2671 values): W1[32], b1[32], W2[32][32]
(row = output unit), b2[32], W3[47][32], b3[47].
"""
import math

import numpy as np
import torch

H, OUT, BINS, NPARAM = 32, 47, 16, 2671
MIN_BIN, MIN_DERIV = 1e-3, 1e-3
ALPHA_LO, ALPHA_HI = 0.5, 30.0


def unpack(p):
    p = torch.as_tensor(p, dtype=torch.float64)
    W1 = p[0:32].reshape(32, 1)
    b1 = p[32:64]
    W2 = p[64:1088].reshape(32, 32)
    b2 = p[1088:1120]
    W3 = p[1120:1120 + 1504].reshape(47, 32)
    b3 = p[2624:2671]
    return W1, b1, W2, b2, W3, b3


def feature(alpha):
    alpha = torch.as_tensor(alpha, dtype=torch.float64)
    return 2 * (torch.log(alpha) - math.log(ALPHA_LO)) / (math.log(ALPHA_HI) - math.log(ALPHA_LO)) - 1


def mlp(p, f):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    h1 = torch.tanh(f[:, None] * W1[:, 0][None, :] + b1)
    h2 = torch.tanh(h1 @ W2.T + b2)
    return h2 @ W3.T + b3


def knots(logits):
    w = MIN_BIN + (1 - BINS * MIN_BIN) * torch.softmax(logits, dim=-1)
    k = torch.cat([torch.full_like(w[:, :1], -1.0), -1.0 + torch.cumsum(2 * w, dim=-1)], dim=-1)
    return torch.cat([k[:, :-1], torch.ones_like(k[:, :1])], dim=-1)


def spline_params(raw):
    x = knots(raw[:, :BINS])
    y = knots(raw[:, BINS:2 * BINS])
    inner = MIN_DERIV + torch.nn.functional.softplus(raw[:, 2 * BINS:])
    one = torch.ones_like(inner[:, :1])
    d = torch.cat([one, inner, one], dim=-1)
    return x, y, d


def log_deriv(x, y, d, xv):
    """ln g'(xv) for each row (bin chosen by the knots, which carry gradients)."""
    k = torch.clamp((xv[:, None] >= x[:, 1:BINS]).sum(dim=-1), 0, BINS - 1)
    g = lambda t, o=0: t.gather(1, (k + o)[:, None])[:, 0]
    W = g(x, 1) - g(x)
    Hh = g(y, 1) - g(y)
    s = Hh / W
    xi = (xv - g(x)) / W
    om = xi * (1 - xi)
    dk, dk1 = g(d), g(d, 1)
    den = s + (dk1 + dk - 2 * s) * om
    num = dk1 * xi * xi + 2 * s * om + dk * (1 - xi) ** 2
    return 2 * torch.log(s) + torch.log(num) - 2 * torch.log(den)


def nll(params, alpha, a0):
    """Mean of -ln q(a0 | alpha) = -ln(1/2) - ln g'(a0)."""
    f = feature(alpha)
    raw = mlp(params, f)
    x, y, d = spline_params(raw)
    ld = log_deriv(x, y, d, torch.as_tensor(a0, dtype=torch.float64))
    return -(math.log(0.5) + ld).mean()


def loss_and_grad(params, alpha, a0):
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    loss = nll(p, alpha, a0)
    loss.backward()
    return float(loss.detach()), p.grad.numpy().copy()


def identity_raw_bias():
    """b3 that makes the spline the identity (uniform proposal) when W3 = 0."""
    b = np.zeros(OUT)
    b[2 * BINS:] = math.log(math.expm1(1.0 - MIN_DERIV))
    return b

"""Pins of the FP64 surrogate-MLP oracle: GELU values, bfloat16 rounding
(against hand-picked ties and torch's own bfloat16 conversion), the backward
pass against central finite differences, the bfloat16 mode of the network
against an independent realisation of the same rounding points, Adam's first
step and its closed forms over three steps."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M


def test_gelu_values_and_derivative():
    # GELU(z) = z Phi(z) with Phi the standard normal CDF: Phi(1) = 0.8413447461
    np.testing.assert_allclose(M.gelu([0.0, 1.0, -1.0, 2.0]),
                               [0.0, 0.8413447460685429, -0.15865525393145707, 1.9544997361036416], rtol=1e-12)
    z = np.linspace(-4, 4, 17)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(z), fd, atol=1e-8)


def test_bf16_rounding():
    ulp = 2.0 ** -7
    vals = [1.0, 1.0 + ulp / 2, 1.0 + 1.5 * ulp, 1.0 + 0.75 * ulp, -3.0, 0.0]
    want = [1.0, 1.0, 1.0 + 2 * ulp, 1.0 + ulp, -3.0, 0.0]  # ties go to the even mantissa
    np.testing.assert_array_equal(M.bf16_round(vals), want)


def _tiny(seed=0, dims=(5, 7, 6, 3)):
    rng = np.random.Generator(np.random.PCG64(seed))
    Ws = [rng.normal(0, 0.5, (dims[l + 1], dims[l])) for l in range(len(dims) - 1)]
    bs = [rng.normal(0, 0.1, dims[l + 1]) for l in range(len(dims) - 1)]
    X = rng.normal(0, 1, (4, dims[0]))
    Y = rng.normal(0, 1, (4, dims[-1]))
    return Ws, bs, X, Y


def test_backward_matches_central_fd():
    Ws, bs, X, Y = _tiny()
    loss, gW, gb = M.loss_and_grads(Ws, bs, X, Y)
    h = 1e-6
    for l in range(len(Ws)):
        for idx in [(0, 0), (1, 2), (Ws[l].shape[0] - 1, Ws[l].shape[1] - 1)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (M.loss_and_grads(Wp, bs, X, Y)[0] - M.loss_and_grads(Wm, bs, X, Y)[0]) / (2 * h)
            assert abs(fd - gW[l][idx]) <= 1e-7 * max(1.0, abs(fd))
        for j in range(bs[l].size):
            bp = [b.copy() for b in bs]
            bm = [b.copy() for b in bs]
            bp[l][j] += h
            bm[l][j] -= h
            fd = (M.loss_and_grads(Ws, bp, X, Y)[0] - M.loss_and_grads(Ws, bm, X, Y)[0]) / (2 * h)
            assert abs(fd - gb[l][j]) <= 1e-7 * max(1.0, abs(fd))


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = M.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-6)


def test_paper_sized_parameter_count():
    # 1536 -> 512 -> 512 -> 512 -> 512 -> 3
    dims = [1536, 512, 512, 512, 512, 3]
    assert sum(dims[l] * dims[l + 1] + dims[l + 1] for l in range(5)) == 1576451


# ---- the bfloat16 mode, pinned by an independent realisation -------------
# The kernels multiply bfloat16 operands with FP32 accumulation: every matrix
# that enters a product is a bfloat16 value -- the input, the weights, each
# hidden activation GELU(z) (forward operands) and each back-propagated
# dL/dz (the operand of both the weight-gradient and the input-gradient
# products).  Below, the same network is written with torch's autograd in
# float64: the chain rule comes from autograd (not from the oracle's
# hand-written backward), GELU and its derivative from torch, the rounding
# from torch's own bfloat16 conversion, and the rounding points are placed
# as identities around the operands: a forward rounding with a pass-through
# gradient on weights and activations, and a gradient rounding on every z.


def _torch_bf16_net(Ws, bs, X, Y):
    import torch
    import torch.nn.functional as F

    def rb(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    class RoundOperand(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            return rb(x)

        @staticmethod
        def backward(ctx, g):
            return g

    class RoundGradient(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            return x.clone()

        @staticmethod
        def backward(ctx, g):
            return rb(g)

    W = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in Ws]
    b = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in bs]
    x = rb(torch.tensor(X, dtype=torch.float64))
    for l in range(len(W)):
        z = RoundGradient.apply(x @ RoundOperand.apply(W[l]).T + b[l])
        if l < len(W) - 1:
            x = RoundOperand.apply(F.gelu(z))
    loss = ((z - torch.tensor(Y, dtype=torch.float64)) ** 2).mean()
    loss.backward()
    return z.detach().numpy(), float(loss.detach()), [w.grad.numpy() for w in W], [v.grad.numpy() for v in b]


def test_bf16_rounding_matches_torch_bfloat16():
    import torch

    rng = np.random.Generator(np.random.PCG64(3))
    vals = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-30, 100), rng.normal(0, 1e30, 100)])
    # exact ties between two bfloat16 neighbours (odd and even lower mantissa)
    mant = rng.integers(0, 1 << 7, 200)
    ties = (1.0 + mant / 128.0 + 1.0 / 256.0) * np.exp2(rng.integers(-20, 20, 200))
    vals = np.concatenate([vals, ties, -ties]).astype(np.float32)
    want = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16_round(vals), want)


@pytest.mark.parametrize("dims,B,seed", [((5, 7, 6, 3), 4, 0), ((12, 16, 16, 16, 2), 9, 1), ((33, 8, 3), 17, 2)])
def test_bf16_network_matches_independent_realisation(dims, B, seed):
    Ws, bs, X, Y = _tiny(seed, dims)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    X = rng.normal(0, 1, (B, dims[0]))
    Y = rng.normal(0, 1, (B, dims[-1]))
    out, loss, gW, gb = _torch_bf16_net(Ws, bs, X, Y)
    ro, _ = M.forward(Ws, bs, X, bf16=True)
    rl, rW, rb_ = M.loss_and_grads(Ws, bs, X, Y, bf16=True)
    np.testing.assert_allclose(ro, out, rtol=1e-12, atol=1e-14)
    assert abs(rl - loss) <= 1e-12 * loss
    for l in range(len(Ws)):
        np.testing.assert_allclose(rW[l], gW[l], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(rb_[l], gb[l], rtol=1e-12, atol=1e-14)
    # and the rounding is not a no-op here: the FP64 network differs
    r64 = M.loss_and_grads(Ws, bs, X, Y, bf16=False)
    assert max(np.abs(a - c).max() for a, c in zip(r64[1], rW)) > 1e-6


# ---- Adam beyond its first step: closed forms ------------------------------
# From zero moments with a constant gradient g the bias-corrected moments are
# exactly g and g^2 at every t, so every step moves -lr g / (|g| + eps).  With
# g, -g, g the corrected first moment is g, -(1 - b1)/(1 + b1) g and
# (1 - b1 + b1^2)/(1 + b1 + b1^2) g, the corrected second moment g^2 each time
# (sum the geometric series of m_t and v_t by hand).


def test_adam_constant_gradient_steps_are_signed_lr():
    g = np.array([0.3, -2.0, 1e-3, 7.5])
    lr, eps = 0.01, 1e-8
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in (1, 2, 3):
        p, m, v = M.adam_step(p, g, m, v, t, lr=lr, eps=eps)
        np.testing.assert_allclose(p, -t * lr * g / (np.abs(g) + eps), rtol=1e-12)


@pytest.mark.parametrize("b1,b2", [(0.9, 0.999), (0.5, 0.75)])
def test_adam_alternating_gradient_closed_form(b1, b2):
    g = np.array([0.3, -2.0, 1e-3, 7.5])
    lr, eps = 0.01, 1e-8
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    unit = g / (np.abs(g) + eps)
    want = [-lr * unit, lr * (1 - b1) / (1 + b1) * unit, -lr * (1 - b1 + b1 * b1) / (1 + b1 + b1 * b1) * unit]
    for t, sgn in ((1, 1.0), (2, -1.0), (3, 1.0)):
        p0 = p
        p, m, v = M.adam_step(p, sgn * g, m, v, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
        np.testing.assert_allclose(p - p0, want[t - 1], rtol=1e-9)

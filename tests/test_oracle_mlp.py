"""Pins of the FP64 surrogate-MLP oracle: GELU values, bfloat16 rounding,
the backward pass against central finite differences, and Adam's first
step."""
import math

import numpy as np

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

"""Surrogate MLP kernels: the BF16 MFMA GEMM against an FP64 product of the
same bfloat16 values, and the network's forward pass, gradients and training
against the FP64 oracle with bfloat16 rounding at the same points, and
against the exact FP64 network within a bound derived from bfloat16's unit
roundoff.

Tolerances (the method fixes none): every GEMM output element within the
error bound of FP32 summation in any order, gamma_K sum_k |a_ik b_kj| with
gamma_K = K u / (1 - K u), u = 2^-24 (products of two bfloat16 values are
exact in FP32, so only the sums round); network outputs against the
bfloat16-mode oracle normwise <= 1e-2 and gradients cosine >= 0.999,
normwise <= 2e-2 (a value that lands near a bfloat16 tie may round either
way, one bfloat16 ulp apart); against the exact network, every element
within the running first-order bound below."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as MO

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24  # FP32 unit roundoff
U16 = 2.0 ** -8   # bfloat16 unit roundoff (8 significant bits)


def _gamma(k, u=U32):
    return k * u / (1.0 - k * u)


def _bf16_bits(a):
    f = np.asarray(MO.bf16_round(a), np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def _gemm_case(ta, tb, shape):
    import torch

    from paper_1911_10274_amd import titan as T

    M, N, K = shape
    print(f"gemm case ta={ta} tb={tb} M={M} N={N} K={K}", flush=True)
    rng = np.random.Generator(np.random.PCG64(M * 7 + N * 3 + K + 11 * ta + 5 * tb))
    A = rng.normal(0, 1, (M, K))
    B = rng.normal(0, 1, (K, N))
    Ab, Bb = MO.bf16_round(A), MO.bf16_round(B)
    a_store = (_bf16_bits(A).T if ta else _bf16_bits(A)).copy()
    b_store = (_bf16_bits(B).T if tb else _bf16_bits(B)).copy()
    dA = torch.from_numpy(a_store.view(np.int16)).cuda()
    dB = torch.from_numpy(b_store.view(np.int16)).cuda()
    C = T.gemm_bf16(dA, dB, ta=bool(ta), tb=bool(tb), M=M, N=N, K=K)
    torch.cuda.synchronize()
    want = Ab @ Bb
    bound = _gamma(K) * (np.abs(Ab) @ np.abs(Bb))
    got = C.cpu().numpy().astype(np.float64)
    err = np.abs(got - want)
    worst = float((err / np.maximum(bound, 1e-300)).max())
    print(f"  worst error / bound {worst:.3g}")
    assert np.all(err <= bound), worst


@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("tb", [0, 1])
# outputs of fewer than 128 tiles of 256 x 256 take the 64 x 64 kernel
@pytest.mark.parametrize("shape", [(64, 64, 32), (100, 70, 48), (1, 3, 512), (257, 129, 1536), (1024, 2048, 96),
                                   (1100, 1900, 200)])
def test_gemm_bf16_layouts(ta, tb, shape):
    _gemm_case(ta, tb, shape)


@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("tb", [0, 1])
# outputs of at least 128 tiles of 256 x 256 take the big-tile kernel: exactly
# 8 x 16 tiles with a K that ends inside a 64-wide K step, and 9 x 17 / 17 x 9
# tiles ragged in M, N and K
@pytest.mark.parametrize("shape", [(2048, 4096, 96), (2085, 4115, 200), (4100, 2100, 200)])
def test_gemm_bf16_layouts_big_tiles(ta, tb, shape):
    M, N, _ = shape
    assert ((M + 255) // 256) * ((N + 255) // 256) >= 128
    _gemm_case(ta, tb, shape)


@pytest.mark.parametrize("shape", [(2085, 4115, 200), (2048, 4096, 61)])
def test_big_tile_layouts_agree_bit_for_bit(shape):
    """A large product whose K is strided in an operand runs on a
    K-contiguous copy of that operand (rows padded to 16 bytes: K = 61 leaves
    three values of padding per row), so all four layouts of one product give
    the same bits."""
    import torch

    from paper_1911_10274_amd import titan as T

    M, N, K = shape
    rng = np.random.Generator(np.random.PCG64(M + N + K))
    a = _bf16_bits(rng.normal(0, 1, (M, K)))
    b = _bf16_bits(rng.normal(0, 1, (K, N)))
    outs = []
    for ta in (0, 1):
        for tb in (0, 1):
            dA = torch.from_numpy((a.T if ta else a).copy().view(np.int16)).cuda()
            dB = torch.from_numpy((b.T if tb else b).copy().view(np.int16)).cuda()
            outs.append(T.gemm_bf16(dA, dB, ta=bool(ta), tb=bool(tb), M=M, N=N, K=K).cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def _init(dims, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    Ws = [rng.uniform(-1, 1, (dims[l + 1], dims[l])) * np.sqrt(3.0 / dims[l]) for l in range(len(dims) - 1)]
    bs = [rng.uniform(-0.1, 0.1, dims[l + 1]) for l in range(len(dims) - 1)]
    flat = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(Ws, bs)]).astype(np.float32)
    return [W.astype(np.float32).astype(np.float64) for W in Ws], [b.astype(np.float32).astype(np.float64) for b in bs], flat


def _split(flat, dims):
    gW, gb, o = [], [], 0
    for l in range(len(dims) - 1):
        n = dims[l] * dims[l + 1]
        gW.append(flat[o:o + n].reshape(dims[l + 1], dims[l]))
        o += n
        gb.append(flat[o:o + dims[l + 1]])
        o += dims[l + 1]
    return gW, gb


def _net_case(dims, B, seed=5, data_seed=6):
    """GPU forward and gradients on one batch against the bfloat16-mode oracle."""
    from paper_1911_10274_amd import titan as T

    print(f"network {dims} batch {B}", flush=True)
    Ws, bs, flat = _init(dims, seed)
    rng = np.random.Generator(np.random.PCG64(data_seed))
    X = rng.normal(0, 1, (B, dims[0])).astype(np.float32)
    Y = rng.normal(0, 1, (B, dims[-1])).astype(np.float32)
    net = T.Mlp(dims)
    assert net.n_params == flat.size
    net.set_params(flat)
    np.testing.assert_array_equal(net.get_params(), flat)
    out = net.predict(X)
    ref, _ = MO.forward(Ws, bs, X.astype(np.float64), bf16=True)
    e = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    print("forward", e)
    assert e <= 1e-2
    loss, g = net.grad(X, Y)
    rl, rW, rb = MO.loss_and_grads(Ws, bs, X.astype(np.float64), Y.astype(np.float64), bf16=True)
    assert abs(loss - rl) <= 1e-2 * rl
    gW, gb = _split(g.astype(np.float64), dims)
    for l in range(len(dims) - 1):
        for got, want in ((gW[l], rW[l]), (gb[l], rb[l])):
            got, want = got.ravel(), want.ravel()
            cos = got @ want / (np.linalg.norm(got) * np.linalg.norm(want))
            rel = np.linalg.norm(got - want) / np.linalg.norm(want)
            print("layer", l, "cos", cos, "rel", rel)
            assert cos >= 0.999 and rel <= 2e-2
    net.close()


# B = 1024 and 1000: the training batch, where the weight-gradient products
# (and their ones column, the bias gradient) run split over K; 1000 is ragged.
# Up to four outputs the output layer, the loss and the first input gradient
# run as one fused kernel (one, three and four outputs; a single layer has no
# input gradient); more outputs take the general products.
@pytest.mark.parametrize("dims,B", [([40, 64, 64, 3], 33), ([1536, 512, 512, 512, 512, 3], 128),
                                    ([1536, 512, 512, 512, 512, 3], 1024), ([1536, 512, 512, 512, 512, 3], 1000),
                                    ([40, 64, 64, 1], 70), ([30, 72, 4], 65), ([24, 4], 50), ([40, 64, 64, 7], 33),
                                    ([100, 9], 77)])
def test_mlp_forward_and_gradients_match_oracle(dims, B):
    _net_case(dims, B)


# Every epilogue through the big-tile kernel (outputs of >= 128 tiles of
# 256 x 256).  Narrow layers at a batch of 32,768 (+ 37: ragged in M): the
# forward products (bias + GELU, and the last layer's bias) and the
# input-gradient product (GELU') have 129 row tiles.  A 2048 -> 4096 layer:
# its weight-gradient product (dz^T [x, 1], 4096 x 2049, the ones column
# giving the bias gradient) has 16 x 9 tiles, over a ragged K = batch = 100.
@pytest.mark.parametrize("dims,B", [([8, 16, 3], 32768 + 37), ([2048, 4096, 3], 100)])
def test_mlp_epilogues_on_big_tiles(dims, B):
    _net_case(dims, B, seed=7, data_seed=8)


# ---- against the exact network -------------------------------------------
# Here the weights are bfloat16 values (the format the products read them in),
# so the GPU network and the exact FP64 network (the oracle without rounding)
# have the same parameters; they differ by the bfloat16 rounding of the
# input, of every hidden activation and of every back-propagated dL/dz, and
# by FP32 sums (about 2^-16 of the bfloat16 terms, neglected).  Model of the
# rounding (probabilistic rounding-error analysis): each rounding multiplies
# a value by (1 + d), d independent and uniform on [-U16, U16], variance
# U16^2 / 3.  Propagated to first order, layer by layer, this gives every
# output and gradient element a standard deviation sigma; the errors are sums
# of many independent roundings, so the test asks for |error| <= 6.5 sigma per
# element and a normwise ratio ||error|| / ||sigma|| <= 2 (3 for arrays of
# fewer than 64 elements).
V16 = U16 * U16 / 3.0


def _exact_network_sigma(Ws, bs, X, Y):
    L = len(Ws)
    out, (xs, zs) = MO.forward(Ws, bs, X, bf16=False)
    W2 = [W * W for W in Ws]
    vx = [V16 * X * X]
    vz = []
    for l in range(L):
        vz.append(vx[l] @ W2[l].T)
        if l < L - 1:
            gp = MO.gelu_grad(zs[l])
            vx.append(gp * gp * vz[l] + V16 * xs[l + 1] ** 2)
    n = out.size
    dz = 2.0 * (out - Y) / n
    vdz = (2.0 / n) ** 2 * vz[-1] + V16 * dz * dz
    gW, gb, sW, sb = [None] * L, [None] * L, [None] * L, [None] * L
    for l in range(L - 1, -1, -1):
        gW[l] = dz.T @ xs[l]
        gb[l] = dz.sum(axis=0)
        sW[l] = np.sqrt(vdz.T @ xs[l] ** 2 + (dz * dz).T @ vx[l])
        sb[l] = np.sqrt(vdz.sum(axis=0))
        if l > 0:
            dx = dz @ Ws[l]
            z = zs[l - 1]
            gp = MO.gelu_grad(z)
            gpp = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi) * (2.0 - z * z)  # GELU''
            vdz = gp * gp * (vdz @ W2[l]) + (dx * gpp) ** 2 * vz[l - 1] + V16 * (dx * gp) ** 2
            dz = dx * gp
    return out, np.sqrt(vz[-1]), gW, gb, sW, sb


def _within_sigma(label, got, want, sigma):
    e = np.abs(np.asarray(got, np.float64) - want).ravel()
    s = np.maximum(np.asarray(sigma).ravel(), 1e-300)
    elem, norm = float((e / s).max()), float(np.linalg.norm(e) / np.linalg.norm(s))
    print(f"{label}: worst error / sigma {elem:.2f}, normwise {norm:.2f}, relative error "
          f"{np.linalg.norm(e) / np.linalg.norm(want):.2e}")
    assert elem <= 6.5 and norm <= (2.0 if e.size >= 64 else 3.0), (label, elem, norm)


def test_mlp_against_exact_network_within_bf16_rounding():
    from paper_1911_10274_amd import titan as T

    dims, B = [1536, 512, 512, 512, 512, 3], 1024
    Ws, bs, _ = _init(dims, 5)
    Ws = [MO.bf16_round(W) for W in Ws]
    flat = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(Ws, bs)]).astype(np.float32)
    rng = np.random.Generator(np.random.PCG64(6))
    X = rng.normal(0, 1, (B, dims[0])).astype(np.float32)
    Y = rng.normal(0, 1, (B, dims[-1])).astype(np.float32)
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    out, sout, gW, gb, sW, sb = _exact_network_sigma(Ws, bs, X64, Y64)
    # the model's own backward recurrence reproduces the oracle's exact gradients
    _, rW, rb = MO.loss_and_grads(Ws, bs, X64, Y64, bf16=False)
    for l in range(len(Ws)):
        np.testing.assert_allclose(gW[l], rW[l], rtol=1e-9, atol=1e-15)
        np.testing.assert_allclose(gb[l], rb[l], rtol=1e-9, atol=1e-15)
    net = T.Mlp(dims)
    net.set_params(flat)
    _within_sigma("output", net.predict(X), out, sout)
    _, g = net.grad(X, Y)
    GW, Gb = _split(g.astype(np.float64), dims)
    for l in range(len(Ws)):
        _within_sigma(f"layer {l} dW", GW[l], gW[l], sW[l])
        _within_sigma(f"layer {l} db", Gb[l], gb[l], sb[l])
    net.close()


def test_gradients_across_batch_sizes_on_one_network():
    """One network, batches of 128, 1024 (its buffers grow) and then 1000
    and 64 (they do not): the activations' ones column, which turns the
    weight-gradient product into the bias gradient too, must hold each time."""
    from paper_1911_10274_amd import titan as T

    dims = [96, 64, 64, 3]
    Ws, bs, flat = _init(dims, 21)
    net = T.Mlp(dims)
    net.set_params(flat)
    for B in (128, 1024, 1000, 64):
        rng = np.random.Generator(np.random.PCG64(B))
        X = rng.normal(0, 1, (B, dims[0])).astype(np.float32)
        Y = rng.normal(0, 1, (B, dims[-1])).astype(np.float32)
        _, g = net.grad(X, Y)
        _, rW, rb = MO.loss_and_grads(Ws, bs, X.astype(np.float64), Y.astype(np.float64), bf16=True)
        gW, gb = _split(g.astype(np.float64), dims)
        for l in range(len(dims) - 1):
            for got, want in ((gW[l], rW[l]), (gb[l], rb[l])):
                got, want = got.ravel(), want.ravel()
                rel = np.linalg.norm(got - want) / np.linalg.norm(want)
                assert rel <= 2e-2, (B, l, rel)
    net.close()


# 21 inputs: the batch gather copies element by element (rows of a multiple
# of 8 values go 16 bytes at a time)
@pytest.mark.parametrize("n_in", [24, 21])
def test_adam_step_matches_reference_and_training_learns(n_in):
    from paper_1911_10274_amd import titan as T

    dims = [n_in, 64, 64, 2]
    Ws, bs, flat = _init(dims, 9)
    rng = np.random.Generator(np.random.PCG64(10))
    X = rng.normal(0, 1, (2048, dims[0])).astype(np.float32)
    wt = rng.normal(0, 1, (dims[0], dims[-1]))
    Y = np.tanh(X.astype(np.float64) @ wt / 3).astype(np.float32)
    net = T.Mlp(dims)
    net.set_params(flat)
    net.set_data(X, Y)
    # three Adam steps on different batches, each against the oracle's update
    # from the same gradient (the bias corrections change with t)
    p = flat.astype(np.float64)
    m = v = 0.0
    for t in (1, 2, 3):
        rows = np.arange(64 * (t - 1), 64 * t, dtype=np.int64)
        loss, g = net.grad(X[rows], Y[rows])
        # the training step gathers the same rows from the resident data set
        # and reports the loss at the parameters it starts from: bit for bit
        # what the gradient call on the uploaded batch gave
        step_loss = net.train(rows[None, :], lr=1e-3)
        assert np.float32(step_loss[0]) == np.float32(loss), (t, step_loss, loss)
        got = net.get_params().astype(np.float64)
        p, m, v = MO.adam_step(p, g.astype(np.float64), m, v, t, lr=1e-3)
        err = np.abs(got - p).max()
        print("adam step", t, "max |GPU - oracle|", err)
        assert err <= 2e-7, (t, err)
        p = got  # continue from the GPU's FP32 parameters
    # a few epochs of mini-batch Adam reduce the loss substantially
    steps = []
    for ep in range(15):
        perm = rng.permutation(2048)
        steps.append(net.train(perm.reshape(-1, 128), lr=3e-3))
    first, last = float(np.mean(steps[0])), float(np.mean(steps[-1]))
    print("loss", first, last)
    assert last < 0.2 * first
    net.close()


def test_long_training_call_reports_every_step_loss():
    """A training call of more steps than the loss buffer holds (its per-row
    squared errors are summed every 1024 steps) equals the same steps taken in
    calls of 100: every step's loss and the final parameters, bit for bit."""
    from paper_1911_10274_amd import titan as T

    dims = [8, 16, 2]
    _, _, flat = _init(dims, 31)
    rng = np.random.Generator(np.random.PCG64(32))
    X = rng.normal(0, 1, (64, dims[0])).astype(np.float32)
    Y = rng.normal(0, 1, (64, dims[-1])).astype(np.float32)
    idx = rng.integers(0, 64, (1100, 4))
    nets = [T.Mlp(dims), T.Mlp(dims)]
    for net in nets:
        net.set_params(flat)
        net.set_data(X, Y)
    one = nets[0].train(idx, lr=1e-3)
    parts = np.concatenate([nets[1].train(idx[a:a + 100], lr=1e-3) for a in range(0, 1100, 100)])
    assert one.shape == (1100,) and np.all(np.isfinite(one))
    assert np.array_equal(one, parts)
    assert np.array_equal(nets[0].get_params(), nets[1].get_params())
    for net in nets:
        net.close()

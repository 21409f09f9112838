"""Surrogate MLP kernels: the BF16 MFMA GEMM against an FP64 product of the
same bfloat16 values, and the network's forward pass, gradients and training
against the FP64 oracle with bfloat16 rounding at the same points.

Tolerances (the method fixes none): GEMM relative error <= 1e-5 (bf16 products
are exact in FP32; only the FP32 sum order differs); network outputs
normwise <= 1e-2 and gradients cosine >= 0.999, normwise <= 2e-2 (rounding a
value that lands near a bfloat16 tie either way moves it by one bf16 ulp)."""
import numpy as np
import pytest

from oracle import mlp_oracle as MO

pytestmark = pytest.mark.gpu


def _bf16_bits(a):
    f = np.asarray(MO.bf16_round(a), np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("tb", [0, 1])
# the last two take the 128 x 128 kernel (outputs of >= 128 such tiles), the
# last one with ragged edges in M, N and K
@pytest.mark.parametrize("shape", [(64, 64, 32), (100, 70, 48), (1, 3, 512), (257, 129, 1536), (1024, 2048, 96),
                                   (1100, 1900, 200)])
def test_gemm_bf16_layouts(ta, tb, shape):
    import torch

    from paper_1911_10274_amd import titan as T

    M, N, K = shape
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
    got = C.cpu().numpy().astype(np.float64)
    err = np.abs(got - want).max() / max(np.abs(want).max(), 1e-30)
    assert err <= 1e-5, err


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


# B = 1024 and 1000: the training batch, where every weight-gradient product
# (and its ones column, the bias gradient) runs split over K; 1000 is ragged
@pytest.mark.parametrize("dims,B", [([40, 64, 64, 3], 33), ([1536, 512, 512, 512, 512, 3], 128),
                                    ([1536, 512, 512, 512, 512, 3], 1024), ([1536, 512, 512, 512, 512, 3], 1000)])
def test_mlp_forward_and_gradients_match_oracle(dims, B):
    from paper_1911_10274_amd import titan as T

    Ws, bs, flat = _init(dims, 5)
    rng = np.random.Generator(np.random.PCG64(6))
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


def test_adam_step_matches_reference_and_training_learns():
    from paper_1911_10274_amd import titan as T

    dims = [24, 64, 64, 2]
    Ws, bs, flat = _init(dims, 9)
    rng = np.random.Generator(np.random.PCG64(10))
    X = rng.normal(0, 1, (2048, dims[0])).astype(np.float32)
    wt = rng.normal(0, 1, (dims[0], dims[-1]))
    Y = np.tanh(X.astype(np.float64) @ wt / 3).astype(np.float32)
    net = T.Mlp(dims)
    net.set_params(flat)
    net.set_data(X, Y)
    idx = np.arange(64, dtype=np.int64)[None, :]
    loss0, g = net.grad(X[:64], Y[:64])
    net.train(idx, lr=1e-3)
    p1 = net.get_params()
    want, _, _ = MO.adam_step(flat.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, lr=1e-3)
    np.testing.assert_allclose(p1, want, rtol=0, atol=1e-6)
    # a few epochs of mini-batch Adam reduce the loss substantially
    steps = []
    for ep in range(15):
        perm = rng.permutation(2048)
        steps.append(net.train(perm.reshape(-1, 128), lr=3e-3))
    first, last = float(np.mean(steps[0])), float(np.mean(steps[-1]))
    print("loss", first, last)
    assert last < 0.2 * first
    net.close()

// Surrogate MLP: BF16 matrix-core (MFMA) GEMMs with FP32 accumulation and
// fused epilogues, its backward pass and Adam, behind the titan_mlp_* C ABI.
//
// Network: x_0 = input; hidden layers z_l = x_l W_l^T + b_l,
// x_{l+1} = GELU(z_l) (exact erf form); the last layer is linear.  Weights
// and activations are stored in bfloat16 for the GEMMs, pre-activations and
// the output in FP32; master weights and Adam moments in FP32.  Loss: mean
// squared error.  Backward: dz_L = 2 (out - y) / (B O);
// dW_l = dz_l^T x_l, db_l = column sums of dz_l,
// dz_{l-1} = (dz_l W_l) * GELU'(z_{l-1})  -- the GELU derivative is applied in
// the epilogue of the dgrad GEMM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "titan.h"
#include "titan_sim.h"

namespace titan {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum Epi { EPI_BIAS_GELU = 1, EPI_BIAS = 2, EPI_GELU_BWD = 3, EPI_F32 = 4, EPI_WGRAD = 5 };

struct GemmEpi {
    const float *bias;  // [N]
    float *Z;           // fp32 out (pre-activation / output / C), row stride ldz
    const float *Zin;   // fp32 pre-activation read by EPI_GELU_BWD, row stride ldz
    uint16_t *Yb;       // bf16 out, row stride ldy
    int ldz, ldy;
    float *db;          // EPI_WGRAD: column ldz (the activations' ones column) -> db[row]
};

constexpr int BM = 64, BN = 64, BK = 64, LDK = BK + 8;

// Epilogue of output element (i, j) with accumulated value v.
template <int EPI>
__device__ __forceinline__ void epi_store(int i, int j, float v, const GemmEpi &ep)
{
    if (EPI == EPI_BIAS_GELU) {
        const float z = v + ep.bias[j];
        ep.Z[(int64_t)i * ep.ldz + j] = z;
        ep.Yb[(int64_t)i * ep.ldy + j] = f2bf(gelu(z));
    } else if (EPI == EPI_BIAS) {
        ep.Z[(int64_t)i * ep.ldz + j] = v + ep.bias[j];
    } else if (EPI == EPI_GELU_BWD) {
        ep.Yb[(int64_t)i * ep.ldy + j] = f2bf(v * gelu_grad(ep.Zin[(int64_t)i * ep.ldz + j]));
    } else if (EPI == EPI_WGRAD) {
        // dW = dz^T x over the activations and their ones column: the last
        // column is the column sum of dz, the bias gradient
        if (j < ep.ldz)
            ep.Z[(int64_t)i * ep.ldz + j] = v;
        else
            ep.db[i] = v;
    } else {
        ep.Z[(int64_t)i * ep.ldz + j] = v;
    }
}

struct GemmArgs {
    int M, N, K;
    const uint16_t *A;
    int lda;
    const uint16_t *B;
    int ldb;
    int kslice;   // K range of one split (a multiple of BK)
    float *part;  // split-K partial sums [splits][M][N], or null: epilogue here
};

// One operand tile (64 rows x BK of K) moved global -> registers -> LDS, the
// LDS tile holding K contiguous per row.  KCONTIG: element (r, k) at
// P[r * ld + k] (K contiguous in memory): each of the 256 threads moves two
// 16-byte chunks of 8 K-values.  Otherwise element (r, k) at P[k * ld + r]:
// each thread moves a block of 8 K-values x 2 rows, read as eight 4-byte
// pieces along the rows (32 consecutive threads cover one 128-byte K row),
// transposed in registers and stored as two 16-byte LDS writes.
template <bool KCONTIG>
struct TileMove {
    u32x4 v[2];

    // FAST: the caller has checked that the whole tile is in range and the
    // vector loads aligned.  Otherwise element loads at clamped positions
    // (R >= 1 rows and K values up to kend >= 1 exist) with zero fill.
    // Neither form branches per lane, so the compiler can count each load's
    // completion exactly instead of waiting for all of them.
    template <bool FAST>
    __device__ __forceinline__ void load(const uint16_t *P, int ld, int r0, int R, int k0, int kend, int tid)
    {
        if (KCONTIG) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int c = tid + 256 * q;
                const int row = r0 + (c >> 3), k = k0 + (c & 7) * 8;
                if (FAST) {
                    v[q] = *(const u32x4 *)(P + (int64_t)row * ld + k);
                } else {
                    // element loads at clamped (always valid) positions, out
                    // of range ones replaced by zero: no branch
                    const int64_t rr = (int64_t)min(row, R - 1) * ld;
                    uint32_t w[4];
#pragma unroll
                    for (int e = 0; e < 8; e += 2) {
                        const uint32_t x0 = P[rr + min(k + e, kend - 1)];
                        const uint32_t x1 = P[rr + min(k + e + 1, kend - 1)];
                        w[e / 2] = (row < R && k + e < kend ? x0 : 0u) | (row < R && k + e + 1 < kend ? x1 : 0u) << 16;
                    }
                    v[q] = u32x4{w[0], w[1], w[2], w[3]};
                }
            }
        } else {
            const int kb = k0 + 8 * (tid >> 5), rb = r0 + 2 * (tid & 31);
            uint32_t in[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = kb + e;
                if (FAST) {
                    in[e] = *(const uint32_t *)(P + (int64_t)k * ld + rb);
                } else {
                    const int64_t kk = (int64_t)min(k, kend - 1) * ld;
                    const uint32_t x0 = P[kk + min(rb, R - 1)];
                    const uint32_t x1 = P[kk + min(rb + 1, R - 1)];
                    in[e] = (k < kend && rb < R ? x0 : 0u) | (k < kend && rb + 1 < R ? x1 : 0u) << 16;
                }
            }
            // v[n] = the 8 K-values of row rb + n
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                uint32_t w[4];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    w[j] = n ? ((in[2 * j] >> 16) | (in[2 * j + 1] & 0xFFFF0000u))
                             : ((in[2 * j] & 0xFFFFu) | (in[2 * j + 1] << 16));
                v[n] = u32x4{w[0], w[1], w[2], w[3]};
            }
        }
    }

    __device__ __forceinline__ void store(uint16_t *S, int tid) const
    {
        if (KCONTIG) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int c = tid + 256 * q;
                *(u32x4 *)&S[(c >> 3) * LDK + (c & 7) * 8] = v[q];
            }
        } else {
            const int kb = 8 * (tid >> 5), rb = 2 * (tid & 31);
#pragma unroll
            for (int n = 0; n < 2; ++n)
                *(u32x4 *)&S[(rb + n) * LDK + kb] = v[n];
        }
    }
};

// One chunk of NK K tiles of the 64 x 64 kernel, from c0: all NK tiles'
// loads first, then per tile the LDS store (alternating buffers, by the
// tile's index in the split), one barrier and four MFMAs per wave.  FA / FB:
// operand A / B of the whole chunk is in range and aligned for vector loads
// (uniform over the workgroup); the chunk's tiles past ke are skipped.
template <bool TA, bool TB, int NK, bool FA, bool FB>
__device__ __forceinline__ void gemm_chunk(const GemmArgs &g, int c0, int kb, int ke, int m0, int n0, int tid,
                                           uint16_t (*sA)[BM * LDK], uint16_t (*sB)[BN * LDK], f32x16_t &acc)
{
    const int lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
    TileMove<!TA> ta[NK];
    TileMove<TB> tb[NK];
    // a stage past the range loads zeros (its K values are all >= ke)
#pragma unroll
    for (int s = 0; s < NK; ++s) {
        ta[s].template load<FA>(g.A, g.lda, m0, g.M, c0 + s * BK, ke, tid);
        tb[s].template load<FB>(g.B, g.ldb, n0, g.N, c0 + s * BK, ke, tid);
    }
    const int t0 = (c0 - kb) / BK;  // K tiles of the split before this chunk
#pragma unroll
    for (int s = 0; s < NK; ++s) {
        if (c0 + s * BK < ke) {  // uniform over the workgroup
            uint16_t *a = sA[(t0 + s) & 1], *b = sB[(t0 + s) & 1];
            ta[s].store(a, tid);
            tb[s].store(b, tid);
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < BK; kk += 16) {
                const bf16x8_t av = *(const bf16x8_t *)&a[(wm * 32 + (lane & 31)) * LDK + kk + 8 * (lane >> 5)];
                const bf16x8_t bv = *(const bf16x8_t *)&b[(wn * 32 + (lane & 31)) * LDK + kk + 8 * (lane >> 5)];
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
            }
        }
    }
}

// C[M,N] = A[M,K] B[K,N] with A(m,k) = TA ? A[k*lda + m] : A[m*lda + k] and
// B(k,n) = TB ? B[n*ldb + k] : B[k*ldb + n], all bf16; FP32 accumulate on
// v_mfma_f32_32x32x16_bf16.  A 64x64 tile per workgroup, 32x32 per wave;
// workgroup z takes K range [z*kslice, (z+1)*kslice).  Tiles are staged in
// LDS with K contiguous per row (A) or column (B), so each lane's 8 K-values
// of an MFMA operand are one 16-byte LDS read.  The K range is taken in
// chunks of NK tiles: the loads of a whole chunk are issued before its first
// product (NK register stages, straight-line code, so each stage waits only
// for its own loads), then each stage goes to one of two alternating LDS
// buffers (one barrier per K tile) and into the MFMAs.
template <bool TA, bool TB, int EPI, int NK>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g, GemmEpi ep)
{
    __shared__ __attribute__((aligned(16))) uint16_t sA[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) uint16_t sB[2][BN * LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wm = wave >> 1, wn = wave & 1;
    const int kb = blockIdx.z * g.kslice, ke = min(g.K, kb + g.kslice);
    // vector loads: 16 bytes along K, or 4 bytes along the rows
    const bool va = TA ? (g.lda % 2 == 0 && ((uintptr_t)g.A & 3) == 0) : (g.lda % 8 == 0 && ((uintptr_t)g.A & 15) == 0);
    const bool vb = TB ? (g.ldb % 8 == 0 && ((uintptr_t)g.B & 15) == 0) : (g.ldb % 2 == 0 && ((uintptr_t)g.B & 3) == 0);
    f32x16_t acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    // D layout of the 32x32 MFMA: lane l holds column l % 32 and, for
    // r = 0..15, row 8 (r / 4) + 4 (l / 32) + r % 4.
    const int j = n0 + wn * 32 + (lane & 31);
    auto row = [&](int r) { return m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); };
    // the epilogue's own inputs are loaded first, so their latency hides
    // behind the K loop (one pass; a split leaves them to the reduction)
    float pre[16];
    if (!g.part && (EPI == EPI_GELU_BWD || EPI == EPI_BIAS_GELU || EPI == EPI_BIAS)) {
        const float bj = (EPI != EPI_GELU_BWD && j < g.N) ? ep.bias[j] : 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r)
            pre[r] = EPI == EPI_GELU_BWD ? ((j < g.N && row(r) < g.M) ? ep.Zin[(int64_t)row(r) * ep.ldz + j] : 0.f)
                                         : bj;
    }
    // Full chunks: an operand whose 64 rows are all in range (and whose
    // vector loads are aligned) is loaded with vector loads, the other with
    // clamped element loads; with both in range all NK tiles' loads are in
    // flight at once, otherwise two tiles'.  The split's last partial chunk
    // goes two K tiles at a time with element loads.
    const bool fa = va && m0 + BM <= g.M, fb = vb && n0 + BN <= g.N;
    int c0 = kb;
    if (fa && fb)
        for (; c0 + NK * BK <= ke; c0 += NK * BK)
            gemm_chunk<TA, TB, NK, true, true>(g, c0, kb, ke, m0, n0, tid, sA, sB, acc);
    else if (fa)
        for (; c0 + 2 * BK <= ke; c0 += 2 * BK)
            gemm_chunk<TA, TB, 2, true, false>(g, c0, kb, ke, m0, n0, tid, sA, sB, acc);
    else if (fb)
        for (; c0 + 2 * BK <= ke; c0 += 2 * BK)
            gemm_chunk<TA, TB, 2, false, true>(g, c0, kb, ke, m0, n0, tid, sA, sB, acc);
    for (; c0 < ke; c0 += 2 * BK)
        gemm_chunk<TA, TB, 2, false, false>(g, c0, kb, ke, m0, n0, tid, sA, sB, acc);

    if (j >= g.N)
        return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = row(r);
        if (i >= g.M)
            continue;
        if (g.part) {
            g.part[((int64_t)blockIdx.z * g.M + i) * g.N + j] = acc[r];
        } else if (EPI == EPI_GELU_BWD) {
            ep.Yb[(int64_t)i * ep.ldy + j] = f2bf(acc[r] * gelu_grad(pre[r]));
        } else if (EPI == EPI_BIAS_GELU) {
            const float z = acc[r] + pre[r];
            ep.Z[(int64_t)i * ep.ldz + j] = z;
            ep.Yb[(int64_t)i * ep.ldy + j] = f2bf(gelu(z));
        } else if (EPI == EPI_BIAS) {
            ep.Z[(int64_t)i * ep.ldz + j] = acc[r] + pre[r];
        } else {
            epi_store<EPI>(i, j, acc[r], ep);
        }
    }
}

// ---- large outputs: big workgroup tiles --------------------------------------
// WM x WN waves, each computing (MI x 32) x (NJ x 32) as MI x NJ MFMA 32x32x16
// tiles: per 16 K-values a wave reads MI + NJ fragments from LDS for MI * NJ
// MFMAs (the 64 x 64 kernel reads two for one).  Operands whose K is not
// contiguous in memory are loaded as 8 (K) x 4 (rows) blocks of 8-byte
// pieces, transposed in registers and stored as 16-byte LDS writes.
#ifndef TITAN_GEMM_BIG
#define TITAN_GEMM_BIG 2
#endif
// Tile shapes (compile-time choice for tuning builds; 8192^3 in TFLOP/s for
// the NN / NT / TN layouts on MI355X with the strided operand loaded inside
// the product: 256 x 256 683 / 987 / 609, 256 x 128 705 / 750 / 355,
// 128 x 128 608 / 833 / 490; NN / NT with the copied operand: 256 x 256 in
// 8 waves 804-836 / 964-1,007, in 4 waves of 128 x 128 (one wave per SIMD,
// 256 accumulators per lane) 737 / 850).
#if TITAN_GEMM_BIG == 1
constexpr int GWM = 2, GWN = 2, GMI = 4, GNJ = 2;  // 256 x 128, 4 waves of 128 x 64
#elif TITAN_GEMM_BIG == 2
constexpr int GWM = 2, GWN = 4, GMI = 4, GNJ = 2;  // 256 x 256, 8 waves of 128 x 64
#elif TITAN_GEMM_BIG == 4
constexpr int GWM = 2, GWN = 2, GMI = 4, GNJ = 4;  // 256 x 256, 4 waves of 128 x 128
#else
constexpr int GWM = 2, GWN = 2, GMI = 2, GNJ = 2;  // 128 x 128, 4 waves of 64 x 64
#endif
// (One LDS buffer per operand: double-buffering, one barrier per K step
// instead of two, measured no faster -- LDS reads per MFMA set the pace.)
constexpr int GBM = GWM * GMI * 32, GBN = GWN * GNJ * 32, GT = GWM * GWN * 64;

template <bool KCONTIG, int ROWS>
struct TileMoveBig {
    static constexpr int CH = ROWS * (BK / 8) / GT;  // 16-byte chunks per thread (K contiguous)
    static constexpr int BL = 2 * ROWS / GT;         // 8 x 4 blocks per thread (K strided)
    static_assert(CH * GT == ROWS * (BK / 8) && BL * GT == 2 * ROWS, "tile must split evenly over the threads");
    uint4 v[KCONTIG ? CH : 4 * BL];

    __device__ __forceinline__ void load(const uint16_t *P, int ld, int r0, int R, int k0, int kend, bool vec,
                                         int tid)
    {
        if (KCONTIG) {
            // element (r, k) at P[r * ld + k]: 16-byte chunks of 8 K-values,
            // chunk c = row c / 8, K offset (c % 8) * 8
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int c = tid + GT * q;
                const int row = r0 + (c >> 3), k = k0 + (c & 7) * 8;
                if (vec && row < R && k + 8 <= kend) {
                    v[q] = *(const uint4 *)(P + (int64_t)row * ld + k);
                } else {
                    uint32_t w[4];
#pragma unroll
                    for (int e = 0; e < 8; e += 2) {
                        const uint32_t x0 = (row < R && k + e < kend) ? P[(int64_t)row * ld + k + e] : 0u;
                        const uint32_t x1 = (row < R && k + e + 1 < kend) ? P[(int64_t)row * ld + k + e + 1] : 0u;
                        w[e / 2] = x0 | x1 << 16;
                    }
                    v[q] = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
        } else {
            // element (r, k) at P[k * ld + r]: block b = K k0 + 8 (b / (ROWS/4))
            // .. +8, rows r0 + 4 (b % (ROWS/4)) .. +4 (consecutive threads read
            // consecutive 8-byte pieces of a K row), transposed in registers
#pragma unroll
            for (int q = 0; q < BL; ++q) {
                const int blk = tid + GT * q;
                const int kb = k0 + 8 * (blk / (ROWS / 4)), rb = r0 + 4 * (blk % (ROWS / 4));
                uint2 in[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = kb + e;
                    if (vec && k < kend && rb + 4 <= R) {
                        in[e] = *(const uint2 *)(P + (int64_t)k * ld + rb);
                    } else {
                        uint32_t h[4];
#pragma unroll
                        for (int n = 0; n < 4; ++n)
                            h[n] = (k < kend && rb + n < R) ? P[(int64_t)k * ld + rb + n] : 0u;
                        in[e] = make_uint2(h[0] | h[1] << 16, h[2] | h[3] << 16);
                    }
                }
                // v[4q + n] = the 8 K-values of row rb + n
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    uint32_t w[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint32_t a = (n < 2) ? in[2 * j].x : in[2 * j].y;
                        const uint32_t b = (n < 2) ? in[2 * j + 1].x : in[2 * j + 1].y;
                        w[j] = (n & 1) ? ((a >> 16) | (b & 0xFFFF0000u)) : ((a & 0xFFFFu) | (b << 16));
                    }
                    v[4 * q + n] = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
        }
    }

    __device__ __forceinline__ void store(uint16_t *S, int tid) const
    {
        if (KCONTIG) {
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int c = tid + GT * q;
                *(uint4 *)&S[(c >> 3) * LDK + (c & 7) * 8] = v[q];
            }
        } else {
#pragma unroll
            for (int q = 0; q < BL; ++q) {
                const int blk = tid + GT * q;
                const int kb = 8 * (blk / (ROWS / 4)), rb = 4 * (blk % (ROWS / 4));
#pragma unroll
                for (int n = 0; n < 4; ++n)
                    *(uint4 *)&S[(rb + n) * LDK + kb] = v[4 * q + n];
            }
        }
    }
};

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(GT) void gemm_big_kernel(GemmArgs g, GemmEpi ep)
{
    __shared__ __attribute__((aligned(16))) uint16_t sA[GBM * LDK];
    __shared__ __attribute__((aligned(16))) uint16_t sB[GBN * LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int wm = wave / GWN, wn = wave % GWN;
    const int K = g.K;
    // vector loads: 16 bytes along K, or 8 bytes along the rows
    const bool va = TA ? (g.lda % 4 == 0 && ((uintptr_t)g.A & 7) == 0) : (g.lda % 8 == 0 && ((uintptr_t)g.A & 15) == 0);
    const bool vb = TB ? (g.ldb % 8 == 0 && ((uintptr_t)g.B & 15) == 0) : (g.ldb % 4 == 0 && ((uintptr_t)g.B & 7) == 0);
    TileMoveBig<!TA, GBM> ta;
    TileMoveBig<TB, GBN> tb;
    f32x16_t acc[GMI][GNJ];
#pragma unroll
    for (int i = 0; i < GMI; ++i)
#pragma unroll
        for (int j = 0; j < GNJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                acc[i][j][r] = 0.f;
    auto multiply = [&](const uint16_t *A_, const uint16_t *B_) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            bf16x8_t a[GMI], b[GNJ];
#pragma unroll
            for (int i = 0; i < GMI; ++i)
                a[i] = *(const bf16x8_t *)&A_[(wm * GMI * 32 + i * 32 + (lane & 31)) * LDK + kk + 8 * (lane >> 5)];
#pragma unroll
            for (int j = 0; j < GNJ; ++j)
                b[j] = *(const bf16x8_t *)&B_[(wn * GNJ * 32 + j * 32 + (lane & 31)) * LDK + kk + 8 * (lane >> 5)];
#pragma unroll
            for (int i = 0; i < GMI; ++i)
#pragma unroll
                for (int j = 0; j < GNJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    };
    if (K > 0) {
        ta.load(g.A, g.lda, m0, g.M, 0, K, va, tid);
        tb.load(g.B, g.ldb, n0, g.N, 0, K, vb, tid);
    }
    // the next K tile is loaded into registers while this one is multiplied
    for (int k0 = 0; k0 < K; k0 += BK) {
        ta.store(sA, tid);
        tb.store(sB, tid);
        __syncthreads();
        if (k0 + BK < K) {
            ta.load(g.A, g.lda, m0, g.M, k0 + BK, K, va, tid);
            tb.load(g.B, g.ldb, n0, g.N, k0 + BK, K, vb, tid);
        }
        multiply(sA, sB);
        __syncthreads();
    }

    // D layout of the 32x32 MFMA: lane l holds column l % 32 and, for
    // r = 0..15, row 8 (r / 4) + 4 (l / 32) + r % 4.
#pragma unroll
    for (int j = 0; j < GNJ; ++j) {
        const int col = n0 + wn * GNJ * 32 + j * 32 + (lane & 31);
        if (col >= g.N)
            continue;
#pragma unroll
        for (int i = 0; i < GMI; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * GMI * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row < g.M)
                    epi_store<EPI>(row, col, acc[i][j][r], ep);
            }
    }
}

// Split-K: sum the partials of each output element in split order, then the
// epilogue.
template <int EPI>
__global__ void gemm_reduce_kernel(int M, int N, int splits, const float *part, GemmEpi ep)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)M * N)
        return;
    float v = 0.f;
    for (int z = 0; z < splits; ++z)
        v += part[(int64_t)z * M * N + q];
    epi_store<EPI>((int)(q / N), (int)(q % N), v, ep);
}

// Q (C x R, row stride ldq) = P^T for P (R x C, row stride ld), bf16, through
// a 64 x 64 LDS tile (rows padded to 72 values, 16-byte aligned): 16-byte
// loads along P's rows when in range and aligned, stored whole; then each
// thread gathers 8 consecutive P rows of one column (a wave reads 64
// neighbouring columns: no bank conflicts) and writes them as 16 bytes of a
// Q row.  Used to give a large product both operands with K contiguous.
__global__ __launch_bounds__(256) void transpose_bf16_kernel(const uint16_t *P, int R, int C, int ld, uint16_t *Q,
                                                             int ldq)
{
    __shared__ __attribute__((aligned(16))) uint16_t t[64][72];
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64, tid = threadIdx.x;
    const bool vec = ld % 8 == 0 && ((uintptr_t)P & 15) == 0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int ch = tid + 256 * q, rr = ch >> 3, cc = (ch & 7) * 8;
        const int r = r0 + rr, c = c0 + cc;
        u32x4 v;
        if (vec && r < R && c + 8 <= C) {
            v = *(const u32x4 *)(P + (int64_t)r * ld + c);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t lo = (r < R && c + 2 * e < C) ? P[(int64_t)r * ld + c + 2 * e] : 0u;
                const uint32_t hi = (r < R && c + 2 * e + 1 < C) ? P[(int64_t)r * ld + c + 2 * e + 1] : 0u;
                v[e] = lo | hi << 16;
            }
        }
        *(u32x4 *)&t[rr][cc] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int ch = tid + 256 * q, rr = (ch >> 6) * 8, cc = ch & 63;
        const int c = c0 + cc, r = r0 + rr;
        if (c >= C)
            continue;
        if (r + 8 <= R && ldq % 8 == 0 && ((uintptr_t)Q & 15) == 0) {
            u32x4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                v[e] = (uint32_t)t[rr + 2 * e][cc] | (uint32_t)t[rr + 2 * e + 1][cc] << 16;
            *(u32x4 *)(Q + (int64_t)c * ldq + r) = v;
        } else {
            for (int e = 0; e < 8 && r + e < R; ++e)
                Q[(int64_t)c * ldq + r + e] = t[rr + e][cc];
        }
    }
}

static hipError_t transpose_bf16(const uint16_t *P, int R, int C, int ld, uint16_t *Q, int ldq, hipStream_t st)
{
    const dim3 grid((unsigned)((C + 63) / 64), (unsigned)((R + 63) / 64));
    hipLaunchKernelGGL(transpose_bf16_kernel, grid, dim3(256), 0, st, P, R, C, ld, Q, ldq);
    return hipGetLastError();
}

// Largest number of K tiles the 64 x 64 kernel loads at once (4 or 8).
#ifndef TITAN_GEMM_MAXNK
#define TITAN_GEMM_MAXNK 8
#endif
constexpr int kGemmMaxNk = TITAN_GEMM_MAXNK;

// Workgroups a GEMM aims for before it splits K (a split costs a partial-sum
// write and a reduce launch).
#ifndef TITAN_GEMM_TARGET
#define TITAN_GEMM_TARGET 128
#endif
constexpr int kGemmTarget = TITAN_GEMM_TARGET;

// part (capacity part_cap floats) enables split-K when the output has too few
// tiles; null: one pass.  A large product uses the same buffer to copy an
// operand whose K is strided into K-contiguous form first (the big-tile
// kernel then loads both operands with 16-byte loads; the MFMAs see the same
// values in the same order, so the result is the same bit for bit).
template <bool TA, bool TB, int EPI>
hipError_t gemm(int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B, int ldb, const GemmEpi &ep,
                hipStream_t st, float *part = nullptr, int64_t part_cap = 0)
{
    if (M <= 0 || N <= 0)
        return hipSuccess;
    // large outputs (at least 128 big tiles): one pass of the big-tile kernel
    const int big_tiles = ((N + GBN - 1) / GBN) * ((M + GBM - 1) / GBM);
    if (big_tiles >= 128) {
        const int Kp = (K + 7) / 8 * 8;  // row stride of the copies: 16-byte rows
        const int64_t need = (TA ? (int64_t)M * Kp : 0) + (TB ? 0 : (int64_t)N * Kp);  // bf16 values
        if (need > 0 && K > 0 && part && 2 * need <= 4 * part_cap) {
            uint16_t *w = (uint16_t *)part;
            const uint16_t *a = A, *b = B;
            int la = lda, lb = ldb;
            if (TA) {  // A (K x M, stride lda) -> M x K, stride Kp
                hipError_t e = transpose_bf16(A, K, M, lda, w, Kp, st);
                if (e != hipSuccess)
                    return e;
                a = w;
                la = Kp;
                w += (int64_t)M * Kp;
            }
            if (!TB) {  // B (K x N, stride ldb) -> N x K, stride Kp
                hipError_t e = transpose_bf16(B, K, N, ldb, w, Kp, st);
                if (e != hipSuccess)
                    return e;
                b = w;
                lb = Kp;
            }
            GemmArgs g{M, N, K, a, la, b, lb, std::max(K, 1), nullptr};
            const dim3 grid((unsigned)((N + GBN - 1) / GBN), (unsigned)((M + GBM - 1) / GBM), 1);
            hipLaunchKernelGGL((gemm_big_kernel<false, true, EPI>), grid, dim3(GT), 0, st, g, ep);
            return hipGetLastError();
        }
        GemmArgs g{M, N, K, A, lda, B, ldb, std::max(K, 1), nullptr};
        const dim3 grid((unsigned)((N + GBN - 1) / GBN), (unsigned)((M + GBM - 1) / GBM), 1);
        hipLaunchKernelGGL((gemm_big_kernel<TA, TB, EPI>), grid, dim3(GT), 0, st, g, ep);
        return hipGetLastError();
    }
    const int tiles = ((N + BN - 1) / BN) * ((M + BM - 1) / BM);
    const int kt = std::max(1, (K + BK - 1) / BK);
    int splits = 1;
    if (part && tiles < kGemmTarget)
        splits = std::max(1, std::min((kGemmTarget + tiles - 1) / tiles, kt / 2));  // at least the target
    while (splits > 1 && (int64_t)splits * M * N > part_cap)
        --splits;
    // K tiles per split, rounded up to the chunk the kernel stages at once
    const int per = (kt + splits - 1) / splits;
    const int nk = per <= 1 ? 1 : per <= 2 ? 2 : per <= 4 || kGemmMaxNk == 4 ? 4 : 8;
    const int kslice = (splits > 1 ? std::min(per, nk) : kt) * BK;
    splits = std::max(1, (K + kslice - 1) / kslice);
    GemmArgs g{M, N, K, A, lda, B, ldb, kslice, splits > 1 ? part : nullptr};
    const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)splits);
    if (nk == 1)
        hipLaunchKernelGGL((gemm_kernel<TA, TB, EPI, 1>), grid, dim3(256), 0, st, g, ep);
    else if (nk == 2)
        hipLaunchKernelGGL((gemm_kernel<TA, TB, EPI, 2>), grid, dim3(256), 0, st, g, ep);
    else if (nk == 4)
        hipLaunchKernelGGL((gemm_kernel<TA, TB, EPI, 4>), grid, dim3(256), 0, st, g, ep);
    else
        hipLaunchKernelGGL((gemm_kernel<TA, TB, EPI, 8>), grid, dim3(256), 0, st, g, ep);
    if (splits > 1) {
        const int64_t n = (int64_t)M * N;
        hipLaunchKernelGGL(gemm_reduce_kernel<EPI>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M, N, splits,
                           part, ep);
    }
    return hipGetLastError();
}

__global__ void to_bf16_kernel(const float *x, uint16_t *y, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n)
        y[q] = f2bf(x[q]);
}

// Rows of n floats to bf16 rows of stride ld.
__global__ void to_bf16_rows_kernel(const float *x, uint16_t *y, int64_t rows, int n, int ld)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < rows * n)
        y[(q / n) * ld + q % n] = f2bf(x[q]);
}

// The padding of activation rows: column n = 1.0 (the ones column that turns
// the weight-gradient product into the bias gradient too), columns n+1 .. ld-1
// zero.  Written once per allocation; the GEMMs write only columns < n.
__global__ void activation_pad_kernel(uint16_t *x, int64_t rows, int n, int ld)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int pad = ld - n;
    if (q < rows * pad) {
        const int64_t r = q / pad;
        const int c = n + (int)(q % pad);
        x[r * ld + c] = c == n ? (uint16_t)0x3F80 : (uint16_t)0;
    }
}

// The batch's rows of the resident data set: inputs (bf16, rows of `in`
// values) into the activation rows (stride ldx) and targets into yb.  Rows
// over blockIdx.y; 16-byte copies when rows hold a multiple of 8 values.
__global__ __launch_bounds__(256) void gather_rows_kernel(const uint16_t *X, const float *Y, const int64_t *idx, int B,
                                                          int in, int out, uint16_t *xb, int ldx, float *yb)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
    for (int b = blockIdx.y; b < B; b += gridDim.y) {
        const int64_t r = idx[b];
        const uint16_t *src = X + r * in;
        uint16_t *dst = xb + (int64_t)b * ldx;
        if (in % 8 == 0) {
            for (int c = t; c < in / 8; c += nt)
                *(u32x4 *)(dst + 8 * c) = *(const u32x4 *)(src + 8 * c);
        } else {
            for (int c = t; c < in; c += nt)
                dst[c] = src[c];
        }
        if (blockIdx.x == 0)
            for (int c = threadIdx.x; c < out; c += blockDim.x)
                yb[(int64_t)b * out + c] = Y[r * out + c];
    }
}

// Output layers with at most kHeadMax outputs (the surrogate's three): the
// last product, the loss and the first backward product in one launch, one
// wave per batch row i (four rows per workgroup):
//   z[i][o] = sum_k x[i][k] W[o][k] + b[o]            (FP32 out)
//   e = z - y, dz[i][o] = bf16(2 e / (B O)), lrow[i] = sum_o e^2
//   dzp[i][j] = bf16((sum_o dz[i][o] W[o][j]) gelu'(zp[i][j]))   (if zp)
// The lane partial sums over k are combined by a butterfly of exchanges, so
// every lane holds the same total and the order is fixed: deterministic.
constexpr int kHeadMax = 4;

template <int O>
__global__ __launch_bounds__(256) void head_kernel(int B, int in, const uint16_t *x, int ldx, const uint16_t *W,
                                                   const float *bias, const float *y, float *z, uint16_t *dz,
                                                   float *lrow, const float *zp, uint16_t *dzp)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= B)
        return;  // a whole wave; no barrier follows
    const uint16_t *xr = x + (int64_t)i * ldx;
    float acc[O];
#pragma unroll
    for (int o = 0; o < O; ++o)
        acc[o] = 0.f;
#pragma unroll 4
    for (int k = lane; k < in; k += 64) {
        const float xv = bf2f(xr[k]);
#pragma unroll
        for (int o = 0; o < O; ++o)
            acc[o] = fmaf(xv, bf2f(W[(int64_t)o * in + k]), acc[o]);
    }
#pragma unroll
    for (int o = 0; o < O; ++o)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            acc[o] += __shfl_xor(acc[o], off, 64);
    const float n = (float)((int64_t)B * O);  // dz as in the general path: 2 e / n
    float dzf[O], l = 0.f;
#pragma unroll
    for (int o = 0; o < O; ++o) {
        const float zo = acc[o] + bias[o];
        const float e = zo - y[(int64_t)i * O + o];
        const uint16_t d = f2bf(2.f * e / n);
        dzf[o] = bf2f(d);
        l = fmaf(e, e, l);
        if (lane == o) {
            z[(int64_t)i * O + o] = zo;
            dz[(int64_t)i * O + o] = d;
        }
    }
    if (lane == 0)
        lrow[i] = l;
    if (!zp)
        return;
    const float *zr = zp + (int64_t)i * in;
    uint16_t *dr = dzp + (int64_t)i * in;
#pragma unroll 4
    for (int j = lane; j < in; j += 64) {
        float g = dzf[0] * bf2f(W[j]);
#pragma unroll
        for (int o = 1; o < O; ++o)
            g = fmaf(dzf[o], bf2f(W[(int64_t)o * in + j]), g);
        dr[j] = f2bf(g * gelu_grad(zr[j]));
    }
}

// The general output layer's loss terms: dz = bf16(2 (out - y) / (B O)) and
// lrow[i] = sum_o (out - y)^2, one thread per row.
__global__ void mse_rows_kernel(const float *out, const float *y, int B, int O, uint16_t *dz, float *lrow)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B)
        return;
    const float n = (float)((int64_t)B * O);
    float l = 0.f;
    for (int o = 0; o < O; ++o) {
        const int64_t q = (int64_t)i * O + o;
        const float d = out[q] - y[q];
        l = fmaf(d, d, l);
        dz[q] = f2bf(2.f * d / n);
    }
    lrow[i] = l;
}

// Loss of step s = sum_i lrow[s][i] / (B O), one workgroup per step, a fixed
// summation order: deterministic.
__global__ __launch_bounds__(256) void loss_rows_kernel(const float *lrow, int B, int O, float *loss)
{
    __shared__ float red[256];
    const int t = threadIdx.x;
    const float *r = lrow + (int64_t)blockIdx.x * B;
    float acc = 0.f;
    for (int i = t; i < B; i += 256)
        acc += r[i];
    red[t] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s)
            red[t] += red[t + s];
        __syncthreads();
    }
    if (t == 0)
        loss[blockIdx.x] = red[0] / (float)((int64_t)B * O);
}

// Where the weight matrices sit in the flat parameters and in the bf16 copy
// the GEMMs read (biases stay FP32).
constexpr int kMaxLayersFused = 8;
struct WeightMap {
    int L;
    int64_t woff[kMaxLayersFused], wn[kMaxLayersFused], wboff[kMaxLayersFused];
};

// Adam on the FP32 master parameters; with wb, also the bf16 copy of every
// updated weight (what a separate conversion pass would write).
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2, WeightMap map, uint16_t *wb)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n)
        return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    const float pq = p[q] - lr * (mq / bc1) / (sqrtf(vq / bc2) + eps);
    p[q] = pq;
    if (wb)
        for (int l = 0; l < map.L; ++l)
            if (q >= map.woff[l] && q < map.woff[l] + map.wn[l])
                wb[map.wboff[l] + (q - map.woff[l])] = f2bf(pq);
}

hipError_t launch1d(void (*k)(const float *, uint16_t *, int64_t), const float *x, uint16_t *y, int64_t n,
                    hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, n);
    return hipGetLastError();
}

}  // namespace
}  // namespace titan

using namespace titan;

// ---------------------------------------------------------------------------
// the titan_mlp object
// ---------------------------------------------------------------------------

struct titan_mlp {
    std::mutex mu;
    hipStream_t stream = nullptr;
    titan_allocator alloc{};
    std::vector<std::pair<void *, size_t>> allocations;
    int device = 0;
    std::vector<int32_t> dims;        // n_layers + 1
    std::vector<int64_t> woff, boff;  // offsets of W_l, b_l in the flat parameter array
    std::vector<int64_t> wboff;       // offsets of W_l in the bf16 weight array
    int64_t nparam = 0, nw = 0;
    float *P = nullptr, *G = nullptr, *Mo = nullptr, *Vo = nullptr;  // params, grads, Adam moments
    uint16_t *Wb = nullptr;                                          // bf16 weights
    int64_t adam_t = 0;
    // dataset
    int64_t n_data = 0;
    uint16_t *X = nullptr;
    float *Y = nullptr;
    // workspace for batches up to cap
    int cap = 0;
    std::vector<uint16_t *> xs;  // x_l, l = 0..L-1 (bf16), row stride xld[l]: dims[l] values, a ones column, zeros
    std::vector<int> xld;
    std::vector<float *> zs;     // z_l (fp32)
    uint16_t *dz[2] = {nullptr, nullptr};
    float *yb = nullptr;
    float *gpart = nullptr;  // split-K partial sums of the GEMMs
    float *lrow = nullptr;   // the current batch's per-row squared errors (owned by the caller)
    int64_t gpart_cap = 0;   // floats in gpart
    int64_t *idx = nullptr;
    float *loss = nullptr;
    int loss_cap = 0;
    int L() const { return (int)dims.size() - 1; }
};

static int mlp_alloc(titan_mlp *m, size_t bytes, void **out)
{
    *out = nullptr;
    bytes = std::max<size_t>(bytes, 256);
    void *p = nullptr;
    if (m->alloc.alloc) {
        p = m->alloc.alloc(bytes, m->alloc.ctx);
        if (!p)
            return fail(TITAN_ENOMEM, "device allocator returned NULL for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(TITAN_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        }
    }
    m->allocations.push_back({p, bytes});
    *out = p;
    return TITAN_OK;
}

static void mlp_free(titan_mlp *m, void *p)
{
    for (size_t q = 0; q < m->allocations.size(); ++q)
        if (m->allocations[q].first == p) {
            (void)hipStreamSynchronize(m->stream);
            if (m->alloc.release)
                m->alloc.release(p, m->alloc.ctx);
            else
                (void)hipFree(p);
            m->allocations.erase(m->allocations.begin() + q);
            return;
        }
}

#define MLP_TRY(expr)                                                         \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess)                                                 \
            return fail(TITAN_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

static int ensure_cap(titan_mlp *m, int B)
{
    if (B <= m->cap)
        return TITAN_OK;
    for (auto *p : m->xs)
        mlp_free(m, p);
    for (auto *p : m->zs)
        mlp_free(m, p);
    for (auto *p : {(void *)m->dz[0], (void *)m->dz[1], (void *)m->yb, (void *)m->idx, (void *)m->gpart})
        if (p)
            mlp_free(m, p);
    m->xs.assign(m->L(), nullptr);
    m->zs.assign(m->L(), nullptr);
    m->xld.assign(m->L(), 0);
    int maxd = 0;
    for (int d : m->dims)
        maxd = std::max(maxd, d);
    for (int l = 0; l < m->L(); ++l) {
        m->xld[l] = (m->dims[l] + 1 + 7) / 8 * 8;  // room for the ones column; 16-byte rows
        if (int rc = mlp_alloc(m, sizeof(uint16_t) * (size_t)B * m->xld[l], (void **)&m->xs[l]))
            return rc;
        const int64_t pad = (int64_t)B * (m->xld[l] - m->dims[l]);
        hipLaunchKernelGGL(activation_pad_kernel, dim3((unsigned)((pad + 255) / 256)), dim3(256), 0, m->stream,
                           m->xs[l], (int64_t)B, m->dims[l], m->xld[l]);
        MLP_TRY(hipGetLastError());
        if (int rc = mlp_alloc(m, sizeof(float) * (size_t)B * m->dims[l + 1], (void **)&m->zs[l]))
            return rc;
    }
    for (int q = 0; q < 2; ++q)
        if (int rc = mlp_alloc(m, sizeof(uint16_t) * (size_t)B * maxd, (void **)&m->dz[q]))
            return rc;
    if (int rc = mlp_alloc(m, sizeof(float) * (size_t)B * m->dims.back(), (void **)&m->yb))
        return rc;
    if (int rc = mlp_alloc(m, sizeof(int64_t) * (size_t)B, (void **)&m->idx))
        return rc;
    m->gpart_cap = 4 * std::max<int64_t>((int64_t)B * maxd, (int64_t)maxd * (maxd + 1));
    if (int rc = mlp_alloc(m, sizeof(float) * (size_t)m->gpart_cap, (void **)&m->gpart))
        return rc;
    m->cap = B;
    return TITAN_OK;
}

static int refresh_bf16(titan_mlp *m)
{
    for (int l = 0; l < m->L(); ++l)
        MLP_TRY(launch1d(to_bf16_kernel, m->P + m->woff[l], m->Wb + m->wboff[l],
                         (int64_t)m->dims[l] * m->dims[l + 1], m->stream));
    return TITAN_OK;
}

// Forward of a batch already in xs[0] through layers [0, upto); the output
// of the whole network (upto = L) in zs[L-1].
static int forward(titan_mlp *m, int B, int upto)
{
    const int L = m->L();
    for (int l = 0; l < upto; ++l) {
        const int in = m->dims[l], out = m->dims[l + 1];
        GemmEpi ep{};
        ep.bias = m->P + m->boff[l];
        ep.Z = m->zs[l];
        ep.ldz = out;
        if (l < L - 1) {
            ep.Yb = m->xs[l + 1];
            ep.ldy = m->xld[l + 1];
            MLP_TRY((gemm<false, true, EPI_BIAS_GELU>(B, out, in, m->xs[l], m->xld[l], m->Wb + m->wboff[l], in, ep,
                                                      m->stream, m->gpart, m->gpart_cap)));
        } else {
            MLP_TRY((gemm<false, true, EPI_BIAS>(B, out, in, m->xs[l], m->xld[l], m->Wb + m->wboff[l], in, ep,
                                                 m->stream, m->gpart, m->gpart_cap)));
        }
    }
    return TITAN_OK;
}

template <int O>
static void launch_head(titan_mlp *m, int B)
{
    const int L = m->L(), in = m->dims[L - 1];
    hipLaunchKernelGGL(head_kernel<O>, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, m->stream, B, in, m->xs[L - 1],
                       m->xld[L - 1], m->Wb + m->wboff[L - 1], m->P + m->boff[L - 1], m->yb, m->zs[L - 1],
                       m->dz[0], m->lrow, L > 1 ? m->zs[L - 2] : nullptr, m->dz[1]);
}

// Loss terms and gradients of a batch in xs[0] / yb: each row's squared
// error summed over the outputs to lrow[0..B).
static int backward(titan_mlp *m, int B, float *lrow)
{
    const int L = m->L();
    const int O = m->dims[L];
    const bool head = O <= kHeadMax;
    m->lrow = lrow;
    if (int rc = forward(m, B, head ? L - 1 : L))
        return rc;
    if (head) {
        // the output layer's product, the loss and dz_{L-2} in one launch
        if (O == 1)
            launch_head<1>(m, B);
        else if (O == 2)
            launch_head<2>(m, B);
        else if (O == 3)
            launch_head<3>(m, B);
        else
            launch_head<4>(m, B);
    } else {
        hipLaunchKernelGGL(mse_rows_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, m->stream, m->zs[L - 1],
                           m->yb, B, O, m->dz[0], lrow);
    }
    MLP_TRY(hipGetLastError());
    int cur = 0;
    for (int l = L - 1; l >= 0; --l) {
        const int in = m->dims[l], out = m->dims[l + 1];
        uint16_t *dz = m->dz[cur];
        // dW and db in one product: dz^T [x_l, 1]
        GemmEpi ew{};
        ew.Z = m->G + m->woff[l];
        ew.ldz = in;
        ew.db = m->G + m->boff[l];
        MLP_TRY((gemm<true, false, EPI_WGRAD>(out, in + 1, B, dz, out, m->xs[l], m->xld[l], ew, m->stream, m->gpart,
                                              m->gpart_cap)));
        if (l > 0 && head && l == L - 1) {
            cur = 1 - cur;  // dz_{L-2} came with the loss
        } else if (l > 0) {
            GemmEpi ed{};
            ed.Zin = m->zs[l - 1];
            ed.ldz = in;
            ed.Yb = m->dz[1 - cur];
            ed.ldy = in;
            MLP_TRY((gemm<false, false, EPI_GELU_BWD>(B, in, out, dz, out, m->Wb + m->wboff[l], in, ed, m->stream,
                                                      m->gpart, m->gpart_cap)));
            cur = 1 - cur;
        }
    }
    return TITAN_OK;
}

static int upload_batch_f32(titan_mlp *m, int B, const float *X, const float *Y)
{
    const int in = m->dims[0];
    float *tmp = nullptr;
    if (int rc = mlp_alloc(m, sizeof(float) * (size_t)B * in, (void **)&tmp))
        return rc;
    MLP_TRY(hipMemcpyAsync(tmp, X, sizeof(float) * (size_t)B * in, hipMemcpyHostToDevice, m->stream));
    hipLaunchKernelGGL(to_bf16_rows_kernel, dim3((unsigned)(((int64_t)B * in + 255) / 256)), dim3(256), 0,
                       m->stream, tmp, m->xs[0], (int64_t)B, in, m->xld[0]);
    MLP_TRY(hipGetLastError());
    if (Y)
        MLP_TRY(hipMemcpyAsync(m->yb, Y, sizeof(float) * (size_t)B * m->dims.back(), hipMemcpyHostToDevice,
                               m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    mlp_free(m, tmp);
    return TITAN_OK;
}

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------

extern "C" int titan_mlp_create(int32_t n_layers, const int32_t *dims, void *stream, const titan_allocator *alloc,
                                titan_mlp **out)
{
    if (!out || !dims || n_layers < 1 || n_layers > 64)
        return fail(TITAN_EINVAL, "need out, dims and 1..64 layers");
    *out = nullptr;
    for (int l = 0; l <= n_layers; ++l)
        if (dims[l] < 1 || dims[l] > (1 << 16))
            return fail(TITAN_EINVAL, "layer width %d out of range", dims[l]);
    if (alloc && (!alloc->alloc || !alloc->release))
        return fail(TITAN_EINVAL, "allocator needs both alloc and release");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
        (void)hipGetLastError();
        return fail(TITAN_EDEVICE, "no usable HIP device");
    }
    titan_mlp *m = new (std::nothrow) titan_mlp();
    if (!m)
        return fail(TITAN_ENOMEM, "out of host memory");
    m->stream = (hipStream_t)stream;
    if (alloc)
        m->alloc = *alloc;
    (void)hipGetDevice(&m->device);
    m->dims.assign(dims, dims + n_layers + 1);
    int64_t off = 0, wb = 0;
    for (int l = 0; l < n_layers; ++l) {
        m->woff.push_back(off);
        off += (int64_t)dims[l] * dims[l + 1];
        m->boff.push_back(off);
        off += dims[l + 1];
        m->wboff.push_back(wb);
        wb += (int64_t)dims[l] * dims[l + 1];
    }
    m->nparam = off;
    m->nw = wb;
    int rc = TITAN_OK;
    if ((rc = mlp_alloc(m, sizeof(float) * off, (void **)&m->P)) || (rc = mlp_alloc(m, sizeof(float) * off, (void **)&m->G)) ||
        (rc = mlp_alloc(m, sizeof(float) * off, (void **)&m->Mo)) ||
        (rc = mlp_alloc(m, sizeof(float) * off, (void **)&m->Vo)) ||
        (rc = mlp_alloc(m, sizeof(uint16_t) * wb, (void **)&m->Wb))) {
        titan_mlp_destroy(m);
        return rc;
    }
    if (hipMemsetAsync(m->P, 0, sizeof(float) * off, m->stream) != hipSuccess ||
        hipMemsetAsync(m->Mo, 0, sizeof(float) * off, m->stream) != hipSuccess ||
        hipMemsetAsync(m->Vo, 0, sizeof(float) * off, m->stream) != hipSuccess) {
        titan_mlp_destroy(m);
        return fail(TITAN_EDEVICE, "hipMemsetAsync failed");
    }
    *out = m;
    return TITAN_OK;
}

extern "C" int titan_mlp_destroy(titan_mlp *m)
{
    if (!m)
        return TITAN_OK;
    {
        std::lock_guard<std::mutex> lk(m->mu);
        (void)hipStreamSynchronize(m->stream);
        for (auto &a : m->allocations) {
            if (m->alloc.release)
                m->alloc.release(a.first, m->alloc.ctx);
            else
                (void)hipFree(a.first);
        }
        m->allocations.clear();
    }
    delete m;
    return TITAN_OK;
}

extern "C" int64_t titan_mlp_param_count(titan_mlp *m) { return m ? m->nparam : -1; }

extern "C" int titan_mlp_set_params(titan_mlp *m, const float *params)
{
    if (!m || !params)
        return fail(TITAN_EINVAL, "mlp or params is NULL");
    std::lock_guard<std::mutex> lk(m->mu);
    for (int64_t q = 0; q < m->nparam; ++q)
        if (!std::isfinite(params[q]))
            return fail(TITAN_EINVAL, "parameter %lld is not finite", (long long)q);
    MLP_TRY(hipMemcpyAsync(m->P, params, sizeof(float) * m->nparam, hipMemcpyHostToDevice, m->stream));
    MLP_TRY(hipMemsetAsync(m->Mo, 0, sizeof(float) * m->nparam, m->stream));
    MLP_TRY(hipMemsetAsync(m->Vo, 0, sizeof(float) * m->nparam, m->stream));
    m->adam_t = 0;
    if (int rc = refresh_bf16(m))
        return rc;
    MLP_TRY(hipStreamSynchronize(m->stream));
    return TITAN_OK;
}

extern "C" int titan_mlp_get_params(titan_mlp *m, float *params)
{
    if (!m || !params)
        return fail(TITAN_EINVAL, "mlp or params is NULL");
    std::lock_guard<std::mutex> lk(m->mu);
    MLP_TRY(hipMemcpyAsync(params, m->P, sizeof(float) * m->nparam, hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    return TITAN_OK;
}

extern "C" int titan_mlp_set_data(titan_mlp *m, int64_t n, const float *X, const float *Y)
{
    if (!m || n < 0 || (n > 0 && (!X || !Y)))
        return fail(TITAN_EINVAL, "bad dataset arguments");
    std::lock_guard<std::mutex> lk(m->mu);
    const int in = m->dims[0], out = m->dims.back();
    if (m->X)
        mlp_free(m, m->X);
    if (m->Y)
        mlp_free(m, m->Y);
    m->X = nullptr;
    m->Y = nullptr;
    m->n_data = 0;
    if (int rc = mlp_alloc(m, sizeof(uint16_t) * (size_t)std::max<int64_t>(n, 1) * in, (void **)&m->X))
        return rc;
    if (int rc = mlp_alloc(m, sizeof(float) * (size_t)std::max<int64_t>(n, 1) * out, (void **)&m->Y))
        return rc;
    // convert in chunks through an FP32 staging buffer
    const int64_t chunk = 16384;
    float *tmp = nullptr;
    if (int rc = mlp_alloc(m, sizeof(float) * (size_t)chunk * in, (void **)&tmp))
        return rc;
    for (int64_t a = 0; a < n; a += chunk) {
        const int64_t c = std::min(chunk, n - a);
        MLP_TRY(hipMemcpyAsync(tmp, X + a * in, sizeof(float) * (size_t)c * in, hipMemcpyHostToDevice, m->stream));
        MLP_TRY(launch1d(to_bf16_kernel, tmp, m->X + a * in, c * in, m->stream));
        MLP_TRY(hipStreamSynchronize(m->stream));
    }
    mlp_free(m, tmp);
    if (n)
        MLP_TRY(hipMemcpyAsync(m->Y, Y, sizeof(float) * (size_t)n * out, hipMemcpyHostToDevice, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    m->n_data = n;
    return TITAN_OK;
}

extern "C" int titan_mlp_train(titan_mlp *m, int64_t nsteps, int32_t batch, const int64_t *idx, float lr, float beta1,
                               float beta2, float eps, float *loss_out)
{
    if (!m || nsteps < 0 || batch < 1 || (nsteps > 0 && !idx))
        return fail(TITAN_EINVAL, "bad training arguments");
    if (!(std::isfinite(lr) && lr >= 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0))
        return fail(TITAN_EINVAL, "bad optimiser settings");
    std::lock_guard<std::mutex> lk(m->mu);
    if (m->n_data == 0)
        return fail(TITAN_ESTATE, "no dataset (titan_mlp_set_data)");
    for (int64_t q = 0; q < nsteps * (int64_t)batch; ++q)
        if (idx[q] < 0 || idx[q] >= m->n_data)
            return fail(TITAN_EINVAL, "sample index %lld out of range", (long long)idx[q]);
    if (int rc = ensure_cap(m, batch))
        return rc;
    int64_t *didx = nullptr;
    float *dloss = nullptr, *dlrow = nullptr;
    if (int rc = mlp_alloc(m, sizeof(int64_t) * (size_t)std::max<int64_t>(nsteps * batch, 1), (void **)&didx))
        return rc;
    if (int rc = mlp_alloc(m, sizeof(float) * (size_t)std::max<int64_t>(nsteps, 1), (void **)&dloss))
        return rc;
    // the per-row squared errors of up to kLossChunk steps; their losses are
    // summed once per chunk (one launch for the chunk's steps)
    constexpr int64_t kLossChunk = 1024;
    const int64_t chunk = std::max<int64_t>(1, std::min(nsteps, kLossChunk));
    if (int rc = mlp_alloc(m, sizeof(float) * (size_t)(chunk * batch), (void **)&dlrow))
        return rc;
    if (nsteps)
        MLP_TRY(hipMemcpyAsync(didx, idx, sizeof(int64_t) * nsteps * batch, hipMemcpyHostToDevice, m->stream));
    const int in = m->dims[0], out = m->dims.back();
    for (int64_t s = 0; s < nsteps; ++s) {
        const int per_row = in % 8 == 0 ? in / 8 : in;
        hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((per_row + 255) / 256), (unsigned)std::min(batch, 65535)),
                           dim3(256), 0, m->stream, m->X, m->Y, didx + s * batch, batch, in, out, m->xs[0], m->xld[0],
                           m->yb);
        MLP_TRY(hipGetLastError());
        if (int rc = backward(m, batch, dlrow + (s % chunk) * batch))
            return rc;
        m->adam_t += 1;
        const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)m->adam_t));
        const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)m->adam_t));
        WeightMap map{};
        const bool fused = m->L() <= kMaxLayersFused;
        if (fused) {
            map.L = m->L();
            for (int l = 0; l < m->L(); ++l) {
                map.woff[l] = m->woff[l];
                map.wn[l] = (int64_t)m->dims[l] * m->dims[l + 1];
                map.wboff[l] = m->wboff[l];
            }
        }
        hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((m->nparam + 255) / 256)), dim3(256), 0, m->stream, m->P,
                           m->G, m->Mo, m->Vo, m->nparam, lr, beta1, beta2, eps, bc1, bc2, map,
                           fused ? m->Wb : nullptr);
        MLP_TRY(hipGetLastError());
        if (!fused)
            if (int rc = refresh_bf16(m))
                return rc;
        // the losses of a completed chunk of steps (also the last, partial one)
        if ((s + 1) % chunk == 0 || s + 1 == nsteps) {
            const int64_t s0 = s - s % chunk;
            hipLaunchKernelGGL(loss_rows_kernel, dim3((unsigned)(s + 1 - s0)), dim3(256), 0, m->stream, dlrow, batch,
                               out, dloss + s0);
            MLP_TRY(hipGetLastError());
        }
    }
    if (loss_out && nsteps)
        MLP_TRY(hipMemcpyAsync(loss_out, dloss, sizeof(float) * nsteps, hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    mlp_free(m, didx);
    mlp_free(m, dloss);
    mlp_free(m, dlrow);
    return TITAN_OK;
}

extern "C" int titan_mlp_predict(titan_mlp *m, int64_t n, const float *X, float *out)
{
    if (!m || n < 0 || (n > 0 && (!X || !out)))
        return fail(TITAN_EINVAL, "bad predict arguments");
    std::lock_guard<std::mutex> lk(m->mu);
    const int in = m->dims[0], O = m->dims.back();
    const int B = 4096;
    if (int rc = ensure_cap(m, std::min<int64_t>(std::max<int64_t>(n, 1), B)))
        return rc;
    for (int64_t a = 0; a < n; a += m->cap) {
        const int c = (int)std::min<int64_t>(m->cap, n - a);
        if (int rc = upload_batch_f32(m, c, X + a * in, nullptr))
            return rc;
        if (int rc = forward(m, c, m->L()))
            return rc;
        MLP_TRY(hipMemcpyAsync(out + a * O, m->zs[m->L() - 1], sizeof(float) * (size_t)c * O, hipMemcpyDeviceToHost,
                               m->stream));
        MLP_TRY(hipStreamSynchronize(m->stream));
    }
    return TITAN_OK;
}

extern "C" int titan_mlp_grad(titan_mlp *m, int32_t batch, const float *X, const float *Y, float *loss,
                              float *grads)
{
    if (!m || batch < 1 || !X || !Y)
        return fail(TITAN_EINVAL, "bad gradient arguments");
    std::lock_guard<std::mutex> lk(m->mu);
    if (int rc = ensure_cap(m, batch))
        return rc;
    if (int rc = upload_batch_f32(m, batch, X, Y))
        return rc;
    float *dloss = nullptr, *dlrow = nullptr;
    if (int rc = mlp_alloc(m, sizeof(float), (void **)&dloss))
        return rc;
    if (int rc = mlp_alloc(m, sizeof(float) * (size_t)batch, (void **)&dlrow))
        return rc;
    if (int rc = backward(m, batch, dlrow))
        return rc;
    hipLaunchKernelGGL(loss_rows_kernel, dim3(1), dim3(256), 0, m->stream, dlrow, batch, m->dims.back(), dloss);
    MLP_TRY(hipGetLastError());
    if (loss)
        MLP_TRY(hipMemcpyAsync(loss, dloss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    if (grads)
        MLP_TRY(hipMemcpyAsync(grads, m->G, sizeof(float) * m->nparam, hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    mlp_free(m, dloss);
    mlp_free(m, dlrow);
    return TITAN_OK;
}

extern "C" int titan_mlp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A_dev, int32_t lda, int32_t ta,
                                   const uint16_t *B_dev, int32_t ldb, int32_t tb, float *C_dev, void *stream)
{
    if (M < 0 || N < 0 || K < 0 || !A_dev || !B_dev || !C_dev)
        return fail(TITAN_EINVAL, "bad gemm arguments");
    GemmEpi ep{};
    ep.Z = C_dev;
    ep.ldz = N;
    hipStream_t st = (hipStream_t)stream;
    // a large product with a K-strided operand copies it K-contiguous first,
    // into stream-ordered memory released behind the product (without that
    // memory it runs on the strided operand directly)
    float *ws = nullptr;
    int64_t ws_floats = 0;
    const int Kp = (K + 7) / 8 * 8;
    const int64_t big_tiles = (int64_t)((N + GBN - 1) / GBN) * ((M + GBM - 1) / GBM);
    const int64_t need = (ta ? (int64_t)M * Kp : 0) + (tb ? 0 : (int64_t)N * Kp);
    if (big_tiles >= 128 && need > 0) {
        const size_t bytes = (size_t)(need + 1) / 2 * 4;
        if (hipMallocAsync((void **)&ws, bytes, st) == hipSuccess)
            ws_floats = (int64_t)(bytes / 4);
        else {
            (void)hipGetLastError();
            ws = nullptr;
        }
    }
    hipError_t e;
    if (!ta && !tb)
        e = gemm<false, false, EPI_F32>(M, N, K, A_dev, lda, B_dev, ldb, ep, st, ws, ws_floats);
    else if (!ta && tb)
        e = gemm<false, true, EPI_F32>(M, N, K, A_dev, lda, B_dev, ldb, ep, st, ws, ws_floats);
    else if (ta && !tb)
        e = gemm<true, false, EPI_F32>(M, N, K, A_dev, lda, B_dev, ldb, ep, st, ws, ws_floats);
    else
        e = gemm<true, true, EPI_F32>(M, N, K, A_dev, lda, B_dev, ldb, ep, st, ws, ws_floats);
    if (ws)
        (void)hipFreeAsync(ws, st);
    if (e != hipSuccess)
        return fail(TITAN_EDEVICE, "gemm launch: %s", hipGetErrorString(e));
    return TITAN_OK;
}

// Batched engine kernel: one workgroup per group of whole, independent bodies
// (robots).  The group's state is loaded into LDS once, stepped `nsteps`
// times with two workgroup barriers per step, and written back once, so the
// only per-step memory traffic is the spring constants, which stay cached
// (L2 / Infinity Cache) across the steps of a launch.  The per-mass force sum
// uses the same incidence order and arithmetic as the gather engines, so the
// result is bitwise identical to stepping the same system with them.
#include "step_device.h"

namespace titan {

namespace {

// LDS a workgroup of the batched kernel may use (160 KB per CU on gfx950).
constexpr size_t kBatchLdsBytes = 160 * 1024;

// DB: the state is double-buffered in LDS (5 arrays instead of 3, when the
// group fits): each step reads one buffer and writes the other, so one
// barrier per step suffices instead of two.
template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, bool YIELD, int T, int MAXM, bool DB>
__global__ __launch_bounds__(T) void batch_step_kernel(GatherGraph g, BatchLayout b, StateIO io, StepConsts sc,
                                                       int nsteps)
{
    extern __shared__ float4 smem[];
    const int cap = b.max_group;
    float4 *sX = smem;
    float4 *sUa = smem + cap, *sVa = smem + 2 * cap;
    float4 *sUb = DB ? smem + 3 * cap : sUa, *sVb = DB ? smem + 4 * cap : sVa;
    // wave law with offset tables: the step's sine of each of the group's
    // distinct offsets, after the state arrays (two tables with DB)
    float *sW = (float *)(smem + (DB ? 5 : 3) * cap);
    const bool wtab = WAVE && b.wave_cls != nullptr;
    if (wtab)
        g.wave_cls = b.wave_cls;
    const int64_t w0 = wtab ? b.wave_off[blockIdx.x] : 0;
    const int nw = wtab ? (int)(b.wave_off[blockIdx.x + 1] - w0) : 0;
    const int64_t m0 = b.mass_off[blockIdx.x];
    const int nm = (int)(b.mass_off[blockIdx.x + 1] - m0);
    const int tid = threadIdx.x;
    auto table = [&](int s) { return sW + ((DB && (s & 1)) ? b.max_wave : 0); };
    // the table of step s is written before a barrier that every reader of
    // that table's previous contents has passed (the staging barrier for
    // step 0; then the last barrier of step s - 1, or with DB any point of
    // step s - 1), so it costs no barrier of its own
    auto fill_table = [&](int s) {
        const double ts = (double)(sc.step + s) * sc.dt64;
        float *tab = table(s);
        for (int c = tid; c < nw; c += T)
            tab[c] = wave_sine(ts, b.wave_t[w0 + c], sc);
    };
    for (int q = tid; q < nm; q += T) {
        sX[q] = g.X0[m0 + q];
        sUa[q] = io.U_in[m0 + q];
        sVa[q] = io.V_in[m0 + q];
    }
    if (wtab && nsteps > 0)
        fill_table(0);
    __syncthreads();

    for (int s = 0; s < nsteps; ++s) {
        const bool odd = DB && (s & 1);
        const float4 *sU = odd ? sUb : sUa, *sV = odd ? sVb : sVa;  // this step's state
        float4 *nU = DB ? (odd ? sUa : sUb) : sUa, *nV = DB ? (odd ? sVa : sVb) : sVa;  // the next
        const Clock ck{(ACT && !WAVE) ? sc.trig[s] : make_float2(0.f, 1.f), (double)(sc.step + s) * sc.dt64,
                       wtab ? table(s) : nullptr};
        float4 nu[DB ? 1 : MAXM], nv[DB ? 1 : MAXM];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < MAXM; ++k) {
            const int q = tid + k * T;
            if (q < nm) {
                const int64_t i = m0 + q;
                const float4 xi = sX[q], ui = sU[q], vi = sV[q];
                const int64_t base = g.slice_off[i >> 6] + (i & 63);
                float fx = 0.f, fy = 0.f, fz = 0.f;
                // a slot's break is recorded and read back by this same thread
                // (a mass's row belongs to one thread for the whole launch)
                sum_forces<ACT, DAMP, DAMPV, REST, false, WAVE, YIELD ? 2 : 0>(
                    g, base, slice_width(g, i), xi, ui, vi, ck, sc, [&](int64_t e) { return (int)b.nbr_group[e]; },
                    [&](int r, float4 &xj, float4 &uj, float4 &vj) {
                        uj = sU[r];
                        xj = sX[r];
                        vj = DAMP ? sV[r] : make_float4(0.f, 0.f, 0.f, 0.f);
                    },
                    fx, fy, fz);
                if (DB) {
                    float4 uo, vo;
                    ok &= integrate_mass(xi, ui, vi, fx, fy, fz, sc, uo, vo);
                    nU[q] = uo;  // nobody reads this buffer during this step
                    nV[q] = vo;
                } else {
                    ok &= integrate_mass(xi, ui, vi, fx, fy, fz, sc, nu[DB ? 0 : k], nv[DB ? 0 : k]);
                }
            }
        }
        if (!ok)
            atomicMin(io.first_bad, (unsigned long long)(sc.step + s));
        if (!DB) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < MAXM; ++k) {
                const int q = tid + k * T;
                if (q < nm) {
                    nU[q] = nu[DB ? 0 : k];
                    nV[q] = nv[DB ? 0 : k];
                }
            }
        }
        if (wtab && s + 1 < nsteps)
            fill_table(s + 1);
        __syncthreads();
    }

    const bool odd = DB && (nsteps & 1);
    const float4 *sU = odd ? sUb : sUa, *sV = odd ? sVb : sVa;
    for (int q = tid; q < nm; q += T) {
        io.U_out[m0 + q] = sU[q];
        io.V_out[m0 + q] = sV[q];
    }
}

template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, bool YIELD, int T, int MAXM, bool DB>
hipError_t launch_db(const GatherGraph &g, const BatchLayout &b, const StateIO &io, const StepConsts &sc,
                     int nsteps, size_t lds, hipStream_t st)
{
    auto kern = batch_step_kernel<ACT, WAVE, DAMP, DAMPV, REST, YIELD, T, MAXM, DB>;
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)b.n_groups), dim3(T), lds, st, g, b, io, sc, nsteps);
    return hipGetLastError();
}

// Double-buffered state when the group (and, with the wave law, two offset
// tables) fits in LDS, else the single-buffered kernel.
template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, bool YIELD, int T, int MAXM>
hipError_t launch_tm(const GatherGraph &g, const BatchLayout &b, const StateIO &io, const StepConsts &sc,
                     int nsteps, hipStream_t st)
{
    const size_t tab = WAVE && b.wave_cls ? (size_t)b.max_wave * sizeof(float) : 0;
    const size_t lds_db = (size_t)b.max_group * 5 * sizeof(float4) + 2 * tab;
    if (lds_db <= kBatchLdsBytes)
        return launch_db<ACT, WAVE, DAMP, DAMPV, REST, YIELD, T, MAXM, true>(g, b, io, sc, nsteps, lds_db, st);
    return launch_db<ACT, WAVE, DAMP, DAMPV, REST, YIELD, T, MAXM, false>(
        g, b, io, sc, nsteps, (size_t)b.max_group * 3 * sizeof(float4) + tab, st);
}

template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, bool YIELD, int T>
hipError_t launch_t(const GatherGraph &g, const BatchLayout &b, const StateIO &io, const StepConsts &sc, int nsteps,
                    hipStream_t st)
{
    const int per = (b.max_group + T - 1) / T;
    if (per <= 1)
        return launch_tm<ACT, WAVE, DAMP, DAMPV, REST, YIELD, T, 1>(g, b, io, sc, nsteps, st);
    if (per <= 2)
        return launch_tm<ACT, WAVE, DAMP, DAMPV, REST, YIELD, T, 2>(g, b, io, sc, nsteps, st);
    if (per <= 4)
        return launch_tm<ACT, WAVE, DAMP, DAMPV, REST, YIELD, T, 4>(g, b, io, sc, nsteps, st);
    if (per <= 8)
        return launch_tm<ACT, WAVE, DAMP, DAMPV, REST, YIELD, T, 8>(g, b, io, sc, nsteps, st);
    return hipErrorInvalidValue;
}

template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, bool YIELD = false>
hipError_t launch4(const GatherGraph &g, const BatchLayout &b, const StateIO &io, const StepConsts &sc, int nsteps,
                   int threads, hipStream_t st)
{
    switch (threads) {
    case 256: return launch_t<ACT, WAVE, DAMP, DAMPV, REST, YIELD, 256>(g, b, io, sc, nsteps, st);
    case 512: return launch_t<ACT, WAVE, DAMP, DAMPV, REST, YIELD, 512>(g, b, io, sc, nsteps, st);
    case 1024: return launch_t<ACT, WAVE, DAMP, DAMPV, REST, YIELD, 1024>(g, b, io, sc, nsteps, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_batch(const GatherGraph &g, const BatchLayout &b, const StateIO &io, const StepConsts &sc,
                        int nsteps, int threads, hipStream_t stream)
{
    if (b.n_groups == 0 || nsteps <= 0)
        return hipSuccess;
    const bool act = g.act_c != nullptr, wave = act && g.t_off != nullptr, dampv = g.c != nullptr,
               rest = g.d0 != nullptr;
    const bool damp = dampv || g.c_uniform != 0.f;
    // breakable springs come with per-slot damping and rest lengths
    const bool yield = g.yield != nullptr;
    if (yield && !(dampv && rest))
        return hipErrorInvalidValue;
    const int key = (act ? 8 : 0) | (damp ? 4 : 0) | (dampv ? 2 : 0) | (rest ? 1 : 0) | (wave ? 16 : 0) |
                    (yield ? 32 : 0);
    switch (key) {
    case 0: return launch4<false, false, false, false, false>(g, b, io, sc, nsteps, threads, stream);
    case 1: return launch4<false, false, false, false, true>(g, b, io, sc, nsteps, threads, stream);
    case 4: return launch4<false, false, true, false, false>(g, b, io, sc, nsteps, threads, stream);
    case 5: return launch4<false, false, true, false, true>(g, b, io, sc, nsteps, threads, stream);
    case 6: return launch4<false, false, true, true, false>(g, b, io, sc, nsteps, threads, stream);
    case 7: return launch4<false, false, true, true, true>(g, b, io, sc, nsteps, threads, stream);
    case 8: return launch4<true, false, false, false, false>(g, b, io, sc, nsteps, threads, stream);
    case 9: return launch4<true, false, false, false, true>(g, b, io, sc, nsteps, threads, stream);
    case 12: return launch4<true, false, true, false, false>(g, b, io, sc, nsteps, threads, stream);
    case 13: return launch4<true, false, true, false, true>(g, b, io, sc, nsteps, threads, stream);
    case 14: return launch4<true, false, true, true, false>(g, b, io, sc, nsteps, threads, stream);
    case 15: return launch4<true, false, true, true, true>(g, b, io, sc, nsteps, threads, stream);
    case 24: return launch4<true, true, false, false, false>(g, b, io, sc, nsteps, threads, stream);
    case 25: return launch4<true, true, false, false, true>(g, b, io, sc, nsteps, threads, stream);
    case 28: return launch4<true, true, true, false, false>(g, b, io, sc, nsteps, threads, stream);
    case 29: return launch4<true, true, true, false, true>(g, b, io, sc, nsteps, threads, stream);
    case 30: return launch4<true, true, true, true, false>(g, b, io, sc, nsteps, threads, stream);
    case 31: return launch4<true, true, true, true, true>(g, b, io, sc, nsteps, threads, stream);
    case 39: return launch4<false, false, true, true, true, true>(g, b, io, sc, nsteps, threads, stream);
    case 47: return launch4<true, false, true, true, true, true>(g, b, io, sc, nsteps, threads, stream);
    case 63: return launch4<true, true, true, true, true, true>(g, b, io, sc, nsteps, threads, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace titan

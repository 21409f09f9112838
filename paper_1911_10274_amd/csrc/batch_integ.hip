// Velocity Verlet and RK4 (Sec. III-B) on the batched engine: one workgroup
// per group of whole bodies, the group's state in LDS, many steps per launch.
// Every force evaluation and stage update uses the same device functions, in
// the same order, as the per-step engines, so all engines give identical bits.
//
// Verlet: each mass's carried acceleration sits in a register for the whole
// launch (read from, and written back to, the sim's acceleration buffer); a
// step drifts every mass in LDS, evaluates the forces at the drifted state
// and kicks (three workgroup barriers).  RK4: the step's starting state and
// the running sums sit in registers; the four stage states pass through LDS
// (two barriers per stage).
#include "step_device.h"
#include "titan.h"

namespace titan {

namespace {

constexpr int kIntegThreads = 512;

template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, bool YIELD, int INTEG, int MAXM>
__global__ __launch_bounds__(kIntegThreads) void batch_integ_kernel(GatherGraph g, BatchLayout b, StateIO io,
                                                                    StepConsts sc, int nsteps, int acc_valid)
{
    constexpr int T = kIntegThreads;
    extern __shared__ float4 smem[];
    const int cap = b.max_group;
    float4 *sX = smem;
    float4 *sU = smem + cap;
    float4 *sV = smem + 2 * cap;
    const int64_t m0 = b.mass_off[blockIdx.x];
    const int nm = (int)(b.mass_off[blockIdx.x + 1] - m0);
    const int tid = threadIdx.x;
    for (int q = tid; q < nm; q += T) {
        sX[q] = g.X0[m0 + q];
        sU[q] = io.U_in[m0 + q];
        sV[q] = io.V_in[m0 + q];
    }
    __syncthreads();

    // smooth acceleration of group mass q at the LDS state, clock ck
    auto accel_at = [&](int q, const Clock &ck) {
        const int64_t i = m0 + q;
        const float4 xi = sX[q], ui = sU[q], vi = sV[q];
        float fx = 0.f, fy = 0.f, fz = 0.f;
        sum_forces<ACT, DAMP, DAMPV, REST, false, WAVE, YIELD ? 2 : 0>(
            g, g.slice_off[i >> 6] + (i & 63), slice_width(g, i), xi, ui, vi, ck, sc,
            [&](int64_t e) { return (int)b.nbr_group[e]; },
            [&](int r, float4 &xj, float4 &uj, float4 &vj) {
                uj = sU[r];
                xj = sX[r];
                vj = DAMP ? sV[r] : make_float4(0.f, 0.f, 0.f, 0.f);
            },
            fx, fy, fz);
        return smooth_accel(xi, ui, fx, fy, fz, sc);
    };
    // clock of step index n at t = n dt + c dt; phasor entry e of the chunk's table
    auto clock = [&](int64_t n, double c, int e) {
        return Clock{(ACT && !WAVE) ? sc.trig[e] : make_float2(0.f, 1.f), step_time(n, sc.dt64, c * sc.dt64)};
    };

    float4 nu[MAXM], nv[MAXM];
    if (INTEG == TITAN_INTEG_VERLET) {
        float4 a[MAXM];
#pragma unroll
        for (int k = 0; k < MAXM; ++k) {
            const int q = tid + k * T;
            a[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (q < nm) {
                if (acc_valid) {
                    a[k] = io.A_in[m0 + q];
                } else {
                    const float3 a3 = accel_at(q, clock(sc.step, 0.0, 0));
                    a[k] = make_float4(a3.x, a3.y, a3.z, 0.f);
                }
            }
        }
        // every neighbour read of that evaluation ends before the first drift
        // writes the state
        if (!acc_valid)
            __syncthreads();
        for (int s = 0; s < nsteps; ++s) {
            const int64_t n = sc.step + s;
            float zb[MAXM];
            // drift (every read of the previous step's state ended at its last barrier)
#pragma unroll
            for (int k = 0; k < MAXM; ++k) {
                const int q = tid + k * T;
                zb[k] = 0.f;
                if (q < nm) {
                    float4 u = sU[q], v = sV[q];
                    zb[k] = sX[q].z + u.z;
                    verlet_drift(u, v, a[k], sc.dt, u, v);
                    sU[q] = u;
                    sV[q] = v;
                }
            }
            __syncthreads();
            const Clock ck = clock(n, 1.0, s + 1);
            bool ok = true;
#pragma unroll
            for (int k = 0; k < MAXM; ++k) {
                const int q = tid + k * T;
                if (q < nm) {
                    const float3 a3 = accel_at(q, ck);
                    verlet_kick(sU[q], sV[q], a3, zb[k], sc, nu[k], nv[k]);
                    a[k] = make_float4(a3.x, a3.y, a3.z, 0.f);
                    ok &= finite4(nu[k], nv[k]);
                }
            }
            if (!ok)
                atomicMin(io.first_bad, (unsigned long long)n);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < MAXM; ++k) {
                const int q = tid + k * T;
                if (q < nm) {
                    sU[q] = nu[k];
                    sV[q] = nv[k];
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < MAXM; ++k) {
            const int q = tid + k * T;
            if (q < nm)
                io.A[m0 + q] = a[k];
        }
    } else {
        float4 ub[MAXM], vb[MAXM], su[MAXM], sv[MAXM];
        for (int s = 0; s < nsteps; ++s) {
            const int64_t n = sc.step + s;
#pragma unroll
            for (int k = 0; k < MAXM; ++k) {
                const int q = tid + k * T;
                ub[k] = vb[k] = su[k] = sv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (q < nm) {
                    ub[k] = sU[q];
                    vb[k] = sV[q];
                }
            }
            bool ok = true;
            for (int st = kStageRk1; st <= kStageRk4; ++st) {
                const double c = st == kStageRk1 ? 0.0 : (st == kStageRk4 ? 1.0 : 0.5);
                const Clock ck = clock(n, c, 2 * s + (int)(2 * c));
#pragma unroll
                for (int k = 0; k < MAXM; ++k) {
                    const int q = tid + k * T;
                    if (q < nm) {
                        const float4 xi = sX[q], ui = sU[q], vi = sV[q];
                        const float3 a3 = accel_at(q, ck);
                        if (ui.w == 0.f) {  // pinned
                            nu[k] = ub[k];
                            nv[k] = vb[k];
                        } else {
                            rk_sums(st, vi, a3, su[k], sv[k]);
                            if (st != kStageRk4) {
                                rk_next(st, ub[k], vb[k], vi, a3, sc.dt, nu[k], nv[k]);
                            } else {
                                rk_final(ub[k], vb[k], su[k], sv[k], xi.z + ub[k].z, sc, nu[k], nv[k]);
                                ok &= finite4(nu[k], nv[k]);
                            }
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < MAXM; ++k) {
                    const int q = tid + k * T;
                    if (q < nm) {
                        sU[q] = nu[k];
                        sV[q] = nv[k];
                    }
                }
                __syncthreads();
            }
            if (!ok)
                atomicMin(io.first_bad, (unsigned long long)n);
        }
    }

    for (int q = tid; q < nm; q += T) {
        io.U_out[m0 + q] = sU[q];
        io.V_out[m0 + q] = sV[q];
    }
}

template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, bool YIELD, int INTEG, int MAXM>
hipError_t launch_m(const GatherGraph &g, const BatchLayout &b, const StateIO &io, const StepConsts &sc, int nsteps,
                    int acc_valid, hipStream_t st)
{
    auto kern = batch_integ_kernel<ACT, WAVE, DAMP, DAMPV, REST, YIELD, INTEG, MAXM>;
    const size_t lds = (size_t)b.max_group * 3 * sizeof(float4);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)b.n_groups), dim3(kIntegThreads), lds, st, g, b, io, sc, nsteps,
                       acc_valid);
    return hipGetLastError();
}

template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, bool YIELD = false>
hipError_t launch4(const GatherGraph &g, const BatchLayout &b, const StateIO &io, const StepConsts &sc, int nsteps,
                   int integ, int acc_valid, hipStream_t st)
{
    const int per = (b.max_group + kIntegThreads - 1) / kIntegThreads;
    if (integ == TITAN_INTEG_VERLET) {
        if (per <= 1)
            return launch_m<ACT, WAVE, DAMP, DAMPV, REST, YIELD, TITAN_INTEG_VERLET, 1>(g, b, io, sc, nsteps,
                                                                                        acc_valid, st);
        if (per <= 2)
            return launch_m<ACT, WAVE, DAMP, DAMPV, REST, YIELD, TITAN_INTEG_VERLET, 2>(g, b, io, sc, nsteps,
                                                                                        acc_valid, st);
        if (per <= 4)
            return launch_m<ACT, WAVE, DAMP, DAMPV, REST, YIELD, TITAN_INTEG_VERLET, 4>(g, b, io, sc, nsteps,
                                                                                        acc_valid, st);
        if (per <= 8)
            return launch_m<ACT, WAVE, DAMP, DAMPV, REST, YIELD, TITAN_INTEG_VERLET, 8>(g, b, io, sc, nsteps,
                                                                                        acc_valid, st);
    } else {
        if (per <= 1)
            return launch_m<ACT, WAVE, DAMP, DAMPV, REST, YIELD, TITAN_INTEG_RK4, 1>(g, b, io, sc, nsteps, acc_valid,
                                                                                     st);
        if (per <= 2)
            return launch_m<ACT, WAVE, DAMP, DAMPV, REST, YIELD, TITAN_INTEG_RK4, 2>(g, b, io, sc, nsteps, acc_valid,
                                                                                     st);
        if (per <= 4)
            return launch_m<ACT, WAVE, DAMP, DAMPV, REST, YIELD, TITAN_INTEG_RK4, 4>(g, b, io, sc, nsteps, acc_valid,
                                                                                     st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool batch_integ_fits(const BatchLayout &b, int integ)
{
    const int per = (b.max_group + kIntegThreads - 1) / kIntegThreads;
    return integ == TITAN_INTEG_VERLET ? per <= 8 : per <= 4;
}

bool batch_integ_preferred(const BatchLayout &b)
{
    // at most two masses per thread: beyond, the serial masses per thread and
    // the extra barriers cost more than the per-step engines' launches
    return (b.max_group + kIntegThreads - 1) / kIntegThreads <= 2;
}

hipError_t launch_batch_integ(const GatherGraph &g, const BatchLayout &b, const StateIO &io, const StepConsts &sc,
                              int nsteps, int integ, int acc_valid, hipStream_t stream)
{
    if (b.n_groups == 0 || nsteps <= 0)
        return hipSuccess;
    const bool act = g.act_c != nullptr, wave = act && g.t_off != nullptr, dampv = g.c != nullptr,
               rest = g.d0 != nullptr;
    const bool damp = dampv || g.c_uniform != 0.f;
    const bool yield = g.yield != nullptr;
    if (yield && !(dampv && rest))
        return hipErrorInvalidValue;
    const int key = (act ? 8 : 0) | (damp ? 4 : 0) | (dampv ? 2 : 0) | (rest ? 1 : 0) | (wave ? 16 : 0) |
                    (yield ? 32 : 0);
#define TITAN_I(...) return launch4<__VA_ARGS__>(g, b, io, sc, nsteps, integ, acc_valid, stream)
    switch (key) {
    case 0: TITAN_I(false, false, false, false, false);
    case 1: TITAN_I(false, false, false, false, true);
    case 4: TITAN_I(false, false, true, false, false);
    case 5: TITAN_I(false, false, true, false, true);
    case 6: TITAN_I(false, false, true, true, false);
    case 7: TITAN_I(false, false, true, true, true);
    case 8: TITAN_I(true, false, false, false, false);
    case 9: TITAN_I(true, false, false, false, true);
    case 12: TITAN_I(true, false, true, false, false);
    case 13: TITAN_I(true, false, true, false, true);
    case 14: TITAN_I(true, false, true, true, false);
    case 15: TITAN_I(true, false, true, true, true);
    case 24: TITAN_I(true, true, false, false, false);
    case 25: TITAN_I(true, true, false, false, true);
    case 28: TITAN_I(true, true, true, false, false);
    case 29: TITAN_I(true, true, true, false, true);
    case 30: TITAN_I(true, true, true, true, false);
    case 31: TITAN_I(true, true, true, true, true);
    case 39: TITAN_I(false, false, true, true, true, true);
    case 47: TITAN_I(true, false, true, true, true, true);
    case 63: TITAN_I(true, true, true, true, true, true);
    default: return hipErrorInvalidValue;
    }
#undef TITAN_I
}

}  // namespace titan

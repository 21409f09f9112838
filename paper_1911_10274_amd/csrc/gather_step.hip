// Step kernels of the gather engine: one thread per mass, fused spring force
// + mass update.
//
// The paper (Sec. III-B) alternates a spring pass that adds Hooke forces to
// both ends (atomics by default) with a mass pass that integrates.  Here each
// mass walks its own incidence list in a fixed order and evaluates every
// incident spring itself, so a spring is evaluated once from each end, no
// atomics are needed and the per-mass sum order -- hence the result -- is the
// same on every run and in both kernels below.
//
// untiled: neighbours' state is read from global memory (L2).
// tiled:   a workgroup owns a tile of kTile consecutive masses; it first
//          stages the tile's state and its halo (the outside masses its
//          springs reach) in LDS, then every neighbour read is an LDS read
//          through a 16-bit tile-local index.  Tiles are assigned to
//          workgroups so that each XCD walks a contiguous range.
#include "step_device.h"

namespace titan {

namespace {

// What a launch does after the force sum: an Euler step, a force query, or
// one stage of another integrator (StepConsts::stage).
constexpr int kModeStep = 0, kModeForces = 1, kModeStage = 2;

// Sum-of-forces mode of a kernel: breakable springs are tested, and their
// breaks recorded unless the launch only queries the forces.
template <bool YIELD, int MODE>
constexpr int yield_mode = YIELD ? (MODE == kModeForces ? 1 : 2) : 0;

// Slots per load batch of the tiled kernel: more in flight for the lean
// phasor-law slots (about 18 more registers, within what three 512-mass tiles
// per CU allow), the default where a slot carries more state.
template <bool WAVE, bool DAMPV, bool REST, bool YIELD>
constexpr int plain_unroll = (WAVE || DAMPV || REST || YIELD) ? kUnroll : kUnrollPlain;

template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, int MODE, bool YIELD>
__global__ __launch_bounds__(256) void untiled_step_kernel(GatherGraph g, StateIO io, StepConsts sc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n)
        return;
    // the Verlet kick evaluates the drifted state of every mass it reads
    const bool drifting = MODE == kModeStage && sc.stage == kStageVerletKick;
    float4 ui = io.U_in[i];
    float4 vi = io.V_in[i];
    if (drifting)
        verlet_drift(ui, vi, io.A_in[i], sc.dt, ui, vi);
    const float4 xi = g.X0[i];
    const int64_t base = g.slice_off[i >> 6] + (i & 63);
    float fx = 0.f, fy = 0.f, fz = 0.f;
    const int64_t n = step_index(sc);
    const Clock ck{(ACT && !WAVE) ? *sc.trig : make_float2(0.f, 1.f), step_time(n, sc.dt64, sc.t_add)};
    sum_forces<ACT, DAMP, DAMPV, REST, TITAN_NT_LOADS != 0, WAVE, yield_mode<YIELD, MODE>>(
        g, base, slice_width(g, i), xi, ui, vi, ck, sc, [&](int64_t e) { return stream_load(g.nbr + e); },
        [&](int j, float4 &xj, float4 &uj, float4 &vj) {
            uj = io.U_in[j];
            xj = g.X0[j];
            if (MODE == kModeStage && drifting) {
                float4 vv = io.V_in[j];
                verlet_drift(uj, vv, io.A_in[j], sc.dt, uj, vv);
                vj = DAMP ? vv : make_float4(0.f, 0.f, 0.f, 0.f);
            } else {
                vj = DAMP ? io.V_in[j] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        },
        fx, fy, fz);
    if (MODE == kModeForces) {
        io.F_out[i] = make_float4(fx, fy, fz, 0.f);
        return;
    }
    if (MODE == kModeStage) {
        if (!stage_update(i, xi, ui, vi, fx, fy, fz, io, sc))
            atomicMin(io.first_bad, (unsigned long long)n);
        return;
    }
    float4 uo, vo;
    const bool ok = integrate_mass(xi, ui, vi, fx, fy, fz, sc, uo, vo);
    io.U_out[i] = uo;
    io.V_out[i] = vo;
    if (!ok)
        atomicMin(io.first_bad, (unsigned long long)n);
}

template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, int MODE, bool YIELD>
__global__ __launch_bounds__(kTile) void tiled_step_kernel(GatherGraph g, StateIO io, StepConsts sc)
{
    extern __shared__ float4 smem[];
    const int L = g.max_local;
    float4 *sU = smem;
    float4 *sX = smem + L;
    float4 *sV = smem + 2 * L;  // only with damping
    // wave law with offset tables: the step's sine of each of the tile's
    // distinct offsets, after the state arrays
    float *sW = (float *)(smem + (DAMP ? 3 : 2) * L);

    const unsigned t = xcd_tile(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)t * kTile + tid;
    const bool valid = i < g.n;
    const bool wtab = WAVE && g.tile_wave_cls != nullptr;
    if (wtab) {
        g.wave_cls = g.tile_wave_cls;
        const double tn = step_time(step_index(sc), sc.dt64, sc.t_add);
        const int64_t w0 = g.tile_wave_off[t];
        const int nw = (int)(g.tile_wave_off[t + 1] - w0);
        for (int c = tid; c < nw; c += kTile)
            sW[c] = wave_sine(tn, g.tile_wave_t[w0 + c], sc);  // read after the staging barrier
    }
    // the Verlet kick stages the drifted state of the tile and its halo
    const bool drifting = MODE == kModeStage && sc.stage == kStageVerletKick;
    float4 ui = make_float4(0.f, 0.f, 0.f, 0.f), vi = ui, xi = ui;
    if (valid) {
        ui = io.U_in[i];
        vi = io.V_in[i];
        if (MODE == kModeStage && drifting)
            verlet_drift(ui, vi, io.A_in[i], sc.dt, ui, vi);
        xi = g.X0[i];
        sU[tid] = ui;
        sX[tid] = xi;
        if (DAMP)
            sV[tid] = vi;
    }
    const int64_t hb = g.halo_off[t], he = g.halo_off[t + 1];
    for (int64_t h = hb + tid; h < he; h += kTile) {
        const int j = g.halo_idx[h];
        const int q = kTile + (int)(h - hb);
        float4 uj = io.U_in[j];
        if (MODE == kModeStage && drifting) {
            float4 vj = io.V_in[j];
            verlet_drift(uj, vj, io.A_in[j], sc.dt, uj, vj);
            if (DAMP)
                sV[q] = vj;
        } else if (DAMP) {
            sV[q] = io.V_in[j];
        }
        sU[q] = uj;
        sX[q] = g.X0[j];
    }
    __syncthreads();
    if (!valid)
        return;

    const int64_t base = g.slice_off[i >> 6] + (i & 63);
    float fx = 0.f, fy = 0.f, fz = 0.f;
    const int64_t n = step_index(sc);
    const Clock ck{(ACT && !WAVE) ? *sc.trig : make_float2(0.f, 1.f), step_time(n, sc.dt64, sc.t_add),
                   wtab ? sW : nullptr};
    sum_forces<ACT, DAMP, DAMPV, REST, TITAN_NT_LOADS != 0, WAVE, yield_mode<YIELD, MODE>,
               plain_unroll<WAVE, DAMPV, REST, YIELD>>(
        g, base, slice_width(g, i), xi, ui, vi, ck, sc, [&](int64_t e) { return (int)stream_load(g.nbr_local + e); },
        [&](int q, float4 &xj, float4 &uj, float4 &vj) {
            uj = sU[q];
            xj = sX[q];
            vj = DAMP ? sV[q] : make_float4(0.f, 0.f, 0.f, 0.f);
        },
        fx, fy, fz);
    if (MODE == kModeForces) {
        io.F_out[i] = make_float4(fx, fy, fz, 0.f);
        return;
    }
    if (MODE == kModeStage) {
        if (!stage_update(i, xi, ui, vi, fx, fy, fz, io, sc))
            atomicMin(io.first_bad, (unsigned long long)n);
        return;
    }
    float4 uo, vo;
    const bool ok = integrate_mass(xi, ui, vi, fx, fy, fz, sc, uo, vo);
    io.U_out[i] = uo;
    io.V_out[i] = vo;
    if (!ok)
        atomicMin(io.first_bad, (unsigned long long)n);
}

template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, bool YIELD, int MODE>
void launch_mode(const GatherGraph &g, const StateIO &io, const StepConsts &sc, bool tiled, hipStream_t st)
{
    if (tiled) {
        const dim3 grid((unsigned)g.n_tiles), block(kTile);
        const size_t lds = (size_t)g.max_local * sizeof(float4) * (DAMP ? 3 : 2) +
                           (WAVE && g.tile_wave_cls ? (size_t)g.max_tile_wave * sizeof(float) : 0);
        hipLaunchKernelGGL((tiled_step_kernel<ACT, WAVE, DAMP, DAMPV, REST, MODE, YIELD>), grid, block, lds, st, g,
                           io, sc);
    } else {
        const dim3 grid((unsigned)((g.n + 255) / 256)), block(256);
        hipLaunchKernelGGL((untiled_step_kernel<ACT, WAVE, DAMP, DAMPV, REST, MODE, YIELD>), grid, block, 0, st, g,
                           io, sc);
    }
}

template <bool ACT, bool WAVE, bool DAMP, bool DAMPV, bool REST, bool YIELD = false>
hipError_t launch4(const GatherGraph &g, const StateIO &io, const StepConsts &sc, int mode, bool tiled,
                   hipStream_t st)
{
    if (mode == kModeForces)
        launch_mode<ACT, WAVE, DAMP, DAMPV, REST, YIELD, kModeForces>(g, io, sc, tiled, st);
    else if (mode == kModeStage)
        launch_mode<ACT, WAVE, DAMP, DAMPV, REST, YIELD, kModeStage>(g, io, sc, tiled, st);
    else
        launch_mode<ACT, WAVE, DAMP, DAMPV, REST, YIELD, kModeStep>(g, io, sc, tiled, st);
    return hipGetLastError();
}

__global__ void trig_table_kernel(float2 *trig, int64_t first, int count, double omega, double dt)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count)
        return;
    const double ph = omega * ((double)(first + s) * dt);
    trig[s] = make_float2((float)sin(ph), (float)cos(ph));
}

// The same table with its first step read from the device clock (a node of a
// captured step loop).
__global__ void trig_table_clock_kernel(float2 *trig, const int64_t *clock, int count, double omega, double dt)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count)
        return;
    const double ph = omega * ((double)(*clock + s) * dt);
    trig[s] = make_float2((float)sin(ph), (float)cos(ph));
}

// *clock = value (add == 0) or *clock += add: one thread, a vector store.
__global__ void clock_kernel(int64_t *clock, int64_t value, int64_t add)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *clock = add ? *clock + add : value;
}

__global__ void scatter_kernel(float *dst, const int64_t *slot, const float *val, int64_t m)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m)
        dst[slot[q]] = val[q];
}

template <class T>
__global__ void scatter_bits_kernel(T *dst, const int64_t *slot, const T *val, int64_t m)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m)
        dst[slot[q]] = val[q];
}

// disp[b] = sum_i w_i u_i over body b's internal masses [off[b], off[b+1]),
// w_i = m_i / M_b: the body's centre-of-mass displacement (one thread per
// body, masses in index order).
__global__ void body_disp_kernel(const float4 *U, const float *w, const int64_t *off, int64_t nb, float *disp)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb)
        return;
    float x = 0.f, y = 0.f, z = 0.f;
    for (int64_t i = off[b]; i < off[b + 1]; ++i) {
        const float4 u = U[i];
        x = fmaf(w[i], u.x, x);
        y = fmaf(w[i], u.y, y);
        z = fmaf(w[i], u.z, z);
    }
    disp[3 * b] = x;
    disp[3 * b + 1] = y;
    disp[3 * b + 2] = z;
}

__global__ void fill_kernel(float *dst, float v, int64_t m)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m)
        dst[q] = v;
}

}  // namespace

hipError_t launch_trig_table_clock(float2 *trig, const int64_t *clock, int count, double omega, double dt,
                                   hipStream_t stream)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(trig_table_clock_kernel, dim3((count + 255) / 256), dim3(256), 0, stream, trig, clock, count,
                       omega, dt);
    return hipGetLastError();
}

hipError_t launch_clock(int64_t *clock, int64_t value, int64_t add, hipStream_t stream)
{
    hipLaunchKernelGGL(clock_kernel, dim3(1), dim3(64), 0, stream, clock, value, add);
    return hipGetLastError();
}

hipError_t launch_scatter(float *dst, const int64_t *slot, const float *val, int64_t m, hipStream_t stream)
{
    if (m <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, dst, slot, val, m);
    return hipGetLastError();
}

hipError_t launch_scatter_bits(void *dst, int bytes, const int64_t *slot, const void *val, int64_t m,
                               hipStream_t stream)
{
    if (m <= 0)
        return hipSuccess;
    const dim3 grid((unsigned)((m + 255) / 256)), block(256);
    if (bytes == 2)
        hipLaunchKernelGGL(scatter_bits_kernel<uint16_t>, grid, block, 0, stream, (uint16_t *)dst, slot,
                           (const uint16_t *)val, m);
    else if (bytes == 4)
        hipLaunchKernelGGL(scatter_bits_kernel<uint32_t>, grid, block, 0, stream, (uint32_t *)dst, slot,
                           (const uint32_t *)val, m);
    else if (bytes == 8)
        hipLaunchKernelGGL(scatter_bits_kernel<uint64_t>, grid, block, 0, stream, (uint64_t *)dst, slot,
                           (const uint64_t *)val, m);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_body_disp(const float4 *U, const float *w, const int64_t *off, int64_t nb, float *disp,
                            hipStream_t stream)
{
    if (nb <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(body_disp_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, stream, U, w, off, nb,
                       disp);
    return hipGetLastError();
}

hipError_t launch_fill(float *dst, float v, int64_t m, hipStream_t stream)
{
    if (m <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, dst, v, m);
    return hipGetLastError();
}

hipError_t launch_trig_table(float2 *trig, int64_t first, int count, double omega, double dt, hipStream_t stream)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(trig_table_kernel, dim3((count + 255) / 256), dim3(256), 0, stream, trig, first, count, omega,
                       dt);
    return hipGetLastError();
}

static hipError_t dispatch_mode(const GatherGraph &g, const StateIO &io, const StepConsts &sc, int mode, bool tiled,
                                hipStream_t stream)
{
    if (g.n == 0)
        return hipSuccess;
    const bool act = g.act_c != nullptr, wave = act && g.t_off != nullptr, dampv = g.c != nullptr,
               rest = g.d0 != nullptr;
    const bool damp = dampv || g.c_uniform != 0.f;
    tiled = tiled && g.nbr_local != nullptr;
    // (ACT, WAVE, DAMP, DAMPV, REST); WAVE implies ACT, DAMPV implies DAMP.
    // breakable springs come with per-slot damping and rest lengths
    const bool yield = g.yield != nullptr;
    if (yield && !(dampv && rest))
        return hipErrorInvalidValue;
    const int key = (act ? 8 : 0) | (damp ? 4 : 0) | (dampv ? 2 : 0) | (rest ? 1 : 0) | (wave ? 16 : 0) |
                    (yield ? 32 : 0);
    switch (key) {
    case 0: return launch4<false, false, false, false, false>(g, io, sc, mode, tiled, stream);
    case 1: return launch4<false, false, false, false, true>(g, io, sc, mode, tiled, stream);
    case 4: return launch4<false, false, true, false, false>(g, io, sc, mode, tiled, stream);
    case 5: return launch4<false, false, true, false, true>(g, io, sc, mode, tiled, stream);
    case 6: return launch4<false, false, true, true, false>(g, io, sc, mode, tiled, stream);
    case 7: return launch4<false, false, true, true, true>(g, io, sc, mode, tiled, stream);
    case 8: return launch4<true, false, false, false, false>(g, io, sc, mode, tiled, stream);
    case 9: return launch4<true, false, false, false, true>(g, io, sc, mode, tiled, stream);
    case 12: return launch4<true, false, true, false, false>(g, io, sc, mode, tiled, stream);
    case 13: return launch4<true, false, true, false, true>(g, io, sc, mode, tiled, stream);
    case 14: return launch4<true, false, true, true, false>(g, io, sc, mode, tiled, stream);
    case 15: return launch4<true, false, true, true, true>(g, io, sc, mode, tiled, stream);
    case 24: return launch4<true, true, false, false, false>(g, io, sc, mode, tiled, stream);
    case 25: return launch4<true, true, false, false, true>(g, io, sc, mode, tiled, stream);
    case 28: return launch4<true, true, true, false, false>(g, io, sc, mode, tiled, stream);
    case 29: return launch4<true, true, true, false, true>(g, io, sc, mode, tiled, stream);
    case 30: return launch4<true, true, true, true, false>(g, io, sc, mode, tiled, stream);
    case 31: return launch4<true, true, true, true, true>(g, io, sc, mode, tiled, stream);
    case 39: return launch4<false, false, true, true, true, true>(g, io, sc, mode, tiled, stream);
    case 47: return launch4<true, false, true, true, true, true>(g, io, sc, mode, tiled, stream);
    case 63: return launch4<true, true, true, true, true, true>(g, io, sc, mode, tiled, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather_step(const GatherGraph &g, const StateIO &io, const StepConsts &sc, bool forces_only,
                              bool tiled, hipStream_t stream)
{
    return dispatch_mode(g, io, sc, forces_only ? kModeForces : kModeStep, tiled, stream);
}

hipError_t launch_gather_stage(const GatherGraph &g, const StateIO &io, const StepConsts &sc, bool tiled,
                               hipStream_t stream)
{
    return dispatch_mode(g, io, sc, kModeStage, tiled, stream);
}


}  // namespace titan

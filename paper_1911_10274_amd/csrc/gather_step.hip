// Gather engine: one thread per mass, fused spring force + mass update.
//
// The paper (Sec. III-B) alternates a spring pass that adds Hooke forces to
// both ends (atomics by default) with a mass pass that integrates.  Here each
// mass instead walks its own incidence list in a fixed order and evaluates
// every incident spring itself, so a spring is evaluated once from each end,
// no atomics are needed and the per-mass sum order -- hence the result -- is
// the same on every run.  The two evaluations of one spring are exact
// negatives of each other (every operand is negated, so every rounding is the
// same), which keeps Newton's third law pairwise exact.
//
// Positions are stored as displacement u = x - x0 next to the read-only
// reference x0.  The stretch is formed without cancellation,
//     l - |R| = (2 R.du + du.du) / (l + |R|),   R = x0_j - x0_i, du = u_j - u_i,
// so that FP32 keeps relative accuracy even when a step moves a mass by less
// than one ulp of its absolute coordinate.
#include "titan_internal.h"

namespace titan {

namespace {

template <bool ACT, bool DAMPV, bool REST, bool FORCES>
__global__ __launch_bounds__(256) void gather_step_kernel(GatherGraph g, StateIO io, StepConsts sc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n)
        return;
    const float4 ui = io.U_in[i];
    const float4 vi = io.V_in[i];
    const float4 xi = g.X0[i];
    const int64_t base = g.slice_off[i >> 6] + (i & 63);
    const int deg = g.deg[i];

    float fx = 0.f, fy = 0.f, fz = 0.f;
    for (int w = 0; w < deg; ++w) {
        const int64_t e = base + (int64_t)w * kSlice;
        const int j = g.nbr[e];
        const float4 uj = io.U_in[j];
        const float4 xj = g.X0[j];
        const float Rx = xj.x - xi.x, Ry = xj.y - xi.y, Rz = xj.z - xi.z;
        const float ax = uj.x - ui.x, ay = uj.y - ui.y, az = uj.z - ui.z;
        const float dx = Rx + ax, dy = Ry + ay, dz = Rz + az;
        const float l2 = dx * dx + dy * dy + dz * dz;
        if (l2 == 0.f)
            continue;  // coincident ends: no direction, no force
        const float l = sqrtf(l2);
        const float il = 1.f / l;
        const float r = sqrtf(Rx * Rx + Ry * Ry + Rz * Rz);
        const float num = 2.f * (Rx * ax + Ry * ay + Rz * az) + (ax * ax + ay * ay + az * az);
        float stretch = num / (l + r);
        if (REST) {
            const float L0 = g.rest[e];
            stretch += g.d0[e];
            if (ACT)
                stretch -= L0 * (g.act_c[e] * sc.sin_wt + g.act_s[e] * sc.cos_wt);
        } else if (ACT) {
            stretch -= r * (g.act_c[e] * sc.sin_wt + g.act_s[e] * sc.cos_wt);
        }
        const float ux = dx * il, uy = dy * il, uz = dz * il;
        float mag = g.k[e] * stretch;
        const float c = DAMPV ? g.c[e] : g.c_uniform;
        if (DAMPV || g.c_uniform != 0.f) {
            const float4 vj = io.V_in[j];
            const float vr = (vj.x - vi.x) * ux + (vj.y - vi.y) * uy + (vj.z - vi.z) * uz;
            mag += c * vr;
        }
        fx += mag * ux;
        fy += mag * uy;
        fz += mag * uz;
    }

    if (FORCES) {
        io.F_out[i] = make_float4(fx, fy, fz, 0.f);
        return;
    }

    const float im = ui.w;  // inverse mass; 0 = pinned
    if (im == 0.f) {
        io.U_out[i] = ui;
        io.V_out[i] = vi;
        return;
    }
    float ax = fx * im + sc.gx;
    float ay = fy * im + sc.gy;
    float az = fz * im + sc.gz;
    const float z = xi.z + ui.z;
    const bool contact = sc.ground && z < 0.f;
    float fn = 0.f;
    if (contact) {
        fn = -sc.ground_k * z;
        az += fn * im;
    }
    float wx = vi.x + sc.dt * ax;
    float wy = vi.y + sc.dt * ay;
    const float wz = vi.z + sc.dt * az;
    if (contact) {
        const float vt = sqrtf(wx * wx + wy * wy);
        if (vt > 0.f) {
            const float s = fmaxf(0.f, 1.f - sc.mu * fn * sc.dt * im / vt);
            wx *= s;
            wy *= s;
        }
    }
    const float4 uo = make_float4(ui.x + sc.dt * wx, ui.y + sc.dt * wy, ui.z + sc.dt * wz, im);
    io.U_out[i] = uo;
    io.V_out[i] = make_float4(wx, wy, wz, 0.f);
    if (!(isfinite(uo.x) && isfinite(uo.y) && isfinite(uo.z) && isfinite(wx) && isfinite(wy) &&
          isfinite(wz)))
        atomicMin(io.first_bad, (unsigned long long)sc.step);
}

template <bool ACT, bool DAMPV, bool REST>
hipError_t launch3(const GatherGraph &g, const StateIO &io, const StepConsts &sc, bool forces,
                   hipStream_t st)
{
    const dim3 block(256);
    const dim3 grid((unsigned)((g.n + 255) / 256));
    if (forces)
        hipLaunchKernelGGL((gather_step_kernel<ACT, DAMPV, REST, true>), grid, block, 0, st, g, io, sc);
    else
        hipLaunchKernelGGL((gather_step_kernel<ACT, DAMPV, REST, false>), grid, block, 0, st, g, io, sc);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gather_step(const GatherGraph &g, const StateIO &io, const StepConsts &sc,
                              bool forces_only, hipStream_t stream)
{
    if (g.n == 0)
        return hipSuccess;
    const bool act = g.act_c != nullptr, dampv = g.c != nullptr, rest = g.d0 != nullptr;
    const int key = (act ? 4 : 0) | (dampv ? 2 : 0) | (rest ? 1 : 0);
    switch (key) {
    case 0: return launch3<false, false, false>(g, io, sc, forces_only, stream);
    case 1: return launch3<false, false, true>(g, io, sc, forces_only, stream);
    case 2: return launch3<false, true, false>(g, io, sc, forces_only, stream);
    case 3: return launch3<false, true, true>(g, io, sc, forces_only, stream);
    case 4: return launch3<true, false, false>(g, io, sc, forces_only, stream);
    case 5: return launch3<true, false, true>(g, io, sc, forces_only, stream);
    case 6: return launch3<true, true, false>(g, io, sc, forces_only, stream);
    default: return launch3<true, true, true>(g, io, sc, forces_only, stream);
    }
}

}  // namespace titan

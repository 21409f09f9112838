// Device-side arithmetic of one mass-spring step, shared by every kernel that
// steps the system so that all engines produce bitwise identical results.
//
// Spring force (Sec. III-B, Eq. 1 read as an axial Hooke law with damping):
// on mass i from its spring to mass j,
//     f = [k (l - L(t)) + c (v_j - v_i) . u] u,   u = (x_j - x_i) / l,
// with L(t) = L0 (1 + amp sin(omega t + phase)) (Sec. IV-B, Eq. 4) written as
// L0 (1 + C sin(omega t) + S cos(omega t)), C = amp cos(phase),
// S = amp sin(phase).  Positions are displacements u from the reference x0,
// and the stretch is formed without cancellation:
//     l - |R| = (2 R.du + du.du) / (l + |R|),  R = x0_j - x0_i,  du = u_j - u_i;
//     l - L(t) = (l - |R|) + d0 - L0 (C sin + S cos),   d0 = |R| - L0.
// When every rest length is the initial length, d0 = 0 and L0 = |R|.
//
// Breakable springs (Sec. III-E, material yield values): a spring whose
// elastic force |k (l - L(t))| exceeds its yield value Y breaks in that force
// evaluation and exerts no force from then on (its damper included).  Per
// slot, Y = +inf never breaks and Y < 0 marks a broken spring; both ends of a
// spring compute the same |k (l - L(t))| (exactly negated operands), so they
// take the same decision and each records it in its own slot.
//
// Mass update (Sec. III-B, Eq. 1: dx = xdot dt + xddot dt^2, semi-implicit
// Euler): a = F/m + g (+ ground normal force -k_g z / m while z < 0),
// v* = v + a dt; in contact, Coulomb friction scales the tangential part of
// v* by max(0, 1 - mu F_n dt / (m |v*_t|)); x += v_new dt.
#pragma once

#include <hip/hip_runtime.h>

#include "titan_internal.h"

namespace titan {

struct SpringConst {
    float k;
    float c;      // damping
    float act_c;  // amp cos(phase)
    float act_s;  // amp sin(phase)
    float d0;     // |R| - L0 (only with explicit rest lengths)
    float L0;     // rest length (only with explicit rest lengths)
    double t_off; // wave-law offset t_o (only with the wave law)
    int cls;      // wave law with a table: the offset's class in the group
    float yield;  // yield value Y; < 0: broken (only with breakable springs)
};

// Actuation clock of one step: (sin, cos)(omega t_n) for the phasor law, and
// t_n = n dt itself in FP64 for the wave law.
struct Clock {
    float2 tr;
    double t;
    const float *wtab = nullptr;  // wave law: this step's sine per offset class (batched engine), or null
};

// The FP64 time of step n plus an offset (an RK4 stage's c dt), rounded the
// same way by every kernel (product, then sum; no fused multiply-add), so
// every engine folds the wave law's period at the same instants.
__device__ __forceinline__ double step_time(int64_t n, double dt64, double add)
{
#pragma clang fp contract(off)
    return (double)n * dt64 + add;
}

// Actuation factor of one incidence: the rest length is L0 (1 + factor).
// Phasor law: C sin(omega t) + S cos(omega t) = amp sin(omega t + phase).
// Wave law (Sec. IV-B, Eqs. 3-4): amp sin(omega tau) with
// tau = (t - t_o) mod t_p in [0, t_p).  The fold is done in FP64 with the same
// operations as its definition, so which period a spring is in -- the
// factor jumps at the period boundary -- does not depend on FP32 rounding.
__device__ __forceinline__ float wave_sine(double t, double t_off, const StepConsts &sc)
{
#pragma clang fp contract(off)
    const double u = t - t_off;
    const double tau = u - sc.period * floor(u / sc.period);
    // omega tau reaches tens of radians: reduce it to [-pi, pi] in FP64
    // before the FP32 sine, so the argument's rounding is that of a number
    // below pi, not of omega tau
    constexpr double kTwoPi = 6.283185307179586, kInvTwoPi = 0.15915494309189535;
    const double arg = sc.omega * tau;
    const double red = arg - kTwoPi * rint(arg * kInvTwoPi);
    return sinf((float)red);
}

template <bool ACT, bool WAVE>
__device__ __forceinline__ float act_factor(const SpringConst &p, const Clock &ck, const StepConsts &sc)
{
#pragma clang fp contract(off)
    if (!ACT)
        return 0.f;
    if (!WAVE)
        return fmaf(p.act_c, ck.tr.x, p.act_s * ck.tr.y);
    // the same sine, from the step's table when there is one
    return p.act_c * (ck.wtab ? ck.wtab[p.cls] : wave_sine(ck.t, p.t_off, sc));
}

// Every floating-point operation below is spelled out: contraction of
// multiplies and adds into FMAs is switched off and the FMAs that are wanted
// are written as fmaf.  The rounding of each operation is therefore fixed by
// this source, not by how the compiler schedules a particular kernel, and all
// engines that step the system give identical bits.

// Force on mass i from one incident spring (xi, ui, vi: mass i; xj, uj, vj:
// the other end).  Evaluating the same spring from its other end gives the
// exact negative: every operand is negated, so every rounding is the same.
// With YIELD, returns true when the spring breaks in this evaluation.
template <bool ACT, bool DAMP, bool REST, bool YIELD = false>
__device__ __forceinline__ bool spring_force(const float4 &xi, const float4 &ui, const float4 &vi,
                                             const float4 &xj, const float4 &uj, const float4 &vj,
                                             const SpringConst &p, float act, float &fx, float &fy, float &fz)
{
#pragma clang fp contract(off)
    const float Rx = xj.x - xi.x, Ry = xj.y - xi.y, Rz = xj.z - xi.z;
    const float ax = uj.x - ui.x, ay = uj.y - ui.y, az = uj.z - ui.z;
    const float dx = Rx + ax, dy = Ry + ay, dz = Rz + az;
    const float l2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    // Coincident ends (also the padding slots, which point a mass at itself)
    // have no direction and exert no force: select zeros, no branch, so the
    // loads of the next incidences need not wait for this test.
    const bool ok = l2 > 0.f;
    const float il = ok ? __builtin_amdgcn_rsqf(l2) : 0.f;  // 1/l (1 ulp)
    const float l = l2 * il;
    const float R2 = fmaf(Rx, Rx, fmaf(Ry, Ry, Rz * Rz));
    const float r = R2 > 0.f ? R2 * __builtin_amdgcn_rsqf(R2) : 0.f;  // |R|
    const float Rda = fmaf(Rx, ax, fmaf(Ry, ay, Rz * az));
    const float ada = fmaf(ax, ax, fmaf(ay, ay, az * az));
    const float num = fmaf(2.f, Rda, ada);  // 2 R.du + du.du = l^2 - |R|^2
    float stretch = ok ? num * __builtin_amdgcn_rcpf(l + r) : 0.f;
    if (REST) {
        stretch += p.d0;
        if (ACT)
            stretch = fmaf(-p.L0, act, stretch);
    } else if (ACT) {
        stretch = fmaf(-r, act, stretch);
    }
    const float ux = dx * il, uy = dy * il, uz = dz * il;
    float mag = p.k * stretch;
    // coincident ends (no direction) are not tested; NaN fails the test
    const bool holds = !YIELD || !ok || fabsf(mag) <= p.yield;
    if (DAMP) {
        const float vr = fmaf(vj.x - vi.x, ux, fmaf(vj.y - vi.y, uy, (vj.z - vi.z) * uz));
        mag = fmaf(p.c, vr, mag);
    }
    if (YIELD)
        mag = holds ? mag : 0.f;
    fx = fmaf(mag, ux, fx);
    fy = fmaf(mag, uy, fy);
    fz = fmaf(mag, uz, fz);
    return YIELD && !holds && p.yield >= 0.f;
}

// Mass update.  Returns false if the new state is not finite.
__device__ __forceinline__ bool integrate_mass(const float4 &xi, const float4 &ui, const float4 &vi, float fx,
                                               float fy, float fz, const StepConsts &sc, float4 &uo, float4 &vo)
{
#pragma clang fp contract(off)
    const float im = ui.w;  // inverse mass; 0 = pinned
    if (im == 0.f) {
        uo = ui;
        vo = vi;
        return true;
    }
    float ax = fmaf(fx, im, sc.gx);
    float ay = fmaf(fy, im, sc.gy);
    float az = fmaf(fz, im, sc.gz);
    const float z = xi.z + ui.z;
    const bool contact = sc.ground && z < 0.f;
    float fn = 0.f;
    if (contact) {
        fn = -sc.ground_k * z;
        az = fmaf(fn, im, az);
    }
    float wx = fmaf(sc.dt, ax, vi.x);
    float wy = fmaf(sc.dt, ay, vi.y);
    const float wz = fmaf(sc.dt, az, vi.z);
    if (contact) {
        const float vt = sqrtf(fmaf(wx, wx, wy * wy));
        if (vt > 0.f) {
            const float s = fmaxf(0.f, 1.f - sc.mu * fn * sc.dt * im / vt);
            wx *= s;
            wy *= s;
        }
    }
    uo = make_float4(fmaf(sc.dt, wx, ui.x), fmaf(sc.dt, wy, ui.y), fmaf(sc.dt, wz, ui.z), im);
    vo = make_float4(wx, wy, wz, 0.f);
    return isfinite(uo.x) && isfinite(uo.y) && isfinite(uo.z) && isfinite(wx) && isfinite(wy) && isfinite(wz);
}

// ---- staged integrators (velocity Verlet, RK4; Sec. III-B) ----------------
// They integrate the smooth forces -- springs with their dampers, gravity and
// the ground's normal force at the evaluated position -- and apply Coulomb
// friction once per step afterwards, as the Euler step does: normal force
// from the step's starting height, tangential velocity scaled by
// max(0, 1 - mu F_n dt / (m |v_t|)), the position moved by the velocity
// change times dt.  Pinned masses keep position and velocity.

// a = f / m + g (+ -k_g z / m while z < 0); 0 for a pinned mass.
__device__ __forceinline__ float3 smooth_accel(const float4 &xi, const float4 &ui, float fx, float fy, float fz,
                                               const StepConsts &sc)
{
#pragma clang fp contract(off)
    const float im = ui.w;
    if (im == 0.f)
        return make_float3(0.f, 0.f, 0.f);
    float az = fmaf(fz, im, sc.gz);
    const float z = xi.z + ui.z;
    if (sc.ground && z < 0.f)
        az = fmaf(-sc.ground_k * z, im, az);
    return make_float3(fmaf(fx, im, sc.gx), fmaf(fy, im, sc.gy), az);
}

// Friction after a smooth update of (u, v); zb: the step's starting height.
__device__ __forceinline__ void friction_after(float zb, float im, const StepConsts &sc, float4 &u, float4 &v)
{
#pragma clang fp contract(off)
    if (im == 0.f || !(sc.ground && zb < 0.f))
        return;
    const float fn = -sc.ground_k * zb;
    const float vt = sqrtf(fmaf(v.x, v.x, v.y * v.y));
    if (!(vt > 0.f))
        return;
    const float s = fmaxf(0.f, 1.f - sc.mu * fn * sc.dt * im / vt);
    const float wx = v.x * s, wy = v.y * s;
    u.x = fmaf(wx - v.x, sc.dt, u.x);
    u.y = fmaf(wy - v.y, sc.dt, u.y);
    v.x = wx;
    v.y = wy;
}

// Verlet drift of one mass: v' = v + a dt/2, x' = x + v' dt (pinned: kept).
__device__ __forceinline__ void verlet_drift(const float4 &u, const float4 &v, const float4 &a, float dt, float4 &uo,
                                             float4 &vo)
{
#pragma clang fp contract(off)
    if (u.w == 0.f) {
        uo = u;
        vo = v;
        return;
    }
    const float half = 0.5f * dt;
    const float4 vh = make_float4(fmaf(half, a.x, v.x), fmaf(half, a.y, v.y), fmaf(half, a.z, v.z), 0.f);
    uo = make_float4(fmaf(dt, vh.x, u.x), fmaf(dt, vh.y, u.y), fmaf(dt, vh.z, u.z), u.w);
    vo = vh;
}

__device__ __forceinline__ bool finite4(const float4 &u, const float4 &v)
{
    return isfinite(u.x) && isfinite(u.y) && isfinite(u.z) && isfinite(v.x) && isfinite(v.y) && isfinite(v.z);
}

// Pieces of the stage updates, shared by every engine so that all of them
// give identical bits.

// RK4 running sums of w_s v_s and w_s a_s, w = 1, 2, 2, 1 (times dt / 6):
// stage 1 starts them.
__device__ __forceinline__ void rk_sums(int stage, const float4 &vi, const float3 &a, float4 &su, float4 &sv)
{
#pragma clang fp contract(off)
    if (stage == kStageRk1) {
        su = make_float4(vi.x, vi.y, vi.z, 0.f);
        sv = make_float4(a.x, a.y, a.z, 0.f);
        return;
    }
    const float w = stage == kStageRk4 ? 1.f : 2.f;
    su = make_float4(fmaf(w, vi.x, su.x), fmaf(w, vi.y, su.y), fmaf(w, vi.z, su.z), 0.f);
    sv = make_float4(fmaf(w, a.x, sv.x), fmaf(w, a.y, sv.y), fmaf(w, a.z, sv.z), 0.f);
}

// The state RK4 stage `stage` (1-3) hands to the next: base + c dt (v_s, a_s),
// c = 1/2, 1/2, 1.
__device__ __forceinline__ void rk_next(int stage, const float4 &ub, const float4 &vb, const float4 &vi,
                                        const float3 &a, float dt, float4 &uo, float4 &vo)
{
#pragma clang fp contract(off)
    const float c = stage == kStageRk1 + 2 ? dt : 0.5f * dt;
    uo = make_float4(fmaf(c, vi.x, ub.x), fmaf(c, vi.y, ub.y), fmaf(c, vi.z, ub.z), ub.w);
    vo = make_float4(fmaf(c, a.x, vb.x), fmaf(c, a.y, vb.y), fmaf(c, a.z, vb.z), 0.f);
}

// RK4's new state from the base state and the complete sums, then friction
// (zb: the step's starting height).
__device__ __forceinline__ void rk_final(const float4 &ub, const float4 &vb, const float4 &su, const float4 &sv,
                                         float zb, const StepConsts &sc, float4 &u, float4 &v)
{
#pragma clang fp contract(off)
    const float h6 = sc.dt / 6.f;
    u = make_float4(fmaf(h6, su.x, ub.x), fmaf(h6, su.y, ub.y), fmaf(h6, su.z, ub.z), ub.w);
    v = make_float4(fmaf(h6, sv.x, vb.x), fmaf(h6, sv.y, vb.y), fmaf(h6, sv.z, vb.z), 0.f);
    friction_after(zb, ub.w, sc, u, v);
}

// Verlet's kick of a drifted mass (ui, vi) = (x', v') with its new
// acceleration a, then friction (zb: the step's starting height).
__device__ __forceinline__ void verlet_kick(const float4 &ui, const float4 &vi, const float3 &a, float zb,
                                            const StepConsts &sc, float4 &u, float4 &v)
{
#pragma clang fp contract(off)
    const float half = 0.5f * sc.dt;
    u = ui;
    v = vi;
    if (ui.w != 0.f) {
        v = make_float4(fmaf(half, a.x, vi.x), fmaf(half, a.y, vi.y), fmaf(half, a.z, vi.z), 0.f);
        friction_after(zb, ui.w, sc, u, v);
    }
}

// The epilogue of one stage for mass i on the per-step engines: (xi, ui, vi)
// is the stage state the force (fx, fy, fz) was evaluated at.  Returns false
// if a new state is not finite.
__device__ __forceinline__ bool stage_update(int64_t i, const float4 &xi, const float4 &ui, const float4 &vi,
                                             float fx, float fy, float fz, const StateIO &io, const StepConsts &sc)
{
    const float3 a = smooth_accel(xi, ui, fx, fy, fz, sc);
    if (sc.stage == kStageVerletInit) {
        io.A[i] = make_float4(a.x, a.y, a.z, 0.f);
        return true;
    }
    if (sc.stage == kStageVerletKick) {
        // (ui, vi) = (x', v'), drifted from the step's starting state U_base
        float4 u, v;
        verlet_kick(ui, vi, a, xi.z + io.U_base[i].z, sc, u, v);
        io.U_out[i] = u;
        io.V_out[i] = v;
        io.A[i] = make_float4(a.x, a.y, a.z, 0.f);
        return finite4(u, v);
    }
    const float4 ub = io.U_base[i], vb = io.V_base[i];
    if (ui.w == 0.f) {  // pinned
        io.U_out[i] = ub;
        io.V_out[i] = vb;
        return true;
    }
    float4 su = make_float4(0.f, 0.f, 0.f, 0.f), sv = su;
    if (sc.stage != kStageRk1) {
        su = io.sum_u[i];
        sv = io.sum_v[i];
    }
    rk_sums(sc.stage, vi, a, su, sv);
    if (sc.stage != kStageRk4) {
        io.sum_u[i] = su;
        io.sum_v[i] = sv;
        float4 uo, vo;
        rk_next(sc.stage, ub, vb, vi, a, sc.dt, uo, vo);
        io.U_out[i] = uo;
        io.V_out[i] = vo;
        return true;
    }
    float4 u, v;
    rk_final(ub, vb, su, sv, xi.z + ub.z, sc, u, v);
    io.U_out[i] = u;
    io.V_out[i] = v;
    return finite4(u, v);
}

// Spring constants are read once per step: optionally as non-temporal loads
// so they do not displace the state arrays from the caches.
template <class T>
__device__ __forceinline__ T stream_load(const T *p)
{
#if TITAN_NT_LOADS
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

template <bool NT, class T>
__device__ __forceinline__ T const_load(const T *p)
{
    if (NT)
        return stream_load(p);
    return *p;
}

// NT: the constants are streamed once per launch (gather engines); the
// batched engine reads them every step of a launch and keeps them cached.
template <bool ACT, bool DAMPV, bool REST, bool NT, bool WAVE = false, bool YIELD = false>
__device__ __forceinline__ SpringConst load_const(const GatherGraph &g, int64_t e)
{
    SpringConst p;
    p.k = g.k ? const_load<NT>(g.k + e) : g.k_uniform;
    p.c = DAMPV ? const_load<NT>(g.c + e) : g.c_uniform;
    p.act_c = ACT ? const_load<NT>(g.act_c + e) : 0.f;
    p.act_s = (ACT && !WAVE) ? const_load<NT>(g.act_s + e) : 0.f;
    p.d0 = REST ? const_load<NT>(g.d0 + e) : 0.f;
    p.L0 = REST ? const_load<NT>(g.rest + e) : 0.f;
    p.t_off = (WAVE && !g.wave_cls) ? const_load<NT>(g.t_off + e) : 0.0;
    p.cls = (WAVE && g.wave_cls) ? (int)g.wave_cls[e] : 0;
    p.yield = YIELD ? const_load<NT>(g.yield + e) : 0.f;
    return p;
}

// Sum the spring forces on one mass over its incidence slots
// [base + w*64 for w < width).  Slots past the mass's own degree are padding
// that points the mass at itself and contributes nothing.  Loads of kUnroll
// slots (neighbour index and spring constants) are issued together before
// any of them is used, so each wave keeps several requests in flight.
// Nbr(e) loads the neighbour reference of slot e; State(ref, xj, uj, vj)
// fetches that neighbour's state.  YIELD: 0 unbreakable springs; 1 apply the
// yield test (a force query); 2 apply it and record breaks in the slot.
constexpr int kUnroll = TITAN_UNROLL;
constexpr int kUnrollPlain = TITAN_UNROLL_PLAIN;

template <bool ACT, bool DAMP, bool DAMPV, bool REST, bool NT, bool WAVE, int YIELD = 0, int UNROLL = kUnroll,
          class Nbr, class State>
__device__ __forceinline__ void sum_forces(const GatherGraph &g, int64_t base, int width, const float4 &xi,
                                           const float4 &ui, const float4 &vi, const Clock &ck,
                                           const StepConsts &sc, Nbr nbr, State state, float &fx, float &fy,
                                           float &fz)
{
    int w = 0;
    for (; w + UNROLL <= width; w += UNROLL) {
        int ref[UNROLL];
        SpringConst p[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t e = base + (int64_t)(w + u) * kSlice;
            ref[u] = nbr(e);
            p[u] = load_const<ACT, DAMPV, REST, NT, WAVE, YIELD != 0>(g, e);
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            float4 xj, uj, vj;
            state(ref[u], xj, uj, vj);
            const bool broke = spring_force<ACT, DAMP, REST, YIELD != 0>(
                xi, ui, vi, xj, uj, vj, p[u], act_factor<ACT, WAVE>(p[u], ck, sc), fx, fy, fz);
            if (YIELD == 2 && broke)
                g.yield[base + (int64_t)(w + u) * kSlice] = -1.f;
        }
    }
    for (; w < width; ++w) {
        const int64_t e = base + (int64_t)w * kSlice;
        const int ref = nbr(e);
        const SpringConst p = load_const<ACT, DAMPV, REST, NT, WAVE, YIELD != 0>(g, e);
        float4 xj, uj, vj;
        state(ref, xj, uj, vj);
        const bool broke = spring_force<ACT, DAMP, REST, YIELD != 0>(xi, ui, vi, xj, uj, vj, p,
                                                                     act_factor<ACT, WAVE>(p, ck, sc), fx, fy, fz);
        if (YIELD == 2 && broke)
            g.yield[e] = -1.f;
    }
}

__device__ __forceinline__ int slice_width(const GatherGraph &g, int64_t i)
{
    return (int)((g.slice_off[(i >> 6) + 1] - g.slice_off[i >> 6]) >> 6);
}

// Workgroup -> tile mapping that gives each XCD a contiguous range of tiles:
// consecutive workgroups are dispatched round-robin over the 8 XCDs, so
// workgroup b runs on XCD b % 8; tile ranges that are contiguous per XCD keep
// neighbouring tiles (and their shared halo data) in the same XCD's L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nblocks)
{
    constexpr unsigned kXcd = 8;
    const unsigned xcd = b % kXcd, k = b / kXcd;
    const unsigned q = nblocks / kXcd, r = nblocks % kXcd;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

}  // namespace titan

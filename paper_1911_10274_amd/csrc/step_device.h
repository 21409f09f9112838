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
};

// Force on mass i from one incident spring (xi, ui, vi: mass i; xj, uj, vj:
// the other end).  Evaluating the same spring from its other end gives the
// exact negative: every operand is negated, so every rounding is the same.
template <bool ACT, bool DAMP, bool REST>
__device__ __forceinline__ void spring_force(const float4 &xi, const float4 &ui, const float4 &vi,
                                             const float4 &xj, const float4 &uj, const float4 &vj,
                                             const SpringConst &p, float sin_wt, float cos_wt,
                                             float &fx, float &fy, float &fz)
{
    const float Rx = xj.x - xi.x, Ry = xj.y - xi.y, Rz = xj.z - xi.z;
    const float ax = uj.x - ui.x, ay = uj.y - ui.y, az = uj.z - ui.z;
    const float dx = Rx + ax, dy = Ry + ay, dz = Rz + az;
    const float l2 = dx * dx + dy * dy + dz * dz;
    // Coincident ends (also the padding slots, which point a mass at itself)
    // have no direction and exert no force: select zeros, no branch, so the
    // loads of the next incidences need not wait for this test.
    const bool ok = l2 > 0.f;
    const float il = ok ? __builtin_amdgcn_rsqf(l2) : 0.f;  // 1/l (1 ulp)
    const float l = l2 * il;
    const float R2 = Rx * Rx + Ry * Ry + Rz * Rz;
    const float r = R2 > 0.f ? R2 * __builtin_amdgcn_rsqf(R2) : 0.f;  // |R|
    const float num = 2.f * (Rx * ax + Ry * ay + Rz * az) + (ax * ax + ay * ay + az * az);
    float stretch = ok ? num * __builtin_amdgcn_rcpf(l + r) : 0.f;
    if (REST) {
        stretch += p.d0;
        if (ACT)
            stretch -= p.L0 * (p.act_c * sin_wt + p.act_s * cos_wt);
    } else if (ACT) {
        stretch -= r * (p.act_c * sin_wt + p.act_s * cos_wt);
    }
    const float ux = dx * il, uy = dy * il, uz = dz * il;
    float mag = p.k * stretch;
    if (DAMP) {
        const float vr = (vj.x - vi.x) * ux + (vj.y - vi.y) * uy + (vj.z - vi.z) * uz;
        mag += p.c * vr;
    }
    fx += mag * ux;
    fy += mag * uy;
    fz += mag * uz;
}

// Mass update.  Returns false if the new state is not finite.
__device__ __forceinline__ bool integrate_mass(const float4 &xi, const float4 &ui, const float4 &vi, float fx,
                                               float fy, float fz, const StepConsts &sc, float4 &uo, float4 &vo)
{
    const float im = ui.w;  // inverse mass; 0 = pinned
    if (im == 0.f) {
        uo = ui;
        vo = vi;
        return true;
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
    uo = make_float4(ui.x + sc.dt * wx, ui.y + sc.dt * wy, ui.z + sc.dt * wz, im);
    vo = make_float4(wx, wy, wz, 0.f);
    return isfinite(uo.x) && isfinite(uo.y) && isfinite(uo.z) && isfinite(wx) && isfinite(wy) && isfinite(wz);
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

// Adjoint (reverse-mode, backward in time) of a rollout on the batched
// layout: one workgroup per group of whole bodies, state in LDS.
//
// Loss: J = sum_b w_b * J_b, J_b = -(CoM_x(x_N) - CoM_x(x_0)) of body b; its
// gradient with respect to x_N is the per-mass seed -w_b m_i / M_b (x).
// Gradients: per spring, dJ/dk and dJ/d(C, S) of the actuation phasor
// (rest length L0 (1 + C sin(omega t) + S cos(omega t))).
//
// One launch per call:
//   1. forward nsteps steps, storing the state every K steps (checkpoints);
//   2. for each segment, newest first: reload its checkpoint, recompute its K
//      states into a segment buffer, then run K reverse steps.
// A reverse step undoes, in reverse order, what a forward step did
// (Sec. III-B's two passes):
//   mass pass:   x' = x + dt v',  v' = friction(w),  w = v + dt F / m
//                -> force adjoint mu_i = dt/m * dJ/dw_i (kept in LDS)
//   spring pass: every spring's force depends on both ends' x and v and on
//                (k, C, S): gather, per mass, the contributions of its springs
//                from mu_i - mu_j; the spring's owner (lower internal index
//                end) adds the parameter gradients.  No atomics.
// Forward steps sum each mass's slots in their fixed order, as every engine
// does (same states, bit for bit).  In the reverse steps, with the host's
// spring tables (groups of at most 1024 masses), each spring's adjoint terms
// and parameter gradients are evaluated once per step, by one thread, into
// LDS records that both ends then add (the other end negated: the value it
// would compute itself, bit for bit), in ascending spring order and in
// chunks when a group's records exceed LDS.  Otherwise every slot evaluates
// its spring's terms itself.
#include "step_device.h"

namespace titan {

namespace {

// dJ/d(spring inputs) for one incidence of mass i: the terms that move the
// adjoints of mass i -- lx_i -= gd, lv_i -= bu -- and the parameter-gradient
// contributions (k, C, S).  Seen from the spring's other end every operand
// is negated, so that end receives exactly -gd and -bu (lx_j += gd,
// lv_j += bu) and the same parameter terms.
template <bool ACT, bool DAMP, bool REST>
__device__ __forceinline__ void spring_adjoint_terms(const float4 &xi, const float4 &ui, const float4 &vi,
                                                     const float4 &xj, const float4 &uj, const float4 &vj,
                                                     const SpringConst &p, float sin_wt, float cos_wt,
                                                     const float4 &mi, const float4 &mj, float3 &gd, float3 &bu,
                                                     float &gk, float &gC, float &gS)
{
#pragma clang fp contract(off)
    const float Rx = xj.x - xi.x, Ry = xj.y - xi.y, Rz = xj.z - xi.z;
    const float ax = uj.x - ui.x, ay = uj.y - ui.y, az = uj.z - ui.z;
    const float dx = Rx + ax, dy = Ry + ay, dz = Rz + az;
    const float l2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    gd = bu = make_float3(0.f, 0.f, 0.f);
    gk = gC = gS = 0.f;
    if (!(l2 > 0.f))
        return;  // no force, no gradient (also the padding slots)
    const float il = __builtin_amdgcn_rsqf(l2);
    const float l = l2 * il;
    const float R2 = fmaf(Rx, Rx, fmaf(Ry, Ry, Rz * Rz));
    const float r = R2 > 0.f ? R2 * __builtin_amdgcn_rsqf(R2) : 0.f;
    const float Rda = fmaf(Rx, ax, fmaf(Ry, ay, Rz * az));
    const float ada = fmaf(ax, ax, fmaf(ay, ay, az * az));
    float e = fmaf(2.f, Rda, ada) * __builtin_amdgcn_rcpf(l + r);
    const float L0 = REST ? p.L0 : r;
    if (REST)
        e += p.d0;
    if (ACT)
        e = fmaf(-L0, fmaf(p.act_c, sin_wt, p.act_s * cos_wt), e);
    const float ux = dx * il, uy = dy * il, uz = dz * il;
    const float dvx = vj.x - vi.x, dvy = vj.y - vi.y, dvz = vj.z - vi.z;
    const float vr = DAMP ? fmaf(dvx, ux, fmaf(dvy, uy, dvz * uz)) : 0.f;
    const float mag = DAMP ? fmaf(p.c, vr, p.k * e) : p.k * e;
    // dm = mu_i - mu_j, pu = dm . u
    const float mx = mi.x - mj.x, my = mi.y - mj.y, mz = mi.z - mj.z;
    const float pu = fmaf(mx, ux, fmaf(my, uy, mz * uz));
    // g_d = pu k u + pu (c / l)(dv - u vr) + (mag / l)(dm - u pu): the gradient
    // with respect to d = x_j - x_i; mass i receives -g_d.
    const float a1 = pu * p.k;
    const float a2 = DAMP ? pu * p.c * il : 0.f;
    const float a3 = mag * il;
    gd.x = fmaf(a1, ux, fmaf(a2, fmaf(-ux, vr, dvx), a3 * fmaf(-ux, pu, mx)));
    gd.y = fmaf(a1, uy, fmaf(a2, fmaf(-uy, vr, dvy), a3 * fmaf(-uy, pu, my)));
    gd.z = fmaf(a1, uz, fmaf(a2, fmaf(-uz, vr, dvz), a3 * fmaf(-uz, pu, mz)));
    if (DAMP) {
        // the damper's pull on v_i: (pu c) u
        const float b = pu * p.c;
        bu = make_float3(b * ux, b * uy, b * uz);
    }
    gk = pu * e;
    if (ACT) {
        gC = -(a1 * L0 * sin_wt);
        gS = -(a1 * L0 * cos_wt);
    }
}

// The same terms applied to mass i's adjoints (lx, lv) at once.
template <bool ACT, bool DAMP, bool REST>
__device__ __forceinline__ void spring_adjoint(const float4 &xi, const float4 &ui, const float4 &vi,
                                               const float4 &xj, const float4 &uj, const float4 &vj,
                                               const SpringConst &p, float sin_wt, float cos_wt,
                                               const float4 &mi, const float4 &mj, float3 &lx, float3 &lv,
                                               float &gk, float &gC, float &gS)
{
#pragma clang fp contract(off)
    float3 gd, bu;
    spring_adjoint_terms<ACT, DAMP, REST>(xi, ui, vi, xj, uj, vj, p, sin_wt, cos_wt, mi, mj, gd, bu, gk, gC, gS);
    lx.x -= gd.x;
    lx.y -= gd.y;
    lx.z -= gd.z;
    if (DAMP) {
        lv.x -= bu.x;
        lv.y -= bu.y;
        lv.z -= bu.z;
    }
}

// Mass pass of a reverse step for one mass: given the summed spring force f
// at the step's starting state and the adjoints (lx, lv) of the state after
// the step, returns the force adjoint mu = dt/m dJ/dw and updates (lx, lv) to
// the adjoints of the starting state (minus the spring terms, added later).
__device__ __forceinline__ float4 mass_adjoint(const float4 &xi, const float4 &ui, const float4 &vi, float fx,
                                               float fy, float fz, const StepConsts &sc, float3 &lx, float3 &lv)
{
#pragma clang fp contract(off)
    const float im = ui.w;
    if (im == 0.f)
        return make_float4(0.f, 0.f, 0.f, 0.f);  // pinned: nothing depends on its force
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
    const float wx = fmaf(sc.dt, ax, vi.x);
    const float wy = fmaf(sc.dt, ay, vi.y);
    // v' moves x' too: adjoint of v' is lv + dt lx
    const float tx = fmaf(sc.dt, lx.x, lv.x), ty = fmaf(sc.dt, lx.y, lv.y), tz = fmaf(sc.dt, lx.z, lv.z);
    float wlx = tx, wly = ty;
    float dzf = 0.f;
    if (contact) {
        const float vt = sqrtf(fmaf(wx, wx, wy * wy));
        if (vt > 0.f) {
            const float beta = sc.mu * fn * sc.dt * im;
            const float s = 1.f - beta / vt;
            if (s > 0.f) {
                const float hx = wx / vt, hy = wy / vt;
                const float wl = fmaf(hx, tx, hy * ty);
                const float bv = beta / vt;
                wlx = fmaf(s, tx, bv * hx * wl);
                wly = fmaf(s, ty, bv * hy * wl);
                dzf = wl * sc.mu * sc.dt * sc.ground_k * im;
            } else {
                wlx = 0.f;
                wly = 0.f;
            }
        }
    }
    const float4 mu = make_float4(sc.dt * im * wlx, sc.dt * im * wly, sc.dt * im * tz, 0.f);
    lv = make_float3(wlx, wly, tz);
    lx.z += dzf;
    if (contact)
        lx.z = fmaf(-sc.ground_k, mu.z, lx.z);
    return mu;
}

// Springs-once loops: springs per thread whose loads are issued together,
// and entries per batch of a mass's sum (tuning builds may set them; on the
// 256-robot gradient 1, 2 and 3 springs measured within 1% of each other and
// 1.5-2% faster than 4, 8 springs 17% slower; 4 and 16 entries 1-3% slower
// than 8).
#ifndef TITAN_ADJ_ONCE_BATCH
#define TITAN_ADJ_ONCE_BATCH 2
#endif
#ifndef TITAN_ADJ_SLOT_BATCH
#define TITAN_ADJ_SLOT_BATCH 8
#endif
constexpr int kOnceBatch = TITAN_ADJ_ONCE_BATCH;
constexpr int kSlotBatch = TITAN_ADJ_SLOT_BATCH;

// ONCE: the reverse steps evaluate every spring once (AdjointIO's spring
// tables), else from both ends, slot by slot.
template <bool ACT, bool DAMP, bool DAMPV, bool REST, int T, int MAXM, bool ONCE>
__global__ __launch_bounds__(T) void adjoint_kernel(GatherGraph g, BatchLayout b, AdjointIO a, StepConsts sc)
{
    extern __shared__ float4 smem[];
    const int cap = b.max_group;
    float4 *sX = smem;
    float4 *sU = smem + cap;
    float4 *sV = smem + 2 * cap;
    float4 *sM = smem + 3 * cap;
    // springs evaluated once: the reverse records (gd, bu.x) and (bu.y, bu.z)
    // of a chunk of springs
    float4 *sF = smem + 4 * cap;
    float2 *sF2 = reinterpret_cast<float2 *>(sF + a.rev_chunk);
    const int64_t n = g.n;
    const int64_t m0 = b.mass_off[blockIdx.x];
    const int nm = (int)(b.mass_off[blockIdx.x + 1] - m0);
    const int tid = threadIdx.x;
    const int K = a.K;
    constexpr bool once = ONCE;
    const int64_t sp0 = once ? a.sp_off[blockIdx.x] : 0;
    const int nsp = once ? (int)(a.sp_off[blockIdx.x + 1] - sp0) : 0;

    auto nbr = [&](int64_t e) { return (int)b.nbr_group[e]; };
    // a group spring's constants, the same values load_const reads from its slots
    auto pconst = [&](int64_t t) {
        SpringConst p{};
        const float4 q = a.sp_kcs[t];
        p.k = q.x;
        p.c = q.y;
        p.act_c = q.z;
        p.act_s = q.w;
        if (REST) {
            const float2 r = a.sp_rest[t];
            p.d0 = r.x;
            p.L0 = r.y;
        }
        return p;
    };
    auto state = [&](int r, float4 &xj, float4 &uj, float4 &vj) {
        uj = sU[r];
        xj = sX[r];
        vj = DAMP ? sV[r] : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    // one forward step of the group in LDS (same arithmetic as every engine);
    // with fout, the summed spring forces are kept too
    auto forward = [&](int s, float4 *fout) {
        const float2 tr = ACT ? a.trig[s] : make_float2(0.f, 1.f);
        float4 nu[MAXM], nv[MAXM];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < MAXM; ++k) {
            const int q = tid + k * T;
            if (q < nm) {
                const int64_t i = m0 + q;
                const float4 xi = sX[q], ui = sU[q], vi = sV[q];
                float fx = 0.f, fy = 0.f, fz = 0.f;
                sum_forces<ACT, DAMP, DAMPV, REST, false, false>(g, g.slice_off[i >> 6] + (i & 63),
                                                                 slice_width(g, i), xi, ui, vi,
                                                                 Clock{tr, 0.0}, sc, nbr, state, fx, fy, fz);
                if (fout)
                    fout[q] = make_float4(fx, fy, fz, 0.f);
                ok &= integrate_mass(xi, ui, vi, fx, fy, fz, sc, nu[k], nv[k]);
            }
        }
        if (!ok)
            atomicMin(a.first_bad, (unsigned long long)(sc.step + s));
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
    };

    for (int q = tid; q < nm; q += T) {
        const float4 u = a.U0[m0 + q], v = a.V0[m0 + q];
        sX[q] = g.X0[m0 + q];
        sU[q] = u;
        sV[q] = v;
        a.ckU[m0 + q] = u;
        a.ckV[m0 + q] = v;
    }
    __syncthreads();

    // 1. forward with checkpoints; the last segment's states and forces go
    // straight to the segment buffers (that segment is reversed first and
    // needs no recompute)
    const int nseg = (a.nsteps + K - 1) / K;
    const int last0 = (nseg - 1) * K;
    for (int s = 0; s < a.nsteps; ++s) {
        if (s >= last0) {
            const int r = s - last0;
            for (int q = tid; q < nm; q += T) {
                a.segU[(int64_t)r * n + m0 + q] = sU[q];
                a.segV[(int64_t)r * n + m0 + q] = sV[q];
            }
            forward(s, a.segF + (int64_t)r * n + m0);
        } else {
            forward(s, nullptr);
        }
        if ((s + 1) % K == 0 && (s + 1) / K < nseg)
            for (int q = tid; q < nm; q += T) {
                a.ckU[(int64_t)((s + 1) / K) * n + m0 + q] = sU[q];
                a.ckV[(int64_t)((s + 1) / K) * n + m0 + q] = sV[q];
            }
    }
    for (int q = tid; q < nm; q += T)
        a.dux[m0 + q] = sU[q].x - a.U0[m0 + q].x;

    // 2. reverse, segment by segment
    float3 lx[MAXM], lv[MAXM];
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
        const int q = tid + k * T;
        lx[k] = make_float3(q < nm ? a.seed[m0 + q] : 0.f, 0.f, 0.f);
        lv[k] = make_float3(0.f, 0.f, 0.f);
    }
    for (int c = nseg - 1; c >= 0; --c) {
        const int s0 = c * K;
        const int len = min(K, a.nsteps - s0);
        const bool kept = c == nseg - 1;  // states and forces stored by the forward pass
        if (!kept) {
            __syncthreads();
            for (int q = tid; q < nm; q += T) {
                sU[q] = a.ckU[(int64_t)c * n + m0 + q];
                sV[q] = a.ckV[(int64_t)c * n + m0 + q];
            }
            __syncthreads();
            for (int r = 0; r < len; ++r) {
                for (int q = tid; q < nm; q += T) {
                    a.segU[(int64_t)r * n + m0 + q] = sU[q];
                    a.segV[(int64_t)r * n + m0 + q] = sV[q];
                }
                if (r + 1 < len)
                    forward(s0 + r, a.segF + (int64_t)r * n + m0);
            }
        }
        // the next reverse step's state and force are fetched into
        // registers while the current spring pass runs (each thread reads
        // only what it wrote itself)
        float4 pu[MAXM], pv[MAXM], pf[MAXM];
        auto fetch = [&](int r) {
#pragma unroll
            for (int k = 0; k < MAXM; ++k) {
                const int q = tid + k * T;
                if (q < nm) {
                    const int64_t o = (int64_t)r * n + m0 + q;
                    pu[k] = a.segU[o];
                    pv[k] = a.segV[o];
                    pf[k] = (kept || r + 1 < len) ? a.segF[o] : make_float4(0.f, 0.f, 0.f, 0.f);
                }
            }
        };
        fetch(len - 1);
        for (int r = len - 1; r >= 0; --r) {
            const int s = s0 + r;
            const float2 tr = ACT ? a.trig[s] : make_float2(0.f, 1.f);
            StepConsts scs = sc;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < MAXM; ++k) {
                const int q = tid + k * T;
                if (q < nm) {
                    sU[q] = pu[k];
                    sV[q] = pv[k];
                }
            }
            __syncthreads();
            // mass pass (the forces of every state but a recomputed
            // segment's last were kept)
#pragma unroll
            for (int k = 0; k < MAXM; ++k) {
                const int q = tid + k * T;
                if (q < nm) {
                    const int64_t i = m0 + q;
                    const float4 xi = sX[q], ui = sU[q], vi = sV[q];
                    float fx = pf[k].x, fy = pf[k].y, fz = pf[k].z;
                    if (!(kept || r + 1 < len)) {
                        fx = fy = fz = 0.f;
                        sum_forces<ACT, DAMP, DAMPV, REST, false, false>(g, g.slice_off[i >> 6] + (i & 63),
                                                                         slice_width(g, i), xi, ui, vi,
                                                                         Clock{tr, 0.0}, sc, nbr, state, fx, fy, fz);
                    }
                    sM[q] = mass_adjoint(xi, ui, vi, fx, fy, fz, scs, lx[k], lv[k]);
                }
            }
            __syncthreads();
            if (r > 0)
                fetch(r - 1);
            // spring pass
            if constexpr (ONCE) {
                // every spring once, in chunks of records that fit LDS: the
                // owner end's terms and the parameter gradients, then each
                // mass adds its springs' terms (the other end negated) in
                // ascending spring order, resuming where the last chunk ended
                int cw[MAXM];
#pragma unroll
                for (int k = 0; k < MAXM; ++k)
                    cw[k] = 0;
                for (int c0 = 0; c0 < nsp; c0 += a.rev_chunk) {
                    const int c1 = min(nsp, c0 + a.rev_chunk);
                    if (c0 > 0)
                        __syncthreads();  // the previous chunk's records are read
                    for (int t0 = c0 + tid; t0 < c1; t0 += kOnceBatch * T) {
                        uint32_t rr[kOnceBatch];
                        SpringConst p[kOnceBatch];
                        float4 acc[kOnceBatch];
#pragma unroll
                        for (int u = 0; u < kOnceBatch; ++u) {
                            const int t = min(t0 + u * T, c1 - 1);
                            rr[u] = a.sp_ends[sp0 + t];
                            p[u] = pconst(sp0 + t);
                            acc[u] = a.gsp[sp0 + t];
                        }
#pragma unroll
                        for (int u = 0; u < kOnceBatch; ++u) {
                            const int t = t0 + u * T;
                            if (t < c1) {
                                const int qa = (int)(rr[u] & 0xffffu), qb = (int)(rr[u] >> 16);
                                float3 gd, bu;
                                float gk, gC, gS;
                                spring_adjoint_terms<ACT, DAMP, REST>(
                                    sX[qa], sU[qa], DAMP ? sV[qa] : make_float4(0.f, 0.f, 0.f, 0.f), sX[qb],
                                    sU[qb], DAMP ? sV[qb] : make_float4(0.f, 0.f, 0.f, 0.f), p[u], tr.x, tr.y,
                                    sM[qa], sM[qb], gd, bu, gk, gC, gS);
                                sF[t - c0] = make_float4(gd.x, gd.y, gd.z, bu.x);
                                if (DAMP)
                                    sF2[t - c0] = make_float2(bu.y, bu.z);
                                acc[u].x += gk;
                                acc[u].y += gC;
                                acc[u].z += gS;
                                a.gsp[sp0 + t] = acc[u];
                            }
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < MAXM; ++k) {
                        const int q = tid + k * T;
                        if (q < nm) {
                            const int64_t i = m0 + q;
                            const int64_t base = g.slice_off[i >> 6] + (i & 63);
                            const int width = slice_width(g, i);
                            // entries of kSlotBatch slots loaded at a time;
                            // stop at a later chunk's entry or the list's end
                            int w = cw[k];
                            bool go = w < width;
                            while (go) {
                                int v[kSlotBatch];
#pragma unroll
                                for (int u = 0; u < kSlotBatch; ++u)
                                    v[u] = a.rev_sp[base + (int64_t)min(w + u, width - 1) * kSlice];
#pragma unroll
                                for (int u = 0; u < kSlotBatch; ++u) {
                                    go = go && w < width && (v[u] >> 1) < c1;
                                    if (go) {
                                        const int t = v[u] >> 1;
                                        const unsigned sg = (unsigned)(~v[u]) << 31;  // negate at the owner end
                                        const float4 r0 = sF[t - c0];
                                        lx[k].x += __uint_as_float(__float_as_uint(r0.x) ^ sg);
                                        lx[k].y += __uint_as_float(__float_as_uint(r0.y) ^ sg);
                                        lx[k].z += __uint_as_float(__float_as_uint(r0.z) ^ sg);
                                        if (DAMP) {
                                            const float2 r1 = sF2[t - c0];
                                            lv[k].x += __uint_as_float(__float_as_uint(r0.w) ^ sg);
                                            lv[k].y += __uint_as_float(__float_as_uint(r1.x) ^ sg);
                                            lv[k].z += __uint_as_float(__float_as_uint(r1.y) ^ sg);
                                        }
                                        ++w;
                                    }
                                }
                            }
                            cw[k] = w;
                        }
                    }
                }
                continue;
            }
#pragma unroll
            for (int k = 0; k < MAXM; ++k) {
                const int q = tid + k * T;
                if (q < nm) {
                    const int64_t i = m0 + q;
                    const float4 xi = sX[q], ui = sU[q], vi = sV[q], mi = sM[q];
                    const int64_t base = g.slice_off[i >> 6] + (i & 63);
                    const int width = slice_width(g, i);
                    // one slot: its adjoint terms, and at the spring's owner
                    // slot (lower internal index end) the parameter gradients
                    auto slot = [&](int64_t e, int jr, const SpringConst &p, float4 acc) {
                        float gk, gC, gS;
                        spring_adjoint<ACT, DAMP, REST>(xi, ui, vi, sX[jr], sU[jr],
                                                        DAMP ? sV[jr] : make_float4(0.f, 0.f, 0.f, 0.f), p, tr.x,
                                                        tr.y, mi, sM[jr], lx[k], lv[k], gk, gC, gS);
                        if (jr > q) {
                            acc.x += gk;
                            acc.y += gC;
                            acc.z += gS;
                            a.gslot[e] = acc;
                        }
                    };
                    // as in the force sum, the global loads of kUnroll slots
                    // (neighbour, constants, then the owners' running
                    // gradients) are issued before any of them is used
                    int w = 0;
                    for (; w + kUnroll <= width; w += kUnroll) {
                        int ref[kUnroll];
                        SpringConst p[kUnroll];
                        float4 acc[kUnroll];
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u) {
                            const int64_t e = base + (int64_t)(w + u) * kSlice;
                            ref[u] = nbr(e);
                            p[u] = load_const<ACT, DAMPV, REST, false>(g, e);
                        }
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
                            acc[u] = ref[u] > q ? a.gslot[base + (int64_t)(w + u) * kSlice]
                                                : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
                            slot(base + (int64_t)(w + u) * kSlice, ref[u], p[u], acc[u]);
                    }
                    for (; w < width; ++w) {
                        const int64_t e = base + (int64_t)w * kSlice;
                        const int jr = nbr(e);
                        slot(e, jr, load_const<ACT, DAMPV, REST, false>(g, e),
                             jr > q ? a.gslot[e] : make_float4(0.f, 0.f, 0.f, 0.f));
                    }
                }
            }
        }
    }
}

template <bool ACT, bool DAMP, bool DAMPV, bool REST, int T, int MAXM, bool ONCE>
hipError_t launch_tm(const GatherGraph &g, const BatchLayout &b, const AdjointIO &a, const StepConsts &sc,
                     hipStream_t st)
{
    auto kern = adjoint_kernel<ACT, DAMP, DAMPV, REST, T, MAXM, ONCE>;
    const size_t lds = (size_t)b.max_group * 4 * sizeof(float4) + (ONCE ? (size_t)a.once_bytes : 0);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)b.n_groups), dim3(T), lds, st, g, b, a, sc);
    return hipGetLastError();
}

// One mass per thread while a group fits 1024 threads: the reverse step is
// a chain of LDS reads and workgroup barriers, so the more waves a CU holds
// the more of that latency is hidden (1024 threads allow 128 VGPRs; the
// actuated, damped kernels take 116-120 at one mass per thread).  Groups up
// to 2048 masses take two masses per thread (125 VGPRs) and the per-slot
// reverse steps.
template <bool ACT, bool DAMP, bool DAMPV, bool REST>
hipError_t launch4(const GatherGraph &g, const BatchLayout &b, const AdjointIO &a, const StepConsts &sc,
                   hipStream_t st)
{
    const int m = b.max_group;
    const bool once = a.sp_ends != nullptr;
    if (m <= 256)
        return once ? launch_tm<ACT, DAMP, DAMPV, REST, 256, 1, true>(g, b, a, sc, st)
                    : launch_tm<ACT, DAMP, DAMPV, REST, 256, 1, false>(g, b, a, sc, st);
    if (m <= 512)
        return once ? launch_tm<ACT, DAMP, DAMPV, REST, 512, 1, true>(g, b, a, sc, st)
                    : launch_tm<ACT, DAMP, DAMPV, REST, 512, 1, false>(g, b, a, sc, st);
    if (m <= 1024)
        return once ? launch_tm<ACT, DAMP, DAMPV, REST, 1024, 1, true>(g, b, a, sc, st)
                    : launch_tm<ACT, DAMP, DAMPV, REST, 1024, 1, false>(g, b, a, sc, st);
    // springs once needs groups of at most 1024 masses
    if (m <= 2048 && !once)
        return launch_tm<ACT, DAMP, DAMPV, REST, 1024, 2, false>(g, b, a, sc, st);
    return hipErrorInvalidValue;
}

// The spring-once tables' constants, one group per workgroup, as load_const
// reads them from each spring's owner slot.
__global__ void pack_spring_consts(GatherGraph g, const int64_t *sp_slot, const int64_t *sp_off, float4 *kcs,
                                   float2 *rest)
{
    for (int64_t t = sp_off[blockIdx.x] + threadIdx.x; t < sp_off[blockIdx.x + 1]; t += blockDim.x) {
        const int64_t e = sp_slot[t];
        kcs[t] = make_float4(g.k ? g.k[e] : g.k_uniform, g.c ? g.c[e] : g.c_uniform, g.act_c ? g.act_c[e] : 0.f,
                             g.act_c ? g.act_s[e] : 0.f);
        if (rest)
            rest[t] = make_float2(g.d0[e], g.rest[e]);
    }
}

__global__ void gather_spring_grads(const float4 *gslot, const int64_t *owner_slot, int64_t ns, float *gk, float *gC,
                                    float *gS)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns)
        return;
    // a removed spring has no slot and no gradient
    const int64_t e = owner_slot[s];
    const float4 v = e >= 0 ? gslot[e] : make_float4(0.f, 0.f, 0.f, 0.f);
    gk[s] = v.x;
    gC[s] = v.y;
    gS[s] = v.z;
}

// Per-voxel actuation gradients (Sec. IV-C drives bodies by per-voxel
// parameters; the adjoint itself is not in the paper).  A voxel-driven
// spring's phasor is the mean of its voxels' a (cos phi, sin phi), so
// dJ/da_v = sum_s (gC_s cos phi_v + gS_s sin phi_v) / n_s and
// dJ/dphi_v = a_v sum_s (gS_s cos phi_v - gC_s sin phi_v) / n_s over the
// springs s of voxel v (n_s: the spring's voxel count).  One thread per voxel,
// its springs in ascending order: deterministic, no atomics.
// vw[v] = (cos phi_v, sin phi_v, a_v, 0); inv_cnt[s] = 1 / n_s.
__global__ void voxel_grads_kernel(int64_t nv, const int64_t *vs_ptr, const int32_t *vs_spring, const float *inv_cnt,
                                   const float4 *vw, const float *gC, const float *gS, float *ga, float *gphi)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv)
        return;
    const float4 w = vw[v];
    float sa = 0.f, sp = 0.f;
    for (int64_t e = vs_ptr[v]; e < vs_ptr[v + 1]; ++e) {
        const int32_t q = vs_spring[e];
        const float r = inv_cnt[q];
        const float c = gC[q] * r, sn = gS[q] * r;
        sa += c * w.x + sn * w.y;
        sp += sn * w.x - c * w.y;
    }
    ga[v] = sa;
    gphi[v] = w.z * sp;
}

// J_b = -sum_{i in b} (m_i / M_b) * dux_i: one wave per body, masses of a
// body contiguous; lane l sums the body's masses l, l + 64, ... in index
// order, then a butterfly of exchanges adds the 64 partial sums (the same
// pairs in the same order on every run: deterministic, no atomics).
__global__ __launch_bounds__(256) void body_loss(const float *dux, const float *coef, const int64_t *body_off,
                                                 int64_t nb, float *loss)
{
    const int64_t bdy = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (bdy >= nb)
        return;  // the whole wave: one body per wave
    float acc = 0.f;
    for (int64_t i = body_off[bdy] + lane; i < body_off[bdy + 1]; i += 64)
        acc = fmaf(coef[i], dux[i], acc);
    for (int o = 32; o > 0; o >>= 1)
        acc += __shfl_xor(acc, o);
    if (lane == 0)
        loss[bdy] = -acc;
}

}  // namespace

hipError_t launch_adjoint(const GatherGraph &g, const BatchLayout &b, const AdjointIO &a, const StepConsts &sc,
                          hipStream_t stream)
{
    if (b.n_groups == 0 || a.nsteps <= 0)
        return hipSuccess;
    const bool act = g.act_c != nullptr, dampv = g.c != nullptr, rest = g.d0 != nullptr;
    // every buffer the chosen path reads or writes must be there
    if (!a.U0 || !a.V0 || !a.ckU || !a.ckV || !a.segU || !a.segV || !a.segF || !a.seed || !a.dux || !a.trig ||
        !a.first_bad || a.K < 1)
        return hipErrorInvalidValue;
    if (a.sp_ends ? (!a.sp_kcs || !a.sp_off || !a.rev_sp || !a.gsp || (rest && !a.sp_rest) || a.rev_chunk < 1 ||
                     a.once_bytes < 24 * a.rev_chunk)
                  : !a.gslot)
        return hipErrorInvalidValue;
    const bool damp = dampv || g.c_uniform != 0.f;
    const int key = (act ? 8 : 0) | (damp ? 4 : 0) | (dampv ? 2 : 0) | (rest ? 1 : 0);
    switch (key) {
    case 0: return launch4<false, false, false, false>(g, b, a, sc, stream);
    case 1: return launch4<false, false, false, true>(g, b, a, sc, stream);
    case 4: return launch4<false, true, false, false>(g, b, a, sc, stream);
    case 5: return launch4<false, true, false, true>(g, b, a, sc, stream);
    case 6: return launch4<false, true, true, false>(g, b, a, sc, stream);
    case 7: return launch4<false, true, true, true>(g, b, a, sc, stream);
    case 8: return launch4<true, false, false, false>(g, b, a, sc, stream);
    case 9: return launch4<true, false, false, true>(g, b, a, sc, stream);
    case 12: return launch4<true, true, false, false>(g, b, a, sc, stream);
    case 13: return launch4<true, true, false, true>(g, b, a, sc, stream);
    case 14: return launch4<true, true, true, false>(g, b, a, sc, stream);
    case 15: return launch4<true, true, true, true>(g, b, a, sc, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pack_spring_consts(const GatherGraph &g, const BatchLayout &b, const int64_t *sp_slot,
                                     const int64_t *sp_off, float4 *kcs, float2 *rest, hipStream_t stream)
{
    if (b.n_groups == 0)
        return hipSuccess;
    if (rest && !g.d0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(pack_spring_consts, dim3((unsigned)b.n_groups), dim3(256), 0, stream, g, sp_slot, sp_off,
                       kcs, rest);
    return hipGetLastError();
}

hipError_t launch_spring_grads(const float4 *gslot, const int64_t *owner_slot, int64_t ns, float *gk, float *gC,
                               float *gS, hipStream_t stream)
{
    if (ns == 0)
        return hipSuccess;
    hipLaunchKernelGGL(gather_spring_grads, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, stream, gslot,
                       owner_slot, ns, gk, gC, gS);
    return hipGetLastError();
}

hipError_t launch_voxel_grads(int64_t nv, const int64_t *vs_ptr, const int32_t *vs_spring, const float *inv_cnt,
                              const float4 *vw, const float *gC, const float *gS, float *ga, float *gphi,
                              hipStream_t stream)
{
    if (nv == 0)
        return hipSuccess;
    hipLaunchKernelGGL(voxel_grads_kernel, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, stream, nv, vs_ptr,
                       vs_spring, inv_cnt, vw, gC, gS, ga, gphi);
    return hipGetLastError();
}

hipError_t launch_body_loss(const float *dux, const float *coef, const int64_t *body_off, int64_t nb, float *loss,
                            hipStream_t stream)
{
    if (nb == 0)
        return hipSuccess;
    hipLaunchKernelGGL(body_loss, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, stream, dux, coef, body_off, nb, loss);
    return hipGetLastError();
}

}  // namespace titan

// Host side of the gather engine: incidence lists in sliced-ELL layout with
// per-incidence spring constants, and the per-step launch loop.
//
// Sec. III-B of the paper describes an accumulation variant in which every
// mass knows its springs in a fixed order and sums their forces; this layout
// is that variant made gather-only: each mass's row lists (neighbour, spring
// constants) sorted by neighbour, so the force sum has one fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "titan_sim.h"

namespace titan {

int build_batch_engine(titan_sim *s);  // engine_batch.hip
int enqueue_batch_steps(titan_sim *s, int64_t first_step, int64_t count);
void destroy_batch_engine(titan_sim *s);

#define HIP_TRY(sim, expr)                                  \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess)                               \
            return titan::hip_fail((sim), e_, #expr);       \
    } while (0)

template <class T>
static int put(titan_sim *s, const std::vector<T> &h, const T **d)
{
    T *p = nullptr;
    if (int rc = dev_alloc(s, h.size() * sizeof(T), (void **)&p))
        return rc;
    if (!h.empty())
        HIP_TRY(s, hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s->stream));
    *d = p;
    return TITAN_OK;
}

static int build_gather(titan_sim *s)
{
    const int64_t n = s->n, ns = s->ns;
    std::vector<int64_t> inv(n);
    for (int64_t i = 0; i < n; ++i)
        inv[s->perm[i]] = i;

    // Incidence rows (internal order), each sorted by (neighbour, spring).
    std::vector<int32_t> deg(n, 0);
    for (int64_t q = 0; q < ns; ++q) {
        ++deg[inv[s->h_ends[2 * q]]];
        ++deg[inv[s->h_ends[2 * q + 1]]];
    }
    std::vector<int64_t> rp(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        rp[i + 1] = rp[i] + deg[i];
    struct Inc {
        int32_t nbr;
        int32_t spring;
    };
    std::vector<Inc> inc(rp[n]);
    {
        std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
        for (int64_t q = 0; q < ns; ++q) {
            const int64_t a = inv[s->h_ends[2 * q]], b = inv[s->h_ends[2 * q + 1]];
            inc[fill[a]++] = {(int32_t)b, (int32_t)q};
            inc[fill[b]++] = {(int32_t)a, (int32_t)q};
        }
    }
    for (int64_t i = 0; i < n; ++i)
        std::sort(inc.begin() + rp[i], inc.begin() + rp[i + 1], [](const Inc &x, const Inc &y) {
            return x.nbr != y.nbr ? x.nbr < y.nbr : x.spring < y.spring;
        });

    // Per-spring constants (FP64 -> FP32).
    bool act = false, rest = false, damp_uniform = true;
    for (int64_t q = 0; q < ns; ++q) {
        act |= s->h_amp[q] != 0.f;
        rest |= s->h_rest[q] > 0.f;
        damp_uniform &= s->h_damp[q] == s->h_damp[0];
    }
    std::vector<float> sC, sS, sD0, sL0;
    if (act) {
        sC.resize(ns);
        sS.resize(ns);
        for (int64_t q = 0; q < ns; ++q) {
            sC[q] = (float)((double)s->h_amp[q] * std::cos((double)s->h_phase[q]));
            sS[q] = (float)((double)s->h_amp[q] * std::sin((double)s->h_phase[q]));
        }
    }
    if (rest) {
        sD0.resize(ns);
        sL0.resize(ns);
        for (int64_t q = 0; q < ns; ++q) {
            const float *a = &s->h_pos[3 * s->h_ends[2 * q]], *b = &s->h_pos[3 * s->h_ends[2 * q + 1]];
            const double dx = (double)b[0] - a[0], dy = (double)b[1] - a[1], dz = (double)b[2] - a[2];
            const double R = std::sqrt(dx * dx + dy * dy + dz * dz);
            const double L = s->h_rest[q] > 0.f ? (double)s->h_rest[q] : R;
            sD0[q] = (float)(R - L);
            sL0[q] = (float)L;
        }
    }

    // Sliced ELL.
    const int64_t nsl = (n + kSlice - 1) / kSlice;
    std::vector<int64_t> off(nsl + 1, 0);
    for (int64_t sl = 0; sl < nsl; ++sl) {
        int32_t w = 0;
        for (int64_t i = sl * kSlice; i < std::min(n, (sl + 1) * kSlice); ++i)
            w = std::max(w, deg[i]);
        off[sl + 1] = off[sl] + (int64_t)w * kSlice;
    }
    const int64_t slots = off[nsl];
    std::vector<int32_t> nbr(slots, 0);
    std::vector<float> kk(slots, 0.f), cc, ac, as, d0, L0;
    if (!damp_uniform)
        cc.assign(slots, 0.f);
    if (act) {
        ac.assign(slots, 0.f);
        as.assign(slots, 0.f);
    }
    if (rest) {
        d0.assign(slots, 0.f);
        L0.assign(slots, 1.f);
    }
    for (int64_t i = 0; i < n; ++i) {
        const int64_t base = off[i / kSlice] + (i % kSlice);
        for (int64_t w = 0; w < deg[i]; ++w) {
            const Inc &x = inc[rp[i] + w];
            const int64_t e = base + w * kSlice;
            nbr[e] = x.nbr;
            kk[e] = s->h_k[x.spring];
            if (!damp_uniform)
                cc[e] = s->h_damp[x.spring];
            if (act) {
                ac[e] = sC[x.spring];
                as[e] = sS[x.spring];
            }
            if (rest) {
                d0[e] = sD0[x.spring];
                L0[e] = sL0[x.spring];
            }
        }
    }

    GatherGraph &g = s->gg;
    g = GatherGraph{};
    g.n = n;
    g.n_slices = nsl;
    g.c_uniform = (ns > 0 && damp_uniform) ? s->h_damp[0] : 0.f;
    if (int rc = put(s, off, &g.slice_off))
        return rc;
    if (int rc = put(s, deg, &g.deg))
        return rc;
    if (int rc = put(s, nbr, &g.nbr))
        return rc;
    if (int rc = put(s, kk, &g.k))
        return rc;
    if (!damp_uniform)
        if (int rc = put(s, cc, &g.c))
            return rc;
    if (act) {
        if (int rc = put(s, ac, &g.act_c))
            return rc;
        if (int rc = put(s, as, &g.act_s))
            return rc;
    }
    if (rest) {
        if (int rc = put(s, d0, &g.d0))
            return rc;
        if (int rc = put(s, L0, &g.rest))
            return rc;
    }
    g.X0 = s->X0;
    // keep the staging alive until the copies have run
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return TITAN_OK;
}

int build_engines(titan_sim *s)
{
    if (s->params.engine == TITAN_ENGINE_BATCHED || s->params.engine == TITAN_ENGINE_AUTO) {
        const int rc = build_batch_engine(s);
        if (rc == TITAN_OK && s->batch) {
            s->engine = TITAN_ENGINE_BATCHED;
        } else if (rc != TITAN_OK && s->params.engine == TITAN_ENGINE_BATCHED) {
            return rc;
        }
    }
    // The gather representation is always built: it serves the plain engine
    // and the force query of either engine.
    return build_gather(s);
}

static StepConsts consts_for(const titan_sim *s, int64_t step)
{
    StepConsts sc{};
    const titan_params &p = s->params;
    sc.dt = (float)p.dt;
    sc.gx = (float)p.gravity[0];
    sc.gy = (float)p.gravity[1];
    sc.gz = (float)p.gravity[2];
    sc.ground = p.ground ? 1 : 0;
    sc.ground_k = (float)p.ground_k;
    sc.mu = (float)p.friction_mu;
    const double ph = p.omega * ((double)step * p.dt);
    sc.sin_wt = (float)std::sin(ph);
    sc.cos_wt = (float)std::cos(ph);
    sc.step = step;
    return sc;
}

int enqueue_steps(titan_sim *s, int64_t first_step, int64_t count)
{
    if (s->engine == TITAN_ENGINE_BATCHED && s->batch)
        return enqueue_batch_steps(s, first_step, count);
    for (int64_t q = 0; q < count; ++q) {
        StateIO io{};
        io.U_in = s->U[s->cur];
        io.V_in = s->V[s->cur];
        io.U_out = s->U[1 - s->cur];
        io.V_out = s->V[1 - s->cur];
        io.first_bad = s->first_bad;
        const StepConsts sc = consts_for(s, first_step + q);
        HIP_TRY(s, launch_gather_step(s->gg, io, sc, false, s->stream));
        s->cur = 1 - s->cur;
    }
    return TITAN_OK;
}

int compute_forces(titan_sim *s)
{
    if (!s->F)
        if (int rc = dev_alloc(s, sizeof(float4) * s->n, (void **)&s->F))
            return rc;
    StateIO io{};
    io.U_in = s->U[s->cur];
    io.V_in = s->V[s->cur];
    io.F_out = s->F;
    io.first_bad = s->first_bad;
    const StepConsts sc = consts_for(s, s->step_enq);
    HIP_TRY(s, launch_gather_step(s->gg, io, sc, true, s->stream));
    return TITAN_OK;
}

void destroy_engines(titan_sim *s) { destroy_batch_engine(s); }

}  // namespace titan

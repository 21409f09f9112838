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
#include <cstring>
#include <memory>
#include <unordered_map>
#include <vector>

#include "titan_sim.h"

namespace titan {

int build_batch_engine(titan_sim *s, bool may_step);  // engine_batch.hip
int enqueue_batch_integ(titan_sim *s, int64_t first_step, int64_t count);
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

// Interleave the low 21 bits of x with two zero bits between each.
static uint64_t spread3(uint64_t x)
{
    x &= 0x1fffffull;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

// Internal mass order: bodies contiguous, largest body first (ties by body
// id); within a body, Morton (Z-order) of the reference positions quantised
// to cells of about one short spring length, so that consecutive masses --
// and therefore each tile -- form compact regions.  Ties keep caller order.
// Then, inside each tile, masses are ordered by degree (below).
void plan_order(titan_sim *s)
{
    const int64_t n = s->n, ns = s->ns;
    s->perm.resize(n);
    if (n == 0)
        return;
    double lo[3] = {1e300, 1e300, 1e300};
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c)
            lo[c] = std::min(lo[c], (double)s->h_pos[3 * i + c]);
    double h = 1.0;
    if (ns > 0) {
        std::vector<double> len;
        const int64_t stride = std::max<int64_t>(1, ns / 65536);
        for (int64_t q = 0; q < ns; q += stride) {
            const float *a = &s->h_pos[3 * s->h_ends[2 * q]], *b = &s->h_pos[3 * s->h_ends[2 * q + 1]];
            const double dx = (double)b[0] - a[0], dy = (double)b[1] - a[1], dz = (double)b[2] - a[2];
            len.push_back(std::sqrt(dx * dx + dy * dy + dz * dz));
        }
        std::nth_element(len.begin(), len.begin() + len.size() / 10, len.end());
        h = len[len.size() / 10];
    }
    // body rank: by size, descending
    int32_t nb = 0;
    for (int32_t b : s->h_body)
        nb = std::max(nb, b + 1);
    std::vector<int64_t> bsize(nb, 0);
    for (int32_t b : s->h_body)
        ++bsize[b];
    std::vector<int32_t> border(nb);
    for (int32_t b = 0; b < nb; ++b)
        border[b] = b;
    std::stable_sort(border.begin(), border.end(), [&](int32_t a, int32_t b) { return bsize[a] > bsize[b]; });
    std::vector<int32_t> brank(nb);
    for (int32_t r = 0; r < nb; ++r)
        brank[border[r]] = r;
    struct Key {
        int32_t rank;
        uint64_t morton;
        int64_t caller;
        bool operator<(const Key &o) const
        {
            if (rank != o.rank)
                return rank < o.rank;
            if (morton != o.morton)
                return morton < o.morton;
            return caller < o.caller;
        }
    };
    std::vector<Key> key(n);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t m = 0;
        for (int c = 0; c < 3; ++c) {
            double q = std::floor(((double)s->h_pos[3 * i + c] - lo[c]) / h + 0.5);
            q = std::min(std::max(q, 0.0), 2097151.0);
            m |= spread3((uint64_t)q) << c;
        }
        key[i] = {brank[s->h_body[i]], m, i};
    }
    std::sort(key.begin(), key.end());
    for (int64_t i = 0; i < n; ++i)
        s->perm[i] = key[i].caller;

    // Within each run of masses that share a tile and a body, masses of
    // higher degree first (stable): the 64-mass slices of the incidence
    // layout then hold masses of similar degree, so their rows need little
    // padding (voxel robots mix degrees 7 to 26).  Tiles and bodies keep
    // their masses, and no result depends on the internal order.
    std::vector<int32_t> deg(n, 0);
    for (int64_t q = 0; q < ns; ++q) {
        ++deg[s->h_ends[2 * q]];
        ++deg[s->h_ends[2 * q + 1]];
    }
    for (int64_t a = 0; a < n;) {
        int64_t b = a + 1;
        while (b < n && b % kTile != 0 && s->h_body[s->perm[b]] == s->h_body[s->perm[a]])
            ++b;
        std::stable_sort(s->perm.begin() + a, s->perm.begin() + b,
                         [&](int64_t x, int64_t y) { return deg[x] > deg[y]; });
        a = b;
    }
}

// Per-spring constants in the layouts' form.
// Phasor actuation: C = amp cos(phase), S = amp sin(phase), kept in the host
// tables (FP32 of the FP64 products, or the values given directly).
static void phasor_consts(const titan_sim *s, int64_t q, float &C, float &S)
{
    C = s->h_C[q];
    S = s->h_S[q];
}

// Does spring q carry actuation (either law)?
static bool actuated(const titan_sim *s, int64_t q)
{
    return s->h_amp[q] != 0.f || s->h_C[q] != 0.f || s->h_S[q] != 0.f;
}

// Explicit rest length L (else the reference length |R|): d0 = |R| - L, L0 = L.
static void rest_consts(const titan_sim *s, int64_t q, float &d0, float &L0)
{
    const float *a = &s->h_pos[3 * s->h_ends[2 * q]], *b = &s->h_pos[3 * s->h_ends[2 * q + 1]];
    const double dx = (double)b[0] - a[0], dy = (double)b[1] - a[1], dz = (double)b[2] - a[2];
    const double R = std::sqrt(dx * dx + dy * dy + dz * dz);
    const double L = s->h_rest[q] > 0.f ? (double)s->h_rest[q] : R;
    d0 = (float)(R - L);
    L0 = (float)L;
}

// Sec. IV-B, Eq. 5: the wave offset t_o of a spring is the smaller reference
// x of its two ends minus the smallest reference x of its body.
static std::vector<double> body_xmin(const titan_sim *s)
{
    int32_t nb = 0;
    for (int32_t b : s->h_body)
        nb = std::max(nb, b + 1);
    std::vector<double> xmin(nb, INFINITY);
    for (size_t i = 0; i < s->h_body.size(); ++i)
        xmin[s->h_body[i]] = std::min(xmin[s->h_body[i]], (double)s->h_pos[3 * i]);
    return xmin;
}

static double wave_offset(const titan_sim *s, const std::vector<double> &xmin, int64_t q)
{
    const int64_t a = s->h_ends[2 * q], b = s->h_ends[2 * q + 1];
    return std::min((double)s->h_pos[3 * a], (double)s->h_pos[3 * b]) - xmin[s->h_body[a]];
}

// Host tables of the gather layout, planned without touching the device.
struct GatherPlan {
    bool allow_tiled = false, tiled = false;
    bool k_uniform = true, damp_uniform = true, act = false, wave = false, rest = false, yield = false;
    int64_t q0 = -1, nt = 0, nsl = 0, slots = 0;
    int32_t max_local = 0;
    std::vector<int32_t> deg, nbr, halo_idx;
    std::vector<int64_t> off, halo_off;
    std::vector<uint16_t> nbr_local;
    std::vector<float> kk, cc, ac, as, d0, L0, yy;
    std::vector<double> to;
    // wave law on the tiled layout: each tile's distinct offsets, per slot
    // its class (see GatherGraph::tile_wave_*)
    std::vector<uint16_t> twc;
    std::vector<int64_t> twoff;
    std::vector<double> twt;
    int32_t max_tw = 0;
};

// Per tile, the distinct offsets of its masses' slots (padding included),
// sorted by bit pattern, and each slot's index among them; none when a tile
// has more than 1,024 or the table would not fit beside the tile's state.
static void plan_tile_wave(GatherPlan &P, int64_t n)
{
    const int64_t nt = P.nt;
    std::vector<uint16_t> cls(P.slots, 0);
    std::vector<int64_t> woff(1, 0);
    std::vector<double> wt;
    int64_t maxw = 0;
    for (int64_t t = 0; t < nt; ++t) {
        std::vector<std::pair<uint64_t, int64_t>> keys;
        for (int64_t i = t * kTile; i < std::min(n, (t + 1) * kTile); ++i) {
            const int64_t sl = i / kSlice, base = P.off[sl] + (i % kSlice);
            const int64_t width = (P.off[sl + 1] - P.off[sl]) / kSlice;
            for (int64_t w = 0; w < width; ++w) {
                uint64_t bits;
                memcpy(&bits, &P.to[base + w * kSlice], 8);
                keys.push_back({bits, base + w * kSlice});
            }
        }
        std::sort(keys.begin(), keys.end());
        int64_t c = -1;
        for (size_t a = 0; a < keys.size(); ++a) {
            if (a == 0 || keys[a].first != keys[a - 1].first) {
                if (++c >= 1024)
                    return;
                double v;
                memcpy(&v, &keys[a].first, 8);
                wt.push_back(v);
            }
            cls[keys[a].second] = (uint16_t)c;
        }
        woff.push_back((int64_t)wt.size());
        maxw = std::max(maxw, c + 1);
    }
    if ((int64_t)P.max_local * 3 * 16 + maxw * 4 > 65536)  // (three state arrays at most)
        return;
    P.twc.swap(cls);
    P.twoff.swap(woff);
    P.twt.swap(wt);
    P.max_tw = (int32_t)maxw;
}

// Plan the gather layout on the host (internal order already in s->perm):
// incidence rows, tiles and halos, sliced-ELL slots and per-slot constants.
// Also fills s->inv_perm and each spring's two slots.  Host work on the host
// tables only; every size may be zero (no springs, no masses).
static void plan_gather(titan_sim *s, bool allow_tiled, GatherPlan &P)
{
    const int64_t n = s->n, ns = s->ns;
    P = GatherPlan{};
    P.allow_tiled = allow_tiled;
    std::vector<int64_t> &inv = s->inv_perm;
    inv.assign(n, 0);
    for (int64_t i = 0; i < n; ++i)
        inv[s->perm[i]] = i;

    // Incidence rows (internal order), each sorted by the neighbour's caller
    // index (then spring index): the summation order, hence the result, does
    // not depend on the internal order or on the tiling.
    auto live = [&](int64_t q) { return s->h_removed.empty() || !s->h_removed[q]; };
    std::vector<int32_t> &deg = P.deg;
    deg.assign(n, 0);
    for (int64_t q = 0; q < ns; ++q) {
        if (!live(q))
            continue;
        ++deg[inv[s->h_ends[2 * q]]];
        ++deg[inv[s->h_ends[2 * q + 1]]];
    }
    std::vector<int64_t> rp(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        rp[i + 1] = rp[i] + deg[i];
    struct Inc {
        int32_t nbr_caller;
        int32_t spring;
    };
    std::vector<Inc> inc(rp[n]);
    {
        std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
        for (int64_t q = 0; q < ns; ++q) {
            if (!live(q))
                continue;
            const int64_t a = s->h_ends[2 * q], b = s->h_ends[2 * q + 1];
            inc[fill[inv[a]]++] = {(int32_t)b, (int32_t)q};
            inc[fill[inv[b]]++] = {(int32_t)a, (int32_t)q};
        }
    }
    for (int64_t i = 0; i < n; ++i)
        std::sort(inc.begin() + rp[i], inc.begin() + rp[i + 1], [](const Inc &x, const Inc &y) {
            return x.nbr_caller != y.nbr_caller ? x.nbr_caller < y.nbr_caller : x.spring < y.spring;
        });

    // Tiles and halos.
    const int64_t nt = (n + kTile - 1) / kTile;
    P.nt = nt;
    std::vector<int64_t> &halo_off = P.halo_off;
    halo_off.assign(nt + 1, 0);
    std::vector<int32_t> &halo_idx = P.halo_idx;
    int32_t &max_local = P.max_local;
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t a = t * kTile, b = std::min(n, a + kTile);
        std::vector<int32_t> h;
        for (int64_t i = a; i < b; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                const int64_t j = inv[inc[e].nbr_caller];
                if (j < a || j >= b)
                    h.push_back((int32_t)j);
            }
        std::sort(h.begin(), h.end());
        h.erase(std::unique(h.begin(), h.end()), h.end());
        halo_idx.insert(halo_idx.end(), h.begin(), h.end());
        halo_off[t + 1] = (int64_t)halo_idx.size();
        max_local = std::max<int32_t>(max_local, kTile + (int32_t)h.size());
    }
    // LDS per tile: 3 float4 per local entry must fit the default 64 KB.
    const bool tiled = P.tiled = allow_tiled && max_local * 3 * (int64_t)sizeof(float4) <= 65536;

    // Per-spring constants (FP64 -> FP32).
    // (over the springs present; q0: the first of them)
    // Breakable springs keep damping and rest lengths per slot (one kernel
    // variant per actuation law).
    const bool yield = P.yield = !s->h_yield.empty();
    int64_t &q0 = P.q0;
    bool &act = P.act, &rest = P.rest, &damp_uniform = P.damp_uniform, &k_uniform = P.k_uniform;
    rest = yield;
    damp_uniform = !yield;
    for (int64_t q = 0; q < ns; ++q) {
        if (!live(q))
            continue;
        if (q0 < 0)
            q0 = q;
        act |= actuated(s, q);
        rest |= s->h_rest[q] > 0.f;
        damp_uniform &= s->h_damp[q] == s->h_damp[q0];
        k_uniform &= s->h_k[q] == s->h_k[q0];
    }
    const bool wave = P.wave = act && s->params.actuation == TITAN_ACT_WAVE;
    std::vector<float> sC, sS, sD0, sL0;
    std::vector<double> sT;
    if (act && !wave) {
        sC.resize(ns);
        sS.resize(ns);
        for (int64_t q = 0; q < ns; ++q)
            phasor_consts(s, q, sC[q], sS[q]);
    }
    if (wave) {
        const std::vector<double> xmin = body_xmin(s);
        sC.resize(ns);
        sT.resize(ns);
        for (int64_t q = 0; q < ns; ++q) {
            sC[q] = s->h_amp[q];
            sT[q] = wave_offset(s, xmin, q);
        }
    }
    if (rest) {
        sD0.resize(ns);
        sL0.resize(ns);
        for (int64_t q = 0; q < ns; ++q)
            rest_consts(s, q, sD0[q], sL0[q]);
    }

    // Sliced ELL (slices of 64 masses; a tile is 4 slices).
    const int64_t nsl = P.nsl = (n + kSlice - 1) / kSlice;
    std::vector<int64_t> &off = P.off;
    off.assign(nsl + 1, 0);
    for (int64_t sl = 0; sl < nsl; ++sl) {
        int32_t w = 0;
        for (int64_t i = sl * kSlice; i < std::min(n, (sl + 1) * kSlice); ++i)
            w = std::max(w, deg[i]);
        w += s->slack;  // spare slots for springs added later (after an edit)
        off[sl + 1] = off[sl] + (int64_t)w * kSlice;
    }
    const int64_t slots = P.slots = off[nsl];
    std::vector<int32_t> &nbr = P.nbr;  // internal index of the other end, per slot
    nbr.assign(slots, 0);
    std::vector<uint16_t> &nbr_local = P.nbr_local;
    if (tiled)
        nbr_local.assign(slots, 0);
    std::vector<float> &kk = P.kk, &cc = P.cc, &ac = P.ac, &as = P.as, &d0 = P.d0, &L0 = P.L0, &yy = P.yy;
    std::vector<double> &to = P.to;
    if (yield)
        yy.assign(slots, INFINITY);  // padding never breaks
    if (!k_uniform)
        kk.assign(slots, 0.f);
    if (!damp_uniform)
        cc.assign(slots, 0.f);
    if (act) {
        ac.assign(slots, 0.f);
        if (wave)
            to.assign(slots, 0.0);
        else
            as.assign(slots, 0.f);
    }
    if (rest) {
        d0.assign(slots, 0.f);
        L0.assign(slots, 1.f);
    }
    s->h_owner_slot.assign(ns, -1);
    s->h_other_slot.assign(ns, -1);
    ++s->slot_gen;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t base = off[i / kSlice] + (i % kSlice);
        const int64_t t = i / kTile, a = t * kTile;
        const int32_t *hb = halo_idx.data() + halo_off[t], *he = halo_idx.data() + halo_off[t + 1];
        // Padding slots (past this mass's degree, up to the slice width) point
        // the mass at itself with zero constants: zero force.
        const int64_t width = (off[i / kSlice + 1] - off[i / kSlice]) / kSlice;
        for (int64_t w = deg[i]; w < width; ++w) {
            if (tiled)
                nbr_local[base + w * kSlice] = (uint16_t)(i - a);
            nbr[base + w * kSlice] = (int32_t)i;
        }
        for (int64_t w = 0; w < deg[i]; ++w) {
            const Inc &x = inc[rp[i] + w];
            const int64_t e = base + w * kSlice;
            const int64_t j = inv[x.nbr_caller];
            if (tiled) {
                if (j >= a && j < a + kTile)
                    nbr_local[e] = (uint16_t)(j - a);
                else
                    nbr_local[e] = (uint16_t)(kTile + (std::lower_bound(hb, he, (int32_t)j) - hb));
            }
            nbr[e] = (int32_t)j;
            if (j > i)
                s->h_owner_slot[x.spring] = e;
            else
                s->h_other_slot[x.spring] = e;
            if (!k_uniform)
                kk[e] = s->h_k[x.spring];
            if (!damp_uniform)
                cc[e] = s->h_damp[x.spring];
            if (act) {
                ac[e] = sC[x.spring];
                if (wave)
                    to[e] = sT[x.spring];
                else
                    as[e] = sS[x.spring];
            }
            if (rest) {
                d0[e] = sD0[x.spring];
                L0[e] = sL0[x.spring];
            }
            if (yield)
                yy[e] = s->h_yield[x.spring];
        }
    }
    if (tiled && wave)
        plan_tile_wave(P, n);
}

// Upload a planned gather layout and make it the current one.
static int upload_gather(titan_sim *s, GatherPlan &P)
{
    const int64_t n = s->n;
    const bool tiled = P.tiled, yield = P.yield, act = P.act, wave = P.wave, rest = P.rest;
    const bool k_uniform = P.k_uniform, damp_uniform = P.damp_uniform;
    const int64_t q0 = P.q0, slots = P.slots;
    GatherGraph &g = s->gg;
    g = GatherGraph{};
    g.n = n;
    g.n_slices = P.nsl;
    g.n_tiles = P.nt;
    g.max_local = P.max_local;
    g.c_uniform = (q0 >= 0 && damp_uniform) ? s->h_damp[q0] : 0.f;
    g.k_uniform = (q0 >= 0 && k_uniform) ? s->h_k[q0] : 0.f;
    if (int rc = put(s, P.off, &g.slice_off))
        return rc;
    if (int rc = put(s, P.deg, &g.deg))
        return rc;
    if (tiled) {
        if (int rc = put(s, P.nbr_local, &g.nbr_local))
            return rc;
        if (int rc = put(s, P.halo_off, &g.halo_off))
            return rc;
        if (int rc = put(s, P.halo_idx, &g.halo_idx))
            return rc;
    } else {
        if (int rc = put(s, P.nbr, &g.nbr))
            return rc;
    }
    if (!k_uniform)
        if (int rc = put(s, P.kk, &g.k))
            return rc;
    if (!damp_uniform)
        if (int rc = put(s, P.cc, &g.c))
            return rc;
    if (act) {
        if (int rc = put(s, P.ac, &g.act_c))
            return rc;
        if (wave) {
            if (int rc = put(s, P.to, &g.t_off))
                return rc;
        } else {
            if (int rc = put(s, P.as, &g.act_s))
                return rc;
        }
    }
    if (rest) {
        if (int rc = put(s, P.d0, &g.d0))
            return rc;
        if (int rc = put(s, P.L0, &g.rest))
            return rc;
    }
    if (yield) {
        const float *p = nullptr;
        if (int rc = put(s, P.yy, &p))
            return rc;
        g.yield = const_cast<float *>(p);  // the step records breaks here
    }
    if (!P.twc.empty()) {
        if (int rc = put(s, P.twc, &g.tile_wave_cls))
            return rc;
        if (int rc = put(s, P.twoff, &g.tile_wave_off))
            return rc;
        if (int rc = put(s, P.twt, &g.tile_wave_t))
            return rc;
        g.max_tile_wave = P.max_tw;
    }
    g.X0 = s->X0;
    s->tiled = tiled;
    s->n_slots = slots;
    // keep the staging alive until the copies have run
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    s->h_slot_nbr.swap(P.nbr);  // for the batched engine's layout
    // what insertion in place needs of the layout
    s->h_deg.swap(P.deg);
    s->h_slice_off.swap(P.off);
    if (tiled) {
        s->h_halo_off.swap(P.halo_off);
        s->h_halo_idx.swap(P.halo_idx);
    } else {
        std::vector<int64_t>().swap(s->h_halo_off);
        std::vector<int32_t>().swap(s->h_halo_idx);
    }
    ++s->layout_builds;
    return TITAN_OK;
}

static int build_gather(titan_sim *s, bool allow_tiled)
{
    // a plan made before the device was set up (finalize) is used once
    std::shared_ptr<GatherPlan> P = std::move(s->gplan);
    if (!P || P->allow_tiled != allow_tiled) {
        P = std::make_shared<GatherPlan>();
        plan_gather(s, allow_tiled, *P);
    }
    return upload_gather(s, *P);
}

void plan_layouts(titan_sim *s)
{
    s->n = (int64_t)s->h_mass.size();
    s->ns = (int64_t)s->h_k.size();
    plan_order(s);
    auto P = std::make_shared<GatherPlan>();
    plan_gather(s, s->params.engine != TITAN_ENGINE_GATHER, *P);
    s->gplan = std::move(P);
}

// Allocations made while an engine's layout is built or updated belong to the
// engine (freed when the layout is rebuilt).
struct EngineAllocs {
    titan_sim *s;
    bool was;
    explicit EngineAllocs(titan_sim *sim) : s(sim), was(sim->engine_allocs) { s->engine_allocs = true; }
    ~EngineAllocs() { s->engine_allocs = was; }
};

int build_engines(titan_sim *s)
{
    EngineAllocs mark(s);
    const int want = s->params.engine;
    if (int rc = dev_alloc(s, sizeof(float2) * (kTrigChunk + 1), (void **)&s->trig))
        return rc;
    // The gather representation is always built: it serves the plain engines
    // and the force query of every engine.
    if (int rc = build_gather(s, want != TITAN_ENGINE_GATHER))
        return rc;
    s->engine = s->tiled ? TITAN_ENGINE_TILED : TITAN_ENGINE_GATHER;
    // The batched layout is built whenever the bodies fit it (the adjoint
    // uses it); it steps the system when asked for, or when AUTO times it
    // faster.
    if (int rc = build_batch_engine(s, want == TITAN_ENGINE_BATCHED || want == TITAN_ENGINE_AUTO))
        return rc;
    // (the Verlet and RK4 kernels hold more per mass: larger groups step with
    // the per-step engines under AUTO)
    if (s->batch && s->batch_step && s->params.integrator != TITAN_INTEG_EULER &&
        !batch_integ_fits(batch_layout(s), s->params.integrator)) {
        if (want == TITAN_ENGINE_BATCHED)
            return fail(TITAN_EINVAL, "the batched engine cannot run this integrator on this system (a group of "
                                      "%d masses is too large)", batch_layout(s).max_group);
        s->batch_step = false;
    }
    const bool integ_ok = s->params.integrator == TITAN_INTEG_EULER || want == TITAN_ENGINE_BATCHED ||
                          (s->batch && batch_integ_preferred(batch_layout(s)));
    if (s->batch && s->batch_step && integ_ok)
        s->engine = TITAN_ENGINE_BATCHED;
    else if (want == TITAN_ENGINE_BATCHED)
        return fail(TITAN_EINVAL, "the batched engine cannot run this system (a body does not fit in LDS)");
    std::vector<int32_t>().swap(s->h_slot_nbr);
    return TITAN_OK;
}

// Spring constants changed after the device layout exists (the new values
// are in the host table): both incidence slots of every listed spring that is
// in the layout are rewritten on the device, in stream order.  A uniform
// stiffness/damping that stops being uniform, or actuation that appears, gets
// its per-slot array first.
int update_spring_list(titan_sim *s, const std::vector<int64_t> &springs, bool k, bool damping, bool amp,
                       bool force)
{
    EngineAllocs mark(s);
    GatherGraph &g = s->gg;
    std::vector<int64_t> slot, of;
    for (int64_t q : springs)
        if (s->h_owner_slot[q] >= 0) {
            slot.push_back(s->h_owner_slot[q]);
            slot.push_back(s->h_other_slot[q]);
            of.push_back(q);
            of.push_back(q);
        }
    const int64_t m = (int64_t)slot.size();
    std::vector<void *> tmp;
    auto cleanup = [&]() {
        for (void *p : tmp)
            dev_free(s, p);
    };
    int64_t *dslot = nullptr;
    float *dval = nullptr;
    if (int rc = dev_alloc(s, sizeof(int64_t) * std::max<int64_t>(m, 1), (void **)&dslot))
        return rc;
    tmp.push_back(dslot);
    if (int rc = dev_alloc(s, sizeof(float) * std::max<int64_t>(m, 1), (void **)&dval)) {
        cleanup();
        return rc;
    }
    tmp.push_back(dval);
    std::vector<float> val(m);
    // one per-slot array: allocate it (filled with `fill`) if absent, then scatter
    auto apply = [&](const float **arr, float fill, auto value_of) -> hipError_t {
        if (!*arr) {
            float *p = nullptr;
            if (dev_alloc(s, sizeof(float) * std::max<int64_t>(s->n_slots, 1), (void **)&p))
                return hipErrorOutOfMemory;
            if (hipError_t e = launch_fill(p, fill, s->n_slots, s->stream))
                return e;
            *arr = p;
        }
        if (m == 0)
            return hipSuccess;
        for (int64_t e = 0; e < m; ++e)
            val[e] = value_of(of[e]);
        if (hipError_t e = hipMemcpyAsync(dval, val.data(), sizeof(float) * m, hipMemcpyHostToDevice, s->stream))
            return e;
        if (hipError_t e = launch_scatter(const_cast<float *>(*arr), dslot, dval, m, s->stream))
            return e;
        // the staging values are reused by the next array: wait for this one
        return hipStreamSynchronize(s->stream);
    };
    // uniform over the springs present?
    auto uniform_of = [&](const std::vector<float> &v, float &u) {
        bool seen = false;
        for (int64_t q = 0; q < s->ns; ++q) {
            if (!s->h_removed.empty() && s->h_removed[q])
                continue;
            if (!seen) {
                u = v[q];
                seen = true;
            } else if (v[q] != u) {
                return false;
            }
        }
        return seen;
    };
    hipError_t e = hipSuccess;
    int rc = TITAN_OK;
    if (m)
        e = hipMemcpyAsync(dslot, slot.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s->stream);
    if (!e && k) {
        float u = 0.f;
        if (!g.k && !force && uniform_of(s->h_k, u))
            g.k_uniform = u;
        else
            e = apply(&g.k, g.k_uniform, [&](int64_t q) { return s->h_k[q]; });
    }
    if (!e && damping) {
        float u = 0.f;
        if (!g.c && !force && uniform_of(s->h_damp, u))
            g.c_uniform = u;
        else
            e = apply(&g.c, g.c_uniform, [&](int64_t q) { return s->h_damp[q]; });
    }
    if (!e && amp && g.t_off) {
        // wave law: the amplitude is the factor; the offsets stay those of Eq. 5
        e = apply(&g.act_c, 0.f, [&](int64_t q) { return s->h_amp[q]; });
    } else if (!e && amp && s->params.actuation == TITAN_ACT_WAVE) {
        rc = fail(TITAN_ESTATE, "wave actuation must be present when the system is finalized");
    } else if (!e && amp) {
        e = apply(&g.act_c, 0.f, [&](int64_t q) { return s->h_C[q]; });
        if (!e)
            e = apply(&g.act_s, 0.f, [&](int64_t q) { return s->h_S[q]; });
    }
    if (e != hipSuccess)
        rc = e == hipErrorOutOfMemory ? fail(TITAN_ENOMEM, "out of device memory updating spring constants")
                                      : hip_fail(s, e, "updating spring constants");
    cleanup();
    return rc;
}

int update_springs(titan_sim *s, int64_t first, int64_t count, const float *k, const float *damping,
                   const float *amp, const float *phase)
{
    (void)phase;
    std::vector<int64_t> list(count);
    for (int64_t q = 0; q < count; ++q)
        list[q] = first + q;
    return update_spring_list(s, list, k != nullptr, damping != nullptr, amp != nullptr, false);
}

StepConsts consts_for(const titan_sim *s, int64_t step, const float2 *trig)
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
    sc.trig = trig;
    sc.step = step;
    sc.dt64 = p.dt;
    sc.period = p.wave_period;
    sc.omega = p.omega;
    return sc;
}

// Buffers of the staged integrators, for the current number of masses.
int ensure_stage_buffers(titan_sim *s, bool rk4)
{
    if (s->stage_n != s->n) {
        for (float4 *&b : s->stage_buf) {
            if (b)
                dev_free(s, b);
            b = nullptr;
        }
        for (float4 *&b : s->verlet_acc) {
            if (b)
                dev_free(s, b);
            b = nullptr;
        }
        s->acc_valid = false;
        s->stage_n = s->n;
    }
    const size_t bytes = sizeof(float4) * std::max<int64_t>(s->n, 1);
    if (rk4) {
        for (float4 *&b : s->stage_buf)
            if (!b)
                if (int rc = dev_alloc(s, bytes, (void **)&b))
                    return rc;
    } else if (!s->verlet_acc[0]) {
        for (float4 *&b : s->verlet_acc)
            if (int rc = dev_alloc(s, bytes, (void **)&b))
                return rc;
        s->acc_valid = false;
    }
    return TITAN_OK;
}

// Velocity Verlet and RK4 (Sec. III-B): one gather launch per force
// evaluation (Verlet's drift is done by its kick launch), on the plain
// engines.
static int enqueue_staged(titan_sim *s, int64_t first_step, int64_t count)
{
    const bool rk4 = s->params.integrator == TITAN_INTEG_RK4;
    if (s->engine == TITAN_ENGINE_BATCHED && s->batch && s->batch_step)
        return enqueue_batch_integ(s, first_step, count);
    if (int rc = ensure_stage_buffers(s, rk4))
        return rc;
    const double dt = s->params.dt;
    // RK4's clock table holds half steps: entry 2q + j is t_(n0+q) + j dt/2
    const int chunk = rk4 ? kTrigChunk / 2 : kTrigChunk;
    for (int64_t c0 = 0; c0 < count; c0 += chunk) {
        const int nc = (int)std::min<int64_t>(chunk, count - c0);
        const int64_t n0 = first_step + c0;
        if (rk4)
            HIP_TRY(s, launch_trig_table(s->trig, 2 * n0, 2 * nc + 1, s->params.omega, 0.5 * dt, s->stream));
        else
            HIP_TRY(s, launch_trig_table(s->trig, n0, nc + 1, s->params.omega, dt, s->stream));
        for (int q = 0; q < nc; ++q) {
            const int64_t n = n0 + q;
            float4 *const U0 = s->U[s->cur], *const V0 = s->V[s->cur];
            float4 *const U1 = s->U[1 - s->cur], *const V1 = s->V[1 - s->cur];
            StateIO io{};
            io.first_bad = s->first_bad;
            if (rk4) {
                // stage s reads the previous stage's state; stages 1-3 write the
                // next one (into alternating buffers), stage 4 the new state
                io.U_base = U0;
                io.V_base = V0;
                io.sum_u = s->stage_buf[4];
                io.sum_v = s->stage_buf[5];
                const float4 *inU = U0, *inV = V0;
                for (int st = kStageRk1; st <= kStageRk4; ++st) {
                    float4 *oU = st == kStageRk4 ? U1 : s->stage_buf[(st & 1) ? 0 : 2];
                    float4 *oV = st == kStageRk4 ? V1 : s->stage_buf[(st & 1) ? 1 : 3];
                    io.U_in = inU;
                    io.V_in = inV;
                    io.U_out = oU;
                    io.V_out = oV;
                    const double c = st == kStageRk1 ? 0.0 : (st == kStageRk4 ? 1.0 : 0.5);
                    StepConsts sc = consts_for(s, n, s->trig + 2 * q + (int)(2 * c));
                    sc.t_add = c * dt;
                    sc.stage = st;
                    HIP_TRY(s, launch_gather_stage(s->gg, io, sc, s->tiled, s->stream));
                    inU = oU;
                    inV = oV;
                }
                s->cur = 1 - s->cur;
                continue;
            }
            // velocity Verlet: one launch drifts every mass it reads (from
            // its state and carried acceleration), kicks, and writes the new
            // state and acceleration into the other buffers
            if (!s->acc_valid) {
                io.U_in = U0;
                io.V_in = V0;
                io.A = s->verlet_acc[s->acc_cur];
                StepConsts sc = consts_for(s, n, s->trig + q);
                sc.stage = kStageVerletInit;
                HIP_TRY(s, launch_gather_stage(s->gg, io, sc, s->tiled, s->stream));
                s->acc_valid = true;
            }
            io.U_in = U0;
            io.V_in = V0;
            io.A_in = s->verlet_acc[s->acc_cur];
            io.U_base = U0;
            io.U_out = U1;
            io.V_out = V1;
            io.A = s->verlet_acc[1 - s->acc_cur];
            StepConsts sc = consts_for(s, n, s->trig + q + 1);
            sc.t_add = dt;
            sc.stage = kStageVerletKick;
            HIP_TRY(s, launch_gather_stage(s->gg, io, sc, s->tiled, s->stream));
            s->cur = 1 - s->cur;
            s->acc_cur = 1 - s->acc_cur;
        }
    }
    return TITAN_OK;
}

void destroy_step_graphs(titan_sim *s)
{
    bool any = false;
    for (hipGraphExec_t g : s->step_graph)
        any |= g != nullptr;
    if (any)
        (void)hipStreamSynchronize(s->stream);  // no replay in flight
    for (hipGraphExec_t &g : s->step_graph) {
        if (g)
            (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    if (s->capture_stream)
        (void)hipStreamDestroy(s->capture_stream);
    s->capture_stream = nullptr;
    (void)hipGetLastError();
}

void invalidate_step_cache(titan_sim *s)
{
    s->acc_valid = false;
    bool any = false;
    for (hipGraphExec_t g : s->step_graph)
        any |= g != nullptr;
    if (!any)
        return;
    (void)hipStreamSynchronize(s->stream);
    for (hipGraphExec_t &g : s->step_graph) {
        if (g)
            (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    (void)hipGetLastError();  // leave no error of this cleanup for the next launch check
}

// Capture graph_steps Euler step launches, for the current parity of cur: a
// clock-table node (first step = *d_clock), the steps (step index = *d_clock
// + q), and a node that advances the clock.  Captured on a stream of the
// sim's own (default priority); kernel nodes only.
static int capture_step_graph(titan_sim *s, hipGraphExec_t *out)
{
    const int G = s->params.graph_steps;
    if (!s->capture_stream)
        HIP_TRY(s, hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = s->capture_stream;
    HIP_TRY(s, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_trig_table_clock(s->trig, s->d_clock, G, s->params.omega, s->params.dt, cs);
    int c = s->cur;
    for (int q = 0; q < G && e == hipSuccess; ++q) {
        StateIO io{};
        io.U_in = s->U[c];
        io.V_in = s->V[c];
        io.U_out = s->U[1 - c];
        io.V_out = s->V[1 - c];
        io.first_bad = s->first_bad;
        StepConsts sc = consts_for(s, q, s->trig + q);
        sc.clock = s->d_clock;
        e = launch_gather_step(s->gg, io, sc, false, s->tiled, cs);
        c = 1 - c;
    }
    if (e == hipSuccess)
        e = launch_clock(s->d_clock, 0, G, cs);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess)
        e = e2;
    if (e == hipSuccess)
        e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    if (graph)
        (void)hipGraphDestroy(graph);
    if (e != hipSuccess)
        return hip_fail(s, e, "capturing the step loop");
    return TITAN_OK;
}

// reps replays of the captured step loop from step `first` (parity of cur
// unchanged: graph_steps is even).
static int replay_step_graph(titan_sim *s, int64_t first, int64_t reps)
{
    if (!s->d_clock) {  // lives as long as the sim (not a layout allocation)
        if (int rc = dev_alloc(s, sizeof(int64_t), (void **)&s->d_clock))
            return rc;
        s->clock_host = -1;
    }
    hipGraphExec_t &ex = s->step_graph[s->cur];
    if (!ex)
        if (int rc = capture_step_graph(s, &ex))
            return rc;
    if (s->clock_host != first)
        HIP_TRY(s, launch_clock(s->d_clock, first, 0, s->stream));
    for (int64_t r = 0; r < reps; ++r)
        HIP_TRY(s, hipGraphLaunch(ex, s->stream));
    s->clock_host = first + reps * s->params.graph_steps;
    return TITAN_OK;
}

int enqueue_steps(titan_sim *s, int64_t first_step, int64_t count)
{
    if (s->params.integrator != TITAN_INTEG_EULER)
        return enqueue_staged(s, first_step, count);
    if (s->engine == TITAN_ENGINE_BATCHED && s->batch && s->batch_step)
        return enqueue_batch_steps(s, first_step, count);
    const int G = s->params.graph_steps;
    if (G > 0 && count >= G) {
        const int64_t reps = count / G;
        if (int rc = replay_step_graph(s, first_step, reps))
            return rc;
        first_step += reps * G;
        count -= reps * G;
    }
    for (int64_t c0 = 0; c0 < count; c0 += kTrigChunk) {
        const int nc = (int)std::min<int64_t>(kTrigChunk, count - c0);
        HIP_TRY(s, launch_trig_table(s->trig, first_step + c0, nc, s->params.omega, s->params.dt, s->stream));
        for (int q = 0; q < nc; ++q) {
            StateIO io{};
            io.U_in = s->U[s->cur];
            io.V_in = s->V[s->cur];
            io.U_out = s->U[1 - s->cur];
            io.V_out = s->V[1 - s->cur];
            io.first_bad = s->first_bad;
            const StepConsts sc = consts_for(s, first_step + c0 + q, s->trig + q);
            HIP_TRY(s, launch_gather_step(s->gg, io, sc, false, s->tiled, s->stream));
            s->cur = 1 - s->cur;
        }
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
    // the clock entry of the current step sits after the chunk table
    HIP_TRY(s, launch_trig_table(s->trig + kTrigChunk, s->step_enq, 1, s->params.omega, s->params.dt, s->stream));
    const StepConsts sc = consts_for(s, s->step_enq, s->trig + kTrigChunk);
    HIP_TRY(s, launch_gather_step(s->gg, io, sc, true, s->tiled, s->stream));
    return TITAN_OK;
}

void destroy_engines(titan_sim *s) { destroy_batch_engine(s); }

// Springs added to a running system go into spare slots of the current
// layouts (Sec. III-C: arrays made larger than needed give O(1) insertion).
// A spring fits when both of its rows have a slot past their degree, the
// other end is reachable from each row (tiled layout: in the row's tile or
// its halo; batched layout: in the row's group), and its constants are
// representable by the arrays the layout has (a uniform stiffness or damping
// that it matches, actuation only where per-slot actuation exists, per-slot
// rest lengths).  The inserted spring is summed after the row's earlier
// springs; a later rebuild sorts it into place.
int insert_springs(titan_sim *s, int64_t first, int64_t count)
{
    GatherGraph &g = s->gg;
    const int64_t n = s->n;
    if (count <= 0)
        return TITAN_OK;
    if ((int64_t)s->h_deg.size() != n || (int64_t)s->h_slice_off.size() != g.n_slices + 1 || !g.d0)
        return 2;
    const bool act = g.act_c != nullptr, wave = g.t_off != nullptr;
    uint16_t *ngroup = batch_nbr_group(s);
    const bool grouped = ngroup != nullptr;
    if (grouped && s->h_group_off.size() < 2)
        return 2;
    auto group_of = [&](int64_t i) {
        return (int64_t)(std::upper_bound(s->h_group_off.begin(), s->h_group_off.end(), i) -
                         s->h_group_off.begin()) - 1;
    };
    // one new incidence: slot e of row r, whose other end is o
    struct Put {
        int64_t e, r, o, q;
        uint16_t local, group;
    };
    std::vector<Put> puts;
    std::unordered_map<int64_t, int32_t> extra;  // slots taken in this call, per row
    for (int64_t q = first; q < first + count; ++q) {
        if ((!g.k && s->h_k[q] != g.k_uniform) || (!g.c && s->h_damp[q] != g.c_uniform) ||
            (!act && actuated(s, q)))
            return 2;
        const int64_t i = s->inv_perm_of(s->h_ends[2 * q]), j = s->inv_perm_of(s->h_ends[2 * q + 1]);
        for (int side = 0; side < 2; ++side) {
            const int64_t r = side ? j : i, o = side ? i : j;
            const int64_t sl = r / kSlice;
            const int64_t width = (s->h_slice_off[sl + 1] - s->h_slice_off[sl]) / kSlice;
            const int64_t w = s->h_deg[r] + extra[r];
            if (w >= width)
                return 1;
            Put p{s->h_slice_off[sl] + (r % kSlice) + w * kSlice, r, o, q, 0, 0};
            if (s->tiled) {
                const int64_t t = r / kTile, a = t * kTile;
                if (o >= a && o < a + kTile) {
                    p.local = (uint16_t)(o - a);
                } else {
                    const int32_t *hb = s->h_halo_idx.data() + s->h_halo_off[t];
                    const int32_t *he = s->h_halo_idx.data() + s->h_halo_off[t + 1];
                    const int32_t *f = std::lower_bound(hb, he, (int32_t)o);
                    if (f == he || *f != (int32_t)o)
                        return 2;
                    p.local = (uint16_t)(kTile + (f - hb));
                }
            }
            if (grouped) {
                const int64_t gr = group_of(r);
                if (gr != group_of(o))
                    return 2;
                p.group = (uint16_t)(o - s->h_group_off[gr]);
            }
            ++extra[r];
            puts.push_back(p);
        }
    }

    // All fit: write the slots, one scatter per array, in stream order.
    const int64_t m = (int64_t)puts.size();
    for (const Put &p : puts)
        if (p.e < 0 || p.e >= s->n_slots || p.r < 0 || p.r >= n || p.o < 0 || p.o >= n)
            return fail(TITAN_EINVAL, "internal: inserted slot out of range");
    std::vector<int64_t> slot(m);
    for (int64_t e = 0; e < m; ++e)
        slot[e] = puts[e].e;
    int64_t *dslot = nullptr;
    void *dval = nullptr;
    if (int rc = dev_alloc(s, sizeof(int64_t) * m, (void **)&dslot))
        return rc;
    if (int rc = dev_alloc(s, sizeof(double) * m, &dval)) {
        dev_free(s, dslot);
        return rc;
    }
    std::vector<uint8_t> val(sizeof(double) * m);
    auto scatter = [&](const void *dst, int bytes, auto value_of) -> hipError_t {
        using V = decltype(value_of(puts[0]));
        static_assert(sizeof(V) == 2 || sizeof(V) == 4 || sizeof(V) == 8, "element size");
        (void)bytes;
        for (int64_t e = 0; e < m; ++e) {
            const V v = value_of(puts[e]);
            memcpy(val.data() + e * sizeof(V), &v, sizeof(V));
        }
        if (hipError_t err = hipMemcpyAsync(dval, val.data(), sizeof(V) * m, hipMemcpyHostToDevice, s->stream))
            return err;
        if (hipError_t err = launch_scatter_bits(const_cast<void *>(dst), sizeof(V), dslot, dval, m, s->stream))
            return err;
        return hipStreamSynchronize(s->stream);  // the staging is reused by the next array
    };
    std::vector<double> xmin;
    if (wave)
        xmin = body_xmin(s);
    hipError_t err = hipMemcpyAsync(dslot, slot.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s->stream);
    if (!err && g.nbr)
        err = scatter(g.nbr, 4, [](const Put &p) { return (int32_t)p.o; });
    if (!err && g.nbr_local)
        err = scatter(g.nbr_local, 2, [](const Put &p) { return p.local; });
    if (!err && grouped)
        err = scatter(ngroup, 2, [](const Put &p) { return p.group; });
    if (!err && g.k)
        err = scatter(g.k, 4, [&](const Put &p) { return s->h_k[p.q]; });
    if (!err && g.c)
        err = scatter(g.c, 4, [&](const Put &p) { return s->h_damp[p.q]; });
    if (!err && act && wave) {
        err = scatter(g.act_c, 4, [&](const Put &p) { return s->h_amp[p.q]; });
        if (!err)
            err = scatter(g.t_off, 8, [&](const Put &p) { return wave_offset(s, xmin, p.q); });
        // the offset tables do not know the new slots
        if (!err && grouped)
            batch_drop_wave_tables(s);
        if (!err && g.tile_wave_cls) {
            dev_free(s, const_cast<uint16_t *>(g.tile_wave_cls));
            dev_free(s, const_cast<int64_t *>(g.tile_wave_off));
            dev_free(s, const_cast<double *>(g.tile_wave_t));
            g.tile_wave_cls = nullptr;
            g.tile_wave_off = nullptr;
            g.tile_wave_t = nullptr;
            g.max_tile_wave = 0;
        }
    } else if (!err && act) {
        err = scatter(g.act_c, 4, [&](const Put &p) {
            float C, S;
            phasor_consts(s, p.q, C, S);
            return C;
        });
        if (!err)
            err = scatter(g.act_s, 4, [&](const Put &p) {
                float C, S;
                phasor_consts(s, p.q, C, S);
                return S;
            });
    }
    if (!err)
        err = scatter(g.d0, 4, [&](const Put &p) {
            float d0, L0;
            rest_consts(s, p.q, d0, L0);
            return d0;
        });
    if (!err)
        err = scatter(g.rest, 4, [&](const Put &p) {
            float d0, L0;
            rest_consts(s, p.q, d0, L0);
            return L0;
        });
    if (!err && g.yield)
        err = scatter(g.yield, 4, [&](const Put &p) { return s->h_yield[p.q]; });
    if (!err) {
        for (const Put &p : puts) {
            ++s->h_deg[p.r];
            if (p.o > p.r)
                s->h_owner_slot[p.q] = p.e;
            else
                s->h_other_slot[p.q] = p.e;
        }
        ++s->slot_gen;
        // the device copy of the row degrees: indexed by row, not by slot
        // (slot holds m >= the number of rows)
        for (int64_t e = 0; e < m; ++e)
            slot[e] = puts[e].r;
        err = hipMemcpyAsync(dslot, slot.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s->stream);
        if (!err)
            err = scatter(g.deg, 4, [&](const Put &p) { return s->h_deg[p.r]; });
    }
    dev_free(s, dslot);
    dev_free(s, dval);
    if (err != hipSuccess)
        return hip_fail(s, err, "inserting springs");
    s->springs_in_place += count;
    return TITAN_OK;
}

// Breaks recorded by the steps so far (in stream order) are copied into the
// host tables: a broken spring is marked broken and removed, so that a
// rebuilt layout leaves it out.
int sync_broken(titan_sim *s)
{
    if (!s->gg.yield || s->n_slots == 0)
        return TITAN_OK;
    std::vector<float> y(s->n_slots);
    HIP_TRY(s, hipMemcpyAsync(y.data(), s->gg.yield, sizeof(float) * s->n_slots, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    const int64_t ns = (int64_t)s->h_k.size();
    if (s->h_removed.empty())
        s->h_removed.assign(ns, 0);
    if (s->h_broken.empty())
        s->h_broken.assign(ns, 0);
    for (int64_t q = 0; q < ns && q < (int64_t)s->h_owner_slot.size(); ++q) {
        const int64_t e = s->h_owner_slot[q];
        if (e >= 0 && y[e] < 0.f && !s->h_broken[q]) {
            s->h_broken[q] = 1;
            s->h_removed[q] = 1;
        }
    }
    return TITAN_OK;
}

// New yield values of the listed springs (host table) written to both of
// their slots; springs that are removed or broken keep theirs.
int update_yield(titan_sim *s, const std::vector<int64_t> &springs)
{
    std::vector<int64_t> slot;
    std::vector<float> val;
    for (int64_t q : springs) {
        if (s->h_owner_slot[q] < 0 || (!s->h_removed.empty() && s->h_removed[q]))
            continue;
        slot.push_back(s->h_owner_slot[q]);
        slot.push_back(s->h_other_slot[q]);
        val.push_back(s->h_yield[q]);
        val.push_back(s->h_yield[q]);
    }
    const int64_t m = (int64_t)slot.size();
    if (m == 0)
        return TITAN_OK;
    int64_t *dslot = nullptr;
    float *dval = nullptr;
    if (int rc = dev_alloc(s, sizeof(int64_t) * m, (void **)&dslot))
        return rc;
    if (int rc = dev_alloc(s, sizeof(float) * m, (void **)&dval)) {
        dev_free(s, dslot);
        return rc;
    }
    hipError_t e = hipMemcpyAsync(dslot, slot.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s->stream);
    if (!e)
        e = hipMemcpyAsync(dval, val.data(), sizeof(float) * m, hipMemcpyHostToDevice, s->stream);
    if (!e)
        e = launch_scatter(s->gg.yield, dslot, dval, m, s->stream);
    if (!e)
        e = hipStreamSynchronize(s->stream);
    dev_free(s, dslot);
    dev_free(s, dval);
    return e == hipSuccess ? TITAN_OK : hip_fail(s, e, "updating yield values");
}

int rebuild_engines(titan_sim *s)
{
    if (int rc = sync_broken(s))
        return rc;
    invalidate_step_cache(s);
    destroy_batch_engine(s);
    dev_free_engine(s);
    s->gg = GatherGraph{};
    s->tiled = false;
    s->trig = nullptr;
    s->n_slots = 0;
    s->h_slot_nbr.clear();
    s->h_group_off.clear();
    if (int rc = build_engines(s))
        return rc;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    s->layout_dirty = false;
    return TITAN_OK;
}

}  // namespace titan

// Host side of the batched engine: groups of whole bodies, their LDS-resident
// stepping kernel, and the autotuner that picks the workgroup size -- and,
// under TITAN_ENGINE_AUTO, whether the batched or the tiled engine runs.
//
// Bodies are laid out contiguously, largest first (see plan_order), so the
// launch order of the groups is a longest-processing-time-first list schedule:
// the hardware hands the next group to whichever compute unit frees up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <utility>
#include <vector>

#include "titan_sim.h"

namespace titan {

#define HIP_TRY(sim, expr)                                  \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess)                               \
            return titan::hip_fail((sim), e_, #expr);       \
    } while (0)

struct BatchEngine {
    BatchLayout lay{};
    int threads = 256;
};

// Bodies are packed into a group until it would exceed the largest body (and
// at least this many masses): every group then uses most of the LDS sized for
// the largest, and groups are of similar cost.
constexpr int64_t kPackMin = 256;
// LDS holds three float4 per mass of a group (x0, u, v): at most 160 KB.
constexpr int64_t kMaxGroup = 160 * 1024 / (3 * 16);
// Steps timed per candidate by the tuner.
constexpr int kTuneSteps = 16;
// Largest group the tuner may form by packing more bodies per group.
constexpr int64_t kMaxPackTuned = 2048;

static bool threads_fit(int threads, int64_t max_group) { return (max_group + threads - 1) / threads <= 8; }

static int time_batch(titan_sim *s, const BatchEngine &be, int threads, float4 *su, float4 *sv, float *ms)
{
    StateIO io{};
    io.U_in = s->U[s->cur];
    io.V_in = s->V[s->cur];
    io.U_out = su;
    io.V_out = sv;
    io.first_bad = s->first_bad;
    const StepConsts sc = consts_for(s, 0, s->trig);
    hipEvent_t a, b;
    HIP_TRY(s, hipEventCreate(&a));
    HIP_TRY(s, hipEventCreate(&b));
    HIP_TRY(s, launch_batch(s->gg, be.lay, io, sc, 2, threads, s->stream));  // warm-up
    HIP_TRY(s, hipEventRecord(a, s->stream));
    HIP_TRY(s, launch_batch(s->gg, be.lay, io, sc, kTuneSteps, threads, s->stream));
    HIP_TRY(s, hipEventRecord(b, s->stream));
    HIP_TRY(s, hipEventSynchronize(b));
    HIP_TRY(s, hipEventElapsedTime(ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return TITAN_OK;
}

static int time_gather(titan_sim *s, float4 *su, float4 *sv, float *ms)
{
    StateIO io{};
    io.U_in = s->U[s->cur];
    io.V_in = s->V[s->cur];
    io.U_out = su;
    io.V_out = sv;
    io.first_bad = s->first_bad;
    hipEvent_t a, b;
    HIP_TRY(s, hipEventCreate(&a));
    HIP_TRY(s, hipEventCreate(&b));
    HIP_TRY(s, launch_gather_step(s->gg, io, consts_for(s, 0, s->trig), false, s->tiled, s->stream));
    HIP_TRY(s, hipEventRecord(a, s->stream));
    for (int q = 0; q < kTuneSteps; ++q)
        HIP_TRY(s, launch_gather_step(s->gg, io, consts_for(s, q, s->trig + q), false, s->tiled, s->stream));
    HIP_TRY(s, hipEventRecord(b, s->stream));
    HIP_TRY(s, hipEventSynchronize(b));
    HIP_TRY(s, hipEventElapsedTime(ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return TITAN_OK;
}

// Groups of whole bodies for a packing size: consecutive body runs of the
// internal order (largest first) are put in one group until the next would
// take it past `pack` masses.  Returns the group offsets and the largest group.
static void make_groups(const titan_sim *s, int64_t pack, std::vector<int64_t> &goff, int64_t &max_group)
{
    const int64_t n = s->n;
    goff.assign(1, 0);
    int64_t gsize = 0;
    max_group = 0;
    for (int64_t a = 0; a < n;) {
        const int32_t body = s->h_body[s->perm[a]];
        int64_t b = a + 1;
        while (b < n && s->h_body[s->perm[b]] == body)
            ++b;
        const int64_t r = b - a;
        if (gsize > 0 && gsize + r > pack) {
            goff.push_back(a);
            max_group = std::max(max_group, gsize);
            gsize = 0;
        }
        gsize += r;
        a = b;
    }
    goff.push_back(n);
    max_group = std::max(max_group, gsize);
}

// Wave law: each group's distinct spring offsets (bit patterns of the FP64
// t_o the slots hold, padding slots included) and every slot's index among
// them, so that the batched kernel evaluates the wave's sine once per
// distinct offset and step instead of once per slot (the same function of
// the same operands: the same bits).  Skipped when a group has more than
// kMaxWaveCls offsets or the table would not fit in LDS beside the state.
constexpr int64_t kMaxWaveCls = 1024;

static int upload_wave_tables(titan_sim *s, const std::vector<int64_t> &goff, const std::vector<int64_t> &hoff,
                              BatchEngine *be)
{
    const GatherGraph &g = s->gg;
    const int64_t ng = (int64_t)goff.size() - 1, slots = (int64_t)s->h_slot_nbr.size();
    if (!g.t_off || slots == 0)
        return TITAN_OK;
    std::vector<double> toff(slots);
    HIP_TRY(s, hipMemcpyAsync(toff.data(), g.t_off, sizeof(double) * slots, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    std::vector<uint16_t> cls(slots, 0);
    std::vector<int64_t> woff(1, 0);
    std::vector<double> wt;
    int64_t max_wave = 0;
    for (int64_t q = 0; q < ng; ++q) {
        std::vector<std::pair<uint64_t, int64_t>> keys;  // (bits, slot)
        for (int64_t i = goff[q]; i < goff[q + 1]; ++i) {
            const int64_t sl = i / kSlice, base = hoff[sl] + (i % kSlice);
            const int64_t width = (hoff[sl + 1] - hoff[sl]) / kSlice;
            for (int64_t w = 0; w < width; ++w) {
                uint64_t bits;
                memcpy(&bits, &toff[base + w * kSlice], 8);
                keys.push_back({bits, base + w * kSlice});
            }
        }
        std::sort(keys.begin(), keys.end());
        int64_t c = -1;
        for (size_t a = 0; a < keys.size(); ++a) {
            if (a == 0 || keys[a].first != keys[a - 1].first) {
                ++c;
                double v;
                memcpy(&v, &keys[a].first, 8);
                wt.push_back(v);
            }
            if (c >= kMaxWaveCls)
                return TITAN_OK;  // too many offsets: no tables
            cls[keys[a].second] = (uint16_t)c;
        }
        woff.push_back((int64_t)wt.size());
        max_wave = std::max(max_wave, c + 1);
    }
    if (be->lay.max_group * 3 * 16 + max_wave * 4 > 160 * 1024)
        return TITAN_OK;
    // the tables are an optimisation: without the memory for them every slot
    // evaluates its own offset
    uint16_t *dc = nullptr;
    int64_t *doff = nullptr;
    double *dt = nullptr;
    if (dev_alloc(s, sizeof(uint16_t) * slots, (void **)&dc) != TITAN_OK ||
        dev_alloc(s, sizeof(int64_t) * woff.size(), (void **)&doff) != TITAN_OK ||
        dev_alloc(s, sizeof(double) * std::max<size_t>(wt.size(), 1), (void **)&dt) != TITAN_OK) {
        dev_free(s, dc);
        dev_free(s, doff);
        dev_free(s, dt);
        return TITAN_OK;
    }
    HIP_TRY(s, hipMemcpyAsync(dc, cls.data(), sizeof(uint16_t) * slots, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipMemcpyAsync(doff, woff.data(), sizeof(int64_t) * woff.size(), hipMemcpyHostToDevice, s->stream));
    if (!wt.empty())
        HIP_TRY(s, hipMemcpyAsync(dt, wt.data(), sizeof(double) * wt.size(), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    be->lay.wave_cls = dc;
    be->lay.wave_off = doff;
    be->lay.wave_t = dt;
    be->lay.max_wave = (int32_t)max_wave;
    return TITAN_OK;
}

static void free_wave_tables(titan_sim *s, BatchEngine *be)
{
    dev_free(s, const_cast<uint16_t *>(be->lay.wave_cls));
    dev_free(s, const_cast<int64_t *>(be->lay.wave_off));
    dev_free(s, const_cast<double *>(be->lay.wave_t));
    be->lay.wave_cls = nullptr;
    be->lay.wave_off = nullptr;
    be->lay.wave_t = nullptr;
    be->lay.max_wave = 0;
}

// The batched layout of the groups `goff` on the device: group offsets and
// each slot's neighbour relative to its group's first mass.
static int upload_groups(titan_sim *s, const std::vector<int64_t> &goff, int64_t max_group,
                         const std::vector<int64_t> &hoff, BatchEngine *be)
{
    const int64_t ng = (int64_t)goff.size() - 1;
    const int64_t slots = (int64_t)s->h_slot_nbr.size();
    std::vector<uint16_t> nbr_group(slots, 0);
    for (int64_t q = 0; q < ng; ++q)
        for (int64_t i = goff[q]; i < goff[q + 1]; ++i) {
            const int64_t sl = i / kSlice, base = hoff[sl] + (i % kSlice);
            const int64_t width = (hoff[sl + 1] - hoff[sl]) / kSlice;
            for (int64_t w = 0; w < width; ++w) {
                const int64_t j = s->h_slot_nbr[base + w * kSlice];
                if (j < goff[q] || j >= goff[q + 1])
                    return fail(TITAN_EINVAL, "internal: a spring leaves its body group");
                nbr_group[base + w * kSlice] = (uint16_t)(j - goff[q]);
            }
        }
    be->lay.n_groups = ng;
    be->lay.max_group = (int32_t)max_group;
    int64_t *d = nullptr;
    if (int rc = dev_alloc(s, sizeof(int64_t) * goff.size(), (void **)&d))
        return rc;
    HIP_TRY(s, hipMemcpyAsync(d, goff.data(), sizeof(int64_t) * goff.size(), hipMemcpyHostToDevice, s->stream));
    be->lay.mass_off = d;
    uint16_t *e = nullptr;
    if (int rc = dev_alloc(s, sizeof(uint16_t) * std::max<int64_t>(slots, 1), (void **)&e))
        return rc;
    if (slots)
        HIP_TRY(s, hipMemcpyAsync(e, nbr_group.data(), sizeof(uint16_t) * slots, hipMemcpyHostToDevice, s->stream));
    be->lay.nbr_group = e;
    // the host table goes away with this call
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return upload_wave_tables(s, goff, hoff, be);
}

static void free_groups(titan_sim *s, BatchEngine *be)
{
    if (!be)
        return;
    dev_free(s, const_cast<int64_t *>(be->lay.mass_off));
    dev_free(s, const_cast<uint16_t *>(be->lay.nbr_group));
    free_wave_tables(s, be);
    delete be;
}

int build_batch_engine(titan_sim *s, bool may_step)
{
    s->batch = nullptr;
    s->batch_step = false;
    const int64_t n = s->n;
    if (n == 0 || (s->h_slot_nbr.empty() && s->ns > 0))
        return TITAN_OK;

    // Packing: bodies go into groups of up to `pack` masses, at least the
    // largest body (the first body run of the internal order is a largest
    // one) and at least kPackMin.
    int64_t pack = kPackMin;
    {
        int64_t b = 1;
        while (b < n && s->h_body[s->perm[b]] == s->h_body[s->perm[0]])
            ++b;
        pack = std::max<int64_t>(pack, b);
    }
    std::vector<int64_t> goff;
    int64_t max_group = 0;
    make_groups(s, pack, goff, max_group);
    if (max_group > kMaxGroup)
        return TITAN_OK;  // a body too large for LDS: not eligible
    std::vector<int64_t> hoff(s->gg.n_slices + 1);
    HIP_TRY(s, hipMemcpy(hoff.data(), s->gg.slice_off, sizeof(int64_t) * hoff.size(), hipMemcpyDeviceToHost));
    BatchEngine *be = new (std::nothrow) BatchEngine();
    if (!be)
        return fail(TITAN_ENOMEM, "out of host memory");
    if (int rc = upload_groups(s, goff, max_group, hoff, be)) {
        free_groups(s, be);
        return rc;
    }
    s->h_group_off = goff;

    if (!may_step) {
        s->batch = be;
        return TITAN_OK;
    }

    // Autotune: workgroup size of the batched kernel, and (AUTO) batched vs
    // the per-step gather engine, by timing kTuneSteps steps of each into
    // scratch buffers (the simulation state is not touched; breaks of
    // breakable springs are recorded in a copy of their yield values).
    struct YieldCopy {
        titan_sim *s;
        float *keep = nullptr, *tmp = nullptr;
        ~YieldCopy()
        {
            if (tmp) {
                (void)hipStreamSynchronize(s->stream);
                s->gg.yield = keep;
                dev_free(s, tmp);
            }
        }
    } ycopy{s};
    if (s->gg.yield && s->n_slots > 0) {
        if (int rc = dev_alloc(s, sizeof(float) * s->n_slots, (void **)&ycopy.tmp)) {
            free_groups(s, be);
            return rc;
        }
        ycopy.keep = s->gg.yield;
        HIP_TRY(s, hipMemcpyAsync(ycopy.tmp, ycopy.keep, sizeof(float) * s->n_slots, hipMemcpyDeviceToDevice,
                                  s->stream));
        s->gg.yield = ycopy.tmp;
    }
    float4 *su = nullptr, *sv = nullptr;
    if (int rc = dev_alloc(s, sizeof(float4) * n, (void **)&su)) {
        free_groups(s, be);
        return rc;
    }
    if (int rc = dev_alloc(s, sizeof(float4) * n, (void **)&sv)) {
        free_groups(s, be);
        return rc;
    }
    HIP_TRY(s, launch_trig_table(s->trig, 0, kTuneSteps, s->params.omega, s->params.dt, s->stream));
    // Candidates: the base packing, then groups of two and four times as many
    // masses while the largest group stays within kMaxPackTuned masses (the
    // adjoint and the batched RK4 take groups of up to 2048), each with every
    // workgroup size that fits.
    std::vector<int64_t> packs{pack};
    for (int64_t f = 2; f <= 4; f *= 2)
        if (pack * f <= kMaxPackTuned)
            packs.push_back(pack * f);
    float best = 1e30f;
    int best_t = 0;
    BatchEngine *best_be = nullptr;
    std::vector<int64_t> best_goff;
    int64_t prev_groups = -1;
    for (int64_t p : packs) {
        BatchEngine *cand = nullptr;
        std::vector<int64_t> cg;
        int64_t cmax = 0;
        if (p == pack) {
            cand = be;
            cg = goff;
            cmax = max_group;
        } else {
            make_groups(s, p, cg, cmax);
            if (cmax > kMaxPackTuned || (int64_t)cg.size() - 1 == prev_groups)
                continue;  // too large, or the same groups as the last candidate
            cand = new (std::nothrow) BatchEngine();
            if (!cand) {
                free_groups(s, best_be != be ? best_be : nullptr);
                free_groups(s, be);
                return fail(TITAN_ENOMEM, "out of host memory");
            }
            if (int rc = upload_groups(s, cg, cmax, hoff, cand)) {
                free_groups(s, cand);
                free_groups(s, best_be != be ? best_be : nullptr);
                free_groups(s, be);
                return rc;
            }
        }
        prev_groups = (int64_t)cg.size() - 1;
        bool won = false;
        for (int t : kBatchThreadChoices) {
            if (!threads_fit(t, cmax))
                continue;
            float ms = 0.f;
            if (int rc = time_batch(s, *cand, t, su, sv, &ms)) {
                if (cand != be)
                    free_groups(s, cand);
                free_groups(s, best_be != be ? best_be : nullptr);
                free_groups(s, be);
                return rc;
            }
            if (ms < best) {
                best = ms;
                best_t = t;
                won = true;
            }
        }
        if (won) {
            if (best_be && best_be != be && best_be != cand)
                free_groups(s, best_be);
            best_be = cand;
            best_goff = cg;
        } else if (cand != be) {
            free_groups(s, cand);
        }
    }
    if (best_t == 0) {
        free_groups(s, be);
        return TITAN_OK;
    }
    if (best_be != be) {
        free_groups(s, be);
        be = best_be;
        s->h_group_off = best_goff;
    }
    be->threads = best_t;
    s->tune_batch_ms = best / kTuneSteps;
    bool use = true;
    if (s->params.engine == TITAN_ENGINE_AUTO) {
        float gms = 0.f;
        if (int rc = time_gather(s, su, sv, &gms)) {
            free_groups(s, be);
            return rc;
        }
        s->tune_gather_ms = gms / kTuneSteps;
        use = best < gms;
    }
    dev_free(s, su);
    dev_free(s, sv);
    // the timing runs may have flagged their own non-finite steps: forget them
    const unsigned long long none = ~0ull;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    HIP_TRY(s, hipMemcpy(s->first_bad, &none, sizeof none, hipMemcpyHostToDevice));
    // The layout is kept whenever the system fits it: the adjoint runs on it
    // even when the per-step gather engine steps the system.
    s->batch = be;
    s->batch_step = use;
    return TITAN_OK;
}

int enqueue_batch_steps(titan_sim *s, int64_t first_step, int64_t count)
{
    BatchEngine *be = s->batch;
    for (int64_t c0 = 0; c0 < count; c0 += kTrigChunk) {
        const int nc = (int)std::min<int64_t>(kTrigChunk, count - c0);
        HIP_TRY(s, launch_trig_table(s->trig, first_step + c0, nc, s->params.omega, s->params.dt, s->stream));
        StateIO io{};
        io.U_in = s->U[s->cur];
        io.V_in = s->V[s->cur];
        io.U_out = s->U[1 - s->cur];
        io.V_out = s->V[1 - s->cur];
        io.first_bad = s->first_bad;
        const StepConsts sc = consts_for(s, first_step + c0, s->trig);
        HIP_TRY(s, launch_batch(s->gg, be->lay, io, sc, nc, be->threads, s->stream));
        s->cur = 1 - s->cur;
    }
    return TITAN_OK;
}

const BatchLayout &batch_layout(const titan_sim *s) { return s->batch->lay; }

// Velocity Verlet / RK4 on the batched layout: chunks of steps per launch,
// the clock tables as the per-step engines build them (RK4: half steps).
int enqueue_batch_integ(titan_sim *s, int64_t first_step, int64_t count)
{
    BatchEngine *be = s->batch;
    const int integ = s->params.integrator;
    const bool rk4 = integ == TITAN_INTEG_RK4;
    if (int rc = ensure_stage_buffers(s, false))  // Verlet's acceleration buffers
        return rc;
    const double dt = s->params.dt;
    const int chunk = rk4 ? kTrigChunk / 2 : kTrigChunk;
    for (int64_t c0 = 0; c0 < count; c0 += chunk) {
        const int nc = (int)std::min<int64_t>(chunk, count - c0);
        const int64_t n0 = first_step + c0;
        if (rk4)
            HIP_TRY(s, launch_trig_table(s->trig, 2 * n0, 2 * nc + 1, s->params.omega, 0.5 * dt, s->stream));
        else
            HIP_TRY(s, launch_trig_table(s->trig, n0, nc + 1, s->params.omega, dt, s->stream));
        StateIO io{};
        io.U_in = s->U[s->cur];
        io.V_in = s->V[s->cur];
        io.U_out = s->U[1 - s->cur];
        io.V_out = s->V[1 - s->cur];
        io.first_bad = s->first_bad;
        io.A_in = s->verlet_acc[s->acc_cur];
        io.A = s->verlet_acc[s->acc_cur];  // each mass's entry: read at the start, written at the end
        const StepConsts sc = consts_for(s, n0, s->trig);
        HIP_TRY(s, launch_batch_integ(s->gg, be->lay, io, sc, nc, integ, s->acc_valid ? 1 : 0, s->stream));
        if (!rk4)
            s->acc_valid = true;
        s->cur = 1 - s->cur;
    }
    return TITAN_OK;
}

void batch_drop_wave_tables(titan_sim *s)
{
    if (s->batch && s->batch->lay.wave_cls) {
        (void)hipStreamSynchronize(s->stream);  // launches in flight may still read them
        free_wave_tables(s, s->batch);
    }
}

uint16_t *batch_nbr_group(titan_sim *s)
{
    return s->batch ? const_cast<uint16_t *>(s->batch->lay.nbr_group) : nullptr;
}

void destroy_batch_engine(titan_sim *s)
{
    delete s->batch;
    s->batch = nullptr;
}

// LDS of one workgroup (gfx950: 160 KB).
constexpr int64_t kLdsBytes = 160 * 1024;

// The spring-once tables of the current layout, built when the slots or the
// groups changed since the last call: each group's springs (owner mass, then
// owner slot, ascending), their ends and owner slots, and per slot the
// reverse sums' entries (see AdjointIO).
static int once_tables(titan_sim *s)
{
    SpringOnceTables &o = s->once;
    const std::vector<int64_t> &goff = s->h_group_off;
    if (o.gen == s->slot_gen && o.goff == goff)
        return TITAN_OK;
    for (void *p : {(void *)o.ends, (void *)o.slot, (void *)o.off, (void *)o.rev_sp, (void *)o.of_spring})
        if (p)
            dev_free(s, p);
    o = SpringOnceTables{};
    const int64_t n = s->n, ns = s->ns;
    const std::vector<int64_t> &off = s->h_slice_off;
    const int64_t ng = (int64_t)goff.size() - 1;
    o.gen = s->slot_gen;
    o.goff = goff;
    if (ng < 1 || (int64_t)off.size() != s->gg.n_slices + 1 || (int64_t)s->h_owner_slot.size() < ns)
        return TITAN_OK;  // no usable layout: the per-slot path
    const int64_t nslots = off.back();
    std::vector<int32_t> group(n);
    for (int64_t q = 0; q < ng; ++q)
        for (int64_t i = goff[q]; i < goff[q + 1]; ++i)
            group[i] = (int32_t)q;
    // (owner mass, owner slot, other mass, caller spring) per group
    struct Rec {
        int64_t io, eo, ix, q;
    };
    std::vector<std::vector<Rec>> per(ng);
    for (int64_t q = 0; q < ns; ++q) {
        const int64_t eo = s->h_owner_slot[q];
        if (eo < 0 || s->h_other_slot[q] < 0)
            continue;
        const int64_t a = s->inv_perm_of(s->h_ends[2 * q]), b = s->inv_perm_of(s->h_ends[2 * q + 1]);
        const int64_t io = std::min(a, b), ix = std::max(a, b);
        if (group[io] != group[ix])
            return fail(TITAN_EINVAL, "internal: a spring leaves its body group");
        per[group[io]].push_back({io, eo, ix, q});
    }
    std::vector<int64_t> sp_off(ng + 1, 0);
    int sp_max = 0;
    for (int64_t g = 0; g < ng; ++g) {
        std::sort(per[g].begin(), per[g].end(),
                  [](const Rec &x, const Rec &y) { return x.io != y.io ? x.io < y.io : x.eo < y.eo; });
        sp_off[g + 1] = sp_off[g] + (int64_t)per[g].size();
        sp_max = std::max<int>(sp_max, (int)per[g].size());
    }
    const int64_t nsp = sp_off[ng];
    if (nsp == 0)
        return TITAN_OK;
    std::vector<uint32_t> ends(nsp);
    std::vector<int64_t> slot(nsp), of(ns, -1);
    std::vector<int32_t> rev_sp(nslots, INT32_MAX);
    // each mass's entries: springs are in owner order, so a mass's entries
    // as owner come in ascending order; merged with its other-end entries
    std::vector<std::vector<int32_t>> ent;
    for (int64_t g = 0; g < ng; ++g) {
        const int64_t m = goff[g + 1] - goff[g];
        ent.assign(m, {});
        for (int64_t t = 0; t < (int64_t)per[g].size(); ++t) {
            const Rec &r = per[g][t];
            const int64_t u = sp_off[g] + t;
            ends[u] = (uint32_t)(r.io - goff[g]) | ((uint32_t)(r.ix - goff[g]) << 16);
            slot[u] = r.eo;
            of[r.q] = u;
            ent[r.io - goff[g]].push_back((int32_t)(2 * t));
            ent[r.ix - goff[g]].push_back((int32_t)(2 * t + 1));
        }
        for (int64_t i = goff[g]; i < goff[g + 1]; ++i) {
            std::vector<int32_t> &v = ent[i - goff[g]];
            std::sort(v.begin(), v.end());
            const int64_t sl = i / kSlice, base = off[sl] + (i % kSlice), width = (off[sl + 1] - off[sl]) / kSlice;
            if ((int64_t)v.size() > width)
                return fail(TITAN_EINVAL, "internal: a mass has more springs than slots");
            for (size_t w = 0; w < v.size(); ++w)
                rev_sp[base + (int64_t)w * kSlice] = v[w];
        }
    }
    int rc = TITAN_OK;
    if ((rc = dev_alloc(s, sizeof(uint32_t) * nsp, (void **)&o.ends)) ||
        (rc = dev_alloc(s, sizeof(int64_t) * nsp, (void **)&o.slot)) ||
        (rc = dev_alloc(s, sizeof(int64_t) * (ng + 1), (void **)&o.off)) ||
        (rc = dev_alloc(s, sizeof(int32_t) * std::max<int64_t>(nslots, 1), (void **)&o.rev_sp)) ||
        (rc = dev_alloc(s, sizeof(int64_t) * std::max<int64_t>(ns, 1), (void **)&o.of_spring))) {
        o.gen = 0;  // built again next time
        return rc;
    }
    HIP_TRY(s, hipMemcpyAsync(o.ends, ends.data(), sizeof(uint32_t) * nsp, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipMemcpyAsync(o.slot, slot.data(), sizeof(int64_t) * nsp, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipMemcpyAsync(o.off, sp_off.data(), sizeof(int64_t) * (ng + 1), hipMemcpyHostToDevice, s->stream));
    if (nslots)
        HIP_TRY(s, hipMemcpyAsync(o.rev_sp, rev_sp.data(), sizeof(int32_t) * nslots, hipMemcpyHostToDevice,
                                  s->stream));
    if (ns)
        HIP_TRY(s, hipMemcpyAsync(o.of_spring, of.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice, s->stream));
    // the host tables go away with this call
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    o.nsp = nsp;
    o.sp_max = sp_max;
    return TITAN_OK;
}

// Adjoint rollout on the batched layout (see adjoint_step.hip).
int rollout_grad(titan_sim *s, int64_t nsteps, int32_t K, const float *body_weights, float *loss, float *gk,
                 float *gC, float *gS, float *gvox_a, float *gvox_phi, bool dev_out)
{
    const bool voxels = gvox_a || gvox_phi;
    const int64_t nv = (int64_t)s->h_vox_a.size();
    if (voxels && s->h_vs_ptr.empty())
        return fail(TITAN_ESTATE, "no voxel actuation (titan_set_voxel_actuation)");
    if (!s->batch)
        return fail(TITAN_ESTATE, "the rollout gradient needs every body to fit one workgroup's LDS");
    if (nsteps < 0 || K < 1)
        return fail(TITAN_EINVAL, "need nsteps >= 0 and checkpoint interval >= 1");
    if (nsteps > (int64_t)1 << 30)
        return fail(TITAN_EINVAL, "nsteps too large");
    if (s->paused && s->steps_req != s->step_enq)
        return fail(TITAN_ESTATE, "steps are held at a pause breakpoint");
    if (s->batch->lay.max_group > 8 * 256)
        return fail(TITAN_ESTATE, "the rollout gradient supports groups of at most 2048 masses");
    const int64_t n = s->n, ns = s->ns;
    if (nsteps == 0) {
        int32_t nb = 0;
        for (int32_t b : s->h_body)
            nb = std::max(nb, b + 1);
        if (dev_out) {
            const std::pair<float *, int64_t> outs[4] = {{loss, nb}, {gk, ns}, {gC, ns}, {gS, ns}};
            for (const auto &o : outs)
                if (o.first && o.second)
                    HIP_TRY(s, hipMemsetAsync(o.first, 0, sizeof(float) * o.second, s->stream));
            HIP_TRY(s, hipStreamSynchronize(s->stream));
            return TITAN_OK;
        }
        if (loss)
            std::fill(loss, loss + nb, 0.f);
        for (float *g : {gk, gC, gS})
            if (g)
                std::fill(g, g + ns, 0.f);
        for (float *g : {gvox_a, gvox_phi})
            if (g)
                std::fill(g, g + nv, 0.f);
        return TITAN_OK;
    }
    K = (int32_t)std::min<int64_t>(K, std::max<int64_t>(nsteps, 1));
    const int64_t nseg = (nsteps + K - 1) / K;

    // Bodies: contiguous internal ranges (plan_order), in rank order.
    int32_t nb = 0;
    for (int32_t b : s->h_body)
        nb = std::max(nb, b + 1);
    std::vector<int64_t> body_off{0};
    std::vector<int32_t> rank_body;
    for (int64_t a = 0; a < n;) {
        const int32_t bd = s->h_body[s->perm[a]];
        int64_t b = a + 1;
        while (b < n && s->h_body[s->perm[b]] == bd)
            ++b;
        rank_body.push_back(bd);
        body_off.push_back(b);
        a = b;
    }
    const int64_t nruns = (int64_t)rank_body.size();
    std::vector<double> mtot(nb, 0.0);
    for (int64_t u = 0; u < n; ++u)
        mtot[s->h_body[u]] += (double)s->h_mass[u];
    std::vector<float> coef(n), seed(n);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t u = s->perm[i];
        const int32_t bd = s->h_body[u];
        const double c = mtot[bd] > 0.0 ? (double)s->h_mass[u] / mtot[bd] : 0.0;
        coef[i] = (float)c;
        seed[i] = (float)(-(body_weights ? (double)body_weights[bd] : 1.0) * c);
    }

    // Buffers (released at the end of the call).
    std::vector<void *> tmp;
    auto get = [&](size_t bytes, void **p) {
        const int rc = dev_alloc(s, bytes, p);
        if (rc == TITAN_OK)
            tmp.push_back(*p);
        return rc;
    };
    auto cleanup = [&]() {
        for (void *p : tmp)
            dev_free(s, p);
    };
    AdjointIO a{};
    float *dseed = nullptr, *dcoef = nullptr, *dloss = nullptr, *dgrad = nullptr;
    int64_t *dboff = nullptr;
    float2 *dtrig = nullptr;
    unsigned long long *dbad = nullptr;
    int64_t nslots = 0;
    {
        std::vector<int64_t> last(1);
        HIP_TRY(s, hipMemcpy(last.data(), s->gg.slice_off + s->gg.n_slices, sizeof(int64_t), hipMemcpyDeviceToHost));
        nslots = last[0];
    }
    // the reverse steps evaluate every spring once when the groups allow it
    // (the environment variable TITAN_ADJOINT_SPRING_ONCE=0 selects the
    // per-slot path)
    const char *once_env = std::getenv("TITAN_ADJOINT_SPRING_ONCE");
    const bool want_once = !(once_env && once_env[0] == '0');
    // (groups of at most 1024 masses, with room for at least 64 records)
    const int64_t avail = kLdsBytes - 4 * 16 * (int64_t)s->batch->lay.max_group;
    const bool eligible = want_once && s->batch->lay.max_group <= 1024 && avail / 24 >= 64;
    int rc = TITAN_OK;
    if (eligible && (rc = once_tables(s)))
        return rc;
    const SpringOnceTables &o = s->once;
    const bool once = eligible && o.nsp > 0;
    const bool rest = s->gg.d0 != nullptr;
    float4 *kcs = nullptr;
    float2 *rst = nullptr;
    if (once) {
        a.rev_chunk = (int)std::min<int64_t>(o.sp_max, avail / 24);
        a.once_bytes = 24 * a.rev_chunk;
        if ((rc = get(sizeof(float4) * o.nsp, (void **)&a.gsp)) || (rc = get(sizeof(float4) * o.nsp, (void **)&kcs)) ||
            (rest && (rc = get(sizeof(float2) * o.nsp, (void **)&rst)))) {
            cleanup();
            return rc;
        }
        a.sp_ends = o.ends;
        a.sp_kcs = kcs;
        a.sp_rest = rst;
        a.sp_off = o.off;
        a.rev_sp = o.rev_sp;
    }
    if ((rc = get(sizeof(float4) * n * std::max<int64_t>(nseg, 1), (void **)&a.ckU)) ||
        (rc = get(sizeof(float4) * n * std::max<int64_t>(nseg, 1), (void **)&a.ckV)) ||
        (rc = get(sizeof(float4) * n * K, (void **)&a.segU)) || (rc = get(sizeof(float4) * n * K, (void **)&a.segV)) ||
        (rc = get(sizeof(float4) * n * K, (void **)&a.segF)) ||
        (rc = get(sizeof(float4) * (once ? 1 : std::max<int64_t>(nslots, 1)), (void **)&a.gslot)) ||
        (rc = get(sizeof(float) * n, (void **)&dseed)) || (rc = get(sizeof(float) * n, (void **)&dcoef)) ||
        (rc = get(sizeof(float) * n, (void **)&a.dux)) || (rc = get(sizeof(float) * nruns, (void **)&dloss)) ||
        (rc = get(sizeof(float) * 3 * ns, (void **)&dgrad)) || (rc = get(sizeof(int64_t) * (nruns + 1), (void **)&dboff)) ||
        (rc = get(sizeof(float2) * std::max<int64_t>(nsteps, 1), (void **)&dtrig)) ||
        (rc = get(sizeof(unsigned long long), (void **)&dbad))) {
        cleanup();
        return rc;
    }
    const unsigned long long none = ~0ull;
#define TRY(expr)                                              \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) {                                \
            cleanup();                                         \
            return titan::hip_fail(s, e_, #expr);              \
        }                                                      \
    } while (0)
    TRY(hipMemcpyAsync(dseed, seed.data(), sizeof(float) * n, hipMemcpyHostToDevice, s->stream));
    TRY(hipMemcpyAsync(dcoef, coef.data(), sizeof(float) * n, hipMemcpyHostToDevice, s->stream));
    TRY(hipMemcpyAsync(dboff, body_off.data(), sizeof(int64_t) * (nruns + 1), hipMemcpyHostToDevice, s->stream));
    // the owner slots stay on the device between calls (sent again only
    // after the layout or the spring set changed)
    if (!once && (s->d_owner_gen != s->slot_gen || s->d_owner_cap < ns)) {
        if (s->d_owner_cap < ns) {
            if (s->d_owner_slot)
                dev_free(s, s->d_owner_slot);
            s->d_owner_slot = nullptr;
            s->d_owner_cap = 0;
            if ((rc = dev_alloc(s, sizeof(int64_t) * std::max<int64_t>(ns, 1), (void **)&s->d_owner_slot))) {
                cleanup();
                return rc;
            }
            s->d_owner_cap = ns;
        }
        if (ns)
            TRY(hipMemcpyAsync(s->d_owner_slot, s->h_owner_slot.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice,
                               s->stream));
        s->d_owner_gen = s->slot_gen;
    }
    TRY(hipMemcpyAsync(dbad, &none, sizeof none, hipMemcpyHostToDevice, s->stream));
    if (once) {
        TRY(hipMemsetAsync(a.gsp, 0, sizeof(float4) * o.nsp, s->stream));
        TRY(launch_pack_spring_consts(s->gg, s->batch->lay, o.slot, o.off, kcs, rst, s->stream));
    } else {
        TRY(hipMemsetAsync(a.gslot, 0, sizeof(float4) * std::max<int64_t>(nslots, 1), s->stream));
    }
    TRY(launch_trig_table(dtrig, s->step_enq, (int)nsteps, s->params.omega, s->params.dt, s->stream));
    a.U0 = s->U[s->cur];
    a.V0 = s->V[s->cur];
    a.seed = dseed;
    a.trig = dtrig;
    a.first_bad = dbad;
    a.nsteps = (int)nsteps;
    a.K = K;
    const StepConsts sc = consts_for(s, s->step_enq, dtrig);
    TRY(launch_adjoint(s->gg, s->batch->lay, a, sc, s->stream));
    if (once)
        TRY(launch_spring_grads(a.gsp, o.of_spring, ns, dgrad, dgrad + ns, dgrad + 2 * ns, s->stream));
    else
        TRY(launch_spring_grads(a.gslot, s->d_owner_slot, ns, dgrad, dgrad + ns, dgrad + 2 * ns, s->stream));
    TRY(launch_body_loss(a.dux, dcoef, dboff, nruns, dloss, s->stream));
    // per-voxel gradients through the mean-phasor map, on the device: each
    // voxel sums over its springs (ascending) the spring's (dJ/dC, dJ/dS)
    // divided by the spring's voxel count, turned by the voxel's phase
    float *dvox = nullptr;
    if (voxels && nv > 0) {
        int64_t *dvptr = nullptr;
        int32_t *dvspring = nullptr;
        float *dinv = nullptr;
        float4 *dvw = nullptr;
        const int64_t nidx = (int64_t)s->h_vs_spring.size();
        std::vector<float> inv(ns, 0.f);
        for (int64_t q = 0; q < ns; ++q)
            if (q < (int64_t)s->h_sv_count.size() && s->h_sv_count[q] > 0)
                inv[q] = (float)(1.0 / (double)s->h_sv_count[q]);
        std::vector<float4> vw(nv);
        for (int64_t v = 0; v < nv; ++v) {
            const double ph = s->h_vox_phi[v];
            vw[v] = make_float4((float)std::cos(ph), (float)std::sin(ph), s->h_vox_a[v], 0.f);
        }
        if ((rc = get(sizeof(int64_t) * (nv + 1), (void **)&dvptr)) ||
            (rc = get(sizeof(int32_t) * std::max<int64_t>(nidx, 1), (void **)&dvspring)) ||
            (rc = get(sizeof(float) * std::max<int64_t>(ns, 1), (void **)&dinv)) ||
            (rc = get(sizeof(float4) * nv, (void **)&dvw)) || (rc = get(sizeof(float) * 2 * nv, (void **)&dvox))) {
            cleanup();
            return rc;
        }
        TRY(hipMemcpyAsync(dvptr, s->h_vs_ptr.data(), sizeof(int64_t) * (nv + 1), hipMemcpyHostToDevice, s->stream));
        if (nidx)
            TRY(hipMemcpyAsync(dvspring, s->h_vs_spring.data(), sizeof(int32_t) * nidx, hipMemcpyHostToDevice,
                               s->stream));
        if (ns)
            TRY(hipMemcpyAsync(dinv, inv.data(), sizeof(float) * ns, hipMemcpyHostToDevice, s->stream));
        TRY(hipMemcpyAsync(dvw, vw.data(), sizeof(float4) * nv, hipMemcpyHostToDevice, s->stream));
        TRY(launch_voxel_grads(nv, dvptr, dvspring, dinv, dvw, dgrad + ns, dgrad + 2 * ns, dvox, dvox + nv,
                               s->stream));
    }
    // the non-finite check first: on failure the caller's arrays are left
    // as they were; then the results straight into them
    unsigned long long bad = ~0ull;
    TRY(hipMemcpyAsync(&bad, dbad, sizeof bad, hipMemcpyDeviceToHost, s->stream));
    TRY(hipStreamSynchronize(s->stream));
    if (bad != ~0ull) {
        cleanup();
        return fail(TITAN_ENONFINITE, "the rollout produced a non-finite state at step %llu", bad);
    }
    std::vector<float> hloss(nruns);
    float *const outs[3] = {gk, gC, gS};
    for (int c = 0; c < 3; ++c)
        if (outs[c] && ns)
            TRY(hipMemcpyAsync(outs[c], dgrad + c * ns, sizeof(float) * ns,
                               dev_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
    if (gvox_a && nv)
        TRY(hipMemcpyAsync(gvox_a, dvox, sizeof(float) * nv, hipMemcpyDeviceToHost, s->stream));
    if (gvox_phi && nv)
        TRY(hipMemcpyAsync(gvox_phi, dvox + nv, sizeof(float) * nv, hipMemcpyDeviceToHost, s->stream));
    if (nruns)
        TRY(hipMemcpyAsync(hloss.data(), dloss, sizeof(float) * nruns, hipMemcpyDeviceToHost, s->stream));
    TRY(hipStreamSynchronize(s->stream));
#undef TRY
    cleanup();
    if (loss) {
        // per body in the caller's numbering (a body without masses: 0)
        std::vector<float> lb(nb, 0.f);
        for (int64_t r = 0; r < nruns; ++r)
            lb[rank_body[r]] = hloss[r];
        if (dev_out)
            HIP_TRY(s, hipMemcpy(loss, lb.data(), sizeof(float) * nb, hipMemcpyHostToDevice));
        else
            std::copy(lb.begin(), lb.end(), loss);
    }
    return TITAN_OK;
}

int batch_threads(const titan_sim *s) { return s->batch && s->batch_step ? s->batch->threads : 0; }

}  // namespace titan

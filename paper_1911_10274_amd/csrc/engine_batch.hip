// Host side of the batched engine: groups of whole bodies, their LDS-resident
// stepping kernel, and the autotuner that picks the workgroup size -- and,
// under TITAN_ENGINE_AUTO, whether the batched or the tiled engine runs.
//
// Bodies are laid out contiguously, largest first (see plan_order), so the
// launch order of the groups is a longest-processing-time-first list schedule:
// the hardware hands the next group to whichever compute unit frees up.
#include <hip/hip_runtime.h>

#include <algorithm>
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

int build_batch_engine(titan_sim *s)
{
    s->batch = nullptr;
    const int64_t n = s->n;
    if (n == 0 || (s->h_slot_nbr.empty() && s->ns > 0))
        return TITAN_OK;

    // Body runs in internal order (largest body first), then groups.
    std::vector<int64_t> goff{0};
    int64_t gsize = 0, max_group = 0;
    int64_t pack = kPackMin;
    {
        int64_t b = 1;
        while (b < n && s->h_body[s->perm[b]] == s->h_body[s->perm[0]])
            ++b;
        pack = std::max<int64_t>(pack, b);  // the first body is a largest one
    }
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
    if (max_group > kMaxGroup)
        return TITAN_OK;  // a body too large for LDS: not eligible
    const int64_t ng = (int64_t)goff.size() - 1;

    // Per-slot neighbour index relative to the group's first mass.
    const int64_t slots = (int64_t)s->h_slot_nbr.size();
    std::vector<uint16_t> nbr_group(slots, 0);
    std::vector<int64_t> hoff(s->gg.n_slices + 1);
    HIP_TRY(s, hipMemcpy(hoff.data(), s->gg.slice_off, sizeof(int64_t) * hoff.size(), hipMemcpyDeviceToHost));
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

    BatchEngine *be = new (std::nothrow) BatchEngine();
    if (!be)
        return fail(TITAN_ENOMEM, "out of host memory");
    be->lay.n_groups = ng;
    be->lay.max_group = (int32_t)max_group;
    {
        int64_t *d = nullptr;
        if (int rc = dev_alloc(s, sizeof(int64_t) * goff.size(), (void **)&d)) {
            delete be;
            return rc;
        }
        HIP_TRY(s, hipMemcpyAsync(d, goff.data(), sizeof(int64_t) * goff.size(), hipMemcpyHostToDevice, s->stream));
        be->lay.mass_off = d;
        uint16_t *e = nullptr;
        if (int rc = dev_alloc(s, sizeof(uint16_t) * std::max<int64_t>(slots, 1), (void **)&e)) {
            delete be;
            return rc;
        }
        if (slots)
            HIP_TRY(s, hipMemcpyAsync(e, nbr_group.data(), sizeof(uint16_t) * slots, hipMemcpyHostToDevice,
                                      s->stream));
        be->lay.nbr_group = e;
    }

    // Autotune: workgroup size of the batched kernel, and (AUTO) batched vs
    // the per-step gather engine, by timing kTuneSteps steps of each into
    // scratch buffers (the simulation state is not touched).
    float4 *su = nullptr, *sv = nullptr;
    if (int rc = dev_alloc(s, sizeof(float4) * n, (void **)&su)) {
        delete be;
        return rc;
    }
    if (int rc = dev_alloc(s, sizeof(float4) * n, (void **)&sv)) {
        delete be;
        return rc;
    }
    HIP_TRY(s, launch_trig_table(s->trig, 0, kTuneSteps, s->params.omega, s->params.dt, s->stream));
    float best = 1e30f;
    int best_t = 0;
    for (int t : kBatchThreadChoices) {
        if (!threads_fit(t, max_group))
            continue;
        float ms = 0.f;
        if (int rc = time_batch(s, *be, t, su, sv, &ms)) {
            delete be;
            return rc;
        }
        if (ms < best) {
            best = ms;
            best_t = t;
        }
    }
    if (best_t == 0) {
        delete be;
        return TITAN_OK;
    }
    be->threads = best_t;
    s->tune_batch_ms = best / kTuneSteps;
    bool use = true;
    if (s->params.engine == TITAN_ENGINE_AUTO) {
        float gms = 0.f;
        if (int rc = time_gather(s, su, sv, &gms)) {
            delete be;
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
    if (!use) {
        delete be;
        return TITAN_OK;
    }
    s->batch = be;
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

void destroy_batch_engine(titan_sim *s)
{
    delete s->batch;
    s->batch = nullptr;
}

int batch_threads(const titan_sim *s) { return s->batch ? s->batch->threads : 0; }

}  // namespace titan

// Host runtime behind the C ABI (include/titan.h): staging and validation of
// masses and springs, construction of the device representation, the
// stream-ordered step queue with breakpoints (the paper's asynchronous
// CPU/GPU model, Sec. III-D), state I/O and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "titan.h"
#include "titan_internal.h"
#include "titan_sim.h"

using namespace titan;

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

int titan::fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int titan::hip_fail(titan_sim *sim, hipError_t e, const char *what)
{
    if (sim)
        sim->dev_error = true;
    return fail(TITAN_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(sim, expr)                                  \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess)                               \
            return titan::hip_fail((sim), e_, #expr);       \
    } while (0)

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------

int titan::dev_alloc(titan_sim *s, size_t bytes, void **out)
{
    *out = nullptr;
    if (bytes == 0)
        bytes = 256;
    void *p = nullptr;
    if (s->alloc.alloc) {
        p = s->alloc.alloc(bytes, s->alloc.ctx);
        if (!p)
            return fail(TITAN_ENOMEM, "device allocator returned NULL for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(e == hipErrorOutOfMemory ? TITAN_ENOMEM : TITAN_EDEVICE,
                        "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        }
    }
    s->allocations.push_back({p, bytes, s->engine_allocs});
    s->device_bytes += (int64_t)bytes;
    *out = p;
    return TITAN_OK;
}

static void release(titan_sim *s, void *p)
{
    if (s->alloc.release)
        s->alloc.release(p, s->alloc.ctx);
    else
        (void)hipFree(p);
}

void titan::dev_free(titan_sim *s, void *p)
{
    for (size_t q = 0; q < s->allocations.size(); ++q)
        if (s->allocations[q].p == p) {
            (void)hipStreamSynchronize(s->stream);
            release(s, p);
            s->device_bytes -= (int64_t)s->allocations[q].bytes;
            s->allocations.erase(s->allocations.begin() + q);
            return;
        }
}

// Free every allocation of the engines' layouts (after the queued work).
void titan::dev_free_engine(titan_sim *s)
{
    (void)hipStreamSynchronize(s->stream);
    std::vector<titan_sim::Allocation> keep;
    for (auto &a : s->allocations) {
        if (a.engine) {
            release(s, a.p);
            s->device_bytes -= (int64_t)a.bytes;
        } else {
            keep.push_back(a);
        }
    }
    s->allocations.swap(keep);
}

static void dev_free_all(titan_sim *s)
{
    for (auto &a : s->allocations)
        release(s, a.p);
    s->allocations.clear();
    s->device_bytes = 0;
}

template <class T>
static int upload(titan_sim *s, const std::vector<T> &h, T **d)
{
    int rc = dev_alloc(s, h.size() * sizeof(T), (void **)d);
    if (rc)
        return rc;
    if (!h.empty())
        HIP_TRY(s, hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s->stream));
    return TITAN_OK;
}

// ---------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------

static bool finite3(const float *p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

static int check_params(const titan_params *p)
{
    if (!p)
        return fail(TITAN_EINVAL, "params is NULL");
    if (!(std::isfinite(p->dt) && p->dt > 0))
        return fail(TITAN_EINVAL, "dt must be finite and > 0 (got %g)", p->dt);
    for (int q = 0; q < 3; ++q)
        if (!std::isfinite(p->gravity[q]))
            return fail(TITAN_EINVAL, "gravity must be finite");
    if (!(std::isfinite(p->ground_k) && p->ground_k >= 0))
        return fail(TITAN_EINVAL, "ground_k must be finite and >= 0");
    if (!(std::isfinite(p->friction_mu) && p->friction_mu >= 0))
        return fail(TITAN_EINVAL, "friction_mu must be finite and >= 0");
    if (!std::isfinite(p->omega))
        return fail(TITAN_EINVAL, "omega must be finite");
    if (p->engine < TITAN_ENGINE_AUTO || p->engine > TITAN_ENGINE_TILED)
        return fail(TITAN_EINVAL, "unknown engine %d", p->engine);
    if (p->actuation != TITAN_ACT_PHASOR && p->actuation != TITAN_ACT_WAVE)
        return fail(TITAN_EINVAL, "unknown actuation %d", p->actuation);
    if (p->actuation == TITAN_ACT_WAVE && !(std::isfinite(p->wave_period) && p->wave_period > 0))
        return fail(TITAN_EINVAL, "wave_period must be finite and > 0 (got %g)", p->wave_period);
    if (p->integrator < TITAN_INTEG_EULER || p->integrator > TITAN_INTEG_RK4)
        return fail(TITAN_EINVAL, "unknown integrator %d", p->integrator);
    if (p->graph_steps < 0 || p->graph_steps > 4096 || (p->graph_steps & 1))
        return fail(TITAN_EINVAL, "graph_steps must be 0 or an even number up to 4096 (got %d)", p->graph_steps);
    return TITAN_OK;
}

// A direct change of the actuation of springs [first, first + count) ends the
// voxel map if any of them was voxel-driven (their phasors no longer follow
// the voxels).
static void drop_voxel_map_over(titan_sim *s, int64_t first, int64_t count)
{
    if (s->h_sv_count.empty())
        return;
    for (int64_t q = first; q < first + count && q < (int64_t)s->h_sv_count.size(); ++q)
        if (s->h_sv_count[q] > 0) {
            s->h_vox_a.clear();
            s->h_vox_phi.clear();
            s->h_vs_ptr.clear();
            s->h_vs_spring.clear();
            s->h_sv_count.clear();
            return;
        }
}

// ---------------------------------------------------------------------------
// ABI: lifetime
// ---------------------------------------------------------------------------

extern "C" int titan_abi_version(void) { return TITAN_ABI_VERSION; }

extern "C" const char *titan_last_error(void) { return g_last_error.c_str(); }

extern "C" int titan_create(const titan_params *p, void *stream, const titan_allocator *alloc, titan_sim **out)
{
    if (!out)
        return fail(TITAN_EINVAL, "out is NULL");
    *out = nullptr;
    if (int rc = check_params(p))
        return rc;
    if (alloc && (!alloc->alloc || !alloc->release))
        return fail(TITAN_EINVAL, "allocator needs both alloc and release");
    titan_sim *s = new (std::nothrow) titan_sim();
    if (!s)
        return fail(TITAN_ENOMEM, "out of host memory");
    s->params = *p;
    s->stream = (hipStream_t)stream;
    if (alloc)
        s->alloc = *alloc;
    *out = s;
    return TITAN_OK;
}

extern "C" int titan_destroy(titan_sim *s)
{
    if (!s)
        return TITAN_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->finalized) {
            (void)hipSetDevice(s->device);
            (void)hipStreamSynchronize(s->stream);
            if (s->side_stream)
                (void)hipStreamSynchronize(s->side_stream);
            for (auto &kv : s->bps)
                if (kv.second.ev)
                    (void)hipEventDestroy(kv.second.ev);
            if (s->side_stream)
                (void)hipStreamDestroy(s->side_stream);
            if (s->host_stage)
                (void)hipHostFree(s->host_stage);
            destroy_step_graphs(s);
            destroy_engines(s);
            dev_free_all(s);
        }
    }
    delete s;
    return TITAN_OK;
}

// ---------------------------------------------------------------------------
// ABI: building the system
// ---------------------------------------------------------------------------

static int add_masses_live(titan_sim *s, int64_t n, const float *pos, const float *vel, const float *mass,
                           const int32_t *body, int64_t *first_out);

extern "C" int titan_add_masses(titan_sim *s, int64_t n, const float *pos, const float *vel, const float *mass,
                                const int32_t *body, int64_t *first_out)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (n < 0)
        return fail(TITAN_EINVAL, "negative count");
    if (n > 0 && (!pos || !mass))
        return fail(TITAN_EINVAL, "pos and mass are required");
    if ((int64_t)s->h_mass.size() + n > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(TITAN_EINVAL, "too many masses (limit 2^31-1)");
    for (int64_t i = 0; i < n; ++i) {
        if (!finite3(pos + 3 * i))
            return fail(TITAN_EINVAL, "mass %lld: non-finite position", (long long)i);
        if (vel && !finite3(vel + 3 * i))
            return fail(TITAN_EINVAL, "mass %lld: non-finite velocity", (long long)i);
        if (!(std::isfinite(mass[i]) && mass[i] >= 0.f))
            return fail(TITAN_EINVAL, "mass %lld: mass must be finite and >= 0", (long long)i);
        if (body && body[i] < 0)
            return fail(TITAN_EINVAL, "mass %lld: negative body id", (long long)i);
    }
    if (s->finalized)
        return add_masses_live(s, n, pos, vel, mass, body, first_out);
    if (first_out)
        *first_out = (int64_t)s->h_mass.size();
    s->h_pos.insert(s->h_pos.end(), pos, pos + 3 * n);
    if (vel)
        s->h_vel.insert(s->h_vel.end(), vel, vel + 3 * n);
    else
        s->h_vel.insert(s->h_vel.end(), (size_t)(3 * n), 0.f);
    s->h_mass.insert(s->h_mass.end(), mass, mass + n);
    if (body)
        s->h_body.insert(s->h_body.end(), body, body + n);
    else
        s->h_body.insert(s->h_body.end(), (size_t)n, 0);
    return TITAN_OK;
}

extern "C" int titan_add_springs(titan_sim *s, int64_t n, const int64_t *ends, const float *k, const float *damping,
                                 const float *rest, const float *amp, const float *phase, int64_t *first_out)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    invalidate_step_cache(s);
    if (s->finalized && s->dev_error)
        return fail(TITAN_EDEVICE, "sim is in a failed device state");
    if (n < 0)
        return fail(TITAN_EINVAL, "negative count");
    if (n > 0 && (!ends || !k))
        return fail(TITAN_EINVAL, "ends and k are required");
    if ((amp == nullptr) != (phase == nullptr))
        return fail(TITAN_EINVAL, "amp and phase must be given together");
    const int64_t nm = (int64_t)s->h_mass.size();
    if ((int64_t)s->h_k.size() + n > (int64_t)std::numeric_limits<int32_t>::max() / 2)
        return fail(TITAN_EINVAL, "too many springs (limit 2^30-1)");
    for (int64_t q = 0; q < n; ++q) {
        const int64_t i = ends[2 * q], j = ends[2 * q + 1];
        if (i < 0 || j < 0 || i >= nm || j >= nm)
            return fail(TITAN_EINVAL, "spring %lld: end out of range [0, %lld)", (long long)q, (long long)nm);
        if (i == j)
            return fail(TITAN_EINVAL, "spring %lld: both ends are mass %lld", (long long)q, (long long)i);
        if (s->h_body[i] != s->h_body[j])
            return fail(TITAN_EINVAL, "spring %lld joins bodies %d and %d", (long long)q, s->h_body[i], s->h_body[j]);
        if (!s->finalized) {
            const float *a = &s->h_pos[3 * i], *b = &s->h_pos[3 * j];
            const double dx = (double)b[0] - a[0], dy = (double)b[1] - a[1], dz = (double)b[2] - a[2];
            if (!(dx * dx + dy * dy + dz * dz > 0))
                return fail(TITAN_EINVAL, "spring %lld: zero initial length", (long long)q);
        }
        if (!(std::isfinite(k[q]) && k[q] >= 0.f))
            return fail(TITAN_EINVAL, "spring %lld: k must be finite and >= 0", (long long)q);
        if (damping && !(std::isfinite(damping[q]) && damping[q] >= 0.f))
            return fail(TITAN_EINVAL, "spring %lld: damping must be finite and >= 0", (long long)q);
        if (rest && !(std::isfinite(rest[q]) && rest[q] > 0.f))
            return fail(TITAN_EINVAL, "spring %lld: rest length must be finite and > 0", (long long)q);
        if (amp && !(std::isfinite(amp[q]) && std::isfinite(phase[q])))
            return fail(TITAN_EINVAL, "spring %lld: non-finite actuation", (long long)q);
    }
    // After the first step a spring without a rest length is at rest at the
    // current positions (the state after the queued steps).
    std::vector<float> live_rest;
    if (s->finalized && n > 0) {
        std::vector<float4> hU(s->n);
        HIP_TRY(s, hipMemcpyAsync(hU.data(), s->U[s->cur], sizeof(float4) * s->n, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(s, hipStreamSynchronize(s->stream));
        live_rest.resize(n);
        for (int64_t q = 0; q < n; ++q) {
            const int64_t a = s->inv_perm_of(ends[2 * q]), b = s->inv_perm_of(ends[2 * q + 1]);
            const double dx = ((double)s->hX0[b].x + hU[b].x) - ((double)s->hX0[a].x + hU[a].x);
            const double dy = ((double)s->hX0[b].y + hU[b].y) - ((double)s->hX0[a].y + hU[a].y);
            const double dz = ((double)s->hX0[b].z + hU[b].z) - ((double)s->hX0[a].z + hU[a].z);
            const double len = std::sqrt(dx * dx + dy * dy + dz * dz);
            if (!(len > 0))
                return fail(TITAN_EINVAL, "spring %lld: zero current length", (long long)q);
            live_rest[q] = rest ? rest[q] : (float)len;
        }
        rest = live_rest.data();
    }
    if (first_out)
        *first_out = (int64_t)s->h_k.size();
    s->h_ends.insert(s->h_ends.end(), ends, ends + 2 * n);
    s->h_k.insert(s->h_k.end(), k, k + n);
    if (damping)
        s->h_damp.insert(s->h_damp.end(), damping, damping + n);
    else
        s->h_damp.insert(s->h_damp.end(), (size_t)n, 0.f);
    if (rest)
        s->h_rest.insert(s->h_rest.end(), rest, rest + n);
    else
        s->h_rest.insert(s->h_rest.end(), (size_t)n, -1.f);  // -1: initial length
    if (amp) {
        s->h_amp.insert(s->h_amp.end(), amp, amp + n);
        s->h_phase.insert(s->h_phase.end(), phase, phase + n);
        for (int64_t q = 0; q < n; ++q) {
            s->h_C.push_back((float)((double)amp[q] * std::cos((double)phase[q])));
            s->h_S.push_back((float)((double)amp[q] * std::sin((double)phase[q])));
        }
    } else {
        s->h_amp.insert(s->h_amp.end(), (size_t)n, 0.f);
        s->h_phase.insert(s->h_phase.end(), (size_t)n, 0.f);
        s->h_C.insert(s->h_C.end(), (size_t)n, 0.f);
        s->h_S.insert(s->h_S.end(), (size_t)n, 0.f);
    }
    if (!s->h_sv_count.empty())
        s->h_sv_count.resize(s->h_k.size(), 0);  // new springs are not voxel-driven
    if (!s->h_removed.empty())
        s->h_removed.resize(s->h_k.size(), 0);
    if (!s->h_yield.empty())
        s->h_yield.resize(s->h_k.size(), INFINITY);
    if (!s->h_broken.empty())
        s->h_broken.resize(s->h_k.size(), 0);
    if (s->finalized && n > 0) {
        const int64_t first = s->ns;
        s->ns = (int64_t)s->h_k.size();
        s->h_owner_slot.resize(s->ns, -1);
        s->h_other_slot.resize(s->ns, -1);
        ++s->slot_gen;
        // into spare slots of the current layouts if they all fit (O(1) per
        // spring), else the layouts are rebuilt before the next step, with
        // more spare slots
        int rc = s->layout_dirty ? 2 : insert_springs(s, first, n);
        if (rc > 0) {
            s->layout_dirty = true;
            s->slack = rc == 1 ? std::min(std::max(2 * s->slack, 2), kMaxSlack) : std::max(s->slack, 2);
            rc = TITAN_OK;
        } else if (rc != TITAN_OK) {
            s->layout_dirty = true;
        }
        return rc;
    }
    return TITAN_OK;
}

// ---------------------------------------------------------------------------
// topology edits after the first step
// ---------------------------------------------------------------------------

// A device float4 array of n_old entries grown to n_old + tail.size(), the new
// entries taken from tail (stream order).
static int grow_state(titan_sim *s, float4 **buf, int64_t n_old, const std::vector<float4> &tail)
{
    const int64_t n_new = n_old + (int64_t)tail.size();
    float4 *p = nullptr;
    if (int rc = dev_alloc(s, sizeof(float4) * n_new, (void **)&p))
        return rc;
    if (n_old)
        HIP_TRY(s, hipMemcpyAsync(p, *buf, sizeof(float4) * n_old, hipMemcpyDeviceToDevice, s->stream));
    if (!tail.empty())
        HIP_TRY(s, hipMemcpyAsync(p + n_old, tail.data(), sizeof(float4) * tail.size(), hipMemcpyHostToDevice,
                                  s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    dev_free(s, *buf);
    *buf = p;
    return TITAN_OK;
}

// Masses added after the first step go after every existing mass in the
// internal order (existing indices, state and snapshots keep their meaning).
// They must start new bodies, or join the only body of a single-body system,
// so that every body stays one contiguous run.
static int add_masses_live(titan_sim *s, int64_t n, const float *pos, const float *vel, const float *mass,
                           const int32_t *body, int64_t *first_out)
{
    invalidate_step_cache(s);
    if (s->dev_error)
        return fail(TITAN_EDEVICE, "sim is in a failed device state");
    int32_t maxb = -1;
    for (int32_t b : s->h_body)
        maxb = std::max(maxb, b);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t b = body ? body[i] : 0;
        if (!(b > maxb || (maxb == 0 && b == 0)))
            return fail(TITAN_EINVAL, "mass %lld: masses added after the first step must start a new body "
                                      "(or join the only body)", (long long)i);
    }
    const int64_t n_old = s->n;
    if (first_out)
        *first_out = n_old;
    std::vector<float4> x0(n), u(n), v(n);
    for (int64_t i = 0; i < n; ++i) {
        x0[i] = make_float4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], 0.f);
        u[i] = make_float4(0.f, 0.f, 0.f, mass[i] > 0.f ? (float)(1.0 / (double)mass[i]) : 0.f);
        v[i] = vel ? make_float4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    if (int rc = grow_state(s, &s->X0, n_old, x0))
        return rc;
    for (int b = 0; b < 2; ++b) {
        if (int rc = grow_state(s, &s->U[b], n_old, u))
            return rc;
        if (int rc = grow_state(s, &s->V[b], n_old, v))
            return rc;
    }
    for (auto &kv : s->bps) {  // a snapshot before the masses existed holds their initial state
        if (int rc = grow_state(s, &kv.second.snapU, n_old, u))
            return rc;
        if (int rc = grow_state(s, &kv.second.snapV, n_old, v))
            return rc;
    }
    if (s->F) {
        dev_free(s, s->F);
        s->F = nullptr;
    }
    HIP_TRY(s, hipHostFree(s->host_stage));
    s->host_stage = nullptr;
    HIP_TRY(s, hipHostMalloc(&s->host_stage, sizeof(float4) * 2 * (n_old + n), hipHostMallocDefault));
    s->hX0.insert(s->hX0.end(), x0.begin(), x0.end());
    s->h_pos.insert(s->h_pos.end(), pos, pos + 3 * n);
    if (vel)
        s->h_vel.insert(s->h_vel.end(), vel, vel + 3 * n);
    else
        s->h_vel.insert(s->h_vel.end(), (size_t)(3 * n), 0.f);
    s->h_mass.insert(s->h_mass.end(), mass, mass + n);
    for (int64_t i = 0; i < n; ++i) {
        s->h_body.push_back(body ? body[i] : 0);
        s->perm.push_back(n_old + i);  // caller index n_old + i is internal index n_old + i
        if (!s->inv_perm.empty())
            s->inv_perm.push_back(n_old + i);
    }
    s->n = n_old + n;
    s->layout_dirty = true;
    return TITAN_OK;
}

// Springs removed: kept in the spring table, dropped from the layouts.  On a
// current layout the removal is a tombstone -- k = 0 and damping 0 in the
// spring's two slots -- so each end adds an exact zero in the spring's place
// and every other bit of the step is unchanged.
static int remove_springs_locked(titan_sim *s, const std::vector<int64_t> &list)
{
    if (s->h_removed.empty())
        s->h_removed.assign(s->h_k.size(), 0);
    std::vector<int64_t> now;
    for (int64_t q : list)
        if (!s->h_removed[q]) {
            s->h_removed[q] = 1;
            s->h_k[q] = 0.f;
            s->h_damp[q] = 0.f;
            now.push_back(q);
        }
    if (!s->finalized || s->layout_dirty || now.empty())
        return TITAN_OK;
    const bool damped = s->gg.c != nullptr || s->gg.c_uniform != 0.f;
    return update_spring_list(s, now, true, damped, false, true);
}

extern "C" int titan_remove_springs(titan_sim *s, int64_t n, const int64_t *springs)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    invalidate_step_cache(s);
    if (n < 0 || (n > 0 && !springs))
        return fail(TITAN_EINVAL, "bad spring list");
    if (s->dev_error)
        return fail(TITAN_EDEVICE, "sim is in a failed device state");
    const int64_t ns = (int64_t)s->h_k.size();
    std::vector<int64_t> list(springs, springs + n);
    for (int64_t q : list)
        if (q < 0 || q >= ns)
            return fail(TITAN_EINVAL, "spring %lld out of range [0, %lld)", (long long)q, (long long)ns);
    return remove_springs_locked(s, list);
}

extern "C" int titan_set_yield(titan_sim *s, int64_t first, int64_t count, const float *yield)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    invalidate_step_cache(s);
    const int64_t ns = (int64_t)s->h_k.size();
    if (first < 0 || count < 0 || first > ns || count > ns - first || (count > 0 && !yield))
        return fail(TITAN_EINVAL, "bad spring range [%lld, +%lld) of %lld", (long long)first, (long long)count,
                    (long long)ns);
    for (int64_t q = 0; q < count; ++q)
        if (!(yield[q] > 0.f))  // NaN fails too
            return fail(TITAN_EINVAL, "spring %lld: yield value must be > 0 (or +inf)", (long long)(first + q));
    if (s->finalized && s->dev_error)
        return fail(TITAN_EDEVICE, "sim is in a failed device state");
    if (s->finalized && !s->layout_dirty)
        if (int rc = sync_broken(s))  // keep the breaks already recorded
            return rc;
    if (s->h_yield.empty())
        s->h_yield.assign(ns, INFINITY);
    std::copy(yield, yield + count, s->h_yield.begin() + first);
    if (!s->finalized || s->layout_dirty || count == 0)
        return TITAN_OK;
    if (!s->gg.yield) {  // the layout has no yield values yet: rebuilt before the next step
        s->layout_dirty = true;
        return TITAN_OK;
    }
    std::vector<int64_t> list(count);
    for (int64_t q = 0; q < count; ++q)
        list[q] = first + q;
    return update_yield(s, list);
}

extern "C" int titan_get_broken(titan_sim *s, int64_t first, int64_t count, uint8_t *broken)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t ns = (int64_t)s->h_k.size();
    if (first < 0 || count < 0 || first > ns || count > ns - first || (count > 0 && !broken))
        return fail(TITAN_EINVAL, "bad spring range [%lld, +%lld) of %lld", (long long)first, (long long)count,
                    (long long)ns);
    if (s->finalized && s->dev_error)
        return fail(TITAN_EDEVICE, "sim is in a failed device state");
    if (s->finalized && !s->layout_dirty)
        if (int rc = sync_broken(s))
            return rc;
    for (int64_t q = 0; q < count; ++q)
        broken[q] = s->h_broken.empty() ? 0 : s->h_broken[first + q];
    return TITAN_OK;
}

extern "C" int titan_remove_masses(titan_sim *s, int64_t n, const int64_t *masses)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    invalidate_step_cache(s);
    if (n < 0 || (n > 0 && !masses))
        return fail(TITAN_EINVAL, "bad mass list");
    if (s->dev_error)
        return fail(TITAN_EDEVICE, "sim is in a failed device state");
    const int64_t nm = (int64_t)s->h_mass.size();
    std::vector<uint8_t> gone(nm, 0);
    for (int64_t k = 0; k < n; ++k) {
        if (masses[k] < 0 || masses[k] >= nm)
            return fail(TITAN_EINVAL, "mass %lld out of range [0, %lld)", (long long)masses[k], (long long)nm);
        gone[masses[k]] = 1;
    }
    std::vector<int64_t> springs;
    for (int64_t q = 0; q < (int64_t)s->h_k.size(); ++q)
        if (gone[s->h_ends[2 * q]] || gone[s->h_ends[2 * q + 1]])
            springs.push_back(q);
    if (int rc = remove_springs_locked(s, springs))
        return rc;
    // a removed mass stays where it is, pinned and at rest
    const float zero4[4] = {0.f, 0.f, 0.f, 0.f};
    for (int64_t k = 0; k < n; ++k) {
        s->h_mass[masses[k]] = 0.f;
        if (s->finalized) {
            const int64_t i = s->inv_perm_of(masses[k]);
            HIP_TRY(s, hipMemcpyAsync(&s->U[s->cur][i].w, zero4, sizeof(float), hipMemcpyHostToDevice, s->stream));
            HIP_TRY(s, hipMemcpyAsync(&s->V[s->cur][i], zero4, sizeof(float4), hipMemcpyHostToDevice, s->stream));
        }
    }
    if (s->finalized)
        HIP_TRY(s, hipStreamSynchronize(s->stream));
    return TITAN_OK;
}

extern "C" int titan_set_params(titan_sim *s, const titan_params *p)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (int rc = check_params(p))
        return rc;
    if (s->finalized && p->engine != s->params.engine && p->engine != TITAN_ENGINE_AUTO)
        return fail(TITAN_ESTATE, "the engine can only be chosen before the first step");
    if (s->finalized && p->actuation != s->params.actuation)
        return fail(TITAN_ESTATE, "the actuation law can only be chosen before the first step");
    const int32_t engine = s->finalized ? s->params.engine : p->engine;
    // which engine steps under the new integrator (decided before anything
    // changes, so that a refused call leaves the sim as it was)
    int32_t new_engine = s->engine;
    if (s->finalized && s->batch && s->batch_step) {
        const bool euler = p->integrator == TITAN_INTEG_EULER;
        const bool fits = euler || batch_integ_fits(batch_layout(s), p->integrator);
        if (engine == TITAN_ENGINE_BATCHED) {
            if (!fits)
                return fail(TITAN_ESTATE, "the batched engine cannot run this integrator on this system");
            new_engine = TITAN_ENGINE_BATCHED;
        } else {  // AUTO: the batched Verlet / RK4 kernels for small groups only
            new_engine = (euler || (fits && batch_integ_preferred(batch_layout(s))))
                             ? TITAN_ENGINE_BATCHED
                             : (s->tiled ? TITAN_ENGINE_TILED : TITAN_ENGINE_GATHER);
        }
    }
    s->params = *p;
    s->params.engine = engine;
    if (s->finalized) {
        invalidate_step_cache(s);
        s->engine = new_engine;
    }
    return TITAN_OK;
}

// ---------------------------------------------------------------------------
// finalize: device representation
// ---------------------------------------------------------------------------

static int ensure_device(titan_sim *s)
{
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) {
        (void)hipGetLastError();
        s->dev_error = true;
        return fail(TITAN_EDEVICE, "no usable HIP device (%s)", e == hipSuccess ? "count 0" : hipGetErrorString(e));
    }
    HIP_TRY(s, hipGetDevice(&s->device));
    return TITAN_OK;
}

static int finalize_locked(titan_sim *s)
{
    if (s->finalized)
        return TITAN_OK;
    if (s->dev_error)
        return fail(TITAN_EDEVICE, "sim is in a failed device state");
    // Host planning first (internal order, incidence layout): it needs no
    // device, and systems of any size, empty ones included, go through it.
    plan_layouts(s);
    if (int rc = ensure_device(s))
        return rc;
    const int64_t n = s->n;

    // Reference positions and initial state in internal (spatial) order.
    std::vector<float4> hX0(n), hU(n), hV(n);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t u = s->perm[i];
        hX0[i] = make_float4(s->h_pos[3 * u], s->h_pos[3 * u + 1], s->h_pos[3 * u + 2], 0.f);
        const float m = s->h_mass[u];
        hU[i] = make_float4(0.f, 0.f, 0.f, m > 0.f ? (float)(1.0 / (double)m) : 0.f);
        hV[i] = make_float4(s->h_vel[3 * u], s->h_vel[3 * u + 1], s->h_vel[3 * u + 2], 0.f);
    }
    s->hX0 = hX0;

    for (int b = 0; b < 2; ++b) {
        if (int rc = dev_alloc(s, sizeof(float4) * n, (void **)&s->U[b]))
            return rc;
        if (int rc = dev_alloc(s, sizeof(float4) * n, (void **)&s->V[b]))
            return rc;
    }
    if (int rc = upload(s, hX0, &s->X0))
        return rc;
    if (n)
        HIP_TRY(s, hipMemcpyAsync(s->U[0], hU.data(), sizeof(float4) * n, hipMemcpyHostToDevice, s->stream));
    if (n)
        HIP_TRY(s, hipMemcpyAsync(s->V[0], hV.data(), sizeof(float4) * n, hipMemcpyHostToDevice, s->stream));
    s->cur = 0;

    if (int rc = dev_alloc(s, sizeof(unsigned long long), (void **)&s->first_bad))
        return rc;
    const unsigned long long none = ~0ull;
    HIP_TRY(s, hipMemcpyAsync(s->first_bad, &none, sizeof none, hipMemcpyHostToDevice, s->stream));

    if (int rc = build_engines(s))
        return rc;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    HIP_TRY(s, hipStreamCreateWithFlags(&s->side_stream, hipStreamNonBlocking));
    HIP_TRY(s, hipHostMalloc(&s->host_stage, sizeof(float4) * (n > 0 ? 2 * n : 2), hipHostMallocDefault));
    s->finalized = true;
    return TITAN_OK;
}

extern "C" int titan_finalize(titan_sim *s)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    return finalize_locked(s);
}

// ---------------------------------------------------------------------------
// stepping and breakpoints
// ---------------------------------------------------------------------------

static int fire_breakpoints(titan_sim *s)
{
    for (auto &kv : s->bps) {
        BP &bp = kv.second;
        if (bp.fired || bp.step != s->step_enq)
            continue;
        if (s->n) {
            HIP_TRY(s, hipMemcpyAsync(bp.snapU, s->U[s->cur], sizeof(float4) * s->n, hipMemcpyDeviceToDevice, s->stream));
            HIP_TRY(s, hipMemcpyAsync(bp.snapV, s->V[s->cur], sizeof(float4) * s->n, hipMemcpyDeviceToDevice, s->stream));
        }
        HIP_TRY(s, hipEventRecord(bp.ev, s->stream));
        bp.fired = true;
        if (bp.kind == TITAN_BP_PAUSE)
            s->paused = true;
    }
    return TITAN_OK;
}

// Layouts invalidated by topology edits are rebuilt before they are used.
static int ensure_layout(titan_sim *s)
{
    if (!s->finalized || !s->layout_dirty)
        return TITAN_OK;
    return rebuild_engines(s);
}

static int pump(titan_sim *s)
{
    if (int rc = ensure_layout(s))
        return rc;
    if (int rc = fire_breakpoints(s))
        return rc;
    while (!s->paused && s->step_enq < s->steps_req) {
        int64_t end = s->steps_req;
        for (auto &kv : s->bps)
            if (!kv.second.fired && kv.second.step > s->step_enq && kv.second.step < end)
                end = kv.second.step;
        if (int rc = enqueue_steps(s, s->step_enq, end - s->step_enq))
            return rc;
        s->step_enq = end;
        if (int rc = fire_breakpoints(s))
            return rc;
    }
    return TITAN_OK;
}

static int ready(titan_sim *s)
{
    if (s->dev_error)
        return fail(TITAN_EDEVICE, "sim is in a failed device state");
    if (!s->finalized)
        if (int rc = finalize_locked(s))
            return rc;
    HIP_TRY(s, hipSetDevice(s->device));
    return TITAN_OK;
}

extern "C" int titan_step(titan_sim *s, int64_t n)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (n < 0)
        return fail(TITAN_EINVAL, "negative step count");
    if (int rc = ready(s))
        return rc;
    s->steps_req += n;
    return pump(s);
}

extern "C" int titan_set_breakpoint(titan_sim *s, int64_t step, int32_t kind, uint64_t *bp_out)
{
    if (!s || !bp_out)
        return fail(TITAN_EINVAL, "sim or bp_out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (kind != TITAN_BP_SNAPSHOT && kind != TITAN_BP_PAUSE)
        return fail(TITAN_EINVAL, "unknown breakpoint kind %d", kind);
    if (int rc = ready(s))
        return rc;
    if (step < s->step_enq)
        return fail(TITAN_EINVAL, "breakpoint step %lld is behind the %lld steps already enqueued",
                    (long long)step, (long long)s->step_enq);
    BP bp;
    bp.id = ++s->next_bp;
    bp.step = step;
    bp.kind = kind;
    HIP_TRY(s, hipEventCreateWithFlags(&bp.ev, hipEventDisableTiming));
    if (int rc = dev_alloc(s, sizeof(float4) * s->n, (void **)&bp.snapU))
        return rc;
    if (int rc = dev_alloc(s, sizeof(float4) * s->n, (void **)&bp.snapV))
        return rc;
    s->bps[bp.id] = bp;
    *bp_out = bp.id;
    return pump(s);
}

static int check_bad(titan_sim *s)
{
    unsigned long long fb = ~0ull;
    HIP_TRY(s, hipMemcpy(&fb, s->first_bad, sizeof fb, hipMemcpyDeviceToHost));
    if (fb != ~0ull) {
        s->first_bad_step = (int64_t)fb;
        return fail(TITAN_ENONFINITE, "non-finite state first produced by step %lld", (long long)fb);
    }
    return TITAN_OK;
}

extern "C" int titan_wait(titan_sim *s, uint64_t id)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->bps.find(id);
    if (it == s->bps.end())
        return fail(TITAN_EINVAL, "unknown breakpoint %llu", (unsigned long long)id);
    if (int rc = ready(s))
        return rc;
    if (!it->second.fired)
        return fail(TITAN_ESTATE, "breakpoint at step %lld is not reached by the %lld steps requested%s",
                    (long long)it->second.step, (long long)s->steps_req, s->paused ? " (paused)" : "");
    HIP_TRY(s, hipEventSynchronize(it->second.ev));
    return check_bad(s);
}

extern "C" int titan_resume(titan_sim *s)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (int rc = ready(s))
        return rc;
    s->paused = false;
    return pump(s);
}

extern "C" int titan_sync(titan_sim *s)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (int rc = ready(s))
        return rc;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return check_bad(s);
}

// ---------------------------------------------------------------------------
// state I/O
// ---------------------------------------------------------------------------

static int check_range(titan_sim *s, int64_t first, int64_t count)
{
    if (first < 0 || count < 0 || first + count > s->n)
        return fail(TITAN_EINVAL, "range [%lld, %lld) outside [0, %lld)", (long long)first,
                    (long long)(first + count), (long long)s->n);
    return TITAN_OK;
}

// Device state (internal order, U/V float4) -> caller arrays for [first, first+count).
static void export_state(titan_sim *s, const float4 *hU, const float4 *hV, int64_t first, int64_t count,
                         float *pos, float *vel, int32_t flags)
{
    for (int64_t q = 0; q < count; ++q) {
        const int64_t i = s->inv_perm_of(first + q);
        if (pos) {
            if (flags & TITAN_STATE_DISPLACEMENT) {
                pos[3 * q] = hU[i].x;
                pos[3 * q + 1] = hU[i].y;
                pos[3 * q + 2] = hU[i].z;
            } else {
                pos[3 * q] = (float)((double)s->hX0[i].x + hU[i].x);
                pos[3 * q + 1] = (float)((double)s->hX0[i].y + hU[i].y);
                pos[3 * q + 2] = (float)((double)s->hX0[i].z + hU[i].z);
            }
        }
        if (vel) {
            vel[3 * q] = hV[i].x;
            vel[3 * q + 1] = hV[i].y;
            vel[3 * q + 2] = hV[i].z;
        }
    }
}

extern "C" int titan_get_state(titan_sim *s, int64_t first, int64_t count, float *pos, float *vel, int32_t flags,
                               int64_t *step_out)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (int rc = ready(s))
        return rc;
    if (int rc = check_range(s, first, count))
        return rc;
    float4 *hU = s->host_stage, *hV = s->host_stage + s->n;
    if (s->n) {
        HIP_TRY(s, hipMemcpyAsync(hU, s->U[s->cur], sizeof(float4) * s->n, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(s, hipMemcpyAsync(hV, s->V[s->cur], sizeof(float4) * s->n, hipMemcpyDeviceToHost, s->stream));
    }
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    if (step_out)
        *step_out = s->step_enq;
    export_state(s, hU, hV, first, count, pos, vel, flags);
    return check_bad(s);
}

extern "C" int titan_get_snapshot(titan_sim *s, uint64_t id, int64_t first, int64_t count, float *pos, float *vel,
                                  int32_t flags, int64_t *step_out)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->bps.find(id);
    if (it == s->bps.end())
        return fail(TITAN_EINVAL, "unknown breakpoint %llu", (unsigned long long)id);
    if (int rc = ready(s))
        return rc;
    if (int rc = check_range(s, first, count))
        return rc;
    BP &bp = it->second;
    if (!bp.fired)
        return fail(TITAN_ESTATE, "breakpoint at step %lld not reached", (long long)bp.step);
    // Copy out on the side stream after the snapshot event: the compute stream
    // keeps running the steps behind the breakpoint.
    float4 *hU = s->host_stage, *hV = s->host_stage + s->n;
    HIP_TRY(s, hipStreamWaitEvent(s->side_stream, bp.ev, 0));
    if (s->n) {
        HIP_TRY(s, hipMemcpyAsync(hU, bp.snapU, sizeof(float4) * s->n, hipMemcpyDeviceToHost, s->side_stream));
        HIP_TRY(s, hipMemcpyAsync(hV, bp.snapV, sizeof(float4) * s->n, hipMemcpyDeviceToHost, s->side_stream));
    }
    HIP_TRY(s, hipStreamSynchronize(s->side_stream));
    if (step_out)
        *step_out = bp.step;
    export_state(s, hU, hV, first, count, pos, vel, flags);
    return TITAN_OK;
}

extern "C" int titan_set_state(titan_sim *s, int64_t first, int64_t count, const float *pos, const float *vel,
                               int32_t flags)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    invalidate_step_cache(s);
    if (int rc = ready(s))
        return rc;
    if (int rc = check_range(s, first, count))
        return rc;
    for (int64_t q = 0; q < count; ++q) {
        if ((pos && !finite3(pos + 3 * q)) || (vel && !finite3(vel + 3 * q)))
            return fail(TITAN_EINVAL, "mass %lld: non-finite state", (long long)(first + q));
    }
    if (!s->n || (!pos && !vel))
        return TITAN_OK;
    float4 *hU = s->host_stage, *hV = s->host_stage + s->n;
    HIP_TRY(s, hipMemcpyAsync(hU, s->U[s->cur], sizeof(float4) * s->n, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipMemcpyAsync(hV, s->V[s->cur], sizeof(float4) * s->n, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    for (int64_t q = 0; q < count; ++q) {
        const int64_t i = s->inv_perm_of(first + q);
        if (pos) {
            float u[3];
            for (int c = 0; c < 3; ++c) {
                const float x0 = c == 0 ? s->hX0[i].x : c == 1 ? s->hX0[i].y : s->hX0[i].z;
                u[c] = (flags & TITAN_STATE_DISPLACEMENT) ? pos[3 * q + c] : (float)((double)pos[3 * q + c] - x0);
            }
            hU[i].x = u[0];
            hU[i].y = u[1];
            hU[i].z = u[2];
        }
        if (vel) {
            hV[i].x = vel[3 * q];
            hV[i].y = vel[3 * q + 1];
            hV[i].z = vel[3 * q + 2];
        }
    }
    HIP_TRY(s, hipMemcpyAsync(s->U[s->cur], hU, sizeof(float4) * s->n, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipMemcpyAsync(s->V[s->cur], hV, sizeof(float4) * s->n, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    // A new state clears a previous non-finite report.
    const unsigned long long none = ~0ull;
    HIP_TRY(s, hipMemcpy(s->first_bad, &none, sizeof none, hipMemcpyHostToDevice));
    s->first_bad_step = -1;
    return TITAN_OK;
}

extern "C" int titan_set_step(titan_sim *s, int64_t step)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    invalidate_step_cache(s);
    if (step < 0)
        return fail(TITAN_EINVAL, "negative step index");
    if (int rc = ready(s))
        return rc;
    if (s->steps_req != s->step_enq)
        return fail(TITAN_ESTATE, "%lld steps are held at a pause breakpoint",
                    (long long)(s->steps_req - s->step_enq));
    s->step_enq = step;
    s->steps_req = step;
    return TITAN_OK;
}

extern "C" int titan_get_forces(titan_sim *s, int64_t first, int64_t count, float *f)
{
    if (!s || (!f && count))
        return fail(TITAN_EINVAL, "sim or f is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (int rc = ready(s))
        return rc;
    if (int rc = check_range(s, first, count))
        return rc;
    if (!s->n)
        return TITAN_OK;
    if (int rc = ensure_layout(s))
        return rc;
    if (int rc = compute_forces(s))
        return rc;
    float4 *hF = s->host_stage;
    HIP_TRY(s, hipMemcpyAsync(hF, s->F, sizeof(float4) * s->n, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    for (int64_t q = 0; q < count; ++q) {
        const int64_t i = s->inv_perm_of(first + q);
        f[3 * q] = hF[i].x;
        f[3 * q + 1] = hF[i].y;
        f[3 * q + 2] = hF[i].z;
    }
    return TITAN_OK;
}

extern "C" int titan_set_springs(titan_sim *s, int64_t first, int64_t count, const float *k, const float *damping,
                                 const float *amp, const float *phase)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    invalidate_step_cache(s);
    if (first < 0 || count < 0 || first + count > (int64_t)s->h_k.size())
        return fail(TITAN_EINVAL, "spring range [%lld, %lld) outside [0, %lld)", (long long)first,
                    (long long)(first + count), (long long)s->h_k.size());
    if ((amp == nullptr) != (phase == nullptr))
        return fail(TITAN_EINVAL, "amp and phase must be given together");
    for (int64_t q = 0; q < count; ++q) {
        if (k && !(std::isfinite(k[q]) && k[q] >= 0.f))
            return fail(TITAN_EINVAL, "spring %lld: k must be finite and >= 0", (long long)(first + q));
        if (damping && !(std::isfinite(damping[q]) && damping[q] >= 0.f))
            return fail(TITAN_EINVAL, "spring %lld: damping must be finite and >= 0", (long long)(first + q));
        if (amp && !(std::isfinite(amp[q]) && std::isfinite(phase[q])))
            return fail(TITAN_EINVAL, "spring %lld: non-finite actuation", (long long)(first + q));
    }
    for (int64_t q = 0; q < count; ++q) {
        if (k)
            s->h_k[first + q] = k[q];
        if (damping)
            s->h_damp[first + q] = damping[q];
        if (amp) {
            s->h_amp[first + q] = amp[q];
            s->h_phase[first + q] = phase[q];
            s->h_C[first + q] = (float)((double)amp[q] * std::cos((double)phase[q]));
            s->h_S[first + q] = (float)((double)amp[q] * std::sin((double)phase[q]));
        }
    }
    if (amp)
        drop_voxel_map_over(s, first, count);
    if (!s->finalized)
        return TITAN_OK;
    if (int rc = ready(s))
        return rc;
    return update_springs(s, first, count, k, damping, amp, phase);
}

extern "C" int titan_set_springs_phasor(titan_sim *s, int64_t first, int64_t count, const float *act_c,
                                        const float *act_s)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (first < 0 || count < 0 || first + count > (int64_t)s->h_k.size())
        return fail(TITAN_EINVAL, "spring range [%lld, %lld) outside [0, %lld)", (long long)first,
                    (long long)(first + count), (long long)s->h_k.size());
    if (count > 0 && (!act_c || !act_s))
        return fail(TITAN_EINVAL, "act_c and act_s are required");
    if (s->params.actuation != TITAN_ACT_PHASOR)
        return fail(TITAN_ESTATE, "(C, S) phasors belong to the phasor actuation law");
    for (int64_t q = 0; q < count; ++q)
        if (!(std::isfinite(act_c[q]) && std::isfinite(act_s[q])))
            return fail(TITAN_EINVAL, "spring %lld: non-finite actuation", (long long)(first + q));
    invalidate_step_cache(s);
    for (int64_t q = 0; q < count; ++q) {
        const int64_t t = first + q;
        s->h_C[t] = act_c[q];
        s->h_S[t] = act_s[q];
        s->h_amp[t] = (float)std::hypot((double)act_c[q], (double)act_s[q]);
        s->h_phase[t] = (float)std::atan2((double)act_s[q], (double)act_c[q]);
    }
    drop_voxel_map_over(s, first, count);
    if (!s->finalized)
        return TITAN_OK;
    if (int rc = ready(s))
        return rc;
    std::vector<float> one(count, 1.f);  // marks "actuation changed" (values come from the tables)
    return update_springs(s, first, count, nullptr, nullptr, one.data(), one.data());
}

extern "C" int titan_set_voxel_actuation(titan_sim *s, int64_t n_voxels, const float *voxel_a, const float *voxel_phi,
                                         const int64_t *sv_ptr, const int32_t *sv_idx)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t ns = (int64_t)s->h_k.size();
    if (n_voxels < 0 || (n_voxels > 0 && (!voxel_a || !voxel_phi)) || !sv_ptr)
        return fail(TITAN_EINVAL, "need n_voxels >= 0, voxel_a, voxel_phi and sv_ptr");
    if (n_voxels > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(TITAN_EINVAL, "too many voxels");
    if (s->params.actuation != TITAN_ACT_PHASOR)
        return fail(TITAN_ESTATE, "voxel actuation drives the phasor actuation law");
    if (sv_ptr[0] != 0)
        return fail(TITAN_EINVAL, "sv_ptr[0] must be 0");
    for (int64_t q = 0; q < ns; ++q)
        if (sv_ptr[q + 1] < sv_ptr[q])
            return fail(TITAN_EINVAL, "sv_ptr decreases at spring %lld", (long long)q);
    const int64_t nidx = sv_ptr[ns];
    if (nidx > 0 && !sv_idx)
        return fail(TITAN_EINVAL, "sv_idx is required");
    for (int64_t e = 0; e < nidx; ++e)
        if (sv_idx[e] < 0 || sv_idx[e] >= n_voxels)
            return fail(TITAN_EINVAL, "voxel index %d out of range [0, %lld)", sv_idx[e], (long long)n_voxels);
    for (int64_t v = 0; v < n_voxels; ++v)
        if (!(std::isfinite(voxel_a[v]) && std::isfinite(voxel_phi[v])))
            return fail(TITAN_EINVAL, "voxel %lld: non-finite actuation", (long long)v);
    for (int64_t q = 0; q < ns; ++q)
        for (int64_t e = sv_ptr[q] + 1; e < sv_ptr[q + 1]; ++e)
            if (sv_idx[e] == sv_idx[e - 1])
                return fail(TITAN_EINVAL, "spring %lld lists voxel %d twice", (long long)q, sv_idx[e]);
    invalidate_step_cache(s);
    // each voxel-driven spring's phasor: the mean of its voxels' a (cos phi,
    // sin phi), in FP64, stored in FP32
    std::vector<int64_t> changed;
    for (int64_t q = 0; q < ns; ++q) {
        const int64_t cnt = sv_ptr[q + 1] - sv_ptr[q];
        if (cnt == 0)
            continue;
        double c = 0.0, sn = 0.0;
        for (int64_t e = sv_ptr[q]; e < sv_ptr[q + 1]; ++e) {
            const double a = voxel_a[sv_idx[e]], ph = voxel_phi[sv_idx[e]];
            c += a * std::cos(ph);
            sn += a * std::sin(ph);
        }
        c /= (double)cnt;
        sn /= (double)cnt;
        s->h_C[q] = (float)c;
        s->h_S[q] = (float)sn;
        s->h_amp[q] = (float)std::hypot(c, sn);
        s->h_phase[q] = (float)std::atan2(sn, c);
        changed.push_back(q);
    }
    // the map, turned around: each voxel's springs in ascending order
    s->h_vox_a.assign(voxel_a, voxel_a + n_voxels);
    s->h_vox_phi.assign(voxel_phi, voxel_phi + n_voxels);
    s->h_sv_count.assign(ns, 0);
    s->h_vs_ptr.assign(n_voxels + 1, 0);
    for (int64_t e = 0; e < nidx; ++e)
        ++s->h_vs_ptr[sv_idx[e] + 1];
    for (int64_t v = 0; v < n_voxels; ++v)
        s->h_vs_ptr[v + 1] += s->h_vs_ptr[v];
    s->h_vs_spring.assign(nidx, 0);
    {
        std::vector<int64_t> fill(s->h_vs_ptr.begin(), s->h_vs_ptr.end() - 1);
        for (int64_t q = 0; q < ns; ++q) {
            s->h_sv_count[q] = (int32_t)(sv_ptr[q + 1] - sv_ptr[q]);
            for (int64_t e = sv_ptr[q]; e < sv_ptr[q + 1]; ++e)
                s->h_vs_spring[fill[sv_idx[e]]++] = (int32_t)q;
        }
    }
    if (!s->finalized || changed.empty())
        return TITAN_OK;
    if (int rc = ready(s))
        return rc;
    return update_spring_list(s, changed, false, false, true, false);
}

// Centre-of-mass displacement, the host part shared by both entry points:
// the body runs of the internal order (bodies are contiguous, largest first)
// and each mass's weight m_i / M_b in internal order.
struct BodyRuns {
    int32_t nb = 0;                  // body ids 0 .. nb - 1
    std::vector<int64_t> off{0};     // run r = internal masses [off[r], off[r+1])
    std::vector<int32_t> rank_body;  // body id of run r
    std::vector<float> w;            // per internal mass
};

static void body_runs(const titan_sim *s, BodyRuns &r)
{
    const int64_t n = s->n;
    for (int32_t b : s->h_body)
        r.nb = std::max(r.nb, b + 1);
    for (int64_t a = 0; a < n;) {
        const int32_t bd = s->h_body[s->perm[a]];
        int64_t b = a + 1;
        while (b < n && s->h_body[s->perm[b]] == bd)
            ++b;
        r.rank_body.push_back(bd);
        r.off.push_back(b);
        a = b;
    }
    std::vector<double> mt(r.nb, 0.0);
    for (int64_t u = 0; u < n; ++u)
        mt[s->h_body[u]] += (double)s->h_mass[u];
    r.w.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t u = s->perm[i];
        const double m = mt[s->h_body[u]];
        r.w[i] = m > 0.0 ? (float)((double)s->h_mass[u] / m) : 0.f;
    }
}

// Device part: weights and run offsets copied into dw / doff, the per-run
// sums into dd (3 floats per run), read back and scattered to disp by body id.
static hipError_t body_disp_device(titan_sim *s, const BodyRuns &r, float *dw, int64_t *doff, float *dd,
                                   float *disp)
{
    const int64_t n = s->n, nr = (int64_t)r.rank_body.size();
    std::vector<float> h(3 * nr);
    hipError_t e = hipSuccess;
    if (n)
        e = hipMemcpyAsync(dw, r.w.data(), sizeof(float) * n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(doff, r.off.data(), sizeof(int64_t) * (nr + 1), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = launch_body_disp(s->U[s->cur], dw, doff, nr, dd, s->stream);
    if (e == hipSuccess && nr)
        e = hipMemcpyAsync(h.data(), dd, sizeof(float) * 3 * nr, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess)
        return e;
    for (int32_t b = 0; b < r.nb; ++b)
        disp[3 * b] = disp[3 * b + 1] = disp[3 * b + 2] = 0.f;
    for (int64_t q = 0; q < nr; ++q)
        for (int c = 0; c < 3; ++c)
            disp[3 * r.rank_body[q] + c] = h[3 * q + c];
    return hipSuccess;
}

extern "C" int titan_get_body_displacement(titan_sim *s, float *disp)
{
    if (!s || !disp)
        return fail(TITAN_EINVAL, "sim or disp is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (int rc = ready(s))
        return rc;
    BodyRuns r;
    body_runs(s, r);
    if (r.nb == 0)
        return TITAN_OK;
    const int64_t n = s->n, nr = (int64_t)r.rank_body.size();
    float *dw = nullptr, *dd = nullptr;
    int64_t *doff = nullptr;
    if (int rc = dev_alloc(s, sizeof(float) * std::max<int64_t>(n, 1), (void **)&dw))
        return rc;
    if (int rc = dev_alloc(s, sizeof(float) * 3 * std::max<int64_t>(nr, 1), (void **)&dd)) {
        dev_free(s, dw);
        return rc;
    }
    if (int rc = dev_alloc(s, sizeof(int64_t) * (nr + 1), (void **)&doff)) {
        dev_free(s, dw);
        dev_free(s, dd);
        return rc;
    }
    const hipError_t e = body_disp_device(s, r, dw, doff, dd, disp);
    dev_free(s, dw);
    dev_free(s, dd);
    dev_free(s, doff);
    if (e != hipSuccess)
        return hip_fail(s, e, "body displacement");
    return check_bad(s);
}

// ---- the same without allocating ---------------------------------------------
// A file-scope device array holds what titan_get_body_displacement allocates
// per call (run offsets, per-run sums, per-mass weights), sized for at most
// kScratchMaxMasses masses in kScratchMaxBodies body runs.  Each device the
// library runs on holds its own copy until the process ends; its address on
// a device comes from hipGetSymbolAddress, taken once per device with that
// device current (the array's name in host code is not a device address).
constexpr int64_t kScratchMaxMasses = (int64_t)1 << 22;  // 4,194,304
constexpr int64_t kScratchMaxBodies = (int64_t)1 << 16;  // 65,536
constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr size_t kScratchOffBytes = align_up(sizeof(int64_t) * (kScratchMaxBodies + 1));
constexpr size_t kScratchSumBytes = align_up(sizeof(float) * 3 * kScratchMaxBodies);
constexpr size_t kScratchBytes = kScratchOffBytes + kScratchSumBytes + sizeof(float) * kScratchMaxMasses;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;  // guards g_scratch and serialises the calls that use the array
static void *g_scratch[kMaxDevices] = {};

// The array's address on the current device (looked up once per device).
static int scratch_on(int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(TITAN_EDEVICE, "device %d beyond the %d devices the scratch table covers", device, kMaxDevices);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(TITAN_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                        hipGetErrorString(e));
        }
        g_scratch[device] = p;
    }
    *out = (unsigned char *)g_scratch[device];
    return TITAN_OK;
}

extern "C" int titan_get_body_displacement_noalloc(titan_sim *s, float *disp)
{
    if (!s || !disp)
        return fail(TITAN_EINVAL, "sim or disp is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->dev_error)
        return fail(TITAN_EDEVICE, "sim is in a failed device state");
    if (!s->finalized)
        return fail(TITAN_ESTATE, "the sim has no device state yet (titan_finalize or titan_step first)");
    HIP_TRY(s, hipSetDevice(s->device));
    BodyRuns r;
    body_runs(s, r);
    if (r.nb == 0)
        return TITAN_OK;
    const int64_t nr = (int64_t)r.rank_body.size();
    if (s->n > kScratchMaxMasses || nr > kScratchMaxBodies)
        return fail(TITAN_EINVAL, "%lld masses in %lld bodies exceed this call's limit of %lld masses and %lld bodies",
                    (long long)s->n, (long long)nr, (long long)kScratchMaxMasses, (long long)kScratchMaxBodies);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    unsigned char *base = nullptr;
    if (int rc = scratch_on(s->device, &base))
        return rc;
    int64_t *doff = (int64_t *)base;
    float *dd = (float *)(base + kScratchOffBytes);
    float *dw = (float *)(base + kScratchOffBytes + kScratchSumBytes);
    const hipError_t e = body_disp_device(s, r, dw, doff, dd, disp);
    if (e != hipSuccess)
        return hip_fail(s, e, "body displacement");
    return check_bad(s);
}

// What every rollout-gradient entry point refuses, then the layout made
// current (caller holds the lock).
static int rollout_ready(titan_sim *s)
{
    if (s->params.actuation != TITAN_ACT_PHASOR)
        return fail(TITAN_ESTATE, "the rollout adjoint covers phasor actuation only");
    if (s->params.integrator != TITAN_INTEG_EULER)
        return fail(TITAN_ESTATE, "the rollout adjoint covers the Euler integrator only");
    if (!s->h_yield.empty())
        return fail(TITAN_ESTATE, "the rollout adjoint covers unbreakable springs only");
    if (int rc = ready(s))
        return rc;
    return ensure_layout(s);
}

extern "C" int titan_rollout_grad(titan_sim *s, int64_t nsteps, int32_t checkpoint_every, const float *body_weights,
                                  float *loss_out, float *grad_k, float *grad_act_c, float *grad_act_s)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (int rc = rollout_ready(s))
        return rc;
    return rollout_grad(s, nsteps, checkpoint_every, body_weights, loss_out, grad_k, grad_act_c, grad_act_s);
}

extern "C" int titan_rollout_grad_device(titan_sim *s, int64_t nsteps, int32_t checkpoint_every,
                                         const float *body_weights, float *loss_out, float *grad_k,
                                         float *grad_act_c, float *grad_act_s)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (int rc = rollout_ready(s))
        return rc;
    // every output given must be device memory of the simulation's GPU
    for (const float *p : {(const float *)loss_out, (const float *)grad_k, (const float *)grad_act_c,
                           (const float *)grad_act_s}) {
        if (!p)
            continue;
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, p) != hipSuccess) {
            (void)hipGetLastError();
            return fail(TITAN_EINVAL, "an output is not device memory");
        }
        if (at.type != hipMemoryTypeDevice || at.device != s->device)
            return fail(TITAN_EINVAL, "an output is not device memory of the simulation's GPU");
    }
    return rollout_grad(s, nsteps, checkpoint_every, body_weights, loss_out, grad_k, grad_act_c, grad_act_s,
                        nullptr, nullptr, true);
}

extern "C" int titan_rollout_grad_voxel(titan_sim *s, int64_t nsteps, int32_t checkpoint_every,
                                        const float *body_weights, float *loss_out, float *grad_k,
                                        float *grad_voxel_a, float *grad_voxel_phi)
{
    if (!s)
        return fail(TITAN_EINVAL, "sim is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->h_vs_ptr.empty())
        return fail(TITAN_ESTATE, "no voxel actuation (titan_set_voxel_actuation)");
    if (int rc = rollout_ready(s))
        return rc;
    std::vector<float> ga(s->h_vox_a.size()), gp(s->h_vox_a.size());
    if (int rc = rollout_grad(s, nsteps, checkpoint_every, body_weights, loss_out, grad_k, nullptr, nullptr,
                              ga.data(), gp.data()))
        return rc;
    if (grad_voxel_a)
        std::copy(ga.begin(), ga.end(), grad_voxel_a);
    if (grad_voxel_phi)
        std::copy(gp.begin(), gp.end(), grad_voxel_phi);
    return TITAN_OK;
}

extern "C" int titan_get_info(titan_sim *s, titan_info *info)
{
    if (!s || !info)
        return fail(TITAN_EINVAL, "sim or info is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(info, 0, sizeof *info);
    info->n_masses = (int64_t)s->h_mass.size();
    info->n_springs = (int64_t)s->h_k.size();
    int32_t maxb = -1;
    for (int32_t b : s->h_body)
        maxb = std::max(maxb, b);
    info->n_bodies = maxb < 0 ? 1 : (int64_t)maxb + 1;
    info->step = s->step_enq;
    info->steps_requested = s->steps_req;
    info->first_bad_step = s->first_bad_step;
    info->finalized = s->finalized;
    info->engine = s->finalized ? s->engine : s->params.engine;
    info->device = s->device;
    info->paused = s->paused;
    info->device_bytes = s->device_bytes;
    info->batch_threads = batch_threads(s);
    info->tune_batch_ms = s->tune_batch_ms;
    info->tune_gather_ms = s->tune_gather_ms;
    info->slack = s->slack;
    info->layout_builds = s->layout_builds;
    info->springs_in_place = s->springs_in_place;
    if (s->batch) {
        info->batch_groups = batch_layout(s).n_groups;
        info->batch_max_group = batch_layout(s).max_group;
    }
    return TITAN_OK;
}

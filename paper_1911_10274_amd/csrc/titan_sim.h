// The titan_sim object and the engine interface of the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "titan.h"
#include "titan_internal.h"

namespace titan {

// Most spare slots per row that insertions after the first step grow the
// layouts to (each slot of slack costs a row slot of traffic per step).
constexpr int32_t kMaxSlack = 8;

struct BP {
    uint64_t id = 0;
    int64_t step = 0;
    int32_t kind = TITAN_BP_SNAPSHOT;
    bool fired = false;
    hipEvent_t ev = nullptr;
    float4 *snapU = nullptr;
    float4 *snapV = nullptr;
};

// The rollout gradient's spring-once tables (see AdjointIO), kept between
// calls for slot generation `gen` and the group offsets `goff`.
struct SpringOnceTables {
    uint64_t gen = 0;
    std::vector<int64_t> goff;
    int64_t nsp = 0;  // springs over all groups (0: no tables)
    int sp_max = 0;   // most springs in one group
    uint32_t *ends = nullptr;
    int64_t *slot = nullptr;       // each group spring's owner slot
    int64_t *off = nullptr;        // [groups + 1]
    int32_t *rev_sp = nullptr;     // [slots]
    int64_t *of_spring = nullptr;  // caller spring -> group spring (-1: no slot)
};

struct BatchEngine;  // defined by the batched engine
struct GatherPlan;   // host tables of the gather layout (engine_gather.hip)

}  // namespace titan

struct titan_sim {
    std::mutex mu;
    titan_params params{};
    hipStream_t stream = nullptr;
    hipStream_t side_stream = nullptr;
    titan_allocator alloc{};

    // host staging, caller order
    std::vector<float> h_pos, h_vel, h_mass;
    std::vector<int32_t> h_body;
    std::vector<int64_t> h_ends;
    std::vector<float> h_k, h_damp, h_rest, h_amp, h_phase;
    // phasor law: each spring's (C, S) = amp (cos phase, sin phase), rounded
    // to FP32 from FP64, or given directly (titan_set_springs_phasor, voxels)
    std::vector<float> h_C, h_S;
    // per-voxel actuation (titan_set_voxel_actuation): each voxel's amplitude
    // and phase, its springs in ascending order, and per spring the number of
    // voxels that drive it (0: not voxel-driven).  Empty: no voxel map.
    std::vector<float> h_vox_a, h_vox_phi;
    std::vector<int64_t> h_vs_ptr;
    std::vector<int32_t> h_vs_spring;
    std::vector<int32_t> h_sv_count;

    // device state
    bool finalized = false;
    bool dev_error = false;
    int device = 0;
    int engine = TITAN_ENGINE_GATHER;
    struct Allocation {
        void *p;
        size_t bytes;
        bool engine;  // part of an engine's layout (freed when the layout is rebuilt)
    };
    std::vector<Allocation> allocations;
    int64_t device_bytes = 0;
    bool engine_allocs = false;  // dev_alloc marks new allocations as the engine's
    int64_t n = 0, ns = 0;
    std::vector<int64_t> perm;      // perm[internal] = caller index
    std::vector<int64_t> inv_perm;  // inv_perm[caller] = internal index (empty: identity)
    std::vector<float4> hX0;        // reference positions, internal order
    float4 *U[2] = {nullptr, nullptr};
    float4 *V[2] = {nullptr, nullptr};
    float4 *X0 = nullptr;
    float4 *F = nullptr;
    int cur = 0;
    unsigned long long *first_bad = nullptr;
    float4 *host_stage = nullptr;  // pinned, 2*n float4

    // gather engine
    titan::GatherGraph gg{};
    bool tiled = false;  // gather engine runs the LDS-tiled kernel
    int64_t n_slots = 0;  // incidence slots of the gather layout
    std::vector<int32_t> h_slot_nbr;  // per-slot neighbour (internal), kept only during finalize
    std::vector<int64_t> h_owner_slot;  // per spring (caller order): its slot at the lower-index end
    std::vector<int64_t> h_other_slot;  // per spring: its slot at the other end
    // bumped whenever springs get slots (layout built, springs inserted):
    // what the rollout gradient keeps between calls is rebuilt after that
    uint64_t slot_gen = 1;
    // device copy of h_owner_slot for the rollout gradient, kept between
    // calls (valid for slot generation d_owner_gen)
    int64_t *d_owner_slot = nullptr;
    int64_t d_owner_cap = 0;
    uint64_t d_owner_gen = 0;
    titan::SpringOnceTables once;
    float2 *trig = nullptr;           // clock table: kTrigChunk entries + 1 for force queries
    std::shared_ptr<titan::GatherPlan> gplan;  // planned before the device was set up; used once

    // topology edits after finalize: the engines' layouts are rebuilt before
    // the next step when dirty; removed springs stay in the spring table
    bool layout_dirty = false;
    std::vector<uint8_t> h_removed;  // per spring (empty: none removed)
    int32_t slack = 0;               // spare slots per row (grown by edits, up to kMaxSlack)
    // host copies of the current layout, for insertions in place
    std::vector<int32_t> h_deg;        // incidences per mass (internal order)
    std::vector<int64_t> h_slice_off;  // sliced-ELL offsets
    std::vector<int64_t> h_halo_off;   // tiled layout: halo lists
    std::vector<int32_t> h_halo_idx;
    std::vector<int64_t> h_group_off;  // batched layout: group ranges (empty: none)
    std::vector<float> h_yield;    // per spring: yield value (+inf: never breaks); empty: none
    std::vector<uint8_t> h_broken; // per spring: broken (as of the last sync_broken)
    // staged integrators: RK4 stage states (two ping-pong pairs) and sums,
    // Verlet's carried acceleration; sized for stage_n masses
    float4 *stage_buf[6] = {};
    float4 *verlet_acc[2] = {};    // ping-pong: the kick reads one, writes the other
    int acc_cur = 0;
    int64_t stage_n = 0;
    // captured step loops (params.graph_steps > 0): one graph per parity of
    // cur, replayed from the device clock d_clock
    hipGraphExec_t step_graph[2] = {};
    int64_t *d_clock = nullptr;
    int64_t clock_host = -1;       // d_clock after the queued work (-1: unknown)
    hipStream_t capture_stream = nullptr;
    bool acc_valid = false;        // verlet_acc[acc_cur] holds the current state's acceleration
    int64_t layout_builds = 0;     // times the layouts were built
    int64_t springs_in_place = 0;  // springs inserted into spare slots

    // batched engine (null unless selected) and the tuner's measurements
    titan::BatchEngine *batch = nullptr;
    bool batch_step = false;  // the batched engine steps the system
    float tune_batch_ms = 0.f;   // per step, best batched workgroup size
    float tune_gather_ms = 0.f;  // per step, gather engine (AUTO only)

    // step queue and breakpoints
    int64_t step_enq = 0;
    int64_t steps_req = 0;
    bool paused = false;
    uint64_t next_bp = 0;
    std::map<uint64_t, titan::BP> bps;
    int64_t first_bad_step = -1;

    int64_t inv_perm_of(int64_t caller) const { return inv_perm.empty() ? caller : inv_perm[caller]; }
};

namespace titan {

int fail(int code, const char *fmt, ...);
int hip_fail(titan_sim *sim, hipError_t e, const char *what);
int dev_alloc(titan_sim *s, size_t bytes, void **out);
void dev_free(titan_sim *s, void *p);
void dev_free_engine(titan_sim *s);
int batch_threads(const titan_sim *s);
int update_springs(titan_sim *s, int64_t first, int64_t count, const float *k, const float *damping,
                   const float *amp, const float *phase);
// Same for a list of springs; the flags say which constants changed.  force:
// write per-slot arrays even where the values stay uniform (removal).
int update_spring_list(titan_sim *s, const std::vector<int64_t> &springs, bool k, bool damping, bool amp,
                       bool force);
// The rollout adjoint; with gvox_a / gvox_phi (either non-null) also the
// gradients of the per-voxel actuation (the sim's voxel map must be set).
// With dev_out, loss / gk / gC / gS are device pointers (no voxel outputs).
int rollout_grad(titan_sim *s, int64_t nsteps, int32_t K, const float *body_weights, float *loss, float *gk,
                 float *gC, float *gS, float *gvox_a = nullptr, float *gvox_phi = nullptr, bool dev_out = false);

// Engines (engine_gather.hip): build the device representation of the
// selected engine after the state buffers exist, enqueue steps, compute the
// spring-force sum, and release engine-private resources.
void plan_order(titan_sim *s);  // fills perm (internal -> caller)
// Host planning of the first layouts (n, ns, perm, inv_perm, the gather
// layout's tables), without the device; build_engines then uploads them.
void plan_layouts(titan_sim *s);
int build_engines(titan_sim *s);
int enqueue_steps(titan_sim *s, int64_t first_step, int64_t count);
int compute_forces(titan_sim *s);
StepConsts consts_for(const titan_sim *s, int64_t step, const float2 *trig);
void destroy_engines(titan_sim *s);
// Place springs [first, first + count) (already in the host tables) into spare
// slots of the current layouts, O(1) per spring.  Returns 0 when all were
// placed; 1 if some row has no spare slot left, 2 if some spring does not fit
// the layout otherwise (in both cases nothing is written and the layouts must
// be rebuilt); or an error code (< 0).
int insert_springs(titan_sim *s, int64_t first, int64_t count);
// The batched engine's layout (s->batch must be set).
const BatchLayout &batch_layout(const titan_sim *s);
// Allocate the staged integrators' buffers for the current masses (RK4's
// stage states and sums, or Verlet's acceleration pair).
int ensure_stage_buffers(titan_sim *s, bool rk4);
// Something the step launches depend on changed: a carried Verlet
// acceleration is recomputed and captured step loops are captured again.
void invalidate_step_cache(titan_sim *s);
// Release the captured step loops and their stream (titan_destroy).
void destroy_step_graphs(titan_sim *s);
// Copy the breaks the steps have recorded into h_broken (and h_removed);
// waits for the stream.
int sync_broken(titan_sim *s);
// Write h_yield of the listed springs into the current layout.
int update_yield(titan_sim *s, const std::vector<int64_t> &springs);
// Device array of the batched layout's group-relative neighbour indices
// (null without a batched layout).
// The batched layout's tables of wave-law offsets are dropped (the kernel
// then evaluates every slot's offset itself), e.g. after springs were
// inserted in place with offsets the tables do not hold.
void batch_drop_wave_tables(titan_sim *s);
uint16_t *batch_nbr_group(titan_sim *s);
// Rebuild the engines' layouts for the current topology, keeping the state,
// the internal order and every device buffer that is not an engine's.
int rebuild_engines(titan_sim *s);

}  // namespace titan

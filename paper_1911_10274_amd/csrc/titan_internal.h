// Internal declarations shared by the host runtime and the kernel translation
// units of libtitan.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace titan {

// Width of a sliced-ELL slice: one wavefront of masses.
constexpr int kSlice = 64;

// Per-step scalars.  The actuation clock (sin, cos)(omega * t_n),
// t_n = n * dt, is read from a device table filled in FP64 by
// launch_trig_table, so every engine uses the same FP32 values.
struct StepConsts {
    float dt;
    float gx, gy, gz;
    float ground_k;
    float mu;
    int32_t ground;
    const float2 *trig;  // entry of this step (gather engines) or of the chunk's first step (batched)
    int64_t step;        // step index n (first step of the chunk, batched)
    double dt64;         // dt in FP64: the wave law's clock t_n = n * dt64
    double period;       // wave law: period t_p
    double omega;        // wave law: angular frequency
    double t_add;        // added to n * dt64 (an RK4 stage's time offset c * dt)
    int32_t stage;       // integrator stage of a staged launch (kStage*)
    const int64_t *clock;  // non-null in a captured step loop: n = *clock + step
};

// The step index n of a gather-engine launch.
__device__ __forceinline__ int64_t step_index(const StepConsts &sc) { return sc.clock ? *sc.clock + sc.step : sc.step; }

// Stages of the other integrators (Sec. III-B names Verlet and RK4): one
// gather launch each, selected by StepConsts::stage.
constexpr int32_t kStageRk1 = 1;         // RK4 stages 1-3: sums, next stage state
constexpr int32_t kStageRk4 = 4;         // RK4 stage 4: the new state (+ friction)
constexpr int32_t kStageVerletKick = 5;  // drift x' = x + v' dt, v' = v + a dt/2 of every mass read;
                                         // a' at (x', v'), v'' = v' + a' dt/2 (+ friction)
constexpr int32_t kStageVerletInit = 6;  // a at (x, v): the acceleration Verlet carries

// Largest number of steps whose clock entries one table holds.
constexpr int kTrigChunk = 4096;

// trig[s] = (sin, cos)(omega * (first + s) * dt) for s < count (FP64, rounded).
hipError_t launch_trig_table(float2 *trig, int64_t first, int count, double omega, double dt,
                             hipStream_t stream);
// The same with first = *clock (read on the device).
hipError_t launch_trig_table_clock(float2 *trig, const int64_t *clock, int count, double omega, double dt,
                                   hipStream_t stream);
// *clock = value, or with add != 0, *clock += add (stream order).
hipError_t launch_clock(int64_t *clock, int64_t value, int64_t add, hipStream_t stream);

// Masses per tile of the tiled kernel (one workgroup, one thread per mass).
// Compile-time tuning of the tiled kernel (overridable with -D for tuning
// builds): tile size, incidence slots whose loads are issued together
// (TITAN_UNROLL_PLAIN in the gather and tiled kernels for the phasor law with
// uniform damping, no per-slot rest lengths and no yields; TITAN_UNROLL
// everywhere else, where each slot carries more state), and non-temporal
// loads for the once-per-step streams of spring constants.
#ifndef TITAN_TILE
#define TITAN_TILE 512
#endif
#ifndef TITAN_UNROLL
#define TITAN_UNROLL 4
#endif
#ifndef TITAN_UNROLL_PLAIN
#define TITAN_UNROLL_PLAIN 8
#endif
#ifndef TITAN_NT_LOADS
#define TITAN_NT_LOADS 1
#endif
constexpr int kTile = TITAN_TILE;

// Device representation used by the gather engine.  Masses are in internal
// order; per-incidence arrays are sliced-ELL: the w-th incidence of the mass
// in lane l of slice s sits at slice_off[s] + w*64 + l.
struct GatherGraph {
    int64_t n;                 // masses
    int64_t n_slices;
    const int64_t *slice_off;  // [n_slices + 1]
    const int32_t *deg;        // [n] incidences of each mass
    const int32_t *nbr;        // [slots] internal index of the other end
    // Tiled layout: tile t holds masses [t*kTile, (t+1)*kTile); its halo is
    // halo_idx[halo_off[t] .. halo_off[t+1]) (internal indices).  Within a
    // tile, index q < kTile is mass t*kTile + q and kTile + h is halo entry h.
    const uint16_t *nbr_local;  // [slots] tile-local index of the other end, or null
    const int64_t *halo_off;    // [n_tiles + 1]
    const int32_t *halo_idx;
    int64_t n_tiles;
    int32_t max_local;          // max over tiles of kTile + halo size
    const float *k;            // [slots] stiffness, or null: k_uniform
    const float *c;            // [slots] damping, or null: c_uniform
    const float *act_c;        // [slots] amp*cos(phase), or null: no actuation
    const float *act_s;        // [slots] amp*sin(phase)
    const double *t_off;       // [slots] wave-law offsets t_o, or null: phasor law (act_s used)
    float *yield;              // [slots] yield values (< 0: broken; written by the step), or null
    const float *d0;           // [slots] |R| - rest (FP64-rounded), or null: rest = |R|
    const float *rest;         // [slots] rest length (with d0)
    const float4 *X0;          // [n] reference positions (w unused)
    // wave law, the kernel at hand's table of distinct offsets: per slot the
    // index of its spring's offset in that table, or null (each slot loads
    // its own offset).  Null in the layout itself; a kernel with a table
    // sets it in its own copy.
    const uint16_t *wave_cls;
    // tiled layout, wave law: each tile's distinct offsets (the tiled
    // kernel's table, as BatchLayout's wave_* for a group), or null
    const uint16_t *tile_wave_cls;  // [slots]
    const int64_t *tile_wave_off;   // [n_tiles + 1]
    const double *tile_wave_t;
    int32_t max_tile_wave;
    float c_uniform;
    float k_uniform;
};

// State buffers: U = (x - x0, inverse mass), V = (v, 0).
struct StateIO {
    const float4 *U_in;
    const float4 *V_in;
    float4 *U_out;
    float4 *V_out;
    float4 *F_out;                   // forces-only mode: summed spring force
    unsigned long long *first_bad;   // min step index that produced a non-finite value
    // staged integrators: the step's starting state (own mass only), the
    // RK4 sums of weighted velocities / accelerations, Verlet's acceleration
    const float4 *U_base;
    const float4 *V_base;
    float4 *sum_u;
    float4 *sum_v;
    const float4 *A_in;  // Verlet: the carried acceleration of every mass
    float4 *A;           // Verlet: the new acceleration (own mass)
};

// dst[slot[q]] = val[q] for q < m; dst[q] = v for q < m.
hipError_t launch_scatter(float *dst, const int64_t *slot, const float *val, int64_t m, hipStream_t stream);
// The same for 16-, 32- and 64-bit elements (bit patterns).
hipError_t launch_scatter_bits(void *dst, int bytes, const int64_t *slot, const void *val, int64_t m,
                               hipStream_t stream);
hipError_t launch_fill(float *dst, float v, int64_t m, hipStream_t stream);
// disp[3b..3b+2] = sum over internal masses [off[b], off[b+1]) of w_i * u_i.xyz
hipError_t launch_body_disp(const float4 *U, const float *w, const int64_t *off, int64_t nb, float *disp,
                            hipStream_t stream);

// Batched engine: independent groups of whole bodies, each stepped by one
// workgroup with its state resident in LDS.  Group q owns internal masses
// [mass_off[q], mass_off[q+1]); nbr_group holds, per incidence slot of the
// gather layout, the neighbour's index relative to its group's first mass.
struct BatchLayout {
    int64_t n_groups;
    const int64_t *mass_off;     // [n_groups + 1]
    const uint16_t *nbr_group;   // [slots]
    int32_t max_group;           // masses of the largest group
    // Wave law: each group's distinct spring offsets t_o are
    // wave_t[wave_off[q] .. wave_off[q+1]) and a slot's offset is
    // wave_t[wave_off[q] + wave_cls[slot]]; every step the batched kernel
    // evaluates the wave's sine once per distinct offset.  Null when absent.
    const uint16_t *wave_cls;    // [slots]
    const int64_t *wave_off;     // [n_groups + 1]
    const double *wave_t;
    int32_t max_wave;            // most distinct offsets in a group
};

// Velocity Verlet / RK4 steps on the batched layout (batch_integ.hip):
// nsteps steps from io.U_in / V_in into io.U_out / V_out; Verlet reads its
// carried acceleration from io.A_in (acc_valid) or computes it, and writes it
// to io.A.  batch_integ_fits: whether the layout's groups fit the kernels.
bool batch_integ_fits(const BatchLayout &b, int integ);
// Whether TITAN_ENGINE_AUTO steps Verlet / RK4 with the batched kernels (small
// groups) rather than the per-step engines.
bool batch_integ_preferred(const BatchLayout &b);
hipError_t launch_batch_integ(const GatherGraph &g, const BatchLayout &b, const StateIO &io, const StepConsts &sc,
                              int nsteps, int integ, int acc_valid, hipStream_t stream);

// Threads per workgroup of the batched kernel (variants the tuner picks from).
constexpr int kBatchThreadChoices[] = {256, 512, 1024};

// Run `nsteps` steps (step indices step0 ..) of every group in one launch:
// state is read from io.U_in/V_in, kept in LDS, written to io.U_out/V_out.
// sc.trig points at the clock entry of step0.
hipError_t launch_batch(const GatherGraph &g, const BatchLayout &b, const StateIO &io, const StepConsts &sc,
                        int nsteps, int threads, hipStream_t stream);

// Buffers of one adjoint rollout (internal order, n = masses).
struct AdjointIO {
    const float4 *U0, *V0;    // starting state
    float4 *ckU, *ckV;        // [ceil(nsteps/K) * n] checkpoints (state at steps 0, K, 2K, ...)
    float4 *segU, *segV;      // [K * n] states of the segment being reversed
    float4 *segF;             // [K * n] summed spring force at those states (w unused)
    float4 *gslot;            // [slots] (dJ/dk, dJ/dC, dJ/dS, 0) on each spring's owner slot; zeroed
    const float *seed;        // [n] dJ/dx_N (x component)
    float *dux;               // [n] x-displacement over the rollout
    const float2 *trig;       // clock entries of rollout steps 0 .. nsteps-1
    unsigned long long *first_bad;
    int nsteps, K;
    // Reverse steps with every spring evaluated once (groups of at most 1024
    // masses; else sp_ends is null): group g's springs are
    // [sp_off[g], sp_off[g+1]), each with its ends (owner end, the lower
    // internal index, in the low 16 bits; group-local) and its constants
    // (k, c, C, S) and (d0, L0).  Per slot, rev_sp holds a mass's entries in
    // ascending order -- 2 * (the spring within its group), + 1 at the
    // spring's other end -- then INT32_MAX.  gsp: each spring's running
    // (dk, dC, dS).
    const uint32_t *sp_ends;
    const float4 *sp_kcs;
    const float2 *sp_rest;
    const int64_t *sp_off;
    const int32_t *rev_sp;
    float4 *gsp;
    int rev_chunk;   // records per chunk
    int once_bytes;  // LDS for the records beyond the state
};

// Per group spring t (AdjointIO's tables): kcs[t] = (k, c, C, S) and
// rest[t] = (d0, L0) (explicit rest lengths only; rest may be null otherwise)
// as load_const reads them from the owner slot sp_slot[t].
hipError_t launch_pack_spring_consts(const GatherGraph &g, const BatchLayout &b, const int64_t *sp_slot,
                                     const int64_t *sp_off, float4 *kcs, float2 *rest, hipStream_t stream);

hipError_t launch_adjoint(const GatherGraph &g, const BatchLayout &b, const AdjointIO &a, const StepConsts &sc,
                          hipStream_t stream);
// gk[s] = gslot[owner_slot[s]].x etc. (caller spring order; owner_slot < 0:
// no gradient).  The spring-once path passes its per-spring array and each
// spring's index in it.
hipError_t launch_spring_grads(const float4 *gslot, const int64_t *owner_slot, int64_t ns, float *gk, float *gC,
                               float *gS, hipStream_t stream);
// loss[b] = -sum over internal masses [body_off[b], body_off[b+1]) of coef * dux
hipError_t launch_voxel_grads(int64_t nv, const int64_t *vs_ptr, const int32_t *vs_spring, const float *inv_cnt,
                              const float4 *vw, const float *gC, const float *gS, float *ga, float *gphi,
                              hipStream_t stream);
hipError_t launch_body_loss(const float *dux, const float *coef, const int64_t *body_off, int64_t nb, float *loss,
                            hipStream_t stream);

// Launch one step (or, with forces_only, only the spring-force sum).  tiled:
// stage each tile's masses and halo in LDS (needs nbr_local); otherwise every
// neighbour is read from global memory.
hipError_t launch_gather_step(const GatherGraph &g, const StateIO &io, const StepConsts &sc,
                              bool forces_only, bool tiled, hipStream_t stream);
// Launch one integrator stage (sc.stage) over the state io.U_in / io.V_in.
hipError_t launch_gather_stage(const GatherGraph &g, const StateIO &io, const StepConsts &sc, bool tiled,
                               hipStream_t stream);

}  // namespace titan

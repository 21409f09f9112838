/*
 * titan.h -- C ABI of the MI355X mass-spring stepper.
 *
 * The library simulates a spring-mass system the way the Titan paper
 * (arXiv:1911.10274) describes it: every step applies Hooke's-law spring
 * forces to the masses (Sec. III-B, Eq. 1) and then integrates every mass
 * (Sec. III-B, Eq. 1's update dx = xdot*dt + xddot*dt^2, i.e. semi-implicit
 * Euler) under gravity and a penalty ground plane with friction (Sec. I and
 * Sec. III-A name plane constraints and friction).  Springs may be actuated by
 * scaling their rest length with 1 + amp*sin(omega*t + phase) (Sec. IV-B,
 * Eq. 4).  The host-side model of the paper's asynchronous CPU/GPU design
 * (Sec. III-D: a simulation that runs on its own until a breakpoint, a CPU
 * that blocks only when it asks to, edits pushed while the simulation is
 * paused) is kept as stream-ordered work plus breakpoints.
 *
 * Conventions for every call:
 *   - Arrays are plain host pointers unless a name ends in _dev (device
 *     pointer on the simulation's device).  Vectors are packed xyz triples
 *     ("n3" = n*3 floats, row-major).  Caller arrays are read or written
 *     during the call only; the library keeps no pointer to them.
 *   - Masses and springs are numbered in the order they were added, from 0.
 *     The library may store them internally in another order; every call
 *     that reads or writes per-mass data uses the caller's numbering.
 *   - Every call returns a status (TITAN_OK = 0 or a negative TITAN_E*);
 *     titan_last_error() then describes the failure of the last failing call
 *     on the calling thread.  No C++ exception crosses this interface.
 *   - A titan_sim is guarded by its own mutex: calls on one sim from several
 *     threads are serialised.  Calls on different sims are independent.
 */
#ifndef TITAN_H
#define TITAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TITAN_ABI_VERSION 8

/* Status codes. */
#define TITAN_OK 0
#define TITAN_EINVAL (-1)     /* bad argument: index out of range, i == j,
                                 zero-length spring, non-finite or negative
                                 input, size mismatch */
#define TITAN_ENOMEM (-2)     /* host or device allocation failed */
#define TITAN_EDEVICE (-3)    /* HIP error or no usable GPU; sticky: the sim
                                 refuses further stepping */
#define TITAN_ESTATE (-4)     /* call not valid in the sim's current phase
                                 (e.g. adding springs after the first step) */
#define TITAN_ENONFINITE (-5) /* the simulation produced a NaN or infinity;
                                 sticky, reported by titan_sync/titan_wait/
                                 titan_get_state; see titan_get_info */

/* Flags of titan_get_state / titan_set_state. */
#define TITAN_STATE_DISPLACEMENT 1 /* pos is x - x0 (x0 = initial position)
                                      instead of absolute x */

/* Breakpoint kinds (titan_set_breakpoint). */
#define TITAN_BP_SNAPSHOT 0 /* keep stepping; the state at the breakpoint
                               step is copied aside for titan_get_snapshot */
#define TITAN_BP_PAUSE 1    /* stop enqueuing steps at the breakpoint until
                               titan_resume (Sec. III-D's halted simulation);
                               also takes a snapshot */

/* Kernel selection (titan_params.engine). */
#define TITAN_ENGINE_AUTO 0    /* library chooses (autotuned) */
#define TITAN_ENGINE_GATHER 1  /* per-mass gather, one launch per step */
#define TITAN_ENGINE_BATCHED 2 /* one workgroup per group of independent
                                  bodies, their state resident in LDS, many
                                  steps per launch; needs body ids
                                  (titan_add_masses).  The tuner picks the
                                  workgroup size and how many bodies a group
                                  holds (up to 2048 masses when packing more
                                  than the largest body) by timing them */
#define TITAN_ENGINE_TILED 3   /* per-mass gather over LDS-staged tiles of
                                  spatially ordered masses, one launch per
                                  step (falls back to GATHER when a tile's
                                  neighbourhood does not fit in LDS) */

/* Actuation law of the rest lengths (titan_params.actuation); L0 is a
 * spring's base rest length and amp its amplitude (titan_add_springs). */
#define TITAN_ACT_PHASOR 0 /* L0 (1 + amp sin(omega t + phase)), t = n dt at
                              the start of step n (Sec. IV-B Eq. 4 with a
                              per-spring phase) */
#define TITAN_ACT_WAVE 1   /* the worm's travelling wave (Sec. IV-B Eqs. 3-5):
                              L0 (1 + amp sin(omega tau)), tau = (t - t_o) mod
                              wave_period taken in [0, wave_period); the
                              offset t_o of a spring is the smaller reference x
                              of its two ends minus the smallest reference x of
                              its body (Eq. 5), computed by the library; the
                              phase array is not used.  No rollout adjoint. */

typedef struct titan_sim titan_sim;

/* Simulation parameters (SI units).  Taken by value at each call that
 * passes them. */
/* Time integrators (Sec. III-B).  EULER: semi-implicit Euler, one force
 * evaluation per step (the default; every engine).  VERLET: velocity Verlet,
 * v' = v + a dt/2, x' = x + v' dt, a' = a(x', v', t + dt), v'' = v' + a' dt/2,
 * one force evaluation per step: the acceleration is carried from step to
 * step and recomputed from the current state after anything changes the
 * system or its state (edits, titan_set_state / _step / _params / _springs /
 * _yield); the end-of-step dampers see the half-step velocity v'.  RK4: the
 * classical four stages on (x, v) at t, t + dt/2, t + dt/2, t + dt, four
 * force evaluations per step.  Verlet and RK4 integrate springs, dampers,
 * gravity and the ground's normal force; Coulomb friction is applied after
 * the step as in the Euler step (normal force from the starting height), the
 * position moving by the velocity change times dt.  Every engine runs them
 * with identical results (the batched engine when its groups hold at most
 * 4096 masses for VERLET, 2048 for RK4; under TITAN_ENGINE_AUTO larger groups
 * step with a per-step engine); the rollout adjoint takes EULER only. */
#define TITAN_INTEG_EULER 0
#define TITAN_INTEG_VERLET 1
#define TITAN_INTEG_RK4 2

typedef struct titan_params {
    double dt;          /* time step, s (> 0) */
    double gravity[3];  /* m/s^2, e.g. {0, 0, -9.81} */
    int32_t ground;     /* nonzero: ground plane z = 0.  A mass with z < 0
                           feels -ground_k*z upward and Coulomb friction */
    int32_t engine;     /* TITAN_ENGINE_* */
    double ground_k;    /* ground penalty stiffness, N/m (>= 0) */
    double friction_mu; /* Coulomb friction coefficient (>= 0) */
    double omega;       /* actuation angular frequency, rad/s */
    int32_t actuation;  /* TITAN_ACT_*; fixed once the system is finalized */
    double wave_period; /* TITAN_ACT_WAVE: period t_p, s (> 0) */
    int32_t integrator; /* TITAN_INTEG_*: the time integrator (Sec. III-B
                           names Euler, Verlet and RK4) */
    int32_t graph_steps; /* 0, or an even number <= 4096: the gather and tiled
                            engines (Euler integrator) replay a captured HIP
                            graph of this many step launches, the step index
                            read from a device clock, for every whole group of
                            graph_steps steps of a titan_step call (the rest
                            launch one by one).  Same results bit for bit;
                            fewer host launches for small systems.  The graph
                            is captured again after anything that changes the
                            system or the parameters. */
} titan_params;

/* Optional device-memory provider.  alloc returns a device pointer aligned
 * to at least 256 bytes or NULL; release frees it.  Both are called with the
 * sim's mutex held, from the thread making the titan_* call.  With a NULL
 * allocator the library uses hipMalloc/hipFree. */
typedef struct titan_allocator {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*release)(void *ptr, void *ctx);
    void *ctx;
} titan_allocator;

/* Read-only facts about a sim (titan_get_info). */
typedef struct titan_info {
    int64_t n_masses;
    int64_t n_springs;
    int64_t n_bodies;        /* distinct body ids (1 if none were given) */
    int64_t step;            /* steps enqueued so far (the current step index) */
    int64_t steps_requested; /* steps asked for by titan_step so far */
    int64_t first_bad_step;  /* first step that produced a non-finite value, or -1 */
    int32_t finalized;       /* nonzero after the first titan_step */
    int32_t engine;          /* engine in use (TITAN_ENGINE_GATHER/TILED/BATCHED) */
    int32_t device;          /* HIP device ordinal */
    int32_t paused;          /* nonzero while held at a pause breakpoint */
    int64_t device_bytes;    /* device memory held by the sim */
    int32_t batch_threads;   /* workgroup size the tuner chose for the batched
                                engine (0 if it is not in use) */
    float tune_batch_ms;     /* tuner's time per step of the batched engine */
    float tune_gather_ms;    /* tuner's time per step of the gather engine
                                (measured only under TITAN_ENGINE_AUTO) */
    int32_t slack;           /* spare slots per row of the current layouts */
    int64_t layout_builds;   /* times the layouts were built (the first step,
                                then each rebuild after a topology edit) */
    int64_t springs_in_place; /* springs added after the first step that went
                                 into spare slots without a rebuild */
    int64_t batch_groups;     /* groups of the batched layout (0 if none) */
    int32_t batch_max_group;  /* masses in its largest group: the packing the
                                 tuner chose (bodies per group) */
} titan_info;

/* ABI version this library implements (TITAN_ABI_VERSION).  Library
 * bookkeeping, not in the paper. */
int titan_abi_version(void);

/* Message of the last failing call on the calling thread ("" if none).  The
 * pointer stays valid until the next titan_* call on this thread.  Error
 * reporting of this interface, not in the paper. */
const char *titan_last_error(void);

/* Create an empty sim (Sec. III-A: a simulation holds the masses, springs
 * and constraints that the library steps).  p: parameters (copied).  stream: a hipStream_t to
 * run on, or NULL for the device's null stream; the caller keeps it alive
 * until titan_destroy.  alloc: NULL or a device allocator (copied).  No device
 * work happens before the first titan_step.  *out receives the sim. */
int titan_create(const titan_params *p, void *stream, const titan_allocator *alloc, titan_sim **out);

/* Wait for the sim's queued work, free all its memory and the sim itself
 * (Sec. III-C: the objects live on the GPU until released).  NULL is
 * accepted. */
int titan_destroy(titan_sim *sim);

/* Append n masses (Sec. III-C: masses are the primitive objects springs act
 * on).  pos_n3: initial positions (m).  vel_n3: initial velocities (m/s) or
 * NULL for zero.  mass_n: kg, >= 0; 0 marks a pinned mass that never moves.
 * body_n: NULL, or the independent body each mass belongs to (>= 0); springs
 * may not join masses of different bodies.  *first_out (may be NULL) gets the
 * index of the first new mass.  After the first step (a topology edit,
 * Sec. III-C, applied from the next enqueued step on): the new masses start
 * with zero displacement from pos and must form new bodies (ids above every
 * existing id) or join the only body of a single-body system; the device
 * layout is rebuilt before the next step. */
int titan_add_masses(titan_sim *sim, int64_t n, const float *pos_n3, const float *vel_n3,
                     const float *mass_n, const int32_t *body_n, int64_t *first_out);

/* Append n springs (Sec. III-B).  ends_n2: mass index pairs (i, j), i != j,
 * both already added; the spring's initial length must be > 0.  k_n:
 * stiffness N/m (>= 0).  damping_n: axial damping N*s/m (>= 0) or NULL for 0.
 * rest_n: rest lengths (> 0) or NULL for the initial lengths.  amp_n,
 * phase_n: actuation (both or neither; Sec. IV-B Eq. 4): the rest length at
 * time t is rest * (1 + amp*sin(omega*t + phase)).  *first_out (may be NULL)
 * gets the first new spring's index.  After the first step (a topology edit,
 * Sec. III-C, applied from the next enqueued step on): a NULL rest length
 * means the distance between the ends after the steps already enqueued (the
 * call waits for them), which must be > 0.  The springs go into spare
 * slots of the current device layout, O(1) each, when all of them fit: both
 * rows have a free slot, the layout reaches the other end from each row, and
 * the spring's constants are representable there (a uniform stiffness or
 * damping it matches, actuation only where per-slot actuation exists,
 * per-slot rest lengths).  Otherwise the layout is rebuilt before the next
 * step, with more spare slots per row (2, doubled when a row ran out, at
 * most 8).  A spring inserted in place is summed after its rows' earlier
 * springs until a rebuild sorts it in.  A sim with breakable springs gives
 * the new springs an infinite yield value (titan_set_yield changes it). */
int titan_add_springs(titan_sim *sim, int64_t n, const int64_t *ends_n2, const float *k_n,
                      const float *damping_n, const float *rest_n, const float *amp_n,
                      const float *phase_n, int64_t *first_out);

/* Remove n springs (indices from titan_add_springs; repeats and springs
 * already removed are ignored) -- Sec. III-C's deletion.  Applies from the
 * next enqueued step on (while paused at a breakpoint: from the breakpoint
 * on).  The spring keeps its index; on a current device layout the removal
 * is O(1) per spring: its two incidence slots get k = 0 and no damping, so the
 * ends add an exact zero where its force was and every other result is
 * bitwise unchanged.  Layouts rebuilt later leave it out. */
int titan_remove_springs(titan_sim *sim, int64_t n, const int64_t *springs_n);

/* Yield values of springs [first, first + count) (Sec. III-E: per-spring
 * material yield values, tested in the force calculation, mark springs as
 * broken).
 * yield_count: > 0, or +inf for a spring that never breaks; springs never
 * given one have +inf.  A spring whose elastic force |k (l - L(t))| (damping
 * excluded) exceeds its yield value in a step's force evaluation breaks: it
 * exerts no force in that step and after, on every engine (both of its ends
 * take the same decision).  Breaks are permanent: a broken spring keeps its
 * state through later yield changes and is left out of rebuilt layouts, and
 * restoring positions (titan_set_state) does not restore it.  A system with
 * breakable springs keeps damping and rest lengths per incidence slot (more
 * traffic per step).  After the first step the new values apply from the
 * next enqueued step on (the call waits for the steps already enqueued).
 * The rollout adjoint refuses breakable springs (TITAN_ESTATE). */
int titan_set_yield(titan_sim *sim, int64_t first, int64_t count, const float *yield_count);

/* Broken flags (1 broken, 0 intact) of springs [first, first + count) after
 * the steps enqueued so far (waits for them); Sec. III-E's yield test.
 * Springs of a sim without yield values are never broken. */
int titan_get_broken(titan_sim *sim, int64_t first, int64_t count, uint8_t *broken_count);

/* Remove n masses (Sec. III-C's deletion of masses): every spring touching
 * them is removed (as above) and the masses stay where they are, pinned
 * (mass 0) and at rest.  Indices are kept.
 * Cost O(springs) to find the touching springs. */
int titan_remove_masses(titan_sim *sim, int64_t n, const int64_t *masses_n);

/* Replace the parameters (Sec. III-A: time resolution, gravity, plane
 * constraint and friction; Sec. III-D: updates queued while the simulation
 * runs are applied when it stops).  Takes effect for steps enqueued after
 * this call (while paused at a breakpoint: from the breakpoint on).  The engine field
 * may change only before the first step; afterwards it must be
 * TITAN_ENGINE_AUTO or the engine first asked for. */
int titan_set_params(titan_sim *sim, const titan_params *p);

/* Build the device representation now (otherwise done by the first
 * titan_step): validation, internal ordering, incidence lists, upload and
 * engine selection (Sec. III-B: each mass's springs in a fixed order for the
 * accumulation-based sum; Sec. III-C: all components reside on the GPU). */
int titan_finalize(titan_sim *sim);

/* Ask for n more steps (n >= 0) of the spring pass and the mass update
 * (Sec. III-B, Eq. 1).  Asynchronous (Sec. III-D: the GPU keeps stepping
 * while the CPU runs freely): work is enqueued on the sim's stream and the
 * call returns; step n of the run uses t = n*dt.  Steps
 * beyond a pause breakpoint are held until titan_resume. */
int titan_step(titan_sim *sim, int64_t n);

/* Breakpoint at absolute step index `step` (the state after `step` steps),
 * which must not be behind the steps already enqueued (Sec. III-D's
 * setBreakpoint).  kind: TITAN_BP_*.
 * *bp_out receives a handle for titan_wait / titan_get_snapshot. */
int titan_set_breakpoint(titan_sim *sim, int64_t step, int32_t kind, uint64_t *bp_out);

/* Block until breakpoint bp has been reached on the GPU (Sec. III-D's
 * waitForEvent).  Returns TITAN_ESTATE if bp will never be reached with the
 * steps requested so far. */
int titan_wait(titan_sim *sim, uint64_t bp);

/* Release a pause breakpoint and enqueue the held steps (Sec. III-D: a CPU
 * thread reactivates the halted simulation). */
int titan_resume(titan_sim *sim);

/* Block until all enqueued work is done; reports non-finite state
 * (Sec. III-D: the CPU blocks only when it issues a blocking call). */
int titan_sync(titan_sim *sim);

/* Copy the state of masses [first, first+count) after all enqueued steps
 * (blocks until they are done; Sec. III-D: copies from the GPU happen when
 * the simulation has stopped).  pos_n3 / vel_n3 may be NULL.  flags:
 * TITAN_STATE_DISPLACEMENT.  *step_out (may be NULL) gets the step index. */
int titan_get_state(titan_sim *sim, int64_t first, int64_t count, float *pos_n3, float *vel_n3,
                    int32_t flags, int64_t *step_out);

/* Copy the state saved at breakpoint bp (blocks until it is reached), while
 * later steps may still be running (Sec. III-D's results read at a
 * breakpoint). */
int titan_get_snapshot(titan_sim *sim, uint64_t bp, int64_t first, int64_t count, float *pos_n3,
                       float *vel_n3, int32_t flags, int64_t *step_out);

/* Overwrite the state of masses [first, first+count), in stream order: it
 * applies after the steps enqueued so far (at the breakpoint if paused;
 * Sec. III-D: state pushed to the GPU while the simulation is stopped).
 * pos_n3 / vel_n3 may be NULL to keep that part.  With
 * TITAN_STATE_DISPLACEMENT pos is x - x0. */
int titan_set_state(titan_sim *sim, int64_t first, int64_t count, const float *pos_n3,
                    const float *vel_n3, int32_t flags);

/* Set the step index of the next step to `step` (>= 0); the time of step n
 * is n*dt.  Together with titan_set_state this restores a checkpoint taken
 * with titan_get_state (Sec. III-D: state pushed while the simulation is
 * stopped).  Only when no steps are held at a pause breakpoint. */
int titan_set_step(titan_sim *sim, int64_t step);

/* Centre-of-mass displacement of every body after all enqueued steps
 * (blocks; Sec. IV-B/IV-C measure locomotion by how far a body moves):
 * disp_nb3[b] = sum_i m_i (x_i - x0_i) / M_b over the masses of
 * body b (n_bodies x 3 floats). */
int titan_get_body_displacement(titan_sim *sim, float *disp_nb3);

/* titan_get_body_displacement for callers that cannot allocate device memory
 * (code under HIP graph capture, tight control loops, harnesses that forbid
 * hipMalloc): same result, bit for bit, with no hipMalloc, hipFree or
 * allocator call.  Its device work uses a fixed array inside the library
 * (about 17 MiB per device, held until the process ends) instead of per-call
 * buffers, so the system is limited to 4,194,304 masses and 65,536 bodies
 * (TITAN_EINVAL beyond).  The sim must already have its device state
 * (TITAN_ESTATE before titan_finalize or the first titan_step).  Calls are
 * serialised within the process (the array is shared by every sim on a
 * device); another process has its own array.  Blocks until the result is
 * on the host. */
int titan_get_body_displacement_noalloc(titan_sim *sim, float *disp_nb3);

/* Change the constants of springs [first, first+count): k, damping and
 * actuation (amp with phase), each array NULL to keep that part (the paper's
 * Sec. IV-D pushes spring constants from the CPU into a running
 * simulation).  In stream order: applies to steps enqueued after the call
 * (while paused: from the breakpoint on).  Same value rules as
 * titan_add_springs. */
int titan_set_springs(titan_sim *sim, int64_t first, int64_t count, const float *k_n, const float *damping_n,
                      const float *amp_n, const float *phase_n);

/* Set the actuation phasor of springs [first, first + count) directly
 * (Sec. IV-B Eq. 4 with a per-spring phase, written as a phasor): the rest
 * length at time t becomes rest (1 + C sin(omega t) + S cos(omega t)) with
 * C = act_c[q], S = act_s[q] exactly as given (titan_set_springs takes amp
 * and phase and rounds C = amp cos(phase), S = amp sin(phase) to FP32).
 * Phasor law only (TITAN_ESTATE under the wave law); values must be finite.
 * In stream order like titan_set_springs.  Ends the voxel map of
 * titan_set_voxel_actuation if a listed spring was voxel-driven. */
int titan_set_springs_phasor(titan_sim *sim, int64_t first, int64_t count, const float *act_c,
                             const float *act_s);

/* Per-voxel actuation (Sec. IV-C drives a swarm's bodies by their own
 * actuation parameters; here each voxel of a voxel robot has an amplitude
 * and a phase).  n_voxels voxels with amplitude voxel_a[v] and phase
 * voxel_phi[v]; sv_ptr (n_springs + 1 entries, sv_ptr[0] = 0, non-decreasing)
 * and sv_idx list, for each spring s, the voxels sv_idx[sv_ptr[s] ..
 * sv_ptr[s+1]) that contain it (each at most once).  A spring with a
 * non-empty list gets the mean of its voxels' phasors a (cos phi, sin phi)
 * (computed in FP64, stored in FP32) as its actuation phasor; springs with
 * an empty list keep theirs.  The map is kept for titan_rollout_grad_voxel
 * until a call changes a voxel-driven spring's actuation directly; springs
 * added later are not voxel-driven.  Phasor law only (TITAN_ESTATE
 * otherwise); TITAN_EINVAL for malformed lists or non-finite values.  In
 * stream order like titan_set_springs. */
int titan_set_voxel_actuation(titan_sim *sim, int64_t n_voxels, const float *voxel_a, const float *voxel_phi,
                              const int64_t *sv_ptr, const int32_t *sv_idx);

/* Gradient of a rollout by the adjoint method (not in the paper; Sec. II
 * names differentiable simulation as related work): backward in time through
 * the steps, with the forward states recomputed from checkpoints taken every
 * `checkpoint_every` steps (memory: one state per checkpoint plus one
 * segment of states and spring forces, 48 bytes per mass per step; the last
 * segment is kept by the forward pass itself, so checkpoint_every >= nsteps
 * recomputes nothing).  The rollout starts from the current state (after all
 * enqueued steps) at the current step index and runs `nsteps` steps; the
 * simulation itself is not advanced.  Loss: J = sum_b w_b J_b with
 * J_b = -(x-displacement of the centre of mass of body b), the
 * mass-weighted mean over the body's masses.  body_weights: w_b per body
 * (n_bodies values) or NULL for all 1.  Outputs (each may be NULL):
 * loss_out[n_bodies] = J_b; grad_k[n_springs] = dJ/dk; grad_act_c and
 * grad_act_s[n_springs] = dJ/dC and dJ/dS for the actuation phasor
 * C = amp cos(phase), S = amp sin(phase) (the rest length at time t is
 * rest (1 + C sin(omega t) + S cos(omega t))).  Needs every body to fit the
 * batched engine's layout (TITAN_ESTATE otherwise); TITAN_ENONFINITE if the
 * rollout blows up.  Differentiates the step exactly as computed, contact
 * and friction included (their switches are not smoothed).  When the
 * largest group of the batched layout holds at most 1024 masses, the
 * reverse steps evaluate each spring once and share its terms between its
 * two ends (the forward states are those of every engine, bit for bit; the
 * gradients differ from each end's own evaluation only by the order of the
 * sums); the tables for this (about 20 bytes per spring and 4 per incidence
 * slot) stay allocated between calls until the springs or the layout
 * change.  Setting the environment variable TITAN_ADJOINT_SPRING_ONCE=0
 * selects the per-slot evaluation. */
int titan_rollout_grad(titan_sim *sim, int64_t nsteps, int32_t checkpoint_every, const float *body_weights,
                       float *loss_out, float *grad_k, float *grad_act_c, float *grad_act_s);

/* The rollout gradient of titan_rollout_grad (same rollout, loss, checkpoints
 * and refusals; not in the paper) with the actuation gradient taken per
 * voxel of the map set by titan_set_voxel_actuation (TITAN_ESTATE if none):
 * through the mean-phasor map, on the device,
 *   grad_voxel_a[v]   = dJ/da_v   = sum_s (dJ/dC_s cos phi_v + dJ/dS_s sin phi_v) / n_s,
 *   grad_voxel_phi[v] = dJ/dphi_v = a_v sum_s (dJ/dS_s cos phi_v - dJ/dC_s sin phi_v) / n_s,
 * over the springs s that voxel v drives, n_s the number of voxels driving
 * spring s; each voxel's sum runs over its springs in ascending order.
 * Outputs (each may be NULL): loss_out[n_bodies], grad_k[n_springs],
 * grad_voxel_a[n_voxels], grad_voxel_phi[n_voxels]. */
int titan_rollout_grad_voxel(titan_sim *sim, int64_t nsteps, int32_t checkpoint_every, const float *body_weights,
                             float *loss_out, float *grad_k, float *grad_voxel_a, float *grad_voxel_phi);

/* The rollout gradient of titan_rollout_grad (same rollout, loss, checkpoints,
 * refusals and bits; not in the paper) with the outputs in device memory, for
 * callers whose parameters and gradients live on the GPU: loss_out[n_bodies],
 * grad_k, grad_act_c and grad_act_s[n_springs] are device pointers of the
 * simulation's GPU (each may be NULL; TITAN_EINVAL for any other pointer).
 * body_weights stays a host array (or NULL).  The outputs are written on the
 * simulation's stream and the call returns once they are complete; on an
 * error (TITAN_ENONFINITE included) they are not written. */
int titan_rollout_grad_device(titan_sim *sim, int64_t nsteps, int32_t checkpoint_every, const float *body_weights,
                              float *loss_out, float *grad_k, float *grad_act_c, float *grad_act_s);

/* Summed spring force on masses [first, first+count) at the current state
 * and the current step's time (blocks): the spring pass of Sec. III-B
 * (Eq. 1) alone.  f_n3 receives N. */
int titan_get_forces(titan_sim *sim, int64_t first, int64_t count, float *f_n3);

/* Fill *info (library bookkeeping, not in the paper). */
int titan_get_info(titan_sim *sim, titan_info *info);

/* ------------------------------------------------------------------------
 * Learned surrogate: a multilayer perceptron trained on the simulator's own
 * rollouts to predict a robot's centre-of-mass displacement from its layout
 * and actuation, used to screen candidates before simulating them.
 * Layers l = 0..L-1: z = x W_l^T + b_l; hidden layers apply GELU (exact erf
 * form), the last is linear.  GEMMs run on BF16 matrix cores with FP32
 * accumulation; weights and activations are rounded to bfloat16 for them,
 * master weights and Adam moments stay FP32.  Loss: mean squared error.
 * Parameters are one flat FP32 array: W_0 (dims[1] x dims[0], row-major),
 * b_0 (dims[1]), W_1, b_1, ...
 * ------------------------------------------------------------------------ */
typedef struct titan_mlp titan_mlp;

/* (The surrogate is not in the paper; every titan_mlp_* call belongs to it.)
 * Create a network of n_layers layers with widths dims[0..n_layers]
 * (1..65536 each).  stream / alloc as in titan_create.  Parameters start at
 * zero: set them with titan_mlp_set_params. */
int titan_mlp_create(int32_t n_layers, const int32_t *dims, void *stream, const titan_allocator *alloc,
                     titan_mlp **out);
/* Free the network and its device memory (not in the paper).  NULL is
 * accepted. */
int titan_mlp_destroy(titan_mlp *mlp);
/* Number of parameters (length of the flat array), or -1 for NULL (not in
 * the paper). */
int64_t titan_mlp_param_count(titan_mlp *mlp);
/* Copy all parameters in (resets the Adam state); not in the paper. */
int titan_mlp_set_params(titan_mlp *mlp, const float *params);
/* Copy all parameters out (not in the paper). */
int titan_mlp_get_params(titan_mlp *mlp, float *params);
/* Keep a training set on the device (not in the paper): X (n x dims[0],
 * stored as bfloat16),
 * Y (n x dims[L], FP32 targets).  Replaces any previous set. */
int titan_mlp_set_data(titan_mlp *mlp, int64_t n, const float *X, const float *Y);
/* nsteps Adam steps (not in the paper; learning rate lr, beta1, beta2, eps) on
 * mini-batches of
 * `batch` rows of the training set; idx (nsteps x batch) lists the rows of
 * each step.  loss_out (nsteps, may be NULL) receives each step's loss. */
int titan_mlp_train(titan_mlp *mlp, int64_t nsteps, int32_t batch, const int64_t *idx, float lr, float beta1,
                    float beta2, float eps, float *loss_out);
/* Outputs (n x dims[L]) for inputs X (n x dims[0]); not in the paper. */
int titan_mlp_predict(titan_mlp *mlp, int64_t n, const float *X, float *out);
/* Loss and the gradient of every parameter (flat layout) on one batch (not
 * in the paper). */
int titan_mlp_grad(titan_mlp *mlp, int32_t batch, const float *X, const float *Y, float *loss, float *grads);
/* The GEMM alone (not in the paper), on device arrays: C (M x N, FP32, row-major) = op(A) op(B)
 * with op(A)[m][k] = ta ? A[k*lda + m] : A[m*lda + k] and
 * op(B)[k][n] = tb ? B[n*ldb + k] : B[k*ldb + n] (bfloat16 bit patterns).
 * Asynchronous on `stream`.  A large product (at least 128 output tiles of
 * 256 x 256) with ta = 1 or tb = 0 first copies that operand with K
 * contiguous into stream-ordered device memory (hipMallocAsync on `stream`,
 * at most (M + N) x K values rounded to 16-byte rows, released on `stream`
 * behind the product); without that memory it reads the operand in place.
 * The result does not depend on which way it ran. */
int titan_mlp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A_dev, int32_t lda, int32_t ta,
                        const uint16_t *B_dev, int32_t ldb, int32_t tb, float *C_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TITAN_H */

/*
 * titan_oracle.c -- plain FP64 CPU reference of the mass-spring step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU path; it is
 * used by the test-suite, by the package's smoke check and by the benchmark's
 * CPU-baseline leg, and by nothing else.  It shares no code, header, table or
 * helper with the GPU library and includes none of its files.
 *
 * What it computes (Titan, arXiv:1911.10274):
 *   - Sec. III-B: each step first applies Hooke's-law spring forces to the
 *     two masses of every spring, then updates every mass from the summed
 *     force.  Eq. 1 gives the mass update dx = xdot*dt + xddot*dt^2, which is
 *     semi-implicit (symplectic) Euler: v += a*dt, then x += v_new*dt.
 *   - Eq. 1 writes Hooke's law without a rest length or direction; the force
 *     used here is the axial law  f = [k (l - L) + c (v_rel . u)] u  on the
 *     first end (u the unit vector from first to second end), -f on the
 *     second, with an axial relative-velocity damper of coefficient c.
 *   - Sec. III-A / Sec. I: masses are subject to plane constraints with
 *     friction; here a penalty ground plane z = 0 (normal force -k_g z while
 *     z < 0) and Coulomb friction applied as a tangential velocity change of
 *     at most mu * F_n * dt / m.
 *   - Sec. IV-B Eq. 4: actuation scales the rest length by
 *     1 + amp * sin(omega * t + phase), t = n * dt at the start of step n.
 *   - Sec. IV-B Eqs. 3-5 (wave mode, the worm): the rest length is scaled by
 *     1 + amp * sin(omega * tau) with tau = (t - t_o) mod period, the modulo
 *     taken non-negative (tau in [0, period)); the per-spring offset t_o is
 *     passed in the phase array.  Eq. 5 defines t_o from the reference
 *     positions: the smaller x of the two ends minus the body's smallest x.
 *   - Sec. III-E (real materials): a spring may carry a yield value; the
 *     force calculation tests it to decide whether the spring has broken.
 *     Reading taken here: the value compared is the magnitude of the spring's
 *     elastic force |k (l - L(t))| (the damper's force is not a material
 *     load); a spring whose elastic force exceeds its yield value breaks in
 *     that force evaluation, exerts no force in it, and stays broken.
 *     Springs with coincident ends (no direction, no force) are not tested.
 *   - Sec. III-B names Verlet and RK4 as alternatives to Euler.  Readings
 *     taken here (integrator 1 and 2; 0 is the semi-implicit Euler above):
 *     both integrate the smooth forces (springs with their dampers, gravity,
 *     the ground's normal force at the evaluated position); Coulomb friction
 *     is then applied once per step as in the Euler step -- normal force from
 *     the step's starting height, tangential velocity scaled by
 *     max(0, 1 - mu F_n dt / (m |v_t|)) -- and the position takes the same
 *     velocity change times dt.  Pinned masses keep position and velocity.
 *     Velocity Verlet: v' = v + a dt/2, x' = x + v' dt, a' = a(x', v', t+dt),
 *     v'' = v' + a' dt/2; the dampers at the end of the step see the
 *     half-step velocity v', and a' is carried to the next step (recomputed
 *     from (x, v, t) when none is carried).  RK4: the classical four stages
 *     on (x, v) at t, t + dt/2, t + dt/2, t + dt, weights 1/6, 2/6, 2/6, 1/6.
 *
 * Accumulation is a serial scatter loop over springs in index order, each
 * spring adding its force to both of its masses (Sec. III-B's spring pass),
 * all in double precision.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double dt;        /* time step, s */
    double g[3];      /* gravitational acceleration, m/s^2 */
    int32_t ground;   /* nonzero: ground plane z = 0 present */
    double ground_k;  /* penalty stiffness, N/m */
    double mu;        /* Coulomb friction coefficient */
    double omega;     /* actuation angular frequency, rad/s */
    int32_t wave;     /* nonzero: wave actuation (Eqs. 3-5), phase = offset t_o */
    double period;    /* wave actuation period t_p, s */
    int32_t integrator; /* 0 semi-implicit Euler, 1 velocity Verlet, 2 RK4 */
} orc_params;

/* Factor by which spring s's rest length exceeds its base length at time t:
 * the rest length is rest * (1 + factor). */
static double act_factor(double amp, double phase, double omega, double t, int wave, double period)
{
    if (!wave)
        return amp * sin(omega * t + phase);
    double u = t - phase;                          /* T - t_o */
    double tau = u - period * floor(u / period);   /* in [0, period) */
    return amp * sin(omega * tau);
}

/* Rest length of every spring = distance between its ends at the given
 * positions (x: n*3 doubles). */
void orc_rest_lengths(int64_t ns, const int64_t *ends, const double *x, double *rest)
{
    for (int64_t s = 0; s < ns; ++s) {
        const double *a = x + 3 * ends[2 * s];
        const double *b = x + 3 * ends[2 * s + 1];
        double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
        rest[s] = sqrt(dx * dx + dy * dy + dz * dz);
    }
}

/* Spring forces of the state (x, v) at time t, summed per mass into f (n*3,
 * overwritten).  amp/phase may be NULL (no actuation); c may be NULL (no
 * damping).  yield may be NULL (no spring breaks); otherwise broken (ns
 * flags, in and out) marks the broken springs and gains those that break in
 * this evaluation. */
void orc_spring_forces(int64_t n, int64_t ns, const int64_t *ends,
                       const double *k, const double *c, const double *rest,
                       const double *amp, const double *phase, double omega,
                       int32_t wave, double period, const double *yield, uint8_t *broken,
                       double t, const double *x, const double *v, double *f)
{
    memset(f, 0, sizeof(double) * 3 * (size_t)n);
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i = ends[2 * s], j = ends[2 * s + 1];
        double d[3], dv[3];
        for (int q = 0; q < 3; ++q) {
            d[q] = x[3 * j + q] - x[3 * i + q];
            dv[q] = v[3 * j + q] - v[3 * i + q];
        }
        double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (len == 0.0)
            continue; /* direction undefined: the spring exerts no force */
        double u[3] = {d[0] / len, d[1] / len, d[2] / len};
        double L = rest[s];
        if (amp)
            L = rest[s] * (1.0 + act_factor(amp[s], phase[s], omega, t, wave, period));
        double mag = k[s] * (len - L);
        if (yield) {
            if (broken[s])
                continue;
            if (!(fabs(mag) <= yield[s])) {
                broken[s] = 1; /* breaks now: no force from here on */
                continue;
            }
        }
        if (c)
            mag += c[s] * (dv[0] * u[0] + dv[1] * u[1] + dv[2] * u[2]);
        for (int q = 0; q < 3; ++q) {
            f[3 * i + q] += mag * u[q];
            f[3 * j + q] -= mag * u[q];
        }
    }
}

/* Mass update of one step given the summed spring force f (n*3).  Pinned
 * masses (mass 0) do not move.  x, v are updated in place. */
void orc_integrate(int64_t n, const double *mass, const orc_params *p,
                   const double *f, double *x, double *v)
{
    const double dt = p->dt;
    for (int64_t i = 0; i < n; ++i) {
        double m = mass[i];
        if (m == 0.0)
            continue;
        double F[3];
        for (int q = 0; q < 3; ++q)
            F[q] = f[3 * i + q] + m * p->g[q];
        double z = x[3 * i + 2];
        int contact = p->ground && z < 0.0;
        double Fn = 0.0;
        if (contact) {
            Fn = -p->ground_k * z;
            F[2] += Fn;
        }
        double w[3];
        for (int q = 0; q < 3; ++q)
            w[q] = v[3 * i + q] + dt * F[q] / m;
        if (contact) {
            double vt = sqrt(w[0] * w[0] + w[1] * w[1]);
            if (vt > 0.0) {
                double scale = 1.0 - p->mu * Fn * dt / (m * vt);
                if (scale < 0.0)
                    scale = 0.0;
                w[0] *= scale;
                w[1] *= scale;
            }
        }
        for (int q = 0; q < 3; ++q) {
            v[3 * i + q] = w[q];
            x[3 * i + q] += dt * w[q];
        }
    }
}

/* Acceleration of the smooth forces: a = f / m + g, plus the ground's normal
 * force -k_g z / m while z < 0 (z of the given positions).  Pinned masses: 0. */
static void accel(int64_t n, const double *mass, const orc_params *p, const double *f, const double *x, double *a)
{
    for (int64_t i = 0; i < n; ++i) {
        double m = mass[i];
        for (int q = 0; q < 3; ++q)
            a[3 * i + q] = 0.0;
        if (m == 0.0)
            continue;
        for (int q = 0; q < 3; ++q)
            a[3 * i + q] = f[3 * i + q] / m + p->g[q];
        double z = x[3 * i + 2];
        if (p->ground && z < 0.0)
            a[3 * i + 2] += -p->ground_k * z / m;
    }
}

/* Coulomb friction after a smooth update (integrators 1 and 2): for a mass
 * whose starting height z0 is below the ground, the tangential velocity is
 * scaled by max(0, 1 - mu F_n dt / (m |v_t|)), F_n = -k_g z0, and the
 * position moves by the velocity change times dt. */
static void friction_after(int64_t n, const double *mass, const orc_params *p, const double *x0, double *x,
                           double *v)
{
    for (int64_t i = 0; i < n; ++i) {
        double m = mass[i];
        double z = x0[3 * i + 2];
        if (m == 0.0 || !(p->ground && z < 0.0))
            continue;
        double Fn = -p->ground_k * z;
        double vt = sqrt(v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1]);
        if (!(vt > 0.0))
            continue;
        double scale = 1.0 - p->mu * Fn * p->dt / (m * vt);
        if (scale < 0.0)
            scale = 0.0;
        for (int q = 0; q < 2; ++q) {
            double w = v[3 * i + q] * scale;
            x[3 * i + q] += (w - v[3 * i + q]) * p->dt;
            v[3 * i + q] = w;
        }
    }
}

/* One velocity-Verlet step from (x, v) at step index `step`.  acc (n*3) holds
 * the carried acceleration when *have_acc, and receives the new one; f
 * receives the spring forces of (x, v, t) (the step's starting state; with a
 * carried acceleration they are evaluated for the caller only: yield tests
 * applied to a copy of the flags, broken in the step proper); w is scratch of
 * 2 * n*3 doubles, bw of ns flags (or NULL without yields).  Returns 0. */
static void verlet_step(int64_t n, const double *mass, int64_t ns, const int64_t *ends, const double *k,
                        const double *c, const double *rest, const double *amp, const double *phase,
                        const orc_params *p, const double *yield, uint8_t *broken, int64_t step, double *x,
                        double *v, double *acc, int32_t *have_acc, double *f, double *w, uint8_t *bw)
{
    const size_t S = 3 * (size_t)n;
    const double dt = p->dt, t = (double)step * dt, t1 = t + dt; /* as RK4's last stage: t + 1 dt */
    double *x0 = w, *f1 = w + S;
    memcpy(x0, x, sizeof(double) * S);
    if (!*have_acc) {
        orc_spring_forces(n, ns, ends, k, c, rest, amp, phase, p->omega, p->wave, p->period, yield, broken, t, x, v,
                          f);
        accel(n, mass, p, f, x, acc);
        *have_acc = 1;
    } else {
        if (yield)
            memcpy(bw, broken, (size_t)ns);
        orc_spring_forces(n, ns, ends, k, c, rest, amp, phase, p->omega, p->wave, p->period, yield,
                          yield ? bw : NULL, t, x, v, f);
    }
    for (int64_t i = 0; i < n; ++i) {
        if (mass[i] == 0.0)
            continue;
        for (int q = 0; q < 3; ++q) {
            v[3 * i + q] += 0.5 * dt * acc[3 * i + q];
            x[3 * i + q] += dt * v[3 * i + q];
        }
    }
    orc_spring_forces(n, ns, ends, k, c, rest, amp, phase, p->omega, p->wave, p->period, yield, broken, t1, x, v, f1);
    accel(n, mass, p, f1, x, acc);
    for (int64_t i = 0; i < n; ++i) {
        if (mass[i] == 0.0)
            continue;
        for (int q = 0; q < 3; ++q)
            v[3 * i + q] += 0.5 * dt * acc[3 * i + q];
    }
    friction_after(n, mass, p, x0, x, v);
}

/* One classical RK4 step on (x, v) from step index `step`; f receives the
 * spring forces of the first stage (the step's starting state); w is scratch
 * of 8 * n*3 doubles. */
static void rk4_step(int64_t n, const double *mass, int64_t ns, const int64_t *ends, const double *k,
                     const double *c, const double *rest, const double *amp, const double *phase,
                     const orc_params *p, const double *yield, uint8_t *broken, int64_t step, double *x, double *v,
                     double *f, double *w)
{
    const size_t S = 3 * (size_t)n;
    const double dt = p->dt, t = (double)step * dt;
    double *x0 = w, *v0 = w + S, *xs = w + 2 * S, *vs = w + 3 * S, *sx = w + 4 * S, *sv = w + 5 * S,
           *a = w + 6 * S, *fs = w + 7 * S;
    memcpy(x0, x, sizeof(double) * S);
    memcpy(v0, v, sizeof(double) * S);
    memcpy(xs, x, sizeof(double) * S);
    memcpy(vs, v, sizeof(double) * S);
    memset(sx, 0, sizeof(double) * S);
    memset(sv, 0, sizeof(double) * S);
    static const double c_time[4] = {0.0, 0.5, 0.5, 1.0};   /* stage times, in dt */
    static const double c_next[3] = {0.5, 0.5, 1.0};        /* next stage offset, in dt */
    static const double weight[4] = {1.0, 2.0, 2.0, 1.0};   /* times 1/6 */
    for (int st = 0; st < 4; ++st) {
        const double ts = t + c_time[st] * dt;
        orc_spring_forces(n, ns, ends, k, c, rest, amp, phase, p->omega, p->wave, p->period, yield, broken, ts, xs,
                          vs, fs);
        if (st == 0)
            memcpy(f, fs, sizeof(double) * S);
        accel(n, mass, p, fs, xs, a);
        for (int64_t i = 0; i < n; ++i) {
            if (mass[i] == 0.0)
                continue;
            for (int q = 0; q < 3; ++q) {
                const size_t e = 3 * (size_t)i + q;
                sx[e] += weight[st] * vs[e];
                sv[e] += weight[st] * a[e];
            }
        }
        if (st < 3)
            for (int64_t i = 0; i < n; ++i) {
                if (mass[i] == 0.0)
                    continue;
                for (int q = 0; q < 3; ++q) {
                    const size_t e = 3 * (size_t)i + q;
                    const double xn = x0[e] + c_next[st] * dt * vs[e];
                    const double vn = v0[e] + c_next[st] * dt * a[e];
                    xs[e] = xn;
                    vs[e] = vn;
                }
            }
    }
    for (int64_t i = 0; i < n; ++i) {
        if (mass[i] == 0.0)
            continue;
        for (int q = 0; q < 3; ++q) {
            const size_t e = 3 * (size_t)i + q;
            x[e] = x0[e] + dt / 6.0 * sx[e];
            v[e] = v0[e] + dt / 6.0 * sv[e];
        }
    }
    friction_after(n, mass, p, x0, x, v);
}

/* nsteps steps of p->integrator starting at step index step0 (t_n = n * dt).
 * Velocity Verlet carries its acceleration in acc (n*3) while *have_acc is
 * set (NULL: none carried in or out).  If f_last is
 * non-NULL it receives the spring forces of the last step's starting state.
 * Scratch of n*3 doubles is allocated here.  Returns 0, or -2 on allocation
 * failure. */
int orc_run(int64_t n, const double *mass, int64_t ns, const int64_t *ends,
            const double *k, const double *c, const double *rest,
            const double *amp, const double *phase, const orc_params *p,
            const double *yield, uint8_t *broken, double *acc, int32_t *have_acc,
            int64_t step0, int64_t nsteps, double *x, double *v, double *f_last)
{
    const size_t S = 3 * (size_t)(n > 0 ? n : 1);
    double *f = (double *)malloc(sizeof(double) * S);
    if (!f)
        return -2;
    if (p->integrator == 1 || p->integrator == 2) {
        double *w = (double *)malloc(sizeof(double) * 8 * S);
        double *own_acc = NULL;
        int32_t own_have = 0;
        uint8_t *bw = yield ? (uint8_t *)malloc((size_t)(ns > 0 ? ns : 1)) : NULL;
        if (p->integrator == 1 && !acc) {
            own_acc = (double *)malloc(sizeof(double) * S);
            acc = own_acc;
            have_acc = &own_have;
        }
        if (!w || (p->integrator == 1 && !acc) || (yield && !bw)) {
            free(w);
            free(own_acc);
            free(bw);
            free(f);
            return -2;
        }
        for (int64_t s = 0; s < nsteps; ++s) {
            if (p->integrator == 1)
                verlet_step(n, mass, ns, ends, k, c, rest, amp, phase, p, yield, broken, step0 + s, x, v, acc,
                            have_acc, f, w, bw);
            else
                rk4_step(n, mass, ns, ends, k, c, rest, amp, phase, p, yield, broken, step0 + s, x, v, f, w);
            if (f_last && s == nsteps - 1)
                memcpy(f_last, f, sizeof(double) * 3 * (size_t)n);
        }
        free(w);
        free(own_acc);
        free(bw);
        free(f);
        return 0;
    }
    for (int64_t s = 0; s < nsteps; ++s) {
        double t = (double)(step0 + s) * p->dt;
        orc_spring_forces(n, ns, ends, k, c, rest, amp, phase, p->omega, p->wave, p->period, yield, broken, t, x,
                          v, f);
        if (f_last && s == nsteps - 1)
            memcpy(f_last, f, sizeof(double) * 3 * (size_t)n);
        orc_integrate(n, mass, p, f, x, v);
    }
    free(f);
    return 0;
}

/* ------------------------------------------------------------------------
 * Reverse-mode gradient of a rollout (the adjoint of the step above).
 *
 * Loss: J = sum_b w_b * J_b,  J_b = -(CoM_x(x_N) - CoM_x(x_0)) over the masses
 * of body b (mass-weighted; pinned masses weigh nothing).
 * Gradients w.r.t. every spring's k and actuation phasor (C, S), where
 * C = amp cos(phase), S = amp sin(phase), so that the rest length at time t
 * is rest * (1 + C sin(omega t) + S cos(omega t)) -- the same function as
 * rest * (1 + amp sin(omega t + phase)).
 *
 * The forward trajectory is stored whole (nsteps + 1 states) and the step is
 * differentiated backwards in the order it was computed: position update,
 * friction, velocity update, forces.  `sig` (optional) receives a hash of
 * every contact and friction-stick decision of the run, so that a
 * finite-difference check can discard perturbations that change them.
 * Returns 0, or -2 when memory runs out.
 * ------------------------------------------------------------------------ */

static uint64_t fnv(uint64_t h, uint64_t v)
{
    for (int b = 0; b < 8; ++b) {
        h ^= (v >> (8 * b)) & 0xff;
        h *= 1099511628211ull;
    }
    return h;
}

/* One forward step that also records the contact/stick decisions in *sig. */
static void step_sig(int64_t n, const double *mass, int64_t ns, const int64_t *ends, const double *k,
                     const double *c, const double *rest, const double *amp, const double *phase,
                     const orc_params *p, int64_t step, double *f, double *x, double *v, uint64_t *sig)
{
    const double dt = p->dt;
    orc_spring_forces(n, ns, ends, k, c, rest, amp, phase, p->omega, p->wave, p->period, NULL, NULL,
                      (double)step * dt, x, v, f);
    for (int64_t i = 0; i < n; ++i) {
        double m = mass[i];
        if (m == 0.0)
            continue;
        double F[3];
        for (int q = 0; q < 3; ++q)
            F[q] = f[3 * i + q] + m * p->g[q];
        double z = x[3 * i + 2];
        int contact = p->ground && z < 0.0;
        double Fn = 0.0;
        if (contact) {
            Fn = -p->ground_k * z;
            F[2] += Fn;
        }
        double w[3];
        for (int q = 0; q < 3; ++q)
            w[q] = v[3 * i + q] + dt * F[q] / m;
        int stick = 0;
        if (contact) {
            double vt = sqrt(w[0] * w[0] + w[1] * w[1]);
            if (vt > 0.0) {
                double scale = 1.0 - p->mu * Fn * dt / (m * vt);
                if (scale < 0.0) {
                    scale = 0.0;
                    stick = 1;
                }
                w[0] *= scale;
                w[1] *= scale;
            }
        }
        if (sig && (contact || stick))
            *sig = fnv(fnv(*sig, (uint64_t)step * 0x9e3779b97f4a7c15ull + (uint64_t)i), (uint64_t)(contact + 2 * stick));
        for (int q = 0; q < 3; ++q) {
            v[3 * i + q] = w[q];
            x[3 * i + q] += dt * w[q];
        }
    }
}

static void com_x(int64_t n, const double *mass, const int32_t *body, int32_t nbody, const double *x,
                  double *com, double *mtot)
{
    for (int32_t b = 0; b < nbody; ++b) {
        com[b] = 0.0;
        mtot[b] = 0.0;
    }
    for (int64_t i = 0; i < n; ++i) {
        com[body[i]] += mass[i] * x[3 * i];
        mtot[body[i]] += mass[i];
    }
    for (int32_t b = 0; b < nbody; ++b)
        com[b] = mtot[b] > 0.0 ? com[b] / mtot[b] : 0.0;
}

/* Forward only: per-body J_b into loss (nbody), decision hash into *sig. */
int orc_rollout_loss(int64_t n, const double *mass, int64_t ns, const int64_t *ends, const double *k,
                     const double *c, const double *rest, const double *amp, const double *phase,
                     const orc_params *p, const int32_t *body, int32_t nbody, int64_t nsteps,
                     const double *x0, const double *v0, double *loss, uint64_t *sig)
{
    if (p->integrator != 0)
        return -1; /* the rollout covers the Euler step only */
    double *x = (double *)malloc(sizeof(double) * 3 * (size_t)(n + 1));
    double *v = (double *)malloc(sizeof(double) * 3 * (size_t)(n + 1));
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)(n + 1));
    double *c0 = (double *)malloc(sizeof(double) * (size_t)(2 * nbody + 2));
    if (!x || !v || !f || !c0) {
        free(x); free(v); free(f); free(c0);
        return -2;
    }
    memcpy(x, x0, sizeof(double) * 3 * (size_t)n);
    memcpy(v, v0, sizeof(double) * 3 * (size_t)n);
    if (sig)
        *sig = 14695981039346656037ull;
    double *mt = c0 + nbody + 1;
    com_x(n, mass, body, nbody, x, c0, mt);
    for (int64_t s = 0; s < nsteps; ++s)
        step_sig(n, mass, ns, ends, k, c, rest, amp, phase, p, s, f, x, v, sig);
    com_x(n, mass, body, nbody, x, loss, mt);
    for (int32_t b = 0; b < nbody; ++b)
        loss[b] = -(loss[b] - c0[b]);
    free(x); free(v); free(f); free(c0);
    return 0;
}

int orc_rollout_grad(int64_t n, const double *mass, int64_t ns, const int64_t *ends, const double *k,
                     const double *c, const double *rest, const double *amp, const double *phase,
                     const orc_params *p, const int32_t *body, int32_t nbody, const double *wbody,
                     int64_t nsteps, const double *x0, const double *v0, double *loss, double *gk,
                     double *gC, double *gS, uint64_t *sig)
{
    if (p->wave || p->integrator != 0)
        return -1; /* the adjoint covers phasor actuation and the Euler step only */
    const double dt = p->dt;
    const size_t S = 3 * (size_t)(n > 0 ? n : 1);
    double *X = (double *)malloc(sizeof(double) * S * (size_t)(nsteps + 1));
    double *V = (double *)malloc(sizeof(double) * S * (size_t)(nsteps + 1));
    double *f = (double *)malloc(sizeof(double) * S);
    double *lx = (double *)malloc(sizeof(double) * S);
    double *lv = (double *)malloc(sizeof(double) * S);
    double *nlx = (double *)malloc(sizeof(double) * S);
    double *nlv = (double *)malloc(sizeof(double) * S);
    double *mu = (double *)malloc(sizeof(double) * S);
    double *cm = (double *)malloc(sizeof(double) * (size_t)(2 * nbody + 2));
    if (!X || !V || !f || !lx || !lv || !nlx || !nlv || !mu || !cm) {
        free(X); free(V); free(f); free(lx); free(lv); free(nlx); free(nlv); free(mu); free(cm);
        return -2;
    }
    /* forward, keeping every state */
    memcpy(X, x0, sizeof(double) * 3 * (size_t)n);
    memcpy(V, v0, sizeof(double) * 3 * (size_t)n);
    if (sig)
        *sig = 14695981039346656037ull;
    for (int64_t s = 0; s < nsteps; ++s) {
        memcpy(X + S * (s + 1), X + S * s, sizeof(double) * 3 * (size_t)n);
        memcpy(V + S * (s + 1), V + S * s, sizeof(double) * 3 * (size_t)n);
        step_sig(n, mass, ns, ends, k, c, rest, amp, phase, p, s, f, X + S * (s + 1), V + S * (s + 1), sig);
    }
    double *mt = cm + nbody + 1;
    double *c0 = cm;
    com_x(n, mass, body, nbody, X, c0, mt);
    double *cN = (double *)malloc(sizeof(double) * (size_t)(nbody + 1));
    if (!cN) {
        free(X); free(V); free(f); free(lx); free(lv); free(nlx); free(nlv); free(mu); free(cm);
        return -2;
    }
    com_x(n, mass, body, nbody, X + S * nsteps, cN, mt);
    for (int32_t b = 0; b < nbody; ++b)
        loss[b] = -(cN[b] - c0[b]);
    free(cN);

    /* dJ/dx_N, dJ/dv_N */
    memset(lx, 0, sizeof(double) * S);
    memset(lv, 0, sizeof(double) * S);
    for (int64_t i = 0; i < n; ++i)
        if (mt[body[i]] > 0.0)
            lx[3 * i] = -wbody[body[i]] * mass[i] / mt[body[i]];
    for (int64_t s = 0; s < ns; ++s)
        gk[s] = gC[s] = gS[s] = 0.0;

    for (int64_t st = nsteps - 1; st >= 0; --st) {
        const double *x = X + S * st, *v = V + S * st;
        const double t = (double)st * dt;
        orc_spring_forces(n, ns, ends, k, c, rest, amp, phase, p->omega, p->wave, p->period, NULL, NULL, t, x, v,
                          f);
        /* masses: position update, friction, velocity update */
        for (int64_t i = 0; i < n; ++i) {
            double m = mass[i];
            for (int q = 0; q < 3; ++q) {
                nlx[3 * i + q] = lx[3 * i + q];
                nlv[3 * i + q] = lv[3 * i + q];
                mu[3 * i + q] = 0.0;
            }
            if (m == 0.0)
                continue; /* pinned: its state never changes */
            double F[3];
            for (int q = 0; q < 3; ++q)
                F[q] = f[3 * i + q] + m * p->g[q];
            double z = x[3 * i + 2];
            int contact = p->ground && z < 0.0;
            double Fn = 0.0;
            if (contact) {
                Fn = -p->ground_k * z;
                F[2] += Fn;
            }
            double w[3];
            for (int q = 0; q < 3; ++q)
                w[q] = v[3 * i + q] + dt * F[q] / m;
            /* v_{n+1} also moves x_{n+1} = x_n + dt v_{n+1} */
            double lvt[3], lw[3];
            for (int q = 0; q < 3; ++q)
                lvt[q] = lv[3 * i + q] + dt * lx[3 * i + q];
            for (int q = 0; q < 3; ++q)
                lw[q] = lvt[q];
            double dz = 0.0; /* extra dJ/dz through the friction bound */
            if (contact) {
                double vt = sqrt(w[0] * w[0] + w[1] * w[1]);
                if (vt > 0.0) {
                    double beta = p->mu * Fn * dt / m;
                    double sc = 1.0 - beta / vt;
                    if (sc > 0.0) {
                        double wh[2] = {w[0] / vt, w[1] / vt};
                        double wl = wh[0] * lvt[0] + wh[1] * lvt[1];
                        lw[0] = sc * lvt[0] + (beta / vt) * wh[0] * wl;
                        lw[1] = sc * lvt[1] + (beta / vt) * wh[1] * wl;
                        dz = wl * p->mu * dt * p->ground_k / m;
                    } else {
                        lw[0] = 0.0;
                        lw[1] = 0.0;
                    }
                }
            }
            for (int q = 0; q < 3; ++q) {
                mu[3 * i + q] = dt / m * lw[q];
                nlv[3 * i + q] = lw[q];
            }
            nlx[3 * i + 2] += dz;
            if (contact)
                nlx[3 * i + 2] += -p->ground_k * mu[3 * i + 2];
        }
        /* springs */
        for (int64_t s = 0; s < ns; ++s) {
            int64_t i = ends[2 * s], j = ends[2 * s + 1];
            double d[3], dv[3];
            for (int q = 0; q < 3; ++q) {
                d[q] = x[3 * j + q] - x[3 * i + q];
                dv[q] = v[3 * j + q] - v[3 * i + q];
            }
            double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (len == 0.0)
                continue;
            double u[3] = {d[0] / len, d[1] / len, d[2] / len};
            double sw = 0.0, cw = 1.0;
            if (amp) {
                sw = sin(p->omega * t);
                cw = cos(p->omega * t);
            }
            double L = rest[s];
            if (amp)
                L = rest[s] * (1.0 + amp[s] * sin(p->omega * t + phase[s]));
            double e = len - L;
            double vr = dv[0] * u[0] + dv[1] * u[1] + dv[2] * u[2];
            double cs = c ? c[s] : 0.0;
            double mag = k[s] * e + cs * vr;
            double dm[3], pu = 0.0;
            for (int q = 0; q < 3; ++q) {
                dm[q] = mu[3 * i + q] - mu[3 * j + q];
                pu += dm[q] * u[q];
            }
            for (int q = 0; q < 3; ++q) {
                double gd = pu * k[s] * u[q] + pu * (cs / len) * (dv[q] - u[q] * vr) +
                            (mag / len) * (dm[q] - u[q] * pu);
                nlx[3 * j + q] += gd;
                nlx[3 * i + q] -= gd;
                double gv = pu * cs * u[q];
                nlv[3 * j + q] += gv;
                nlv[3 * i + q] -= gv;
            }
            gk[s] += pu * e;
            if (amp) {
                gC[s] += pu * k[s] * (-rest[s] * sw);
                gS[s] += pu * k[s] * (-rest[s] * cw);
            }
        }
        double *tmp = lx;
        lx = nlx;
        nlx = tmp;
        tmp = lv;
        lv = nlv;
        nlv = tmp;
    }
    free(X); free(V); free(f); free(lx); free(lv); free(nlx); free(nlv); free(mu); free(cm);
    return 0;
}

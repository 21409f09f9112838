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
 *
 * Accumulation is a serial scatter loop over springs in index order
 * (Sec. III-B's "apply to each corresponding mass"), all in double precision.
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
} orc_params;

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
 * damping). */
void orc_spring_forces(int64_t n, int64_t ns, const int64_t *ends,
                       const double *k, const double *c, const double *rest,
                       const double *amp, const double *phase, double omega,
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
            L = rest[s] * (1.0 + amp[s] * sin(omega * t + phase[s]));
        double mag = k[s] * (len - L);
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

/* nsteps steps starting at step index step0 (t_n = n * dt).  If f_last is
 * non-NULL it receives the spring forces of the last step's starting state.
 * Scratch of n*3 doubles is allocated here.  Returns 0, or -2 on allocation
 * failure. */
int orc_run(int64_t n, const double *mass, int64_t ns, const int64_t *ends,
            const double *k, const double *c, const double *rest,
            const double *amp, const double *phase, const orc_params *p,
            int64_t step0, int64_t nsteps, double *x, double *v, double *f_last)
{
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!f)
        return -2;
    for (int64_t s = 0; s < nsteps; ++s) {
        double t = (double)(step0 + s) * p->dt;
        orc_spring_forces(n, ns, ends, k, c, rest, amp, phase, p->omega, t, x, v, f);
        if (f_last && s == nsteps - 1)
            memcpy(f_last, f, sizeof(double) * 3 * (size_t)n);
        orc_integrate(n, mass, p, f, x, v);
    }
    free(f);
    return 0;
}

"""Pins of the FP64 oracle to facts that do not come from the oracle itself:
closed forms of the integrator, conservation laws, hand-worked forces and
values printed in the paper.  A plausible slip anywhere in the oracle (a
dropped term, a flipped sign, the wrong end of a spring, forward instead of
symplectic Euler, friction on the wrong velocity) fails at least one test.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_10274_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")
NO_FORCES = O.Params(dt=1e-4, gravity=(0.0, 0.0, 0.0), ground=False, ground_k=0.0, mu=0.0, omega=0.0)


def _scene(pos, mass, ends=(), k=(), c=None, vel=None, amp=None, phase=None):
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    ends = np.asarray(ends, np.int64).reshape(-1, 2)
    return dict(pos=pos, vel=np.zeros_like(pos) if vel is None else np.asarray(vel, np.float64),
                mass=np.asarray(mass, np.float64), ends=ends, k=np.asarray(k, np.float64),
                damping=None if c is None else np.asarray(c, np.float64),
                amp=None if amp is None else np.asarray(amp, np.float64),
                phase=None if phase is None else np.asarray(phase, np.float64))


# ---------------------------------------------------------------------------
# Values printed in the paper
# ---------------------------------------------------------------------------

def test_lattice_count_matches_paper():
    g = json.load(open(GOLDEN))["lattice_50_springs"]
    assert scenes.lattice_spring_count(50) == g["value"]
    assert scenes.lattice_topology(50).shape[0] == g["value"]


def test_lattice_topology_brute_force_small():
    # every pair of grid points within sqrt(3) spacing, found by brute force
    for dims in [(2, 2, 2), (3, 4, 5), (10, 10, 10)]:
        nx, ny, nz = dims
        sc = scenes.lattice(nx, ny, nz, spacing=1.0, origin=(0, 0, 0))
        p = sc["pos"].astype(np.float64)
        d2 = ((p[:, None, :] - p[None, :, :]) ** 2).sum(-1)
        iu = np.triu_indices(p.shape[0], 1)
        want = set(zip(*[a[d2[iu] <= 3.0 + 1e-9] for a in iu]))
        got = set(map(tuple, sc["ends"].tolist()))
        assert got == want
        assert len(got) == scenes.lattice_spring_count(nx, ny, nz)


def test_rate_unit_matches_paper():
    # spring updates per second = springs * steps / wall seconds
    g = json.load(open(GOLDEN))["lattice_50_rate"]
    assert round(g["springs"] * g["steps"] / g["seconds"]) == g["rate"]


# ---------------------------------------------------------------------------
# Hand-worked forces
# ---------------------------------------------------------------------------

def test_hand_forces_three_masses():
    # mass 0 at origin; mass 1 at (3,4,0): length 5, rest 4, k 10, c 2,
    # relative velocity (1,0,0) -> axial speed 0.6 -> |f| = 10*1 + 2*0.6 = 11.2
    # along u = (0.6, 0.8, 0): f0 = (6.72, 8.96, 0), f1 = -f0.
    # mass 2 at (0,0,2) joined to mass 0 at rest length 2 and moving
    # perpendicular to that spring: no force from it.
    sc = _scene([[0, 0, 0], [3, 4, 0], [0, 0, 2]], [1, 1, 1], [[0, 1], [0, 2]], [10, 7],
                c=[2, 3], vel=[[0, 0, 0], [1, 0, 0], [5, 0, 0]])
    sysm = O.System(sc, rest=[4.0, 2.0])
    f = sysm.spring_forces(sc["pos"], sc["vel"], 0.0, 0.0)
    np.testing.assert_allclose(f, [[6.72, 8.96, 0], [-6.72, -8.96, 0], [0, 0, 0]], atol=1e-12)


def test_hand_force_actuated_rest_length():
    # rest 4, amp 0.5, phase pi/2, omega pi, t = 1: sin(pi + pi/2) = -1, so the
    # rest length is 4 * (1 - 0.5) = 2 and the stretch of the 5-long spring is 3:
    # |f| = 10 * 3 = 30 along (0.6, 0.8, 0).
    sc = _scene([[0, 0, 0], [3, 4, 0]], [1, 1], [[0, 1]], [10], amp=[0.5], phase=[math.pi / 2])
    sysm = O.System(sc, rest=[4.0])
    f = sysm.spring_forces(sc["pos"], sc["vel"], 1.0, math.pi)
    np.testing.assert_allclose(f, [[18.0, 24.0, 0], [-18.0, -24.0, 0]], atol=1e-12)
    # same rest length at t = 0 with phase 3*pi/2
    sc["phase"] = np.array([1.5 * math.pi])
    f0 = O.System(sc, rest=[4.0]).spring_forces(sc["pos"], sc["vel"], 0.0, math.pi)
    np.testing.assert_allclose(f0, f, atol=1e-12)


def test_actuation_time_is_start_of_step():
    # One free mass tied to a pinned anchor at its base rest length 1, no
    # damping, gravity or ground.  Step n uses t = n*dt, so after one step
    # started at step index n the velocity is -dt/m * k * (1 - L(t_n)) along
    # the spring, with L(t) = 1 + 0.25 sin(omega t + 0.3).
    dt, k, m, w = 1e-3, 50.0, 2.0, 7.0
    sc = _scene([[0, 0, 0], [0, 1, 0]], [0, m], [[0, 1]], [k], amp=[0.25], phase=[0.3])
    sysm = O.System(sc)
    p = O.Params(dt=dt, gravity=(0, 0, 0), ground=False, ground_k=0, mu=0, omega=w)
    for n in (0, 1, 17, 1234):
        x, v, _ = sysm.run(p, sc["pos"], sc["vel"], n, 1)
        L = 1.0 + 0.25 * math.sin(w * n * dt + 0.3)
        want_vy = -dt / m * k * (1.0 - L)
        np.testing.assert_allclose(v[1], [0, want_vy, 0], atol=1e-15)
        np.testing.assert_allclose(x[1], [0, 1 + dt * want_vy, 0], atol=1e-15)
        np.testing.assert_array_equal(x[0], [0, 0, 0])  # pinned


def test_uniform_dilation_corner_force():
    # 2x2x2 cube of spacing a, all 28 springs at rest length for the cube,
    # positions scaled by (1+eps): each spring is stretched by eps*L0, so the
    # corner at the origin feels k*eps*sum(L0*u) = k*eps*a*(4,4,4).
    a, eps, k = 0.1, 1e-3, 1e4
    sc = scenes.lattice(2, spacing=a, origin=(0, 0, 0))
    sysm = O.System(sc)
    f = sysm.spring_forces(sysm.x0 * (1 + eps), sysm.v0, 0.0, 0.0)
    a32 = float(np.float32(a))  # scene positions are FP32
    np.testing.assert_allclose(f[0], k * eps * a32 * np.array([4.0, 4.0, 4.0]), rtol=1e-9)
    np.testing.assert_allclose(f[7], -k * eps * a32 * np.array([4.0, 4.0, 4.0]), rtol=1e-9)
    # interior mass of a 3x3x3 lattice: symmetric neighbourhood, zero net force
    sc3 = scenes.lattice(3, spacing=a, origin=(0, 0, 0))
    s3 = O.System(sc3)
    f3 = s3.spring_forces(s3.x0 * (1 + eps), s3.v0, 0.0, 0.0)
    assert np.abs(f3[13]).max() < 1e-12


# ---------------------------------------------------------------------------
# Closed forms of the integrator
# ---------------------------------------------------------------------------

def test_free_fall_closed_form():
    # symplectic Euler under constant g: v_n = v0 + n g dt,
    # z_n = z0 + v0 n dt + g dt^2 n (n+1) / 2   (not g t^2 / 2)
    dt, g, z0, v0 = 1e-4, -9.81, 0.5, 0.3
    sc = _scene([[0, 0, z0]], [0.1], vel=[[0, 0, v0]])
    sysm = O.System(sc)
    p = O.Params(dt=dt, gravity=(0, 0, g), ground=False, ground_k=0, mu=0, omega=0)
    x, v = sysm.x0, sysm.v0
    for n in (1, 2, 10, 1000):
        xs, vs, _ = sysm.run(p, x, v, 0, n)
        assert abs(vs[0, 2] - (v0 + n * g * dt)) < 1e-13
        assert abs(xs[0, 2] - (z0 + v0 * n * dt + g * dt * dt * n * (n + 1) / 2)) < 1e-13


def _anchor_oscillator(m=0.1, k=1e4, c=0.0, X=0.01, v0=0.5, L0=0.3):
    e = np.array([1.0, 2.0, 2.0]) / 3.0  # skew axis exercises the 3-D projection
    sc = _scene([[0, 0, 0], (L0 + X) * e], [0.0, m], [[0, 1]], [k], c=[c],
                vel=[[0, 0, 0], v0 * e])
    return O.System(sc, rest=[L0]), e, L0


def test_oscillator_closed_form_and_period():
    # undamped spring on a pinned anchor under symplectic Euler:
    # x_n = X cos(n th) + B sin(n th), cos th = 1 - (w dt)^2 / 2,
    # x_1 = X (1 - w^2 dt^2) + dt v0.
    m, k, X, v0, dt = 0.1, 1e4, 0.01, 0.5, 1e-4
    sysm, e, L0 = _anchor_oscillator(m, k, 0.0, X, v0)
    w = math.sqrt(k / m)
    th = math.acos(1 - (w * dt) ** 2 / 2)
    B = (X * (1 - w * w * dt * dt) + dt * v0 - X * math.cos(th)) / math.sin(th)
    p = O.Params(dt=dt, gravity=(0, 0, 0), ground=False, ground_k=0, mu=0, omega=0)
    x, v = sysm.x0, sysm.v0
    worst = 0.0
    for chunk in range(20):
        x, v, _ = sysm.run(p, x, v, chunk * 1000, 1000)
        n = (chunk + 1) * 1000
        q = x[1] @ e - L0
        worst = max(worst, abs(q - (X * math.cos(n * th) + B * math.sin(n * th))))
        perp = x[1] - (x[1] @ e) * e
        assert np.abs(perp).max() < 1e-13
    assert worst < 1e-11
    # discrete period vs the continuous 2 pi sqrt(m/k): O((w dt)^2) apart
    per = 2 * math.pi / th * dt
    assert abs(per / (2 * math.pi * math.sqrt(m / k)) - 1) < (w * dt) ** 2 / 24 * 1.01


def test_damped_oscillator_closed_form():
    # with axial damping c the recurrence is x_{n+1} = (2 - h^2 w^2 - h g) x_n - (1 - h g) x_{n-1},
    # g = c/m, so x_n = r^n (A cos n th + B sin n th) with r = sqrt(1 - h g),
    # cos th = (2 - h^2 w^2 - h g) / (2 r).  The envelope r^n ~ exp(-c t / 2m)
    # is the continuous damped oscillator's.
    m, k, c, X, v0, h = 0.1, 1e4, 2.0, 0.01, 0.0, 1e-4
    sysm, e, L0 = _anchor_oscillator(m, k, c, X, v0)
    w2, g = k / m, c / m
    r = math.sqrt(1 - h * g)
    th = math.acos((2 - h * h * w2 - h * g) / (2 * r))
    x1 = X + h * (v0 + h * (-w2 * X - g * v0))
    A = X
    B = (x1 / r - A * math.cos(th)) / math.sin(th)
    p = O.Params(dt=h, gravity=(0, 0, 0), ground=False, ground_k=0, mu=0, omega=0)
    x, v = sysm.x0, sysm.v0
    for chunk in range(10):
        x, v, _ = sysm.run(p, x, v, chunk * 500, 500)
        n = (chunk + 1) * 500
        want = r ** n * (A * math.cos(n * th) + B * math.sin(n * th))
        assert abs(x[1] @ e - L0 - want) < 1e-12
        # envelope vs exp(-c t / 2m): ln r^n = -(n/2)(hg + (hg)^2/2 + ...)
        assert abs(r ** n / math.exp(-c / (2 * m) * n * h) - 1) < n * (h * g) ** 2 / 4 * 1.01


def test_ground_contact_oscillation_closed_form():
    # a lone mass inside the ground plane (no friction velocity, gravity on)
    # oscillates about z* = m g / k_g with w^2 = k_g / m while it stays below z = 0.
    m, kg, g, h = 0.1, 1e5, -9.81, 1e-4
    zs = m * g / kg
    dz = 0.5 * zs
    sc = _scene([[0, 0, zs + dz]], [m])
    sysm = O.System(sc)
    p = O.Params(dt=h, gravity=(0, 0, g), ground=True, ground_k=kg, mu=0.5, omega=0)
    w = math.sqrt(kg / m)
    th = math.acos(1 - (w * h) ** 2 / 2)
    x1 = dz * (1 - w * w * h * h)
    B = (x1 - dz * math.cos(th)) / math.sin(th)
    x, v = sysm.x0, sysm.v0
    for n in range(1, 400):
        x, v, _ = sysm.run(p, x, v, n - 1, 1)
        assert abs(x[0, 2] - zs - (dz * math.cos(n * th) + B * math.sin(n * th))) < 1e-17
        assert x[0, 2] < 0


def test_friction_slide_closed_form():
    # a mass resting at equilibrium penetration z* = m g / k_g feels normal force
    # m|g|, so Coulomb friction removes mu |g| dt of tangential speed per step,
    # along a fixed direction, until it stops (and then stays stopped).
    m, kg, g, h, mu = 0.1, 1e5, -9.81, 1e-4, 0.5
    zs = m * g / kg
    vt0 = np.array([0.3, -0.4])  # speed 0.5
    sc = _scene([[0.2, 0.1, zs]], [m], vel=[[vt0[0], vt0[1], 0.0]])
    sysm = O.System(sc)
    p = O.Params(dt=h, gravity=(0, 0, g), ground=True, ground_k=kg, mu=mu, omega=0)
    dec = mu * abs(g) * h
    x, v = sysm.x0, sysm.v0
    dirn = vt0 / 0.5
    travelled = 0.0
    nstop = int(0.5 // dec) + 3
    for n in range(1, nstop + 20):
        x, v, _ = sysm.run(p, x, v, n - 1, 1)
        speed = max(0.0, 0.5 - n * dec)
        travelled += h * speed
        np.testing.assert_allclose(v[0, :2], speed * dirn, atol=1e-12)
        np.testing.assert_allclose(x[0, :2], [0.2, 0.1] + travelled * dirn, atol=1e-12)
        assert abs(x[0, 2] - zs) < 1e-15
    assert np.all(v[0, :2] == 0.0)


def test_ground_is_strict_and_no_friction_at_rest():
    # z == 0 is not contact; a contact mass with zero tangential speed gets no
    # friction and no NaN
    sc = _scene([[0, 0, 0.0], [1, 0, -1e-3]], [1.0, 1.0])
    sysm = O.System(sc)
    p = O.Params(dt=1e-3, gravity=(0, 0, 0), ground=True, ground_k=100.0, mu=0.5, omega=0)
    x, v, _ = sysm.run(p, sysm.x0, sysm.v0, 0, 1)
    np.testing.assert_array_equal(v[0], [0, 0, 0])
    np.testing.assert_allclose(v[1], [0, 0, 1e-3 * 100.0 * 1e-3], atol=1e-18)


def test_friction_sticks_when_impulse_exceeds_speed():
    # friction impulse mu*Fn*dt/m = 1.5x the tangential speed: the mass stops
    # (friction never reverses the sliding direction)
    m, kg, h, mu = 1.0, 1e3, 1e-2, 1.0
    z = -1e-3  # Fn = 1 N, impulse 1e-2 m/s
    sc = _scene([[0, 0, z]], [m], vel=[[0.01 / 1.5, 0, 0]])
    sysm = O.System(sc)
    p = O.Params(dt=h, gravity=(0, 0, 0), ground=True, ground_k=kg, mu=mu, omega=0)
    x, v, _ = sysm.run(p, sysm.x0, sysm.v0, 0, 1)
    assert v[0, 0] == 0.0 and v[0, 1] == 0.0
    assert abs(v[0, 2] - h * kg * 1e-3 / m) < 1e-15


def test_pinned_mass_does_not_move():
    sc = _scene([[0, 0, 0.5], [0, 0, 0.7]], [0.0, 0.1], [[0, 1]], [1e3], c=[1.0], vel=[[1, 2, 3], [0, 0, 0]])
    sysm = O.System(sc, rest=[0.1])
    p = O.Params(dt=1e-4, gravity=(0, 0, -9.81), ground=True, ground_k=1e5, mu=0.5, omega=0)
    x, v, _ = sysm.run(p, sysm.x0, sysm.v0, 0, 50)
    np.testing.assert_array_equal(x[0], sc["pos"][0])
    np.testing.assert_array_equal(v[0], [1, 2, 3])


# ---------------------------------------------------------------------------
# Conservation laws on a random 3-D lattice
# ---------------------------------------------------------------------------

def _perturbed_lattice(n=4, seed=11, damping=1.0, dx=0.01, dv=0.3):
    rng = np.random.Generator(np.random.PCG64(seed))
    sc = scenes.lattice(n, origin=(0.0, 0.0, 0.0), damping=damping)
    pos = sc["pos"].astype(np.float64)
    sysm = O.System(sc)  # rest = unperturbed lengths
    x = pos + rng.uniform(-dx, dx, pos.shape)
    v = rng.uniform(-dv, dv, pos.shape)
    return sysm, x, v


def test_newton_third_law_sum_zero():
    sysm, x, v = _perturbed_lattice()
    f = sysm.spring_forces(x, v, 0.0, 0.0)
    assert np.abs(f).sum() > 1.0
    assert np.abs(f.sum(axis=0)).max() < 1e-12 * np.abs(f).sum()


def test_momentum_and_angular_momentum_conserved():
    # gravity and ground off: internal central pair forces (spring + axial
    # damping) conserve linear momentum, and symplectic Euler conserves angular
    # momentum exactly for central forces (x_{n+1} x v_{n+1} = x_n x v_{n+1}).
    sysm, x, v = _perturbed_lattice(damping=1.0)
    P0 = sysm.momentum(v)
    L0 = sysm.angular_momentum(x, v)
    xs, vs, _ = sysm.run(NO_FORCES, x, v, 0, 3000)
    scale = np.abs(sysm.mass[:, None] * v).sum()
    assert np.abs(sysm.momentum(vs) - P0).max() < 1e-12 * scale
    assert np.abs(sysm.angular_momentum(xs, vs) - L0).max() < 1e-11 * scale


def test_modified_energy_bounded_undamped():
    # undamped, unactuated, no gravity/ground: the energy H of symplectic Euler
    # oscillates with O(w dt) amplitude but H~ = H + dt/2 sum v.F(x) is
    # conserved to O(dt^2) (exactly for linear springs): no drift.
    sysm, x, v = _perturbed_lattice(damping=0.0, dx=0.002, dv=0.05)
    sysm.c = None
    H, Ht = [], []
    for s in range(40):
        f = sysm.spring_forces(x, v, 0.0, 0.0)
        h = sysm.kinetic(v) + sysm.spring_energy(x)
        H.append(h)
        Ht.append(h + 0.5 * NO_FORCES.dt * float(np.sum(v * f)))
        x, v, _ = sysm.run(NO_FORCES, x, v, s * 250, 250)
    H, Ht = np.array(H), np.array(Ht)
    assert np.ptp(H) / H.mean() > 1e-2
    assert np.ptp(Ht) < np.ptp(H) / 500
    assert np.ptp(Ht) / Ht.mean() < 5e-5


def test_modified_energy_exact_linear():
    sysm, e, L0 = _anchor_oscillator(c=0.0)
    x, v = sysm.x0, sysm.v0
    vals = []
    for s in range(50):
        f = sysm.spring_forces(x, v, 0.0, 0.0)
        h = sysm.kinetic(v) + sysm.spring_energy(x)
        vals.append(h + 0.5 * NO_FORCES.dt * float(np.sum(v * f)))
        x, v, _ = sysm.run(NO_FORCES, x, v, s * 97, 97)
    vals = np.array(vals)
    assert np.ptp(vals) / vals.mean() < 1e-12


def test_uniform_translation_is_rigid():
    sc = scenes.lattice(3, origin=(0, 0, 0))
    sysm = O.System(sc)
    v = np.tile([0.7, -0.2, 0.1], (sysm.n, 1))
    xs, vs, f = sysm.run(NO_FORCES, sysm.x0, v, 0, 200, want_forces=True)
    np.testing.assert_allclose(xs, sysm.x0 + 200 * NO_FORCES.dt * v, atol=1e-14)
    np.testing.assert_allclose(vs, v, atol=1e-14)
    assert np.abs(f).max() < 1e-9


def test_damping_dissipates():
    # with damping, gravity/ground off and no actuation, H~ decreases
    sysm, x, v = _perturbed_lattice(damping=5.0)
    def Ht(x, v):
        f = sysm.spring_forces(x, v, 0.0, 0.0)
        return sysm.kinetic(v) + sysm.spring_energy(x)
    e0 = Ht(x, v)
    x, v, _ = sysm.run(NO_FORCES, x, v, 0, 2000)
    assert Ht(x, v) < 0.5 * e0

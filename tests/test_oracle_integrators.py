"""Pins of the oracle's other integrators (Sec. III-B names Verlet and RK4
beside Euler).

Closed forms fix the arithmetic of each scheme: on a linear spring the RK4
step is the matrix polynomial I + Z + Z^2/2 + Z^3/6 + Z^4/24 of Z = dt A (A
the system matrix, damping included), and the velocity-Verlet step the
textbook matrix below; both are exact for constant acceleration.  Orders of
convergence against the exact solution of a spring whose rest length is
driven in time pin the stage times (t, t + dt/2, t + dt/2, t + dt) and
Verlet's end-of-step force time.  A sliding mass at its ground equilibrium
pins friction after the step (velocity and position), and conservation of
momentum and pinned masses pin the rest."""
import math

import numpy as np
import pytest

from oracle import oracle as O

K, M, L0 = 100.0, 0.5, 1.0
W2 = K / M


def _spring(u0=0.1, v0=0.0, c=None, amp=None, phase=None):
    """Mass 1 (M) on a spring of stiffness K and rest length L0 to a pinned
    mass 0 at the origin, displaced by u0 along x."""
    sc = dict(pos=np.array([[0.0, 0.0, 0.0], [L0 + u0, 0.0, 0.0]]),
              vel=np.array([[0.0, 0.0, 0.0], [v0, 0.0, 0.0]]),
              mass=np.array([0.0, M]), ends=np.array([[0, 1]]), k=np.array([K]),
              damping=None if c is None else np.array([c]),
              amp=None if amp is None else np.array([amp]), phase=None if phase is None else np.array([phase]))
    return O.System(sc, rest=np.array([L0]))


def _free(integrator, dt, omega=0.0):
    return O.Params(dt=dt, gravity=(0.0, 0.0, 0.0), ground=False, omega=omega, integrator=integrator)


def _run(sysm, p, nsteps):
    sysm.acc = None
    x, v, _ = sysm.run(p, sysm.x0, sysm.v0, 0, nsteps)
    return x[1, 0] - L0, v[1, 0]


def _rk4_map(A, h):
    Z = h * A
    I = np.eye(A.shape[0])
    return I + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24


@pytest.mark.parametrize("c", [None, 0.8])
def test_rk4_is_the_matrix_polynomial_of_the_linear_spring(c):
    h = 2e-3
    A = np.array([[0.0, 1.0], [-W2, -(0.0 if c is None else c / M)]])
    s = _spring(u0=0.1, v0=0.3, c=c)
    for n in (1, 50):
        u, v = _run(s, _free("rk4", h), n)
        want = np.linalg.matrix_power(_rk4_map(A, h), n) @ np.array([0.1, 0.3])
        assert np.allclose([u, v], want, rtol=1e-11, atol=1e-13), (n, [u, v], want)


def test_velocity_verlet_is_the_textbook_matrix():
    h = 2e-3
    q = h * h * W2
    Mv = np.array([[1 - q / 2, h], [-W2 * h * (1 - q / 4), 1 - q / 2]])
    s = _spring(u0=0.1, v0=0.3)
    for n in (1, 50):
        u, v = _run(s, _free("verlet", h), n)
        want = np.linalg.matrix_power(Mv, n) @ np.array([0.1, 0.3])
        assert np.allclose([u, v], want, rtol=1e-11, atol=1e-13), (n, [u, v], want)


@pytest.mark.parametrize("integrator", ["verlet", "rk4"])
def test_free_fall_is_exact(integrator):
    dt, n = 1e-3, 200
    sc = dict(pos=np.array([[0.0, 0.0, 5.0]]), vel=np.array([[0.2, 0.0, 1.5]]), mass=np.array([0.3]),
              ends=np.zeros((0, 2), np.int64), k=np.zeros(0))
    s = O.System(sc, rest=np.zeros(0))
    p = O.Params(dt=dt, gravity=(0.0, 0.0, -9.81), ground=False, integrator=integrator)
    x, v, _ = s.run(p, s.x0, s.v0, 0, n)
    t = n * dt
    assert abs(x[0, 2] - (5.0 + 1.5 * t - 9.81 * t * t / 2)) < 1e-12
    assert abs(v[0, 2] - (1.5 - 9.81 * t)) < 1e-12 and abs(x[0, 0] - 0.2 * t) < 1e-14


def _driven_exact(t, amp, Om, phi):
    """u'' + w^2 u = w^2 L0 amp sin(Om t + phi), u(0) = u'(0) = 0."""
    w = math.sqrt(W2)
    B = W2 * L0 * amp / (W2 - Om * Om)
    c1 = -B * math.sin(phi)
    c2 = -B * Om * math.cos(phi) / w
    return c1 * math.cos(w * t) + c2 * math.sin(w * t) + B * math.sin(Om * t + phi)


def _max_error(integrator, dt, amp, Om, phi, T):
    s = _spring(u0=0.0, amp=amp, phase=phi)
    s.acc = None
    p = _free(integrator, dt, omega=Om)
    x, v, err = s.x0, s.v0, 0.0
    for n in range(int(round(T / dt))):
        x, v, _ = s.run(p, x, v, n, 1)
        err = max(err, abs(x[1, 0] - L0 - _driven_exact((n + 1) * dt, amp, Om, phi)))
    return err


@pytest.mark.parametrize("integrator,order", [("euler", 1), ("verlet", 2), ("rk4", 4)])
def test_order_of_convergence_with_a_driven_rest_length(integrator, order):
    """The rest length L0 (1 + amp sin(Om t + phi)) drives the spring; the
    largest error over 0.5 s against the exact solution falls as dt^order
    (measured 1.00, 2.00, 4.00)."""
    amp, Om, phi, T = 0.05, 7.0, 0.4, 0.5
    errs = [_max_error(integrator, dt, amp, Om, phi, T) for dt in (2e-3, 1e-3, 5e-4)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - order) < 0.1 for r in rates), (errs, rates)


@pytest.mark.parametrize("integrator", ["verlet", "rk4"])
def test_friction_slide_after_the_step(integrator):
    """A mass at rest on the ground at its equilibrium depth, sliding at
    0.3 m/s: friction takes mu g dt off the speed each step and the position
    moves with the reduced speed, until it stops."""
    m, kg, mu, g, dt = 0.1, 1e5, 0.5, 9.81, 1e-3
    z0 = -m * g / kg
    sc = dict(pos=np.array([[0.0, 0.0, z0]]), vel=np.array([[0.3, 0.0, 0.0]]), mass=np.array([m]),
              ends=np.zeros((0, 2), np.int64), k=np.zeros(0))
    s = O.System(sc, rest=np.zeros(0))
    p = O.Params(dt=dt, gravity=(0.0, 0.0, -g), ground=True, ground_k=kg, mu=mu, integrator=integrator)
    x, v = s.x0, s.v0
    want_x, want_v = 0.0, 0.3
    for _ in range(80):
        x, v, _ = s.run(p, x, v, 0, 1)
        want_v = max(0.0, want_v - mu * g * dt)
        want_x += want_v * dt
        assert abs(v[0, 0] - want_v) < 1e-9 and abs(x[0, 0] - want_x) < 1e-9
        assert abs(x[0, 2] - z0) < 1e-12
    assert want_v == 0.0  # it stopped inside the window


@pytest.mark.parametrize("integrator", ["verlet", "rk4"])
def test_momentum_is_conserved_and_pinned_masses_stay(integrator):
    rng = np.random.Generator(np.random.PCG64(8))
    n = 12
    pos = rng.uniform(0, 1, (n, 3))
    vel = rng.normal(0, 0.5, (n, 3))
    mass = rng.uniform(0.1, 1.0, n)
    ends = np.array([(i, j) for i in range(n) for j in range(i + 1, n) if (i + 2 * j) % 3 == 0])
    sc = dict(pos=pos, vel=vel, mass=mass, ends=ends, k=rng.uniform(10, 100, len(ends)),
              damping=rng.uniform(0, 0.5, len(ends)), amp=rng.uniform(0, 0.1, len(ends)),
              phase=rng.uniform(0, 6.28, len(ends)))
    s = O.System(sc)
    p = O.Params(dt=1e-3, gravity=(0.0, 0.0, 0.0), ground=False, omega=5.0, integrator=integrator)
    x, v, _ = s.run(p, s.x0, s.v0, 0, 200)
    assert np.allclose((mass[:, None] * v).sum(0), (mass[:, None] * vel).sum(0), atol=1e-12)
    # a pinned mass keeps its position and its (nonzero) velocity
    sc2 = dict(sc, mass=np.concatenate([[0.0], mass[1:]]))
    s2 = O.System(sc2)
    x2, v2, _ = s2.run(p, s2.x0, s2.v0, 0, 50)
    assert np.array_equal(x2[0], pos[0]) and np.array_equal(v2[0], vel[0])


def test_verlet_carries_its_acceleration_across_calls():
    s = _spring(u0=0.1, v0=0.0, c=0.7)
    p = _free("verlet", 1e-3)
    s.acc = None
    xa, va, _ = s.run(p, s.x0, s.v0, 0, 40)
    s.acc = None
    x, v, _ = s.run(p, s.x0, s.v0, 0, 20)
    xb, vb, _ = s.run(p, x, v, 20, 20)  # continues with the carried acceleration
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    s.acc = None  # afresh: the damper now sees the synchronized velocity
    xc, vc, _ = s.run(p, x, v, 20, 20)
    assert not np.array_equal(vc, vb)
    # without damping the recomputed acceleration is the carried one
    u = _spring(u0=0.1, v0=0.2)
    u.acc = None
    xa, va, _ = u.run(p, u.x0, u.v0, 0, 40)
    u.acc = None
    x, v, _ = u.run(p, u.x0, u.v0, 0, 20)
    u.acc = None
    xb, vb, _ = u.run(p, x, v, 20, 20)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)


def test_rollouts_refuse_other_integrators():
    s = _spring(amp=0.1, phase=0.0)
    for integ in ("verlet", "rk4"):
        p = O.Params(dt=1e-3, omega=1.0, integrator=integ)
        with pytest.raises(ValueError):
            s.rollout_loss(p, 5)
        with pytest.raises(ValueError):
            s.rollout_grad(p, 5)

"""Long runs on the GPU against what the method fixes (the first-10-steps
parity tests live elsewhere):

* free fall with dt = 2^-10 and g = -9.8125 (both exact in FP32): every
  velocity and displacement of the first 400 steps is exactly representable,
  so the GPU must reproduce the closed form of the semi-implicit Euler
  recurrence, v_n = n g dt and z_n - z_0 = g dt^2 n (n + 1) / 2, bit for bit;
* a mass on a spring: after up to 30,000 steps the state equals M^n (u_0,
  v_0) with M the exact one-step map of the integrator on the linear spring
  (its discrete period 2 pi / theta, cos theta = 1 - (omega dt)^2 / 2);
* momentum: with gravity and ground off, internal forces cancel pairwise, so
  total momentum stays where it started (to FP32 accumulation);
* energy: undamped, the total energy stays bounded (no drift) and follows
  the FP64 oracle's."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_10274_amd import scenes

pytestmark = pytest.mark.gpu


def _T():
    from paper_1911_10274_amd import titan as T

    return T


def _sim(sc, **kw):
    T = _T()
    base = dict(dt=1e-4, gravity=(0.0, 0.0, 0.0), ground=False, ground_k=1e5, friction_mu=0.5, omega=0.0,
                engine=T.ENGINE_TILED)
    base.update(kw)
    return T.sim_from_scene(sc, T.Params(**base))


def test_free_fall_is_the_closed_form_bit_for_bit():
    dt, g = 2.0 ** -10, -9.8125
    sc = dict(pos=np.array([[0.0, 0.0, 1000.0], [5.0, 0.0, 1000.0]], np.float32),
              vel=np.zeros((2, 3), np.float32), mass=np.array([0.5, 2.0], np.float32),
              ends=np.zeros((0, 2), np.int64), k=np.zeros(0, np.float32))
    sim = _sim(sc, dt=dt, gravity=(0.0, 0.0, g))
    for n in (1, 2, 3, 50, 400):
        sim.step(n - sim.info()["step"])
        p, v, step = sim.get_state(displacement=True)
        assert step == n
        vz = n * g * dt
        dz = g * dt * dt * n * (n + 1) / 2
        assert np.all(v[:, 2] == np.float32(vz)) and np.all(v[:, :2] == 0.0)
        assert np.all(p[:, 2] == np.float32(dz)), (n, p[:, 2], dz)
    sim.close()


@pytest.mark.parametrize("engine", ["tiled", "batched"])
def test_spring_oscillator_follows_the_exact_discrete_map(engine):
    T = _T()
    k, m, L0, dt = 100.0, 0.5, 1.0, 1e-4
    w2 = k / m
    u0, v0 = 0.05, 0.2
    sc = dict(pos=np.array([[0.0, 0.0, 0.0], [L0 + u0, 0.0, 0.0]], np.float32),
              vel=np.array([[0.0, 0.0, 0.0], [v0, 0.0, 0.0]], np.float32), mass=np.array([0.0, m], np.float32),
              ends=np.array([[0, 1]]), k=np.array([k], np.float32))
    eng = T.ENGINE_TILED if engine == "tiled" else T.ENGINE_BATCHED
    sim = _sim(sc, dt=dt, engine=eng)
    # the rest length is the initial length, so the displacement from rest
    # starts at 0 with velocity v0
    M = np.array([[1.0 - dt * dt * w2, dt], [-dt * w2, 1.0]])  # (u, v) -> (u', v'), semi-implicit Euler
    theta = math.acos(1.0 - (math.sqrt(w2) * dt) ** 2 / 2)
    assert abs(2 * math.pi / theta * dt - 2 * math.pi / math.sqrt(w2)) < 1e-6  # ~ the continuous period
    amp = math.hypot(0.0, float(np.float32(v0)) / math.sqrt(w2))
    for n in (1000, 10000, 30000):
        sim.step(n - sim.info()["step"])
        p, v, _ = sim.get_state(displacement=True)
        want = np.linalg.matrix_power(M, n) @ np.array([0.0, float(np.float32(v0))])
        err = math.hypot(float(p[1, 0]) - want[0], (float(v[1, 0]) - want[1]) / math.sqrt(w2))
        print(engine, n, "relative state error", err / amp)
        assert err <= 1e-4 * amp, (n, want, err / amp)
    sim.close()


def test_momentum_is_conserved_over_a_long_run():
    sc = scenes.jittered_actuated_lattice(n=8, seed=7)
    rng = np.random.Generator(np.random.PCG64(3))
    sc = dict(sc, vel=rng.normal(0, 0.05, sc["pos"].shape).astype(np.float32))
    sim = _sim(sc, dt=5e-5, omega=2 * math.pi * 2)
    m = sc["mass"].astype(np.float64)[:, None]
    p0 = (m * sc["vel"].astype(np.float64)).sum(0)
    scale = float((m * np.abs(sc["vel"].astype(np.float64))).sum())
    worst = 0.0
    for n in (1000, 5000, 20000):
        sim.step(n - sim.info()["step"])
        _, v, _ = sim.get_state()
        worst = max(worst, float(np.abs((m * v.astype(np.float64)).sum(0) - p0).max()) / scale)
    sim.close()
    print("momentum drift", worst)
    assert worst <= 1e-5  # measured 1.2e-6


def test_undamped_energy_is_bounded_and_follows_the_oracle():
    sc = scenes.lattice(5, origin=(0.0, 0.0, 1.0))
    rng = np.random.Generator(np.random.PCG64(4))
    sc = dict(sc, damping=np.zeros(sc["ends"].shape[0], np.float32),
              vel=rng.normal(0, 0.2, sc["pos"].shape).astype(np.float32))
    dt = 1e-4
    sim = _sim(sc, dt=dt)
    sysm = O.System(sc)
    op = O.Params(dt=dt, gravity=(0.0, 0.0, 0.0), ground=False, omega=0.0)

    def energy(x, v):
        return sysm.kinetic(v) + sysm.spring_energy(x)

    e0 = energy(sysm.x0, sysm.v0)
    x, v, step = sysm.x0, sysm.v0, 0
    drift = follow = 0.0
    for n in (2000, 10000, 40000):
        x, v, _ = sysm.run(op, x, v, step, n - step)
        step = n
        sim.step(n - sim.info()["step"])
        p, vg, _ = sim.get_state(displacement=True)
        eg = energy(sysm.x0 + p.astype(np.float64), vg.astype(np.float64))
        er = energy(x, v)
        drift = max(drift, abs(eg - e0) / e0)
        follow = max(follow, abs(eg - er) / e0)
    sim.close()
    print("energy drift", drift, "vs oracle", follow)
    assert drift <= 1e-2 and follow <= 1e-3

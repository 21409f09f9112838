"""Pins of the oracle's breakable springs (Sec. III-E, material yield values
compared against in the force calculation).

Reading: the value compared is the magnitude of the elastic force
|k (l - L(t))|; a spring whose elastic force exceeds its yield value breaks
in that evaluation, exerts no force in it, and stays broken.  Hand-worked
single springs fix the comparison (magnitude, strictness, the actuated rest
length, damping excluded, coincident ends); whole-system identities fix the
bookkeeping (infinite yield = no yield; a broken spring = a deleted one)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_10274_amd import scenes


def _pair(x1, yield_, k=100.0, c=None, amp=None, phase=None, rest=1.0):
    """Mass 0 pinned at the origin, mass 1 at (x1, 0, 0); one spring."""
    sc = dict(pos=np.array([[0.0, 0.0, 0.0], [x1, 0.0, 0.0]]), mass=np.array([0.0, 1.0]),
              ends=np.array([[0, 1]]), k=np.array([k]), damping=None if c is None else np.array([c]),
              amp=None if amp is None else np.array([amp]), phase=None if phase is None else np.array([phase]),
              **{"yield": np.array([yield_])})
    return O.System(sc, rest=np.array([rest]))


def _forces(sysm, x=None, v=None, t=0.0, omega=0.0):
    x = sysm.x0 if x is None else x
    v = np.zeros_like(sysm.x0) if v is None else v
    return sysm.spring_forces(x, v, t, omega)


def test_stretched_spring_breaks_only_above_its_yield():
    # l = 1.1, L = 1: elastic force k (l - L) = 10 N along +x on mass 0
    s = _pair(1.1, 9.99)
    f = _forces(s)
    assert s.broken[0] == 1 and np.all(f == 0.0)
    s = _pair(1.1, 10.01)
    f = _forces(s)
    assert s.broken[0] == 0
    assert np.allclose(f[0], [10.0, 0, 0], rtol=1e-12) and np.allclose(f[1], [-10.0, 0, 0], rtol=1e-12)


def test_compressed_spring_compares_the_magnitude():
    s = _pair(0.9, 9.99)  # k (l - L) = -10 N
    _forces(s)
    assert s.broken[0] == 1
    s = _pair(0.9, 10.01)
    f = _forces(s)
    assert s.broken[0] == 0 and np.allclose(f[1], [10.0, 0, 0], rtol=1e-12)


def test_equal_to_the_yield_holds():
    # positions and rest chosen so that k (l - L) is exactly 8: l = 1.5, L = 1.25, k = 32
    s = _pair(1.5, 8.0, k=32.0, rest=1.25)
    f = _forces(s)
    assert s.broken[0] == 0 and f[0, 0] == 8.0


def test_broken_stays_broken():
    s = _pair(1.1, 9.99)
    _forces(s)
    assert s.broken[0] == 1
    x_rest = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    f = _forces(s, x=x_rest)
    assert s.broken[0] == 1 and np.all(f == 0.0)
    # a trajectory keeps it broken: the free mass only falls
    p = O.Params(dt=1e-3, gravity=(0.0, 0.0, -9.81), ground=False, omega=0.0)
    x, v, _ = s.run(p, x_rest, np.zeros((2, 3)), 0, 100)
    assert np.allclose(v[1], [0, 0, -9.81 * 0.1], rtol=1e-12) and x[1, 0] == 1.0


def test_damping_force_does_not_break():
    # at its rest length the elastic force is exactly zero; the damper pulls
    # with c * v_rel = 5 N, far above the yield value
    s = _pair(1.0, 1e-6, c=1.0)
    v = np.array([[0.0, 0, 0], [5.0, 0, 0]])
    f = _forces(s, v=v)
    assert s.broken[0] == 0 and np.allclose(f[0], [5.0, 0, 0], rtol=1e-12)


def test_coincident_ends_are_not_tested():
    s = _pair(0.0, 0.0)  # no direction: no force, and no break even at yield 0
    f = _forces(s)
    assert s.broken[0] == 0 and np.all(f == 0.0)


def test_actuated_rest_length_is_the_one_compared():
    # amp 0.5, phase pi/2 at t = 0: L = 1 * (1 + 0.5) = 1.5, l = 1: k (l - L) = -50 N
    s = _pair(1.0, 49.0, amp=0.5, phase=math.pi / 2)
    _forces(s, omega=3.0)
    assert s.broken[0] == 1
    s = _pair(1.0, 51.0, amp=0.5, phase=math.pi / 2)
    f = _forces(s, omega=3.0)
    assert s.broken[0] == 0 and np.allclose(f[1], [50.0, 0, 0], rtol=1e-12)
    # a quarter period later (omega t = pi/2): sin(pi) = 0, L = 1, no force
    s = _pair(1.0, 1e-9, amp=0.5, phase=math.pi / 2)
    f = _forces(s, t=math.pi / 6, omega=3.0)
    assert s.broken[0] == 0 and np.abs(f).max() < 1e-9


PRM = O.Params(dt=5e-5, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, mu=0.5, omega=2 * math.pi * 2)


def test_infinite_yield_is_no_yield():
    sc = scenes.jittered_actuated_lattice(n=5, seed=3)
    a = O.System(sc)
    b = O.System(dict(sc, **{"yield": np.full(sc["ends"].shape[0], np.inf)}))
    xa, va, fa = a.run(PRM, a.x0, a.v0, 0, 60, want_forces=True)
    xb, vb, fb = b.run(PRM, b.x0, b.v0, 0, 60, want_forces=True)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(fa, fb)
    assert not b.broken.any()


def test_a_broken_spring_is_a_deleted_spring():
    sc = scenes.jittered_actuated_lattice(n=5, seed=3)
    ns = sc["ends"].shape[0]
    gone = np.arange(3, ns, 11)
    keep = np.setdiff1d(np.arange(ns), gone)
    a = O.System(dict(sc, **{"yield": np.full(ns, np.inf)}))
    a.broken[gone] = 1
    b = O.System({**{k: (v[keep] if k in ("ends", "k", "damping", "amp", "phase") else v) for k, v in sc.items()}},
                 rest=O.System(sc).rest[keep])
    xa, va, fa = a.run(PRM, a.x0, a.v0, 0, 60, want_forces=True)
    xb, vb, fb = b.run(PRM, b.x0, b.v0, 0, 60, want_forces=True)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(fa, fb)


def test_springs_break_under_a_falling_load():
    """A cube dropped on the ground: springs with low yields break at the
    impact and the broken set only grows."""
    sc = scenes.cube_drop(5)
    ns = sc["ends"].shape[0]
    rng = np.random.Generator(np.random.PCG64(1))
    y = rng.uniform(1.0, 60.0, ns)
    s = O.System(dict(sc, **{"yield": y}))
    p = O.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, mu=0.5)
    x, v = s.x0, s.v0
    prev = s.broken.copy()
    for n in range(0, 4000, 200):  # the cube reaches the ground near step 3200
        x, v, _ = s.run(p, x, v, n, 200)
        assert np.all(s.broken >= prev)
        prev = s.broken.copy()
    assert 0 < s.broken.sum() < ns


def test_rollouts_refuse_breakable_springs():
    s = _pair(1.1, 20.0)
    p = O.Params(dt=1e-3, omega=1.0)
    with pytest.raises(ValueError):
        s.rollout_loss(p, 5)
    with pytest.raises(ValueError):
        s.rollout_grad(p, 5)

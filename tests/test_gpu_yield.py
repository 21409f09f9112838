"""Breakable springs (Sec. III-E yield values) on the GPU, through the C ABI.

A break is an integer decision taken from a floating-point value: the GPU
takes it in FP32, the oracle in FP64.  The parity test uses yields whose
decisions all clear the oracle's force by a margin far above FP32 rounding
(checked in the test), so both sides must break the same springs at the same
steps; the impact test compares each step's decisions from the GPU's own
state and excuses only decisions within that rounding."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_10274_amd import scenes
from tests.parity import TOL, assert_parity, compare_series, gpu_series, rel

pytestmark = pytest.mark.gpu

DT = 5e-5
OMEGA = 2 * math.pi * 2


def _T():
    from paper_1911_10274_amd import titan as T

    return T


def _params(engine=None, dt=DT, omega=OMEGA):
    T = _T()
    return T.Params(dt=dt, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5, omega=omega,
                    engine=T.ENGINE_TILED if engine is None else engine)


def _oparams(dt=DT, omega=OMEGA):
    return O.Params(dt=dt, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, mu=0.5, omega=omega)


def _elastic(sysm, x, t, omega):
    """|k (l - L(t))| per spring (for the margin checks only)."""
    d = x[sysm.ends[:, 1]] - x[sysm.ends[:, 0]]
    l = np.sqrt((d * d).sum(1))
    L = sysm.rest if sysm.amp is None else sysm.rest * (1 + sysm.amp * np.sin(omega * t + sysm.phase))
    return np.abs(sysm.k * (l - L))


def _lattice_with_yields(seed=4):
    sc = scenes.jittered_actuated_lattice(n=9, seed=6)
    s0 = O.System(sc)
    f0 = _elastic(s0, s0.x0, 0.0, OMEGA)
    rng = np.random.Generator(np.random.PCG64(seed))
    y = np.maximum((f0 * rng.uniform(0.6, 3.0, f0.size)).astype(np.float32), np.float32(1e-3))
    return dict(sc, **{"yield": y})


@pytest.mark.parametrize("engine", ["gather", "tiled", "batched"])
def test_first_10_steps_with_breaks_match_the_oracle(engine):
    T = _T()
    eng = {"gather": T.ENGINE_GATHER, "tiled": T.ENGINE_TILED, "batched": T.ENGINE_BATCHED}[engine]
    sc = _lattice_with_yields()
    sysm = O.System(dict(sc, **{"yield": sc["yield"].astype(np.float64)}))
    # every decision of the oracle's run clears the yield by >= 1e-4 (relative)
    x, v = sysm.x0, sysm.v0
    probe = O.System(dict(sc, **{"yield": sc["yield"].astype(np.float64)}))
    broken_per_step = []
    for n in range(10):
        e = _elastic(probe, x, n * DT, OMEGA)
        live = probe.broken == 0
        assert (np.abs(e[live] - probe.yield_[live]) / probe.yield_[live]).min() > 1e-4
        x, v, _ = probe.run(_oparams(), x, v, n, 1)
        broken_per_step.append(probe.broken.copy())
    sim = T.sim_from_scene(sc, _params(eng))
    gpu = gpu_series(sim, 10)
    assert sim.info()["engine"] == eng
    gb = sim.get_broken()
    sim.close()
    ref = sysm.trajectory(_oparams(), 10)
    assert np.array_equal(gb, sysm.broken.astype(bool))
    assert 1000 < gb.sum() < gb.size and not np.array_equal(broken_per_step[0], broken_per_step[-1])
    err = compare_series(gpu, ref, sysm.mass)
    print("yield", engine, err, int(gb.sum()))
    assert_parity(err)


def test_breaks_through_an_impact_step_by_step():
    """A cube hits the ground at 2 m/s; from the GPU's state at each step of
    the impact the oracle decides which springs break and computes the step's
    forces and velocity change with the GPU's broken set.  The cube starts
    with its lowest layer 1 mm above the ground, so that the FP32 sum
    reference z + displacement that the contact test reads is exact to
    ~1e-10 m (at a reference height of 0.5 m its rounding alone would move
    the penalty force by ~1e-4 of itself)."""
    T = _T()
    sc = scenes.contact_slide(6, v0=(0.3, 0.1, -2.0))
    rng = np.random.Generator(np.random.PCG64(12))
    y = rng.uniform(5.0, 80.0, sc["ends"].shape[0]).astype(np.float32)
    sc = dict(sc, **{"yield": y})
    dt = 1e-4
    sysm = O.System(dict(sc, **{"yield": y.astype(np.float64)}))
    sim = T.sim_from_scene(sc, _params(T.ENGINE_TILED, dt=dt, omega=0.0))
    floor = float(np.linalg.norm(sysm.mass * 9.81))
    worst = {"F": 0.0, "dV": 0.0}
    excused = 0
    b_prev = sim.get_broken()
    assert not b_prev.any()
    for n in range(0, 300):
        p, v, step = sim.get_state(displacement=True)
        assert step == n
        x = sysm.x0 + p.astype(np.float64)
        v = v.astype(np.float64)
        f_gpu = sim.get_forces().astype(np.float64)
        sim.step(1)
        b_new = sim.get_broken()
        assert np.all(b_new >= b_prev)  # breaks are permanent
        # the oracle's decisions from the GPU's state
        e = _elastic(sysm, x, n * dt, 0.0)
        want = b_prev | (e > y.astype(np.float64))
        close = np.abs(e - y) <= 1e-4 * y
        differ = (want != b_new) & ~b_prev
        assert not (differ & ~close).any(), np.nonzero(differ & ~close)
        excused += int(differ.sum())
        # the step's forces and velocity change with the GPU's decisions (an
        # excused spring the GPU kept is kept by the oracle too)
        flags = b_new.astype(np.uint8)
        sysm.yield_ = np.where(differ & ~b_new, np.inf, y.astype(np.float64))
        f_ref = sysm.spring_forces(x, v, n * dt, 0.0, broken=flags.copy())
        worst["F"] = max(worst["F"], rel(f_gpu, f_ref, floor))
        p2, v2, _ = sim.get_state(displacement=True)
        x1, v1, _ = sysm.run(_oparams(dt=dt, omega=0.0), x, v, n, 1, broken=flags.copy())
        # masses falling at ~2 m/s gain only g dt ~ 1e-3 m/s a step: one FP32
        # ulp of the stored velocity (2.4e-7) is already ~2e-4 of that, so each
        # component of the GPU's change is allowed its storage rounding first
        d = (v2 - v) - (v1 - v)
        d = np.sign(d) * np.maximum(np.abs(d) - np.spacing(np.abs(v2)).astype(np.float64), 0.0)
        worst["dV"] = max(worst["dV"], float(np.linalg.norm(d) / np.linalg.norm(v1 - v)))
        b_prev = b_new
    sim.close()
    print("impact", worst, "broken", int(b_prev.sum()), "excused", excused)
    assert b_prev.sum() > 300 and excused <= 2
    assert max(worst.values()) <= TOL


def test_engines_agree_bitwise_with_breaks():
    T = _T()
    sc = _lattice_with_yields(seed=2)
    outs = []
    for eng in (T.ENGINE_GATHER, T.ENGINE_TILED, T.ENGINE_BATCHED):
        sim = T.sim_from_scene(sc, _params(eng))
        sim.step(400)
        assert sim.info()["engine"] == eng
        outs.append(sim.get_state(displacement=True)[:2] + (sim.get_forces(), sim.get_broken()))
        sim.close()
    assert outs[0][3].sum() > 1300
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


def test_broken_springs_exert_exactly_nothing():
    """Forces of a state with broken springs are bitwise those of the same
    state in a system where the broken springs were removed (and the rest
    unbreakable, so that both run the same kernel)."""
    T = _T()
    sc = _lattice_with_yields(seed=3)
    a = T.sim_from_scene(sc, _params())
    a.step(50)
    p, v, _ = a.get_state(displacement=True)
    fa = a.get_forces()  # leaves out the springs that break in step 50 too
    a.step(1)
    gone = np.nonzero(a.get_broken())[0]
    a.close()
    assert gone.size > 1000
    b = T.sim_from_scene(dict(sc, **{"yield": np.full(sc["ends"].shape[0], np.inf, np.float32)}), _params())
    b.step(1)
    b.set_state(p, v, displacement=True)
    b.set_step(50)
    b.remove_springs(gone)
    fb = b.get_forces()
    b.close()
    assert np.array_equal(fa, fb)


def test_yields_set_while_running():
    """Yields set after the first step rebuild the layout (no yields before)
    or are written in place (infinite yields before): the same bits."""
    T = _T()
    sc = scenes.cube_drop(6)
    ns = sc["ends"].shape[0]
    y = np.random.Generator(np.random.PCG64(5)).uniform(5.0, 80.0, ns).astype(np.float32)
    runs = []
    for before in (None, np.full(ns, np.inf, np.float32)):
        sim = T.sim_from_scene(dict(sc, **{"yield": before}), _params(T.ENGINE_TILED, dt=1e-4, omega=0.0))
        sim.step(3000)
        builds = sim.info()["layout_builds"]
        sim.set_yield(y)
        sim.step(400)
        i = sim.info()
        assert i["layout_builds"] == builds + (1 if before is None else 0)
        runs.append(sim.get_state(displacement=True) + (sim.get_broken(),))
        sim.close()
    (pa, va, sa, ba), (pb, vb, sb, bb) = runs
    assert sa == sb == 3400 and ba.sum() > 20
    assert np.array_equal(pa, pb) and np.array_equal(va, vb) and np.array_equal(ba, bb)


def test_breaks_survive_edits_and_yield_changes():
    T = _T()
    sc = _lattice_with_yields(seed=4)
    sim = T.sim_from_scene(sc, _params())
    sim.step(5)
    b5 = sim.get_broken()
    assert b5.any()
    # raising every yield does not mend a broken spring
    sim.set_yield(np.full(b5.size, np.inf, np.float32))
    sim.step(5)
    assert np.array_equal(sim.get_broken(), b5)
    # a rebuild (a mass added) keeps them, and a spring added after it is intact
    builds = sim.info()["layout_builds"]
    sim.add_masses([[5.0, 5.0, 5.0]], [0.1])
    sim.step(5)
    assert sim.info()["layout_builds"] == builds + 1
    assert np.array_equal(sim.get_broken(), b5)
    first = sim.add_springs([[0, 1]], [1e3])
    sim.step(5)
    b = sim.get_broken()
    assert np.array_equal(b[:first], b5) and not b[first]
    sim.close()


def test_yield_errors():
    T = _T()
    sc = scenes.lattice(3, origin=(0.0, 0.0, 1.0))
    sim = T.sim_from_scene(sc, _params())
    ns = sc["ends"].shape[0]
    for bad in (0.0, -1.0, np.nan):
        with pytest.raises(T.TitanError) as ei:
            sim.set_yield([bad])
        assert ei.value.code == T.EINVAL
    with pytest.raises(T.TitanError) as ei:
        sim.set_yield(np.ones(2, np.float32), first=ns - 1)
    assert ei.value.code == T.EINVAL
    sim.set_yield(np.full(ns, 1e6, np.float32))
    sim.step(2)
    with pytest.raises(T.TitanError) as ei:
        sim.rollout_grad(4, 2)
    assert ei.value.code == T.ESTATE
    assert not sim.get_broken().any()
    sim.close()

"""Captured step loops (titan_params.graph_steps): a HIP graph of step
launches replayed with the step index read from a device clock must give the
bits of launching the steps one by one -- on every replay, with the
program's own work and synchronisations between replays (reads of the state,
edits, parameter changes, breakpoints), under both actuation laws."""
import math

import numpy as np
import pytest

from paper_1911_10274_amd import scenes

pytestmark = pytest.mark.gpu


def _T():
    from paper_1911_10274_amd import titan as T

    return T


def _params(graph_steps, engine=None, **kw):
    T = _T()
    base = dict(dt=5e-5, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5,
                omega=2 * math.pi * 2, engine=T.ENGINE_TILED if engine is None else engine)
    base.update(kw)
    return T.Params(graph_steps=graph_steps, **base)


@pytest.mark.parametrize("engine", ["gather", "tiled"])
def test_replays_match_one_by_one_launches(engine):
    T = _T()
    eng = T.ENGINE_GATHER if engine == "gather" else T.ENGINE_TILED
    sc = scenes.jittered_actuated_lattice(n=9, seed=2)
    a = T.sim_from_scene(sc, _params(64, eng))
    b = T.sim_from_scene(sc, _params(0, eng))
    for chunk in (300, 7, 128, 1, 513, 64, 66):  # whole replays, remainders, odd parities
        a.step(chunk)
        b.step(chunk)
        pa, va, sa = a.get_state(displacement=True)
        pb, vb, sb = b.get_state(displacement=True)
        assert sa == sb
        assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    assert np.array_equal(a.get_forces(), b.get_forces())
    a.close()
    b.close()


def test_replays_across_edits_parameters_and_breakpoints():
    T = _T()
    sc = scenes.jittered_actuated_lattice(n=8, seed=5)
    runs = []
    for g in (32, 0):
        sim = T.sim_from_scene(sc, _params(g))
        sim.step(100)
        sim.remove_springs([3, 50, 400])
        sim.step(100)
        sim.set_params(_params(g, gravity=(0.0, 0.0, -3.0)))
        bp = sim.set_breakpoint(260, T.BP_PAUSE)
        sim.step(200)
        sim.wait(bp)
        sim.set_springs(0, np.full(10, 123.0, np.float32))
        sim.resume()
        p, v, s = sim.get_state(displacement=True)
        runs.append((p, v, s))
        sim.close()
    (pa, va, sa), (pb, vb, sb) = runs
    assert sa == sb == 400
    assert np.array_equal(pa, pb) and np.array_equal(va, vb)


def test_wave_law_clock_in_a_graph():
    """The wave law reads the step's time in FP64 from the device clock:
    2400 steps of the worm cross period boundaries inside replays."""
    T = _T()
    sc = scenes.worm_batch(2, nx=10)
    outs = []
    for g in (256, 0):
        tp = _params(g, dt=1e-4, omega=20.0, actuation=T.ACT_WAVE, wave_period=1.0)
        sim = T.sim_from_scene(sc, tp)
        sim.step(2400)
        outs.append(sim.get_state(displacement=True)[:2])
        sim.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_graph_steps_rules():
    T = _T()
    sc = scenes.lattice(3, origin=(0.0, 0.0, 1.0))
    for bad in (3, -2, 8192):
        with pytest.raises(T.TitanError) as ei:
            T.sim_from_scene(sc, _params(bad))
        assert ei.value.code == T.EINVAL

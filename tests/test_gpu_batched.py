"""Batched engine: many independent voxel robots stepped by one launch, each
group of robots resident in LDS.  Checked against the FP64 oracle per step,
and bitwise against the per-step tiled engine over long runs (both engines
use the same per-mass summation order and arithmetic)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_10274_amd import scenes
from tests.parity import assert_parity, both_params, compare_series, gpu_series

pytestmark = pytest.mark.gpu

BATCHED, TILED, AUTO = 2, 3, 0


def _batch(count=48, seed=3, lo=3, hi=12):
    return scenes.concat(scenes.robot_batch(count, seed=seed, side_lo=lo, side_hi=hi))


def test_batched_engine_is_selected_and_tuned():
    from paper_1911_10274_amd import titan as T

    sc = _batch()
    tp, _ = both_params(dt=1e-4, omega=2 * math.pi * 2, engine=BATCHED)
    sim = T.sim_from_scene(sc, tp)
    sim.finalize()
    info = sim.info()
    assert info["engine"] == BATCHED
    assert info["batch_threads"] in (256, 512, 1024)
    assert info["tune_batch_ms"] > 0
    assert info["n_bodies"] == 48
    # the packing the tuner chose: at least the largest robot per group, more
    # only up to 2048 masses
    largest = max(np.bincount(sc["body"]))
    assert largest <= info["batch_max_group"] <= max(largest, 2048)
    assert 1 <= info["batch_groups"] <= 48
    sim.close()


@pytest.mark.parametrize("lo,hi", [(3, 4), (4, 6)])
def test_packing_choice_keeps_the_bits(lo, hi):
    """Small robots leave the tuner several packings (bodies per group);
    whichever it picks, the run equals the tiled engine's bit for bit."""
    from paper_1911_10274_amd import titan as T

    sc = _batch(count=300, seed=17, lo=lo, hi=hi)
    outs = []
    for eng in (BATCHED, TILED):
        tp, _ = both_params(dt=1e-4, omega=2 * math.pi * 2, engine=eng)
        sim = T.sim_from_scene(sc, tp)
        sim.finalize()
        info = sim.info()
        assert info["engine"] == eng
        if eng == BATCHED:
            print("packing", lo, hi, "groups", info["batch_groups"], "largest group", info["batch_max_group"],
                  "threads", info["batch_threads"])
        sim.step(300)
        outs.append(sim.get_state(displacement=True))
        sim.close()
    for a, b in zip(outs[0][:2], outs[1][:2]):
        assert np.array_equal(a, b)


def test_batched_parity_10_steps():
    from paper_1911_10274_amd import titan as T

    sc = _batch()
    tp, op = both_params(dt=1e-4, omega=2 * math.pi * 2, engine=BATCHED)
    sim = T.sim_from_scene(sc, tp)
    gpu = gpu_series(sim, 10)
    assert sim.info()["engine"] == BATCHED
    sim.close()
    sysm = O.System(sc)
    err = compare_series(gpu, sysm.trajectory(op, 10), sysm.mass)
    print("batched robots", err)
    assert_parity(err)


@pytest.mark.parametrize("steps", [1, 37, 2000])
def test_batched_equals_tiled_bitwise(steps):
    from paper_1911_10274_amd import titan as T

    sc = _batch(count=40, seed=11)
    outs = []
    for eng in (BATCHED, TILED):
        tp, _ = both_params(dt=1e-4, omega=2 * math.pi * 2, engine=eng)
        sim = T.sim_from_scene(sc, tp)
        sim.step(steps)
        assert sim.info()["engine"] == eng
        outs.append(sim.get_state(displacement=True))
        sim.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_batched_single_cube_matches_oracle_and_chunks():
    # one body: the whole 1000-mass cube lives in one workgroup's LDS
    from paper_1911_10274_amd import titan as T

    sc = scenes.contact_slide()
    tp, op = both_params(dt=1e-4, engine=BATCHED)
    sim = T.sim_from_scene(sc, tp)
    bp = sim.set_breakpoint(150)
    sim.step(300)  # one launch split at the breakpoint
    sim.wait(bp)
    p150, v150, step = sim.get_snapshot(bp, displacement=True)
    assert step == 150 and sim.info()["engine"] == BATCHED
    sysm = O.System(sc)
    x, v, _ = sysm.run(op, sysm.x0, sysm.v0, 0, 150)
    assert np.linalg.norm(p150 - (x - sysm.x0)) / np.linalg.norm(x - sysm.x0) < 1e-4
    assert np.linalg.norm(v150 - v) / np.linalg.norm(v) < 1e-4
    sim.close()


def test_auto_picks_a_valid_engine_and_reports_timings():
    from paper_1911_10274_amd import titan as T

    sc = _batch(count=64, seed=5, lo=3, hi=8)
    tp, _ = both_params(dt=1e-4, omega=2 * math.pi * 2, engine=AUTO)
    sim = T.sim_from_scene(sc, tp)
    sim.finalize()
    info = sim.info()
    print("auto", info)
    assert info["engine"] in (BATCHED, TILED)
    assert info["tune_gather_ms"] > 0 and info["tune_batch_ms"] > 0
    sim.close()


def test_tiny_bodies_and_isolated_masses():
    # bodies of one mass (no springs) and of two masses, packed into groups
    from paper_1911_10274_amd import titan as T

    rng = np.random.Generator(np.random.PCG64(1))
    n1 = 300
    pos = np.concatenate([rng.uniform(0, 5, (n1, 3)), rng.uniform(0, 5, (2 * n1, 3))]).astype(np.float32)
    pos[:, 2] += 0.5
    body = np.concatenate([np.arange(n1), n1 + np.repeat(np.arange(n1), 2)]).astype(np.int32)
    ends = np.stack([n1 + 2 * np.arange(n1), n1 + 2 * np.arange(n1) + 1], 1)
    sc = dict(pos=pos, vel=rng.uniform(-1, 1, pos.shape).astype(np.float32),
              mass=np.full(3 * n1, 0.1, np.float32), ends=ends, k=np.full(n1, 50.0, np.float32),
              damping=np.full(n1, 0.1, np.float32), amp=None, phase=None, body=body)
    tp, op = both_params(dt=1e-3, engine=BATCHED)
    sim = T.sim_from_scene(sc, tp)
    gpu = gpu_series(sim, 10)
    assert sim.info()["engine"] == BATCHED
    sim.close()
    sysm = O.System(sc)
    err = compare_series(gpu, sysm.trajectory(op, 10), sysm.mass)
    print("tiny bodies", err)
    assert_parity(err)


def test_batched_ineligible_body_is_rejected():
    # a single 100^3 lattice cannot sit in one workgroup's LDS
    from paper_1911_10274_amd import titan as T

    sc = scenes.lattice(20)  # 8000 masses > LDS capacity of one group
    tp, _ = both_params(dt=1e-4, engine=BATCHED)
    sim = T.sim_from_scene(sc, tp)
    with pytest.raises(T.TitanError) as ei:
        sim.finalize()
    assert ei.value.code == T.EINVAL
    sim.close()

"""The entry point that allocates nothing (titan_get_body_displacement_noalloc)
against titan_get_body_displacement, through the C ABI: equal bit for bit on
two calls in a row, the second on a smaller system (the library's fixed
device array keeps the first call's contents), and refusals beyond its
limits."""
import numpy as np
import pytest

from paper_1911_10274_amd import scenes

pytestmark = pytest.mark.gpu


def _sim(robots, steps):
    from paper_1911_10274_amd import titan as T

    sc = scenes.concat(robots)
    p = T.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5,
                 omega=2 * np.pi * 2)
    sim = T.sim_from_scene(sc, p)
    sim.step(steps)
    return sim


def test_noalloc_body_displacement_equals_the_allocating_call():
    from paper_1911_10274_amd import titan as T

    print("no-alloc: 64 robots, then 5 robots", flush=True)
    big = _sim(scenes.robot_batch(64, seed=21, side_lo=3, side_hi=8), 300)
    small = _sim(scenes.robot_batch(5, seed=22, side_lo=3, side_hi=4), 200)
    want_big = big.body_displacement()
    want_small = small.body_displacement()
    got_big = big.body_displacement_noalloc()
    got_small = small.body_displacement_noalloc()
    assert want_big.shape == (64, 3) and want_small.shape == (5, 3)
    assert np.abs(want_big).max() > 0 and np.abs(want_small).max() > 0
    np.testing.assert_array_equal(got_big, want_big)
    np.testing.assert_array_equal(got_small, want_small)
    # and again on the first system after the second: nothing left over
    np.testing.assert_array_equal(big.body_displacement_noalloc(), want_big)
    big.close()
    small.close()


def test_noalloc_limits_and_state():
    from paper_1911_10274_amd import titan as T

    print("no-alloc: refusals", flush=True)
    # before the device state exists
    sim = T.Sim(T.Params())
    sim.add_masses([[0, 0, 1.0]], [0.1])
    with pytest.raises(T.TitanError) as ei:
        sim.body_displacement_noalloc()
    assert ei.value.code == T.ESTATE
    sim.close()
    # more bodies than the fixed array holds (65,537 one-mass bodies)
    n = 65537
    sim = T.Sim(T.Params(ground=False, engine=T.ENGINE_GATHER))
    pos = np.zeros((n, 3), np.float32)
    pos[:, 0] = np.arange(n, dtype=np.float32)
    sim.add_masses(pos, np.full(n, 0.1, np.float32), body=np.arange(n, dtype=np.int32))
    sim.step(1)
    with pytest.raises(T.TitanError) as ei:
        sim.body_displacement_noalloc()
    assert ei.value.code == T.EINVAL
    want = sim.body_displacement()  # the allocating call has no such limit
    assert want.shape == (n, 3)
    sim.close()

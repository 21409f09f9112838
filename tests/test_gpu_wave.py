"""The worm's wave actuation (Sec. IV-B, Eqs. 3-5) on the GPU against the
FP64 oracle, through the C ABI.

The rest length is L0 (1 + c sin(omega tau)), tau = (T - t_o) mod t_p in
[0, t_p), t_o from Eq. 5; the oracle computes its own offsets from the same
reference positions (oracle.wave_offsets)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_10274_amd import scenes
from tests.parity import TOL, assert_parity, compare_series, gpu_series, rel

pytestmark = pytest.mark.gpu

OMEGA, PERIOD, DT = 20.0, 1.0, 1e-4  # the paper's worm: omega = 20, t_p = 1 s, c = 0.2


def _T():
    from paper_1911_10274_amd import titan as T

    return T


def _params(engine):
    T = _T()
    tp = T.Params(dt=DT, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5, omega=OMEGA,
                  engine=engine, actuation=T.ACT_WAVE, wave_period=PERIOD)
    op = O.Params(dt=DT, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, mu=0.5, omega=OMEGA, wave=True,
                  period=PERIOD)
    return tp, op


def _oracle(sc):
    return O.System(dict(sc, phase=O.wave_offsets(sc["pos"], sc["ends"], sc.get("body"))))


@pytest.mark.parametrize("engine", ["gather", "tiled"])
def test_worm_first_10_steps(engine):
    T = _T()
    sc = scenes.worm()
    tp, op = _params(T.ENGINE_GATHER if engine == "gather" else T.ENGINE_TILED)
    sim = T.sim_from_scene(sc, tp)
    sysm = _oracle(sc)
    gpu = gpu_series(sim, 10)
    sim.close()
    err = compare_series(gpu, sysm.trajectory(op, 10), sysm.mass)
    print("worm", engine, err)
    assert_parity(err)


def test_worm_window_across_a_period_boundary():
    """Steps 995-1010: springs whose offset is 0.1 s wrap from tau ~ t_p to
    tau ~ 0 between steps 1000 and 1001 (their actuation factor jumps from
    c sin(20) to ~0).  Each step is compared locally: the oracle's spring
    force and one oracle step's velocity change from the GPU's own state
    (<= 1e-5), and one step's position change to within what FP32 storage
    allows: the spacing of the stored displacement (centimetres after 1000
    steps), the velocity difference times dt, and the FP32 rounding of dt
    itself times the velocity (the worm's masses move at metres per second)."""
    T = _T()
    sc = scenes.worm()
    tp, op = _params(T.ENGINE_TILED)
    sim = T.sim_from_scene(sc, tp)
    sysm = _oracle(sc)
    t_o = sysm.phase
    sim.step(995)
    floor = float(np.linalg.norm(sysm.mass * 9.81))
    worst = {"F": 0.0, "dV": 0.0}
    eps32 = float(np.finfo(np.float32).eps)
    dt32_err = abs(float(np.float32(DT)) - DT)
    for n in range(995, 1011):
        p, v, step = sim.get_state(displacement=True)
        assert step == n
        x = sysm.x0 + p.astype(np.float64)
        v = v.astype(np.float64)
        f_gpu = sim.get_forces().astype(np.float64)
        f_ref = sysm.spring_forces(x, v, n * DT, OMEGA, wave=True, period=PERIOD)
        worst["F"] = max(worst["F"], rel(f_gpu, f_ref, floor))
        x1, v1, _ = sysm.run(op, x, v, n, 1)
        sim.step(1)
        p2, v2, _ = sim.get_state(displacement=True)
        # one step's change of velocity and position, GPU vs oracle
        worst["dV"] = max(worst["dV"], rel(v2 - v, v1 - v))
        dx_err = np.abs((sysm.x0 + p2 - x) - (x1 - x))
        bound = 2 * eps32 * np.abs(p2) + DT * np.abs(v2 - v1) + dt32_err * np.abs(v2) + 1e-12
        assert np.all(dx_err <= bound), float((dx_err / bound).max())
    sim.close()
    # the window holds a wrap: some spring's tau falls by most of a period
    u0 = 1000 * DT - t_o
    u1 = 1001 * DT - t_o
    tau0 = u0 - PERIOD * np.floor(u0 / PERIOD)
    tau1 = u1 - PERIOD * np.floor(u1 / PERIOD)
    assert np.any(tau0 - tau1 > 0.5 * PERIOD)
    print("wrap window", worst)
    assert max(worst.values()) <= TOL


def test_worm_batch_engines_agree_bitwise():
    T = _T()
    sc = scenes.worm_batch(3, nx=12)
    outs = []
    for eng in (T.ENGINE_GATHER, T.ENGINE_TILED, T.ENGINE_BATCHED):
        tp, _ = _params(eng)
        sim = T.sim_from_scene(sc, tp)
        sim.step(1200)  # crosses period boundaries of several offsets
        assert sim.info()["engine"] == eng
        outs.append(sim.get_state(displacement=True)[:2] + (sim.get_forces(),))
        sim.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


def test_hundred_worms_full_size_10_steps():
    """The paper's 100-worm swarm (339,200 springs) on the batched engine."""
    T = _T()
    sc = scenes.worm_batch(100)
    assert sc["ends"].shape[0] == 339200
    tp, op = _params(T.ENGINE_BATCHED)
    sim = T.sim_from_scene(sc, tp)
    assert sim.info()["engine"] == T.ENGINE_BATCHED
    sysm = _oracle(sc)
    gpu = gpu_series(sim, 10)
    sim.close()
    err = compare_series(gpu, sysm.trajectory(op, 10), sysm.mass)
    print("100 worms", err)
    assert_parity(err)


def test_wave_law_refusals():
    T = _T()
    sc = scenes.worm(6, 3, 2)
    tp, _ = _params(T.ENGINE_TILED)
    sim = T.sim_from_scene(sc, tp)
    sim.step(1)
    with pytest.raises(T.TitanError) as ei:
        sim.rollout_grad(10, 5)
    assert ei.value.code == T.ESTATE
    phasor = T.Params(dt=DT, omega=OMEGA, engine=T.ENGINE_TILED)
    with pytest.raises(T.TitanError) as ei:
        sim.set_params(phasor)
    assert ei.value.code == T.ESTATE
    sim.close()
    bad = T.Params(dt=DT, omega=OMEGA, actuation=T.ACT_WAVE, wave_period=0.0)
    with pytest.raises(T.TitanError) as ei:
        T.sim_from_scene(sc, bad)
    assert ei.value.code == T.EINVAL

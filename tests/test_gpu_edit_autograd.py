"""Spring constants pushed into a built simulation (titan_set_springs) and the
torch.autograd.Function over the adjoint."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_10274_amd import scenes

pytestmark = pytest.mark.gpu

OMEGA = 2 * math.pi * 2


def _tp(engine=0):
    from paper_1911_10274_amd import titan as T

    return T.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5, omega=OMEGA,
                    engine=engine)


def test_set_springs_equals_building_with_them():
    from paper_1911_10274_amd import titan as T

    robots = scenes.robot_batch(6, seed=21, side_lo=3, side_hi=6)
    sc = scenes.concat(robots)
    rng = np.random.Generator(np.random.PCG64(0))
    ns = sc["ends"].shape[0]
    k2 = rng.uniform(5e3, 2e4, ns).astype(np.float32)
    amp2 = rng.uniform(0, 0.2, ns).astype(np.float32)
    ph2 = rng.uniform(0, 2 * np.pi, ns).astype(np.float32)
    sc2 = dict(sc, k=k2, amp=amp2, phase=ph2)
    for eng in (T.ENGINE_TILED, T.ENGINE_BATCHED):
        a = T.sim_from_scene(sc2, _tp(eng))
        a.step(60)
        pa = a.get_state(displacement=True)
        b = T.sim_from_scene(sc, _tp(eng))
        b.finalize()  # uniform k layout first, then per-slot k appears
        b.set_springs(0, k=k2, amp=amp2, phase=ph2)
        b.step(60)
        pb = b.get_state(displacement=True)
        assert np.array_equal(pa[0], pb[0]) and np.array_equal(pa[1], pb[1])
        a.close()
        b.close()


def test_set_springs_at_a_pause_applies_at_that_step():
    from paper_1911_10274_amd import titan as T

    sc = scenes.jittered_actuated_lattice(n=10, seed=3)
    ns = sc["ends"].shape[0]
    k2 = (sc["k"] * 1.5).astype(np.float32)
    a = T.sim_from_scene(sc, _tp(T.ENGINE_TILED))
    bp = a.set_breakpoint(20, T.BP_PAUSE)
    a.step(50)
    a.wait(bp)
    a.set_springs(0, k=k2)
    a.resume()
    pa = a.get_state(displacement=True)
    b = T.sim_from_scene(sc, _tp(T.ENGINE_TILED))
    b.step(20)
    b.set_springs(0, k=k2)
    b.step(30)
    pb = b.get_state(displacement=True)
    assert pa[2] == pb[2] == 50
    assert np.array_equal(pa[0], pb[0]) and np.array_equal(pa[1], pb[1])
    # and the oracle agrees that the stiffness changed at step 20
    sysm = O.System(sc)
    op = O.Params(dt=1e-4, gravity=(0, 0, -9.81), ground=True, ground_k=1e5, mu=0.5, omega=OMEGA)
    x, v, _ = sysm.run(op, sysm.x0, sysm.v0, 0, 20)
    sysm.k = k2.astype(np.float64)
    x, v, _ = sysm.run(op, x, v, 20, 30)
    assert np.linalg.norm(pa[0] - (x - sysm.x0)) / np.linalg.norm(x - sysm.x0) < 1e-4
    a.close()
    b.close()


def test_autograd_function_matches_adjoint_and_oracle():
    import torch

    from paper_1911_10274_amd import titan as T
    from paper_1911_10274_amd.autograd import TitanRollout

    robots = scenes.robot_batch(4, seed=4, side_lo=4, side_hi=6)
    sc = scenes.concat(robots)
    sim = T.sim_from_scene(sc, _tp())
    ns = sc["ends"].shape[0]
    c = (sc["amp"].astype(np.float64) * np.cos(sc["phase"])).astype(np.float32)
    s = (sc["amp"].astype(np.float64) * np.sin(sc["phase"])).astype(np.float32)
    k = torch.tensor(sc["k"], requires_grad=True)
    C = torch.tensor(c, requires_grad=True)
    S = torch.tensor(s, requires_grad=True)
    spring_body = torch.tensor(sc["body"][sc["ends"][:, 0]], dtype=torch.int64)
    J = TitanRollout.apply(k, C, S, sim, 300, 50, spring_body)
    w = torch.tensor([1.0, -2.0, 0.5, 3.0])
    (J * w).sum().backward()
    # the oracle's adjoint of the same weighted loss
    sysm = O.System(dict(sc, amp=np.hypot(c, s), phase=np.arctan2(s, c)))
    op = O.Params(dt=1e-4, gravity=(0, 0, -9.81), ground=True, ground_k=1e5, mu=0.5, omega=OMEGA)
    ref = sysm.rollout_grad(op, 300, body=sc["body"], weights=w.numpy().astype(np.float64))
    np.testing.assert_allclose(J.detach().numpy(), ref["loss"], rtol=1e-3)
    for got, want in ((k.grad, ref["gk"]), (C.grad, ref["gC"]), (S.grad, ref["gS"])):
        g = got.numpy().astype(np.float64)
        assert np.linalg.norm(g - want) / np.linalg.norm(want) <= 1e-3
    sim.close()


def test_gradient_ascent_moves_the_robot_further():
    # a few steps of gradient descent on J = -(x-displacement) using the
    # simulator's own gradients must make the robot travel further in x
    import torch

    from paper_1911_10274_amd import titan as T
    from paper_1911_10274_amd.autograd import TitanRollout

    r = scenes.robot_batch(1, seed=31, side_lo=5, side_hi=5)[0]
    sim = T.sim_from_scene(r, _tp())
    c = torch.tensor((r["amp"].astype(np.float64) * np.cos(r["phase"])).astype(np.float32), requires_grad=True)
    s = torch.tensor((r["amp"].astype(np.float64) * np.sin(r["phase"])).astype(np.float32), requires_grad=True)
    k = torch.tensor(r["k"])
    body = torch.zeros(r["ends"].shape[0], dtype=torch.int64)
    opt = torch.optim.Adam([c, s], lr=0.01)
    losses = []
    for _ in range(6):
        opt.zero_grad()
        J = TitanRollout.apply(k, c, s, sim, 800, 100, body)
        J.sum().backward()
        opt.step()
        with torch.no_grad():  # keep amplitudes physical
            a = torch.clamp(torch.hypot(c, s), max=0.3)
            ph = torch.atan2(s, c)
            c.copy_(a * torch.cos(ph))
            s.copy_(a * torch.sin(ph))
        losses.append(float(J.detach().sum()))
    print("losses", losses)
    assert losses[-1] < losses[0]
    sim.close()


def test_autograd_function_on_gpu_tensors_equals_cpu_tensors():
    # parameters on the GPU: loss and gradients come back through the
    # device-output call and are the same bits as the host-output path
    import torch

    from paper_1911_10274_amd import titan as T
    from paper_1911_10274_amd.autograd import TitanRollout

    robots = scenes.robot_batch(3, seed=6, side_lo=3, side_hi=5)
    sc = scenes.concat(robots)
    sim = T.sim_from_scene(sc, _tp())
    c = (sc["amp"].astype(np.float64) * np.cos(sc["phase"])).astype(np.float32)
    s = (sc["amp"].astype(np.float64) * np.sin(sc["phase"])).astype(np.float32)
    spring_body = torch.tensor(sc["body"][sc["ends"][:, 0]], dtype=torch.int64)
    w = [1.0, -0.5, 2.0]
    got = []
    for dev in ("cpu", "cuda"):
        k = torch.tensor(sc["k"], device=dev, requires_grad=True)
        C = torch.tensor(c, device=dev, requires_grad=True)
        S = torch.tensor(s, device=dev, requires_grad=True)
        J = TitanRollout.apply(k, C, S, sim, 200, 40, spring_body.to(dev))
        assert J.device.type == dev
        (J * torch.tensor(w, device=dev)).sum().backward()
        assert k.grad.device.type == dev
        got.append([t.detach().cpu().numpy() for t in (J, k.grad, C.grad, S.grad)])
    for a, b in zip(*got):
        assert np.array_equal(a, b)
    sim.close()

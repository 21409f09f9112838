"""Pins of the FP64 oracle's rollout gradient (the adjoint of the step):
central finite differences of the oracle's own forward rollout, and the
derivative of the oscillator's discrete closed form."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_10274_amd import scenes

P = O.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, mu=0.5, omega=2 * math.pi * 2)


def _robot_system(r, va=None, vphi=None):
    """A voxel robot as an FP64 oracle system whose spring actuation comes from
    the voxel parameters in FP64 (so finite differences see the same map)."""
    va = r["voxel_a"] if va is None else va
    vphi = r["voxel_phi"] if vphi is None else vphi
    amp, ph = scenes.voxel_to_spring_actuation(va, vphi, r["sv_ptr"], r["sv_idx"])
    sc = dict(r)
    sc["amp"], sc["phase"] = amp, ph
    return O.System(sc)


def test_adjoint_oscillator_closed_form():
    # spring on a pinned anchor along x, no gravity/ground: x_N from the
    # discrete closed form; J = -(x_N - x_0), so dJ/dk = -dx_N/dk, taken here
    # by differencing the closed form (no simulation involved).
    m, L0, X, v0, dt, N = 0.1, 0.3, 0.01, 0.5, 1e-4, 700

    def xN(k):
        w = math.sqrt(k / m)
        th = math.acos(1 - (w * dt) ** 2 / 2)
        x1 = X * (1 - w * w * dt * dt) + dt * v0
        B = (x1 - X * math.cos(th)) / math.sin(th)
        return X * math.cos(N * th) + B * math.sin(N * th)

    k = 1e4
    h = 1e-3
    want = -(xN(k + h) - xN(k - h)) / (2 * h)
    sc = dict(pos=np.array([[0, 0, 0], [L0 + X, 0, 0]]), vel=np.array([[0, 0, 0], [v0, 0, 0]]),
              mass=np.array([0.0, m]), ends=np.array([[0, 1]]), k=np.array([k]), damping=np.array([0.0]))
    sysm = O.System(sc, rest=[L0])
    p = O.Params(dt=dt, gravity=(0, 0, 0), ground=False, ground_k=0, mu=0, omega=0)
    g = sysm.rollout_grad(p, N)
    assert abs(g["loss"][0] - (-(xN(k) - X))) < 1e-12
    assert abs(g["gk"][0] - want) <= 1e-6 * abs(want)


def _fd(f, x0, h):
    return (f(x0 + h) - f(x0 - h)) / (2 * h)


@pytest.mark.parametrize("seed", [4, 7])
def test_adjoint_matches_central_fd_on_robots(seed):
    # small robots sitting on the ground, actuated at 2 Hz, 300 steps: contact,
    # friction and actuation all act.  Components whose +-h runs change a
    # contact or stick decision are skipped (and counted).
    robots = scenes.robot_batch(2, seed=seed, side_lo=3, side_hi=4)
    N, h = 300, 1e-6
    skipped = checked = 0
    for r in robots:
        sysm = _robot_system(r)
        g = sysm.rollout_grad(P, N)
        base_sig = g["sig"]
        ga, gp = O.voxel_grads(g["gC"], g["gS"], r["voxel_a"], r["voxel_phi"], r["sv_ptr"], r["sv_idx"])
        scale = max(np.abs(ga).max(), np.abs(gp).max())

        def loss_with(va, vp):
            s2 = _robot_system(r, va, vp)
            l, sig = s2.rollout_loss(P, N)
            return l[0], sig

        for v in range(len(r["voxel_a"])):
            for which, grad in (("a", ga), ("phi", gp)):
                if abs(grad[v]) < 1e-3 * scale:
                    continue
                vals = []
                ok = True
                for sgn in (+1, -1):
                    va = r["voxel_a"].copy()
                    vp = r["voxel_phi"].copy()
                    (va if which == "a" else vp)[v] += sgn * h
                    l, sig = loss_with(va, vp)
                    ok &= sig == base_sig
                    vals.append(l)
                if not ok:
                    skipped += 1
                    continue
                fd = (vals[0] - vals[1]) / (2 * h)
                checked += 1
                assert abs(fd - grad[v]) <= 1e-5 * scale + 1e-5 * abs(grad[v]), (which, v, fd, grad[v])
        # stiffness of a few springs
        kscale = np.abs(g["gk"]).max()
        for s in np.argsort(-np.abs(g["gk"]))[:8]:
            s2 = _robot_system(r)
            vals = []
            ok = True
            for sgn in (+1, -1):
                s2.k = sysm.k.copy()
                s2.k[s] += sgn * h * sysm.k[s]
                l, sig = s2.rollout_loss(P, N)
                ok &= sig == base_sig
                vals.append(l[0])
            if not ok:
                skipped += 1
                continue
            fd = (vals[0] - vals[1]) / (2 * h * sysm.k[s])
            checked += 1
            assert abs(fd - g["gk"][s]) <= 1e-5 * kscale, (s, fd, g["gk"][s])
    print("checked", checked, "skipped", skipped)
    assert checked >= 20 and skipped <= checked // 4


def test_adjoint_body_weights_are_linear():
    # two independent robots in one system: weighted sum of per-body gradients
    robots = scenes.robot_batch(2, seed=9, side_lo=3, side_hi=3)
    sc = scenes.concat(robots)
    sysm = O.System(sc)
    N = 100
    g1 = sysm.rollout_grad(P, N, body=sc["body"], weights=[1.0, 0.0])
    g2 = sysm.rollout_grad(P, N, body=sc["body"], weights=[0.0, 1.0])
    g3 = sysm.rollout_grad(P, N, body=sc["body"], weights=[2.0, -3.0])
    for key in ("gk", "gC", "gS"):
        np.testing.assert_allclose(g3[key], 2 * g1[key] - 3 * g2[key], atol=1e-12 * np.abs(g3[key]).max())
    # springs of body 0 get nothing from body 1's loss
    s0 = slice(0, robots[0]["ends"].shape[0])
    assert np.all(g2["gk"][s0] == 0.0)
    # the per-body losses agree with the forward-only rollout
    l, _ = sysm.rollout_loss(P, N, body=sc["body"])
    np.testing.assert_allclose(g1["loss"], l, rtol=0, atol=1e-15)


def _variant_scene(variant, seed):
    """One small robot with the constants the library's kernel variants take:
    explicit rest lengths (+-3% of the initial lengths) with per-spring
    damping, actuated; or no actuation and no damping, thrown sideways."""
    r = scenes.robot_batch(1, seed=seed, side_lo=3, side_hi=4)[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    ns, nm = r["ends"].shape[0], r["pos"].shape[0]
    if variant == "rest_damping":
        d = r["pos"][r["ends"][:, 1]].astype(np.float64) - r["pos"][r["ends"][:, 0]]
        rest = np.linalg.norm(d, axis=1) * rng.uniform(0.97, 1.03, ns)
        return dict(r, damping=rng.uniform(0.5, 1.5, ns)), rest
    vel = rng.uniform(-0.2, 0.2, (nm, 3)) + np.array([0.5, 0.0, 0.0])
    return dict(r, amp=None, phase=None, damping=np.zeros(ns), vel=vel), None


@pytest.mark.parametrize("variant", ["rest_damping", "plain"])
def test_adjoint_matches_central_fd_on_constant_variants(variant):
    # dJ/dk of the largest springs, and (actuated) dJ/d(amp) and dJ/d(phase)
    # of the springs with the largest phasor gradients, which combine the
    # gradients in C = amp cos(phase) and S = amp sin(phase) two independent
    # ways; runs whose +-h rollouts change a contact or stick decision are
    # skipped (and counted)
    sc, rest = _variant_scene(variant, 23)
    N, h = 300, 1e-6
    sysm = O.System(sc, rest=rest)
    g = sysm.rollout_grad(P, N)
    base = g["sig"]
    checked = skipped = 0

    def loss(mod):
        s2 = O.System(sc, rest=rest)
        mod(s2)
        l, sig = s2.rollout_loss(P, N)
        return l[0], sig

    def fd_check(mod_plus, mod_minus, step, want, scale):
        nonlocal checked, skipped
        (lp, sp), (lm, sm) = loss(mod_plus), loss(mod_minus)
        if sp != base or sm != base:
            skipped += 1
            return
        checked += 1
        fd = (lp - lm) / (2 * step)
        assert abs(fd - want) <= 1e-5 * scale, (fd, want)

    kscale = np.abs(g["gk"]).max()
    for s in np.argsort(-np.abs(g["gk"]))[:8]:
        dk = h * sysm.k[s]

        def mk(sgn, s=s, dk=dk):
            def mod(s2):
                s2.k = s2.k.copy()
                s2.k[s] += sgn * dk
            return mod
        fd_check(mk(+1), mk(-1), dk, g["gk"][s], kscale)
    if variant == "rest_damping":
        amp, ph = sysm.amp, sysm.phase
        ga = g["gC"] * np.cos(ph) + g["gS"] * np.sin(ph)
        gp = amp * (g["gS"] * np.cos(ph) - g["gC"] * np.sin(ph))
        for which, grad in (("amp", ga), ("phase", gp)):
            scale = np.abs(grad).max()
            for s in np.argsort(-np.abs(grad))[:8]:
                def mk(sgn, s=s, which=which):
                    def mod(s2):
                        arr = (s2.amp if which == "amp" else s2.phase).copy()
                        arr[s] += sgn * h
                        if which == "amp":
                            s2.amp = arr
                        else:
                            s2.phase = arr
                    return mod
                fd_check(mk(+1), mk(-1), h, grad[s], scale)
    print(variant, "checked", checked, "skipped", skipped)
    assert checked >= (20 if variant == "rest_damping" else 6) and skipped <= checked // 4

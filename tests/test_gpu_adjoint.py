"""GPU FP32 adjoint (titan_rollout_grad) against the FP64 oracle's adjoint and
against FP64 central finite differences of the oracle's forward rollout.

Tolerances (the paper gives none; FP32 through 500 steps of contact and
friction): per-spring gradients normwise relative error <= 1e-3 and cosine
>= 0.9999 against the FP64 adjoint; per-voxel gradients within 1e-3 of the
largest against FP64 finite differences (h = 1e-6)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_10274_amd import scenes

pytestmark = pytest.mark.gpu

OMEGA = 2 * math.pi * 2
OP = O.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, mu=0.5, omega=OMEGA)


def _tp(engine=0):
    from paper_1911_10274_amd import titan as T

    return T.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5, omega=OMEGA,
                    engine=engine)


def _gpu_grad(sc, nsteps, K=50, weights=None, engine=0):
    from paper_1911_10274_amd import titan as T

    sim = T.sim_from_scene(sc, _tp(engine))
    out = sim.rollout_grad(nsteps, K, weights)
    info = sim.info()
    sim.close()
    return out, info


def _cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def test_adjoint_matches_oracle_adjoint_8_robots():
    robots = scenes.robot_batch(8, seed=4, side_lo=4, side_hi=8)
    sc = scenes.concat(robots)
    (loss, gk, gC, gS), _ = _gpu_grad(sc, 500, 50)
    sysm = O.System(sc)
    ref = sysm.rollout_grad(OP, 500, body=sc["body"])
    for name, g, r in (("k", gk, ref["gk"]), ("C", gC, ref["gC"]), ("S", gS, ref["gS"])):
        e = np.linalg.norm(g - r) / np.linalg.norm(r)
        c = _cos(g.astype(np.float64), r)
        print(name, "rel", e, "cos", c)
        assert e <= 1e-3 and c >= 0.9999
    print("loss", loss, ref["loss"])
    np.testing.assert_allclose(loss, ref["loss"], rtol=1e-3)


@pytest.mark.parametrize("side,seed,occ,lo,hi", [
    (4, 40, 0.6, 1, 256),       # 112 masses: 256-thread groups
    (7, 41, 0.6, 257, 512),     # 445 masses: 512-thread groups
    (9, 42, 0.6, 513, 1024),    # 934 masses: 1024-thread groups
    (11, 20, 0.7, 1025, 2048),  # 1,699 masses: two masses per thread
])
def test_adjoint_every_group_size_matches_oracle(side, seed, occ, lo, hi):
    # one body, so the group is that body whatever packing the batched
    # engine's tuner picks: each launch shape of the adjoint kernel is run
    robots = scenes.robot_batch(1, seed=seed, side_lo=side, side_hi=side, p_occ=occ)
    sc = scenes.concat(robots)
    (loss, gk, gC, gS), info = _gpu_grad(sc, 300, 50)
    assert lo <= info["batch_max_group"] <= hi
    ref = O.System(sc).rollout_grad(OP, 300, body=sc["body"])
    for name, g, r in (("k", gk, ref["gk"]), ("C", gC, ref["gC"]), ("S", gS, ref["gS"])):
        e = np.linalg.norm(g - r) / np.linalg.norm(r)
        c = _cos(g.astype(np.float64), r)
        print(side, name, "rel", e, "cos", c)
        assert e <= 1e-3 and c >= 0.9999
    np.testing.assert_allclose(loss, ref["loss"], rtol=1e-3)


def _voxel_scene(robots):
    """The robots side by side with their voxel maps, voxel values rounded to
    FP32 (what the library receives) and the springs' phasors recomputed in
    FP64 from those values (what the oracle receives)."""
    sc = scenes.concat(robots)
    sc["voxel_a"] = sc["voxel_a"].astype(np.float32)
    sc["voxel_phi"] = sc["voxel_phi"].astype(np.float32)
    amp, ph = scenes.voxel_to_spring_actuation(sc["voxel_a"], sc["voxel_phi"], sc["sv_ptr"], sc["sv_idx"])
    return sc, dict(sc, amp=amp, phase=ph)


def _gpu_voxel_grad(sc, nsteps, K=50):
    from paper_1911_10274_amd import titan as T

    sim = T.sim_from_scene(sc, _tp())
    sim.set_voxel_actuation(sc["voxel_a"], sc["voxel_phi"], sc["sv_ptr"], sc["sv_idx"])
    out = sim.rollout_grad_voxel(nsteps, K)
    per_spring = sim.rollout_grad(nsteps, K)
    sim.close()
    return out, per_spring


def test_voxel_grads_match_oracle_adjoint_8_robots():
    """Config 4's check set (8 robots of the 256-robot batch generator):
    per-voxel amplitude and phase gradients from the library (mapped on the
    device) against the oracle's FP64 adjoint mapped by the oracle's chain
    rule; and the device map against the same chain rule applied to the
    library's own per-spring gradients (FP32 sums of at most 28 terms)."""
    robots = scenes.robot_batch(8, seed=4, side_lo=4, side_hi=8)
    sc, osc = _voxel_scene(robots)
    (loss, gk, ga, gp), (loss2, gk2, gC2, gS2) = _gpu_voxel_grad(sc, 500, 50)
    np.testing.assert_array_equal(loss, loss2)
    np.testing.assert_array_equal(gk, gk2)
    ref = O.System(osc).rollout_grad(OP, 500, body=sc["body"])
    ra, rp = O.voxel_grads(ref["gC"], ref["gS"], sc["voxel_a"], sc["voxel_phi"], sc["sv_ptr"], sc["sv_idx"])
    for name, g, r in (("a", ga, ra), ("phi", gp, rp), ("k", gk, ref["gk"])):
        e = np.linalg.norm(g - r) / np.linalg.norm(r)
        c = _cos(g.astype(np.float64), r)
        print("voxel", name, "rel", e, "cos", c)
        assert e <= 1e-3 and c >= 0.9999
    np.testing.assert_allclose(loss, ref["loss"], rtol=1e-3)
    # the device map itself: same chain rule on the library's per-spring output
    ma, mp = O.voxel_grads(gC2.astype(np.float64), gS2.astype(np.float64), sc["voxel_a"], sc["voxel_phi"],
                           sc["sv_ptr"], sc["sv_idx"])
    absg = np.abs(gC2.astype(np.float64)) + np.abs(gS2.astype(np.float64))
    bound_a, _ = O.voxel_grads(absg, absg, np.ones(sc["voxel_a"].size), np.zeros(sc["voxel_a"].size),
                               sc["sv_ptr"], sc["sv_idx"])
    tol = 64 * 2.0 ** -24 * bound_a
    assert np.all(np.abs(ga - ma) <= tol)
    assert np.all(np.abs(gp - mp) <= tol * np.abs(sc["voxel_a"]))


def test_adjoint_voxel_grads_match_fp64_fd():
    # the 8-robot check of the adjoint batch: FP64 central differences
    # (h = 1e-6) of the oracle's 500-step rollout, in the voxel amplitudes and
    # phases, against the library's per-voxel gradients, for the largest
    # voxel gradients of each robot
    robots = scenes.robot_batch(8, seed=4, side_lo=4, side_hi=8)
    sc, _ = _voxel_scene(robots)
    (loss, gk, ga_all, gp_all), _ = _gpu_voxel_grad(sc, 500, 50)
    h = 1e-6
    checked = skipped = 0
    for b, r in enumerate(robots):
        v0, v1 = sc["voxel_ptr"][b], sc["voxel_ptr"][b + 1]
        ga, gp = ga_all[v0:v1].astype(np.float64), gp_all[v0:v1].astype(np.float64)
        va0 = sc["voxel_a"][v0:v1].astype(np.float64)
        vp0 = sc["voxel_phi"][v0:v1].astype(np.float64)
        scale = max(np.abs(ga).max(), np.abs(gp).max())

        def loss_at(va, vp):
            amp, ph = scenes.voxel_to_spring_actuation(va, vp, r["sv_ptr"], r["sv_idx"])
            s2 = dict(r)
            s2["amp"], s2["phase"] = amp, ph
            l, sig = O.System(s2).rollout_loss(OP, 500)
            return l[0], sig

        _, base_sig = loss_at(va0, vp0)
        for which, grad in (("a", ga), ("phi", gp)):
            for v in np.argsort(-np.abs(grad))[:4]:
                vals, sigs = [], []
                for sgn in (1, -1):
                    va, vp = va0.copy(), vp0.copy()
                    (va if which == "a" else vp)[v] += sgn * h
                    l, sg = loss_at(va, vp)
                    vals.append(l)
                    sigs.append(sg)
                if sigs[0] != base_sig or sigs[1] != base_sig:
                    skipped += 1
                    continue
                fd = (vals[0] - vals[1]) / (2 * h)
                checked += 1
                assert abs(fd - grad[v]) <= 1e-3 * scale, (b, which, v, fd, grad[v], scale)
    print("checked", checked, "skipped", skipped)
    assert checked >= 48


def _mean_phasor(va, vp, sv_ptr, sv_idx):
    # each spring's mean of a (cos phi, sin phi) over its voxels, in list
    # order in FP64, rounded to FP32
    C = np.zeros(len(sv_ptr) - 1, np.float32)
    S = np.zeros(len(sv_ptr) - 1, np.float32)
    for q in range(len(sv_ptr) - 1):
        c = s = 0.0
        for e in range(sv_ptr[q], sv_ptr[q + 1]):
            a, ph = float(va[sv_idx[e]]), float(vp[sv_idx[e]])
            c += a * math.cos(ph)
            s += a * math.sin(ph)
        n = sv_ptr[q + 1] - sv_ptr[q]
        C[q], S[q] = c / n, s / n
    return C, S


def test_voxel_actuation_sets_mean_phasors_and_map_ends_on_direct_change():
    from paper_1911_10274_amd import titan as T

    robots = scenes.robot_batch(3, seed=15, side_lo=3, side_hi=5)
    sc, osc = _voxel_scene(robots)
    # a sim whose springs start unactuated gets its phasors from the voxels:
    # the same run as a sim built with the oracle's phasors
    bare = dict(sc, amp=None, phase=None)
    a = T.sim_from_scene(bare, _tp())
    a.set_voxel_actuation(sc["voxel_a"], sc["voxel_phi"], sc["sv_ptr"], sc["sv_idx"])
    c, s_ = _mean_phasor(sc["voxel_a"], sc["voxel_phi"], sc["sv_ptr"], sc["sv_idx"])
    b = T.sim_from_scene(bare, _tp())
    b.set_springs_phasor(0, c, s_)
    a.step(200)
    b.step(200)
    pa, va, _ = a.get_state(displacement=True)
    pb, vb, _ = b.get_state(displacement=True)
    assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    # voxels changed while running: still equal to setting the phasors
    va2 = (sc["voxel_a"] * 0.5).astype(np.float32)
    a.set_voxel_actuation(va2, sc["voxel_phi"], sc["sv_ptr"], sc["sv_idx"])
    b.set_springs_phasor(0, *_mean_phasor(va2, sc["voxel_phi"], sc["sv_ptr"], sc["sv_idx"]))
    a.step(100)
    b.step(100)
    pa, va, _ = a.get_state(displacement=True)
    pb, vb, _ = b.get_state(displacement=True)
    assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    a.rollout_grad_voxel(20, 10)
    # a direct change of a voxel-driven spring ends the map
    a.set_springs_phasor(0, [0.0], [0.0])
    with pytest.raises(T.TitanError) as ei:
        a.rollout_grad_voxel(20, 10)
    assert ei.value.code == T.ESTATE
    a.close()
    b.close()


@pytest.mark.parametrize("K", [1, 7, 500])
def test_adjoint_checkpoint_interval_does_not_change_bits(K):
    robots = scenes.robot_batch(6, seed=12, side_lo=3, side_hi=6)
    sc = scenes.concat(robots)
    a, _ = _gpu_grad(sc, 300, 50)
    b, _ = _gpu_grad(sc, 300, K)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_adjoint_same_on_every_engine_and_leaves_state():
    from paper_1911_10274_amd import titan as T

    robots = scenes.robot_batch(5, seed=13, side_lo=3, side_hi=5)
    sc = scenes.concat(robots)
    ga, ia = _gpu_grad(sc, 200, 50, engine=T.ENGINE_TILED)
    gb, ib = _gpu_grad(sc, 200, 50, engine=T.ENGINE_BATCHED)
    assert ia["engine"] == T.ENGINE_TILED and ib["engine"] == T.ENGINE_BATCHED
    for x, y in zip(ga, gb):
        assert np.array_equal(x, y)
    sim = T.sim_from_scene(sc, _tp())
    sim.step(30)
    p0, v0, s0 = sim.get_state(displacement=True)
    sim.rollout_grad(100, 25)
    p1, v1, s1 = sim.get_state(displacement=True)
    assert s0 == s1 == 30 and np.array_equal(p0, p1) and np.array_equal(v0, v1)
    # the rollout starts at the current step: equal to a fresh sim advanced 30 steps
    loss_a, gk_a, _, _ = sim.rollout_grad(100, 25)
    sim.close()


def test_adjoint_body_weights():
    robots = scenes.robot_batch(3, seed=14, side_lo=3, side_hi=5)
    sc = scenes.concat(robots)
    (l1, k1, c1, s1), _ = _gpu_grad(sc, 150, 30, weights=[1.0, 0.0, 0.0])
    (l2, k2, c2, s2), _ = _gpu_grad(sc, 150, 30, weights=[0.0, 1.0, 1.0])
    (l3, k3, c3, s3), _ = _gpu_grad(sc, 150, 30)
    np.testing.assert_array_equal(l1, l3)  # losses do not depend on the weights
    for a, b, c in ((k1, k2, k3), (c1, c2, c3), (s1, s2, s3)):
        np.testing.assert_allclose(a + b, c, rtol=0, atol=1e-6 * np.abs(c).max())
    r0 = slice(0, robots[0]["ends"].shape[0])
    assert np.all(k2[r0] == 0.0)


def test_adjoint_needs_fitting_bodies():
    from paper_1911_10274_amd import titan as T

    sc = scenes.lattice(20)  # one 8000-mass body: does not fit one workgroup
    sim = T.sim_from_scene(sc, _tp(T.ENGINE_TILED))
    with pytest.raises(T.TitanError) as ei:
        sim.rollout_grad(10, 5)
    assert ei.value.code == T.ESTATE
    sim.close()


def test_device_outputs_equal_host_outputs_bit_for_bit():
    """titan_rollout_grad_device: the same bits as the host-output call, into
    device memory; any output may be left out; host pointers refused; a
    zero-step rollout writes zeros."""
    import ctypes

    import torch

    from paper_1911_10274_amd import titan as T

    robots = scenes.robot_batch(6, seed=15, side_lo=3, side_hi=6)
    sc = scenes.concat(robots)
    w = np.linspace(0.5, 1.5, len(robots)).astype(np.float32)
    sim = T.sim_from_scene(sc, _tp())
    host = sim.rollout_grad(120, 40, w)
    dev = sim.rollout_grad_device(120, 40, w)
    assert all(t.is_cuda and t.dtype == torch.float32 for t in dev)
    for h, d in zip(host, dev):
        assert np.array_equal(h, d.cpu().numpy())
    # only dJ/dk and dJ/dC wanted (NULL for the others)
    ns = host[1].size
    gk = torch.full((ns,), 7.0, device="cuda")
    gc = torch.empty(ns, device="cuda")
    sim.rollout_grad_device(120, 40, w, out=(None, gk, gc, None))
    assert np.array_equal(gk.cpu().numpy(), host[1])
    assert np.array_equal(gc.cpu().numpy(), host[2])
    # a host array is not device memory: refused before any work
    arr = np.zeros(ns, np.float32)
    rc = T.lib.titan_rollout_grad_device(sim._h, 10, 5, None, None, ctypes.c_void_p(arr.ctypes.data), None, None)
    assert rc == T.EINVAL
    # zero steps: zeros
    outs = tuple(torch.full((n,), 3.0, device="cuda") for n in (len(robots), ns, ns, ns))
    sim.rollout_grad_device(0, 5, out=outs)
    assert all(bool((t == 0).all()) for t in outs)
    sim.close()


@pytest.mark.parametrize("seed,lo,hi,count", [
    (16, 3, 5, 12),   # small robots packed several to a group
    (17, 4, 8, 8),    # the adjoint workload's sizes
    (41, 7, 7, 1),    # one 445-mass body: 512-thread groups
    (42, 9, 9, 1),    # one 934-mass body: 1024-thread groups, records in chunks
])
def test_adjoint_springs_once_equals_per_slot(seed, lo, hi, count, monkeypatch):
    """Reverse steps with every spring evaluated once (records shared through
    LDS, the default) against each end evaluating every spring itself
    (TITAN_ADJOINT_SPRING_ONCE=0): the same forward rollout (the loss, bit for
    bit); the reverse sums run in another order (each element within 1e-5 of
    the largest gradient)."""
    robots = scenes.robot_batch(count, seed=seed, side_lo=lo, side_hi=hi)
    sc = scenes.concat(robots)
    monkeypatch.setenv("TITAN_ADJOINT_SPRING_ONCE", "0")
    slot, _ = _gpu_grad(sc, 300, 50)
    monkeypatch.delenv("TITAN_ADJOINT_SPRING_ONCE")
    once, _ = _gpu_grad(sc, 300, 50)
    assert np.array_equal(slot[0], once[0])
    for a, b in zip(slot[1:], once[1:]):
        assert np.abs(a - b).max() <= 1e-5 * np.abs(a).max()


@pytest.mark.parametrize("once", ["0", "1"])
@pytest.mark.parametrize("variant", ["rest_damping", "plain"])
def test_adjoint_spring_constant_variants_match_oracle(variant, once, monkeypatch):
    """The kernel variants beyond the robots' own constants, on both reverse
    paths (TITAN_ADJOINT_SPRING_ONCE): explicit rest lengths with per-spring
    damping (actuated), and springs with neither actuation nor damping (the
    robots thrown sideways so the loss moves); against the FP64 adjoint."""
    from paper_1911_10274_amd import titan as T

    robots = scenes.robot_batch(6, seed=18, side_lo=3, side_hi=6)
    sc = scenes.concat(robots)
    rng = np.random.Generator(np.random.PCG64(19))
    ns, nm = sc["ends"].shape[0], sc["pos"].shape[0]
    rest = None
    if variant == "rest_damping":
        d = sc["pos"][sc["ends"][:, 1]].astype(np.float64) - sc["pos"][sc["ends"][:, 0]]
        rest = (np.linalg.norm(d, axis=1) * rng.uniform(0.97, 1.03, ns)).astype(np.float32)
        sc = dict(sc, damping=rng.uniform(0.5, 1.5, ns).astype(np.float32))
    else:
        vel = rng.uniform(-0.2, 0.2, (nm, 3)) + np.array([0.5, 0.0, 0.0])
        sc = dict(sc, amp=None, phase=None, damping=np.zeros(ns, np.float32), vel=vel.astype(np.float32))
    monkeypatch.setenv("TITAN_ADJOINT_SPRING_ONCE", once)
    sim = T.sim_from_scene(sc, _tp(), rest=rest)
    loss, gk, gC, gS = sim.rollout_grad(300, 50)
    sim.close()
    ref = O.System(sc, rest=rest).rollout_grad(OP, 300, body=sc["body"])
    pairs = [("k", gk, ref["gk"])]
    if variant == "rest_damping":
        pairs += [("C", gC, ref["gC"]), ("S", gS, ref["gS"])]
    for name, g, r in pairs:
        e = np.linalg.norm(g - r) / np.linalg.norm(r)
        c = _cos(g.astype(np.float64), r)
        print(variant, once, name, "rel", e, "cos", c)
        assert e <= 1e-3 and c >= 0.9999
    np.testing.assert_allclose(loss, ref["loss"], rtol=1e-3)


def test_adjoint_after_topology_edits_matches_oracle():
    """One sim's rollout gradient across topology edits -- springs removed
    (tombstones), then springs added twice within a body (a layout rebuild
    with spare slots, then insertion in place) -- each time against the FP64
    adjoint of the edited system: the spring tables the gradient keeps
    between calls follow every change of the slots."""
    from paper_1911_10274_amd import titan as T

    robots = scenes.robot_batch(4, seed=31, side_lo=3, side_hi=5)
    sc = scenes.concat(robots)
    rng = np.random.Generator(np.random.PCG64(31))
    ns0 = sc["ends"].shape[0]
    pos, body = sc["pos"], sc["body"]
    b0 = np.flatnonzero(body == 0)
    existing = set(map(tuple, np.sort(sc["ends"], axis=1).tolist()))

    def new_pairs(count):
        out = []
        while len(out) < count:
            a, b = sorted(int(x) for x in rng.choice(b0, 2, replace=False))
            if (a, b) in existing or np.linalg.norm(pos[a].astype(np.float64) - pos[b]) > 0.35:
                continue
            existing.add((a, b))
            out.append((a, b))
        return np.array(out, np.int64)

    cols = {key: sc[key].copy() for key in ("ends", "k", "damping", "amp", "phase")}
    sim = T.sim_from_scene(sc, _tp())
    sim.rollout_grad(100, 25)  # the tables of the first layout
    removed = rng.choice(ns0, 6, replace=False)
    sim.remove_springs(removed)
    before = sim.info()
    for rnd in range(2):
        add = new_pairs(5)
        new = dict(ends=add, k=rng.uniform(5e3, 2e4, 5).astype(np.float32), damping=np.ones(5, np.float32),
                   amp=rng.uniform(0.0, 0.15, 5).astype(np.float32),
                   phase=rng.uniform(0.0, 2 * np.pi, 5).astype(np.float32))
        sim.add_springs(new["ends"], new["k"], damping=new["damping"], amp=new["amp"], phase=new["phase"])
        for key in cols:
            cols[key] = np.concatenate([cols[key], new[key]])
        keep = np.ones(cols["k"].shape[0], bool)
        keep[removed] = False
        edited = dict(sc, **{key: v[keep] for key, v in cols.items()})
        loss, gk, gC, gS = sim.rollout_grad(200, 50)
        ref = O.System(edited).rollout_grad(OP, 200, body=body)
        for name, g, r in (("k", gk[keep], ref["gk"]), ("C", gC[keep], ref["gC"]), ("S", gS[keep], ref["gS"])):
            e = np.linalg.norm(g - r) / np.linalg.norm(r)
            c = _cos(g.astype(np.float64), r)
            print("after edit", rnd, name, "rel", e, "cos", c)
            assert e <= 1e-3 and c >= 0.9999
        np.testing.assert_allclose(loss, ref["loss"], rtol=1e-3)
    after = sim.info()
    sim.close()
    assert after["layout_builds"] + after["springs_in_place"] > before["layout_builds"] + before["springs_in_place"]

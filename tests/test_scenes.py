"""Seeded scene generators: determinism and the structural rules they follow."""
import numpy as np

from paper_1911_10274_amd import scenes


def test_lattice_counts_and_order():
    sc = scenes.cube_drop(10)
    assert sc["pos"].shape == (1000, 3) and sc["ends"].shape == (10476, 2)
    e = sc["ends"]
    assert np.all(e[:, 0] < e[:, 1])
    # sorted by lower end (stable w.r.t. offset order)
    assert np.all(np.diff(e[:, 0]) >= 0)
    assert abs(float(sc["pos"][:, 2].min()) - 0.5) < 1e-7


def test_jittered_lattice_deterministic_and_bounded():
    a = scenes.jittered_actuated_lattice(n=12, seed=5)
    b = scenes.jittered_actuated_lattice(n=12, seed=5)
    c = scenes.jittered_actuated_lattice(n=12, seed=6)
    for key in ("pos", "k", "phase"):
        np.testing.assert_array_equal(a[key], b[key])
    assert not np.array_equal(a["pos"], c["pos"])
    base = scenes.lattice(12)["pos"].astype(np.float64)
    assert np.abs(a["pos"] - base).max() <= 0.002 + 1e-6
    assert a["k"].min() >= 5e3 and a["k"].max() <= 2e4
    assert a["phase"].min() >= 0 and a["phase"].max() <= 2 * np.pi + 1e-6
    assert np.all(a["amp"] == np.float32(0.1))


def test_voxel_robot_structure():
    robots = scenes.robot_batch(40, seed=123, side_lo=3, side_hi=6)
    from scipy import ndimage
    for r in robots:
        s = r["side"]
        assert 3 <= s <= 6
        n = r["pos"].shape[0]
        e = r["ends"]
        assert np.all(e[:, 0] < e[:, 1]) and e.max() < n
        # unique springs, sorted
        key = e[:, 0] * n + e[:, 1]
        assert np.all(np.diff(key) > 0)
        # lowest corners on the ground, corners on the 0.1 m grid
        assert float(r["pos"][:, 2].min()) == 0.0
        g = r["pos"].astype(np.float64) / 0.1
        assert np.abs(g - np.round(g)).max() < 1e-4
        # kept voxels form one face-connected component
        occ = np.zeros(s ** 3, bool)
        occ[r["voxel_index"]] = True
        lab, nl = ndimage.label(occ.reshape(s, s, s), ndimage.generate_binary_structure(3, 1))
        assert nl == 1
        # each voxel contributes its 28 corner pairs to the membership lists
        assert r["sv_ptr"][-1] == 28 * r["voxel_index"].size
        cnt = np.diff(r["sv_ptr"])
        assert cnt.min() >= 1 and cnt.max() <= 4
        # spring lengths are edges (0.1), face diagonals or body diagonals
        d = np.linalg.norm(r["pos"][e[:, 1]].astype(np.float64) - r["pos"][e[:, 0]], axis=1) / 0.1
        assert np.all(np.min(np.abs(d[:, None] - np.sqrt([1.0, 2.0, 3.0])[None, :]), axis=1) < 1e-5)
        # amplitudes within the voxel range, phasor mean never exceeds it
        assert r["amp"].min() >= 0 and r["amp"].max() <= 0.15 + 1e-6


def test_robot_batch_deterministic():
    a = scenes.robot_batch(5, seed=9, side_lo=3, side_hi=12)
    b = scenes.robot_batch(5, seed=9, side_lo=3, side_hi=12)
    for ra, rb in zip(a, b):
        np.testing.assert_array_equal(ra["ends"], rb["ends"])
        np.testing.assert_array_equal(ra["phase"], rb["phase"])


def test_concat_offsets():
    robots = scenes.robot_batch(3, seed=1, side_lo=3, side_hi=4)
    sc = scenes.concat(robots)
    assert sc["mass_ptr"][-1] == sc["pos"].shape[0]
    assert sc["spring_ptr"][-1] == sc["ends"].shape[0]
    for b in range(3):
        e = sc["ends"][sc["spring_ptr"][b]:sc["spring_ptr"][b + 1]]
        assert e.min() >= sc["mass_ptr"][b] and e.max() < sc["mass_ptr"][b + 1]
        assert np.all(sc["body"][sc["mass_ptr"][b]:sc["mass_ptr"][b + 1]] == b)

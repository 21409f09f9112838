"""C ABI: the library loads, exports every function the header declares, and
its host-side validation works without a GPU (no compute calls here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "titan.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(titan_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    from paper_1911_10274_amd import titan as T

    names = _declared()
    assert "titan_step" in names and "titan_create" in names
    for name in names:
        assert hasattr(T.lib, name), name


def test_abi_version():
    from paper_1911_10274_amd import titan as T

    src = open(HEADER).read()
    want = int(re.search(r"#define TITAN_ABI_VERSION (\d+)", src).group(1))
    assert T.lib.titan_abi_version() == want


def _host_sim():
    from paper_1911_10274_amd import titan as T

    return T.Sim(T.Params(), memory="hip")


def test_validation_errors_without_gpu():
    from paper_1911_10274_amd import titan as T

    sim = _host_sim()
    pos = np.array([[0, 0, 0], [1, 0, 0], [1, 0, 0]], np.float32)
    assert sim.add_masses(pos, [1, 1, 0]) == 0
    cases = [
        dict(ends=[[0, 3]], k=[1.0]),                 # out of range
        dict(ends=[[1, 1]], k=[1.0]),                 # self spring
        dict(ends=[[1, 2]], k=[1.0]),                 # zero initial length
        dict(ends=[[0, 1]], k=[-1.0]),                # negative k
        dict(ends=[[0, 1]], k=[np.nan]),              # non-finite
        dict(ends=[[0, 1]], k=[1.0], rest=[0.0]),     # zero rest
        dict(ends=[[0, 1]], k=[1.0], damping=[-1.0]),
    ]
    for c in cases:
        with pytest.raises(T.TitanError) as ei:
            sim.add_springs(**c)
        assert ei.value.code == T.EINVAL
        assert T.last_error()
    with pytest.raises(T.TitanError):
        sim.add_springs([[0, 1]], [1.0], amp=[0.1])  # amp without phase
    assert sim.add_springs([[0, 1]], [1.0]) == 0
    assert sim.add_springs([[0, 2], [1, 0]], [1.0, 2.0]) == 1
    with pytest.raises(T.TitanError):
        sim.add_masses([[0, 0, np.inf]], [1.0])
    with pytest.raises(T.TitanError):
        sim.add_masses([[0, 0, 0]], [-1.0])
    info = sim.info()
    assert info["n_masses"] == 3 and info["n_springs"] == 3 and info["finalized"] == 0
    sim.close()


def test_bodies_cannot_be_joined():
    from paper_1911_10274_amd import titan as T

    sim = _host_sim()
    sim.add_masses([[0, 0, 0], [1, 0, 0]], [1, 1], body=[0, 1])
    with pytest.raises(T.TitanError) as ei:
        sim.add_springs([[0, 1]], [1.0])
    assert ei.value.code == T.EINVAL
    assert sim.info()["n_bodies"] == 2
    sim.close()


def test_bad_params_rejected():
    from paper_1911_10274_amd import titan as T

    for p in [T.Params(dt=0.0), T.Params(dt=-1.0), T.Params(ground_k=-1.0), T.Params(friction_mu=float("nan")),
              T.Params(engine=7)]:
        with pytest.raises(T.TitanError) as ei:
            T.Sim(p, memory="hip")
        assert ei.value.code == T.EINVAL


def test_null_sim_is_rejected():
    from paper_1911_10274_amd import titan as T

    assert T.lib.titan_step(None, 1) == T.EINVAL
    assert T.lib.titan_destroy(None) == T.OK


def test_step_without_device_reports_edevice():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1911_10274_amd import titan as T

    sim = _host_sim()
    sim.add_masses([[0, 0, 1]], [1.0])
    with pytest.raises(T.TitanError) as ei:
        sim.step(1)
    assert ei.value.code == T.EDEVICE
    sim.close()


def _declarations_with_comments():
    """(name, comment block right above its declaration) for every titan_*
    function the header declares."""
    lines = open(HEADER).read().split("\n")
    out = []
    for q, line in enumerate(lines):
        m = re.match(r"^(?:const char \*|int64_t |int )(titan_[a-z_0-9]+)\(", line)
        if not m:
            continue
        p = q - 1
        block = []
        if p >= 0 and lines[p].rstrip().endswith("*/"):
            while p >= 0:
                block.append(lines[p])
                if "/*" in lines[p]:
                    break
                p -= 1
        out.append((m.group(1), "\n".join(reversed(block))))
    return out


def test_every_declaration_cites_its_passage():
    """Each call says where in the paper its operation is defined (a section,
    equation or figure), that it is not in the paper, or -- for the entry point
    that allocates nothing -- which callers it is for."""
    decls = _declarations_with_comments()
    assert {n for n, _ in decls} == set(_declared())
    flat = {n: " ".join(re.sub(r"^\s*(/\*|\*/|\*)", " ", ln) for ln in c.split("\n")) for n, c in decls}
    flat = {n: re.sub(r"\s+", " ", c) for n, c in flat.items()}
    missing = [n for n, c in flat.items()
               if not re.search(r"Sec\. [IV]+|Eq\. \d|not in the paper|cannot allocate", c)]
    assert not missing, missing


_PLAN_SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
from paper_1911_10274_amd import titan as T
from paper_1911_10274_amd import scenes

def finalize(build, engine):
    sim = T.Sim(T.Params(engine=engine), memory="hip")
    build(sim)
    rc = T.lib.titan_finalize(sim._h)
    assert rc in (T.OK, T.EDEVICE), (rc, T.last_error())
    sim.close()

cube = scenes.lattice(4)
cases = {{
    "no masses": lambda s: None,
    "one mass, no springs": lambda s: s.add_masses([[0, 0, 1.0]], [0.1]),
    "pinned masses, no springs": lambda s: s.add_masses([[0, 0, 0], [1, 0, 0]], [0.0, 0.0]),
    "bodies without springs": lambda s: s.add_masses([[0, 0, 0], [1, 0, 0], [2, 0, 0]], [1, 1, 1], body=[0, 1, 1]),
    "masses at one point": lambda s: s.add_masses(np.zeros((600, 3)), np.ones(600)),
    "cube": lambda s: (s.add_masses(cube["pos"], cube["mass"]), s.add_springs(cube["ends"], cube["k"])),
}}
for engine in (T.ENGINE_AUTO, T.ENGINE_GATHER, T.ENGINE_TILED, T.ENGINE_BATCHED):
    for name, build in cases.items():
        print(engine, name, flush=True)
        finalize(build, engine)
print("PLANNED")
"""


def test_host_layout_planning_of_degenerate_systems():
    """titan_finalize plans the internal order and the incidence layout on the
    host before it needs a device, so this runs here without a GPU: systems
    with no masses, no springs (a spring-less step once crashed in this host
    path), only pinned masses, springless bodies, coincident masses and a
    small cube.  In a child process, so a crash fails the test."""
    import subprocess
    import sys

    r = subprocess.run([sys.executable, "-c", _PLAN_SCRIPT.format(root=ROOT)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "PLANNED" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])


def test_voxel_actuation_validation_without_gpu():
    from paper_1911_10274_amd import titan as T

    sim = _host_sim()
    sim.add_masses([[0, 0, 0], [1, 0, 0], [0, 1, 0]], [1, 1, 1])
    sim.add_springs([[0, 1], [1, 2], [0, 2]], [1.0, 1.0, 1.0])
    a = np.array([0.1, 0.2], np.float32)
    ph = np.array([0.5, 1.0], np.float32)
    good_ptr, good_idx = [0, 1, 3, 3], [0, 0, 1]
    sim.set_voxel_actuation(a, ph, good_ptr, good_idx)  # host tables only before the first step
    bad = [
        (a, ph, [1, 1, 3, 3], good_idx),            # sv_ptr[0] != 0
        (a, ph, [0, 2, 1, 3], [0, 0, 1]),           # decreasing
        (a, ph, [0, 1, 3, 3], [0, 0, 2]),           # voxel out of range
        (a, ph, [0, 1, 3, 3], [0, 1, 1]),           # a voxel listed twice for one spring
        (np.array([np.nan, 0.2], np.float32), ph, good_ptr, good_idx),
    ]
    for va, vp, ptr, idx in bad:
        with pytest.raises(T.TitanError) as ei:
            sim.set_voxel_actuation(va, vp, ptr, idx)
        assert ei.value.code == T.EINVAL
    with pytest.raises(T.TitanError) as ei:
        sim.set_springs_phasor(0, [np.inf], [0.0])
    assert ei.value.code == T.EINVAL
    with pytest.raises(T.TitanError) as ei:
        sim.set_springs_phasor(2, [0.1, 0.1], [0.0, 0.0])  # past the last spring
    assert ei.value.code == T.EINVAL
    sim.set_springs_phasor(0, [0.1, 0.0, -0.2], [0.0, 0.3, 0.1])
    sim.close()
    wave = T.Sim(T.Params(actuation=T.ACT_WAVE), memory="hip")
    wave.add_masses([[0, 0, 0], [1, 0, 0]], [1, 1])
    wave.add_springs([[0, 1]], [1.0])
    for call in (lambda: wave.set_springs_phasor(0, [0.1], [0.0]),
                 lambda: wave.set_voxel_actuation([0.1], [0.0], [0, 1], [0])):
        with pytest.raises(T.TitanError) as ei:
            call()
        assert ei.value.code == T.ESTATE
    wave.close()

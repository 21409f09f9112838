"""Helpers shared by the GPU parity tests: run the native path and the FP64
oracle on the same seeded scene and compare per step."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

TOL = 1e-5  # relative error per step over the first 10 steps (normwise over all masses)
# Per mass: |error_i| / max(|ref_i|, floor) with the floor the step's RMS over
# all masses of the reference quantity (for the spring force: at least the
# mass's weight m_i g), so that masses that barely move are measured against
# the step's typical motion.  A normwise bound alone lets a large error on a
# few masses hide in a million-mass norm; this bound does not.
MASS_TOL = 1e-5


def both_params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, mu=0.5, omega=0.0, engine=None):
    from paper_1911_10274_amd import titan as T

    tp = T.Params(dt=dt, gravity=gravity, ground=ground, ground_k=ground_k, friction_mu=mu, omega=omega,
                  engine=T.ENGINE_TILED if engine is None else engine)
    op = O.Params(dt=dt, gravity=gravity, ground=ground, ground_k=ground_k, mu=mu, omega=omega)
    return tp, op


def rel(a, b, floor=0.0):
    num = float(np.linalg.norm(np.asarray(a, np.float64) - b))
    den = max(float(np.linalg.norm(b)), floor)
    return num / den if den > 0 else num


def gpu_series(sim, nsteps, with_start_states=False):
    """Per step n = 1..nsteps of the native path: displacement, velocity and
    the spring force of step n's starting state.  With ``with_start_states``
    also the (displacement, velocity) each step started from."""
    dX, V, F, S = [], [], [], []
    p, v, _ = sim.get_state(displacement=True)
    for _ in range(nsteps):
        S.append((p.astype(np.float64), v.astype(np.float64)))
        F.append(sim.get_forces().astype(np.float64))
        sim.step(1)
        p, v, _ = sim.get_state(displacement=True)
        dX.append(p.astype(np.float64))
        V.append(v.astype(np.float64))
    out = np.array(dX), np.array(V), np.array(F)
    return (out, S) if with_start_states else out


def compare_series(gpu, ref, mass, g=9.81, label=""):
    """Worst per-step relative errors (displacement, velocity, force).

    The spring-force error is taken relative to the larger of the reference
    force norm and the weight norm ||m g|| over all masses: where springs are
    at rest (free fall, rigid sliding) the exact spring force is zero and only
    its size against the forces that drive the motion is meaningful."""
    gdX, gV, gF = gpu
    rdX, rV, rF = ref
    m = np.asarray(mass, np.float64)
    ffloor = float(np.linalg.norm(m * g))
    out = {"dX": 0.0, "V": 0.0, "F": 0.0, "dX_mass": 0.0, "V_mass": 0.0, "F_mass": 0.0}
    for s in range(gdX.shape[0]):
        out["dX"] = max(out["dX"], rel(gdX[s], rdX[s]))
        out["V"] = max(out["V"], rel(gV[s], rV[s]))
        out["F"] = max(out["F"], rel(gF[s], rF[s], ffloor))
        out["dX_mass"] = max(out["dX_mass"], per_mass(gdX[s], rdX[s]))
        out["V_mass"] = max(out["V_mass"], per_mass(gV[s], rV[s]))
        out["F_mass"] = max(out["F_mass"], per_mass(gF[s], rF[s], m * g))
    return out


def per_mass(a, b, floor_i=None):
    """Largest per-mass error |a_i - b_i| / max(|b_i|, RMS_j |b_j|, floor_i)."""
    a = np.asarray(a, np.float64).reshape(-1, 3)
    b = np.asarray(b, np.float64).reshape(-1, 3)
    if b.shape[0] == 0:
        return 0.0
    nb = np.linalg.norm(b, axis=1)
    den = np.maximum(nb, np.sqrt(np.mean(nb * nb)))
    if floor_i is not None:
        den = np.maximum(den, np.asarray(floor_i, np.float64))
    num = np.linalg.norm(a - b, axis=1)
    return float(np.max(np.where(den > 0, num / np.where(den > 0, den, 1.0), num)))


def assert_parity(err, label=""):
    """Normwise errors within TOL and per-mass errors within MASS_TOL."""
    norm = {k: v for k, v in err.items() if not k.endswith("_mass")}
    mass = {k: v for k, v in err.items() if k.endswith("_mass")}
    assert max(norm.values()) <= TOL, (label, err)
    assert not mass or max(mass.values()) <= MASS_TOL, (label, err)

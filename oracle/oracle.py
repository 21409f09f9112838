"""FP64 CPU oracle of the mass-spring step (Python front end).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the package smoke check and the
benchmark's CPU-baseline leg; never by the GPU library or its binding.

The arithmetic lives in ``titan_oracle.c`` (plain C, double precision,
serial scatter over springs); this module compiles it with gcc on first use,
promotes the FP32 scene arrays to FP64 and adds the observables (energies,
momenta, centre of mass) as plain numpy sums.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "titan_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)


class _Params(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("ground", ctypes.c_int32),
        ("ground_k", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("wave", ctypes.c_int32),
        ("period", ctypes.c_double),
        ("integrator", ctypes.c_int32),
    ]


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` (plain -O2, no FMA
    contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def build_native(out_dir: str) -> str:
    """The same source compiled for the host it runs on (-O3 -march=native,
    still no FMA contraction and no fast-math), into ``out_dir``: the build
    the CPU baseline times.  The tests use ``build()``'s portable library."""
    out = os.path.join(out_dir, "liboracle_native.so")
    subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", _SRC,
                           "-o", out, "-lm"])
    return out


def use_library(path: str) -> None:
    """Load the oracle from ``path`` (a build of the same source) instead of
    the default library; call before any other use."""
    global _lib
    _lib = None
    _load(path)


_lib = None


def _load(path: str | None = None):
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(path or build())
        lib.orc_rest_lengths.argtypes = [ctypes.c_int64, _lp, _dp, _dp]
        _u8p = ctypes.POINTER(ctypes.c_uint8)
        lib.orc_spring_forces.argtypes = [ctypes.c_int64, ctypes.c_int64, _lp, _dp, _dp, _dp, _dp, _dp,
                                          ctypes.c_double, ctypes.c_int32, ctypes.c_double, _dp, _u8p,
                                          ctypes.c_double, _dp, _dp, _dp]
        lib.orc_integrate.argtypes = [ctypes.c_int64, _dp, ctypes.POINTER(_Params), _dp, _dp, _dp]
        lib.orc_run.argtypes = [ctypes.c_int64, _dp, ctypes.c_int64, _lp, _dp, _dp, _dp, _dp, _dp,
                                ctypes.POINTER(_Params), _dp, _u8p, _dp, ctypes.POINTER(ctypes.c_int32),
                                ctypes.c_int64, ctypes.c_int64, _dp, _dp, _dp]
        lib.orc_run.restype = ctypes.c_int
        _i32p = ctypes.POINTER(ctypes.c_int32)
        _u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.orc_rollout_loss.argtypes = [ctypes.c_int64, _dp, ctypes.c_int64, _lp, _dp, _dp, _dp, _dp, _dp,
                                         ctypes.POINTER(_Params), _i32p, ctypes.c_int32, ctypes.c_int64, _dp, _dp,
                                         _dp, _u64p]
        lib.orc_rollout_loss.restype = ctypes.c_int
        lib.orc_rollout_grad.argtypes = [ctypes.c_int64, _dp, ctypes.c_int64, _lp, _dp, _dp, _dp, _dp, _dp,
                                         ctypes.POINTER(_Params), _i32p, ctypes.c_int32, _dp, ctypes.c_int64, _dp,
                                         _dp, _dp, _dp, _dp, _dp, _u64p]
        lib.orc_rollout_grad.restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


INTEGRATORS = {"euler": 0, "verlet": 1, "rk4": 2}


@dataclass
class Params:
    dt: float = 1.0e-4
    gravity: tuple = (0.0, 0.0, -9.81)
    ground: bool = True
    ground_k: float = 1.0e5
    mu: float = 0.5
    omega: float = 0.0
    wave: bool = False    # wave actuation (Eqs. 3-5): a scene's phase holds the offsets t_o
    period: float = 1.0   # wave period t_p, s
    integrator: str = "euler"  # "euler" (semi-implicit), "verlet" (velocity Verlet) or "rk4"

    @classmethod
    def from_dict(cls, d: dict) -> "Params":
        return cls(dt=d["dt"], gravity=tuple(d["gravity"]), ground=bool(d["ground"]),
                   ground_k=d["ground_k"], mu=d["mu"], omega=d["omega"], wave=bool(d.get("wave", False)),
                   period=d.get("period", 1.0), integrator=d.get("integrator", "euler"))

    def _c(self) -> _Params:
        p = _Params()
        p.dt = self.dt
        p.g[:] = list(self.gravity)
        p.ground = 1 if self.ground else 0
        p.ground_k = self.ground_k
        p.mu = self.mu
        p.omega = self.omega
        p.wave = 1 if self.wave else 0
        p.period = self.period
        p.integrator = INTEGRATORS[self.integrator]
        return p


def wave_offsets(pos, ends, body=None) -> np.ndarray:
    """Per-spring actuation offsets of the wave mode (Sec. IV-B, Eq. 5): the
    smaller reference x of the spring's two ends minus the smallest reference
    x of its body, in FP64 from the given positions."""
    x = _d(pos).reshape(-1, 3)[:, 0]
    e = np.asarray(ends, dtype=np.int64).reshape(-1, 2)
    b = np.zeros(x.shape[0], np.int64) if body is None else np.asarray(body, dtype=np.int64)
    xmin = np.full(int(b.max()) + 1 if b.size else 1, np.inf)
    np.minimum.at(xmin, b, x)
    return np.minimum(x[e[:, 0]], x[e[:, 1]]) - xmin[b[e[:, 0]]]


class System:
    """A scene promoted to FP64.  ``rest`` defaults to the initial lengths,
    computed in FP64 from the (FP32) initial positions.

    A scene with a ``yield`` array (per spring; inf = never breaks) has
    breakable springs (Sec. III-E): ``broken`` holds one flag per spring,
    starts all clear and is updated by ``run``, ``trajectory`` and
    ``spring_forces`` unless they are given a flag array of their own (then
    that array is updated in place).

    Velocity Verlet carries the acceleration of each step's end into the
    next step: ``run`` and ``trajectory`` keep it in ``acc`` (None: none
    carried, recomputed from the starting state), so that consecutive calls
    continue one run; set ``acc = None`` to start afresh."""

    def __init__(self, scene: dict, rest=None):
        self.x0 = _d(scene["pos"]).reshape(-1, 3).copy()
        self.v0 = _d(scene["vel"]).reshape(-1, 3).copy() if scene.get("vel") is not None \
            else np.zeros_like(self.x0)
        self.n = self.x0.shape[0]
        self.mass = _d(scene["mass"])
        self.ends = np.ascontiguousarray(scene["ends"], dtype=np.int64).reshape(-1, 2)
        self.ns = self.ends.shape[0]
        self.k = _d(scene["k"])
        self.c = _d(scene.get("damping"))
        self.amp = _d(scene.get("amp"))
        self.phase = _d(scene.get("phase"))
        if (self.amp is None) != (self.phase is None):
            raise ValueError("amp and phase go together")
        if rest is None:
            rest = np.empty(self.ns, np.float64)
            _load().orc_rest_lengths(self.ns, _ptr(self.ends, _lp), _ptr(self.x0), _ptr(rest))
        self.rest = _d(rest)
        self.yield_ = _d(scene.get("yield"))
        self.broken = np.zeros(self.ns, np.uint8) if self.yield_ is not None else None
        self.acc = None

    def _flags(self, broken):
        if self.yield_ is None:
            return None
        b = self.broken if broken is None else broken
        if b.dtype != np.uint8 or b.shape != (self.ns,) or not b.flags.c_contiguous:
            raise ValueError("broken must be a contiguous uint8 array with one flag per spring")
        return b

    def spring_forces(self, x, v, t, omega, wave=False, period=1.0, broken=None):
        x = _d(x).reshape(-1, 3)
        v = _d(v).reshape(-1, 3)
        f = np.empty((self.n, 3), np.float64)
        b = self._flags(broken)
        _load().orc_spring_forces(self.n, self.ns, _ptr(self.ends, _lp), _ptr(self.k), _ptr(self.c),
                                  _ptr(self.rest), _ptr(self.amp), _ptr(self.phase), omega, 1 if wave else 0,
                                  period, _ptr(self.yield_), _ptr(b, ctypes.POINTER(ctypes.c_uint8)), t, _ptr(x),
                                  _ptr(v), _ptr(f))
        return f

    def run(self, params: Params, x, v, step0: int, nsteps: int, want_forces: bool = False, broken=None):
        """Advance copies of (x, v) by ``nsteps`` steps from step index
        ``step0``.  Returns (x, v, f) with f the spring forces of the last
        step's starting state (or None)."""
        x = _d(x).reshape(-1, 3).copy()
        v = _d(v).reshape(-1, 3).copy()
        f = np.empty((self.n, 3), np.float64) if want_forces else None
        p = params._c()
        b = self._flags(broken)
        acc, have = None, ctypes.c_int32(0)
        if params.integrator == "verlet":
            acc = np.zeros((self.n, 3), np.float64) if self.acc is None else self.acc
            have.value = 0 if self.acc is None else 1
        rc = _load().orc_run(self.n, _ptr(self.mass), self.ns, _ptr(self.ends, _lp), _ptr(self.k),
                             _ptr(self.c), _ptr(self.rest), _ptr(self.amp), _ptr(self.phase),
                             ctypes.byref(p), _ptr(self.yield_), _ptr(b, ctypes.POINTER(ctypes.c_uint8)),
                             _ptr(acc), ctypes.byref(have) if acc is not None else None, step0,
                             nsteps, _ptr(x), _ptr(v), _ptr(f))
        if acc is not None and have.value:
            self.acc = acc
        if rc != 0:
            raise MemoryError("oracle run failed")
        return x, v, f

    def trajectory(self, params: Params, nsteps: int, x=None, v=None, step0: int = 0, broken=None):
        """Per-step series for n = 1..nsteps: displacement X(n) - X(0),
        velocity V(n) and spring force F of step n's starting state (F(n-1)).
        Returns three arrays of shape (nsteps, n, 3)."""
        x = self.x0 if x is None else _d(x).reshape(-1, 3)
        v = self.v0 if v is None else _d(v).reshape(-1, 3)
        xs0 = x.copy()
        dX = np.empty((nsteps, self.n, 3))
        V = np.empty((nsteps, self.n, 3))
        F = np.empty((nsteps, self.n, 3))
        for s in range(nsteps):
            x, v, f = self.run(params, x, v, step0 + s, 1, want_forces=True, broken=broken)
            dX[s] = x - xs0
            V[s] = v
            F[s] = f
        return dX, V, F

    # ---- rollout loss and its adjoint ---------------------------------------------

    def _body(self, body):
        b = np.zeros(self.n, np.int32) if body is None else np.ascontiguousarray(body, dtype=np.int32)
        return b, int(b.max()) + 1 if b.size else 1

    def rollout_loss(self, params: Params, nsteps: int, body=None):
        """Per-body J_b = -(CoM_x after nsteps - CoM_x at start), and a hash of
        every contact / friction-stick decision of the run."""
        if self.yield_ is not None:
            raise ValueError("the rollout covers unbreakable springs only")
        if params.integrator != "euler":
            raise ValueError("the rollout covers the Euler step only")
        b, nb = self._body(body)
        loss = np.empty(nb, np.float64)
        sig = ctypes.c_uint64()
        rc = _load().orc_rollout_loss(self.n, _ptr(self.mass), self.ns, _ptr(self.ends, _lp), _ptr(self.k),
                                      _ptr(self.c), _ptr(self.rest), _ptr(self.amp), _ptr(self.phase),
                                      ctypes.byref(params._c()), b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      nb, nsteps, _ptr(self.x0), _ptr(self.v0), _ptr(loss), ctypes.byref(sig))
        if rc != 0:
            raise MemoryError("oracle rollout failed")
        return loss, sig.value

    def rollout_grad(self, params: Params, nsteps: int, body=None, weights=None):
        """Adjoint of J = sum_b w_b J_b: per-spring dJ/dk, dJ/dC, dJ/dS with
        C = amp cos(phase), S = amp sin(phase).  Returns a dict with loss,
        gk, gC, gS and the decision hash."""
        if params.wave:
            raise ValueError("the rollout adjoint covers phasor actuation only")
        if self.yield_ is not None:
            raise ValueError("the rollout adjoint covers unbreakable springs only")
        if params.integrator != "euler":
            raise ValueError("the rollout adjoint covers the Euler step only")
        b, nb = self._body(body)
        w = np.ones(nb) if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        loss = np.empty(nb, np.float64)
        gk, gC, gS = (np.empty(self.ns, np.float64) for _ in range(3))
        sig = ctypes.c_uint64()
        rc = _load().orc_rollout_grad(self.n, _ptr(self.mass), self.ns, _ptr(self.ends, _lp), _ptr(self.k),
                                      _ptr(self.c), _ptr(self.rest), _ptr(self.amp), _ptr(self.phase),
                                      ctypes.byref(params._c()), b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      nb, _ptr(w), nsteps, _ptr(self.x0), _ptr(self.v0), _ptr(loss), _ptr(gk),
                                      _ptr(gC), _ptr(gS), ctypes.byref(sig))
        if rc != 0:
            raise MemoryError("oracle rollout failed")
        return dict(loss=loss, gk=gk, gC=gC, gS=gS, sig=sig.value)

    # ---- observables (plain sums) -------------------------------------------------

    def spring_stretch(self, x, t=0.0, omega=0.0):
        x = _d(x).reshape(-1, 3)
        d = x[self.ends[:, 1]] - x[self.ends[:, 0]]
        L = self.rest.copy()
        if self.amp is not None:
            L = L * (1.0 + self.amp * np.sin(omega * t + self.phase))
        return np.linalg.norm(d, axis=1) - L

    def kinetic(self, v):
        v = _d(v).reshape(-1, 3)
        return 0.5 * float(np.sum(self.mass[:, None] * v * v))

    def spring_energy(self, x, t=0.0, omega=0.0):
        e = self.spring_stretch(x, t, omega)
        return 0.5 * float(np.sum(self.k * e * e))

    def gravity_energy(self, x, g):
        x = _d(x).reshape(-1, 3)
        return -float(np.sum(self.mass[:, None] * x * np.asarray(g)[None, :]))

    def ground_energy(self, x, ground_k):
        z = _d(x).reshape(-1, 3)[:, 2]
        return 0.5 * ground_k * float(np.sum(np.where(z < 0.0, z * z, 0.0)))

    def momentum(self, v):
        return np.sum(self.mass[:, None] * _d(v).reshape(-1, 3), axis=0)

    def angular_momentum(self, x, v):
        x = _d(x).reshape(-1, 3)
        v = _d(v).reshape(-1, 3)
        return np.sum(np.cross(x, self.mass[:, None] * v), axis=0)

    def com(self, x):
        x = _d(x).reshape(-1, 3)
        return np.sum(self.mass[:, None] * x, axis=0) / np.sum(self.mass)


def voxel_grads(gC, gS, voxel_a, voxel_phi, sv_ptr, sv_idx):
    """Chain rule from per-spring actuation-phasor gradients to per-voxel
    amplitude and phase gradients.  A spring's phasor is the mean of its
    voxels' a*(cos phi, sin phi), so with n_s voxels on spring s:
    dJ/da_v   = sum_s (gC_s cos phi_v + gS_s sin phi_v) / n_s,
    dJ/dphi_v = sum_s a_v (-gC_s sin phi_v + gS_s cos phi_v) / n_s."""
    va = np.asarray(voxel_a, np.float64)
    vp = np.asarray(voxel_phi, np.float64)
    ga = np.zeros(va.size)
    gp = np.zeros(va.size)
    for s in range(len(sv_ptr) - 1):
        vs = sv_idx[sv_ptr[s]:sv_ptr[s + 1]]
        ns_ = len(vs)
        for v in vs:
            ga[v] += (gC[s] * np.cos(vp[v]) + gS[s] * np.sin(vp[v])) / ns_
            gp[v] += va[v] * (-gC[s] * np.sin(vp[v]) + gS[s] * np.cos(vp[v])) / ns_
    return ga, gp

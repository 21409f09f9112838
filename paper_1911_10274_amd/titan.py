"""Python binding of ``libtitan`` (include/titan.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels.  PyTorch
supplies the device memory (through its caching allocator, passed to the
library as a ``titan_allocator``) and the stream (the current torch stream by
default).  If ``libtitan.so`` has not been built, importing this module
raises ``ImportError``: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TITAN_LIBRARY") or os.path.join(_HERE, "libtitan.so")

OK = 0
EINVAL = -1
ENOMEM = -2
EDEVICE = -3
ESTATE = -4
ENONFINITE = -5
STATE_DISPLACEMENT = 1
BP_SNAPSHOT = 0
BP_PAUSE = 1
ENGINE_AUTO = 0
ENGINE_GATHER = 1
ENGINE_BATCHED = 2
ENGINE_TILED = 3
ACT_PHASOR = 0
ACT_WAVE = 1
INTEG_EULER = 0
INTEG_VERLET = 1
INTEG_RK4 = 2

_ERR_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ESTATE: "ESTATE", ENONFINITE: "ENONFINITE"}


class TitanError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"titan {_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double),
        ("gravity", ctypes.c_double * 3),
        ("ground", ctypes.c_int32),
        ("engine", ctypes.c_int32),
        ("ground_k", ctypes.c_double),
        ("friction_mu", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("actuation", ctypes.c_int32),
        ("wave_period", ctypes.c_double),
        ("integrator", ctypes.c_int32),
        ("graph_steps", ctypes.c_int32),
    ]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("release", _RELEASE_FN), ("ctx", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [
        ("n_masses", ctypes.c_int64),
        ("n_springs", ctypes.c_int64),
        ("n_bodies", ctypes.c_int64),
        ("step", ctypes.c_int64),
        ("steps_requested", ctypes.c_int64),
        ("first_bad_step", ctypes.c_int64),
        ("finalized", ctypes.c_int32),
        ("engine", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("paused", ctypes.c_int32),
        ("device_bytes", ctypes.c_int64),
        ("batch_threads", ctypes.c_int32),
        ("tune_batch_ms", ctypes.c_float),
        ("tune_gather_ms", ctypes.c_float),
        ("slack", ctypes.c_int32),
        ("layout_builds", ctypes.c_int64),
        ("springs_in_place", ctypes.c_int64),
        ("batch_groups", ctypes.c_int64),
        ("batch_max_group", ctypes.c_int32),
    ]


_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_vp = ctypes.c_void_p


def _load():
    # PyTorch is imported first so that libtitan binds to the HIP runtime
    # torch already carries (same soname): one runtime per process, so torch
    # streams and torch-allocated memory are valid handles inside libtitan.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1911_10274_amd/build.py (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "titan_abi_version": ([], ctypes.c_int),
        "titan_last_error": ([], ctypes.c_char_p),
        "titan_create": ([ctypes.POINTER(_Params), _vp, ctypes.POINTER(_Allocator), ctypes.POINTER(_vp)], ctypes.c_int),
        "titan_destroy": ([_vp], ctypes.c_int),
        "titan_add_masses": ([_vp, ctypes.c_int64, _fp, _fp, _fp, _i32p, _i64p], ctypes.c_int),
        "titan_add_springs": ([_vp, ctypes.c_int64, _i64p, _fp, _fp, _fp, _fp, _fp, _i64p], ctypes.c_int),
        "titan_set_params": ([_vp, ctypes.POINTER(_Params)], ctypes.c_int),
        "titan_finalize": ([_vp], ctypes.c_int),
        "titan_step": ([_vp, ctypes.c_int64], ctypes.c_int),
        "titan_set_breakpoint": ([_vp, ctypes.c_int64, ctypes.c_int32, _u64p], ctypes.c_int),
        "titan_wait": ([_vp, ctypes.c_uint64], ctypes.c_int),
        "titan_resume": ([_vp], ctypes.c_int),
        "titan_sync": ([_vp], ctypes.c_int),
        "titan_get_state": ([_vp, ctypes.c_int64, ctypes.c_int64, _fp, _fp, ctypes.c_int32, _i64p], ctypes.c_int),
        "titan_get_snapshot": ([_vp, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, _fp, _fp, ctypes.c_int32,
                                _i64p], ctypes.c_int),
        "titan_set_state": ([_vp, ctypes.c_int64, ctypes.c_int64, _fp, _fp, ctypes.c_int32], ctypes.c_int),
        "titan_get_forces": ([_vp, ctypes.c_int64, ctypes.c_int64, _fp], ctypes.c_int),
        "titan_set_step": ([_vp, ctypes.c_int64], ctypes.c_int),
        "titan_get_body_displacement": ([_vp, _fp], ctypes.c_int),
        "titan_get_body_displacement_noalloc": ([_vp, _fp], ctypes.c_int),
        "titan_set_springs": ([_vp, ctypes.c_int64, ctypes.c_int64, _fp, _fp, _fp, _fp], ctypes.c_int),
        "titan_remove_springs": ([_vp, ctypes.c_int64, _i64p], ctypes.c_int),
        "titan_remove_masses": ([_vp, ctypes.c_int64, _i64p], ctypes.c_int),
        "titan_set_yield": ([_vp, ctypes.c_int64, ctypes.c_int64, _fp], ctypes.c_int),
        "titan_get_broken": ([_vp, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint8)], ctypes.c_int),
        "titan_rollout_grad": ([_vp, ctypes.c_int64, ctypes.c_int32, _fp, _fp, _fp, _fp, _fp], ctypes.c_int),
        "titan_set_springs_phasor": ([_vp, ctypes.c_int64, ctypes.c_int64, _fp, _fp], ctypes.c_int),
        "titan_set_voxel_actuation": ([_vp, ctypes.c_int64, _fp, _fp, _i64p, _i32p], ctypes.c_int),
        "titan_rollout_grad_voxel": ([_vp, ctypes.c_int64, ctypes.c_int32, _fp, _fp, _fp, _fp, _fp], ctypes.c_int),
        "titan_rollout_grad_device": ([_vp, ctypes.c_int64, ctypes.c_int32, _fp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "titan_get_info": ([_vp, ctypes.POINTER(_Info)], ctypes.c_int),
        "titan_mlp_create": ([ctypes.c_int32, _i32p, _vp, ctypes.POINTER(_Allocator), ctypes.POINTER(_vp)],
                             ctypes.c_int),
        "titan_mlp_destroy": ([_vp], ctypes.c_int),
        "titan_mlp_param_count": ([_vp], ctypes.c_int64),
        "titan_mlp_set_params": ([_vp, _fp], ctypes.c_int),
        "titan_mlp_get_params": ([_vp, _fp], ctypes.c_int),
        "titan_mlp_set_data": ([_vp, ctypes.c_int64, _fp, _fp], ctypes.c_int),
        "titan_mlp_train": ([_vp, ctypes.c_int64, ctypes.c_int32, _i64p, ctypes.c_float, ctypes.c_float,
                             ctypes.c_float, ctypes.c_float, _fp], ctypes.c_int),
        "titan_mlp_predict": ([_vp, ctypes.c_int64, _fp, _fp], ctypes.c_int),
        "titan_mlp_grad": ([_vp, ctypes.c_int32, _fp, _fp, _fp, _fp], ctypes.c_int),
        "titan_mlp_gemm_bf16": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int32,
                                 ctypes.c_int32, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def last_error() -> str:
    return lib.titan_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise TitanError(rc, last_error())


def _f32(a, shape=None):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        arr = arr.reshape(shape)
    return arr, arr.ctypes.data_as(_fp)


@dataclass
class Params:
    dt: float = 1.0e-4
    gravity: tuple = (0.0, 0.0, -9.81)
    ground: bool = True
    ground_k: float = 1.0e5
    friction_mu: float = 0.5
    omega: float = 0.0
    engine: int = ENGINE_AUTO
    actuation: int = ACT_PHASOR
    wave_period: float = 1.0
    integrator: int = INTEG_EULER
    graph_steps: int = 0

    def _c(self) -> _Params:
        p = _Params()
        p.dt = self.dt
        p.gravity[:] = list(self.gravity)
        p.ground = 1 if self.ground else 0
        p.engine = int(self.engine)
        p.ground_k = self.ground_k
        p.friction_mu = self.friction_mu
        p.omega = self.omega
        p.actuation = int(self.actuation)
        p.wave_period = self.wave_period
        p.integrator = int(self.integrator)
        p.graph_steps = int(self.graph_steps)
        return p


class _TorchMemory:
    """Device memory from PyTorch's caching allocator, on the sim's stream."""

    def __init__(self, device: int, stream_handle: int):
        import torch

        self._torch = torch
        self.device = device
        self.stream = stream_handle

        def _alloc(nbytes, ctx):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream))
            except Exception:  # out of memory: the library reports ENOMEM
                return None

        def _release(ptr, ctx):
            torch.cuda.caching_allocator_delete(int(ptr))

        self._alloc_cb = _ALLOC_FN(_alloc)
        self._release_cb = _RELEASE_FN(_release)
        self.c = _Allocator(self._alloc_cb, self._release_cb, None)


class Sim:
    """One simulation (a ``titan_sim``).

    ``stream``: a ``torch.cuda.Stream``, a raw hipStream_t handle (int), or
    None for torch's current stream.  ``memory``: "torch" (default) routes
    device allocations through torch's caching allocator; "hip" lets the
    library call hipMalloc itself.
    """

    def __init__(self, params: Params | None = None, stream=None, memory: str = "torch"):
        self.params = params or Params()
        self._mem = None
        handle = None
        if memory not in ("torch", "hip"):
            raise ValueError("memory must be 'torch' or 'hip'")
        if stream is not None or memory == "torch":
            import torch

            if stream is None:
                stream = torch.cuda.current_stream()
            handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
            device = stream.device.index if hasattr(stream, "device") else torch.cuda.current_device()
            if memory == "torch":
                self._mem = _TorchMemory(device if device is not None else 0, handle)
        self.stream_handle = handle
        h = _vp()
        _check(lib.titan_create(ctypes.byref(self.params._c()), _vp(handle) if handle else None,
                                ctypes.byref(self._mem.c) if self._mem else None, ctypes.byref(h)))
        self._h = h

    # -- lifetime ---------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib.titan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- building ---------------------------------------------------------------
    def add_masses(self, pos, mass, vel=None, body=None) -> int:
        p, pp = _f32(pos, (-1, 3))
        n = p.shape[0]
        m, mp = _f32(mass, (n,))
        v, vp = _f32(vel, (n, 3)) if vel is not None else (None, None)
        b = None if body is None else np.ascontiguousarray(body, dtype=np.int32).reshape(n)
        first = ctypes.c_int64()
        _check(lib.titan_add_masses(self._h, n, pp, vp, mp, None if b is None else b.ctypes.data_as(_i32p),
                                    ctypes.byref(first)))
        return first.value

    def add_springs(self, ends, k, damping=None, rest=None, amp=None, phase=None) -> int:
        e = np.ascontiguousarray(ends, dtype=np.int64).reshape(-1, 2)
        n = e.shape[0]
        kk, kp = _f32(k, (n,))
        c, cp = _f32(damping, (n,)) if damping is not None else (None, None)
        r, rp = _f32(rest, (n,)) if rest is not None else (None, None)
        a, ap = _f32(amp, (n,)) if amp is not None else (None, None)
        ph, php = _f32(phase, (n,)) if phase is not None else (None, None)
        first = ctypes.c_int64()
        _check(lib.titan_add_springs(self._h, n, e.ctypes.data_as(_i64p), kp, cp, rp, ap, php, ctypes.byref(first)))
        return first.value

    def remove_springs(self, springs):
        """Remove springs (titan_remove_springs)."""
        q = np.ascontiguousarray(springs, dtype=np.int64).reshape(-1)
        _check(lib.titan_remove_springs(self._h, q.size, q.ctypes.data_as(_i64p)))

    def remove_masses(self, masses):
        """Remove masses and their springs (titan_remove_masses)."""
        q = np.ascontiguousarray(masses, dtype=np.int64).reshape(-1)
        _check(lib.titan_remove_masses(self._h, q.size, q.ctypes.data_as(_i64p)))

    def set_yield(self, yield_values, first: int = 0):
        """Yield values of springs first.. (titan_set_yield; inf: never breaks)."""
        y = np.ascontiguousarray(yield_values, dtype=np.float32).reshape(-1)
        _check(lib.titan_set_yield(self._h, first, y.size, y.ctypes.data_as(_fp)))

    def get_broken(self, first: int = 0, count: int | None = None) -> np.ndarray:
        """Broken flags of springs first.. (titan_get_broken), as bools."""
        count = self.info()["n_springs"] - first if count is None else count
        out = np.zeros(count, np.uint8)
        _check(lib.titan_get_broken(self._h, first, count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return out.astype(bool)

    def set_params(self, params: Params):
        _check(lib.titan_set_params(self._h, ctypes.byref(params._c())))
        self.params = params

    def finalize(self):
        _check(lib.titan_finalize(self._h))

    # -- running ----------------------------------------------------------------
    def step(self, n: int = 1):
        _check(lib.titan_step(self._h, int(n)))

    def set_breakpoint(self, step: int, kind: int = BP_SNAPSHOT) -> int:
        bp = ctypes.c_uint64()
        _check(lib.titan_set_breakpoint(self._h, int(step), int(kind), ctypes.byref(bp)))
        return bp.value

    def wait(self, bp: int):
        _check(lib.titan_wait(self._h, int(bp)))

    def resume(self):
        _check(lib.titan_resume(self._h))

    def sync(self):
        _check(lib.titan_sync(self._h))

    # -- state ------------------------------------------------------------------
    def info(self) -> dict:
        i = _Info()
        _check(lib.titan_get_info(self._h, ctypes.byref(i)))
        return {name: getattr(i, name) for name, _ in _Info._fields_}

    @property
    def n_masses(self) -> int:
        return self.info()["n_masses"]

    def get_state(self, first: int = 0, count: int | None = None, displacement: bool = False):
        count = self.n_masses - first if count is None else count
        pos = np.empty((count, 3), np.float32)
        vel = np.empty((count, 3), np.float32)
        step = ctypes.c_int64()
        _check(lib.titan_get_state(self._h, first, count, pos.ctypes.data_as(_fp), vel.ctypes.data_as(_fp),
                                   STATE_DISPLACEMENT if displacement else 0, ctypes.byref(step)))
        return pos, vel, step.value

    def get_snapshot(self, bp: int, first: int = 0, count: int | None = None, displacement: bool = False):
        count = self.n_masses - first if count is None else count
        pos = np.empty((count, 3), np.float32)
        vel = np.empty((count, 3), np.float32)
        step = ctypes.c_int64()
        _check(lib.titan_get_snapshot(self._h, int(bp), first, count, pos.ctypes.data_as(_fp),
                                      vel.ctypes.data_as(_fp), STATE_DISPLACEMENT if displacement else 0,
                                      ctypes.byref(step)))
        return pos, vel, step.value

    def set_state(self, pos=None, vel=None, first: int = 0, displacement: bool = False):
        p, pp = _f32(pos, (-1, 3)) if pos is not None else (None, None)
        v, vp = _f32(vel, (-1, 3)) if vel is not None else (None, None)
        count = (p if p is not None else v).shape[0]
        _check(lib.titan_set_state(self._h, first, count, pp, vp, STATE_DISPLACEMENT if displacement else 0))

    def body_displacement(self):
        """(n_bodies, 3) centre-of-mass displacement of every body."""
        nb = self.info()["n_bodies"]
        out = np.empty((nb, 3), np.float32)
        _check(lib.titan_get_body_displacement(self._h, out.ctypes.data_as(_fp)))
        return out

    def body_displacement_noalloc(self):
        """``body_displacement`` through titan_get_body_displacement_noalloc
        (no device allocation; the sim must have stepped or been finalized)."""
        nb = self.info()["n_bodies"]
        out = np.empty((nb, 3), np.float32)
        _check(lib.titan_get_body_displacement_noalloc(self._h, out.ctypes.data_as(_fp)))
        return out

    def set_springs(self, first: int = 0, k=None, damping=None, amp=None, phase=None):
        """Change spring constants (see titan_set_springs)."""
        arrs = [a for a in (k, damping, amp, phase) if a is not None]
        if not arrs:
            return
        count = int(np.asarray(arrs[0]).size)
        ptrs, keep = [], []
        for a in (k, damping, amp, phase):
            arr, p = _f32(a, (count,)) if a is not None else (None, None)
            keep.append(arr)
            ptrs.append(p)
        _check(lib.titan_set_springs(self._h, int(first), count, *ptrs))

    def rollout_grad(self, nsteps: int, checkpoint_every: int = 50, body_weights=None):
        """Adjoint gradient of J = sum_b w_b J_b (J_b = -CoM x-displacement of
        body b after ``nsteps`` steps from the current state).  Returns
        (loss per body, dJ/dk, dJ/dC, dJ/dS) as numpy arrays."""
        info = self.info()
        nb, ns = info["n_bodies"], info["n_springs"]
        w, wp = _f32(body_weights, (nb,)) if body_weights is not None else (None, None)
        loss = np.empty(nb, np.float32)
        gk, gc, gs = (np.empty(ns, np.float32) for _ in range(3))
        _check(lib.titan_rollout_grad(self._h, int(nsteps), int(checkpoint_every), wp, loss.ctypes.data_as(_fp),
                                      gk.ctypes.data_as(_fp), gc.ctypes.data_as(_fp), gs.ctypes.data_as(_fp)))
        return loss, gk, gc, gs

    def rollout_grad_device(self, nsteps: int, checkpoint_every: int = 50, body_weights=None, out=None):
        """As ``rollout_grad`` with the results in GPU memory: returns torch
        float32 tensors (loss per body, dJ/dk, dJ/dC, dJ/dS) on the current
        device, or writes into ``out`` (four contiguous float32 CUDA tensors
        of those sizes, or None for an output not wanted)."""
        import torch

        info = self.info()
        nb, ns = info["n_bodies"], info["n_springs"]
        w, wp = _f32(body_weights, (nb,)) if body_weights is not None else (None, None)
        if out is None:
            out = (torch.empty(nb, dtype=torch.float32, device="cuda"),
                   *(torch.empty(ns, dtype=torch.float32, device="cuda") for _ in range(3)))
        ptrs = []
        for t, n in zip(out, (nb, ns, ns, ns)):
            if t is None:
                ptrs.append(None)
                continue
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == n):
                raise ValueError("outputs must be contiguous float32 CUDA tensors of n_bodies / n_springs values")
            ptrs.append(_vp(t.data_ptr()))
        _check(lib.titan_rollout_grad_device(self._h, int(nsteps), int(checkpoint_every), wp, *ptrs))
        return tuple(out)

    def set_springs_phasor(self, first: int = 0, act_c=None, act_s=None):
        """Actuation phasors (C, S) of springs [first, first + len) as given."""
        c, cp = _f32(act_c, (-1,))
        s_, sp = _f32(act_s, (c.size,))
        _check(lib.titan_set_springs_phasor(self._h, int(first), c.size, cp, sp))

    def set_voxel_actuation(self, voxel_a, voxel_phi, sv_ptr, sv_idx):
        """Per-voxel amplitude and phase; sv_ptr / sv_idx list each spring's
        voxels (n_springs + 1 offsets)."""
        a, ap = _f32(voxel_a, (-1,))
        ph, pp = _f32(voxel_phi, (a.size,))
        ptr = np.ascontiguousarray(sv_ptr, dtype=np.int64)
        idx = np.ascontiguousarray(sv_idx, dtype=np.int32)
        _check(lib.titan_set_voxel_actuation(self._h, a.size, ap, pp, ptr.ctypes.data_as(_i64p),
                                             idx.ctypes.data_as(_i32p)))
        self._n_voxels = a.size

    def rollout_grad_voxel(self, nsteps: int, checkpoint_every: int = 50, body_weights=None, n_voxels=None):
        """As ``rollout_grad`` with the actuation gradient per voxel: returns
        (loss per body, dJ/dk, dJ/da per voxel, dJ/dphi per voxel)."""
        info = self.info()
        nb, ns = info["n_bodies"], info["n_springs"]
        w, wp = _f32(body_weights, (nb,)) if body_weights is not None else (None, None)
        nv = int(n_voxels if n_voxels is not None else getattr(self, "_n_voxels", 0))
        loss = np.empty(nb, np.float32)
        gk = np.empty(ns, np.float32)
        ga, gp = np.empty(nv, np.float32), np.empty(nv, np.float32)
        _check(lib.titan_rollout_grad_voxel(self._h, int(nsteps), int(checkpoint_every), wp, loss.ctypes.data_as(_fp),
                                            gk.ctypes.data_as(_fp), ga.ctypes.data_as(_fp), gp.ctypes.data_as(_fp)))
        return loss, gk, ga, gp

    def set_step(self, step: int):
        _check(lib.titan_set_step(self._h, int(step)))

    def get_forces(self, first: int = 0, count: int | None = None):
        count = self.n_masses - first if count is None else count
        f = np.empty((count, 3), np.float32)
        _check(lib.titan_get_forces(self._h, first, count, f.ctypes.data_as(_fp)))
        return f


def sim_from_scene(scene: dict, params: Params, rest=None, **kw) -> Sim:
    """A Sim holding ``scene`` (a dict from ``scenes``)."""
    sim = Sim(params, **kw)
    sim.add_masses(scene["pos"], scene["mass"], vel=scene.get("vel"), body=scene.get("body"))
    if scene["ends"].shape[0]:
        sim.add_springs(scene["ends"], scene["k"], damping=scene.get("damping"), rest=rest,
                        amp=scene.get("amp"), phase=scene.get("phase"))
        if scene.get("yield") is not None:
            sim.set_yield(scene["yield"])
    return sim


class Mlp:
    """The surrogate network (``titan_mlp``).  ``dims``: layer widths."""

    def __init__(self, dims, stream=None, memory: str = "torch"):
        import torch

        self.dims = [int(d) for d in dims]
        if stream is None:
            stream = torch.cuda.current_stream()
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self._mem = _TorchMemory(torch.cuda.current_device(), handle) if memory == "torch" else None
        d = np.asarray(self.dims, np.int32)
        h = _vp()
        _check(lib.titan_mlp_create(len(self.dims) - 1, d.ctypes.data_as(_i32p), _vp(handle) if handle else None,
                                    ctypes.byref(self._mem.c) if self._mem else None, ctypes.byref(h)))
        self._h = h
        self.n_params = int(lib.titan_mlp_param_count(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib.titan_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        p, pp = _f32(flat, (self.n_params,))
        _check(lib.titan_mlp_set_params(self._h, pp))

    def get_params(self):
        out = np.empty(self.n_params, np.float32)
        _check(lib.titan_mlp_get_params(self._h, out.ctypes.data_as(_fp)))
        return out

    def set_data(self, X, Y):
        x, xp = _f32(X, (-1, self.dims[0]))
        y, yp = _f32(Y, (-1, self.dims[-1]))
        _check(lib.titan_mlp_set_data(self._h, x.shape[0], xp, yp))

    def train(self, idx, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """Adam steps over the rows listed by idx (nsteps x batch)."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        nsteps, batch = idx.shape
        loss = np.empty(nsteps, np.float32)
        _check(lib.titan_mlp_train(self._h, nsteps, batch, idx.ctypes.data_as(_i64p), lr, beta1, beta2, eps,
                                   loss.ctypes.data_as(_fp)))
        return loss

    def predict(self, X):
        x, xp = _f32(X, (-1, self.dims[0]))
        out = np.empty((x.shape[0], self.dims[-1]), np.float32)
        _check(lib.titan_mlp_predict(self._h, x.shape[0], xp, out.ctypes.data_as(_fp)))
        return out

    def grad(self, X, Y):
        x, xp = _f32(X, (-1, self.dims[0]))
        y, yp = _f32(Y, (-1, self.dims[-1]))
        loss = np.empty(1, np.float32)
        g = np.empty(self.n_params, np.float32)
        _check(lib.titan_mlp_grad(self._h, x.shape[0], xp, yp, loss.ctypes.data_as(_fp), g.ctypes.data_as(_fp)))
        return float(loss[0]), g


def gemm_bf16(A, B, ta=False, tb=False, M=None, N=None, K=None, stream=None):
    """C = op(A) op(B) on the MFMA GEMM kernel; A, B are torch int16/uint16
    (bfloat16 bit patterns) CUDA tensors, C a new float32 CUDA tensor."""
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    if M is None:
        M = A.shape[1] if ta else A.shape[0]
        K = A.shape[0] if ta else A.shape[1]
        N = B.shape[0] if tb else B.shape[1]
    lda = A.shape[1]
    ldb = B.shape[1]
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(lib.titan_mlp_gemm_bf16(M, N, K, _vp(A.data_ptr()), lda, int(ta), _vp(B.data_ptr()), ldb, int(tb),
                                   _vp(C.data_ptr()), _vp(stream.cuda_stream) if stream.cuda_stream else None))
    return C

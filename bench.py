#!/usr/bin/env python3
"""Throughput benchmark of the mass-spring step on one MI355X.

Workload: the large actuated lattice -- 100^3 masses (1,000,000), the
26-neighbourhood springs (12,731,796), positions jittered by +-2% of the
0.1 m spacing, k ~ U(5e3, 2e4) N/m, every rest length actuated as
L0 (1 + 0.1 sin(2 pi 2 t + phi)), phi ~ U(0, 2 pi), damping 1 N s/m, ground
contact on (k_g = 1e5 N/m, mu = 0.5), dt = 5e-5 s.  Inputs are seeded and
synthetic and are resident in GPU memory before the timed region.

One "step" is one simulation step of the whole system.  The metric is spring
updates per second (springs x steps / wall time), the unit the paper uses for
its lattice benchmark (Sec. IV-A).

Prints ONE JSON line.  ``roofline`` reports the step kernel against the HBM
bandwidth peak using the algorithmic byte count per step; ``cpu_baseline``
times the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "tiled_step_lattice100.md")
# the kernel and the host code that lays out its input (the counters depend on both)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1911_10274_amd", "csrc", f)
                  for f in ("gather_step.hip", "step_device.h", "titan_internal.h", "engine_gather.hip")]


def algorithmic_bytes(n_masses: int, n_springs: int) -> int:
    """Bytes one step must move under the minimal model: per spring its two
    int32 end indices and four FP32 constants (k, rest, actuation phasor C, S)
    = 24 B; per mass the state read (u, v, x0: 3 x 16 B), the state written
    (u, v: 2 x 16 B) and one int32 of incidence bookkeeping = 84 B."""
    return 24 * n_springs + 84 * n_masses


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if there is none or the kernel source changed since it was taken."""
    if not os.path.exists(PROFILE_SUMMARY):
        return None
    txt = open(PROFILE_SUMMARY).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    hsh = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", txt)
    if not m or not hsh or hsh.group(1) != kernel_source_hash():
        return None
    return float(m.group(1))


def build_workload(n: int, seed: int):
    from paper_1911_10274_amd import scenes

    return scenes.jittered_actuated_lattice(n=n, seed=seed)


PARAMS = dict(dt=5e-5, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, mu=0.5, omega=2 * math.pi * 2)


def _host_cores() -> int:
    """Cores this process may use: the affinity mask, capped by the thread
    budget the environment sets (OMP_NUM_THREADS), if any."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS")
    return max(1, min(n, int(cap))) if cap and cap.isdigit() else n


def cpu_baseline(scene, steps: int, repeats: int = 3):
    """The FP64 oracle, as it stands, on the first ``steps`` steps of the same
    workload, built for this host (gcc -O3 -march=native, no FMA
    contraction): the median of ``repeats`` single-thread runs, and the
    aggregate rate of one copy of the same window per host core, run
    concurrently (independent processes; the oracle is a serial loop).  Each
    measurement times the step loop alone, in its own process."""
    import statistics
    import subprocess
    import tempfile

    import numpy as np

    from oracle import oracle as O

    ns = scene["ends"].shape[0]
    with tempfile.TemporaryDirectory(prefix="titan_cpu_") as tmp:
        lib = O.build_native(tmp)
        path = os.path.join(tmp, "scene.npz")
        np.savez(path, pos=scene["pos"], vel=scene["vel"], mass=scene["mass"], ends=scene["ends"], k=scene["k"],
                 damping=scene["damping"], amp=scene["amp"], phase=scene["phase"], dt=PARAMS["dt"],
                 g=np.asarray(PARAMS["gravity"]), ground=PARAMS["ground"], ground_k=PARAMS["ground_k"],
                 mu=PARAMS["mu"], omega=PARAMS["omega"])
        cmd = [sys.executable, "-m", "oracle.baseline", path, str(steps), lib]
        env = dict(os.environ, OMP_NUM_THREADS="1")

        def run(count):
            procs = [subprocess.Popen(cmd, cwd=ROOT, env=env, stdout=subprocess.PIPE, text=True) for _ in range(count)]
            outs = [p.communicate()[0] for p in procs]
            if any(p.returncode for p in procs):
                raise RuntimeError("CPU baseline worker failed")
            return [json.loads(o.strip().splitlines()[-1])["seconds"] for o in outs]

        single = [run(1)[0] for _ in range(repeats)]
        cores = _host_cores()
        many = run(cores)
    sec = statistics.median(single)
    return {
        "value": ns * steps / sec,
        "unit": "spring updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {steps} steps of the same {scene['pos'].shape[0]}-mass / {ns}-spring lattice, serial FP64 "
                  f"C oracle (gcc -O3 -march=native), median of {repeats} runs: "
                  + ", ".join(f"{x:.2f}" for x in single) + " s",
        "all_cores": {
            "value": cores * ns * steps / max(many),
            "cores": cores,
            "sample": f"{cores} concurrent single-thread oracle processes, each the same {steps}-step window "
                      f"(slowest {max(many):.2f} s): aggregate host throughput",
        },
    }


def copy_calibration(mib: int = 1024, reps: int = 5):
    """A plain device copy of known size, for scaling rocprofv3 FETCH_SIZE /
    WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch

    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4, "reps": reps}))


def copy_bandwidth(mib: int = 2048, reps: int = 10):
    """What this GPU's HBM delivers to a plain device-to-device copy (bytes
    read + written per second): context for the roofline, whose peak stays
    the published 8 TB/s."""
    import torch

    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    sec = ev0.elapsed_time(ev1) / reps * 1e-3
    del a, b
    return {"bytes": 2 * n * 4, "gbs": 2 * n * 4 / sec / 1e9}


def _timed_steps(sim, steps, stream):
    """Milliseconds of ``steps`` steps, HIP events on the sim's stream."""
    import torch

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    sim.step(steps)
    end.record(stream)
    end.synchronize()
    sim.sync()
    return start.elapsed_time(end)


def bench_batched(T, robots_n: int, steps: int, loop_sample: int):
    """Uneven voxel robots: the batched engine (one launch runs every robot
    for all steps, each robot group resident in LDS) against the plain tiled
    engine on the same system and against the plain per-robot loop (each
    robot its own simulation, one launch per step), the latter timed on a
    sample of robots at evenly spaced size ranks and scaled to all robots."""
    import numpy as np
    import torch

    from paper_1911_10274_amd import scenes

    robots = scenes.robot_batch(robots_n, seed=3, side_lo=3, side_hi=12)
    sc = scenes.concat(robots)
    nm, ns = sc["pos"].shape[0], sc["ends"].shape[0]
    stream = torch.cuda.current_stream()
    res = {"workload": f"{robots_n} voxel robots, side U{{3..12}}, Bernoulli(0.6) voxels, largest "
                       f"6-connected component, {steps} steps", "robots": robots_n, "masses": nm,
           "springs": ns, "steps": steps, "unit": "spring updates/s"}

    def mk(engine):
        tp = T.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5,
                      omega=2 * math.pi * 2, engine=engine)
        sim = T.sim_from_scene(sc, tp)
        sim.finalize()
        return sim

    def other_integrators(sim, engine, isteps=200):
        """Verlet and RK4 on the same sim (switched by set_params, same layout)."""
        out = {}
        for name, integ in (("verlet", T.INTEG_VERLET), ("rk4", T.INTEG_RK4)):
            tp = T.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5,
                          omega=2 * math.pi * 2, engine=engine, integrator=integ)
            try:
                sim.set_params(tp)
            except T.TitanError as e:
                out[name] = {"not_run": str(e)}
                continue
            sim.step(5)
            sim.sync()
            ims = _timed_steps(sim, isteps, stream)
            out[name] = {"ms_per_step": ims / isteps, "engine": {T.ENGINE_BATCHED: "batched",
                                                                  T.ENGINE_TILED: "tiled",
                                                                  T.ENGINE_GATHER: "gather"}[sim.info()["engine"]]}
        return out

    sim = mk(T.ENGINE_BATCHED)
    info = sim.info()
    sim.step(20)
    sim.sync()
    ms = _timed_steps(sim, steps, stream)
    integ_batched = other_integrators(sim, T.ENGINE_BATCHED)
    sim.close()
    res.update(value=ns * steps / (ms / 1e3), ms_per_step=ms / steps, engine="batched",
               workgroup_threads=info["batch_threads"], groups=info["batch_groups"],
               largest_group_masses=info["batch_max_group"])
    sim = mk(T.ENGINE_TILED)
    sim.step(20)
    sim.sync()
    ms_plain = _timed_steps(sim, steps, stream)
    integ_plain = other_integrators(sim, T.ENGINE_TILED)
    sim.close()
    res["integrators"] = {"batched": integ_batched, "plain": integ_plain, "steps": 200}
    res["plain_same_system"] = {"value": ns * steps / (ms_plain / 1e3), "ms_per_step": ms_plain / steps,
                                "engine": "tiled"}

    order = np.argsort([r["ends"].shape[0] for r in robots], kind="stable")
    pick = order[np.linspace(0, len(robots) - 1, loop_sample).round().astype(int)]
    tot_ms, tot_springs = 0.0, 0
    for b in pick:
        r = robots[b]
        tp = T.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5,
                      omega=2 * math.pi * 2, engine=T.ENGINE_TILED)
        one = T.sim_from_scene(r, tp)
        one.finalize()
        one.step(5)
        one.sync()
        tot_ms += _timed_steps(one, steps, stream)
        tot_springs += r["ends"].shape[0]
        one.close()
    loop_ms = tot_ms / len(pick) * len(robots)
    res["per_robot_loop"] = {"value": ns * steps / (loop_ms / 1e3), "ms_total": loop_ms,
                             "sample": f"{len(pick)} robots at evenly spaced spring-count ranks, each "
                                       f"{steps} steps on its own; mean time x {len(robots)} robots",
                             "extrapolated": True}
    res["speedup_vs_per_robot_loop"] = loop_ms / ms
    res["speedup_vs_plain_same_system"] = ms_plain / ms
    return res


def bench_adjoint(T, robots_n: int, steps: int, K: int):
    """Gradient of the 500-step rollout loss (-CoM x-displacement) of 256
    voxel robots with respect to every spring's stiffness and actuation, by
    the checkpointed adjoint; timed against the forward rollout alone."""
    import time as _t

    import torch

    from paper_1911_10274_amd import scenes

    robots = scenes.robot_batch(robots_n, seed=4, side_lo=4, side_hi=8)
    sc = scenes.concat(robots)
    nm, ns = sc["pos"].shape[0], sc["ends"].shape[0]
    tp = T.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5,
                  omega=2 * math.pi * 2, engine=T.ENGINE_BATCHED)
    sim = T.sim_from_scene(sc, tp)
    sim.finalize()
    reps = 3
    # outputs in HBM (titan_rollout_grad_device): the device-resident rate;
    # the host-output call adds the copy of the gradients to host memory
    outs = (torch.empty(len(robots), dtype=torch.float32, device="cuda"),
            *(torch.empty(ns, dtype=torch.float32, device="cuda") for _ in range(3)))

    def timed(k, device):
        run = (lambda: sim.rollout_grad_device(steps, k, out=outs)) if device else (lambda: sim.rollout_grad(steps, k))
        run()  # warm-up
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        for _ in range(reps):
            run()
        return (_t.perf_counter() - t0) / reps

    sec = timed(K, True)
    sec_host = timed(K, False)
    # every state kept (one segment, no recompute): 48 B per mass per step
    sec_all = timed(steps, True)
    sec_all_host = timed(steps, False)
    ms_fwd = _timed_steps(sim, steps, torch.cuda.current_stream())
    sim.close()
    return {"workload": f"{robots_n} voxel robots, side U{{4..8}}, {steps}-step rollout, checkpoints every {K} "
                        f"steps, gradients w.r.t. every spring's k and actuation phasor (outputs in HBM)",
            "robots": robots_n, "masses": nm, "springs": ns, "steps": steps, "checkpoint_every": K,
            "value": steps / sec, "unit": "adjoint steps/s",
            "robot_steps_per_s": robots_n * steps / sec,
            "ms_per_gradient": sec * 1e3,
            "ms_per_gradient_host_outputs": sec_host * 1e3,
            "forward_ms": ms_fwd, "gradient_over_forward": sec * 1e3 / ms_fwd,
            "all_states_kept": {"checkpoint_every": steps, "segment_bytes": 48 * nm * steps,
                                "ms_per_gradient": sec_all * 1e3, "value": steps / sec_all,
                                "ms_per_gradient_host_outputs": sec_all_host * 1e3,
                                "gradient_over_forward": sec_all * 1e3 / ms_fwd}}


def bench_worms(T, count: int = 100, steps: int = 10000):
    """The paper's worm swarm (Sec. IV-B): ``count`` 27 x 5 x 3 worms
    (339,200 springs for 100), wave actuation omega = 20, t_p = 1 s, c = 0.2,
    dt = 1e-4: one simulated second, batched engine and plain engine."""
    import torch

    from paper_1911_10274_amd import scenes

    sc = scenes.worm_batch(count)
    ns = sc["ends"].shape[0]
    out = {"workload": f"{count} worms (27x5x3 lattice each), wave actuation, {steps} steps of dt = 1e-4",
           "worms": count, "masses": sc["pos"].shape[0], "springs": ns, "steps": steps}
    for name, eng in (("batched", T.ENGINE_BATCHED), ("plain", T.ENGINE_TILED)):
        tp = T.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5, omega=20.0,
                      engine=eng, actuation=T.ACT_WAVE, wave_period=1.0)
        sim = T.sim_from_scene(sc, tp)
        sim.finalize()
        sim.step(100)
        sim.sync()
        ms = _timed_steps(sim, steps, torch.cuda.current_stream())
        if name == "batched":
            out["com_dx_m_after_1s"] = [float(d) for d in sim.body_displacement()[:, 0][:3]]
        sim.close()
        out[name] = {"spring_updates_per_s": ns * steps / (ms * 1e-3), "ms_per_step": ms / steps,
                     "times_real_time": steps * 1e-4 / (ms * 1e-3)}
    return out


def bench_surrogate(T, batch: int = 1024, steps: int = 60, gemm_n: int = 8192):
    """Training throughput of the surrogate network (1536 -> 512 x 4 -> 3,
    Adam) on the library's BF16 MFMA kernels at the training batch size, and
    the MFMA GEMM kernel alone on one large square product."""
    import numpy as np
    import torch

    dims = [1536, 512, 512, 512, 512, 3]
    rng = np.random.Generator(np.random.PCG64(11))
    n = 16 * batch
    X = rng.standard_normal((n, dims[0])).astype(np.float32)
    Y = rng.standard_normal((n, dims[-1])).astype(np.float32)
    net = T.Mlp(dims)
    params = np.concatenate([np.concatenate([rng.uniform(-1, 1, dims[l] * dims[l + 1]) * math.sqrt(3.0 / dims[l]),
                                             np.zeros(dims[l + 1])]) for l in range(len(dims) - 1)])
    net.set_params(params.astype(np.float32))
    net.set_data(X, Y)
    idx = rng.integers(0, n, (steps, batch))
    net.train(idx[:5])  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.train(idx)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    net.close()
    macs = sum(dims[l] * dims[l + 1] for l in range(len(dims) - 1))
    train_flops = 3 * 2 * macs * batch * steps  # forward, data gradient, weight gradient
    # bf16 bit patterns of magnitude below 1 (sign and top exponent bit clear)
    A = torch.randint(-2**15, 2**15, (gemm_n, gemm_n), dtype=torch.int16, device="cuda") & 0x3F7F
    B = torch.randint(-2**15, 2**15, (gemm_n, gemm_n), dtype=torch.int16, device="cuda") & 0x3F7F
    gemm = {"shape": [gemm_n, gemm_n, gemm_n]}
    # NN: both operands row-major; NT: B given as its transpose (K contiguous
    # in both operands), the layout of the network's forward product x W^T
    for name, tb in (("nn", False), ("nt", True)):
        T.gemm_bf16(A, B, tb=tb)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        ev0.record()
        for _ in range(reps):
            T.gemm_bf16(A, B, tb=tb)
        ev1.record()
        torch.cuda.synchronize()
        gms = ev0.elapsed_time(ev1) / reps
        gflops = 2.0 * gemm_n ** 3 / (gms * 1e-3)
        gemm[name] = {"ms": gms, "tflops": gflops / 1e12, "frac_of_bf16_peak": gflops / 2.5e15}
    return {"workload": f"surrogate MLP 1536-512x4-3 (1,576,451 parameters), batch {batch}, {steps} Adam steps",
            "train_ms_per_step": sec * 1e3 / steps, "train_tflops": train_flops / sec / 1e12,
            "train_frac_of_bf16_peak": train_flops / sec / 2.5e15, "gemm": gemm}


def bench_integrators(T, scene, steps: int = 1000):
    """Velocity Verlet and RK4 (Sec. III-B) on the benchmark lattice, tiled
    engine: time per step against the Euler step's.  A Verlet step is one
    force evaluation plus a drift pass over the masses; an RK4 step is four
    force evaluations."""
    import torch

    ns = scene["ends"].shape[0]
    out = {"workload": f"the same lattice ({ns} springs), tiled engine, {steps} steps each"}
    for name, integ, evals in (("verlet", T.INTEG_VERLET, 1), ("rk4", T.INTEG_RK4, 4)):
        tp = T.Params(dt=PARAMS["dt"], gravity=PARAMS["gravity"], ground=PARAMS["ground"],
                      ground_k=PARAMS["ground_k"], friction_mu=PARAMS["mu"], omega=PARAMS["omega"],
                      engine=T.ENGINE_TILED, integrator=integ)
        sim = T.sim_from_scene(scene, tp)
        sim.finalize()
        sim.step(20)
        sim.sync()
        ms = _timed_steps(sim, steps, torch.cuda.current_stream())
        sim.close()
        out[name] = {"ms_per_step": ms / steps, "steps_per_s": steps / (ms * 1e-3),
                     "spring_evaluations_per_s": evals * ns * steps / (ms * 1e-3)}
    return out


def bench_graphs(T, steps: int = 10000, graph_steps: int = 512):
    """A small system, where launches rather than bytes bound a step: the
    10^3 falling cube (10,476 springs, dt = 1e-4) on the tiled engine, one
    launch per step against replays of a captured graph of graph_steps
    launches."""
    import torch

    from paper_1911_10274_amd import scenes

    sc = scenes.cube_drop(10)
    ns = sc["ends"].shape[0]
    out = {"workload": f"10^3 cube ({ns} springs), tiled engine, {steps} steps", "graph_steps": graph_steps}
    for name, g in (("launches", 0), ("graph", graph_steps)):
        tp = T.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5,
                      engine=T.ENGINE_TILED, graph_steps=g)
        sim = T.sim_from_scene(sc, tp)
        sim.finalize()
        sim.step(2 * graph_steps)
        sim.sync()
        ms = _timed_steps(sim, steps, torch.cuda.current_stream())
        sim.close()
        out[name] = {"us_per_step": 1e3 * ms / steps, "spring_updates_per_s": ns * steps / (ms * 1e-3)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=100, help="lattice side (masses per edge)")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate training / GEMM figures")
    ap.add_argument("--worms", type=int, default=100, help="worms in the wave-actuation workload (0: skip)")
    ap.add_argument("--engine", choices=("tiled", "gather"), default="tiled")
    ap.add_argument("--robots", type=int, default=4096, help="voxel robots in the batched workload (0: skip)")
    ap.add_argument("--robot-steps", type=int, default=2000)
    ap.add_argument("--loop-sample", type=int, default=32)
    ap.add_argument("--adjoint-robots", type=int, default=256, help="robots in the adjoint workload (0: skip)")
    ap.add_argument("--integrator-steps", type=int, default=1000,
                    help="steps of Verlet and of RK4 on the lattice (0: skip)")
    ap.add_argument("--no-graphs", action="store_true", help="skip the captured-step-loop figure")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the stepper has no multi-GPU path "
              "(one lattice per GPU; see the sharding design notes)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        copy_calibration()
        return

    import torch

    from paper_1911_10274_amd import titan as T

    torch.cuda.set_device(0)
    scene = build_workload(args.n, args.seed)
    nm, ns = scene["pos"].shape[0], scene["ends"].shape[0]
    tp = T.Params(dt=PARAMS["dt"], gravity=PARAMS["gravity"], ground=PARAMS["ground"], ground_k=PARAMS["ground_k"],
                  friction_mu=PARAMS["mu"], omega=PARAMS["omega"],
                  engine=T.ENGINE_TILED if args.engine == "tiled" else T.ENGINE_GATHER)
    sim = T.sim_from_scene(scene, tp)
    sim.finalize()
    engine = {T.ENGINE_TILED: "tiled", T.ENGINE_GATHER: "gather"}[sim.info()["engine"]]
    stream = torch.cuda.current_stream()

    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    sim.step(args.steps)
    end.record(stream)
    end.synchronize()
    torch.cuda.synchronize()
    sim.sync()  # raises on a non-finite state
    ms = start.elapsed_time(end)
    ms_per_step = ms / args.steps
    value = ns * args.steps / (ms / 1e3)

    abytes = algorithmic_bytes(nm, ns)
    achieved = abytes / (ms_per_step / 1e3) / 1e9
    traffic = measured_traffic()
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
    }
    roofline["copy_gbs"] = round(copy_bandwidth()["gbs"], 1)  # context: a plain 2 GiB copy on this GPU
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(scene, args.cpu_steps)

    out = {
        "metric": "spring updates/s",
        "value": value,
        "unit": "spring updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"actuated jittered lattice {args.n}^3 (plain fused step, {engine} kernel)",
            "masses": nm,
            "springs": ns,
            "dt": PARAMS["dt"],
            "seed": args.seed,
            "engine": engine,
            "algorithmic_bytes_per_step": abytes,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    sim.close()
    if args.integrator_steps > 0:
        out["integrators"] = bench_integrators(T, scene, args.integrator_steps)
        out["integrators"]["euler_ms_per_step"] = ms_per_step
    if not args.no_graphs:
        out["graphs"] = bench_graphs(T)
    if args.robots > 0:
        out["batched"] = bench_batched(T, args.robots, args.robot_steps, args.loop_sample)
    if args.adjoint_robots > 0:
        out["adjoint"] = bench_adjoint(T, args.adjoint_robots, 500, 50)
    if args.worms > 0:
        out["worms"] = bench_worms(T, args.worms)
    if not args.no_surrogate:
        out["surrogate"] = bench_surrogate(T)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""Learned surrogate of the simulator: dataset, training, screening.

A voxel robot (side <= 8) is described by its 8x8x8 occupancy and, per voxel,
the actuation phasor (a cos(phi), a sin(phi)): 1536 numbers.  The target is
the robot's centre-of-mass displacement after 2000 steps (dt = 1e-4,
actuation at 2 Hz, ground with friction), computed by the simulator itself
(batched engine).  The network (1536 -> 512 x 4 GELU -> 3) is trained on the
GPU by the library's own BF16-MFMA kernels (titan_mlp_*).  Screening ranks
held-out robots by the predicted x-displacement and re-simulates only the
best fraction: the simulator is the fallback and the judge.

Run as ``python -m paper_1911_10274_amd.surrogate`` (see ``--help``); prints
one JSON line of metrics.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import scenes

GRID = 8
IN_DIM = 3 * GRID ** 3
DIMS = [IN_DIM, 512, 512, 512, 512, 3]
STEPS = 2000
OMEGA = 2 * math.pi * 2


def featurize(batch: dict) -> np.ndarray:
    """(robots, 1536) float32: occupancy, a cos(phi), a sin(phi) per voxel of
    the 8^3 frame (zero outside the robot)."""
    count = batch["occ"].shape[0]
    occ = batch["occ"].reshape(count, -1).astype(np.float64)
    a = batch["vox_a"].reshape(count, -1)
    ph = batch["vox_phi"].reshape(count, -1)
    return np.concatenate([occ, a * np.cos(ph), a * np.sin(ph)], axis=1).astype(np.float32)


def sim_params(engine=None):
    from . import titan as T

    return T.Params(dt=1e-4, gravity=(0.0, 0.0, -9.81), ground=True, ground_k=1e5, friction_mu=0.5, omega=OMEGA,
                    engine=T.ENGINE_BATCHED if engine is None else engine)


def simulate(batch: dict, steps: int = STEPS, engine=None):
    """Centre-of-mass displacement (robots, 3) after ``steps`` steps, and the
    GPU seconds of the stepping."""
    import torch

    from . import titan as T

    sim = T.sim_from_scene(batch, sim_params(engine))
    sim.finalize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    sec = time.perf_counter() - t0
    d = sim.body_displacement()
    sim.close()
    return d, sec


def chunk_seed(seed: int, c: int) -> int:
    return seed * 1_000_003 + c


def dataset(count: int, seed: int, chunk: int = 16384, log=None):
    """Features, targets and total GPU stepping seconds for ``count`` robots,
    generated in chunks (chunk c drawn with seed ``seed * 1000003 + c``)."""
    X, Y, gpu = [], [], 0.0
    for c, a in enumerate(range(0, count, chunk)):
        n = min(chunk, count - a)
        b = scenes.small_robot_batch(n, chunk_seed(seed, c))
        d, sec = simulate(b)
        X.append(featurize(b))
        Y.append(d)
        gpu += sec
        if log:
            log(f"chunk {c}: {n} robots, {b['ends'].shape[0]} springs, {sec:.3f} s")
    return np.concatenate(X), np.concatenate(Y), gpu


def init_params(dims, seed: int) -> np.ndarray:
    """Flat parameters: W_l ~ U(-sqrt(3/in), sqrt(3/in)) (unit-variance
    preserving for unit inputs), b_l = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for l in range(len(dims) - 1):
        lim = math.sqrt(3.0 / dims[l])
        parts.append(rng.uniform(-lim, lim, dims[l] * dims[l + 1]))
        parts.append(np.zeros(dims[l + 1]))
    return np.concatenate(parts).astype(np.float32)


class Surrogate:
    def __init__(self, dims=DIMS, seed: int = 0):
        from . import titan as T

        self.net = T.Mlp(dims)
        self.net.set_params(init_params(dims, seed))
        self.mu = np.zeros(dims[-1])
        self.sd = np.ones(dims[-1])

    def fit(self, X, Y, epochs: int = 30, batch: int = 1024, lr: float = 1e-3, seed: int = 1, log=None,
            X_val=None, Y_val=None):
        """Adam on standardised targets, cosine-decayed learning rate.
        Returns a dict: the mean training loss of every epoch, the held-out
        loss (standardised MSE) after every epoch when a validation set is
        given, the seconds spent in the training calls alone (the upload of
        the data set and the validation passes excluded) and the steps run."""
        import torch

        rng = np.random.Generator(np.random.PCG64(seed))
        self.mu = Y.mean(axis=0)
        self.sd = Y.std(axis=0) + 1e-12
        self.net.set_data(X, ((Y - self.mu) / self.sd).astype(np.float32))
        n = X.shape[0]
        steps = n // batch
        hist, val, train_s = [], [], 0.0
        for ep in range(epochs):
            e_lr = lr * 0.5 * (1 + math.cos(math.pi * ep / epochs))
            idx = rng.permutation(n)[: steps * batch].reshape(steps, batch)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            losses = self.net.train(idx, lr=e_lr)  # returns after the last step
            train_s += time.perf_counter() - t0
            hist.append(float(np.mean(losses)))
            if X_val is not None:
                pz = (self.predict(X_val) - self.mu) / self.sd
                val.append(float(np.mean((pz - (Y_val - self.mu) / self.sd) ** 2)))
            if log:
                log(f"epoch {ep}: loss {hist[-1]:.4f}" + (f", held out {val[-1]:.4f}" if val else ""))
        return {"train_loss": hist, "val_loss": val, "train_s": train_s, "steps": steps * epochs}

    def predict(self, X):
        return self.net.predict(X).astype(np.float64) * self.sd + self.mu

    def close(self):
        self.net.close()


def spearman(a, b) -> float:
    ra = np.argsort(np.argsort(a)).astype(np.float64)
    rb = np.argsort(np.argsort(b)).astype(np.float64)
    return float(np.corrcoef(ra, rb)[0, 1])


def screen(model: Surrogate, Xe, Ye, batch_eval: dict, frac: float = 0.01, seed: int = 7):
    """Rank held-out robots by predicted x-displacement, re-simulate the top
    ``frac`` with the plain simulator, and score the choice against the
    simulated ground truth ``Ye``."""
    import torch

    from . import titan as T

    n = Xe.shape[0]
    k = max(1, int(round(frac * n)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = model.predict(Xe)
    t_pred = time.perf_counter() - t0
    top = np.argsort(-pred[:, 0], kind="stable")[:k]
    # the judge: re-simulate the chosen robots on their own, plain engine
    picked = subset(batch_eval, top)
    d, t_sim = simulate(picked, engine=T.ENGINE_TILED)
    true_top = np.argsort(-Ye[:, 0], kind="stable")[:k]
    rng = np.random.Generator(np.random.PCG64(seed))
    rand = rng.choice(n, k, replace=False)
    best = float(Ye[:, 0].max())
    return {
        "held_out": n, "picked": k,
        "recall_top": float(np.intersect1d(top, true_top).size / k),
        "recall_random_expected": k / n,
        "recall_random_draw": float(np.intersect1d(rand, true_top).size / k),
        "best_true_dx": best,
        "best_picked_dx": float(d[:, 0].max()),
        "regret": best - float(d[:, 0].max()),
        "regret_random": best - float(Ye[rand, 0].max()),
        "mean_picked_dx": float(d[:, 0].mean()), "mean_random_dx": float(Ye[rand, 0].mean()),
        "judge_matches_dataset": bool(np.allclose(d, Ye[top], rtol=0, atol=1e-6)),
        "spearman_dx": spearman(pred[:, 0], Ye[:, 0]),
        "mae_m": [float(v) for v in np.abs(pred - Ye).mean(axis=0)],
        "std_target_m": [float(v) for v in Ye.std(axis=0)],
        "predict_s": t_pred, "resimulate_s": t_sim,
    }


def subset(batch: dict, robots) -> dict:
    """The robots ``robots`` (indices) of a small_robot_batch, as a scene."""
    robots = np.asarray(robots)
    mp, sp = batch["mass_ptr"], batch["spring_ptr"]
    parts = []
    for r in robots:
        m0, m1, s0, s1 = mp[r], mp[r + 1], sp[r], sp[r + 1]
        parts.append(dict(pos=batch["pos"][m0:m1], vel=batch["vel"][m0:m1], mass=batch["mass"][m0:m1],
                          ends=batch["ends"][s0:s1] - m0, k=batch["k"][s0:s1], damping=batch["damping"][s0:s1],
                          amp=batch["amp"][s0:s1], phase=batch["phase"][s0:s1]))
    return scenes.concat(parts)


def main(argv=None):
    ap = argparse.ArgumentParser(description="train and evaluate the surrogate")
    ap.add_argument("--train", type=int, default=200000)
    ap.add_argument("--eval", type=int, default=20000)
    ap.add_argument("--train-seed", type=int, default=5)
    ap.add_argument("--eval-seed", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--chunk", type=int, default=16384)
    args = ap.parse_args(argv)

    import torch

    torch.cuda.set_device(0)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    Xt, Yt, gpu_t = dataset(args.train, args.train_seed, args.chunk, log)
    t_data = time.perf_counter() - t0
    eval_batch = scenes.small_robot_batch(args.eval, chunk_seed(args.eval_seed, 0))
    Ye, gpu_e = simulate(eval_batch)
    Xe = featurize(eval_batch)
    log(f"eval set simulated: {gpu_e:.3f} s")
    model = Surrogate(seed=3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fit = model.fit(Xt, Yt, args.epochs, args.batch, args.lr, log=log, X_val=Xe, Y_val=Ye)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t1
    hist = fit["train_loss"]
    t_train = fit["train_s"]
    flops = 3 * 2 * sum(DIMS[l] * DIMS[l + 1] for l in range(len(DIMS) - 1)) * args.batch * fit["steps"]
    res = screen(model, Xe, Ye, eval_batch)
    out = {
        "metric": "surrogate screening", "train_robots": args.train, "eval_robots": args.eval,
        "epochs": args.epochs, "batch": args.batch, "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
        "train_loss_per_epoch": hist, "held_out_loss_per_epoch": fit["val_loss"],
        "train_steps": fit["steps"], "train_s": t_train, "train_ms_per_step": t_train / fit["steps"] * 1e3,
        "train_tflops": flops / t_train / 1e12, "fit_s_incl_data_upload_and_validation": t_fit,
        "dataset_s": t_data, "dataset_gpu_step_s": gpu_t, "eval_simulate_all_s": gpu_e,
        "screen_s": res["predict_s"] + res["resimulate_s"],
        "screen_speedup_vs_simulate_all": gpu_e / (res["predict_s"] + res["resimulate_s"]),
        **res,
    }
    model.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()

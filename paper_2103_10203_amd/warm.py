"""Learned warm start: data generation with the library's own solver, training
with the library's network kernels, and warm-started batched solves.

The network maps features of a microstructure's adapted pattern (the phase
spectrum at the first `nslots` selected conjugate pairs, their frequencies,
the volume fraction) to the per-unit-macro-strain strain response at those
pairs, as a correction to the first-order (Born) term that the cold start's
first iteration produces; the warm start is prior plus correction contracted
with the RVE's macro strain.
Linear elasticity makes the converged response exactly linear in the macro
strain, so three unit-strain solves per training microstructure give complete
targets.  The prediction only seeds the fixed-point iteration, which still
runs to tolerance.
"""
from __future__ import annotations

import math
import time
from concurrent.futures import ProcessPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import _native as nat

UNIT = np.eye(3)


@dataclass
class WarmConfig:
    nslots: int = 256
    hidden: int = 512
    seed: int = 0
    epochs: int = 60
    batch: int = 512
    lr: float = 1e-3
    lr_final: float = 1e-4


def _gen_micro(args):
    import synth
    seed, n = args
    return synth.fibre_rve_256(seed, n).g


def generate_microstructures(seeds, n=256, workers=8):
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_gen_micro, [(s, n) for s in seeds], chunksize=16))


@dataclass
class TrainingSet:
    X: object                 # torch [n][4 S + 1]
    T: object                 # torch [n][18 S]
    solves: int = 0
    gen_s: dict = field(default_factory=dict)


def build_training_set(gs, M, phases, nslots, tol=1e-6, chunk=512, log=None):
    """Features and targets for microstructures `gs`: three unit-strain solves
    each (RVE order (b, k)), converged coefficients gathered to slot targets."""
    import torch
    Xs, Ts = [], []
    t_plan = t_solve = 0.0
    solves = 0
    for c0 in range(0, len(gs), chunk):
        part = gs[c0:c0 + chunk]
        t = time.perf_counter()
        plans = nat.make_plans(part, M)
        t_plan += time.perf_counter() - t
        nb = len(part)
        plan_of = np.repeat(np.arange(nb), 3)
        ebs = np.tile(UNIT, (nb, 1))
        t = time.perf_counter()
        out = nat.solve_multi(plans, plan_of, ebs, phases, tol, want_coeffs=True)
        torch.cuda.synchronize()
        t_solve += time.perf_counter() - t
        solves += 3 * nb
        po = np.arange(nb)
        Xs.append(nat.warm_features(plans, po, nslots))
        Ts.append(nat.warm_targets(plans, po, nslots, phases, out.coeffs))
        del plans
        if log:
            log(f"training set: {c0 + nb} of {len(gs)} microstructures solved")
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    return TrainingSet(X=X, T=T, solves=solves, gen_s={"plans": t_plan, "solves": t_solve})


def train(net: nat.MLP, data: TrainingSet, cfg: WarmConfig, log=None):
    """Mini-batch Adam on the MSE of the slot targets; cosine-decayed rate."""
    import torch
    n = data.X.shape[0]
    g = torch.Generator(device="cpu")
    g.manual_seed(cfg.seed)
    hist = []
    steps = cfg.epochs * math.ceil(n / cfg.batch)
    k = 0
    t0 = time.perf_counter()
    for ep in range(cfg.epochs):
        perm = torch.randperm(n, generator=g).to(data.X.device)
        tot = 0.0
        nb = 0
        for b0 in range(0, n, cfg.batch):
            idx = perm[b0:b0 + cfg.batch]
            xb = data.X.index_select(0, idx).contiguous()
            tb = data.T.index_select(0, idx).contiguous()
            lr = cfg.lr_final + 0.5 * (cfg.lr - cfg.lr_final) * (1 + math.cos(math.pi * k / max(steps, 1)))
            tot += net.grad(xb, tb)
            net.adam(lr)
            nb += 1
            k += 1
        hist.append(tot / nb)
        if log:
            log(f"epoch {ep} loss {hist[-1]:.4e}")
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def predict_warm(net: nat.MLP, plans, plan_of, macro, phases, nslots, precision=nat.MLP_BF16):
    X = nat.warm_features(plans, plan_of, nslots)
    Y = net.forward(X, precision)
    return nat.warm_apply(plans, plan_of, nslots, phases, Y, macro)


def born_warm(plans, plan_of, macro, phases, nslots):
    """The prior alone (zero network output): the cold start's first iterate."""
    import torch
    Y = torch.zeros((len(plan_of), 18 * nslots), dtype=torch.float32, device="cuda")
    return nat.warm_apply(plans, plan_of, nslots, phases, Y, macro)


def relative_error(net: nat.MLP, data: TrainingSet, precision=nat.MLP_FP32):
    """Relative L2 error of the prediction against the targets."""
    import torch
    Y = net.forward(data.X, precision)
    return float(torch.linalg.norm(Y - data.T) / torch.linalg.norm(data.T))

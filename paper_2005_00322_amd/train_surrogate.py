"""Train and evaluate the DCT-basis neural-operator surrogate on solver-generated pairs.

    python -m paper_2005_00322_amd.train_surrogate [--train 20000] [--test 2000] [--epochs 20]
        [--batch 64] [--lr 2e-3] [--save weights.npz] [--init weights.npz] [--time-budget SECONDS]

Inputs are the seeded 128 x 128 pairs of ``workloads.nop_inputs`` (1-3 Gaussian blobs, smooth c0 map in
[1400, 1600] m/s); targets are the pressure after ``workloads.NOP_STEPS`` steps of the FP32 batched PSTD
solver with the same c0 map (x faces Dirichlet, y faces Neumann).  Training runs the library's forward,
backward and Adam kernels; this module only schedules batches and the learning rate.  Prints one JSON
line with the held-out relative L2 errors against the solver.  ``--init`` starts from saved parameters (a
warm restart: fresh Adam moments and a new cosine schedule) instead of the seeded initialisation.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import sys
import time

import numpy as np


def _inputs_chunk(args):
    import workloads
    count, n, offset = args
    return workloads.nop_inputs(count, n=n, index_offset=offset)


def make_inputs(count, n=128, offset=0, workers=8):
    """(p0s, c0s) float32 arrays of shape (count, n, n), drawn in parallel host processes."""
    chunk = max(1, math.ceil(count / (4 * workers)))
    jobs = [(min(chunk, count - s), n, offset + s) for s in range(0, count, chunk)]
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_inputs_chunk, jobs))
    p = np.concatenate([a for a, _ in parts]).astype(np.float32)
    c = np.concatenate([b for _, b in parts]).astype(np.float32)
    return p, c


def targets(p0s, c0s, batch=256):
    import workloads
    from .surrogate import solver_targets
    return solver_targets(p0s, c0s, workloads.DX, workloads.NOP_DT, workloads.NOP_STEPS, workloads.NOP_BCS,
                          batch=batch)


def train(net, p, c, t, epochs, batch, lr, time_budget=None, log=sys.stderr, seed=0):
    """Adam with a cosine learning-rate schedule over `epochs` passes of shuffled batches."""
    import torch
    n = int(p.shape[0])
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    step = 0
    history = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(p.device)
        losses = []
        for i in range(steps_per_epoch):
            idx = perm[i * batch:(i + 1) * batch]
            net.forward(p[idx], c[idx])
            losses.append(net.backward(t[idx]))
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * step / max(1, total)))
            net.adam_step(max(cur, 1e-3 * lr))
            step += 1
        history.append(float(np.mean(losses)))
        print("epoch %d loss %.5f (%.1f s)" % (ep, history[-1], time.perf_counter() - t0), file=log, flush=True)
        if time_budget is not None and time.perf_counter() - t0 > time_budget:
            break
    torch.cuda.synchronize()
    return history, time.perf_counter() - t0, step


def evaluate(net, p, c, t, batch):
    import torch
    errs = []
    out = torch.empty_like(t[:batch])
    for s in range(0, int(p.shape[0]), batch):
        e = min(int(p.shape[0]), s + batch)
        o = net.infer(p[s:e], c[s:e], out=out[:e - s])
        errs.append(net.relative_errors(o, t[s:e]))
    return np.concatenate(errs)


def main(argv=None):
    import torch

    import workloads
    from .surrogate import Surrogate, SurrogateConfig, param_shapes

    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--test", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--time-budget", type=float, default=None)
    ap.add_argument("--save", default=None)
    ap.add_argument("--init", default=None, help="npz with 'theta' to start from")
    ap.add_argument("--workers", type=int, default=8)
    a = ap.parse_args(argv)
    # host inputs first, in child processes started before this process touches the GPU
    t0 = time.perf_counter()
    ptr, ctr = make_inputs(a.train, offset=0, workers=a.workers)
    pte, cte = make_inputs(a.test, offset=10 ** 6, workers=a.workers)
    t_inputs = time.perf_counter() - t0
    torch.cuda.set_device(0)
    print("inputs %.1f s" % t_inputs, file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    ttr = targets(ptr, ctr)
    tte = targets(pte, cte)
    torch.cuda.synchronize()
    t_targets = time.perf_counter() - t1
    print("targets %.1f s" % t_targets, file=sys.stderr, flush=True)
    dev = torch.device("cuda")
    ptr_d, ctr_d = torch.from_numpy(ptr).to(dev), torch.from_numpy(ctr).to(dev)
    pte_d, cte_d = torch.from_numpy(pte).to(dev), torch.from_numpy(cte).to(dev)
    cfg = SurrogateConfig()
    net = Surrogate(cfg, max_batch=a.batch)
    if a.init:
        with np.load(a.init) as z:
            net.set_params(np.asarray(z["theta"], dtype=np.float32))
    else:
        net.set_params(workloads.nop_init(param_shapes(cfg), seed=a.seed))
    hist, t_train, steps = train(net, ptr_d, ctr_d, ttr, a.epochs, a.batch, a.lr, a.time_budget, seed=a.seed)
    err = evaluate(net, pte_d, cte_d, tte, a.batch)
    theta = net.get_params()
    if a.save:
        np.savez_compressed(a.save, theta=theta, train=a.train, epochs=len(hist), batch=a.batch, lr=a.lr,
                            seed=a.seed, init=a.init or "")
    print(json.dumps({
        "train_pairs": a.train, "test_pairs": a.test, "epochs": len(hist), "steps": steps, "batch": a.batch,
        "lr": a.lr, "init": a.init, "loss_history": [round(x, 5) for x in hist], "train_s": round(t_train, 2),
        "targets_s": round(t_targets, 2), "inputs_s": round(t_inputs, 2),
        "heldout_rel_l2": {"mean": float(err.mean()), "median": float(np.median(err)),
                           "p95": float(np.quantile(err, 0.95)), "max": float(err.max())},
        "params": int(theta.size)}))
    net.close()


if __name__ == "__main__":
    main()

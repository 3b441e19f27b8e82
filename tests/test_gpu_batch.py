"""GPU parity of the batched persistent 2D solver against the FP64 oracle, solve by solve."""
import os

import numpy as np
import pytest

import workloads
from gpu_helpers import TOL, rel_l2
from oracle import pstd as opstd

pytestmark = pytest.mark.gpu
N, D = opstd.NEUMANN, opstd.DIRICHLET


def _random_solves(seed, count, lo, hi):
    rng = np.random.default_rng(seed)
    solves, p0s = [], []
    for _ in range(count):
        shape = tuple(int(v) for v in rng.integers(lo, hi + 1, size=2))
        faces = rng.integers(0, 2, size=4)
        c0 = float(rng.uniform(1400, 1600))
        solves.append({"shape": shape, "bcs": ((int(faces[0]), int(faces[1])), (int(faces[2]), int(faces[3]))),
                       "dx": 1e-4, "dt": 0.3e-4 / c0, "c0": c0})
        p0s.append(rng.standard_normal(shape))
    return solves, p0s


def _run(solves, p0s, steps, config=None, chunks=None):
    import torch
    from paper_2005_00322_amd import Batch
    with Batch(solves) as b:
        if config:
            b.set_config(**config)
        st = b.new_states(p0s)
        b.init_states(st)
        for n in (chunks or [steps]):
            b.step(st, n)
        b.synchronize()   # raises if a grid barrier timed out
        return [s.p.double().cpu().numpy() for s in st], [[u.double().cpu().numpy() for u in s.u] for s in st]


@pytest.mark.parametrize("seed,count,lo,hi", [(1, 5, 5, 40), (2, 7, 30, 140), (3, 3, 3, 12)])
def test_batch_matches_oracle(seed, count, lo, hi):
    solves, p0s = _random_solves(seed, count, lo, hi)
    print("batch", [s["shape"] for s in solves], flush=True)
    ps, us = _run(solves, p0s, 30)
    for s, p0, p, u in zip(solves, p0s, ps, us):
        prob = opstd.Problem(s["shape"], s["bcs"], s["dx"], s["dt"], s["c0"])
        po, uo = prob.run(p0, 30)
        assert rel_l2(p, po) < TOL["fp32"]
        for a in range(2):
            assert rel_l2(u[a], uo[a]) < TOL["fp32"]


@pytest.mark.parametrize("config", [{"blocks": 0, "order": 1}, {"blocks": 256, "order": 0},
                                    {"blocks": 0, "order": 0, "tile": 64}, {"blocks": 300, "order": 1, "tile": 64}])
def test_batch_configs_agree(config):
    solves, p0s = _random_solves(4, 6, 20, 100)
    a, _ = _run(solves, p0s, 20, config={"tile": config.get("tile", 32)})
    b, _ = _run(solves, p0s, 20, config=config)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)      # same tiles, same arithmetic: order and block count do not matter
    if config.get("tile", 32) != 32:
        # another tile edge sums in another order: equal to rounding
        c, _ = _run(solves, p0s, 20)
        for x, y in zip(b, c):
            assert np.max(np.abs(x - y)) <= 1e-6 * np.max(np.abs(y))


def test_batch_chunks_bitwise():
    solves, p0s = _random_solves(5, 4, 20, 70)
    a, _ = _run(solves, p0s, 23)
    b, _ = _run(solves, p0s, 23, chunks=[1, 10, 12])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_batch_combine_pairs():
    import torch
    from paper_2005_00322_amd import Batch
    rng = np.random.default_rng(11)
    solves, p0s, R, pairs = [], [], [], []
    for i in range(3):
        shape = tuple(int(v) for v in rng.integers(20, 70, size=2))
        c0 = float(rng.uniform(1400, 1600))
        g = workloads.gaussian(shape, 1e-4, (shape[0] * 0.5e-4, shape[1] * 0.5e-4), 4e-4)
        for bc in (D, N):
            solves.append({"shape": shape, "bcs": ((bc, bc), (bc, bc)), "dx": 1e-4, "dt": 0.3e-4 / c0, "c0": c0})
            p0s.append(g)
        pairs.append((2 * i, 2 * i + 1))
        R.append(float(rng.uniform(-1, 1)))
    with Batch(solves) as b:
        st = b.new_states(p0s)
        b.init_states(st)
        b.step(st, 40)
        outs = b.combine_R(st, pairs, R)
        b.synchronize()
        got = [o.double().cpu().numpy() for o in outs]
    for (d, n), r, g in zip(pairs, R, got):
        sd, sn = solves[d], solves[n]
        pd, _ = opstd.Problem(sd["shape"], sd["bcs"], 1e-4, sd["dt"], sd["c0"]).run(p0s[d], 40)
        pn, _ = opstd.Problem(sn["shape"], sn["bcs"], 1e-4, sn["dt"], sn["c0"]).run(p0s[n], 40)
        assert rel_l2(g, opstd.combine_R(pd, pn, r)) < TOL["fp32"]


def test_batch_autotune_cache(tmp_path):
    from paper_2005_00322_amd import Batch
    solves, p0s = _random_solves(6, 5, 30, 90)
    cache = os.path.join(str(tmp_path), "tune.json")
    with Batch(solves) as b:
        cfg = b.autotune(trial_steps=3, cache_path=cache)
        assert not cfg["from_cache"] and os.path.exists(cache)
        cfg2 = b.autotune(trial_steps=3, cache_path=cache)
        assert cfg2["from_cache"] and cfg2["blocks"] == cfg["blocks"] and cfg2["order"] == cfg["order"]
    a, _ = _run(solves, p0s, 15)
    c, _ = _run(solves, p0s, 15, config={"blocks": cfg["blocks"], "order": cfg["order"], "tile": cfg["tile"]})
    for x, y in zip(a, c):
        assert np.array_equal(x, y)


def test_batch_autotune_cache_keeps_tile(tmp_path):
    """A cached tile-16 (fused phase launch) choice is reused for a one-shape batch; an entry edited to tile
    16 for a batch of mixed shapes is ignored and the trials run again."""
    import json
    from paper_2005_00322_amd import Batch
    rng = np.random.default_rng(8)
    same = [{"shape": (64, 48), "bcs": ((int(a), int(b)), (int(c), int(d))), "dx": 1e-4, "dt": 0.3e-4 / 1500,
             "c0": 1500.0} for a, b, c, d in rng.integers(0, 2, size=(8, 4))]
    cache = os.path.join(str(tmp_path), "same.json")
    with Batch(same) as b:
        cfg = b.autotune(trial_steps=3, cache_path=cache)
        cfg2 = b.autotune(trial_steps=3, cache_path=cache)
    assert not cfg["from_cache"] and cfg2["from_cache"]
    assert (cfg2["blocks"], cfg2["order"], cfg2["tile"]) == (cfg["blocks"], cfg["order"], cfg["tile"])
    mixed, _ = _random_solves(9, 4, 30, 90)
    cache = os.path.join(str(tmp_path), "mixed.json")
    with Batch(mixed) as b:
        first = b.autotune(trial_steps=3, cache_path=cache)
        assert first["tile"] in (32, 64)
        entry = json.load(open(cache))
        entry["tile"] = 16
        json.dump(entry, open(cache, "w"))
        again = b.autotune(trial_steps=3, cache_path=cache)
    assert not again["from_cache"] and again["tile"] in (32, 64)


def test_batched_workload_full():
    """The 128-instance workload (paired all-Neumann / all-Dirichlet solves, sides 96..512, 1000 steps)
    against the oracle's closed form for every solve, and the combination for every instance."""
    import torch
    from paper_2005_00322_amd import Batch
    wl = workloads.batched()
    solves, p0s, pairs, R = [], [], [], []
    for i, inst in enumerate(wl["instances"]):
        for bc in (D, N):
            solves.append({"shape": inst.shape, "bcs": ((bc, bc), (bc, bc)), "dx": wl["dx"], "dt": inst.dt,
                           "c0": inst.c0})
            p0s.append(inst.p0)
        pairs.append((2 * i, 2 * i + 1))
        R.append(inst.R)
    steps = wl["steps"]
    with Batch(solves) as b:
        st = b.new_states(p0s)
        b.init_states(st)
        b.step(st, steps)
        outs = b.combine_R(st, pairs, R)
        b.synchronize()
        ps = [s.p.double().cpu().numpy() for s in st]
        comb = [o.double().cpu().numpy() for o in outs]
    worst = 0.0
    for i, inst in enumerate(wl["instances"]):
        refs = []
        for k, bc in enumerate((D, N)):
            prob = opstd.Problem(inst.shape, ((bc, bc), (bc, bc)), wl["dx"], inst.dt, inst.c0)
            ref = prob.modal_solution(inst.p0, steps)
            refs.append(ref)
            worst = max(worst, rel_l2(ps[2 * i + k], ref))
        worst = max(worst, rel_l2(comb[i], opstd.combine_R(refs[0], refs[1], inst.R)))
    print("batched workload worst rel L2", worst, flush=True)
    assert worst < TOL["fp32"]


def _uniform_solves(seed, count, shape):
    rng = np.random.default_rng(seed)
    solves, p0s = [], []
    for _ in range(count):
        faces = rng.integers(0, 2, size=4)
        c0 = float(rng.uniform(1400, 1600))
        solves.append({"shape": shape, "bcs": ((int(faces[0]), int(faces[1])), (int(faces[2]), int(faces[3]))),
                       "dx": 1e-4, "dt": 0.3e-4 / c0, "c0": c0})
        p0s.append(rng.standard_normal(shape))
    return solves, p0s


@pytest.mark.parametrize("seed,count,shape", [(11, 6, (40, 52)), (12, 3, (17, 9)), (13, 4, (300, 130))])
def test_phase_path_matches_oracle(seed, count, shape):
    """Tile 16: solves of one shape stepped by two fused phase launches per step."""
    solves, p0s = _uniform_solves(seed, count, shape)
    print("phase batch", shape, count, flush=True)
    ps, us = _run(solves, p0s, 30, config={"tile": 16})
    for s, p0, p, u in zip(solves, p0s, ps, us):
        prob = opstd.Problem(s["shape"], s["bcs"], s["dx"], s["dt"], s["c0"])
        po, uo = prob.run(p0, 30)
        assert rel_l2(p, po) < TOL["fp32"]
        for a in range(2):
            assert rel_l2(u[a], uo[a]) < TOL["fp32"]


def test_phase_path_sound_speed_maps():
    import torch
    from paper_2005_00322_amd import Batch
    rng = np.random.default_rng(21)
    shape, dx = (36, 44), 1e-4
    solves, p0s, maps = [], [], []
    for bc in (((1, 1), (0, 0)), ((0, 1), (1, 0)), ((0, 0), (0, 0))):
        cm = workloads.smooth_c0_map(rng, shape, corr_nodes=6.0)
        dt = 0.25 * dx / cm.max()
        solves.append({"shape": shape, "bcs": bc, "dx": dx, "dt": dt, "c0": float(cm.max())})
        p0s.append(workloads.gaussian(shape, dx, (shape[0] * dx / 2, shape[1] * dx / 2.5), 4 * dx))
        maps.append(cm)
    maps[2] = None                              # one homogeneous solve among them
    with Batch(solves) as b:
        b.set_c0_maps([None if m is None else torch.from_numpy(m.astype(np.float32)) for m in maps])
        b.set_config(tile=16)
        st = b.new_states(p0s)
        b.init_states(st)
        b.step(st, 80)
        b.synchronize()
        for i, (s, m) in enumerate(zip(solves, maps)):
            kw = {} if m is None else {"c0_map": m.astype(np.float32).astype(np.float64)}
            ref, _ = opstd.Problem(s["shape"], s["bcs"], dx, s["dt"], s["c0"], **kw).run(p0s[i], 80)
            assert rel_l2(st[i].p.double().cpu().numpy(), ref) < TOL["fp32"]


def test_phase_path_needs_one_shape():
    from paper_2005_00322_amd import Batch, PstdError
    solves, _ = _random_solves(14, 3, 20, 40)
    solves[1]["shape"] = (21, 33)
    with Batch(solves) as b:
        with pytest.raises(PstdError):
            b.set_config(tile=16)

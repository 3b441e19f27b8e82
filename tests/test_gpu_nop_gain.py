"""What the trained surrogate gains over the method without it.

The shipped network (weights/) against FP32 PSTD of the same 128 held-out inputs on coarser grids of the
same box (the accuracy-versus-cost knob of the convergence study, §4.2): inputs resampled spectrally onto
m x m nodes, the coarse solve over the same final time, its result evaluated back on the 128 x 128 nodes,
both measured against the fine FP32 solver.  The coarse error falls as the grid is refined; the cheapest
coarse grid whose 95th-percentile error is at or below the surrogate's takes longer than the surrogate's
inference of the same batch.
"""
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_surrogate_against_coarse_pstd():
    import torch

    from bench import coarse_pstd
    from paper_2005_00322_amd.surrogate import Surrogate, SurrogateConfig, solver_targets

    torch.cuda.set_device(0)
    cfg = SurrogateConfig()
    B = 128
    p0s, c0s = workloads.nop_inputs(B, n=cfg.H, index_offset=2 * 10 ** 6)
    p = torch.from_numpy(p0s.astype(np.float32)).cuda()
    c = torch.from_numpy(c0s.astype(np.float32)).cuda()
    ref = solver_targets(p, c, workloads.DX, workloads.NOP_DT, workloads.NOP_STEPS, workloads.NOP_BCS, batch=B)
    net = Surrogate(cfg, max_batch=B)
    net.set_params(np.load(os.path.join(ROOT, "paper_2005_00322_amd", "weights", "nop_128x128_c32_m48_l4.npz"))["theta"])
    out = torch.empty_like(p)
    for _ in range(3):
        net.infer(p, c, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(net._stream)
    for _ in range(5):
        net.infer(p, c, out=out)
    e1.record(net._stream)
    torch.cuda.synchronize()
    nop_ms = e0.elapsed_time(e1) / 5
    err = net.relative_errors(out, ref)
    net.close()
    p95 = float(np.quantile(err, 0.95))
    coarse = coarse_pstd(p, c, ref, cfg.H, sizes=(64, 40, 32))
    print("surrogate: %.2f ms, mean %.3f, p95 %.3f" % (nop_ms, err.mean(), p95), flush=True)
    for x in coarse:
        print("coarse %s: %.2f ms (+%.2f ms resampling), mean %.3f, p95 %.3f" % (
            x["grid"], x["solve_ms"], x["resample_ms"], x["rel_l2_vs_fp32_pstd"]["mean"],
            x["rel_l2_vs_fp32_pstd"]["p95"]), flush=True)
    p95s = [x["rel_l2_vs_fp32_pstd"]["p95"] for x in coarse]
    assert p95s[0] < p95s[1] < p95s[2]                   # refinement converges toward the fine solver
    assert p95s[0] < 0.2
    match = [x for x in coarse if x["rel_l2_vs_fp32_pstd"]["p95"] <= p95]
    assert match, "no coarse grid reaches the surrogate's error"
    cheapest = min(x["solve_ms"] + x["resample_ms"] for x in match)
    assert nop_ms < cheapest

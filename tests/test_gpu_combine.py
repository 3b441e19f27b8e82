"""GPU parity of the reflection-coefficient combination (§5) against the oracle."""
import numpy as np
import pytest

from gpu_helpers import rel_l2
from oracle import pstd as opstd

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("count", [0, 1, 5, 4099, 1 << 20])
@pytest.mark.parametrize("R", [-1.0, -0.3, 0.0, 0.77, 1.0])
def test_combine_R(count, R):
    import torch
    from paper_2005_00322_amd import combine_R
    rng = np.random.default_rng(count + 7)
    pd = rng.standard_normal(count).astype(np.float32)
    pn = rng.standard_normal(count).astype(np.float32)
    tD = torch.as_tensor(pd, device="cuda")
    tN = torch.as_tensor(pn, device="cuda")
    out = combine_R(tD, tN, R).cpu().numpy()
    ref = opstd.combine_R(pd, pn, R)
    if count:
        assert np.max(np.abs(out - ref)) <= 4e-7 * max(1.0, np.max(np.abs(ref)))
    # in place over the Neumann field, from an unaligned view
    if count > 8:
        tN2 = torch.as_tensor(pn, device="cuda")
        v = tN2[1:]
        combine_R(tD[1:], v, R, out=v)
        assert np.max(np.abs(v.cpu().numpy() - ref[1:])) <= 4e-7 * max(1.0, np.max(np.abs(ref)))


def test_combine_fields_four_basic_fields():
    import torch
    from paper_2005_00322_amd import combine_fields
    rng = np.random.default_rng(3)
    fields = [rng.standard_normal(10007).astype(np.float32) for _ in range(4)]
    w = opstd.combination_weights_1d(0.0, 0.5)
    out = combine_fields([torch.as_tensor(f, device="cuda") for f in fields], w).cpu().numpy()
    ref = sum(wi * f.astype(np.float64) for wi, f in zip(w, fields))
    assert rel_l2(out, ref) < 1e-7

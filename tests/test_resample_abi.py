"""Host-side checks of the collocated-derivative and interpolation tables (§3.3, §3.4) that the library
builds: equal to the oracle's matrices for every wall pair, argument errors."""
import numpy as np
import pytest

from oracle import pstd as o
from paper_2005_00322_amd import (GRAD_NODES, GRAD_STAG, NODES_TO_STAG, PERIODIC, STAG_TO_NODES, PstdError,
                                  axis_operator)

N, D = o.NEUMANN, o.DIRICHLET
KINDS = [GRAD_NODES, GRAD_STAG, NODES_TO_STAG, STAG_TO_NODES]


@pytest.mark.parametrize("which", KINDS)
@pytest.mark.parametrize("bcl,bcr", [(N, N), (N, D), (D, N), (D, D)])
@pytest.mark.parametrize("n", [3, 4, 5, 16, 17, 64, 129])
def test_tables_equal_oracle(which, bcl, bcr, n):
    dx = 0.013
    got = axis_operator(n, bcl, bcr, dx, which)
    want = o.Axis(n, bcl, bcr, dx).resample_matrix(which)
    assert got.shape == want.shape
    scale = np.max(np.abs(want))
    assert np.max(np.abs(got - want)) < 1e-12 * scale * n


def test_errors():
    with pytest.raises(PstdError):
        axis_operator(16, PERIODIC, PERIODIC, 1.0, GRAD_NODES)
    with pytest.raises(PstdError):
        axis_operator(16, N, N, 1.0, 6)

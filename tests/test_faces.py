"""Per-face reflection coefficients (§5 extended to every face, CPU only): the library's basic fields
and weights (pstd_face_weights) against the oracle's combination weights, formed independently, and
against the weights printed in §5."""
import json
import os

import numpy as np
import pytest

from oracle import pstd as opstd
from paper_2005_00322_amd import PstdError, face_weights

N, D = opstd.NEUMANN, opstd.DIRICHLET


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_weights_match_oracle(ndim, seed):
    rng = np.random.default_rng(100 + 10 * ndim + seed)
    R = [tuple(rng.uniform(-1.0, 1.0, 2)) for _ in range(ndim)]
    cases, w = face_weights(R)
    ref = opstd.combination_weights(R)
    assert len(cases) == 4 ** ndim == len(ref)
    assert len(set(cases)) == len(cases)
    for cs, wi in zip(cases, w):
        assert abs(wi - ref[cs]) < 1e-15
    assert abs(w.sum() - 1.0) < 1e-14    # a uniform field is reproduced: the weights sum to one


def test_printed_weights(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "combination.json")))
    for c in g["cases"]:
        cases, w = face_weights([(c["RL"], c["RR"])])
        assert cases == [((N, N),), ((N, D),), ((D, N),), ((D, D),)]
        assert np.allclose(w, np.array(c["w_num"], float) / c["w_den"], atol=1e-15)


@pytest.mark.parametrize("walls", [(N, N, D, N), (D, D, N, D), (N, D, D, D)])
def test_basic_walls_select_their_field(walls):
    R = [(1.0 if walls[0] == N else -1.0, 1.0 if walls[1] == N else -1.0),
         (1.0 if walls[2] == N else -1.0, 1.0 if walls[3] == N else -1.0)]
    cases, w = face_weights(R)
    own = cases.index(((walls[0], walls[1]), (walls[2], walls[3])))
    assert w[own] == 1.0 and np.count_nonzero(w) == 1


def test_separable_product():
    R = [(0.3, -0.7), (0.0, 0.5)]
    _, w = face_weights(R)
    _, wx = face_weights([R[0]])
    _, wy = face_weights([R[1]])
    assert np.allclose(w.reshape(4, 4), np.outer(wx, wy), atol=1e-16)


def test_argument_errors():
    with pytest.raises(PstdError):
        face_weights([])
    with pytest.raises(PstdError):
        face_weights([(0.0, 0.0)] * 4)
    with pytest.raises(PstdError):
        face_weights([(float("nan"), 0.0)])

"""Pins of the reflection-coefficient combination (§5, CPU only).

* The image matrix and the two worked weight vectors printed in §5 (golden fixture); M/2 is unitary.
* Each basic boundary pair selects its own field.
* Non-reflecting walls (R_L = R_R = 0): the weighted sum of the four basic 1D fields equals the
  free-space solution (no images) until T = 3L/c0, and is zero to rounding once the pulse has left.
* (R_L, R_R) = (0, 0.5): the sum equals the image solution with amplitudes r up to T = 2L/c0.
* 2D, a different partial R on each face: the 16 weighted basic fields equal the image solution in
  which each image carries the product of its per-face reflection factors.
* The two-field op p_R = (1+R)/2 p_N + (1-R)/2 p_D equals the four-field result until doubly reflected
  arrivals and differs after them.
"""
import json
import os

import numpy as np
import pytest

from oracle import images, pstd

N, D = pstd.NEUMANN, pstd.DIRICHLET


def test_printed_weights(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "combination.json")))
    assert np.array_equal(pstd.IMAGE_MATRIX, np.array(g["M"], dtype=float))
    half = pstd.IMAGE_MATRIX / 2
    assert np.allclose(half.T @ half, np.eye(4))
    for c in g["cases"]:
        w = pstd.combination_weights_1d(c["RL"], c["RR"])
        assert np.allclose(w, np.array(c["w_num"], float) / c["w_den"], atol=1e-15)


@pytest.mark.parametrize("i,case", list(enumerate(pstd.BASIC_CASES)))
def test_basic_cases_select_their_field(i, case):
    R = [1.0 if b == N else -1.0 for b in case]
    w = pstd.combination_weights_1d(*R)
    assert np.allclose(w, np.eye(4)[i])
    wd = pstd.combination_weights([tuple(R), tuple(R)])
    assert abs(wd[(case, case)] - 1.0) < 1e-15 and abs(sum(wd.values()) - 1.0) < 1e-15


def _four_fields(n, dx, c0, dt, m, p0):
    out = []
    for case in pstd.BASIC_CASES:
        prob = pstd.Problem((n,), (case,), dx, dt, c0)
        out.append(prob.modal_solution(p0, m))
    return out


def _free_space_1d(n, dx, c0, dt, m, xs, sigma):
    r = np.abs(np.arange(n) * dx - xs)
    return images.free_space_gaussian(r, 1, 1.0, sigma, c0, dt, m)


def test_non_reflecting_matches_free_space():
    n, dx, c0 = 257, 1e-4, 1500.0
    L = (n - 1) * dx
    dt = 0.2 * dx / c0
    xs, sigma = 0.3 * L, 4 * dx
    x = np.arange(n) * dx
    p0 = np.exp(-0.5 * (x - xs) ** 2 / sigma ** 2)
    w = pstd.combination_weights_1d(0.0, 0.0)
    for frac in (0.5, 1.2, 2.0, 2.9):
        m = int(round(frac * L / (c0 * dt)))
        fields = _four_fields(n, dx, c0, dt, m, p0)
        comb = sum(wi * f for wi, f in zip(w, fields))
        ref = _free_space_1d(n, dx, c0, dt, m, xs, sigma)
        assert np.max(np.abs(comb - ref)) < 1e-11
        if frac >= 1.2:                         # both halves have left the box
            assert np.max(np.abs(comb)) < 1e-11


def test_partial_reflection_matches_images():
    n, dx, c0 = 201, 1e-4, 1500.0
    L = (n - 1) * dx
    dt = 0.2 * dx / c0
    xs, sigma = 0.4 * L, 4 * dx
    RL, RR = 0.0, 0.5
    x = np.arange(n) * dx
    p0 = np.exp(-0.5 * (x - xs) ** 2 / sigma ** 2)
    w = pstd.combination_weights_1d(RL, RR)
    m = int(round(1.5 * L / (c0 * dt)))
    fields = _four_fields(n, dx, c0, dt, m, p0)
    comb = sum(wi * f for wi, f in zip(w, fields))
    # within one period: source, left image (R_L), right image (R_R), double image (R_L R_R)
    ref = np.zeros(n)
    for pos, amp in ((xs, 1.0), (-xs, RL), (2 * L - xs, RR), (2 * L + xs, RL * RR), (xs - 2 * L, RL * RR)):
        ref += amp * images.free_space_gaussian(np.abs(x - pos), 1, 1.0, sigma, c0, dt, m)
    assert np.max(np.abs(comb - ref)) < 1e-11


def test_two_field_combination_window():
    n, dx, c0 = 257, 1e-4, 1500.0
    L = (n - 1) * dx
    dt = 0.2 * dx / c0
    xs, sigma, R = 0.3 * L, 4 * dx, 0.5
    x = np.arange(n) * dx
    p0 = np.exp(-0.5 * (x - xs) ** 2 / sigma ** 2)
    w4 = pstd.combination_weights_1d(R, R)
    for frac, same in ((0.9, True), (1.6, False)):
        m = int(round(frac * L / (c0 * dt)))
        fields = _four_fields(n, dx, c0, dt, m, p0)
        four = sum(wi * f for wi, f in zip(w4, fields))
        two = pstd.combine_R(fields[3], fields[0], R)
        diff = np.max(np.abs(two - four))
        if same:
            assert diff < 1e-12
        else:
            assert diff > 1e-2
    # R = +1 / -1 reproduce the basic fields exactly
    assert np.array_equal(pstd.combine_R(fields[3], fields[0], 1.0), fields[0])
    assert np.array_equal(pstd.combine_R(fields[3], fields[0], -1.0), fields[3])


def test_partial_images_reduce_to_basic_walls():
    """R = +-1 on both walls: the partial-reflection image series is the basic walls' series."""
    L, xs, reach = 1.0, 0.37, 5.0
    for bl, br in pstd.BASIC_CASES:
        RL, RR = (1.0 if bl == N else -1.0), (1.0 if br == N else -1.0)
        a = sorted(images.image_positions_1d(xs, L, bl, br, reach))
        b = sorted(images.partial_image_positions_1d(xs, L, RL, RR, reach))
        assert len(a) == len(b)
        for (pa, sa), (pb, sb) in zip(a, b):
            assert abs(pa - pb) < 1e-14 and sa == sb


def _mixed_faces_case():
    shape, dx, c0 = (57, 69), 1e-4, 1500.0
    dt = 0.2 * dx / c0
    L = [(n - 1) * dx for n in shape]
    centre, sigma = (0.45 * L[0], 0.5 * L[1]), 3 * dx
    x = [np.arange(n) * dx for n in shape]
    X, Y = np.meshgrid(*x, indexing="ij")
    p0 = np.exp(-0.5 * ((X - centre[0]) ** 2 + (Y - centre[1]) ** 2) / sigma ** 2)
    m = int(round(1.9 * min(L) / (c0 * dt)))        # doubly reflected images inside, before 2 L_min / c0
    return shape, dx, c0, dt, centre, sigma, p0, m


def _weighted_fields(shape, dx, c0, dt, p0, m, weights):
    out = np.zeros(shape)
    for cases, w in weights.items():
        if w != 0.0:
            out += w * pstd.Problem(shape, cases, dx, dt, c0).modal_solution(p0, m)
    return out


def test_mixed_partial_faces_2d_match_images():
    """A different real R on each face of a 2D box: the 16 weighted basic-wall fields (§5, extended to
    d dimensions by separable images) equal the physical image solution in which every image carries
    the product of its per-face reflection factors, while no wave has met one pair of walls twice.

    The weights come from ``combination_weights`` and the reference from ``partial_image_solution``,
    which forms no weight at all.  The doubly reflected images have entered the box, so planted errors
    in the weights (axes exchanged, left and right exchanged, the R_L R_R term dropped or of the wrong
    sign) each move the weighted sum by 2e-2 or more, against 1e-14 agreement."""
    R = [(0.0, 0.5), (-0.3, 0.8)]
    shape, dx, c0, dt, centre, sigma, p0, m = _mixed_faces_case()
    comb = _weighted_fields(shape, dx, c0, dt, p0, m, pstd.combination_weights(R))
    ref = images.partial_image_solution(shape, R, dx, c0, dt, m, centre, 1.0, sigma)
    assert np.max(np.abs(ref)) > 0.02
    assert np.max(np.abs(comb - ref)) < 1e-9
    # the reference tells the faces apart: swapped axes or mirrored walls are far from it
    for other in ([R[1], R[0]], [R[0][::-1], R[1]], [R[0], R[1][::-1]]):
        alt = images.partial_image_solution(shape, other, dx, c0, dt, m, centre, 1.0, sigma)
        assert np.max(np.abs(alt - ref)) > 1e-2

"""Pins of the oracle's sampled-Fisher-row interpolation and fiducial iteration
(the Fisher matrix's smoothness and near translation invariance, sec. 3.1; the iterated
fiducial spectrum, sec. 2.3 after eq. pilin), against values fixed by hand or by closed
forms rather than by re-running the same code."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1810_00503_amd import workloads as WL


def _toeplitz(nb, f):
    return np.array([[f(l - l2) for l2 in range(nb)] for l in range(nb)], np.float64)


def test_all_columns_sampled_is_the_symmetrised_response():
    rng = np.random.default_rng(3)
    Fr = rng.normal(size=(7, 7))
    got = O.fisher_from_columns(Fr, list(range(7)), 7)
    np.testing.assert_array_equal(got, 0.5 * (Fr + Fr.T))


@pytest.mark.parametrize("rows", [[0, 11], [0, 4, 7, 11], [0, 1, 2, 9, 11], [0, 5, 6, 11]])
def test_toeplitz_response_is_reproduced_exactly(rows):
    """A response that depends only on the diagonal offset (asymmetric on purpose) is
    reproduced exactly from any columns that include both end bands: every missing
    column reads the same diagonal values from its neighbours."""
    nb = 12
    Fr = _toeplitz(nb, lambda d: math.exp(-abs(d) / 2.5) * (1.0 + 0.1 * d))
    got = O.fisher_from_columns(Fr[:, rows], rows, nb)
    np.testing.assert_allclose(got, 0.5 * (Fr + Fr.T), rtol=0, atol=1e-15)


def test_block_toeplitz_with_two_groups():
    """Two groups (E bands 0-5, B bands 6-11): each block depends only on the offset of the
    positions inside the groups; reproduced exactly from the end bands plus one more each."""
    nb, h = 12, 6
    fs = {(0, 0): lambda d: 2.0 * math.exp(-abs(d)), (1, 1): lambda d: 1.0 / (1.0 + d * d),
          (0, 1): lambda d: 0.3 * math.exp(-abs(d - 1)), (1, 0): lambda d: 0.2 * math.exp(-abs(d + 1))}
    Fr = np.zeros((nb, nb))
    for l in range(nb):
        for l2 in range(nb):
            Fr[l, l2] = fs[(l // h, l2 // h)]((l % h) - (l2 % h))
    groups = [0] * h + [1] * h
    rows = [0, 2, 5, 6, 9, 11]
    got = O.fisher_from_columns(Fr[:, rows], rows, nb, groups)
    np.testing.assert_allclose(got, 0.5 * (Fr + Fr.T), rtol=0, atol=1e-15)


def test_interpolation_weights_by_hand():
    """Five bands, columns 0 and 4 simulated: the diagonal of column l2 is
    Fr[0,0] + (Fr[4,4] - Fr[0,0]) l2 / 4, off-diagonal entries read the one neighbour
    whose shifted row stays inside the group."""
    Fr = np.zeros((5, 5))
    Fr[:, 0] = [1.0, 0.5, 0.25, 0.125, 0.0625]
    Fr[:, 4] = [0.03, 0.06, 0.12, 0.6, 5.0]
    got = O.fisher_from_columns(Fr[:, [0, 4]], [0, 4], 5)
    R = np.zeros((5, 5))
    R[:, 0] = Fr[:, 0]
    R[:, 4] = Fr[:, 4]
    # column 1: row l reads Fr[l-1, 0] (a = 0) and Fr[l+3, 4] (b = 4), weight 1/4 on b.
    # row 0: a-row -1 is outside, b-row 3 -> 0.6; row 1: both (1.0, 5.0) -> 2.0;
    # rows 2..4: b-rows 5..7 outside -> a-rows 1..3
    R[:, 1] = [0.6, 1.0 + 0.25 * (5.0 - 1.0), 0.5, 0.25, 0.125]
    # column 2: rows 0, 1: a-rows -2, -1 outside -> b-rows 2, 3; row 2: both -> 3.0;
    # rows 3, 4: b-rows outside -> a-rows 1, 2
    R[:, 2] = [0.12, 0.6, 1.0 + 0.5 * 4.0, 0.5, 0.25]
    # column 3: rows 0..2: a-rows -3..-1 outside -> b-rows 1..3; row 3: both -> 4.0;
    # row 4: a-row 1
    R[:, 3] = [0.06, 0.12, 0.6, 1.0 + 0.75 * 4.0, 0.5]
    np.testing.assert_allclose(got, 0.5 * (R + R.T), rtol=0, atol=1e-15)


def test_extrapolation_clamps_into_the_group():
    """Beyond the last simulated column the one neighbour is used; a shifted row that
    leaves the group is clamped to the group's edge."""
    Fr = np.zeros((4, 4))
    Fr[:, 0] = [4.0, 3.0, 2.0, 1.0]
    Fr[:, 2] = [7.0, 8.0, 9.0, 10.0]
    got = O.fisher_from_columns(Fr[:, [0, 2]], [0, 2], 4)
    R = np.zeros((4, 4))
    R[:, 0] = Fr[:, 0]
    R[:, 2] = Fr[:, 2]
    R[:, 1] = [8.0, 4.0 + 0.5 * 5.0, 3.0 + 0.5 * 7.0, 2.0]   # a = 0, b = 2: rows l - 1 and l + 1
    R[:, 3] = [7.0, 7.0, 8.0, 9.0]                  # a = 2 only: rows -1 (clamped to 0), 0, 1, 2
    np.testing.assert_allclose(got, 0.5 * (R + R.T), rtol=0, atol=1e-15)


def test_group_without_simulated_column_is_an_error():
    with pytest.raises(ValueError):
        O.fisher_from_columns(np.zeros((4, 1)), [0], 4, [0, 0, 1, 1])


def test_fiducial_iteration_homogeneous_expected_moments_converge_in_one_step():
    """Unmasked homogeneous noise with the expected E (closed forms): the Newton step of
    a linear prior lands on Theta_true from any fiducial, so the iteration stops after
    the second estimate with Theta_true."""
    n = 16
    pshape = WL.density_pshape(n, kd=n / 3.0)
    band = WL.log_band_map(n, 3)[None].astype(np.int32)
    nb, sigma2 = 3, 0.7
    theta_true = np.array([0.6, 1.3, 0.9])

    def est(th):
        mean, b, F = O.homogeneous_band_moments(pshape, band, th, theta_true, nb, sigma2)
        return O.newton_update(th, F, mean, b)

    th, hist = O.fiducial_iteration(est, np.array([0.1, 3.0, 0.5]), 10, 1e-12, 0.01)
    assert len(hist) == 3
    np.testing.assert_allclose(hist[1], theta_true, rtol=1e-12)
    np.testing.assert_allclose(th, theta_true, rtol=1e-12)


def test_fiducial_iteration_contraction_history():
    """estimate(T) = T* + (T - T*)/2: the fiducials follow T* + 2^-t (T0 - T*) and the loop
    stops at the first relative change below the tolerance."""
    ts = np.array([1.0, 2.0])
    t0 = np.array([3.0, 1.0])
    th, hist = O.fiducial_iteration(lambda t: ts + 0.5 * (t - ts), t0, 50, 1e-3, 0.01)
    for t, h in enumerate(hist):
        np.testing.assert_allclose(h, ts + 0.5 ** t * (t0 - ts), rtol=1e-14)
    rel = [np.max(np.abs(hist[t] - hist[t - 1]) / hist[t - 1]) for t in range(1, len(hist))]
    assert rel[-1] <= 1e-3 and all(r > 1e-3 for r in rel[:-1])


def test_fiducial_iteration_floor():
    """Negative estimates are held at floor times the previous fiducial."""
    t0 = np.array([2.0, 0.5])
    th, hist = O.fiducial_iteration(lambda t: -t, t0, 3, 0.0, 0.1)
    np.testing.assert_allclose(np.array(hist), [t0, 0.1 * t0, 0.01 * t0, 0.001 * t0], rtol=1e-15)
    np.testing.assert_allclose(th, -0.01 * t0, rtol=1e-15)


def test_scaled_toeplitz_is_reproduced_exactly_with_its_scale():
    """Fr = diag(sqrt D) T diag(sqrt D) with T depending only on the diagonal offset (a
    correlation-like response whose diagonal spans orders of magnitude) is reproduced
    exactly when the interpolation works in units of D."""
    nb = 10
    T = _toeplitz(nb, lambda d: math.exp(-abs(d) / 1.5) * (1.0 - 0.05 * d))
    D = np.geomspace(1e3, 1e-6, nb)
    sq = np.sqrt(D)
    Fr = sq[:, None] * T * sq[None, :]
    rows = [0, 3, 4, 9]
    got = O.fisher_from_columns(Fr[:, rows], rows, nb, None, D)
    want = 0.5 * (Fr + Fr.T)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)
    # without the scale the interpolation of such a matrix is far off
    raw = O.fisher_from_columns(Fr[:, rows], rows, nb)
    assert np.abs(raw - want).max() > 1e-3 * np.abs(want).max()


def test_fisher_scale_is_the_sample_variance():
    Es = np.array([[1.0, 2.0, 5.0], [3.0, 2.0, 1.0], [2.0, 2.0, 3.0]])
    np.testing.assert_allclose(O.fisher_scale(Es), [1.0, 1.0, 4.0], rtol=1e-15)
    np.testing.assert_array_equal(O.fisher_scale(Es[:1]), np.ones(3))

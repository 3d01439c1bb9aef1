"""Planted mistakes: each test plants one plausible error in an oracle function (on the CPU,
through monkeypatch, for the duration of the test) and checks that a pin of that function
fails.  This is evidence that the pins constrain the oracle: a dropped term, a wrong sign, a
missing factor or a conjugated transform anywhere in it is caught by a check that does not
use the oracle's own formula.

Only the oracle is modified, and only inside these tests; nothing here touches the GPU."""
import numpy as np
import pytest

import oracle as O
import oracle.philox as OP
import oracle.wf_oracle as OW
from tests import test_oracle_catalog as TC
from tests import test_oracle_estimator_pins as TE
from tests import test_oracle_fisher_rows as TF
from tests import test_oracle_leakage as TL
from tests import test_oracle_posterior as TP
from tests import test_oracle_solver as TS
from tests import test_oracle_transforms as TT


def _plant(monkeypatch, name, fn, module=OW):
    """Replace oracle function `name` (the package attribute and the module global that the
    oracle's own functions call)."""
    monkeypatch.setattr(module, name, fn)
    if hasattr(O, name):
        monkeypatch.setattr(O, name, fn)


def _free_prior_term(s, S):
    """4 S^-1 s on the free entries (the prior's part of the stored-coefficient gradient)."""
    fr = O.free_mask(S.shape[1])[None] & (S > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(fr, 4.0 * np.where(fr, s, 0) / np.where(fr, S, 1.0), 0)


def _m_forward_b_sign(orig):
    # spin-2: the B coefficient enters the rotation with the wrong sign
    return lambda s, free=None: orig(np.stack([s[0], -s[1]]) if s.shape[0] == 2 else s, free)


def _m_forward_norm(orig):
    # the inverse DFT without its 1/n
    return lambda s, free=None: orig(s, free) * s.shape[1]


def _m_adjoint_b_sign(orig):
    # the adjoint rotates B the wrong way (forward unchanged)
    def f(x):
        a = orig(x)
        return np.stack([a[0], -a[1]]) if a.shape[0] == 2 else a
    return f


def _m_adjoint_conj(orig):
    # forward DFT with the exponent's sign flipped
    return lambda x: np.conj(orig(x))


def _m_grad_no_prior(orig):
    return lambda s, d, W, S: orig(s, d, W, S) - _free_prior_term(s, S)


def _m_grad_data_sign(orig):
    def f(s, d, W, S):
        p = _free_prior_term(s, S)
        return p - (orig(s, d, W, S) - p)
    return f


def _m_chi2_half_prior(orig):
    # the prior summed over the stored half plane only (each mode once instead of with its mirror)
    return lambda s, d, W, S: orig(s, d, W, S) - 0.5 * orig(s, d, 0.0 * W, S)


def _m_hvp_no_identity(orig):
    def f(p, W, S):
        fr = O.free_mask(S.shape[1])[None] & (S > 0)
        return orig(p, W, S) - np.where(fr, p, 0)
    return f


def _m_band_E_double(orig):
    return lambda *a, **k: 2.0 * orig(*a, **k)


def _m_wiener_variance(orig):
    # the noise variance in place of its inverse
    def f(d, W, S):
        with np.errstate(divide="ignore"):
            return orig(d, np.where(W > 0, 1.0 / np.where(W > 0, W, 1.0), 0.0), S)
    return f


def _m_lbfgs_early(orig):
    def f(d, W, S, *a, **k):
        k["tol"] = 1e-3
        return orig(d, W, S, *a, **k)
    return f


def _m_simulate_no_noise(orig):
    return lambda draw, S_true, W: OW.sim_signal(draw, S_true)


def _m_newton_sign(orig):
    return lambda th, F, E, b: 2.0 * np.asarray(th, np.float64) - orig(th, F, E, b)


def _m_dense_fisher_diag(orig):
    def f(*a, **k):
        b, F = orig(*a, **k)
        return b, np.diag(np.diag(F))
    return f


def _m_sim_fisher_half(orig):
    def f(*a, **k):
        out = orig(*a, **k)
        return (out[0], 0.5 * out[1]) + tuple(out[2:])
    return f


def _m_catalog_phase(orig):
    # the plane waves evaluated with the opposite phase (at -r)
    def f(s, pos, free=None):
        n = s.shape[1]
        return orig(s, np.mod(-np.asarray(pos, np.float64), n), free)
    return f


def _m_lbfgs_no_history(orig):
    # the curvature pairs are never kept (steepest descent with exact steps)
    def f(d, W, S, *a, **k):
        k["m"] = 0
        return orig(d, W, S, *a, **k)
    return f


def _m_dot_real_parts(orig):
    # the solver's inner product over the real parts only
    return lambda a, b: float(np.sum(a.real * b.real))


def _m_catalog_adjoint_b_sign(orig):
    # the catalog adjoint rotates B the wrong way
    def f(r, pos, n):
        a = orig(r, pos, n)
        return np.stack([a[0], -a[1]]) if a.shape[0] == 2 else a
    return f


def _m_dtheta_one_power(orig):
    # d chi^2 / d Theta_b with 1 / Theta_b where the prior term gives 1 / Theta_b^2
    return lambda s, pshape, band, theta, nbands: orig(s, pshape, band, theta, nbands) * np.asarray(theta)


def _m_posterior_half(orig):
    # the simulation variance of one coordinate only (real part) per stored entry
    def f(*a, **k):
        vm, vp = orig(*a, **k)
        return 0.5 * vm, vp
    return f


def _m_dense_posterior_half(orig):
    def f(W, S):
        vm, vp = orig(W, S)
        return 0.5 * vm, vp
    return f


def _m_fisher_scale_ignored(orig):
    # the sample-variance scale of the response dropped
    return lambda Fcols, rows, nbands, groups=None, scale=None: orig(Fcols, rows, nbands, groups, None)


def _m_fiducial_no_floor(orig):
    return lambda estimate, theta0, max_iter, rel_tol, floor: orig(estimate, theta0, max_iter, rel_tol, 0.0)


def _m_leakage_fisher_half(orig):
    def f(*a, **k):
        th, EB, bB, FBB = orig(*a, **k)
        return th, EB, bB, 0.5 * FBB
    return f


def _m_cosmic_variance_one_mode(orig):
    # sqrt(1 / N_l): each free entry counted once instead of with its mirror
    return lambda S, band, nbands: orig(S, band, nbands) / np.sqrt(2.0)


def _m_sim_signal_full_variance(orig):
    # each of the real and imaginary parts drawn with variance S instead of S / 2
    return lambda draw, S_true: np.sqrt(2.0) * orig(draw, S_true)


def _m_philox_bit(orig):
    def f(*a, **k):
        r = np.array(orig(*a, **k), dtype=np.uint64, copy=True)
        r.flat[0] ^= 1
        return r.astype(np.uint32)
    return f


CASES = [
    ("spin-2 B sign in R", "forward", _m_forward_b_sign, lambda: TT.test_spin2_matches_plane_wave_derivatives(16)),
    ("1/n missing in R", "forward", _m_forward_norm, lambda: TT.test_forward_is_bruteforce_inverse_dft(4)),
    ("B sign in R^T", "adjoint", _m_adjoint_b_sign, lambda: TT.test_adjoint_dot_product_and_parseval(8, 2)),
    ("conjugated R^T", "adjoint", _m_adjoint_conj, lambda: TT.test_adjoint_is_bruteforce_forward_dft(4)),
    ("prior term dropped from the gradient", "grad_chi2", _m_grad_no_prior,
     lambda: TT.test_gradient_equals_central_differences(1)),
    ("data term of the gradient with the wrong sign", "grad_chi2", _m_grad_data_sign,
     lambda: TT.test_gradient_equals_central_differences(2)),
    ("prior of chi^2 over the half plane", "chi2", _m_chi2_half_prior,
     lambda: TT.test_gradient_equals_central_differences(1)),
    ("identity dropped from the curvature", "whitened_hvp", _m_hvp_no_identity,
     lambda: TT.test_whitened_curvature_is_gradient_difference(1)),
    ("factor 1/2 missing in E_b", "band_E", _m_band_E_double, lambda: TS.test_band_E_is_minus_half_theta_derivative(1)),
    ("noise variance for its inverse in the dense Wiener filter", "wiener_dense", _m_wiener_variance,
     lambda: TS.test_map_equals_dense_wiener_filter(1, 12)),
    ("L-BFGS stopped at 1e-3", "lbfgs_solve", _m_lbfgs_early, lambda: TS.test_map_equals_dense_wiener_filter(2, 12)),
    ("L-BFGS history never kept", "lbfgs_solve", _m_lbfgs_no_history,
     lambda: TS.test_lbfgs_iterates_equal_conjugate_gradients(1, 10, False)),
    ("solver dot products over real parts only", "_dot", _m_dot_real_parts,
     lambda: TS.test_lbfgs_iterates_equal_conjugate_gradients(2, 3, False)),
    ("simulation without noise", "simulate", _m_simulate_no_noise,
     lambda: TS.test_simulation_matches_prior_and_noise_statistics()),
    ("Newton step with the wrong sign", "newton_update", _m_newton_sign, lambda: TS.test_bandpower_estimate_unbiased()),
    ("off-diagonal Fisher couplings dropped", "dense_bias_fisher", _m_dense_fisher_diag,
     lambda: TE.test_dense_bias_fisher_are_lndet_derivatives(1, 12, 3)),
    ("simulation Fisher matrix halved", "sim_fisher", _m_sim_fisher_half,
     lambda: TS.test_sim_bias_and_fisher_converge_to_closed_forms()),
    ("catalog plane waves with the opposite phase", "catalog_forward", _m_catalog_phase,
     lambda: TC.test_integer_positions_reduce_to_the_map_response(1)),
    ("catalog adjoint's B rotation with the wrong sign", "catalog_adjoint", _m_catalog_adjoint_b_sign,
     lambda: TC.test_catalog_adjoint_dot_product(2)),
    ("d chi^2 / d theta with one power of theta", "dchi2_dtheta", _m_dtheta_one_power,
     lambda: TE.test_dchi2_dtheta_central_differences(1)),
    ("posterior variance of one coordinate", "posterior_error", _m_posterior_half,
     lambda: TP.test_posterior_error_simulations_match_dense_diagonal()),
    ("dense posterior variance of one coordinate", "dense_posterior_variance", _m_dense_posterior_half,
     lambda: TP.test_dense_posterior_variance_homogeneous_closed_form()),
    ("Fisher rows' sample-variance scale dropped", "fisher_from_columns", _m_fisher_scale_ignored,
     lambda: TF.test_scaled_toeplitz_is_reproduced_exactly_with_its_scale()),
    ("fiducial iteration without its floor", "fiducial_iteration", _m_fiducial_no_floor,
     lambda: TF.test_fiducial_iteration_floor()),
    ("B-mode leakage Fisher halved", "bmode_leakage_qe", _m_leakage_fisher_half,
     lambda: TL.test_unmasked_leakage_bias_is_the_noise_only_mean()),
    ("cosmic variance counting each mode once", "cosmic_variance", _m_cosmic_variance_one_mode,
     lambda: TP.test_cosmic_variance_counts_modes()),
    ("simulated signal with twice the variance", "sim_signal", _m_sim_signal_full_variance,
     lambda: TP.test_sim_signal_has_the_prior_variance()),
]


@pytest.mark.filterwarnings("ignore::RuntimeWarning")   # a planted mistake may drive a value to 0 or inf
@pytest.mark.parametrize("what,name,mutate,pin", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_is_caught(monkeypatch, what, name, mutate, pin):
    _plant(monkeypatch, name, mutate(getattr(OW, name)))
    with pytest.raises(AssertionError):
        pin()


def test_unplanted_pins_pass():
    """The same pins pass on the unmodified oracle (so the failures above come from the
    planted mistakes)."""
    for _, _, _, pin in CASES:
        pin()


def test_planted_philox_constant_is_caught(monkeypatch):
    """A wrong word in the counter-based generator is caught by the published known answers."""
    orig = OP.philox4x32_10
    monkeypatch.setattr(OP, "philox4x32_10", _m_philox_bit(orig))
    monkeypatch.setattr(O, "philox4x32_10", _m_philox_bit(orig))
    with pytest.raises(AssertionError):
        TS.test_philox_known_answers()

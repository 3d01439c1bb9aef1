"""GPU checks of the autograd wrappers: the hand-written adjoint and the chi^2 gradients
against central finite differences (exact for linear and quadratic functions, O(h^2) in
theta) and against the FP64 oracle's adjoint.  Bar: 1e-4 relative (float32) and 1e-10
(float64, oracle)."""
import numpy as np
import pytest

import oracle as O
from paper_1810_00503_amd import workloads as WL
from tests.gpu_util import make_problem, random_half

pytestmark = pytest.mark.gpu


def _shear(n=32, seed=4):
    return WL.shear_workload(n, seed, nbands_e=3, nbands_b=3)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("masked", [False, True])
def test_response_adjoint_vs_finite_differences_and_oracle(lib, dtype, masked):
    import torch
    print(f"[autograd response {dtype} masked={masked}]", flush=True)
    wl = _shear()
    prob = make_problem(lib, torch, wl, dtype)
    n = wl.n
    rng = np.random.default_rng(1)
    s0 = random_half(rng, 2, n)
    wts = rng.standard_normal((2, n, n))
    s = torch.tensor(s0, dtype=prob.cdtype, device="cuda:0", requires_grad=True)
    wt = torch.tensor(wts, dtype=prob.rdtype, device="cuda:0")
    x = lib.autograd.response(s, prob, masked=masked)
    L = (x * wt).sum()
    L.backward()
    g = s.grad.cpu().numpy()
    # oracle: dL/ds = 2 R^T (M wts) on the free modes
    M = (wl.W > 0)[None] if masked else np.ones((1, n, n), bool)
    ref = np.where(O.free_mask(n)[None], 2.0 * O.adjoint(M * wts), 0)
    tol = 1e-5 if dtype == "f32" else 1e-11
    assert np.linalg.norm(g - ref) <= tol * np.linalg.norm(ref)
    # central differences along random free directions (L is linear in s)
    for _ in range(3):
        e = random_half(rng, 2, n)
        et = torch.tensor(e, dtype=prob.cdtype, device="cuda:0")
        h = 0.5
        with torch.no_grad():
            lp = (lib.autograd.response(s + h * et, prob, masked) * wt).sum().item()
            lm = (lib.autograd.response(s - h * et, prob, masked) * wt).sum().item()
        fd = (lp - lm) / (2 * h)
        an = float(np.sum((np.conj(g) * e).real))
        assert abs(fd - an) <= (1e-4 if dtype == "f32" else 1e-10) * (abs(an) + np.abs(g).sum() * 1e-3)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_chi2_gradients_vs_finite_differences(lib, dtype):
    import torch
    print(f"[autograd chi2 {dtype}]", flush=True)
    wl = _shear(seed=9)
    n = wl.n
    rng = np.random.default_rng(3)
    d = rng.standard_normal((2, n, n))
    prob = make_problem(lib, torch, wl, dtype, d=d)
    S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
    fr = O.free_mask(n)[None] & (S > 0)
    B = 2
    s0 = np.stack([np.where(fr, np.sqrt(S) * (rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape)), 0)
                   for _ in range(B)])
    s = torch.tensor(s0, dtype=prob.cdtype, device="cuda:0", requires_grad=True)
    theta = torch.tensor(wl.theta_fid, dtype=torch.float64, requires_grad=True)
    chi = lib.autograd.chi2(s, theta, prob)
    wts = torch.tensor([0.7, 1.3], dtype=torch.float64, device="cuda:0")
    (chi * wts).sum().backward()
    gs = s.grad.cpu().numpy()
    gth = theta.grad.numpy()
    # oracle values
    for b in range(B):
        ref = O.grad_chi2(s0[b], d, wl.W, S) * [0.7, 1.3][b]
        tol = 2e-5 if dtype == "f32" else 1e-11
        assert np.linalg.norm(gs[b] - ref) <= tol * np.linalg.norm(ref)
    # finite differences in s (quadratic: exact up to round-off)
    e = np.where(fr, rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape), 0)
    et = torch.tensor(np.stack([e, 0 * e]), dtype=prob.cdtype, device="cuda:0")
    h = 0.05
    with torch.no_grad():
        cp = lib.autograd.chi2(s + h * et, theta, prob).cpu().numpy()
        cm = lib.autograd.chi2(s - h * et, theta, prob).cpu().numpy()
    fd = 0.7 * (cp[0] - cm[0]) / (2 * h)
    an = float(np.sum((np.conj(gs[0]) * e).real))
    assert abs(fd - an) <= (1e-4 if dtype == "f32" else 1e-9) * abs(an)
    # finite differences in theta (O(h^2))
    for bnd in range(wl.nbands):
        # truncation ~ (h/theta)^2 of the 1/theta prior term; float32 rounding of S ~ 6e-8 / (h/theta)
        hh = (3e-3 if dtype == "f32" else 1e-4) * wl.theta_fid[bnd]
        tp = theta.detach().clone()
        tm = theta.detach().clone()
        tp[bnd] += hh
        tm[bnd] -= hh
        with torch.no_grad():
            cpp = (lib.autograd.chi2(s, tp, prob) * wts).sum().item()
            cmm = (lib.autograd.chi2(s, tm, prob) * wts).sum().item()
        fd = (cpp - cmm) / (2 * hh)
        assert abs(fd - gth[bnd]) <= (1e-4 if dtype == "f32" else 1e-6) * abs(gth[bnd]) + 1e-9
    # and the closed form against the oracle: -2 E_b(theta, s)
    Eo = sum(w * O.band_E(s0[b], S, wl.band, wl.theta_fid, wl.nbands) for b, w in enumerate([0.7, 1.3]))
    np.testing.assert_allclose(gth, -2.0 * Eo, rtol=1e-5 if dtype == "f32" else 1e-11)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_chi2_dtheta_through_the_c_abi(lib, dtype):
    """wf_chi2_dtheta: sum_i gout_i d chi^2_i / d theta_b against the oracle's derivative."""
    import torch
    print(f"[wf_chi2_dtheta {dtype}]", flush=True)
    wl = _shear(n=48, seed=12)
    n = wl.n
    rng = np.random.default_rng(21)
    prob = make_problem(lib, torch, wl, dtype, d=rng.standard_normal((2, n, n)))
    S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
    fr = O.free_mask(n)[None] & (S > 0)
    s0 = np.stack([np.where(fr, np.sqrt(S) * (rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape)), 0)
                   for _ in range(3)])
    st = torch.tensor(s0, dtype=prob.cdtype, device="cuda:0")
    gout = np.array([0.5, -1.25, 2.0])
    got = lib.wf_chi2_dtheta(prob, st, gout)
    ref = sum(w * O.dchi2_dtheta(s0[i], wl.pshape, wl.band, wl.theta_fid, wl.nbands) for i, w in enumerate(gout))
    tol = 1e-5 if dtype == "f32" else 1e-12
    np.testing.assert_allclose(got, ref, rtol=tol, atol=tol * np.abs(ref).max())
    one = lib.wf_chi2_dtheta(prob, st[1])
    np.testing.assert_allclose(one, O.dchi2_dtheta(s0[1], wl.pshape, wl.band, wl.theta_fid, wl.nbands), rtol=tol)


def test_shear512_masked_autograd_full_size(lib):
    """Config 3 at its own size: the masked response M R s of the 512^2 E/B shear map (the
    register-staged passes) with its hand-written adjoint under autograd, against the oracle's
    adjoint and central differences; chi^2 with the workload's mask and noise, its s- and
    theta-gradients by central differences."""
    import torch
    print("[autograd 512^2 shear masked]", flush=True)
    wl = WL.shear_eb()
    n = wl.n
    rng = np.random.default_rng(512)
    d = rng.standard_normal((2, n, n))
    prob = make_problem(lib, torch, wl, "f32", d=d)
    S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
    fr = O.free_mask(n)[None] & (S > 0)
    s0 = np.where(fr, np.sqrt(S) * (rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape)), 0)
    wts = rng.standard_normal((2, n, n))
    s = torch.tensor(s0, dtype=prob.cdtype, device="cuda:0", requires_grad=True)
    wt = torch.tensor(wts, dtype=prob.rdtype, device="cuda:0")
    (lib.autograd.response(s, prob, masked=True) * wt).sum().backward()
    g = s.grad.cpu().numpy()
    ref = np.where(O.free_mask(n)[None], 2.0 * O.adjoint((wl.W > 0)[None] * wts), 0)
    assert np.linalg.norm(g - ref) <= 1e-5 * np.linalg.norm(ref)
    for k in range(3):
        e = np.where(fr, rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape), 0) * np.sqrt(S)
        et = torch.tensor(e, dtype=prob.cdtype, device="cuda:0")
        with torch.no_grad():
            lp = (lib.autograd.response(s + 0.5 * et, prob, True).double() * wt.double()).sum().item()
            lm = (lib.autograd.response(s - 0.5 * et, prob, True).double() * wt.double()).sum().item()
        an = float(np.sum((np.conj(g) * e).real))
        assert abs((lp - lm) - an) <= 1e-4 * abs(an), (k, lp - lm, an)
    # chi^2: s-gradient and theta-gradient
    s2 = torch.tensor(s0, dtype=prob.cdtype, device="cuda:0", requires_grad=True)
    theta = torch.tensor(wl.theta_fid, dtype=torch.float64, requires_grad=True)
    lib.autograd.chi2(s2, theta, prob).backward()
    gs, gth = s2.grad.cpu().numpy(), theta.grad.numpy()
    refg = O.grad_chi2(s0, d, wl.W, S)
    assert np.linalg.norm(gs - refg) <= 2e-5 * np.linalg.norm(refg)
    e = np.where(fr, rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape), 0) * np.sqrt(S)
    et = torch.tensor(e, dtype=prob.cdtype, device="cuda:0")
    # chi^2 is quadratic, so the central difference is exact at any step; a unit step keeps the
    # difference far above the float32 rounding of the 512^2 data term
    with torch.no_grad():
        cp = lib.autograd.chi2(s2 + et, theta, prob).item()
        cm = lib.autograd.chi2(s2 - et, theta, prob).item()
    an = float(np.sum((np.conj(gs) * e).real))
    assert abs((cp - cm) / 2.0 - an) <= 1e-4 * abs(an), (cp - cm, an)
    np.testing.assert_allclose(gth, O.dchi2_dtheta(s0, wl.pshape, wl.band, wl.theta_fid, wl.nbands), rtol=1e-5)
    for bnd in (0, 9, 10, 19):
        hh = 3e-3 * wl.theta_fid[bnd]
        tp, tm = theta.detach().clone(), theta.detach().clone()
        tp[bnd] += hh
        tm[bnd] -= hh
        with torch.no_grad():
            fd = (lib.autograd.chi2(s2, tp, prob).item() - lib.autograd.chi2(s2, tm, prob).item()) / (2 * hh)
        assert abs(fd - gth[bnd]) <= 1e-4 * abs(gth[bnd]), (bnd, fd, gth[bnd])

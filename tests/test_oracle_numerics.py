"""Pins for the oracle's coefficients, bounds, density matrices, moments and mu.

Each check is against mathematics the oracle does not itself encode: the
interpolation property of the Chebyshev-Gauss projection, the closed form of
the step-function expansion, symmetry, Gershgorin's theorem on diagonal
matrices, three independent routes to the same matrix polynomial, the exact
Fermi operator in the converged regime, and scipy's root finder.
"""
import numpy as np
import pytest
import scipy.optimize

import synth
from oracle import chebyshev as ch


# ---------------------------------------------------------------- coefficients

@pytest.mark.parametrize("order,beta_s,mu_s", [(16, 5.0, 0.3), (64, 40.0, -0.2), (127, 80.0, 0.71)])
def test_coeffs_interpolate_at_nodes(order, beta_s, mu_s):
    # With M = L+1 nodes the projection is the interpolant: p(x_j) = f(x_j).
    M = order + 1
    c = ch.chebyshev_coeffs(order, beta_s, mu_s, M)
    theta = np.pi * (np.arange(M) + 0.5) / M
    x = np.cos(theta)
    np.testing.assert_allclose(ch.cheb_eval(c, x), ch.fermi(x, beta_s, mu_s), atol=2e-14)


def test_coeffs_step_limit_closed_form():
    # beta' -> infinity: f is the step 1[x < mu~]; c_0 = (pi - t)/pi, c_n = -2 sin(n t)/(n pi).
    order, mu_s, beta_s = 40, 0.37, 1e7
    M = 1 << 22
    c = ch.chebyshev_coeffs(order, beta_s, mu_s, M)
    t = np.arccos(mu_s)
    n = np.arange(1, order + 1)
    want = np.concatenate([[(np.pi - t) / np.pi], -2.0 * np.sin(n * t) / (n * np.pi)])
    np.testing.assert_allclose(c, want, atol=2e-6)


def test_coeffs_half_filling_symmetry():
    # f(x; mu~=0) - 1/2 is odd: c_0 = 1/2 and every even coefficient vanishes.
    c = ch.chebyshev_coeffs(200, 150.0, 0.0)
    assert abs(c[0] - 0.5) < 1e-15
    assert np.max(np.abs(c[2::2])) < 1e-15


def test_coeffs_quadrature_converged():
    order, beta_s, mu_s = 512, 1350.0, 0.1
    M = ch.quadrature_size(order, beta_s)
    c1 = ch.chebyshev_coeffs(order, beta_s, mu_s, M)
    c2 = ch.chebyshev_coeffs(order, beta_s, mu_s, 2 * M)
    assert np.max(np.abs(c1 - c2)) < 1e-15 * max(1.0, np.abs(c1).sum())


def test_quadrature_size_rule():
    assert ch.quadrature_size(128, 400.0) == 4096
    assert ch.quadrature_size(512, 1350.0) == 16384
    assert ch.quadrature_size(2048, 1e4) == 131072
    assert ch.quadrature_size(0, 0.0) == 64


def test_fermi_function():
    assert ch.fermi(0.2, 30.0, 0.2) == 0.5
    assert ch.fermi(-1.0, 1e4, 0.0) == 1.0
    assert ch.fermi(1.0, 1e4, 0.0) == 0.0


# --------------------------------------------------------------------- bounds

def test_bounds_diagonal_exact():
    d = np.array([3.0, -1.5, 0.25, 7.0])
    assert ch.gershgorin_bounds(np.diag(d)) == (-1.5, 7.0)


@pytest.mark.parametrize("law", synth.LAWS)
def test_bounds_contain_spectrum(law):
    h, q, lam = synth.hamiltonian(96, law, seed=5)
    lo, hi = ch.gershgorin_bounds(h)
    ev = np.linalg.eigvalsh(h)
    assert lo <= ev.min() and ev.max() <= hi


def test_bounds_by_hand_2x2():
    h = np.array([[1.0, -2.0], [-2.0, 3.0]])
    assert ch.gershgorin_bounds(h) == (-1.0, 5.0)


# ------------------------------------------------------------ density matrices

@pytest.mark.parametrize("law,n,order", [("uniform", 64, 40), ("gaussmix6", 96, 64), ("highdos", 80, 33)])
def test_density_three_routes_agree(law, n, order):
    h, q, lam = synth.hamiltonian(n, law, seed=11)
    emin, emax = ch.gershgorin_bounds(h)
    c = ch.chebyshev_coeffs(order, 30.0 * 0.5 * (emax - emin), 0.05)
    d_gen = ch.density_from_eigs(q, lam, c, emin, emax)
    d_eig = ch.density_eigh(h, c, emin, emax)
    d_rec = ch.density_recursion(h, c, emin, emax)
    np.testing.assert_allclose(d_eig, d_gen, atol=1e-12)
    np.testing.assert_allclose(d_rec, d_gen, atol=1e-12)


def test_density_symmetric_and_commutes():
    h, q, lam = synth.hamiltonian(120, "uniform", seed=2)
    emin, emax = ch.gershgorin_bounds(h)
    c = ch.chebyshev_coeffs(128, 50.0 * 0.5 * (emax - emin), 0.0)
    d = ch.density_eigh(h, c, emin, emax)
    assert np.max(np.abs(d - d.T)) < 1e-13
    assert np.max(np.abs(h @ d - d @ h)) < 1e-12
    assert ch.commutator_max(h, d) < 1e-12


def test_commutator_closed_form_for_diagonal_h():
    # (diag(a) D - D diag(a))_ij = (a_i - a_j) D_ij
    rng = np.random.default_rng(3)
    a = rng.normal(size=9)
    d = rng.normal(size=(9, 9))
    d = d + d.T
    assert abs(ch.commutator_max(np.diag(a), d) - np.max(np.abs((a[:, None] - a[None, :]) * d))) < 1e-15
    assert ch.commutator_max(np.diag(a), np.diag(rng.normal(size=9))) == 0.0


def test_density_diagonal_hamiltonian():
    diag = np.linspace(-2.0, 3.0, 17)
    h = np.diag(diag)
    emin, emax = ch.gershgorin_bounds(h)
    c = ch.chebyshev_coeffs(50, 8.0, 0.1)
    d = ch.density_recursion(h, c, emin, emax)
    cen, a = ch.scaling(emin, emax)
    np.testing.assert_allclose(np.diag(d), ch.cheb_eval(c, (diag - cen) / a), atol=1e-14)
    assert np.max(np.abs(d - np.diag(np.diag(d)))) == 0.0


def test_density_converges_to_fermi_dirac():
    # Tight bounds and a small beta': the truncated expansion reaches the exact Fermi operator.
    n, order = 100, 128
    h, q, lam = synth.hamiltonian(n, "uniform", seed=9)
    emin, emax = float(lam.min()) - 1e-3, float(lam.max()) + 1e-3
    cen, a = ch.scaling(emin, emax)
    beta, mu = 20.0 / a, 0.1
    c = ch.chebyshev_coeffs(order, beta * a, (mu - cen) / a)
    d_l = ch.density_from_eigs(q, lam, c, emin, emax)
    d_fd = ch.fermi_dirac_density(q, lam, beta, mu)
    assert np.max(np.abs(d_l - d_fd)) < 1e-8


def test_gapped_large_beta_is_idempotent():
    n = 60
    lam = np.concatenate([np.linspace(-1.0, -0.4, 30), np.linspace(0.4, 1.0, 30)])
    h, q, lam = synth.hamiltonian(n, lam=lam, seed=4)
    # beta' = 100 puts f(+-0.4) at e^-40; L = 1000 brings the tail to ~e^{-L pi/beta'}.
    c = ch.chebyshev_coeffs(1000, 100.0, 0.0)
    d = ch.density_from_eigs(q, lam, c, -1.0, 1.0)
    assert np.max(np.abs(d @ d - d)) < 1e-9
    assert abs(np.trace(d) - 30.0) < 1e-9


# ------------------------------------------------------------------- moments

def test_moments_match_matrix_traces():
    n, order = 48, 30
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=13)
    emin, emax = ch.gershgorin_bounds(h)
    tau = ch.moments_from_eigs(lam, emin, emax, order)
    ht = ch.scaled_hamiltonian(h, emin, emax)
    t0, t1 = np.eye(n), ht
    traces = [np.trace(t0), np.trace(t1)]
    for _ in range(order - 1):
        t0, t1 = t1, 2 * ht @ t1 - t0
        traces.append(np.trace(t1))
    np.testing.assert_allclose(tau, traces, atol=1e-11)
    assert tau[0] == n
    assert np.all(np.abs(tau) <= n + 1e-9)


def test_trace_identity():
    h, q, lam = synth.hamiltonian(70, "uniform", seed=21)
    emin, emax = ch.gershgorin_bounds(h)
    c = ch.chebyshev_coeffs(90, 120.0, -0.05)
    tau = ch.moments_from_eigs(lam, emin, emax, 90)
    d = ch.density_eigh(h, c, emin, emax)
    assert abs(np.trace(d) - ch.trace_of_series(c, tau)) < 1e-11


# ------------------------------------------------------------------------- mu

def test_mu_symmetric_spectrum_is_zero_first_sweep():
    n = 64
    lam = synth.symmetric_pairs_spectrum(n, seed=1)
    b = 1.25
    tau = ch.moments_from_eigs(lam, -b, b, 64)
    mu_s, iters, t, status = ch.bisect_mu(tau, 64, 40.0, n / 2, tol=1e-9)
    assert status == ch.OK and iters == 1 and mu_s == 0.0
    assert abs(t - n / 2) < 1e-9


def test_mu_bisection_matches_brentq():
    n, order = 256, 128
    h, q, lam = synth.hamiltonian(n, "uniform", seed=1000)
    emin, emax = ch.gershgorin_bounds(h)
    cen, a = ch.scaling(emin, emax)
    beta_s = 50.0 * a
    M = ch.quadrature_size(order, beta_s)
    tau = ch.moments_from_eigs(lam, emin, emax, order)
    mu_s, iters, t, status = ch.bisect_mu(tau, order, beta_s, 128.0, tol=1e-10, M=M)
    assert status == ch.OK and abs(t - 128.0) < 1e-10

    def g(x):
        return ch.trace_of_series(ch.chebyshev_coeffs(order, beta_s, x, M), tau) - 128.0

    root = scipy.optimize.brentq(g, -1.0, 1.0, xtol=1e-15, rtol=1e-15)
    slope = (g(root + 1e-7) - g(root - 1e-7)) / 2e-7
    assert slope > 0
    assert abs(mu_s - root) <= 2e-10 / slope + 1e-15


def test_mu_bracket_error():
    tau = ch.moments_from_eigs(np.linspace(-0.5, 0.5, 10), -1.0, 1.0, 16)
    assert ch.bisect_mu(tau, 16, 10.0, 10.5)[3] == ch.BRACKET
    assert ch.bisect_mu(tau, 16, 10.0, -0.5)[3] == ch.BRACKET


def test_mu_search_density_end_to_end_small():
    n = 128
    h, q, lam = synth.hamiltonian(n, "uniform", seed=1001)
    out = ch.mu_search_density(h, 50.0, 64.0, 128)
    assert out["status"] == ch.OK
    assert abs(np.trace(out["D"]) - 64.0) < 1e-9
    out2 = ch.mu_search_density(h, 50.0, 64.0, 128, eig=(q, lam))
    np.testing.assert_allclose(out2["D"], out["D"], atol=1e-12)


# ---------------------------------------------------------------- Jackson damping (option)

def test_jackson_factors_by_hand():
    g = ch.jackson_kernel(1)              # N = 2 terms: g_1 = (2 cos(pi/3) + cos(pi/3)) / 3 = 1/2
    assert g[0] == 1.0
    assert abs(g[1] - 0.5) < 1e-15
    g = ch.jackson_kernel(200)
    assert g[0] == 1.0 and np.all(np.diff(g) < 0) and g[-1] > 0


def test_jackson_damped_series_stays_in_unit_interval():
    # a positive kernel with unit weight: the damped expansion of 0 <= f <= 1 stays in [0, 1]
    # (no Gibbs overshoot), while the plain truncation overshoots near a sharp step
    order, beta_s, mu_s = 128, 2000.0, 0.13
    M = ch.quadrature_size(order, beta_s)
    x = np.linspace(-1, 1, 20001)
    plain = ch.cheb_eval(ch.chebyshev_coeffs(order, beta_s, mu_s, M), x)
    damped = ch.cheb_eval(ch.chebyshev_coeffs(order, beta_s, mu_s, M, "jackson"), x)
    assert plain.max() > 1.05 and plain.min() < -0.05
    assert damped.min() > -1e-12 and damped.max() < 1.0 + 1e-12
    # damping keeps c_0 (the mean of f over the Chebyshev measure)
    c_p = ch.chebyshev_coeffs(order, beta_s, mu_s, M)
    c_d = ch.chebyshev_coeffs(order, beta_s, mu_s, M, "jackson")
    assert c_d[0] == c_p[0]


def test_jackson_damped_mu_search_counts_electrons():
    h, q, lam = synth.hamiltonian(60, "uniform", seed=5)
    lo, hi = ch.gershgorin_bounds(h)
    cen, a = ch.scaling(lo, hi)
    order, beta = 64, 20.0
    tau = ch.moments_from_eigs(lam, lo, hi, order)
    mu_s, it, t, st = ch.bisect_mu(tau, order, beta * a, 27.5, damping="jackson")
    assert st == ch.OK
    c = ch.chebyshev_coeffs(order, beta * a, mu_s, damping="jackson")
    d = ch.density_from_eigs(q, lam, c, lo, hi)
    assert abs(np.trace(d) - 27.5) < 1e-9

"""Pins of the oracle's Lanczos bounds (CPU, float64).

What fixes them besides the oracle itself:
* SplitMix64: the published outputs of the reference generator for seed 0;
* the Lanczos relation H V^T = V^T T + beta_{k-1} v_k e_{k-1}^T and the
  orthonormality of the basis (a dropped term, a wrong sign or a missing
  reorthogonalisation breaks one of them);
* Cauchy interlacing: Ritz values lie inside [lambda_min, lambda_max];
* n steps on an n x n matrix reproduce its eigenvalues (LAPACK eigvalsh);
* invariant subspaces (few distinct eigenvalues, H = c I, n = 1) stop the
  recurrence early with exact extremes;
* the bounds enclose the spectrum of every synthetic law and stay inside
  Gershgorin's interval.
"""
import numpy as np
import pytest

import synth
from oracle import chebyshev as ch


def test_splitmix64_published_outputs():
    # first outputs of the reference SplitMix64 for seed 0
    assert ch.splitmix64(3, 0) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_splitmix64_uniform_map():
    z = ch.splitmix64(5, 123)
    u = ch.splitmix64_uniform(5, 123)
    assert np.array_equal(u, np.array([2.0 * (x >> 11) / 2.0 ** 53 - 1.0 for x in z]))
    big = ch.splitmix64_uniform(20000, 7)
    assert big.min() >= -1.0 and big.max() < 1.0
    assert abs(big.mean()) < 0.02 and abs(np.mean(big ** 2) - 1.0 / 3.0) < 0.01


def _random_sym(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n, n))
    return (a + a.T) / 2


@pytest.mark.parametrize("n,steps", [(60, 20), (200, 40), (17, 17)])
def test_lanczos_relation_and_orthonormal_basis(n, steps):
    h = _random_sym(n, n)
    alpha, beta, V = ch.lanczos(h, steps, seed=3)
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    assert np.max(np.abs(V @ V.T - np.eye(k))) < 1e-12
    R = h @ V.T - V.T @ T
    scale = np.linalg.norm(h, 2)
    assert np.max(np.abs(R[:, :-1])) < 1e-12 * scale
    # the last column is the residual beta_{k-1} v_k, orthogonal to the basis
    assert abs(np.linalg.norm(R[:, -1]) - beta[-1]) < 1e-12 * scale
    assert np.max(np.abs(V @ R[:, -1])) < 1e-12 * scale


def test_ritz_values_interlace():
    h = _random_sym(150, 1)
    lam = np.linalg.eigvalsh(h)
    alpha, beta, _ = ch.lanczos(h, 30)
    theta = ch.tridiag_eigvals(alpha, beta)
    assert theta[0] >= lam[0] - 1e-12 and theta[-1] <= lam[-1] + 1e-12


def test_full_length_reproduces_the_spectrum():
    h = _random_sym(40, 2)
    alpha, beta, _ = ch.lanczos(h, 40)
    theta = ch.tridiag_eigvals(alpha, beta)
    assert np.max(np.abs(theta - np.linalg.eigvalsh(h))) < 1e-10


def test_invariant_subspace_stops_early():
    # three distinct eigenvalues: the Krylov space has dimension 3
    rng = np.random.default_rng(4)
    q, _ = np.linalg.qr(rng.normal(size=(50, 50)))
    lam = np.repeat([-2.0, 0.5, 3.0], [10, 25, 15])
    h = (q * lam) @ q.T
    alpha, beta, _ = ch.lanczos(h, 40)
    assert len(alpha) == 3
    assert np.max(np.abs(ch.tridiag_eigvals(alpha, beta) - [-2.0, 0.5, 3.0])) < 1e-12
    lo, hi, _, _ = ch.lanczos_bounds(h, 40, margin=0.01)
    r = beta[-1]
    w = 5.0 + 2 * r
    g_lo, g_hi = ch.gershgorin_bounds(h)
    assert abs(lo - max(-2.0 - r - 0.01 * w, g_lo)) < 1e-12 and abs(hi - min(3.0 + r + 0.01 * w, g_hi)) < 1e-12


@pytest.mark.parametrize("h,val", [(3.0 * np.eye(5), 3.0), (np.array([[2.0]]), 2.0), (np.diag(np.full(4, -1.5)), -1.5)])
def test_scalar_matrix_bounds_are_exact(h, val):
    lo, hi, alpha, _ = ch.lanczos_bounds(h, 40)
    assert lo == val and hi == val and len(alpha) == 1


def test_diagonal_matrix():
    h = np.diag(np.arange(10.0))
    lo, hi, alpha, _ = ch.lanczos_bounds(h, 40)
    assert len(alpha) == 10 and (lo, hi) == (0.0, 9.0)   # Gershgorin is exact here


@pytest.mark.parametrize("law", synth.LAWS)
@pytest.mark.parametrize("n", [64, 300])
def test_bounds_enclose_spectrum_inside_gershgorin(law, n):
    h, _, lam = synth.hamiltonian(n, law, seed=n)
    lo, hi, alpha, beta = ch.lanczos_bounds(h, 40)
    g_lo, g_hi = ch.gershgorin_bounds(h)
    assert g_lo <= lo <= lam.min() and lam.max() <= hi <= g_hi
    # dense synthetic H: Gershgorin's discs are loose, the Lanczos interval is not
    assert hi - lo < 0.5 * (g_hi - g_lo)
    assert hi - lo < 2.0 * (lam.max() - lam.min())


def test_chain_keeps_the_tighter_gershgorin_side():
    # nearest-neighbour chain: Gershgorin [-2, 2] already hugs 2 cos(pi/(n+1))
    n = 200
    h = -(np.eye(n, k=1) + np.eye(n, k=-1))
    lo, hi, _, _ = ch.lanczos_bounds(h, 40)
    assert (lo, hi) == (-2.0, 2.0)
    edge = 2 * np.cos(np.pi / (n + 1))
    assert lo <= -edge and edge <= hi


def test_seed_changes_start_vector_not_enclosure():
    h, _, lam = synth.hamiltonian(200, "gaussmix6", seed=9)
    for seed in (0, 1, 2**63 + 5):
        lo, hi, _, _ = ch.lanczos_bounds(h, 30, seed=seed)
        assert lo <= lam.min() and lam.max() <= hi


def test_tighter_bounds_cut_the_truncation_error():
    # same order, same H: the expansion on the Lanczos interval is far closer to the exact
    # Fermi operator than on Gershgorin's (beta' = beta (emax - emin)/2 drops about 6x)
    n, beta, order = 200, 100.0, 256
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=31)
    errs = {}
    for name, b in (("gershgorin", ch.gershgorin_bounds(h)), ("lanczos", ch.lanczos_bounds(h, 40)[:2])):
        r = ch.mu_search_density(h, beta, n / 2, order, bounds=b, eig=(q, lam))
        assert r["status"] == ch.OK
        errs[name] = np.max(np.abs(r["D"] - ch.fermi_dirac_density(q, lam, beta, r["mu"])))
    assert errs["lanczos"] < 0.05 * errs["gershgorin"], errs

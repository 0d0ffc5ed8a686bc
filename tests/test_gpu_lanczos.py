"""GPU parity of the Lanczos bounds (chebdm_bounds_lanczos and opts.bounds = LANCZOS).

The device recurrence and the oracle's take the same steps from the same
SplitMix64 start vector but sum in different orders, so the tridiagonal and
the bounds agree to rounding, not bit for bit: 1e-10 times the Gershgorin
scale max(|g_lo|, |g_hi|) on alpha, beta and both bounds (40 steps of
float64 dot products over n <= 2100 terms stay many orders below that).  The
steps done before a breakdown are integers and must agree exactly.  Density
matrices at the Lanczos bounds are held to the float64 target of 1e-10
against the oracle evaluated at the same bounds.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import chebyshev as ch
from refcheck import checked_lanczos_bounds, checked_quadrature

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_12616_amd as chebdm

    chebdm.load_library()
    return chebdm


@pytest.fixture(scope="module")
def handle(cd):
    h = cd.Handle(0)
    yield h
    h.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _compare(cd, handle, h, steps, margin=0.01, seed=0, H=None):
    lo, hi, a, b = cd.chebdm_bounds_lanczos(handle, _dev(h) if H is None else H, steps, margin, seed)
    rlo, rhi, ra, rb = ch.lanczos_bounds(h, steps, margin, seed)
    g_lo, g_hi = ch.gershgorin_bounds(h)
    scale = max(abs(g_lo), abs(g_hi), 1e-300)
    assert len(a) == len(ra), (len(a), len(ra))
    ea = float(np.max(np.abs(a - ra))) / scale
    eb = float(np.max(np.abs(b - rb))) / scale
    _say(f"  steps done {len(a)}: bounds [{lo:.12f}, {hi:.12f}] oracle [{rlo:.12f}, {rhi:.12f}] "
         f"rel err alpha {ea:.1e} beta {eb:.1e}")
    assert ea <= 1e-10 and eb <= 1e-10
    assert abs(lo - rlo) <= 1e-10 * scale and abs(hi - rhi) <= 1e-10 * scale
    return lo, hi


@pytest.mark.parametrize("n,law,steps", [(2, "uniform", 40), (5, "gaussmix6", 40), (64, "uniform", 40),
                                         (300, "gaussmix6", 40), (1500, "highdos", 40), (2100, "gaussmix6", 24),
                                         (333, "uniform", 128), (700, "uniform", 1)])
def test_bounds_match_oracle(cd, handle, n, law, steps):
    _say(f"lanczos n={n} law={law} steps={steps}")
    h, _, lam = synth.hamiltonian(n, law, seed=500 + n)
    lo, hi = _compare(cd, handle, h, steps)
    if steps >= 8:   # one or two steps give no enclosure: the extreme Ritz values have not settled
        assert lo <= lam.min() and lam.max() <= hi


@pytest.mark.parametrize("kind", ["scalar", "one", "diag", "three_levels", "chain"])
def test_special_matrices(cd, handle, kind):
    _say(f"lanczos special {kind}")
    if kind == "scalar":
        h = 3.0 * np.eye(37)
    elif kind == "one":
        h = np.array([[-0.75]])
    elif kind == "diag":
        h = np.diag(np.linspace(-1.0, 2.0, 50))
    elif kind == "three_levels":
        rng = np.random.default_rng(4)
        q, _ = np.linalg.qr(rng.normal(size=(90, 90)))
        h = (q * np.repeat([-2.0, 0.5, 3.0], [20, 40, 30])) @ q.T
        h = (h + h.T) / 2
    else:
        h = -(np.eye(1100, k=1) + np.eye(1100, k=-1))
    lo, hi = _compare(cd, handle, h, 40)
    lam = np.linalg.eigvalsh(h)
    assert lo <= lam.min() + 1e-12 and lam.max() - 1e-12 <= hi
    if kind in ("scalar", "one"):
        assert lo == hi == h[0, 0]


def test_leading_dimension_and_seed(cd, handle):
    n, ld = 301, 384
    h, _, _ = synth.hamiltonian(n, "uniform", seed=8)
    big = torch.zeros((n, ld), dtype=torch.float64, device="cuda:0")
    big[:, :n] = _dev(h)
    _compare(cd, handle, h, 30, margin=0.0, seed=12345, H=big[:, :n])
    _compare(cd, handle, h, 30, margin=0.2, seed=2**64 - 1, H=big[:, :n])


def test_arguments_are_checked(cd, handle):
    H = _dev(np.eye(8))
    for steps, margin in ((0, 0.01), (129, 0.01), (10, -1.0), (10, float("nan"))):
        with pytest.raises(cd.ChebdmError) as e:
            cd.chebdm_bounds_lanczos(handle, H, steps, margin)
        assert e.value.code == -1
    bad = np.eye(8)
    bad[3, 5] = np.nan
    with pytest.raises(cd.ChebdmError) as e:
        cd.chebdm_bounds_lanczos(handle, _dev(bad), 8)
    assert e.value.code == -4


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_mu_search_with_lanczos_bounds(cd, handle, prec, tol):
    n, order, beta = 700, 256, 100.0
    ne = n / 2 + 0.5
    _say(f"mu search with Lanczos bounds n={n} order={order} prec={prec}")
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=44)
    H = _dev(h)
    opts = cd.make_opts(prec, bounds="lanczos")
    mu, D, info = cd.chebdm_mu_search(handle, H, beta, ne, order, opts)
    lo, hi, _, _ = cd.chebdm_bounds_lanczos(handle, H, 40, 0.01, 0)
    assert (info["emin"], info["emax"]) == (lo, hi)   # same kernels, same seed: bit-identical
    assert info["status"] == 0
    lo, hi = checked_lanczos_bounds(h, (lo, hi))       # the reference takes the oracle's bounds
    cen, a = ch.scaling(lo, hi)
    M = checked_quadrature(order, beta, lo, hi, info)
    c = ch.chebyshev_coeffs(order, beta * a, (mu - cen) / a, M)
    ref = ch.density_from_eigs(q, lam, c, lo, hi)
    err = float(np.max(np.abs(D.cpu().numpy() - ref)))
    exact = ch.fermi_dirac_density(q, lam, beta, mu)
    trunc = float(np.max(np.abs(ref - exact)))
    _say(f"  bounds [{lo:.6f}, {hi:.6f}] mu={mu:.12f} err vs oracle {err:.2e}, oracle vs exact f {trunc:.2e}")
    assert err <= tol
    t_or = ch.trace_of_series(c, ch.moments_from_eigs(lam, lo, hi, order))
    assert abs(t_or - ne) <= (1e-9 if prec == "fp64" else 1e-5 * n)


def test_lanczos_bounds_beat_gershgorin_at_fixed_order(cd, handle):
    # the gain of the option: same H, same order, distance to the exact Fermi operator
    n, order, beta = 1000, 512, 100.0
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=2002)
    H = _dev(h)
    errs = {}
    for name in ("gershgorin", "lanczos"):
        mu, D, info = cd.chebdm_mu_search(handle, H, beta, n / 2, order, cd.make_opts(bounds=name))
        exact = ch.fermi_dirac_density(q, lam, beta, mu)
        errs[name] = float(np.max(np.abs(D.cpu().numpy() - exact)))
        _say(f"  {name}: [{info['emin']:.4f}, {info['emax']:.4f}] beta'={beta * (info['emax'] - info['emin']) / 2:.0f}"
             f" max|D - f(H)| = {errs[name]:.2e}")
    assert errs["lanczos"] < 1e-2 * errs["gershgorin"]


def test_replayed_bounds_follow_new_contents(cd, handle):
    # the Lanczos launches are captured once per argument set; new contents under the same
    # pointer must give the new matrix's bounds
    n = 400
    h1, _, _ = synth.hamiltonian(n, "uniform", seed=1)
    h2, _, _ = synth.hamiltonian(n, "gaussmix6", seed=2)
    H = _dev(h1)
    first = cd.chebdm_bounds_lanczos(handle, H, 40)
    again = cd.chebdm_bounds_lanczos(handle, H, 40)
    assert first[:2] == again[:2]
    H.copy_(_dev(2.0 * h2))
    lo, hi, _, _ = cd.chebdm_bounds_lanczos(handle, H, 40)
    rlo, rhi, _, _ = ch.lanczos_bounds(2.0 * h2, 40)
    scale = max(abs(rlo), abs(rhi))
    assert abs(lo - rlo) <= 1e-10 * 8 * scale and abs(hi - rhi) <= 1e-10 * 8 * scale

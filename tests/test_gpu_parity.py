"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle.

Tolerances (max-abs, float64 path): 1e-10 on D as the target states; bounds
and coefficients are single reductions, compared at 1e-13 relative.  The
chemical potential is compared through the oracle's own trace at the GPU's
mu (several mu are correct to within the tolerance).  Same seeded inputs on
both sides (``synth``); the oracle uses the generator's eigenpairs.  Where the
library computes the bounds itself, the reference uses the oracle's bounds
and quadrature size, after asserting that the GPU's agree with them.
"""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import chebyshev as ch
from oracle import decomposition as dec
from refcheck import checked_bounds, checked_lanczos_bounds, checked_quadrature

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


def _oracle_density(q, lam, order, beta, mu, emin, emax, M):
    cen, a = ch.scaling(emin, emax)
    c = ch.chebyshev_coeffs(order, beta * a, (mu - cen) / a, M)
    return ch.density_from_eigs(q, lam, c, emin, emax), c


# ------------------------------------------------------------------ bounds

@pytest.mark.parametrize("n,law", [(1, "uniform"), (7, "uniform"), (256, "uniform"), (333, "gaussmix6"),
                                   (1000, "highdos")])
def test_bounds_match_oracle(cd, handle, n, law):
    _say(f"bounds n={n} law={law}")
    h, q, lam = synth.hamiltonian(n, law, seed=17 + n)
    lo, hi = cd.chebdm_bounds(handle, _dev(h))
    rlo, rhi = ch.gershgorin_bounds(h)
    scale = max(abs(rlo), abs(rhi))
    assert abs(lo - rlo) <= 1e-13 * scale and abs(hi - rhi) <= 1e-13 * scale


def test_bounds_with_leading_dimension(cd, handle):
    n, ld = 150, 211
    h, _, _ = synth.hamiltonian(n, "uniform", seed=3)
    big = torch.zeros((n, ld), dtype=torch.float64, device="cuda:0")
    big[:, :n] = _dev(h)
    view = big[:, :n]
    lo, hi = cd.chebdm_bounds(handle, view)
    rlo, rhi = ch.gershgorin_bounds(h)
    assert abs(lo - rlo) < 1e-13 * abs(rlo) and abs(hi - rhi) < 1e-13 * abs(rhi)


def test_bounds_nonfinite_error(cd, handle):
    h, _, _ = synth.hamiltonian(64, "uniform", seed=1)
    h[3, 5] = np.nan
    with pytest.raises(cd.ChebdmError) as e:
        cd.chebdm_bounds(handle, _dev(h))
    assert e.value.code == -4


# ------------------------------------------------------------ coefficients

@pytest.mark.parametrize("order,beta,mu,emin,emax,M", [(128, 50.0, 0.1, -8.0, 8.0, 0), (512, 100.0, -0.3, -13.5, 13.6, 0),
                                                       (40, 3.0, 0.0, -1.0, 1.0, 41), (2048, 400.0, 0.02, -25.0, 25.0, 0)])
def test_coeffs_match_oracle(cd, handle, order, beta, mu, emin, emax, M):
    _say(f"coeffs order={order} beta={beta}")
    c = cd.chebdm_coeffs(handle, beta, mu, emin, emax, order, M)
    cen, a = ch.scaling(emin, emax)
    Mo = M or ch.quadrature_size(order, beta * a)
    ref = ch.chebyshev_coeffs(order, beta * a, (mu - cen) / a, Mo)
    assert np.max(np.abs(c - ref)) <= 1e-13


@pytest.mark.parametrize("order,form,kov", [(128, "composition", 0), (128, "power", 0), (512, "composition", 0),
                                            (24, "power", 0), (99, "power", 7), (2048, "composition", 0),
                                            (0, "composition", 0), (5, "power", 1)])
def test_block_coeffs_match_oracle(cd, handle, order, form, kov):
    rng = np.random.default_rng(order + kov)
    c = rng.uniform(-1, 1, order + 1) * np.exp(-0.01 * np.arange(order + 1))
    k, m, coef = cd.chebdm_block_coeffs(handle, c, order, form, kov)
    assert (k, m) == dec.split_order(order, kov or None)
    if form == "composition":
        ref = dec.composition_form_e(c, k, m)
    else:
        ref = dec.power_form_d(c, k, m).T     # d_{i,l} stored as [l][i]
    scale = max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(coef - ref)) <= 1e-12 * scale


# --------------------------------------------------------------- densities

CASES = [
    # n, law, order, beta, mu, form, k_override
    (256, "uniform", 128, 50.0, 0.05, "composition", 0),
    (256, "uniform", 128, 50.0, 0.05, "power", 0),
    (300, "gaussmix6", 200, 80.0, -0.1, "composition", 0),
    (130, "highdos", 63, 30.0, 0.0, "composition", 5),
    (1, "uniform", 10, 20.0, 0.1, "composition", 0),
    (70, "uniform", 0, 20.0, 0.1, "composition", 0),
    (70, "uniform", 3, 20.0, 0.1, "power", 0),
    (64, "uniform", 30, 20.0, 0.1, "composition", 1),
    (520, "uniform", 255, 40.0, 0.2, "composition", 0),
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}-L{c[2]}-{c[5]}-k{c[6]}" for c in CASES])
def test_density_fp64_matches_oracle(cd, handle, case):
    n, law, order, beta, mu, form, kov = case
    _say(f"density fp64 {case}")
    h, q, lam = synth.hamiltonian(n, law, seed=1000 + n + order)
    opts = cd.make_opts("fp64", form, k_override=kov)
    D, info = cd.chebdm_density(handle, _dev(h), beta, mu, order, opts)
    torch.cuda.synchronize()
    if n == 1:
        # a 1 x 1 H has e_a = e_b: the library returns f(H_00) exactly
        assert info["emin"] == info["emax"] == h[0, 0] and info["n_quad"] == 0
        assert abs(D.item() - 1.0 / (1.0 + math.exp(beta * (h[0, 0] - mu)))) <= 1e-15
        return
    emin, emax = checked_bounds(h, info)
    M = checked_quadrature(order, beta, emin, emax, info)
    ref, c = _oracle_density(q, lam, order, beta, mu, emin, emax, M)
    err = np.max(np.abs(D.cpu().numpy() - ref))
    _say(f"  max|D - D_oracle| = {err:.3e}  k={info['k']} m={info['m']} gemms={info['n_gemm']}")
    assert err <= 1e-10
    assert abs(info["trace"] - np.trace(ref)) <= 1e-9
    k, m = info["k"], info["m"]
    assert info["n_gemm"] == max(k - 1, 0) + (m - 1)


def test_density_writes_only_n_by_n(cd, handle):
    n, ldd = 90, 101
    h, q, lam = synth.hamiltonian(n, "uniform", seed=5)
    out = torch.full((n, ldd), 7.0, dtype=torch.float64, device="cuda:0")
    D, info = cd.chebdm_density(handle, _dev(h), 20.0, 0.0, 50, None, D=out[:, :n])
    torch.cuda.synchronize()
    assert torch.all(out[:, n:] == 7.0)
    lo, hi = checked_bounds(h, info)
    ref, _ = _oracle_density(q, lam, 50, 20.0, 0.0, lo, hi, checked_quadrature(50, 20.0, lo, hi, info))
    assert np.max(np.abs(D.cpu().numpy() - ref)) <= 1e-10


def test_density_given_bounds(cd, handle):
    n, order, beta, mu = 200, 100, 10.0, 0.1
    h, q, lam = synth.hamiltonian(n, "uniform", seed=8)
    emin, emax = float(lam.min()) - 0.01, float(lam.max()) + 0.01
    D, info = cd.chebdm_density(handle, _dev(h), beta, mu, order, None, emin, emax)
    torch.cuda.synchronize()
    assert (info["emin"], info["emax"]) == (emin, emax)
    ref, _ = _oracle_density(q, lam, order, beta, mu, emin, emax, checked_quadrature(order, beta, emin, emax, info))
    assert np.max(np.abs(D.cpu().numpy() - ref)) <= 1e-10


def test_density_scalar_hamiltonian(cd, handle):
    n, c0, beta, mu = 50, 0.3, 7.0, 0.1
    h = c0 * np.eye(n)
    D, info = cd.chebdm_density(handle, _dev(h), beta, mu, 64)
    torch.cuda.synchronize()
    occ = 1.0 / (1.0 + math.exp(beta * (c0 - mu)))
    assert np.max(np.abs(D.cpu().numpy() - occ * np.eye(n))) <= 1e-15


def test_power_form_refuses_reduced_precision(cd, handle):
    h, _, _ = synth.hamiltonian(32, "uniform", seed=2)
    with pytest.raises(cd.ChebdmError) as e:
        cd.chebdm_density(handle, _dev(h), 10.0, 0.0, 20, cd.make_opts("fp32", "power"))
    assert e.value.code == -6


# ------------------------------------------------------------------ moments

@pytest.mark.parametrize("n,order,kov", [(256, 128, 0), (300, 257, 0), (100, 50, 4), (64, 5, 0)])
def test_moments_match_oracle(cd, handle, n, order, kov):
    _say(f"moments n={n} order={order}")
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=n + order)
    tau = cd.chebdm_moments(handle, _dev(h), order, cd.make_opts(k_override=kov))
    lo, hi = checked_bounds(h, gpu_bounds=cd.chebdm_bounds(handle, _dev(h)))
    ref = ch.moments_from_eigs(lam, lo, hi, order)
    assert tau[0] == n
    err = np.max(np.abs(tau - ref))
    _say(f"  max|tau - tau_oracle| = {err:.3e}")
    assert err <= 1e-11 * n


# ------------------------------------------------------------------ mu search

MU_CASES = [
    # n, law, order, beta, n_elec, form, search
    (256, "uniform", 128, 50.0, 128.0, "composition", "bisection"),     # the N = 256 reference workload
    (256, "uniform", 128, 50.0, 128.0, "power", "bisection"),
    (300, "gaussmix6", 200, 80.0, 101.5, "composition", "bisection"),
    (520, "highdos", 255, 60.0, 260.0, "composition", "bisection"),
    (300, "gaussmix6", 200, 80.0, 101.5, "composition", "newton"),
    (520, "highdos", 255, 60.0, 260.0, "composition", "newton"),
    # giant steps forced to one chain, or to two chains (m = 4, 5 and 10: the smallest splits)
    (256, "uniform", 128, 50.0, 128.0, "one_chain", "bisection"),
    (200, "uniform", 15, 20.0, 100.5, "two_chains", "bisection"),
    (200, "gaussmix6", 24, 20.0, 100.5, "two_chains", "bisection"),
    (333, "highdos", 99, 40.0, 166.5, "two_chains", "newton"),
    # four chains: m = 8, 9 (last chain a single block), 10, and 23
    (200, "uniform", 63, 20.0, 100.5, "four_chains", "bisection"),
    (200, "gaussmix6", 80, 20.0, 100.5, "four_chains", "bisection"),
    (257, "highdos", 99, 40.0, 128.5, "four_chains", "newton"),
    (300, "gaussmix6", 512, 80.0, 150.5, "four_chains", "bisection"),
    # the search's node window at both extremes: beta' ~ 10 (every node inside) and ~ 10^4
    (300, "uniform", 64, 1.0, 150.5, "composition", "bisection"),
    (400, "highdos", 1024, 400.0, 200.5, "composition", "newton"),
]


@pytest.mark.parametrize("case", MU_CASES, ids=[f"n{c[0]}-L{c[2]}-{c[5]}-{c[6]}" for c in MU_CASES])
def test_mu_search_matches_oracle(cd, handle, case):
    n, law, order, beta, ne, form, search = case
    _say(f"mu_search {case}")
    h, q, lam = synth.hamiltonian(n, law, seed=2000 + n)
    mu, D, info = cd.chebdm_mu_search(handle, _dev(h), beta, ne, order, cd.make_opts("fp64", form, search=search))
    if search == "newton":
        _, _, info_b = cd.chebdm_mu_search(handle, _dev(h), beta, ne, order, cd.make_opts("fp64", form),
                                           want_density=False)
        _say(f"  evaluations: newton {info['iters']} vs bisection {info_b['iters']}")
        assert info["iters"] < info_b["iters"]
    torch.cuda.synchronize()
    assert info["status"] == 0, info
    emin, emax = checked_bounds(h, info)
    cen, a = ch.scaling(emin, emax)
    M = checked_quadrature(order, beta, emin, emax, info)
    ref, c = _oracle_density(q, lam, order, beta, mu, emin, emax, M)
    tau = ch.moments_from_eigs(lam, emin, emax, order)
    t_or = ch.trace_of_series(c, tau)
    err = np.max(np.abs(D.cpu().numpy() - ref))
    _say(f"  mu={mu:.15f} iters={info['iters']} |t_gpu-Ne|={info['trace_err']:.2e} "
         f"|t_oracle(mu)-Ne|={abs(t_or - ne):.2e} |trD-Ne|={abs(info['trace'] - ne):.2e} maxerr={err:.2e}")
    assert info["trace_err"] < 1e-10
    assert abs(t_or - ne) <= 1e-9
    assert abs(info["trace"] - ne) <= 1e-9
    assert err <= 1e-10
    # the oracle's own bisection lands on the same mu up to the flat-trace resolution
    mu_s, _, _, st = ch.bisect_mu(tau, order, beta * a, ne, 1e-10, M=M)
    slope = (ch.trace_of_series(ch.chebyshev_coeffs(order, beta * a, mu_s + 1e-7, M), tau)
             - ch.trace_of_series(ch.chebyshev_coeffs(order, beta * a, mu_s - 1e-7, M), tau)) / 2e-7
    assert abs((mu - cen) / a - mu_s) <= 4e-9 / slope + 1e-15


def test_mu_search_symmetric_spectrum_first_sweep(cd, handle):
    n = 128
    lam = synth.symmetric_pairs_spectrum(n, seed=4)
    h, q, lam = synth.hamiltonian(n, lam=lam, seed=4)
    mu, D, info = cd.chebdm_mu_search(handle, _dev(h), 30.0, n / 2, 64, None, -1.5, 1.5)
    assert info["iters"] == 1 and mu == 0.0
    mu, D, info = cd.chebdm_mu_search(handle, _dev(h), 30.0, n / 2, 64, cd.make_opts(search="newton"), -1.5, 1.5)
    assert info["iters"] == 1 and mu == 0.0


def test_mu_search_without_density(cd, handle):
    h, q, lam = synth.hamiltonian(200, "uniform", seed=6)
    mu1, D, info1 = cd.chebdm_mu_search(handle, _dev(h), 40.0, 77.0, 100, None, want_density=False)
    mu2, D2, info2 = cd.chebdm_mu_search(handle, _dev(h), 40.0, 77.0, 100, None)
    assert D is None and mu1 == mu2 and info1["iters"] == info2["iters"]
    assert info1["n_gemm"] < info2["n_gemm"]


def test_mu_search_errors_and_warnings(cd, handle):
    h, q, lam = synth.hamiltonian(64, "uniform", seed=9)
    H = _dev(h)
    with pytest.raises(cd.ChebdmError) as e:
        cd.chebdm_mu_search(handle, H, 10.0, 64.0, 32)
    assert e.value.code == -1
    with pytest.raises(cd.ChebdmError) as e:
        cd.chebdm_mu_search(handle, H, 10.0, 0.0, 32)
    assert e.value.code == -1
    # max_iter = 1 cannot reach 1e-10: the result is flagged, not an error
    mu, D, info = cd.chebdm_mu_search(handle, H, 10.0, 20.0, 32, cd.make_opts(max_iter=1))
    assert info["status"] == 1 and info["iters"] == 1
    # the bracket check fires when the requested count is outside (t(-1), t(1))
    with pytest.raises(cd.ChebdmError) as e:
        cd.chebdm_mu_search(handle, H, 10.0, 63.99, 4, None, -100.0, 100.0)
    assert e.value.code == -5


def test_mu_search_scalar_hamiltonian(cd, handle):
    n, c0, beta, ne = 40, -0.2, 5.0, 10.0
    mu, D, info = cd.chebdm_mu_search(handle, _dev(c0 * np.eye(n)), beta, ne, 16)
    occ = ne / n
    assert abs(1.0 / (1.0 + math.exp(beta * (c0 - mu))) - occ) < 1e-15
    assert np.max(np.abs(D.cpu().numpy() - occ * np.eye(n))) <= 1e-15


# ------------------------------------------------------- structure and options

@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_density_is_exactly_symmetric(cd, handle, prec):
    # only upper-triangle tiles are computed and mirrored: D == D^T bit for bit
    h, q, lam = synth.hamiltonian(333, "gaussmix6", seed=12)
    D, info = cd.chebdm_density(handle, _dev(h), 40.0, 0.0, 150, cd.make_opts(prec))
    torch.cuda.synchronize()
    d = D.cpu().numpy()
    assert np.array_equal(d, d.T)


@pytest.mark.parametrize("baby", ["stages", "sequential", "odd_chains"])
@pytest.mark.parametrize("n,order", [(256, 128), (700, 512), (300, 2048)])   # k = 12, 23, 46: chain steps 3, 5, 7
def test_baby_schedules_match_oracle(cd, handle, baby, n, order):
    _say(f"baby={baby} n={n} order={order}")
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=40 + n)
    D, info = cd.chebdm_density(handle, _dev(h), 100.0, 0.02, order, cd.make_opts("fp64", baby=baby))
    torch.cuda.synchronize()
    lo, hi = checked_bounds(h, info)
    ref, _ = _oracle_density(q, lam, order, 100.0, 0.02, lo, hi, checked_quadrature(order, 100.0, lo, hi, info))
    err = np.max(np.abs(D.cpu().numpy() - ref))
    _say(f"  max|D - D_oracle| = {err:.3e}")
    assert err <= 1e-10


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_reduced_precision_ladder_schedules(cd, handle, prec):
    # The mu search's ladder T_{lk} = T_l(T_k) runs in stages by default for float32 products
    # (baby steps in odd chains): both orders hold the moments to the reduced-precision bound
    # against the oracle, the default in 12 launches instead of 43 at a few times the sequential
    # order's moment error (measured 1.7e-4 against 5.4e-5: the staged launches of two to four
    # products run unsplit float32 48-tiles, whose K sums are one accumulator long; both two
    # orders of magnitude under the 1e-5 N bound).  The split-bf16 products keep the sequential
    # ladder by default (staged, their moment error grows about eightfold).
    n, order = 1000, 512
    _say(f"ladder schedules {prec} n={n} order={order}")
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=77)
    H = _dev(h)
    lo, hi = checked_bounds(h, gpu_bounds=cd.chebdm_bounds(handle, H))
    ref = ch.moments_from_eigs(lam, lo, hi, order)
    res = {}
    for baby in ("auto", "sequential"):
        cd.chebdm_profile_enable(handle, True)
        tau = cd.chebdm_moments(handle, H, order, cd.make_opts(prec, baby=baby))
        prof = cd.chebdm_profile_read(handle)
        cd.chebdm_profile_enable(handle, False)
        res[baby] = (float(np.max(np.abs(tau - ref))), prof["gemm_launches"], prof["gemm_products"])
        _say(f"  {baby:10s} max|tau - tau_oracle| = {res[baby][0]:.3e} in {res[baby][1]} launches "
             f"({res[baby][2]} products)")
    assert res["auto"][2] == res["sequential"][2]
    for err, _, _ in res.values():
        assert err <= 1e-5 * n
    if prec == "fp32":
        assert res["auto"][1] < res["sequential"][1]
        assert res["auto"][0] <= 4.0 * res["sequential"][0]
    else:
        assert res["auto"][:2] == res["sequential"][:2]


@pytest.mark.parametrize("order", [3, 8, 15, 24, 35])   # k = 2..6: the sequential fallback and the first chains
def test_odd_chains_small_orders_match_oracle(cd, handle, order):
    n = 150
    _say(f"odd chains n={n} order={order}")
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=60 + order)
    D, info = cd.chebdm_density(handle, _dev(h), 20.0, 0.05, order, cd.make_opts("fp64", baby="odd_chains"))
    torch.cuda.synchronize()
    lo, hi = checked_bounds(h, info)
    ref, _ = _oracle_density(q, lam, order, 20.0, 0.05, lo, hi, checked_quadrature(order, 20.0, lo, hi, info))
    err = np.max(np.abs(D.cpu().numpy() - ref))
    _say(f"  k={info['k']} max|D - D_oracle| = {err:.3e}")
    assert err <= 1e-10


@pytest.mark.parametrize("bounds", ["gershgorin", "lanczos"])
def test_float32_baby_schedules(cd, handle, bounds):
    # float32 baby steps default to odd chains: as accurate as the sequential order (within a
    # factor of 2) on loose and on tight bounds, in fewer launches
    n, order, beta, mu = 1000, 512, 100.0, 0.02
    _say(f"float32 baby schedules n={n} order={order} bounds={bounds}")
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=91)
    H = _dev(h)
    res = {}
    for baby in ("auto", "sequential"):
        cd.chebdm_profile_enable(handle, True)
        D, info = cd.chebdm_density(handle, H, beta, mu, order, cd.make_opts("fp32", baby=baby, bounds=bounds))
        prof = cd.chebdm_profile_read(handle)
        cd.chebdm_profile_enable(handle, False)
        gpu_b = (info["emin"], info["emax"])
        lo, hi = checked_bounds(h, gpu_bounds=gpu_b) if bounds == "gershgorin" else checked_lanczos_bounds(h, gpu_b)
        ref, _ = _oracle_density(q, lam, order, beta, mu, lo, hi, checked_quadrature(order, beta, lo, hi, info))
        res[baby] = (float(np.max(np.abs(D.cpu().numpy() - ref))), prof["gemm_launches"], prof["gemm_products"])
        _say(f"  {baby:10s} max|D - D_oracle| = {res[baby][0]:.3e} in {res[baby][1]} launches")
    assert res["auto"][2] == res["sequential"][2] and res["auto"][1] < res["sequential"][1]
    assert res["auto"][0] <= 1e-5 and res["sequential"][0] <= 1e-5
    assert res["auto"][0] <= 2.0 * res["sequential"][0]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_stream_k_products_match_oracle(cd, handle, prec, tol):
    # n = 1530: 300 64-tiles per product with a ragged edge (1530 = 23 * 64 + 58), so launches of
    # one to nine products run as stream-K (K pieces shared between work-groups, summed by the
    # fix-up launch); the whole D is held to the precision's bound against the oracle
    n, order, beta = 1530, 120, 60.0
    _say(f"stream-K products n={n} order={order} {prec}")
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=1530)
    mu, D, info = cd.chebdm_mu_search(handle, _dev(h), beta, n / 2 + 0.5, order, cd.make_opts(prec))
    torch.cuda.synchronize()
    assert info["status"] == 0
    lo, hi = checked_bounds(h, info)
    ref, _ = _oracle_density(q, lam, order, beta, mu, lo, hi, checked_quadrature(order, beta, lo, hi, info))
    err = float(np.max(np.abs(D.cpu().numpy() - ref)))
    _say(f"  mu={mu:.12f} max|D - D_oracle| = {err:.3e}")
    assert err <= tol
    Dn = D.cpu().numpy()
    assert np.array_equal(Dn, Dn.T)


def test_profile_counts_products(cd, handle):
    h, q, lam = synth.hamiltonian(300, "uniform", seed=31)
    H = _dev(h)
    cd.chebdm_profile_enable(handle, True)
    mu, D, info = cd.chebdm_mu_search(handle, H, 50.0, 150.0, 128)
    prof = cd.chebdm_profile_read(handle)
    cd.chebdm_profile_enable(handle, False)
    assert prof["gemm_products"] == info["n_gemm"]
    assert prof["gemm_flop"] == info["n_gemm"] * 300.0 * 300.0 * 301.0
    assert prof["gemm_ms"] > 0 and prof["combine_calls"] == 1 and prof["gram_calls"] == 1
    # read clears the counters
    assert cd.chebdm_profile_read(handle)["gemm_launches"] == 0


def test_replayed_graph_matches_eager_and_tracks_arguments(cd, handle):
    # the device part of a call is captured once and replayed while its arguments are unchanged;
    # launch timing forces the eager path, which must agree bit for bit
    h, q, lam = synth.hamiltonian(333, "gaussmix6", seed=44)
    H = _dev(h)
    D1 = torch.empty_like(H)
    mu1, _, i1 = cd.chebdm_mu_search(handle, H, 40.0, 150.5, 200, None, D=D1)       # capture
    D2 = torch.empty_like(H)
    mu2, _, i2 = cd.chebdm_mu_search(handle, H, 40.0, 150.5, 200, None, D=D2)       # new D pointer: capture
    mu3, _, i3 = cd.chebdm_mu_search(handle, H, 40.0, 150.5, 200, None, D=D2)       # replay
    cd.chebdm_profile_enable(handle, True)
    D4 = torch.empty_like(H)
    mu4, _, i4 = cd.chebdm_mu_search(handle, H, 40.0, 150.5, 200, None, D=D4)       # eager
    cd.chebdm_profile_read(handle)
    cd.chebdm_profile_enable(handle, False)
    assert mu1 == mu2 == mu3 == mu4
    assert torch.equal(D1, D2) and torch.equal(D1, D4)
    assert i1["n_gemm"] == i3["n_gemm"] == i4["n_gemm"] and i3["iters"] == i4["iters"]
    # new contents under the same pointer, same arguments (a replay): H + I/2 moves the bounds,
    # which the replayed graph reads on the device, and mu by 1/2; D is unchanged
    H.add_(0.5 * torch.eye(333, dtype=torch.float64, device=H.device))
    mu5, _, i5 = cd.chebdm_mu_search(handle, H, 40.0, 150.5, 200, None, D=D2)
    assert abs(mu5 - (mu1 + 0.5)) <= 1e-9
    assert float(torch.max(torch.abs(D2 - D1))) <= 1e-9
    # a different electron count changes the key
    mu6, _, i6 = cd.chebdm_mu_search(handle, H, 40.0, 100.5, 200, None, D=D2)
    assert mu6 < mu5 and abs(i6["trace"] - 100.5) <= 1e-9
    # density at fixed mu: replay equals eager
    Da = torch.empty_like(H)
    cd.chebdm_density(handle, H, 40.0, mu5, 200, None, D=Da)
    cd.chebdm_density(handle, H, 40.0, mu5, 200, None, D=Da)
    cd.chebdm_profile_enable(handle, True)
    Db = torch.empty_like(H)
    cd.chebdm_density(handle, H, 40.0, mu5, 200, None, D=Db)
    cd.chebdm_profile_read(handle)
    cd.chebdm_profile_enable(handle, False)
    assert torch.equal(Da, Db)


def test_bounds_survive_scalar_workspace_growth(cd):
    # a fresh handle sized by a small quadrature, then a call whose quadrature needs a larger
    # workspace: the Gershgorin bounds computed before the growth must carry over
    h2 = cd.Handle(0)
    try:
        hm, q, lam = synth.hamiltonian(300, "uniform", seed=61)
        H = _dev(hm)
        cd.chebdm_mu_search(h2, H, 5.0, 150.5, 64, None)                       # small M
        mu, D, info = cd.chebdm_mu_search(h2, H, 400.0, 150.5, 256, None)      # M grows
        assert info["status"] == 0, info
        emin, emax = checked_bounds(hm, info)
        cen, a = ch.scaling(emin, emax)
        c = ch.chebyshev_coeffs(256, 400.0 * a, (mu - cen) / a, checked_quadrature(256, 400.0, emin, emax, info))
        t_or = ch.trace_of_series(c, ch.moments_from_eigs(lam, emin, emax, 256))
        assert abs(t_or - 150.5) <= 1e-9
    finally:
        h2.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_jackson_damping_matches_oracle(cd, handle, prec, tol):
    n, order, beta, ne = 260, 150, 60.0, 120.5
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=77)
    mu, D, info = cd.chebdm_mu_search(handle, _dev(h), beta, ne, order, cd.make_opts(prec, damping="jackson"))
    assert info["status"] == 0
    emin, emax = checked_bounds(h, info)
    cen, a = ch.scaling(emin, emax)
    c = ch.chebyshev_coeffs(order, beta * a, (mu - cen) / a, checked_quadrature(order, beta, emin, emax, info),
                            "jackson")
    ref = ch.density_from_eigs(q, lam, c, emin, emax)
    err = float(np.max(np.abs(D.cpu().numpy() - ref)))
    t_or = ch.trace_of_series(c, ch.moments_from_eigs(lam, emin, emax, order))
    _say(f"  jackson {prec}: err={err:.2e} |t_oracle-Ne|={abs(t_or - ne):.2e}")
    assert err <= tol
    assert abs(t_or - ne) <= (1e-9 if prec == "fp64" else 1e-5 * n)
    # the damped occupations stay in [0, 1]: D's eigenvalues p_J(lam~) are in [0, 1]
    p = ch.cheb_eval(c, (lam - cen) / a)
    assert p.min() > -1e-12 and p.max() < 1 + 1e-12


# ------------------------------------------------------------------ commutator check

@pytest.mark.parametrize("n", [1, 70, 300, 1000])
def test_commutator_norm_matches_oracle(cd, handle, n):
    _say(f"commutator n={n}")
    rng = np.random.default_rng(n)
    h, _, _ = synth.hamiltonian(n, "uniform", seed=40 + n)
    d = rng.normal(size=(n, n))
    d = (d + d.T) / 2
    got = cd.chebdm_commutator_norm(handle, _dev(h), _dev(d))
    ref = ch.commutator_max(h, d)
    scale = n * np.max(np.abs(h)) * np.max(np.abs(d))
    _say(f"  max|HD-DH| gpu {got:.15e} oracle {ref:.15e}")
    assert abs(got - ref) <= 1e-14 * scale


def test_commutator_of_expansion_is_rounding_level(cd, handle):
    n, ld = 500, 640
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=9)
    big = torch.zeros((n, ld), dtype=torch.float64, device="cuda:0")
    big[:, :n] = _dev(h)
    H = big[:, :n]
    mu, D, info = cd.chebdm_mu_search(handle, H, 60.0, n / 2, 256)
    got = cd.chebdm_commutator_norm(handle, H, D)
    ref = ch.commutator_max(h, D.cpu().numpy())
    _say(f"  ||[H, D_L]||_max gpu {got:.3e} oracle {ref:.3e}")
    assert got < 1e-11 and abs(got - ref) <= 1e-12
    # a matrix that is not a function of H is flagged
    E = D.clone()
    E[0, 1] += 1e-3
    E[1, 0] += 1e-3
    assert cd.chebdm_commutator_norm(handle, H, E) > 1e-5
    bad = D.clone()
    bad[2, 3] = float("nan")
    assert math.isnan(cd.chebdm_commutator_norm(handle, H, bad))


# ------------------------------------------------------------------ tight-binding model inputs

@pytest.mark.parametrize("bounds", ["gershgorin", "lanczos"])
@pytest.mark.parametrize("kind", ["metal", "semiconductor", "softmatter", "metal_accuracy"])
def test_mu_search_tight_binding(cd, handle, kind, bounds):
    # the paper's model-Hamiltonian family (Sec. III.C); the oracle diagonalises H itself
    n, order, beta = 601, 256, 20.0
    ne = n / 2
    _say(f"tight-binding {kind} bounds={bounds}")
    h = synth.tight_binding(n, kind, seed=11)
    lam, q = np.linalg.eigh(h)
    mu, D, info = cd.chebdm_mu_search(handle, _dev(h), beta, ne, order, cd.make_opts(bounds=bounds))
    assert info["status"] == 0, info
    gpu_b = (info["emin"], info["emax"])
    emin, emax = checked_bounds(h, gpu_bounds=gpu_b) if bounds == "gershgorin" else checked_lanczos_bounds(h, gpu_b)
    assert emin <= lam.min() and lam.max() <= emax
    cen, a = ch.scaling(emin, emax)
    c = ch.chebyshev_coeffs(order, beta * a, (mu - cen) / a, checked_quadrature(order, beta, emin, emax, info))
    err = float(np.max(np.abs(D.cpu().numpy() - ch.density_from_eigs(q, lam, c, emin, emax))))
    t_or = ch.trace_of_series(c, ch.moments_from_eigs(lam, emin, emax, order))
    _say(f"  [{emin:.3f}, {emax:.3f}] beta'={beta * a:.0f} mu={mu:.10f} |t_oracle-Ne|={abs(t_or - ne):.1e} "
         f"max|D-D_oracle|={err:.1e}")
    assert err <= 1e-10
    assert abs(t_or - ne) <= 1e-9


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1e-5), ("bf16x3", 2e-5)])
def test_one_and_two_giant_chains_agree(cd, handle, prec, tol):
    # same polynomial, different association: D agrees to rounding; same product count
    n, order, beta = 700, 512, 100.0
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=2000)
    H = _dev(h)
    out = {}
    for form in ("one_chain", "two_chains", "four_chains"):
        mu, D, info = cd.chebdm_mu_search(handle, H, beta, n / 2, order, cd.make_opts(prec, form))
        out[form] = (mu, D.cpu().numpy(), info)
    mu1, d1, i1 = out["one_chain"]
    for form in ("two_chains", "four_chains"):
        mu2, d2, i2 = out[form]
        assert mu1 == mu2 and i1["n_gemm"] == i2["n_gemm"] and i1["iters"] == i2["iters"]
        err = float(np.max(np.abs(d1 - d2)))
        _say(f"  {prec}: max|D_one - D_{form}| = {err:.2e}, n_gemm {i1['n_gemm']}")
        assert err <= tol

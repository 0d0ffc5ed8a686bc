"""GPU parity of the reduced-precision products and of the full-size workloads.

Reduced precision (float32 MFMA, split-bf16 "bf16x3"): the products run in
lower precision while bounds, coefficients, traces and the bisection stay
float64.  The error is measured against the float64 oracle at the *same*
chemical potential, so it isolates the products; the target is a max-abs
error of 1e-5 for both forms.

Full size: the benchmark shapes (N = 1000/2000/4000, order 512; N = 5000,
order 2048) are compared on the whole D, which the oracle forms from the
generator's eigenpairs as Q diag(p(lam~)) Q^T.  Every reference uses the
oracle's own Gershgorin bounds and quadrature size, after asserting that the
GPU's agree with them.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import chebyshev as ch
from refcheck import checked_bounds, checked_quadrature, density, trace_error

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


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("n,law,order,beta", [(256, "uniform", 128, 50.0), (520, "gaussmix6", 255, 60.0),
                                              (700, "highdos", 512, 100.0)])
def test_reduced_precision_density(cd, handle, prec, n, law, order, beta):
    _say(f"density {prec} n={n} order={order}")
    h, q, lam = synth.hamiltonian(n, law, seed=3000 + n)
    mu = 0.05
    D, info = cd.chebdm_density(handle, _dev(h), beta, mu, order, cd.make_opts(prec))
    torch.cuda.synchronize()
    lo, hi = checked_bounds(h, info)
    M = checked_quadrature(order, beta, lo, hi, info)
    ref, _ = density(q, lam, order, beta, mu, lo, hi, M)
    err = float(np.max(np.abs(D.cpu().numpy() - ref)))
    _say(f"  max|D_{prec} - D_oracle| = {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_reduced_precision_mu_search(cd, handle, prec):
    n, order, beta, ne = 300, 200, 80.0, 150.0
    _say(f"mu_search {prec}")
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=77)
    mu, D, info = cd.chebdm_mu_search(handle, _dev(h), beta, ne, order, cd.make_opts(prec))
    torch.cuda.synchronize()
    lo, hi = checked_bounds(h, info)
    M = checked_quadrature(order, beta, lo, hi, info)
    ref, c = density(q, lam, order, beta, mu, lo, hi, M)
    t_err = trace_error(lam, c, lo, hi, order, ne)
    err = float(np.max(np.abs(D.cpu().numpy() - ref)))
    _say(f"  |t_oracle(mu_{prec}) - Ne| = {t_err:.3e}  iters={info['iters']}  max|D - D_oracle| = {err:.3e}")
    assert err <= 1e-5
    # moments from reduced-precision matrices: electron count within 1e-5 * N
    assert t_err <= 1e-5 * n
    assert abs(info["trace"] - ne) <= 1e-5 * n


BF16X3_CONFIG4 = ("the three-term split (hi*hi + hi*lo + lo*hi) carries about 16 bits per product; over the "
                  "132 products of order 2048 at beta' ~ 1e4 it ends near 5e-5, above the 1e-5 target: the "
                  "six-term split (bf16x6) is the split-bf16 form for this shape")

FULL = [
    # n, law, order, beta, prec, seed
    (1000, "gaussmix6", 512, 100.0, "fp64", 2000),
    (2000, "gaussmix6", 512, 100.0, "fp64", 2001),
    (4000, "gaussmix6", 512, 100.0, "fp64", 2002),
    (1000, "gaussmix6", 512, 100.0, "fp32", 2000),
    (2000, "gaussmix6", 512, 100.0, "fp32", 2001),
    (4000, "gaussmix6", 512, 100.0, "fp32", 2002),
    (1000, "gaussmix6", 512, 100.0, "bf16x3", 2000),
    (2000, "gaussmix6", 512, 100.0, "bf16x3", 2001),
    (4000, "gaussmix6", 512, 100.0, "bf16x3", 2002),
    (4000, "gaussmix6", 512, 100.0, "bf16x6", 2002),
    (1800, "uniform", 512, 100.0, "bf16x3", 2003),     # LDS-staged split products, ragged 128-tiles
    (5000, "highdos", 2048, 400.0, "fp64", 4000),
    (5000, "highdos", 2048, 400.0, "fp32", 4000),
    (5000, "highdos", 2048, 400.0, "bf16x6", 4000),
    pytest.param((5000, "highdos", 2048, 400.0, "bf16x3", 4000), id="n5000-L2048-bf16x3",
                 marks=pytest.mark.xfail(strict=True, reason=BF16X3_CONFIG4)),
]


def _case_id(c):
    return f"n{c[0]}-L{c[2]}-{c[4]}"


@pytest.mark.parametrize("case", FULL, ids=_case_id)
def test_full_size_mu_search_whole_density(cd, handle, case):
    # the whole D against the oracle's Q diag(p) Q^T: every tile of every launch shape the
    # library picks at these sizes (full rounds, tail-split slices, stream-K pieces, LDS tiles)
    n, law, order, beta, prec, seed = case
    _say(f"full-size mu_search {case}")
    h, q, lam = synth.hamiltonian(n, law, seed=seed)
    mu, D, info = cd.chebdm_mu_search(handle, _dev(h), beta, n / 2, order, cd.make_opts(prec))
    torch.cuda.synchronize()
    lo, hi = checked_bounds(h, info)
    M = checked_quadrature(order, beta, lo, hi, info)
    ref, c = density(q, lam, order, beta, mu, lo, hi, M)
    d = D.cpu().numpy()
    del D
    err = float(np.max(np.abs(d - ref)))
    t_err = trace_error(lam, c, lo, hi, order, n / 2)
    _say(f"  status={info['status']} iters={info['iters']} max|D-D_oracle|={err:.3e} "
         f"|t_oracle(mu)-Ne|={t_err:.3e} |trD-Ne|={abs(info['trace'] - n / 2):.3e}")
    assert np.array_equal(d, d.T)
    if prec == "fp64":
        assert info["status"] == 0 and err <= 1e-10 and t_err <= 1e-8
    else:
        assert err <= 1e-5 and t_err <= 1e-5 * n


def test_six_term_split_grouped_stage_launches(cd, handle):
    # Algorithm-1 stages put several products in one launch: at this size the six-term
    # split then runs on the LDS-staged kernel (ragged 128-tiles: 1800 = 14 * 128 + 8)
    n, order, beta, seed = 1800, 512, 100.0, 2004
    h, q, lam = synth.hamiltonian(n, "gaussmix6", seed=seed)
    mu, D, info = cd.chebdm_mu_search(handle, _dev(h), beta, n / 2, order, cd.make_opts("bf16x6", baby="stages"))
    torch.cuda.synchronize()
    lo, hi = checked_bounds(h, info)
    M = checked_quadrature(order, beta, lo, hi, info)
    ref, _ = density(q, lam, order, beta, mu, lo, hi, M)
    err = float(np.max(np.abs(D.cpu().numpy() - ref)))
    _say(f"  bf16x6 stages n={n}: max|D-D_oracle|={err:.3e} status={info['status']}")
    assert err <= 1e-5
    assert abs(info["trace"] - n / 2) <= 1e-5 * n

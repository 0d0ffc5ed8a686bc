"""Accuracy against the order (float64, GPU), the analogue of the paper's truncation study
(Sec. III.D): distance of D_L to the exact Fermi operator on the high-density-of-states
spectrum at beta = 400, mu = 0, for the spectrum's own extremes, Lanczos and Gershgorin bounds.

Each GPU density is first held to the float64 target (1e-10) against the oracle at the same
bounds and order; the claims are then checked on the oracle-verified values: the error falls
exponentially once L exceeds beta' (spectrum bounds: below 1e-6 at L = 2048, a 100-fold drop
from L = 512), and at every order the tighter interval is the more accurate one.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import chebyshev as ch
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


def test_error_against_order_and_bounds(cd, handle):
    n, beta, mu = 300, 400.0, 0.0
    orders = (128, 512, 2048)
    h, q, lam = synth.hamiltonian(n, "highdos", seed=4001)
    H = torch.from_numpy(h).to("cuda:0")
    exact = ch.fermi_dirac_density(q, lam, beta, mu)
    # the oracle's bounds, after checking the library's against them; both sides then take them
    bounds = {"spectrum": (float(lam.min()), float(lam.max())),
              "lanczos": checked_lanczos_bounds(h, cd.chebdm_bounds_lanczos(handle, H, 40, 0.01, 0)[:2]),
              "gershgorin": checked_bounds(h, gpu_bounds=cd.chebdm_bounds(handle, H))}
    err = {}
    for name, (lo, hi) in bounds.items():
        cen, a = ch.scaling(lo, hi)
        err[name] = []
        for L in orders:
            D, info = cd.chebdm_density(handle, H, beta, mu, L, cd.make_opts("fp64"), lo, hi)
            d = D.cpu().numpy()
            c = ch.chebyshev_coeffs(L, beta * a, (mu - cen) / a, checked_quadrature(L, beta, lo, hi, info))
            parity = float(np.max(np.abs(d - ch.density_from_eigs(q, lam, c, lo, hi))))
            assert parity <= 1e-10, (name, L, parity)
            err[name].append(float(np.max(np.abs(d - exact))))
        _say(f"  {name:10s} beta'={beta * a:8.1f} max|D_L - f(H)| at L={orders}: "
             + " ".join(f"{e:.2e}" for e in err[name]))
    s, lz, g = err["spectrum"], err["lanczos"], err["gershgorin"]
    assert s[2] < 1e-6 and s[2] < 0.01 * s[1] and s[1] < s[0]
    for i in range(len(orders)):
        assert s[i] <= lz[i] <= g[i]
    assert g[2] > 1e-3   # beta' ~ 6000 on Gershgorin's interval: L = 2048 is far too short

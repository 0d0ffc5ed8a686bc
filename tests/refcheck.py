"""Oracle-side references for the GPU parity tests.

Every end-to-end reference is built from quantities the oracle computes
itself: Gershgorin bounds of the stored H, the quadrature size from the
oracle's rule, coefficients at the GPU's mu, and D = Q diag(p(lam~)) Q^T
from the generator's eigenpairs (or LAPACK's, where the generator has none).
The GPU's own bounds and quadrature size are asserted against the oracle's
before anything is compared, so a wrong bound cannot leak into a reference.
The spectrum map through the extreme eigenvalues is the paper's Sec. II.B.
"""
import numpy as np

from oracle import chebyshev as ch

BOUNDS_REL = 1e-13   # single reductions summed in another order


def checked_bounds(h, info=None, gpu_bounds=None, rel=BOUNDS_REL):
    """Oracle Gershgorin bounds of h, after asserting the GPU's agree to `rel` of their scale."""
    lo, hi = ch.gershgorin_bounds(h)
    got = gpu_bounds if gpu_bounds is not None else (info["emin"], info["emax"])
    scale = max(abs(lo), abs(hi), 1e-300)
    assert abs(got[0] - lo) <= rel * scale and abs(got[1] - hi) <= rel * scale, (got, (lo, hi))
    return lo, hi


def checked_lanczos_bounds(h, gpu_bounds, steps=40, margin=0.01, seed=0, rel=1e-10):
    """Oracle Lanczos bounds after asserting the GPU's agree to `rel` of the Gershgorin scale."""
    lo, hi, _, _ = ch.lanczos_bounds(h, steps, margin, seed)
    g_lo, g_hi = ch.gershgorin_bounds(h)
    scale = max(abs(g_lo), abs(g_hi))
    assert abs(gpu_bounds[0] - lo) <= rel * scale and abs(gpu_bounds[1] - hi) <= rel * scale, (gpu_bounds, (lo, hi))
    return lo, hi


def checked_quadrature(order, beta, lo, hi, info=None):
    """The oracle's quadrature size M for these bounds; the GPU must have used the same."""
    _, a = ch.scaling(lo, hi)
    M = ch.quadrature_size(order, beta * a)
    if info is not None:
        assert info["n_quad"] == M, (info["n_quad"], M)
    return M


def coeffs(order, beta, mu, lo, hi, M, damping=None):
    cen, a = ch.scaling(lo, hi)
    return ch.chebyshev_coeffs(order, beta * a, (mu - cen) / a, M, damping)


def density(q, lam, order, beta, mu, lo, hi, M, rows=None, damping=None):
    """D_L (or its rows) at mu from eigenpairs: Q[rows] diag(p_L(lam~)) Q^T."""
    c = coeffs(order, beta, mu, lo, hi, M, damping)
    cen, a = ch.scaling(lo, hi)
    p = ch.cheb_eval(c, (lam - cen) / a)
    qr = q if rows is None else q[rows]
    return (qr * p) @ q.T, c


def trace_error(lam, c, lo, hi, order, n_elec):
    """|t_oracle(mu) - N_e| with the moments from the exact spectrum."""
    return abs(ch.trace_of_series(c, ch.moments_from_eigs(lam, lo, hi, order)) - n_elec)


def band_rows(n, band=64):
    """One row per `band`-row band (first, middle and last of alternating bands), always including
    rows 0 and n - 1, so every tile row of the products' grids is represented."""
    rows = set([0, n - 1])
    for b, start in enumerate(range(0, n, band)):
        stop = min(start + band, n)
        rows.add(start + (b % 3) * (stop - 1 - start) // 2)
    return np.array(sorted(rows))

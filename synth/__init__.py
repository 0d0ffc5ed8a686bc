"""Seeded synthetic Hamiltonians shared by the oracle and the HIP path.

This module only draws inputs.  It holds none of the method's arithmetic
(no Chebyshev polynomials, no Fermi function, no bounds): both the oracle and
the GPU path receive the same matrices from here and compute independently.

The paper benchmarks on tight-binding model Hamiltonians (Sec. III.C) that are
not available; these generators stand in for them.  Every matrix is
``H = Q diag(lam) Q^T`` with a Haar-random orthogonal ``Q`` and a chosen
eigenvalue law, so the exact spectrum is known.  The eigenvalue laws:

``uniform``    lam ~ U[-1, 1]                             (gap-free, flat DOS)
``gaussmix6``  six equal-weight Gaussians, means -0.75..0.75 in steps of 0.3,
               sigma 0.15 (overlapping, so gap-free; metallic-like)
``highdos``    40 % ~ N(0, 0.01^2), 60 % ~ U[-1, 1]  (high DOS at the Fermi
               level, the hard case of the accuracy study, Sec. III.D)

Recipe (seeded, PCG64): draw lam first, then G (n x n standard normal),
Q = qr(G) with the signs of diag(R) folded in (Haar measure), then
H = (Q * lam) @ Q^T in float64, symmetrised exactly as (H + H^T) / 2.
"""
from __future__ import annotations

import numpy as np

LAWS = ("uniform", "gaussmix6", "highdos")


def eigenvalues(law: str, n: int, rng: np.random.Generator) -> np.ndarray:
    """Draw ``n`` eigenvalues from one of ``LAWS`` (unsorted, float64)."""
    if law == "uniform":
        return rng.uniform(-1.0, 1.0, size=n)
    if law == "gaussmix6":
        means = -0.75 + 0.3 * np.arange(6)
        comp = rng.integers(0, 6, size=n)
        return means[comp] + 0.15 * rng.standard_normal(n)
    if law == "highdos":
        n_peak = int(round(0.4 * n))
        lam = np.concatenate([0.01 * rng.standard_normal(n_peak),
                              rng.uniform(-1.0, 1.0, size=n - n_peak)])
        return lam[rng.permutation(n)]
    raise ValueError(f"unknown eigenvalue law {law!r}; expected one of {LAWS}")


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian, signs of diag(R) folded in."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))


def hamiltonian(n: int, law: str = "uniform", seed: int = 0,
                lam: np.ndarray | None = None):
    """Return ``(H, Q, lam)`` with ``H = Q diag(lam) Q^T`` (float64, exactly symmetric).

    ``lam`` overrides the law (used for symmetric-spectrum and diagonal cases).
    """
    rng = np.random.default_rng(seed)
    if lam is None:
        lam = eigenvalues(law, n, rng)
    lam = np.asarray(lam, dtype=np.float64)
    q = haar_orthogonal(n, rng)
    h = (q * lam) @ q.T
    h = 0.5 * (h + h.T)
    return np.ascontiguousarray(h), q, lam


def symmetric_pairs_spectrum(n: int, seed: int = 0) -> np.ndarray:
    """Eigenvalues in exact +/- pairs (n even): a spectrum symmetric about zero."""
    if n % 2:
        raise ValueError("symmetric_pairs_spectrum needs an even n")
    rng = np.random.default_rng(seed)
    half = rng.uniform(0.05, 1.0, size=n // 2)
    return np.concatenate([half, -half])


def batch_problems(count: int, seed: int = 3000, n_lo: int = 96, n_hi: int = 1024,
                   step: int = 32, beta_lo: float = 30.0, beta_hi: float = 200.0):
    """Sizes and inverse temperatures of a batch of uneven-N problems.

    N ~ U{n_lo, n_lo+step, ..., n_hi}, beta ~ U[beta_lo, beta_hi]; returns two arrays.
    """
    rng = np.random.default_rng(seed)
    sizes = rng.integers(0, (n_hi - n_lo) // step + 1, size=count) * step + n_lo
    betas = rng.uniform(beta_lo, beta_hi, size=count)
    return sizes.astype(np.int64), betas

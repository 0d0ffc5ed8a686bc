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


def _cholesky_qr2(torch, g, chunk: int = 16):
    """Orthogonal factor of G (positive-diagonal R) by two Cholesky QR passes; None on failure.

    The triangular solves run ``chunk`` matrices at a time (the batched BLAS
    solve asks for workspace in proportion to the batch).
    """
    q = g
    for _ in range(2):
        a = torch.matmul(q.transpose(-1, -2).contiguous(), q)
        low, info = torch.linalg.cholesky_ex(a)
        if bool((info != 0).any()):
            return None
        up = low.transpose(-1, -2).contiguous()
        q = torch.cat([torch.linalg.solve_triangular(up[i:i + chunk], q[i:i + chunk], upper=True, left=False)
                       for i in range(0, q.shape[0], chunk)])
    return q


def hamiltonians_torch(sizes, law: str = "uniform", seed: int = 0, device="cuda"):
    """Many Hamiltonians assembled on ``device`` with torch (same recipe, faster at scale).

    The eigenvalues come from numpy's PCG64 (``seed``), in the order of
    ``sizes``; the Gaussian matrices from a torch generator on ``device``
    seeded with ``seed``, drawn size group by size group in increasing n.
    Q is the orthogonal factor of G with a positive diagonal R (the Haar
    measure, as in :func:`haar_orthogonal`), computed by Cholesky QR applied
    twice (R^T R = G^T G, Q = G R^-1, then once more on Q: orthogonal to
    rounding, and much faster on a GPU than a Householder QR of many small
    matrices); a group whose Cholesky factorisation fails falls back to
    Householder QR.  H = (Q * lam) Q^T in float64, symmetrised exactly.
    Returns a list of ``(H, lam)`` with H a contiguous float64 device tensor
    and lam a numpy array.
    """
    import torch

    sizes = [int(n) for n in sizes]
    rng = np.random.default_rng(seed)
    lams = [eigenvalues(law, n, rng) for n in sizes]
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    out = [None] * len(sizes)
    for n in sorted(set(sizes)):
        idx = [i for i, v in enumerate(sizes) if v == n]
        g = torch.randn((len(idx), n, n), generator=gen, device=device, dtype=torch.float64)
        q = _cholesky_qr2(torch, g)
        if q is None:
            q, r = torch.linalg.qr(g)
            q = q * torch.sign(torch.diagonal(r, dim1=-2, dim2=-1)).unsqueeze(-2)
            del r
        del g
        lam = torch.from_numpy(np.stack([lams[i] for i in idx])).to(device)
        h = torch.matmul(q * lam.unsqueeze(-2), q.transpose(-1, -2).contiguous())
        h = 0.5 * (h + h.transpose(-1, -2))
        for j, i in enumerate(idx):
            out[i] = (h[j].contiguous(), lams[i])
        del q, h, lam
    return out


def mu_problems(sizes, seed: int, device="cuda"):
    """Problems of the learned-mu workload for the given sizes.

    Per problem: eigenvalue law uniform over ``LAWS``, beta ~ U[30, 200],
    electron fraction f ~ U[0.3, 0.7] with N_e = round(f n) + 1/2.  The
    Hamiltonians come from :func:`hamiltonians_torch` (one seed per law).
    Returns ``(Hs, lams, betas, n_elecs)``.
    """
    sizes = [int(n) for n in sizes]
    count = len(sizes)
    rng = np.random.default_rng(seed)
    law_of = rng.integers(0, len(LAWS), size=count)
    betas = rng.uniform(30.0, 200.0, size=count)
    frac = rng.uniform(0.3, 0.7, size=count)
    n_elecs = [float(np.round(f * n)) + 0.5 for f, n in zip(frac, sizes)]
    Hs, lams = [None] * count, [None] * count
    for li, law in enumerate(LAWS):
        idx = [i for i in range(count) if law_of[i] == li]
        if not idx:
            continue
        made = hamiltonians_torch([sizes[i] for i in idx], law, seed=8 * seed + li, device=device)
        for i, (h, lam) in zip(idx, made):
            Hs[i], lams[i] = h, lam
    return Hs, lams, betas, n_elecs


def mu_training_sizes(count: int, seed: int = 100):
    """Training sizes of the learned-mu workload: n ~ U{64, 80, ..., 512}."""
    return 64 + 16 * np.random.default_rng(seed).integers(0, 29, size=count)


# ---------------------------------------------------------------------------
# two-level tight-binding model Hamiltonians (Sec. III.C, the paper's workload family)

TB_KINDS = {
    # alpha (A-A), beta (B-B), gamma (A-B), eps_a, eps_b, decay k, noise amplitude r
    "metal": dict(alpha=-1.0, beta=-1.0, gamma=0.0, eps_a=0.0, eps_b=0.0, k=-1.0, r=0.0),
    "semiconductor": dict(alpha=0.0, beta=-1.0, gamma=-2.0, eps_a=0.0, eps_b=0.0, k=-0.01, r=0.0),
    "softmatter": dict(alpha=0.0, beta=-1.0, gamma=-1.0, eps_a=-10.0, eps_b=0.0, k=-0.1, r=1.0),
    # the accuracy study's metallic case (Sec. III.D): wide spectrum, DOS piled at the Fermi level
    "metal_accuracy": dict(alpha=-1.0, beta=1.0, gamma=0.0, eps_a=1.0, eps_b=-1.0, k=-1.0, r=0.0),
}


def tight_binding(n: int, kind: str = "metal", seed: int = 0, **override) -> np.ndarray:
    """Two-level tight-binding model, n orbitals (float64, exactly symmetric).

    Orbital i is the A orbital of site i // 2 for even i and its B orbital for
    odd i (the layout is a reading; the paper does not give it).  Off-diagonal
    H_ij = c(type_i, type_j) exp(-|k| |s_i - s_j|) with c = alpha (A-A), beta
    (B-B), gamma (A-B) and s the site index (so gamma couples the two orbitals
    of one site at full strength, as in the paper's two-level schematic; the
    paper's negative k is read as the decay rate |k|); H_ii = eps_a or eps_b.  With r > 0
    every onsite energy and every coupling pair is multiplied by (1 + r eta),
    eta ~ U[-1, 1] drawn once per upper-triangle entry (PCG64, ``seed``).
    Parameters: ``TB_KINDS[kind]``, then the keyword overrides.
    """
    p = dict(TB_KINDS[kind])
    p.update(override)
    idx = np.arange(n)
    is_b = (idx % 2).astype(bool)
    ta, tb = ~is_b[:, None], is_b[:, None]
    sa, sb = ~is_b[None, :], is_b[None, :]
    coup = np.where(ta & sa, p["alpha"], 0.0) + np.where(tb & sb, p["beta"], 0.0) \
        + np.where((ta & sb) | (tb & sa), p["gamma"], 0.0)
    site = idx // 2
    dist = np.abs(site[:, None] - site[None, :]).astype(np.float64)
    h = coup * np.exp(-abs(p["k"]) * dist)
    np.fill_diagonal(h, np.where(is_b, p["eps_b"], p["eps_a"]))
    if p["r"] > 0.0:
        rng = np.random.default_rng(seed)
        eta = rng.uniform(-1.0, 1.0, size=(n, n))
        eta = np.triu(eta) + np.triu(eta, 1).T
        h = h * (1.0 + p["r"] * eta)
    return h

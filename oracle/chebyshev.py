"""Dense Chebyshev Fermi-operator expansion, plain FP64 (oracle; test infrastructure only).

Paper, Sec. II.A (eqs. D from diag, fermifunc) and Sec. II.B (eq. fermi,
the expansion sum c_n T_n, the spectral map by the extreme eigenvalues).
The readings where the paper is silent are stated per function:

* spectrum map: H~ = (2H - (e_a + e_b) I)/(e_b - e_a), T_0 = I, T_1 = H~;
* extreme eigenvalues e_a, e_b: Gershgorin discs (an outer bound), or optionally a
  few Lanczos steps with a residual widening (tighter, see lanczos_bounds);
* coefficients: Chebyshev-Gauss projection with M nodes (a DCT-II), no damping;
* chemical potential: bisection of tr D_L(mu) = N_e on the scaled interval [-1, 1].

The density matrix is evaluated through the eigen-decomposition,
``Q diag(p_L(lam~)) Q^T`` - the plain definition of the polynomial of a
symmetric matrix - never through the baby/giant-step schedule.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft

# ---------------------------------------------------------------------------
# spectrum bounds and scaling (Sec. II.B: e_a, e_b lowest and highest eigenvalues)


def gershgorin_bounds(h: np.ndarray):
    """Outer bounds [e_a, e_b] of the spectrum from Gershgorin's discs.

    e_a = min_i (H_ii - r_i), e_b = max_i (H_ii + r_i), r_i = sum_{j != i} |H_ij|.
    Reading of Sec. II.B, which asks for the extreme eigenvalues without a method.
    """
    h = np.asarray(h, dtype=np.float64)
    diag = np.diag(h)
    radius = np.abs(h).sum(axis=1) - np.abs(diag)
    return float(np.min(diag - radius)), float(np.max(diag + radius))


def splitmix64(count: int, seed: int = 0):
    """The first `count` outputs of SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) seeded with
    `seed`: state_i = seed + (i + 1) * 0x9E3779B97F4A7C15 (mod 2^64), then two
    xor-shift-multiply rounds and a final xor-shift (the published finaliser)."""
    mask = (1 << 64) - 1
    out = []
    for i in range(count):
        z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & mask
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        out.append(z ^ (z >> 31))
    return out


def splitmix64_uniform(count: int, seed: int = 0) -> np.ndarray:
    """count doubles in [-1, 1): u = (top 53 bits of output i) * 2^-53, returned as 2u - 1 (exact)."""
    return np.array([2.0 * ((z >> 11) * 2.0 ** -53) - 1.0 for z in splitmix64(count, seed)])


LANCZOS_BREAKDOWN = 1e-12   # beta_j <= this * max(|g_lo|, |g_hi|) ends the recurrence


def lanczos(h: np.ndarray, steps: int, seed: int = 0, scale: float | None = None):
    """Lanczos tridiagonalisation with one full reorthogonalisation pass per step.

    Start vector: SplitMix64 doubles in [-1, 1) of `seed`, normalised.  Step j:
    w = H v_j;  alpha_j = v_j . w;  w -= alpha_j v_j + beta_{j-1} v_{j-1};
    w -= V (V^T w) over v_0..v_j;  beta_j = ||w||;  v_{j+1} = w / beta_j.
    The recurrence stops after min(steps, n) steps, or after step j when
    beta_j <= LANCZOS_BREAKDOWN * scale (an invariant subspace: the Ritz values
    are then eigenvalues).  scale defaults to the Gershgorin bound max(|g_lo|, |g_hi|).
    Returns (alpha, beta, V) with len(alpha) = len(beta) = steps done and V of shape
    (steps done, n).
    """
    n = h.shape[0]
    if scale is None:
        g_lo, g_hi = gershgorin_bounds(h)
        scale = max(abs(g_lo), abs(g_hi))
    k = min(steps, n)
    v = splitmix64_uniform(n, seed)
    v = v / np.linalg.norm(v)
    V = np.zeros((k, n))
    alpha, beta = np.zeros(k), np.zeros(k)
    for j in range(k):
        V[j] = v
        w = h @ v
        alpha[j] = v @ w
        w = w - alpha[j] * v
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        w = w - V[: j + 1].T @ (V[: j + 1] @ w)
        beta[j] = np.linalg.norm(w)
        if beta[j] <= LANCZOS_BREAKDOWN * scale:
            k = j + 1
            break
        v = w / beta[j]
    return alpha[:k], beta[:k], V[:k]


def tridiag_eigvals(alpha, beta) -> np.ndarray:
    """Eigenvalues (ascending) of the symmetric tridiagonal matrix with diagonal alpha and
    off-diagonal beta[0..k-2]."""
    k = len(alpha)
    t = np.diag(np.asarray(alpha, dtype=np.float64))
    if k > 1:
        off = np.asarray(beta[: k - 1], dtype=np.float64)
        t = t + np.diag(off, 1) + np.diag(off, -1)
    return np.linalg.eigvalsh(t)


def lanczos_bounds(h: np.ndarray, steps: int = 40, margin: float = 0.01, seed: int = 0):
    """Outer spectral bounds from a few Lanczos steps (the paper needs e_a, e_b, Sec. II.B, and
    names no method; this is the tight alternative to Gershgorin's discs).

    With theta_min, theta_max the extreme Ritz values after k steps and beta_{k-1} the norm of
    the last residual, the estimate is [theta_min - beta_{k-1}, theta_max + beta_{k-1}] widened
    on both sides by margin times its width, then intersected with the Gershgorin interval
    (which always holds the spectrum); if that intersection is empty (rounding, H = cI) the
    Gershgorin interval is returned.  Returns (emin, emax, alpha, beta).
    """
    g_lo, g_hi = gershgorin_bounds(h)
    alpha, beta, _ = lanczos(h, steps, seed, max(abs(g_lo), abs(g_hi)))
    theta = tridiag_eigvals(alpha, beta)
    r = beta[-1]
    lo, hi = theta[0] - r, theta[-1] + r
    pad = margin * (hi - lo)
    lo, hi = max(lo - pad, g_lo), min(hi + pad, g_hi)
    if lo > hi:
        lo, hi = g_lo, g_hi
    return lo, hi, alpha, beta


def scaling(emin: float, emax: float):
    """Centre c and half-width a of [e_a, e_b]; H~ = (H - c I)/a (reading of Sec. II.B)."""
    return 0.5 * (emin + emax), 0.5 * (emax - emin)


def scaled_hamiltonian(h, emin, emax):
    c, a = scaling(emin, emax)
    n = h.shape[0]
    return (h - c * np.eye(n)) / a


# ---------------------------------------------------------------------------
# Fermi function and coefficients


def fermi(x, beta_s: float, mu_s: float):
    """Fermi-Dirac occupation 1/(1 + exp(beta'(x - mu~))) (eq. fermifunc, scaled variables).

    beta' = beta * a and mu~ = (mu - c)/a, so beta'(x - mu~) = beta(e - mu).
    """
    z = beta_s * (np.asarray(x, dtype=np.float64) - mu_s)
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(z))


def quadrature_nodes(M: int):
    """Chebyshev-Gauss nodes x_j = cos(theta_j), theta_j = pi (j + 1/2)/M."""
    theta = np.pi * (np.arange(M) + 0.5) / M
    return np.cos(theta)


def quadrature_size(order: int, beta_s: float) -> int:
    """Number of Chebyshev-Gauss nodes M (reading; the paper does not say how c_n are obtained).

    M = 2^ceil(log2 max(2(L+1), L/2 + 7 beta' + 64)).  The coefficients of the
    Fermi function decay like exp(-n pi/beta'), so the aliasing error of an
    M-node projection, about exp(-(2M - L) pi/beta'), stays below 1e-17.
    """
    need = max(2.0 * (order + 1), 0.5 * order + 7.0 * float(beta_s) + 64.0)
    return 1 << int(math.ceil(math.log2(need)))


def jackson_kernel(order: int):
    """Jackson damping factors g_0..g_L for a series of N = L + 1 terms.

    Not in the paper (it notes the Gibbs oscillations of the truncated series,
    Sec. III.D, but applies no damping): an option, off by default.  The kernel
    polynomial method's Jackson kernel (Weisse, Wellein, Alvermann, Fehske,
    Rev. Mod. Phys. 78, 275 (2006)):
        g_n = [(N - n + 1) cos(pi n / (N+1)) + sin(pi n / (N+1)) cot(pi / (N+1))] / (N + 1).
    """
    N = order + 1
    n = np.arange(order + 1, dtype=np.float64)
    q = np.pi / (N + 1)
    return ((N - n + 1) * np.cos(q * n) + np.sin(q * n) / np.tan(q)) / (N + 1)


def chebyshev_coeffs(order: int, beta_s: float, mu_s: float, M: int | None = None, damping: str | None = None):
    """Coefficients c_0..c_L of sum c_n T_n approximating f (Sec. II.B; projection is a reading).

    c_n = (2 - delta_{n0})/M * sum_{j<M} f(x_j) cos(n theta_j): the DCT-II of
    f sampled at the Chebyshev-Gauss nodes.  c_0 carries the factor 1/2.
    damping="jackson" multiplies c_n by the Jackson factors g_n.
    """
    if M is None:
        M = quadrature_size(order, beta_s)
    f = fermi(quadrature_nodes(M), beta_s, mu_s)
    f[np.abs(f) < 1e-250] = 0.0          # keeps the FFT out of denormals
    y = scipy.fft.dct(f, type=2)         # y_n = 2 sum_j f_j cos(pi n (2j+1)/(2M))
    c = y[: order + 1] / M
    c[0] *= 0.5
    if order + 1 > M:
        raise ValueError("order + 1 must not exceed M")
    if damping == "jackson":
        c = c * jackson_kernel(order)
    elif damping is not None:
        raise ValueError(f"unknown damping {damping!r}")
    return c


def cheb_eval(c, x):
    """p(x) = sum_n c_n T_n(x) by Clenshaw's recurrence (numpy's chebval)."""
    return np.polynomial.chebyshev.chebval(np.asarray(x, dtype=np.float64), np.asarray(c))


# ---------------------------------------------------------------------------
# density matrices


def density_from_eigs(q: np.ndarray, lam: np.ndarray, c, emin: float, emax: float):
    """D_L = Q diag(p_L(lam~)) Q^T (eq. D from diag applied to the polynomial p_L)."""
    cen, a = scaling(emin, emax)
    p = cheb_eval(c, (lam - cen) / a)
    return (q * p) @ q.T


def density_eigh(h: np.ndarray, c, emin: float, emax: float):
    """D_L through LAPACK's symmetric eigensolver on the stored H (self-check route)."""
    lam, q = np.linalg.eigh(h)
    return density_from_eigs(q, lam, c, emin, emax)


def density_recursion(h: np.ndarray, c, emin: float, emax: float):
    """D_L = sum_n c_n T_n(H~) with the plain three-term recursion, L GEMMs (small N only)."""
    ht = scaled_hamiltonian(h, emin, emax)
    n = h.shape[0]
    t_prev, t_cur = np.eye(n), ht
    d = c[0] * t_prev
    if len(c) > 1:
        d = d + c[1] * t_cur
    for cn in c[2:]:
        t_prev, t_cur = t_cur, 2.0 * ht @ t_cur - t_prev
        d = d + cn * t_cur
    return d


def commutator_max(h: np.ndarray, d: np.ndarray) -> float:
    """max_ij |(H D - D H)_ij| by two plain products (zero for any function of H, Sec. II.A)."""
    return float(np.max(np.abs(h @ d - d @ h)))


def fermi_dirac_density(q, lam, beta: float, mu: float):
    """Exact Fermi operator Q f(Lambda) Q^T (eqs. D from diag, fermifunc) - truncation reference."""
    with np.errstate(over="ignore"):
        occ = 1.0 / (1.0 + np.exp(beta * (lam - mu)))
    return (q * occ) @ q.T


# ---------------------------------------------------------------------------
# trace moments and the chemical potential (reading: the paper takes mu as given)


def moments_from_eigs(lam, emin: float, emax: float, order: int):
    """tau_n = tr T_n(H~) = sum_i T_n(lam~_i), n = 0..L, by the three-term recurrence."""
    cen, a = scaling(emin, emax)
    x = (np.asarray(lam, dtype=np.float64) - cen) / a
    tau = np.empty(order + 1)
    t_prev, t_cur = np.ones_like(x), x
    tau[0] = t_prev.sum()
    if order >= 1:
        tau[1] = t_cur.sum()
    for n in range(2, order + 1):
        t_prev, t_cur = t_cur, 2.0 * x * t_cur - t_prev
        tau[n] = t_cur.sum()
    return tau


def trace_of_series(c, tau):
    """tr sum_n c_n T_n(H~) = sum_n c_n tau_n."""
    return float(np.dot(np.asarray(c), np.asarray(tau)))


OK, NOCONV, BRACKET = 0, 1, -5


def bisect_mu(tau, order: int, beta_s: float, n_elec: float, tol: float = 1e-10,
              max_iter: int = 200, M: int | None = None, damping: str | None = None):
    """Scaled chemical potential mu~ with tr D_L(mu~) = N_e, by bisection (reading).

    Bracket [-1, 1]; it must hold t(-1) < N_e < t(1), else status BRACKET.
    Each sweep evaluates t at the midpoint; it stops when |t - N_e| < tol
    (status OK), when the bracket is narrower than 4 ulp of the midpoint or
    after max_iter sweeps (status NOCONV).  Returns (mu~, sweeps, t(mu~), status).
    """
    if M is None:
        M = quadrature_size(order, beta_s)

    def t_of(mu_s):
        return trace_of_series(chebyshev_coeffs(order, beta_s, mu_s, M, damping), tau)

    lo, hi = -1.0, 1.0
    if not (t_of(lo) < n_elec < t_of(hi)):
        return float("nan"), 0, float("nan"), BRACKET
    mid, t_mid = 0.0, float("nan")
    for it in range(1, max_iter + 1):
        mid = 0.5 * (lo + hi)
        t_mid = t_of(mid)
        if abs(t_mid - n_elec) < tol:
            return mid, it, t_mid, OK
        if t_mid < n_elec:
            lo = mid
        else:
            hi = mid
        if hi - lo < 4.0 * np.spacing(abs(mid) if mid != 0.0 else 1e-300):
            return mid, it, t_mid, NOCONV
    return mid, max_iter, t_mid, NOCONV


# ---------------------------------------------------------------------------
# the whole hot path at the oracle's level (the CPU baseline times this)


def mu_search_density(h: np.ndarray, beta: float, n_elec: float, order: int,
                      tol: float = 1e-10, bounds=None, eig=None):
    """Bounds -> moments -> bisection -> coefficients -> D_L, from the stored H.

    ``eig`` = (q, lam) may be given to skip LAPACK (the generator's own
    eigenpairs); otherwise ``numpy.linalg.eigh`` of H is used.  Returns a dict.
    """
    emin, emax = gershgorin_bounds(h) if bounds is None else bounds
    if eig is None:
        lam, q = np.linalg.eigh(h)
    else:
        q, lam = eig
    cen, a = scaling(emin, emax)
    beta_s = beta * a
    M = quadrature_size(order, beta_s)
    tau = moments_from_eigs(lam, emin, emax, order)
    mu_s, iters, t, status = bisect_mu(tau, order, beta_s, n_elec, tol, M=M)
    c = chebyshev_coeffs(order, beta_s, mu_s, M)
    d = density_from_eigs(q, lam, c, emin, emax)
    return dict(emin=emin, emax=emax, beta_s=beta_s, M=M, tau=tau, mu_s=mu_s,
                mu=cen + a * mu_s, iters=iters, trace=t, status=status, c=c, D=d)

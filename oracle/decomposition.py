"""Coefficient-matching algebra of the O(sqrt(L)) expansion (oracle; test infrastructure only).

Paper, Sec. II.B (eqs. ansatz, ansatz2, ansatz3, identity, power_of_Tk,
coeff recursion, example A, formula for d0, formula for d, X) and the
Appendix.  Every routine works either in exact rationals
(``fractions.Fraction``) or in float64, selected by ``exact``.

Two re-associations of the same polynomial ``sum_{n<km} c_n T_n`` are built:

* power form (the paper's):  ``sum_j T_k^j S_j``, ``S_j = sum_{i<k} d_{i,j} T_i``,
  with d from the upper-triangular system ``c = X d`` (eq. X);
* composition form (reading: same identity, other basis): ``sum_l T_l(T_k) R_l``,
  ``R_l = sum_{i<k} e_{l,i} T_i``, evaluated by Clenshaw over l.  Because
  ``T_l(T_k) = T_{lk}`` it is the same polynomial with bounded coefficients.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def split_order(order: int, k: int | None = None):
    """Baby/giant split for degree ``order`` = L (Sec. II.B, eq. ansatz; reading of L).

    L + 1 coefficients are padded with zeros to k*m; by default
    k = ceil(sqrt(L+1)) and m = ceil((L+1)/k), the choice that minimises the
    GEMM count (k-1)+(m-1) in Sec. II.B.
    """
    if order < 0:
        raise ValueError("order must be >= 0")
    n_coef = order + 1
    if k is None or k <= 0:
        k = math.isqrt(n_coef)
        if k * k < n_coef:
            k += 1
    m = -(-n_coef // k)
    return k, m


def power_matrix_A(m: int, exact: bool = False):
    """Matrix A of the expansions T_k^j = sum_l a_{j,l} T_{lk} (eqs. power_of_Tk, coeff recursion).

    Built row by row from the recurrence of Sec. II.B: a_{0,0}=1, a_{1,0}=0,
    a_{1,1}=1, and for j > 1
      a_{j,0} = a_{j-1,1}/2,  a_{j,1} = a_{j-1,0} + a_{j-1,2}/2,
      a_{j,l} = (a_{j-1,l-1} + a_{j-1,l+1})/2 for 1 < l < j,  a_{j,j} = a_{j-1,j-1}/2.
    Entries with l > j are zero (A is lower-triangular).
    """
    one = Fraction(1) if exact else 1.0
    zero = Fraction(0) if exact else 0.0
    half = Fraction(1, 2) if exact else 0.5
    a = [[zero] * m for _ in range(m)]
    if m >= 1:
        a[0][0] = one
    if m >= 2:
        a[1][0] = zero
        a[1][1] = one

    def prev(j, l):
        return a[j][l] if 0 <= l < m and l <= j else zero

    for j in range(2, m):
        for l in range(0, j + 1):
            if l == 0:
                a[j][l] = half * prev(j - 1, 1)
            elif l == 1:
                a[j][l] = prev(j - 1, 0) + half * prev(j - 1, 2)
            elif l < j:
                a[j][l] = half * (prev(j - 1, l - 1) + prev(j - 1, l + 1))
            else:
                a[j][l] = half * prev(j - 1, l - 1)
    if exact:
        return a
    return np.array(a, dtype=np.float64)


def assemble_X(k: int, m: int, exact: bool = False):
    """The km x km matrix X with c = X d (eqs. formula for d0, formula for d, X).

    Unknown ordering (as in the paper): d_{0,0}, d_{1,0}, ..., d_{k-1,0}, ...,
    d_{k-1,m-1}, i.e. d_{i,j} sits at column j*k + i.  Equation for c_{l*k+i}
    sits at row l*k + i:

    * i = 0:           c_{lk}     = d_0^T a_l
    * i > 0, l = 0:    c_i        = d_i^T a_0 + 1/2 d_{k-i}^T a_1
    * i > 0, 0<l<m-1:  c_{lk+i}   = 1/2 d_i^T a_l + 1/2 d_{k-i}^T a_{l+1}
    * i > 0, l = m-1:  c_{(m-1)k+i} = 1/2 d_i^T a_{m-1}

    with d_i^T a_l = sum_j a_{j,l} d_{i,j}.  For m = 1 the l = 0 row has no
    a_1 term (there is no giant step).  X is upper-triangular in this ordering.
    """
    A = power_matrix_A(m, exact=exact)
    zero = Fraction(0) if exact else 0.0
    half = Fraction(1, 2) if exact else 0.5
    n = k * m
    X = [[zero] * n for _ in range(n)]

    def a(j, l):
        return A[j][l] if (l < m and j < m) else zero

    for l in range(m):
        # i = 0 rows
        for j in range(m):
            X[l * k][j * k] += a(j, l)
        for i in range(1, k):
            row = l * k + i
            own = 1 if l == 0 else half
            for j in range(m):
                X[row][j * k + i] += own * a(j, l)
                if l + 1 < m:
                    X[row][j * k + (k - i)] += half * a(j, l + 1)
    if exact:
        return X
    return np.array(X, dtype=np.float64)


def solve_upper(X, rhs, exact: bool = False):
    """Back-substitution on an upper-triangular system (Appendix: "solved using back substitution")."""
    n = len(rhs)
    if exact:
        x = [Fraction(0)] * n
        for r in range(n - 1, -1, -1):
            s = Fraction(rhs[r])
            for cidx in range(r + 1, n):
                if X[r][cidx] != 0:
                    s -= X[r][cidx] * x[cidx]
            x[r] = s / X[r][r]
        return x
    import scipy.linalg

    return scipy.linalg.solve_triangular(np.asarray(X, dtype=np.float64),
                                         np.asarray(rhs, dtype=np.float64), lower=False)


def pad_coeffs(c, k: int, m: int, exact: bool = False):
    """Pad c_0..c_L with zeros up to k*m entries (L <= km - 1, eq. ansatz)."""
    c = list(c)
    if len(c) > k * m:
        raise ValueError("more coefficients than k*m")
    zero = Fraction(0) if exact else 0.0
    return c + [zero] * (k * m - len(c))


def power_form_d(c, k: int, m: int, exact: bool = False):
    """Coefficients d_{i,j} of the power form (paper, eq. ansatz3), returned as a k x m array/list."""
    cp = pad_coeffs(c, k, m, exact)
    X = assemble_X(k, m, exact)
    dvec = solve_upper(X, cp, exact)
    if exact:
        return [[dvec[j * k + i] for j in range(m)] for i in range(k)]
    return np.asarray(dvec).reshape(m, k).T.copy()


def composition_form_e(c, k: int, m: int, exact: bool = False):
    """Coefficients e_{l,i} of the composition form sum_l T_l(T_k) R_l (reading; m x k).

    Matching coefficients with 2 T_{lk} T_i = T_{lk+i} + T_{lk-i} (eq. identity),
    exactly as the paper does for d:
      c_{lk} = e_{l,0};  c_i = e_{0,i} + e_{1,k-i}/2;
      c_{lk+i} = (e_{l,i} + e_{l+1,k-i})/2 for l >= 1, with e_{m,.} = 0.
    Solved from l = m-1 downwards.
    """
    cp = pad_coeffs(c, k, m, exact)
    zero = Fraction(0) if exact else 0.0
    half = Fraction(1, 2) if exact else 0.5
    e = [[zero] * k for _ in range(m + 1)]
    for l in range(m - 1, -1, -1):
        e[l][0] = cp[l * k]
        for i in range(1, k):
            upper = e[l + 1][k - i]
            if l == 0:
                e[l][i] = cp[i] - half * upper
            else:
                e[l][i] = 2 * cp[l * k + i] - upper
    e = e[:m]
    if exact:
        return e
    return np.array(e, dtype=np.float64)


# ---------------------------------------------------------------------------
# scalar evaluators of the three forms (exact or float), used by the pins


def cheb_T(n: int, x):
    """T_n(x) by the three-term recurrence T_{n+1} = 2x T_n - T_{n-1} (textbook)."""
    t0, t1 = type(x)(1) if not isinstance(x, np.ndarray) else np.ones_like(x), x
    if n == 0:
        return t0
    for _ in range(n - 1):
        t0, t1 = t1, 2 * x * t1 - t0
    return t1


def eval_series(c, x):
    """sum_n c_n T_n(x) term by term (the left-hand side of eq. ansatz)."""
    return sum(cn * cheb_T(n, x) for n, cn in enumerate(c))


def eval_power_form(d, k: int, m: int, x):
    """sum_j T_k(x)^j sum_i d_{i,j} T_i(x) (eq. ansatz3)."""
    tk = cheb_T(k, x)
    total = 0
    for j in range(m):
        s = sum(d[i][j] * cheb_T(i, x) for i in range(k))
        total = total + tk ** j * s
    return total


def eval_composition_form(e, k: int, m: int, x):
    """sum_l T_l(T_k(x)) sum_i e_{l,i} T_i(x) (composition form, term by term)."""
    tk = cheb_T(k, x)
    total = 0
    for l in range(m):
        r = sum(e[l][i] * cheb_T(i, x) for i in range(k))
        total = total + cheb_T(l, tk) * r
    return total

"""Pins for the oracle's coefficient-matching algebra (paper Sec. II.B and Appendix).

Each test fixes the oracle against something other than itself: values the
paper prints (golden files), the binomial closed form of cos^j, exact
rational polynomial identities, and structural facts the Appendix states.
"""
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import decomposition as dec


def _read_rational_rows(path):
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line)
    return rows


def test_A_matches_paper_worked_example(golden_dir):
    rows = _read_rational_rows(os.path.join(golden_dir, "A_m5.txt"))
    expected = [[Fraction(tok) for tok in r.split()] for r in rows]
    assert dec.power_matrix_A(5, exact=True) == expected


def test_powers_match_paper_worked_expansions(golden_dir):
    A = dec.power_matrix_A(6, exact=True)
    for r in _read_rational_rows(os.path.join(golden_dir, "powers_Tk.txt")):
        j, vals = r.split(":")
        j = int(j)
        expected = [Fraction(tok) for tok in vals.split()]
        assert A[j][: j + 1] == expected


def _binomial_a(j, l):
    # cos^j(t) = 2^{-j} sum_r C(j, r) cos((j - 2r) t): collect cos(l t).
    if (j - l) % 2:
        return Fraction(0)
    if l == 0:
        return Fraction(math.comb(j, j // 2), 2 ** j)
    return Fraction(math.comb(j, (j - l) // 2), 2 ** (j - 1))


@pytest.mark.parametrize("m", [1, 2, 3, 8, 13])
def test_A_closed_form_from_binomial_expansion(m):
    A = dec.power_matrix_A(m, exact=True)
    for j in range(m):
        for l in range(m):
            want = _binomial_a(j, l) if l <= j else Fraction(0)
            assert A[j][l] == want, (j, l)


def test_A_structure_lower_triangular_parity():
    A = dec.power_matrix_A(9, exact=True)
    for j in range(9):
        for l in range(9):
            if l > j or (j - l) % 2:
                assert A[j][l] == 0


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_powers_of_Tk_identity_exact(k):
    # T_k(x)^j == sum_l a_{j,l} T_{lk}(x) at rational points (eq. power_of_Tk)
    A = dec.power_matrix_A(7, exact=True)
    for x in [Fraction(1, 3), Fraction(-5, 7), Fraction(2, 11)]:
        tk = dec.cheb_T(k, x)
        for j in range(7):
            rhs = sum(A[j][l] * dec.cheb_T(l * k, x) for l in range(j + 1))
            assert tk ** j == rhs


@pytest.mark.parametrize("k,m", [(5, 5), (4, 6), (3, 4), (6, 3), (2, 2)])
def test_X_upper_triangular_with_paper_diagonal(k, m):
    X = dec.assemble_X(k, m, exact=True)
    A = dec.power_matrix_A(m, exact=True)
    n = k * m
    for r in range(n):
        for c in range(r):
            assert X[r][c] == 0
    # Diagonal: a_{l,l} on scalar rows, a_{l,l}/2 on the I blocks, except the
    # first row block whose I block has no factor 1/2 (Appendix, first row block).
    for l in range(m):
        assert X[l * k][l * k] == A[l][l]
        for i in range(1, k):
            want = A[l][l] if l == 0 else A[l][l] / 2
            assert X[l * k + i][l * k + i] == want


@pytest.mark.parametrize("k,m", [(5, 5), (4, 7)])
def test_X_block_pattern_matches_appendix(k, m):
    # Row block l (l >= 1) carries (1/2) a_{l+1,l+1} J in the next column block
    # and (1/2) a_{l+2,l} I two blocks further (eq. X and the Appendix blocks).
    X = dec.assemble_X(k, m, exact=True)
    A = dec.power_matrix_A(m, exact=True)
    for l in range(1, m - 1):
        for i in range(1, k):
            assert X[l * k + i][(l + 1) * k + (k - i)] == A[l + 1][l + 1] / 2
            if l + 2 < m:
                assert X[l * k + i][(l + 2) * k + i] == A[l + 2][l] / 2
                # scalar row: a_{l+2,l} two blocks to the right, zero one block over
                assert X[l * k][(l + 2) * k] == A[l + 2][l]
            assert X[l * k][(l + 1) * k] == 0
    # First row block: a_{j,0} I for even j, (1/2) a_{j,1} J for odd j.
    for j in range(m):
        for i in range(1, k):
            if j % 2 == 0:
                assert X[i][j * k + i] == A[j][0]
            else:
                assert X[i][j * k + (k - i)] == A[j][1] / 2


def _random_rationals(n, seed):
    rnd = random.Random(seed)
    return [Fraction(rnd.randint(-50, 50), rnd.randint(1, 9)) for _ in range(n)]


@pytest.mark.parametrize("k,m", [(1, 4), (4, 1), (2, 2), (3, 4), (5, 5), (4, 6), (6, 3), (3, 7)])
def test_power_form_reproduces_series_exactly(k, m):
    # sum_n c_n T_n(x) == sum_j T_k(x)^j sum_i d_{i,j} T_i(x) in exact rationals (eq. ansatz3)
    c = _random_rationals(k * m, seed=k * 100 + m)
    d = dec.power_form_d(c, k, m, exact=True)
    for x in [Fraction(1, 3), Fraction(-3, 4), Fraction(7, 5), Fraction(0)]:
        assert dec.eval_series(c, x) == dec.eval_power_form(d, k, m, x)


@pytest.mark.parametrize("k,m", [(1, 4), (4, 1), (2, 2), (3, 4), (5, 5), (4, 6), (6, 3), (3, 7)])
def test_composition_form_reproduces_series_exactly(k, m):
    c = _random_rationals(k * m, seed=k * 31 + m)
    e = dec.composition_form_e(c, k, m, exact=True)
    for x in [Fraction(1, 3), Fraction(-3, 4), Fraction(7, 5), Fraction(0)]:
        assert dec.eval_series(c, x) == dec.eval_composition_form(e, k, m, x)


def test_planted_sign_error_is_caught():
    # A plausible slip in the oracle (wrong sign of the mirrored term) must
    # break the exact identity, so the identity pin can detect it.
    k, m = 4, 5
    c = _random_rationals(k * m, seed=7)
    e = dec.composition_form_e(c, k, m, exact=True)
    e[2][1] = -e[2][1] if e[2][1] != 0 else Fraction(1)
    x = Fraction(2, 9)
    assert dec.eval_series(c, x) != dec.eval_composition_form(e, k, m, x)


def test_float_forms_match_exact():
    k, m = 6, 7
    c = _random_rationals(k * m, seed=3)
    d_exact = dec.power_form_d(c, k, m, exact=True)
    d_float = dec.power_form_d([float(v) for v in c], k, m)
    e_exact = dec.composition_form_e(c, k, m, exact=True)
    e_float = dec.composition_form_e([float(v) for v in c], k, m)
    np.testing.assert_allclose(d_float, np.array(d_exact, dtype=float), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(e_float, np.array(e_exact, dtype=float), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("order,k,m", [(128, 12, 11), (512, 23, 23), (256, 17, 16), (2048, 46, 45),
                                       (0, 1, 1), (1, 2, 1), (3, 2, 2), (24, 5, 5)])
def test_split_order(order, k, m):
    assert dec.split_order(order) == (k, m)
    kk, mm = dec.split_order(order)
    assert kk * mm >= order + 1

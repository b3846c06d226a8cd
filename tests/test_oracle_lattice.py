"""Pins for oracle.lattice: eq. (iso) by brute force in exact arithmetic."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import lattice

W_EXACT = {"D2Q9": [Fraction(4, 9)] + [Fraction(1, 9)] * 4 + [Fraction(1, 36)] * 4,
           "D3Q19": [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12}
T0 = Fraction(1, 3)


def delta(i, j):
    return 1 if i == j else 0


def iso_rhs(idx, t0=T0):
    """T0^(n/2) * (sum over all pairings of products of deltas)."""
    if len(idx) == 0:
        return Fraction(1)
    first, rest = idx[0], idx[1:]
    tot = Fraction(0)
    for k in range(len(rest)):
        tot += delta(first, rest[k]) * iso_rhs(rest[:k] + rest[k + 1:], t0)
    return tot * t0


# weights per shell (sorted |c| components), written out as exact fractions
SHELL_W = {"D3Q39": {(0, 0, 0): Fraction(1, 12), (0, 0, 1): Fraction(1, 12), (1, 1, 1): Fraction(1, 27),
                     (0, 0, 2): Fraction(2, 135), (0, 2, 2): Fraction(1, 432), (0, 0, 3): Fraction(1, 1620)},
           "D2Q21": {(0, 0): Fraction(91, 324), (0, 1): Fraction(1, 12), (1, 1): Fraction(2, 27),
                     (0, 2): Fraction(7, 360), (2, 2): Fraction(1, 432), (0, 3): Fraction(1, 1620)}}
SHELL_N = {"D3Q39": {(0, 0, 0): 1, (0, 0, 1): 6, (1, 1, 1): 8, (0, 0, 2): 6, (0, 2, 2): 12, (0, 0, 3): 6},
           "D2Q21": {(0, 0): 1, (0, 1): 4, (1, 1): 4, (0, 2): 4, (2, 2): 4, (0, 3): 4}}


@pytest.mark.parametrize("name", ["D2Q21", "D3Q39"])
def test_sixth_order_isotropy_exact(name):
    """Eq. (iso) to sixth order (and the odd moments to seventh) with T0 = 2/3,
    in exact arithmetic; every shell complete; the float weights are the
    fractions."""
    lat = lattice.by_name(name)
    t0 = Fraction(2, 3)
    assert lat.T0 == float(t0)
    c = [tuple(int(v) for v in row) for row in lat.c]
    assert len(set(c)) == lat.Q
    keys = [tuple(sorted(abs(v) for v in row)) for row in c]
    assert {k: keys.count(k) for k in set(keys)} == SHELL_N[name]
    w = [SHELL_W[name][k] for k in keys]
    assert np.allclose(lat.w, [float(x) for x in w], rtol=1e-15, atol=0)
    for order in range(0, 8):
        for idx in itertools.product(range(lat.d), repeat=order):
            lhs = sum(w[a] * np.prod([c[a][i] for i in idx], dtype=object) for a in range(lat.Q))
            rhs = iso_rhs(list(idx), t0) if order % 2 == 0 else Fraction(0)
            assert Fraction(lhs) == rhs, (name, idx)


def test_d3q39_weights_solve_the_isotropy_conditions():
    """The D3Q39 weights follow from eq. (iso) on its shells: with
    S[shell][moment] the shell sums of c_x^2, c_x^4, c_x^2 c_y^2, c_x^6,
    c_x^4 c_y^2, c_x^2 c_y^2 c_z^2, the seven conditions (normalisation and six
    moments) have the unique solution T0 = 2/3 and the tabulated weights."""
    shells = [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 0, 0), (2, 2, 0), (3, 0, 0)]
    members = []
    for rep in shells:
        vs = set()
        for perm in itertools.permutations(rep):
            for sg in itertools.product((1, -1), repeat=3):
                vs.add(tuple(p * s for p, s in zip(perm, sg)))
        members.append(sorted(vs))
    mom = [lambda v: 1, lambda v: v[0] ** 2, lambda v: v[0] ** 4, lambda v: v[0] ** 2 * v[1] ** 2,
           lambda v: v[0] ** 6, lambda v: v[0] ** 4 * v[1] ** 2, lambda v: v[0] ** 2 * v[1] ** 2 * v[2] ** 2]
    S = [[sum(f(v) for v in m) for m in members] for f in mom]
    t0 = Fraction(2, 3)
    rhs = [1, t0, 3 * t0 ** 2, t0 ** 2, 15 * t0 ** 3, 3 * t0 ** 3, t0 ** 3]
    # exact Gaussian elimination on the 7 x 6 system
    A = [[Fraction(x) for x in row] + [Fraction(r)] for row, r in zip(S, rhs)]
    n = 6
    for col in range(n):
        piv = next(r for r in range(col, len(A)) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        for r in range(len(A)):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
    w = [A[k][n] / A[k][k] for k in range(n)]
    assert A[n][n] == 0   # the seventh condition is consistent: T0 = 2/3 is the solvable value
    want = [SHELL_W["D3Q39"][tuple(sorted(abs(x) for x in rep))] for rep in shells]
    assert w == want


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19"])
def test_isotropy_to_fourth_order_exact(name):
    lat = lattice.by_name(name)
    w = W_EXACT[name]
    assert np.allclose(lat.w, [float(x) for x in w], rtol=0, atol=0)
    assert float(lat.T0) == float(T0)
    c = [tuple(int(v) for v in row) for row in lat.c]
    for order in (0, 1, 2, 3, 4, 5):
        for idx in itertools.product(range(lat.d), repeat=order):
            lhs = sum(w[a] * np.prod([c[a][i] for i in idx], dtype=object) for a in range(lat.Q))
            rhs = iso_rhs(list(idx)) if order % 2 == 0 else Fraction(0)
            assert Fraction(lhs) == rhs, (name, idx)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19"])
def test_sixth_order_isotropy_fails(name):
    # the paper notes D3Q19 reaches only fourth order; sum w c_x^6 = 1/3 vs 15 T0^3 = 5/9
    lat = lattice.by_name(name)
    w = W_EXACT[name]
    lhs = sum(w[a] * int(lat.c[a][0]) ** 6 for a in range(lat.Q))
    assert lhs == Fraction(1, 3)
    assert iso_rhs([0] * 6) == Fraction(5, 9)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D2Q21", "D3Q39"])
def test_opposites_and_order(name):
    lat = lattice.by_name(name)
    assert np.all(lat.c[0] == 0)
    for a in range(1, lat.Q, 2):
        assert lat.opp[a] == a + 1 and lat.opp[a + 1] == a
    assert np.all(lat.c[lat.opp] == -lat.c)
    assert len({tuple(r) for r in lat.c}) == lat.Q

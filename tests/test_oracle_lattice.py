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


def iso_rhs(idx):
    """T0^(n/2) * (sum over all pairings of products of deltas)."""
    if len(idx) == 0:
        return Fraction(1)
    first, rest = idx[0], idx[1:]
    tot = Fraction(0)
    for k in range(len(rest)):
        tot += delta(first, rest[k]) * iso_rhs(rest[:k] + rest[k + 1:])
    return tot * T0


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


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19"])
def test_opposites_and_order(name):
    lat = lattice.by_name(name)
    assert np.all(lat.c[0] == 0)
    for a in range(1, lat.Q, 2):
        assert lat.opp[a] == a + 1 and lat.opp[a + 1] == a
    assert np.all(lat.c[lat.opp] == -lat.c)
    assert len({tuple(r) for r in lat.c}) == lat.Q

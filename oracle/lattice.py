"""Discrete velocity sets (Sec. 2.1, eq. (lattice) and eq. (iso)).

The paper prints the D3Q19 velocity set and T0 = 1/3 but not the weights; the
weights used here are the textbook ones for which eq. (iso) holds to fourth
order (the paper notes D3Q19 does not reach sixth order).  D2Q9 is the planar
analogue with T0 = 1/3.  The velocity ordering is a convention shared with the
C header by documentation only (each side holds its own table): rest first,
then opposite pairs (2k-1, 2k).

Pinned by: brute-force evaluation of eq. (iso) in exact rational arithmetic
(tests/test_oracle_lattice.py).
"""
import numpy as np

T0 = 1.0 / 3.0

_D2Q9_C = [(0, 0),
           (1, 0), (-1, 0),
           (0, 1), (0, -1),
           (1, 1), (-1, -1),
           (1, -1), (-1, 1)]
_D2Q9_W = [4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4

_D3Q19_C = [(0, 0, 0),
            (1, 0, 0), (-1, 0, 0),
            (0, 1, 0), (0, -1, 0),
            (0, 0, 1), (0, 0, -1),
            (1, 1, 0), (-1, -1, 0),
            (1, -1, 0), (-1, 1, 0),
            (1, 0, 1), (-1, 0, -1),
            (1, 0, -1), (-1, 0, 1),
            (0, 1, 1), (0, -1, -1),
            (0, 1, -1), (0, -1, 1)]
_D3Q19_W = [1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12


class Lattice:
    """A DdQq velocity set: c (Q, d) integer, w (Q,), opp (Q,), T0."""

    def __init__(self, name, c, w):
        self.name = name
        self.c = np.array(c, dtype=np.int64)
        self.w = np.array(w, dtype=np.float64)
        self.Q, self.d = self.c.shape
        self.T0 = T0
        opp = []
        for a in range(self.Q):
            match = [b for b in range(self.Q) if np.all(self.c[b] == -self.c[a])]
            assert len(match) == 1
            opp.append(match[0])
        self.opp = np.array(opp, dtype=np.int64)
        self.cf = self.c.astype(np.float64)


D2Q9 = Lattice("D2Q9", _D2Q9_C, _D2Q9_W)
D3Q19 = Lattice("D3Q19", _D3Q19_C, _D3Q19_W)


def by_name(name):
    return {"D2Q9": D2Q9, "D3Q19": D3Q19}[name]


def hermite2(lat):
    """H2_a^{ij} = c^i c^j / T0 - delta^{ij}, the tensor of eq. (deltaN) and of
    the second-order term of eq. (equilibrium).  Shape (Q, d, d)."""
    c = lat.cf
    return np.einsum("ai,aj->aij", c, c) / lat.T0 - np.eye(lat.d)[None]


def hermite3(lat):
    """H3_a^{ijk} = c^i c^j c^k - T0 (c^i d^{jk} + c^j d^{ki} + c^k d^{ij}), the
    tensor of the third-order term of eq. (equilibrium).  Shape (Q, d, d, d)."""
    c = lat.cf
    I = np.eye(lat.d)
    t = np.einsum("ai,aj,ak->aijk", c, c, c)
    t -= lat.T0 * (np.einsum("ai,jk->aijk", c, I)
                   + np.einsum("aj,ki->aijk", c, I)
                   + np.einsum("ak,ij->aijk", c, I))
    return t

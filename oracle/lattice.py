"""Discrete velocity sets (Sec. 2.1, eq. (lattice) and eq. (iso)).

The paper prints the D3Q19 velocity set and T0 = 1/3 but not the weights; the
weights used here are the textbook ones for which eq. (iso) holds to fourth
order (the paper notes D3Q19 does not reach sixth order).  D2Q9 is the planar
analogue with T0 = 1/3.

Eq. (iso) asks for isotropy up to sixth order for the full Navier-Stokes
limit.  D3Q39 reaches it with integer velocities: the shells 0, (1,0,0),
(1,1,1), (2,0,0), (2,2,0), (3,0,0) and T0 = 2/3.  The weights and T0 are the
solution of eq. (iso) on those shells: the x^2 y^2 z^2, x^4 y^2 and x^2 y^2
conditions fix w(1,1,1) = T0^3 / 8, w(2,2,0) = T0^3 / 128 and T0 = 2/3; the
remaining conditions are linear in the other weights.  D2Q21 is its planar
projection (weights summed over c_z), sixth-order isotropic with the same T0.

The velocity ordering is a convention shared with the C header by
documentation only (each side holds its own table): rest first, then opposite
pairs (2k-1, 2k).

Pinned by: brute-force evaluation of eq. (iso) in exact rational arithmetic
(tests/test_oracle_lattice.py).
"""
import itertools

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


def _shells(d, shells):
    """Velocities of the given (representative, weight) shells, every sign and
    axis permutation, ordered rest first and then opposite pairs."""
    c, w = [], []
    for rep, wt in shells:
        rep = tuple(rep) + (0,) * (d - len(rep))
        seen = set()
        for perm in itertools.permutations(rep):
            for signs in itertools.product((1, -1), repeat=d):
                v = tuple(p * s for p, s in zip(perm, signs))
                m = tuple(-x for x in v)
                if v in seen or m in seen:
                    continue
                seen.add(v)
                seen.add(m)
                if any(v):
                    c += [v, m]
                    w += [wt, wt]
                else:
                    c.insert(0, v)
                    w.insert(0, wt)
    return c, w


_D3Q39_SHELLS = [((0, 0, 0), 1.0 / 12.0), ((1, 0, 0), 1.0 / 12.0), ((1, 1, 1), 1.0 / 27.0),
                 ((2, 0, 0), 2.0 / 135.0), ((2, 2, 0), 1.0 / 432.0), ((3, 0, 0), 1.0 / 1620.0)]
# projection of D3Q39 on (c_x, c_y): weights summed over c_z
_D2Q21_SHELLS = [((0, 0), 1.0 / 12.0 + 2.0 / 12.0 + 4.0 / 135.0 + 2.0 / 1620.0), ((1, 0), 1.0 / 12.0),
                 ((1, 1), 2.0 / 27.0), ((2, 0), 2.0 / 135.0 + 2.0 / 432.0), ((2, 2), 1.0 / 432.0),
                 ((3, 0), 1.0 / 1620.0)]


class Lattice:
    """A DdQq velocity set: c (Q, d) integer, w (Q,), opp (Q,), T0."""

    def __init__(self, name, c, w, t0=T0):
        self.name = name
        self.c = np.array(c, dtype=np.int64)
        self.w = np.array(w, dtype=np.float64)
        self.Q, self.d = self.c.shape
        self.T0 = float(t0)
        self.speed = int(np.abs(self.c).max())   # longest link, in cells per axis
        opp = []
        for a in range(self.Q):
            match = [b for b in range(self.Q) if np.all(self.c[b] == -self.c[a])]
            assert len(match) == 1
            opp.append(match[0])
        self.opp = np.array(opp, dtype=np.int64)
        self.cf = self.c.astype(np.float64)


D2Q9 = Lattice("D2Q9", _D2Q9_C, _D2Q9_W)
D3Q19 = Lattice("D3Q19", _D3Q19_C, _D3Q19_W)
D2Q21 = Lattice("D2Q21", *_shells(2, _D2Q21_SHELLS), t0=2.0 / 3.0)
D3Q39 = Lattice("D3Q39", *_shells(3, _D3Q39_SHELLS), t0=2.0 / 3.0)


def by_name(name):
    return {"D2Q9": D2Q9, "D3Q19": D3Q19, "D2Q21": D2Q21, "D3Q39": D3Q39}[name]


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

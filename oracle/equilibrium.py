"""Curvilinear equilibrium distribution (Sec. 2.2, eq. (equilibrium)).

    f^eq_a = rho w_a { 1 + c_a.U / T0
                       + (1 / 2T0) H2_a^{ij} [ (g^{ij} - d^{ij}) T0 + Ut^i Ut^j ]
                       + (1 / 6T0^3) H3_a^{ijk} [ T0 ( (g^{ij} Ut^k - d^{ij} U^k)
                                                     + (g^{jk} Ut^i - d^{jk} U^i)
                                                     + (g^{ki} Ut^j - d^{ki} U^j) )
                                                + Ut^i Ut^j Ut^k ] }

with H2, H3 the Hermite tensors of oracle.lattice.  The first-order term
carries U (the population first moment), the higher ones the shifted velocity
Ut = U + a/2 (rho a = F).  Reading of the nested brackets: T0 multiplies only
the three parenthesised differences of the third-order term.

Pinned by: eq. (equilmoments) orders 0-2 exactly for arbitrary SPD g^{ij} and
Ut != U; the third-order moments where the lattice supports them (D2Q9 xxy,
xyy); reduction to the textbook third-order Hermite equilibrium when
g^{ij} = delta and Ut = U (tests/test_oracle_equilibrium.py).
"""
import numpy as np

from .lattice import hermite2, hermite3


def feq(lat, rho, U, Ut, gup):
    """f^eq on a batch of cells.

    rho (*s), U (d, *s), Ut (d, *s), gup (d, d, *s) -> (Q, *s).
    """
    d = lat.d
    T0 = lat.T0
    I = np.eye(d).reshape((d, d) + (1,) * np.ndim(rho))
    G = (gup - I) * T0 + np.einsum("i...,j...->ij...", Ut, Ut)
    R = T0 * (np.einsum("ij...,k...->ijk...", gup, Ut) - np.einsum("ij...,k...->ijk...", I, U)
              + np.einsum("jk...,i...->ijk...", gup, Ut) - np.einsum("jk...,i...->ijk...", I, U)
              + np.einsum("ki...,j...->ijk...", gup, Ut) - np.einsum("ki...,j...->ijk...", I, U)) \
        + np.einsum("i...,j...,k...->ijk...", Ut, Ut, Ut)
    H2 = hermite2(lat)
    H3 = hermite3(lat)
    t1 = np.einsum("ai,i...->a...", lat.cf, U) / T0
    t2 = np.einsum("aij,ij...->a...", H2, G) / (2.0 * T0)
    t3 = np.einsum("aijk,ijk...->a...", H3, R) / (6.0 * T0 ** 3)
    w = lat.w.reshape((-1,) + (1,) * np.ndim(rho))
    return rho[None] * w * (1.0 + t1 + t2 + t3)

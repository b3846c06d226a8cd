"""Pins for oracle.equilibrium: eq. (equilmoments) and the Cartesian reduction."""
import numpy as np
import pytest

from oracle import lattice
from oracle.equilibrium import feq


def random_spd(rng, d, n):
    M = np.eye(d)[None] + 0.4 * rng.standard_normal((n, d, d))
    S = np.einsum("nij,nkj->nik", M, M)
    return np.moveaxis(S, 0, -1)  # (d, d, n)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D2Q21", "D3Q39"])
def test_moments_orders_0_to_2(name):
    """sum f = rho; sum c f = rho U; sum c c f = g^{ij} rho T0 + rho Ut Ut for any
    SPD g^{ij} and Ut != U (eq. (equilmoments))."""
    lat = lattice.by_name(name)
    rng = np.random.default_rng(1)
    n, d = 200, lat.d
    rho = 1 + 0.2 * rng.standard_normal(n)
    U = 0.1 * rng.standard_normal((d, n))
    Ut = U + 0.1 * rng.standard_normal((d, n))
    gup = random_spd(rng, d, n)
    f = feq(lat, rho, U, Ut, gup)
    c = lat.cf
    assert np.allclose(f.sum(0), rho, rtol=0, atol=1e-14)
    assert np.allclose(np.einsum("ai,an->in", c, f), rho * U, rtol=0, atol=1e-14)
    Pi = np.einsum("ai,aj,an->ijn", c, c, f)
    expect = gup * rho * lat.T0 + rho * np.einsum("in,jn->ijn", Ut, Ut)
    assert np.allclose(Pi, expect, rtol=0, atol=5e-14)


def test_third_moment_where_d2q9_supports_it():
    """Q^{ijk} = [g^{ij} Ut^k + g^{jk} Ut^i + g^{ki} Ut^j] rho T0 + rho Ut Ut Ut holds
    for the mixed components xxy and xyy on D2Q9 (not for xxx, yyy: the lattice
    is only fourth-order isotropic, eq. (iso))."""
    lat = lattice.D2Q9
    rng = np.random.default_rng(2)
    n = 50
    rho = 1 + 0.2 * rng.standard_normal(n)
    U = 0.1 * rng.standard_normal((2, n))
    Ut = U + 0.1 * rng.standard_normal((2, n))
    gup = random_spd(rng, 2, n)
    f = feq(lat, rho, U, Ut, gup)
    c = lat.cf
    Q = np.einsum("ai,aj,ak,an->ijkn", c, c, c, f)
    T0 = lat.T0
    E = rho * T0 * (np.einsum("ijn,kn->ijkn", gup, Ut) + np.einsum("jkn,in->ijkn", gup, Ut)
                    + np.einsum("kin,jn->ijkn", gup, Ut)) + rho * np.einsum("in,jn,kn->ijkn", Ut, Ut, Ut)
    for idx in [(0, 0, 1), (0, 1, 1), (1, 0, 0), (1, 1, 0)]:
        assert np.allclose(Q[idx], E[idx], rtol=0, atol=1e-14), idx
    assert not np.allclose(Q[0, 0, 0], E[0, 0, 0], atol=1e-6)


@pytest.mark.parametrize("name", ["D2Q21", "D3Q39"])
def test_third_moments_exact_on_sixth_order_lattices(name):
    """Every component of Q^{ijk} = [g^{ij} Ut^k + g^{jk} Ut^i + g^{ki} Ut^j] rho T0
    + rho Ut Ut Ut (eq. (equilmoments)) holds on the sixth-order isotropic
    lattices, for any SPD g^{ij} and Ut != U; D3Q19 misses them all."""
    rng = np.random.default_rng(4)
    n = 60
    for nm in (name, "D3Q19" if name == "D3Q39" else "D2Q9"):
        lat = lattice.by_name(nm)
        d = lat.d
        rho = 1 + 0.2 * rng.standard_normal(n)
        U = 0.1 * rng.standard_normal((d, n))
        Ut = U + 0.1 * rng.standard_normal((d, n))
        gup = random_spd(rng, d, n)
        f = feq(lat, rho, U, Ut, gup)
        c = lat.cf
        Q = np.einsum("ai,aj,ak,an->ijkn", c, c, c, f)
        T0 = lat.T0
        E = rho * T0 * (np.einsum("ijn,kn->ijkn", gup, Ut) + np.einsum("jkn,in->ijkn", gup, Ut)
                        + np.einsum("kin,jn->ijkn", gup, Ut)) + rho * np.einsum("in,jn,kn->ijkn", Ut, Ut, Ut)
        if nm == name:
            assert np.allclose(Q, E, rtol=0, atol=5e-14)
        else:
            assert not np.allclose(Q[0, 0, 0], E[0, 0, 0], atol=1e-6)


@pytest.mark.parametrize("name", ["D2Q21", "D3Q39"])
def test_textbook_equilibrium_with_general_t0(name):
    """g^{ij} = delta, Ut = U: the third-order Hermite equilibrium with T0 = 2/3,
    w rho [1 + cu/T0 + (cu)^2/(2 T0^2) - u^2/(2 T0) + (cu)^3/(6 T0^3) - cu u^2/(2 T0^2)]."""
    lat = lattice.by_name(name)
    rng = np.random.default_rng(5)
    n, d = 100, lat.d
    rho = 1 + 0.2 * rng.standard_normal(n)
    u = 0.1 * rng.standard_normal((d, n))
    gup = np.repeat(np.eye(d)[:, :, None], n, axis=2)
    f = feq(lat, rho, u, u, gup)
    t = lat.T0
    cu = lat.cf @ u
    u2 = np.sum(u * u, axis=0)[None]
    text = lat.w[:, None] * rho[None] * (1 + cu / t + cu ** 2 / (2 * t * t) - u2 / (2 * t)
                                         + cu ** 3 / (6 * t ** 3) - cu * u2 / (2 * t * t))
    assert np.allclose(f, text, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19"])
def test_reduces_to_textbook_third_order_equilibrium(name):
    """With g^{ij} = delta and Ut = U the form is the standard third-order Hermite
    equilibrium (remark after eq. (equilibrium)):
    w rho [1 + 3 cu + 9/2 cu^2 - 3/2 u^2 + 9/2 cu^3 - 9/2 cu u^2]."""
    lat = lattice.by_name(name)
    rng = np.random.default_rng(3)
    n, d = 100, lat.d
    rho = 1 + 0.2 * rng.standard_normal(n)
    u = 0.1 * rng.standard_normal((d, n))
    gup = np.repeat(np.eye(d)[:, :, None], n, axis=2)
    f = feq(lat, rho, u, u, gup)
    cu = lat.cf @ u
    u2 = np.sum(u * u, axis=0)[None]
    text = lat.w[:, None] * rho[None] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u2 + 4.5 * cu ** 3 - 4.5 * cu * u2)
    assert np.allclose(f, text, rtol=0, atol=1e-15)

"""Pins for oracle.geometry (Sec. 2.1) against identities, closed forms and the
continuum limit of Sec. 3 / App. B-C."""
import numpy as np
import pytest

from oracle import geometry, lattice
from paper_2401_17183_amd import workloads as W
from tests.oracle_helpers import mesh_of


def lower_metric(g):
    return np.einsum("ik...,jk...->ij...", g, g)


@pytest.mark.parametrize("wl", [W.tanh_channel_2d(16, 12), W.wavy_channel_3d(8, 8, 6),
                                W.ogrid_3d(8, 16, 4), W.wavy_periodic("D2Q9", (10, 12), 0.2)])
def test_basis_identities(wl):
    """g_i . g^j = delta; [g^{ij}] = [g_ij]^-1; det g_ij = J^2 (eqs. (covectors),
    (inverse), (determinant))."""
    m = mesh_of(wl)
    b = geometry.basis(m)
    d = m.d
    I = np.eye(d).reshape((d, d) + (1,) * d)
    dots = np.einsum("ik...,jk...->ij...", b["g"], b["gco"])
    assert np.max(np.abs(dots - I)) < 1e-13
    gl = lower_metric(b["g"])
    prod = np.einsum("ik...,kj...->ij...", gl, b["gup"])
    assert np.max(np.abs(prod - I)) < 1e-12
    det = np.linalg.det(np.moveaxis(gl.reshape(d, d, -1), -1, 0))
    assert np.max(np.abs(det / b["J"].ravel() ** 2 - 1)) < 1e-12


def test_beta_is_one_on_straight_grid_lines():
    """beta = 1 when D_i and -D_-i are parallel (remark after eq. (tangent))."""
    m = mesh_of(W.tanh_channel_2d(16, 12))
    b = geometry.basis(m)
    assert np.max(np.abs(b["beta"] - 1)) < 1e-14
    # and then g_2 is exactly the centred difference over 2 dx
    y = m.coords[:, 0, 1]
    g2 = (y[2:] - y[:-2]) / (2 * m.dx)
    assert np.allclose(b["g"][1][1][:, 0], g2[:], rtol=1e-14, atol=0)


def test_beta_on_a_circle_closed_form():
    """On circular theta-lines beta = 1/cos(dtheta/2), so |g_theta| is the chord
    length over dx: |g_theta| = 2 r sin(dtheta/2)/dx."""
    wl = W.ogrid_3d(6, 16, 4)
    m = mesh_of(wl)
    b = geometry.basis(m)
    dth = 2 * np.pi / 16
    assert np.allclose(b["beta"][1], 1.0 / np.cos(dth / 2), rtol=1e-13)
    k = np.arange(-1, 7)
    r = 20.0 ** (k / 5.0)
    norm = np.sqrt(np.sum(b["g"][1] ** 2, axis=0))
    expect = 2 * r * np.sin(dth / 2) / m.dx
    assert np.allclose(norm, expect[None, None, :], rtol=1e-13)
    assert np.allclose(b["beta"][0], 1.0, atol=1e-14)


def test_parity_of_tangent():
    """g_-i = -g_i: the formula with the roles of D_i and D_-i exchanged."""
    m = mesh_of(W.wavy_channel_3d(8, 8, 6))
    P = np.moveaxis(geometry.padded_coords(m), -1, 0)
    x0 = P[:, 1:-1, 1:-1, 1:-1]
    Dp = P[:, 1:-1, 1:-1, 2:] - x0
    Dm = P[:, 1:-1, 1:-1, :-2] - x0
    def tangent(a, b_):
        return (np.linalg.norm(a, axis=0) + np.linalg.norm(b_, axis=0)) / np.linalg.norm(a - b_, axis=0) * (a - b_) / (2 * m.dx)
    assert np.allclose(tangent(Dm, Dp), -tangent(Dp, Dm), rtol=0, atol=1e-15)
    b = geometry.basis(m)
    assert np.allclose(tangent(Dp, Dm), b["g"][0], rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("lat,n", [("D2Q9", (6, 5)), ("D3Q19", (5, 4, 6))])
@pytest.mark.parametrize("periodic", [True, False])
def test_affine_mesh_has_zero_theta(lat, n, periodic):
    """Theta vanishes on a uniform lattice (after eq. (gamma)); more generally on
    any affine mesh, where g_i is constant: A = 0 and g^{ij} = (M^T M)^-1."""
    rng = np.random.default_rng(3)
    d = len(n)
    M = np.eye(d) + 0.3 * rng.standard_normal((d, d))
    if np.linalg.det(M) < 0:
        M[:, 0] *= -1
    wl = W.affine_mesh(lat, n, M, origin=rng.standard_normal(d), periodic=periodic)
    m = mesh_of(wl)
    g = geometry.Geometry(m)
    assert np.max(np.abs(g.A)) < 1e-13
    gup = np.linalg.inv(M.T @ M)
    assert np.allclose(g.gup.reshape(d, d, -1), gup[:, :, None], atol=1e-13)
    assert np.allclose(g.J, abs(np.linalg.det(M)), rtol=1e-13)
    if np.allclose(M, np.eye(d)):
        assert np.all(g.A == 0)


def polar_annulus(nr, nth, r0=1.0, r1=2.0):
    """2-D polar mesh, r = r0 + (k + 1/2) h_r, theta periodic."""
    hr = (r1 - r0) / nr
    k = np.arange(-2, nr + 2)
    r = r0 + (k + 0.5) * hr
    th = 2 * np.pi * np.arange(nth) / nth
    X = np.empty((nth, len(r), 2))
    X[..., 0] = r[None, :] * np.cos(th)[:, None]
    X[..., 1] = r[None, :] * np.sin(th)[:, None]
    lat = lattice.D2Q9
    m = geometry.Mesh(lat, (nr, nth), X, [(1, 1), (0, 0)], [(0, 0), (0, 0)], hr)
    return m, r[2:-2], hr, 2 * np.pi / nth


def central_gamma(m, bas):
    d = m.d
    G = np.zeros((d, d, d) + m.shape)   # G[i, j, k] = Gamma^i_jk in index units
    for k in range(d):
        e = [0] * d
        e[k] = 1
        G[:, :, k] = 0.5 * (geometry.theta(m, bas, e) - geometry.theta(m, bas, [-v for v in e]))
    return G


def test_christoffel_convergence_polar():
    """Theta -> c^k Gamma^i_jk in the continuum limit (Sec. 3): the centred
    discrete symbol converges at second order to the analytic polar ones
    Gamma^r_{theta theta} = -r, Gamma^theta_{r theta} = 1/r."""
    errs = []
    for nr, nth in ((16, 64), (32, 128)):
        m, r, hr, hth = polar_annulus(nr, nth)
        bas = geometry.basis(m)
        G = central_gamma(m, bas)
        h = np.array([hr, hth])
        # convert index-unit symbols to (r, theta) units: Gamma_xi = Gamma_q h_i / (h_j h_k)
        Gx = G * h[:, None, None, None, None] / (h[None, :, None, None, None] * h[None, None, :, None, None])
        ex = np.zeros_like(Gx)
        ex[0, 1, 1] = -r[None, :]
        ex[1, 0, 1] = 1.0 / r[None, :]
        ex[1, 1, 0] = 1.0 / r[None, :]
        errs.append(np.max(np.abs(Gx - ex)))
    assert errs[1] < errs[0] / 3.5, errs
    assert errs[1] < 2e-3


def refine_wavy(n0, level, amp=0.04):
    """x = xi + amp * (smooth periodic functions of all of xi), xi = q h on the
    unit torus; every coordinate depends on every index axis."""
    n = n0 * 2 ** level
    h = 1.0 / n
    q = np.arange(n) * h
    Z, Y, X = np.meshgrid(q, q, q, indexing="ij")
    tp = 2 * np.pi
    C = np.empty((n, n, n, 3))
    C[..., 0] = X + amp * np.sin(tp * (X + Y)) + 0.5 * amp * np.cos(tp * Z)
    C[..., 1] = Y + amp * np.sin(tp * (Y - 2 * Z)) + 0.5 * amp * np.sin(tp * X)
    C[..., 2] = Z + amp * np.cos(tp * (Z + X)) + 0.5 * amp * np.sin(tp * Y)
    m = geometry.Mesh(lattice.D3Q19, (n, n, n), C, [(0, 0)] * 3,
                      [(1, 0, 0), (0, 1, 0), (0, 0, 1)], h)
    return m, h


def test_flat_space_and_jacobian_identities_converge():
    """Discrete forms of (1/J) d_j (J g^{ij}) + Gamma^i_jk g^{jk} = 0 (eq. (flat)),
    Gamma^i_ij = d_j ln J (App. C) and Gamma^i_jk = Gamma^i_kj converge at second
    order on a smooth curvilinear mesh."""
    res = {"flat": [], "lnJ": [], "sym": []}
    for level in (1, 2):
        m, h = refine_wavy(8, level)
        bas = geometry.basis(m)
        d = 3
        G = central_gamma(m, bas)
        J = bas["J"]
        gupb = bas["gup"]
        Jr = geometry.real(J, 0, d)
        gup = geometry.real(gupb, 2, d)

        def dcent(f, lead, k):
            e = [0] * d
            e[k] = 1
            return 0.5 * (geometry._view(f, lead, e, 1, 0) - geometry._view(f, lead, [-v for v in e], 1, 0))
        div = sum(dcent(J[None, None] * gupb, 2, k)[:, k] for k in range(d)) / Jr[None]
        term = np.einsum("ijk...,jk...->i...", G, gup)
        scale = np.max(np.abs(term))
        res["flat"].append(np.max(np.abs(div + term)) / scale)
        trace = np.einsum("iik...->k...", G)
        dlnJ = np.stack([dcent(J, 0, k) for k in range(d)]) / Jr[None]
        res["lnJ"].append(np.max(np.abs(trace - dlnJ)) / np.max(np.abs(dlnJ)))
        res["sym"].append(np.max(np.abs(G - np.swapaxes(G, 1, 2))) / np.max(np.abs(G)))
    for k, v in res.items():
        assert v[1] < v[0] / 3.0, (k, v)
        assert v[1] < 0.05, (k, v)

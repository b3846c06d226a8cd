"""Collision with the inertial force (Sec. 2.2).

One time step at a cell takes the arrived populations N_a (eq. (adv)) to the
post-collision ones

    N'_a = N_a + Omega_a + dN_a                                   eq. (lbe)
    Omega_a = sum_b M_ab (N_b - J f^eq_b)                         eq. (collide)
            = -(N_a - J f^eq_a) / tau                             BGK, M = -I / tau
    dN_a = w_a J [ c_a.F / T0 + H2_a : dPi / T0 ]                 eq. (deltaN)
    J F^i = -1/2 sum_a [ A^i_a N'_a + A^i_opp(a) N_a ]            eq. (compo-constr)
    dPi^{ij} = -1/2 (1 - 1/2tau) sum_a c^i_a (A^j_a + A^j_opp(a)) f^eq_a
                                                                  eq. (delta-flux)
    Ut = U + F / (2 rho)                                          (below eq. (equilmoments))

with A the contracted Theta of oracle.geometry.  F depends on N', which
depends on F (through dN, and through Ut inside f^eq): the paper leaves the
solution method open.

Readings:
* the implicit relation is solved as a per-cell fixed point on F, started at
  F = 0 and iterated until max_i |F_k - F_(k-1)| <= tol * rho; the N' of the
  last iteration is the output.  The converged fixed point is unique (the map
  contracts), so any solver that converges gives the same step;
* dPi is symmetrised: only its symmetric part reaches dN (H2 is symmetric),
  which removes the index-order difference between the two places the paper
  writes it (eq. (delta-flux) and eq. (delta-fluxa));
* an external Euclidean body acceleration G (not in the paper) enters as
  F_tot = F + rho a_ext, a_ext^i = G . g^i, in dN and in Ut, and adds
  1/2 (1 - 1/2tau) (Ut^i rho a_ext^j + rho a_ext^i Ut^j) to dPi; on a uniform
  Cartesian mesh this is second-order (Guo-type) forcing.

General collision matrix (eq. (collide) with eq. (matrix)).  The paper only
asks of M that it relax the second moment at 1/tau (eq. (matrix)).  The
library's M is the two-rate family
    M = -(1/tau_g) I + (1/tau_g - 1/tau) H,
    H_ab = w_a [1 + c_a.c_b / T0 + H2_a : H2_b / 2],
H the projector onto the Hermite content up to second order (the span of w,
w c^i and w H2^{ij}; a projector because the lattice is fourth-order
isotropic).  The hydrodynamic part of f - f^eq relaxes at 1/tau and all the
rest (third and higher Hermite content) at 1/tau_g.  tau_g = tau is BGK,
tau_g = 1 is the regularised collision (the non-hydrodynamic content is
removed in one step).  Eq. (matrix) and its inverse eq. (matrix2) hold for any
tau_g as matrix identities, and sum Omega = sum c Omega = 0 because f - f^eq
carries no mass or momentum.

Pinned by: sum Omega = 0 and sum c Omega = 0 (eq. (conserv)/(omcons)), the three
moment constraints on dN (eqs. (constraints), (constraint2), (constraint3)),
F = 0 on a uniform lattice, eqs. (matrix) and (matrix2) and the spectrum of
the general M, its reduction to BGK at tau_g = tau and to the textbook
regularised collision on a uniform lattice at tau_g = 1, and the per-cell
mid-link momentum identity
    sum_a (c_a + A_a / 2) N'_a = sum_a (c_a - A_opp(a) / 2) N_a + J rho a_ext
which follows from eq. (constraint2) and eq. (compo-constr) once the fixed
point has converged (tests/test_oracle_collide.py).
"""
import numpy as np

from .equilibrium import feq
from .lattice import hermite2


def moments(lat, J, N):
    """rho = sum_a N_a / J, U^i = sum_a c^i_a N_a / (J rho)  (eqs. (dist), (moments), (vcurvi))."""
    rhoJ = N.sum(axis=0)
    rho = rhoJ / J
    U = np.einsum("ai,a...->i...", lat.cf, N) / rhoJ
    return rho, U


def delta_pi(lat, tau, A, fe, Ut, rho, aext, A_in=None):
    """Symmetrised dPi of eq. (delta-flux) plus the body-force reading.
    A_in: the incoming link coefficients (default A_opp(a); see oracle.moving)."""
    opp = lat.opp
    k = 1.0 - 1.0 / (2.0 * tau)
    S = A + (A[opp] if A_in is None else A_in)
    P = -0.5 * k * np.einsum("ai,aj...,a...->ij...", lat.cf, S, fe)
    ra = rho[None] * aext
    P = P + 0.5 * k * (np.einsum("i...,j...->ij...", Ut, ra) + np.einsum("i...,j...->ij...", ra, Ut))
    return 0.5 * (P + np.swapaxes(P, 0, 1))


def delta_n(lat, J, Ft, dPi):
    """dN_a = w_a J [c_a.F / T0 + H2_a : dPi / T0]  (eq. (deltaN))."""
    H2 = hermite2(lat)
    T0 = lat.T0
    w = lat.w.reshape((-1,) + (1,) * J.ndim)
    return w * J[None] * (np.einsum("ai,i...->a...", lat.cf, Ft) / T0
                          + np.einsum("aij,ij...->a...", H2, dPi) / T0)


def inertial_force(lat, J, A, N, Np, A_in=None):
    """F^i of eq. (compo-constr): J F^i = -1/2 sum_a [A^i_a N'_a + A^i_opp(a) N_a]
    (A_in in place of A_opp(a) when given: the incoming coefficients of
    oracle.moving)."""
    Ai = A[lat.opp] if A_in is None else A_in
    return (-0.5 * np.einsum("ai...,a...->i...", A, Np)
            - 0.5 * np.einsum("ai...,a...->i...", Ai, N)) / J[None]


def hydrodynamic_projector(lat):
    """H (Q, Q): H_ab = w_a [1 + c_a.c_b / T0 + H2_a : H2_b / 2]."""
    H2 = hermite2(lat)
    w = lat.w[:, None]
    return w * (1.0 + lat.cf @ lat.cf.T / lat.T0 + 0.5 * np.einsum("aij,bij->ab", H2, H2))


def collision_matrix(lat, tau, tau_g):
    """M (Q, Q) of eq. (collide): -(1/tau_g) I + (1/tau_g - 1/tau) H."""
    return -np.eye(lat.Q) / tau_g + (1.0 / tau_g - 1.0 / tau) * hydrodynamic_projector(lat)


def collide(geom, tau, N, tol=1e-14, max_iter=50, tau_g=None, A_in=None):
    """Post-collision populations and the converged inertial force.

    N (Q, *n) -> (N', info) with info = {F, Ut, U, rho, iters (*n), converged}.
    iters is the per-cell number of fixed-point iterations needed to meet the
    stopping rule (max_iter + 1 where it never did).  tau_g None: BGK;
    otherwise the general collision matrix collision_matrix(lat, tau, tau_g).
    A_in: incoming link coefficients in place of A_opp(a) (moving meshes,
    oracle.moving); geom.A holds the outgoing ones.
    """
    lat = geom.lat
    M = None if tau_g is None else collision_matrix(lat, tau, tau_g)
    J, A, gup, aext = geom.J, geom.A, geom.gup, geom.aext
    rho, U = moments(lat, J, N)
    F = np.zeros_like(U)
    iters = np.full(rho.shape, max_iter + 1, dtype=np.int64)
    Np = None
    Ut = None
    for k in range(1, max_iter + 1):
        Ft = F + rho[None] * aext
        Ut = U + Ft / (2.0 * rho[None])
        fe = feq(lat, rho, U, Ut, gup)
        dPi = delta_pi(lat, tau, A, fe, Ut, rho, aext, A_in)
        if M is None:
            Om = -(N - J[None] * fe) / tau
        else:
            Om = np.einsum("ab,b...->a...", M, N - J[None] * fe)
        Np = N + Om + delta_n(lat, J, Ft, dPi)
        Fn = inertial_force(lat, J, A, N, Np, A_in)
        change = np.max(np.abs(Fn - F), axis=0)
        newly = (change <= tol * rho) & (iters > max_iter)
        iters[newly] = k
        F = Fn
        if np.all(iters <= max_iter):
            break
    info = {"F": F, "Ut": Ut, "U": U, "rho": rho, "iters": iters,
            "converged": bool(np.all(iters <= max_iter))}
    return Np, info


def consistent_equilibrium(geom, tau, rho, Ut_target, tol=1e-14, max_iter=50):
    """Populations N = J f^eq(rho, U, Ut) whose own collision fixed point
    reproduces the prescribed shifted velocity Ut (reading for the initial and
    the far-field state; the paper gives neither).

    Fixed point on F: U = Ut - F_tot / (2 rho), N = J f^eq(rho, U, Ut),
    N' = N + dN (Omega = 0 because f = f^eq at that Ut), F <- eq. (compo-constr)
    with the arrived populations equal to N.  At convergence the collision of N
    (collide above) has the same F and hence Ut.
    """
    lat = geom.lat
    J, A, gup, aext = geom.J, geom.A, geom.gup, geom.aext
    F = np.zeros_like(Ut_target)
    N = None
    done = False
    for _ in range(max_iter):
        Ft = F + rho[None] * aext
        U = Ut_target - Ft / (2.0 * rho[None])
        fe = feq(lat, rho, U, Ut_target, gup)
        N = J[None] * fe
        dPi = delta_pi(lat, tau, A, fe, Ut_target, rho, aext)
        Np = N + delta_n(lat, J, Ft, dPi)
        Fn = inertial_force(lat, J, A, N, Np)
        change = np.max(np.abs(Fn - F), axis=0)
        F = Fn
        if np.all(change <= tol * rho):
            done = True
            break
    if not done:
        raise RuntimeError("initial-state fixed point did not converge")
    Ft = F + rho[None] * aext
    U = Ut_target - Ft / (2.0 * rho[None])
    return J[None] * feq(lat, rho, U, Ut_target, gup)

// Per-cell dynamics of the volumetric curvilinear LBM (Sec. 2.2), templated on
// the lattice L and the arithmetic type T.  Everything here runs in registers
// of one thread; the kernels around it do the data movement.
#pragma once

#include "common.hpp"

namespace vlbm {

// Per-cell geometry as the collision needs it.
template <class L, class T> struct CellGeo {
  T J;
  T gup[nup<L::D>()];     // g^{ij}, upper triangle
  T A[L::Q][L::D];        // A^i_a (A[0] = 0)
  T aext[L::D];           // a_ext^i = G . g^i
};

template <class L, class T>
__device__ __forceinline__ T gval(const CellGeo<L, T>& g, int i, int j) {
  return g.gup[up<L::D>(i, j)];
}

// Per-cell scalars of the equilibrium that do not depend on the direction.
template <class L, class T> struct EqCoef {
  T rho, trG, U[L::D], Ut[L::D], r[L::D];
};

// Build the direction-independent parts of eq. (equilibrium):
//  G^{ij} = (g^{ij} - d^{ij}) T0 + Ut^i Ut^j        -> trace
//  R^{ijk} (fully symmetric)                          -> r^i = sum_j R^{ijj}
//         = T0 [2 (g Ut)^i + tr(g) Ut^i - (D + 2) U^i] + |Ut|^2 Ut^i
template <class L, class T>
__device__ __forceinline__ EqCoef<L, T> eq_coef(const CellGeo<L, T>& g, T rho, const T* U, const T* Ut) {
  constexpr int D = L::D;
  const T t0 = T(T0);
  EqCoef<L, T> e;
  e.rho = rho;
  T uu = 0, trg = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    e.U[i] = U[i];
    e.Ut[i] = Ut[i];
    uu += Ut[i] * Ut[i];
    trg += gval(g, i, i);
  }
  e.trG = t0 * (trg - T(D)) + uu;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T gu = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) gu += gval(g, i, j) * Ut[j];
    e.r[i] = t0 * (T(2) * gu + trg * Ut[i] - T(D + 2) * U[i]) + uu * Ut[i];
  }
  return e;
}

// f^eq_a of eq. (equilibrium) for a compile-time direction a:
//   rho w [1 + cU/T0 + H2:G/(2 T0) + H3:R/(6 T0^3)]
// with H2:G = c.G.c/T0 - tr G and H3:R = R(c,c,c) - 3 T0 c.r,
//   c.G.c = T0 (c.g.c - c.c) + (c.Ut)^2,
//   R(c,c,c) = 3 T0 [(c.g.c)(c.Ut) - (c.c)(c.U)] + (c.Ut)^3.
template <class L, class T, int a>
__device__ __forceinline__ T feq_dir(const CellGeo<L, T>& g, const EqCoef<L, T>& e) {
  constexpr int D = L::D;
  const T t0 = T(T0);
  T cU = 0, cUt = 0, cr = 0, cgc = 0;
  int cc = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    constexpr int dummy = 0;
    (void)dummy;
    const int ci = L::c(a, i);
    if (ci == 0) continue;
    cc += ci * ci;
    cU += T(ci) * e.U[i];
    cUt += T(ci) * e.Ut[i];
    cr += T(ci) * e.r[i];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int cj = L::c(a, j);
      if (cj == 0) continue;
      cgc += T(ci * cj) * gval(g, i, j);
    }
  }
  const T cGc = t0 * (cgc - T(cc)) + cUt * cUt;
  const T H2G = cGc * T(3) - e.trG;                       // / T0 = * 3
  const T H3R = T(3) * t0 * (cgc * cUt - T(cc) * cU) + cUt * cUt * cUt - T(3) * t0 * cr;
  // 1/(2 T0) = 3/2, 1/(6 T0^3) = 27/6 = 9/2, 1/T0 = 3
  return e.rho * T(L::w(a)) * (T(1) + T(3) * cU + T(1.5) * H2G + T(4.5) * H3R);
}

template <class L, class T, int a = 0>
__device__ __forceinline__ void feq_all(const CellGeo<L, T>& g, const EqCoef<L, T>& e, T* fe) {
  if constexpr (a < L::Q) {
    fe[a] = feq_dir<L, T, a>(g, e);
    feq_all<L, T, a + 1>(g, e, fe);
  }
}

// Symmetrised dPi of eq. (delta-flux) (A contracted with c, S_a = A_a + A_opp(a)),
// using the pair symmetry S_a = S_opp(a), c_opp(a) = -c_a:
//   sum_a c^i S^j f_a = sum_pairs c^i_p S^j_p (f_p - f_opp(p)),
// plus the body-force reading 1/2 k (Ut^i rho a^j + rho a^i Ut^j), k = 1 - 1/(2 tau).
template <class L, class T>
__device__ __forceinline__ void delta_pi(const CellGeo<L, T>& g, const T* fe, const T* Ut, T rho, T k,
                                         T* dpi /* nup */) {
  constexpr int D = L::D;
  T M[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) M[i][j] = 0;
#pragma unroll
  for (int p = 1; p < L::Q; p += 2) {
    const T df = fe[p] - fe[p + 1];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const int ci = L::c(p, i);
      if (ci == 0) continue;
#pragma unroll
      for (int j = 0; j < D; ++j) M[i][j] += T(ci) * (g.A[p][j] + g.A[p + 1][j]) * df;
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      const T fi = T(-0.25) * k * (M[i][j] + M[j][i]);
      const T fb = T(0.5) * k * rho * (Ut[i] * g.aext[j] + g.aext[i] * Ut[j]);
      dpi[up<D>(i, j)] = fi + fb;
    }
}

// dN_a = w_a J [c.F/T0 + H2_a:dPi/T0],  H2:dPi = c.dPi.c/T0 - tr dPi  (eq. (deltaN))
template <class L, class T, int a>
__device__ __forceinline__ T delta_n_dir(T J, const T* Ft, const T* dpi, T trdpi) {
  constexpr int D = L::D;
  T cF = 0, cpc = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const int ci = L::c(a, i);
    if (ci == 0) continue;
    cF += T(ci) * Ft[i];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int cj = L::c(a, j);
      if (cj == 0) continue;
      cpc += T(ci * cj) * dpi[up<D>(i, j)];
    }
  }
  return T(L::w(a)) * J * (T(3) * cF + T(3) * (T(3) * cpc - trdpi));
}

// N'_a = N_a - (N_a - J f^eq_a)/tau + dN_a (eqs. (lbe), (collide)) and the
// accumulation of -1/2 sum_a A^i_a N'_a for the next force (eq. (compo-constr)).
template <class L, class T, int a = 0>
__device__ __forceinline__ void post_collision(const CellGeo<L, T>& g, const T* N, const T* fe, const T* Ft,
                                               const T* dpi, T trdpi, T inv_tau, T* Np, T* acc) {
  if constexpr (a < L::Q) {
    const T v = N[a] - (N[a] - g.J * fe[a]) * inv_tau + delta_n_dir<L, T, a>(g.J, Ft, dpi, trdpi);
    Np[a] = v;
    if constexpr (a > 0) {
#pragma unroll
      for (int i = 0; i < L::D; ++i) acc[i] -= T(0.5) * g.A[a][i] * v;
    }
    post_collision<L, T, a + 1>(g, N, fe, Ft, dpi, trdpi, inv_tau, Np, acc);
  }
}

struct CollideOut {
  int iters;   // iterations used; max_iter + 1 when the cap was hit
};

// The collision of one cell: moments (eqs. (dist), (moments), (vcurvi)), then
// the implicit inertial force (eq. (compo-constr), remark after eq. (deltaN))
// solved as a fixed point on F from F = 0, iterated until
// max_i |F_k - F_(k-1)| <= tol * rho; Np receives the N' of the last iteration.
template <class L, class T>
__device__ __forceinline__ CollideOut collide(const CellGeo<L, T>& g, const T* N, T tau, T tol, int max_iter, T* Np,
                                              T* F_out, T* Ut_out, T* U_out, T& rho_out) {
  constexpr int D = L::D;
  constexpr int Q = L::Q;
  T rhoJ = 0;
  T mom[D];
#pragma unroll
  for (int i = 0; i < D; ++i) mom[i] = 0;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    rhoJ += N[a];
#pragma unroll
    for (int i = 0; i < D; ++i)
      if (L::c(a, i) != 0) mom[i] += T(L::c(a, i)) * N[a];
  }
  const T rho = rhoJ / g.J;
  T U[D], B[D], F[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    U[i] = mom[i] / rhoJ;
    B[i] = 0;
    F[i] = 0;
  }
  // B^i = -1/2 sum_a A^i_opp(a) N_a (the incoming part of eq. (compo-constr))
#pragma unroll
  for (int a = 1; a < Q; ++a)
#pragma unroll
    for (int i = 0; i < D; ++i) B[i] -= T(0.5) * g.A[opp(a)][i] * N[a];
  const T k = T(1) - T(0.5) / tau;
  const T inv_tau = T(1) / tau;
  const T invJ = T(1) / g.J;
  const T half_inv_rho = T(0.5) / rho;
  T Ut[D];
  int it = 1;
  int done = 0;
  for (; it <= max_iter; ++it) {
    T Ft[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      Ft[i] = F[i] + rho * g.aext[i];
      Ut[i] = U[i] + Ft[i] * half_inv_rho;
    }
    const EqCoef<L, T> e = eq_coef<L, T>(g, rho, U, Ut);
    T fe[Q];
    feq_all<L, T>(g, e, fe);
    T dpi[nup<D>()];
    delta_pi<L, T>(g, fe, Ut, rho, k, dpi);
    T trdpi = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) trdpi += dpi[up<D>(i, i)];
    T acc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] = B[i];
    post_collision<L, T>(g, N, fe, Ft, dpi, trdpi, inv_tau, Np, acc);
    T change = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const T Fn = acc[i] * invJ;
      const T dd = Fn - F[i];
      change = fmax(change, dd < T(0) ? -dd : dd);
      F[i] = Fn;
    }
    if (change <= tol * rho) {
      done = 1;
      break;
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    F_out[i] = F[i];
    Ut_out[i] = Ut[i];
    U_out[i] = U[i];
  }
  rho_out = rho;
  CollideOut o;
  o.iters = done ? it : max_iter + 1;
  return o;
}

// Consistent equilibrium (the library's reading for initial and imposed
// states): find F such that with U = Ut - F_tot/(2 rho) the populations
// N = J f^eq(rho, U, Ut) have that F as their collision fixed point.
template <class L, class T>
__device__ __forceinline__ int consistent_equilibrium(const CellGeo<L, T>& g, T rho, const T* Ut, T tau, T tol,
                                                      int max_iter, T* N) {
  constexpr int D = L::D;
  constexpr int Q = L::Q;
  const T k = T(1) - T(0.5) / tau;
  const T invJ = T(1) / g.J;
  const T half_inv_rho = T(0.5) / rho;
  T F[D];
#pragma unroll
  for (int i = 0; i < D; ++i) F[i] = 0;
  int ok = 0;
  for (int it = 0; it < max_iter; ++it) {
    T Ft[D], U[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      Ft[i] = F[i] + rho * g.aext[i];
      U[i] = Ut[i] - Ft[i] * half_inv_rho;
    }
    const EqCoef<L, T> e = eq_coef<L, T>(g, rho, U, Ut);
    T fe[Q];
    feq_all<L, T>(g, e, fe);
    T dpi[nup<D>()];
    delta_pi<L, T>(g, fe, Ut, rho, k, dpi);
    T trdpi = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) trdpi += dpi[up<D>(i, i)];
    T Nc[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) Nc[a] = g.J * fe[a];
    // N' = N + dN (Omega = 0 since f = f^eq at this Ut); B uses the arrived N = N
    T acc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] = 0;
#pragma unroll
    for (int a = 1; a < Q; ++a)
#pragma unroll
      for (int i = 0; i < D; ++i) acc[i] -= T(0.5) * g.A[opp(a)][i] * Nc[a];
    T Np[Q];
    post_collision<L, T>(g, Nc, fe, Ft, dpi, trdpi, T(0), Np, acc);
    T change = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const T Fn = acc[i] * invJ;
      const T dd = Fn - F[i];
      change = fmax(change, dd < T(0) ? -dd : dd);
      F[i] = Fn;
    }
    if (change <= tol * rho) {
      ok = 1;
      break;
    }
  }
  T Ft[D], U[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    Ft[i] = F[i] + rho * g.aext[i];
    U[i] = Ut[i] - Ft[i] * half_inv_rho;
  }
  const EqCoef<L, T> e = eq_coef<L, T>(g, rho, U, Ut);
  T fe[Q];
  feq_all<L, T>(g, e, fe);
#pragma unroll
  for (int a = 0; a < Q; ++a) N[a] = g.J * fe[a];
  return ok;
}

// Far-field population J f^eq(rho_inf, U_inf, U_inf) for direction a (runtime a).
template <class L, class T>
__device__ __forceinline__ void feq_farfield(const CellGeo<L, T>& g, T rho_inf, const T* Uinf, T* fe) {
  const EqCoef<L, T> e = eq_coef<L, T>(g, rho_inf, Uinf, Uinf);
  feq_all<L, T>(g, e, fe);
}

}  // namespace vlbm

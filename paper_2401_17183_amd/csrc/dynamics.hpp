// Per-cell dynamics of the volumetric curvilinear LBM (Sec. 2.2), templated on
// the lattice L, the arithmetic type T and the register type AT of the link
// coefficients A (FP32 registers halve their footprint when T is FP64; every
// use converts to T).  Everything here runs in registers of one thread; the
// kernels around it do the data movement.
#pragma once

#include "common.hpp"

namespace vlbm {

// Per-cell geometry as the collision needs it, held in registers of type AT
// (the storage type) and converted to the arithmetic type T at each use.  The
// link coefficients live either in registers (STRIDE = 0) or in LDS, word
// (a - 1) * D + i at lds[word * STRIDE] (STRIDE = threads per block).
//
// Static meshes hold them in pair form: every direction a >= 1 has its
// opposite at a + 1 (odd a), and slot a holds S_a = A_a + A_(a+1), slot a + 1
// D_a = A_a - A_(a+1).  Every sum of the collision over directions pairs the
// coefficients that way (the incoming coefficient of a is A_opp(a)), so the
// pair form saves the sums and differences in each fixed-point iteration.
// Moving meshes hold the outgoing coefficients A_a and the incoming ones.
template <class L, class T, class AT = T, int STRIDE = 0> struct CellGeo {
  // g^{ij} carries a low word when the words are narrower than the arithmetic
  static constexpr bool LO = sizeof(AT) < sizeof(T);
  // a moving mesh staged in LDS keeps the incoming coefficients of its first
  // KR directions in registers.  D3Q19: with all 108 words in LDS two 64-thread
  // blocks fit a CU's 160 KiB; with 10 directions kept (78 words, 39,936
  // bytes per block) four, one wavefront per SIMD; keeping 16 (60 words,
  // 30,720 bytes, 510 VGPRs and no spills) reads fewer words from LDS in each
  // fixed-point iteration and measured 8 % faster than 10 (14: 476 VGPRs, 1 %
  // slower than 16; 18 spills)
  static constexpr int KR = (L::MOVING && STRIDE) ? 16 : 0;
  static_assert(KR < L::Q, "more kept directions than the lattice has");
  // a static D3Q39 mesh keeps the outgoing coefficients of its first KA
  // directions in registers where that fits more blocks into a CU's 160 KiB
  // of LDS: FP64 words, 105 of 114 in LDS take 53,760 bytes per 64 threads,
  // three blocks instead of two (454 VGPRs, measured 33 % faster); FP32 words
  // with FP32 arithmetic, 26,880 bytes, six blocks instead of five (238
  // VGPRs, 7 % faster).  D3Q19 with FP32 arithmetic (FP32C, FP16S, BF16S)
  // keeps one direction: 52,224 bytes per 256 threads, three blocks per CU
  // with the kernel held to three wavefronts per SIMD (164 VGPRs; 16-bit
  // storage 9 % faster, FP32C unchanged at its HBM limit).  FP32 words with
  // FP64 arithmetic have no registers to spare.
  static constexpr int KA =
      (!L::MOVING && STRIDE && (sizeof(AT) == 8 || (L::Q > 21 && sizeof(T) == 4))) ? 3
      : (!L::MOVING && STRIDE && L::Q == 19 && sizeof(T) == 4) ? 1 : 0;
  // LDS words per thread: the outgoing coefficients, then the incoming ones
  // of the directions after the first KR
  static constexpr int LDS_WORDS = (L::Q - 1 - KA) * L::D + (L::MOVING ? (L::Q - 1 - KR) * L::D : 0);
  AT J;
  AT gup[nup<L::D>()];     // g^{ij}, upper triangle
  AT gup_lo[LO ? nup<L::D>() : 1];   // g^{ij} - gup (FP32 words, FP64 arithmetic)
  AT aext[L::D];           // a_ext^i = G . g^i
  AT Areg[STRIDE ? (KA ? KA : 1) : L::Q][L::D];   // (with LDS staging, row al - 1 holds direction al <= KA)
  // moving meshes: the incoming coefficients, after the outgoing ones in LDS
  // (with LDS staging, row al - 1 holds direction al <= KR)
  AT Ainreg[(L::MOVING && !STRIDE) ? L::Q : (KR ? KR : 1)][L::D];
  const AT* lds;
  int lofs;                // added to every LDS index (0); re-defined per fixed-point iteration
  __device__ __forceinline__ T j() const { return T(J); }
  __device__ __forceinline__ T ae(int i) const { return T(aext[i]); }
  // coefficient slot al: on a moving mesh the outgoing link coefficient A^i_al
  // (eq. (gamma) contracted with c_al), on a static one S or D of its pair
  __device__ __forceinline__ AT a(int al, int i) const {
    if constexpr (STRIDE == 0) {
      return Areg[al][i];
    } else if constexpr (KA > 0) {
      if (al == 0) return AT(0);
      if (al <= KA) return Areg[al - 1][i];
      return lds[lofs + ((al - 1 - KA) * L::D + i) * STRIDE];
    } else {
      return al == 0 ? AT(0) : lds[lofs + ((al - 1) * L::D + i) * STRIDE];
    }
  }
  // moving meshes: the incoming coefficient of al
  __device__ __forceinline__ AT ain(int al, int i) const {
    static_assert(L::MOVING, "a static mesh takes the opposite outgoing coefficient (pair form)");
    if constexpr (STRIDE == 0) return Ainreg[al][i];
    else if (al == 0) return AT(0);
    else if (al <= KR) return Ainreg[al - 1][i];
    else return lds[lofs + ((L::Q - 1) * L::D + (al - 1 - KR) * L::D + i) * STRIDE];
  }
};

// Pair form of the outgoing coefficients A_a, A_(a+1) of an opposite pair.
template <class T>
__host__ __device__ __forceinline__ void pair_form(T ap, T am, T& s, T& d) {
  s = ap + am;
  d = ap - am;
}

template <class L, class T, class AT, int ST>
__device__ __forceinline__ T gval(const CellGeo<L, T, AT, ST>& g, int i, int j) {
  if constexpr (CellGeo<L, T, AT, ST>::LO) return T(g.gup[up<L::D>(i, j)]) + T(g.gup_lo[up<L::D>(i, j)]);
  else return T(g.gup[up<L::D>(i, j)]);
}

template <class V>
__device__ __forceinline__ void pin(V& v) {
  if constexpr (sizeof(V) == 8) {
    asm volatile("" : "+v"(v));
  } else {
    asm volatile("" : "+v"(v));
  }
}

template <class L, class T, class AT, int ST>
__device__ __forceinline__ void pin_scalars(CellGeo<L, T, AT, ST>& g, T& rho) {
  if constexpr (ST != 0) asm volatile("" : "+s"(g.lofs));   // wave-uniform: a scalar register
  pin(g.J);
#pragma unroll
  for (int k = 0; k < nup<L::D>(); ++k) {
    pin(g.gup[k]);
    if constexpr (CellGeo<L, T, AT, ST>::LO) pin(g.gup_lo[k]);
  }
#pragma unroll
  for (int i = 0; i < L::D; ++i) pin(g.aext[i]);
  pin(rho);
}

// A^i_a in the arithmetic type.  When A is held narrower than T, the empty
// register constraint keeps the widening inside the fixed-point loop instead
// of letting it be hoisted (which would keep a wide copy of every A live).
template <class T, class AT>
__device__ __forceinline__ T widen(AT v) {
  if constexpr (sizeof(AT) < sizeof(T)) asm volatile("" : "+v"(v));
  return T(v);
}

// A_p and A_q (all components) in the arithmetic type.  From LDS (ST > 0) the
// loads carry the per-iteration offset lofs, so neither they nor their
// widening can be hoisted out of the fixed point and no register barrier is
// needed: the waits for the loads fall where the values are used.
template <class L, class T, class AT, int ST>
__device__ __forceinline__ void a_pair(const CellGeo<L, T, AT, ST>& g, int p, int q, T* ap, T* aq) {
#pragma unroll
  for (int i = 0; i < L::D; ++i) {
    if constexpr (ST != 0) {
      ap[i] = T(g.a(p, i));
      aq[i] = T(g.a(q, i));
    } else {
      ap[i] = widen<T>(g.a(p, i));
      aq[i] = widen<T>(g.a(q, i));
    }
  }
}

// S and D of the opposite pair (p, p + 1) of a static mesh in the arithmetic type.
template <class L, class T, class AT, int ST>
__device__ __forceinline__ void sd_pair(const CellGeo<L, T, AT, ST>& g, int p, T* s, T* d) {
  static_assert(!L::MOVING, "moving meshes keep outgoing and incoming coefficients");
  a_pair<L, T, AT, ST>(g, p, p + 1, s, d);
}

// Incoming coefficients of the pair (p, q) in the arithmetic type (moving
// meshes only; a static mesh takes the pair's outgoing ones crosswise).
template <class L, class T, class AT, int ST>
__device__ __forceinline__ void ain_pair(const CellGeo<L, T, AT, ST>& g, int p, int q, T* ip, T* iq) {
#pragma unroll
  for (int i = 0; i < L::D; ++i) {
    if constexpr (ST != 0) {
      ip[i] = T(g.ain(p, i));
      iq[i] = T(g.ain(q, i));
    } else {
      ip[i] = widen<T>(g.ain(p, i));
      iq[i] = widen<T>(g.ain(q, i));
    }
  }
}

// Collision matrix of eq. (collide): M = -s I + (s - 1/tau) H, with H the
// projector onto the Hermite content of order <= 2 (the span of w, w c and
// w H2).  Every such M satisfies eq. (matrix); s = 1/tau is BGK and s = 1 the
// regularised collision.  Applied to f - f^eq, which carries no mass and no
// momentum,
//   Omega_a = -s (N_a - J f^eq_a) + (s - 1/tau) w_a H2_a : Pi_neq / (2 T0),
//   Pi_neq  = sum_a c_a c_a (N_a - J f^eq_a) = S2 - J rho (T0 g + Ut Ut),
// S2 = sum_a c_a c_a N_a (the second moment of f^eq is exact on the lattice).
// The second term has the w H2 : . / T0 form of dN, so the collision is BGK at
// rate s with c1 Pi_neq / J (c1 = (s - 1/tau) / 2) added to dPi inside dN.
template <class T> struct Relax {
  T tau;
  T s;          // rate of the non-hydrodynamic part (1/tau for BGK)
  T c1;         // (s - 1/tau) / 2
  int general;  // 0: BGK (c1 = 0, the stress terms are skipped)
};

template <class T>
__device__ __forceinline__ Relax<T> make_relax(T tau, T tau_g, int general) {
  Relax<T> r;
  const T inv_tau = T(1) / tau;
  r.tau = tau;
  r.general = general;
  r.s = general ? T(1) / tau_g : inv_tau;
  r.c1 = general ? T(0.5) * (r.s - inv_tau) : T(0);
  return r;
}

// S2 = sum_a c_a c_a N_a (upper triangle) scaled by f; returns its trace.
template <class L, class T, class NS>
__device__ __forceinline__ T second_moment(const NS* N, T f, T* S2) {
  constexpr int D = L::D;
#pragma unroll
  for (int k = 0; k < nup<D>(); ++k) S2[k] = 0;
#pragma unroll
  for (int a = 1; a < L::Q; ++a) {
    const T n = T(N[a]);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j) {
        const int cc = L::c(a, i) * L::c(a, j);
        if (cc != 0) S2[up<D>(i, j)] += T(cc) * n;
      }
  }
  T tr = 0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      S2[up<D>(i, j)] *= f;
      if (i == j) tr += S2[up<D>(i, j)];
    }
  return tr;
}

// Per-cell scalars of the equilibrium that do not depend on the direction.
template <class L, class T> struct EqCoef {
  T rho, trG, U[L::D], Ut[L::D], r[L::D];
};

// Direction-independent parts of eq. (equilibrium):
//  G^{ij} = (g^{ij} - d^{ij}) T0 + Ut^i Ut^j        -> its trace
//  R^{ijk} (fully symmetric)                          -> r^i = sum_j R^{ijj}
//         = T0 [2 (g Ut)^i + tr(g) Ut^i - (D + 2) U^i] + |Ut|^2 Ut^i
template <class L, class T, class AT, int ST>
__device__ __forceinline__ EqCoef<L, T> eq_coef(const CellGeo<L, T, AT, ST>& g, T rho, const T* U, const T* Ut) {
  constexpr int D = L::D;
  const T t0 = T(L::T0);
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
template <class L, class T, class AT, int ST, int a>
__device__ __forceinline__ T feq_dir(const CellGeo<L, T, AT, ST>& g, const EqCoef<L, T>& e) {
  constexpr int D = L::D;
  const T t0 = T(L::T0);
  T cU = 0, cUt = 0, cr = 0, cgc = 0;
  int cc = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
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
  const T H2G = cGc * T(L::INV_T0) - e.trG;
  const T H3R = T(3) * t0 * (cgc * cUt - T(cc) * cU) + cUt * cUt * cUt - T(3) * t0 * cr;
  // factors 1/T0, 1/(2 T0), 1/(6 T0^3) of the lattice (3, 3/2, 9/2 for T0 = 1/3)
  return e.rho * T(L::w(a)) * (T(1) + T(L::INV_T0) * cU + T(L::INV_2T0) * H2G + T(L::INV_6T03) * H3R);
}

// Directions a and a + 1 are opposite (c_(a+1) = -c_a) for every odd a.
template <class L>
constexpr bool opposite_pair(int a) {
  if (a < 1 || a + 1 >= L::Q || L::w(a) != L::w(a + 1)) return false;
  for (int i = 0; i < L::D; ++i)
    if (L::c(a + 1, i) != -L::c(a, i)) return false;
  return true;
}

// f^eq of an opposite pair (a, a + 1): the part of eq. (equilibrium) even in c,
// rho w (1 + H2:G/(2 T0)), is shared and the odd part, rho w (c.U/T0 +
// H3:R/(6 T0^3)), changes sign, so f^eq_a = even + odd and f^eq_(a+1) =
// even - odd cost one evaluation.
template <class L, class T, class AT, int ST, int a>
__device__ __forceinline__ void feq_parts(const CellGeo<L, T, AT, ST>& g, const EqCoef<L, T>& e, T& even, T& odd) {
  constexpr int D = L::D;
  static_assert(opposite_pair<L>(a), "feq_parts takes a direction a whose opposite is a + 1");
  const T t0 = T(L::T0);
  T cU = 0, cUt = 0, cr = 0, cgc = 0;
  int cc = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
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
  const T H2G = cGc * T(L::INV_T0) - e.trG;
  const T H3R = T(3) * t0 * (cgc * cUt - T(cc) * cU) + cUt * cUt * cUt - T(3) * t0 * cr;
  const T rw = e.rho * T(L::w(a));
  even = rw * (T(1) + T(L::INV_2T0) * H2G);
  odd = rw * (T(L::INV_T0) * cU + T(L::INV_6T03) * H3R);
}

template <class L, class T, class AT, int ST, int a = 0>
__device__ __forceinline__ void feq_all(const CellGeo<L, T, AT, ST>& g, const EqCoef<L, T>& e, T* fe) {
  if constexpr (a < L::Q) {
    fe[a] = feq_dir<L, T, AT, ST, a>(g, e);
    feq_all<L, T, AT, ST, a + 1>(g, e, fe);
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
  return T(L::w(a)) * J * (T(L::INV_T0) * cF + T(L::INV_T0) * (T(L::INV_T0) * cpc - trdpi));
}

// Pass 1 of one fixed-point iteration, with the equilibrium at the current Ut:
//   X^i  = sum_a A^i_a f^eq_a,   Xo^i = sum_a A^i_opp(a) f^eq_a (if wanted),
//   M^{ij} = sum_a c^i_a S^j_a f^eq_a,  S_a = A_a + A_opp(a),
// accumulated over opposite pairs (S_a = S_opp(a), c_opp(a) = -c_a) without
// storing f^eq.  With f^eq = even +- odd over the pair, a static mesh's pair
// adds S even + D odd to X, S even - D odd to Xo and 2 c S odd to M; M is
// returned halved (the factor 2 sits in finish_dpi).
template <class L, class T, class AT, int ST, bool WITH_XO, int p = 1>
__device__ __forceinline__ void pass_feq(const CellGeo<L, T, AT, ST>& g, const EqCoef<L, T>& e, T* X, T* Xo,
                                         T (*M)[L::D]) {
  if constexpr (p < L::Q) {
    T even, odd;
    feq_parts<L, T, AT, ST, p>(g, e, even, odd);
    if constexpr (!L::MOVING) {
      T sp[L::D], dp[L::D];
      sd_pair<L, T, AT, ST>(g, p, sp, dp);
#pragma unroll
      for (int i = 0; i < L::D; ++i) {
        X[i] += sp[i] * even + dp[i] * odd;
        if constexpr (WITH_XO) Xo[i] += sp[i] * even - dp[i] * odd;
      }
#pragma unroll
      for (int i = 0; i < L::D; ++i) {
        const int ci = L::c(p, i);
        if (ci == 0) continue;
#pragma unroll
        for (int j = 0; j < L::D; ++j) M[i][j] += T(ci) * sp[j] * odd;
      }
    } else {
      T ap[L::D], am[L::D];
      a_pair<L, T, AT, ST>(g, p, p + 1, ap, am);
      const T fp = even + odd, fm = even - odd;
      // S_a = A_a + Ain_a differs between the two members of the pair
      T ip[L::D], im[L::D];
      ain_pair<L, T, AT, ST>(g, p, p + 1, ip, im);
#pragma unroll
      for (int i = 0; i < L::D; ++i) {
        X[i] += ap[i] * fp + am[i] * fm;
        if constexpr (WITH_XO) Xo[i] += ip[i] * fp + im[i] * fm;
      }
#pragma unroll
      for (int i = 0; i < L::D; ++i) {
        const int ci = L::c(p, i);
        if (ci == 0) continue;
#pragma unroll
        for (int j = 0; j < L::D; ++j) M[i][j] += T(0.5 * ci) * ((ap[j] + ip[j]) * fp - (am[j] + im[j]) * fm);
      }
    }
    pass_feq<L, T, AT, ST, WITH_XO, p + 2>(g, e, X, Xo, M);
  }
}

// dN of an opposite pair (a, a + 1): the stress part w J H2:dPi/T0 is even in
// c and the force part w J c.F/T0 odd, so dN_a = even + odd and dN_(a+1) =
// even - odd.
template <class L, class T, int a>
__device__ __forceinline__ void delta_n_parts(T J, const T* Ft, const T* dpi, T trdpi, T& even, T& odd) {
  constexpr int D = L::D;
  static_assert(opposite_pair<L>(a), "delta_n_parts takes a direction a whose opposite is a + 1");
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
  const T wJ = T(L::w(a)) * J;
  even = wJ * (T(L::INV_T0) * (T(L::INV_T0) * cpc - trdpi));
  odd = wJ * (T(L::INV_T0) * cF);
}

// Pass 2: Y^i = sum_a A^i_a dN_a, dN with the volume J (a static mesh's pair
// adds S even + D odd).
template <class L, class T, class AT, int ST, int a = 1>
__device__ __forceinline__ void pass_dn_j(const CellGeo<L, T, AT, ST>& g, T J, const T* Ft, const T* dpi, T trdpi,
                                          T* Y) {
  if constexpr (a < L::Q) {
    T even, odd;
    delta_n_parts<L, T, a>(J, Ft, dpi, trdpi, even, odd);
    if constexpr (!L::MOVING) {
      T sp[L::D], dp[L::D];
      sd_pair<L, T, AT, ST>(g, a, sp, dp);
#pragma unroll
      for (int i = 0; i < L::D; ++i) Y[i] += sp[i] * even + dp[i] * odd;
    } else {
      T ap[L::D], am[L::D];
      a_pair<L, T, AT, ST>(g, a, a + 1, ap, am);
      const T dp = even + odd, dm = even - odd;
#pragma unroll
      for (int i = 0; i < L::D; ++i) Y[i] += ap[i] * dp + am[i] * dm;
    }
    pass_dn_j<L, T, AT, ST, a + 2>(g, J, Ft, dpi, trdpi, Y);
  }
}

template <class L, class T, class AT, int ST>
__device__ __forceinline__ void pass_dn(const CellGeo<L, T, AT, ST>& g, const T* Ft, const T* dpi, T trdpi, T* Y) {
  pass_dn_j<L, T, AT, ST>(g, g.j(), Ft, dpi, trdpi, Y);
}

// Output pass: N'_a = N_a - s (N_a - J f^eq_a) + dN_a  (eqs. (lbe), (collide));
// s = 1/tau for BGK, and dPi carries the stress term of a general M.
template <class L, class T, class AT, int ST, class NS, int a = 1>
__device__ __forceinline__ void pass_out(const CellGeo<L, T, AT, ST>& g, const EqCoef<L, T>& e, const NS* N, const T* Ft,
                                         const T* dpi, T trdpi, T s, T* Np) {
  if constexpr (a == 1) {   // rest direction: c = 0, no force part
    const T n = T(N[0]);
    Np[0] = n - (n - g.j() * feq_dir<L, T, AT, ST, 0>(g, e)) * s + delta_n_dir<L, T, 0>(g.j(), Ft, dpi, trdpi);
  }
  if constexpr (a < L::Q) {
    T fe, fo, de, dd;
    feq_parts<L, T, AT, ST, a>(g, e, fe, fo);
    delta_n_parts<L, T, a>(g.j(), Ft, dpi, trdpi, de, dd);
    const T np = T(N[a]), nm = T(N[a + 1]);
    Np[a] = np - (np - g.j() * (fe + fo)) * s + (de + dd);
    Np[a + 1] = nm - (nm - g.j() * (fe - fo)) * s + (de - dd);
    pass_out<L, T, AT, ST, NS, a + 2>(g, e, N, Ft, dpi, trdpi, s, Np);
  }
}

// Symmetrised dPi of eq. (delta-flux) from M of pass 1 (halved), plus the
// body-force reading 1/2 k (Ut^i rho a^j + rho a^i Ut^j), k = 1 - 1/(2 tau).
// Returns tr dPi.
template <class L, class T, class AT, int ST>
__device__ __forceinline__ T finish_dpi(const CellGeo<L, T, AT, ST>& g, T (*M)[L::D], const T* Ut, T rho, T k, T* dpi) {
  constexpr int D = L::D;
  T tr = 0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      const T v = T(-0.5) * k * (M[i][j] + M[j][i]) + T(0.5) * k * rho * (Ut[i] * g.ae(j) + g.ae(i) * Ut[j]);
      dpi[up<D>(i, j)] = v;
      if (i == j) tr += v;
    }
  return tr;
}

// State of one cell's collision between its phases.
template <class L, class T, class MT = T> struct CollState {
  T rho, invJ, half_inv_rho, cJ;
  T U[L::D], BC[L::D];          // BC = B - (1 - s) C / 2 - Z / 2 (constant part of J F)
  T Ut[L::D], Ft[L::D];
  T dpi[nup<L::D>()], trdpi;
  EqCoef<L, T> e;
  MT lm[L::D * (L::D + nup<L::D>() + 1)];      // link moments P, Q, R (add_link_moments), type of A
  int iters;                    // iterations used; max_iter + 1 when the cap was hit
};

// sum_a A^i_a dN_a is linear in Ft and dPi (eq. (deltaN)):
//   sum_a A^i_a dN_a = J/T0 [P^{ik} Ft_k + Q^{i,jk} dPi_jk / T0 - R^i tr dPi],
//   P^{ik} = sum_a A^i_a w_a c^k_a,  Q^{i,jk} = sum_a A^i_a w_a c^j_a c^k_a,
//   R^i = sum_a A^i_a w_a,
// with geometry-only moments, so the fixed point needs no pass over the
// directions for it.  Held in the storage type of A (words [P | Q over the
// upper triangle, the off-diagonal entries doubled | R] per component i): in
// FP32 they weight the small force and stress corrections only, where their
// rounding stays far below the fixed point's tolerance.
template <class L> constexpr int lm_words() { return L::D + nup<L::D>() + 1; }

// Adds the opposite pair (a, a + 1) to the link moments m[i][word]: with
// c_(a+1) = -c_a, P takes D = A_a - A_(a+1) and Q, R take S = A_a + A_(a+1).
template <class L, class T, int a>
__device__ __forceinline__ void add_link_moments(const T* sp, const T* dp, T (*m)[lm_words<L>()]) {
  constexpr int D = L::D;
  constexpr int NU = nup<D>();
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const T dif = dp[i];
    const T sum = sp[i];
#pragma unroll
    for (int k = 0; k < D; ++k)
      if (L::c(a, k) != 0) m[i][k] += T(L::w(a) * L::c(a, k)) * dif;
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int k = j; k < D; ++k) {
        const int cc = (j == k ? 1 : 2) * L::c(a, j) * L::c(a, k);
        if (cc != 0) m[i][D + up<D>(j, k)] += T(L::w(a) * cc) * sum;
      }
    m[i][D + NU] += T(L::w(a)) * sum;
  }
}

// sum_a A^i_a dN_a from the link moments (narrow words are widened at each use).
template <class L, class T, class MT>
__device__ __forceinline__ void dn_from_moments(const MT* lm, T J, const T* Ft, const T* dpi, T trdpi, T* Y) {
  constexpr int D = L::D;
  constexpr int NU = nup<D>();
  constexpr int W = lm_words<L>();
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T f = 0, q = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) f += widen<T>(lm[i * W + k]) * Ft[k];
#pragma unroll
    for (int k = 0; k < NU; ++k) q += widen<T>(lm[i * W + D + k]) * dpi[k];
    Y[i] = J * T(L::INV_T0) * (f + T(L::INV_T0) * q - widen<T>(lm[i * W + D + NU]) * trdpi);
  }
}

// The sums of phase 1 over the opposite pairs (a, a + 1), each pair's
// coefficients read and widened once: rho J, J rho U, C, B and (ST > 0) the
// link moments.  A static mesh's pair (sigma = N_a + N_(a+1), delta = N_a -
// N_(a+1)) adds (S sigma + D delta) / 2 to C and -(S sigma - D delta) / 4 to
// B; C and B collect sum S sigma and sum D delta, and collide_prepare forms
// C and B from them.
template <class L, class T, class AT, int ST, class NS, int a = 1>
__device__ __forceinline__ void prepare_pairs(const CellGeo<L, T, AT, ST>& g, const NS* N, T& rhoJ, T* mom, T* C, T* B,
                                              T (*m)[lm_words<L>()]) {
  if constexpr (a < L::Q) {
    constexpr int D = L::D;
    static_assert(opposite_pair<L>(a), "prepare_pairs walks opposite pairs (a, a + 1)");
    const T np = T(N[a]), nm = T(N[a + 1]);
    const T sn = np + nm, dn = np - nm;
    rhoJ += sn;
#pragma unroll
    for (int i = 0; i < D; ++i)
      if (L::c(a, i) != 0) mom[i] += T(L::c(a, i)) * dn;
    if constexpr (!L::MOVING) {
      T sp[D], dp[D];
      sd_pair<L, T, AT, ST>(g, a, sp, dp);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        C[i] += sp[i] * sn;
        B[i] += dp[i] * dn;
      }
      if constexpr (ST != 0) add_link_moments<L, T, a>(sp, dp, m);
    } else {
      T ap[D], am[D], ip[D], im[D];   // outgoing and incoming coefficients of the pair
      a_pair<L, T, AT, ST>(g, a, a + 1, ap, am);
      ain_pair<L, T, AT, ST>(g, a, a + 1, ip, im);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        C[i] += ap[i] * np + am[i] * nm;
        B[i] -= T(0.5) * (ip[i] * np + im[i] * nm);
      }
      if constexpr (ST != 0) {
        T sp[D], dp[D];
#pragma unroll
        for (int i = 0; i < D; ++i) pair_form(ap[i], am[i], sp[i], dp[i]);
        add_link_moments<L, T, a>(sp, dp, m);
      }
    }
    prepare_pairs<L, T, AT, ST, NS, a + 2>(g, N, rhoJ, mom, C, B, m);
  }
}

// Phase 1: moments (eqs. (dist), (moments), (vcurvi)) and the parts of
// eq. (compo-constr) that do not change during the fixed point:
//   B^i = -1/2 sum_a A^i_opp(a) N_a,  C^i = sum_a A^i_a N_a  and, for a general
//   M, Z^i = sum_a A^i_a dN_a(F = 0, dPi = c1 S2 / J) (the population part of
//   the stress term, linear in dPi).
template <class L, class T, class AT, int ST, class NS>
__device__ __forceinline__ void collide_prepare(const CellGeo<L, T, AT, ST>& g, const NS* N, const Relax<T>& r,
                                                CollState<L, T, AT>& st) {
  constexpr int D = L::D;
  constexpr int Q = L::Q;
  constexpr int W = lm_words<L>();
  T rhoJ = T(N[0]);
  T mom[D], C[D], B[D], m[ST ? D : 1][W];
#pragma unroll
  for (int i = 0; i < D; ++i) mom[i] = C[i] = B[i] = 0;
  if constexpr (ST != 0)
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < W; ++k) m[i][k] = 0;
  prepare_pairs<L, T, AT, ST, NS>(g, N, rhoJ, mom, C, B, m);
  if constexpr (!L::MOVING)
#pragma unroll
    for (int i = 0; i < D; ++i) {   // C, B from sum S sigma (in C) and sum D delta (in B)
      const T ss = C[i], dd = B[i];
      C[i] = T(0.5) * (ss + dd);
      B[i] = T(-0.25) * (ss - dd);
    }
  // two divisions: 1/J and 1/(rho J)
  const T inv_rhoJ = T(1) / rhoJ;
  st.invJ = T(1) / g.j();
  st.rho = rhoJ * st.invJ;
  st.half_inv_rho = T(0.5) * g.j() * inv_rhoJ;
  st.cJ = g.j() * r.s;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    st.U[i] = mom[i] * inv_rhoJ;
    st.BC[i] = B[i] - T(0.5) * (T(1) - r.s) * C[i];
  }
  // with A in LDS the registers hold the link moments instead of a pass over A
  if constexpr (ST != 0)
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < W; ++k) st.lm[i * W + k] = AT(m[i][k]);
  if (r.general) {   // wave-uniform
    // dN is J times a function of dPi: with J = 1 and dPi = c1 S2 the product
    // J dPi = c1 S2 is the same.  Z and the stress term of the iterations
    // cancel to the small non-equilibrium part, so both take the same moments.
    T S2[nup<D>()], Z[D], zero[D];
    const T tr = second_moment<L, T, NS>(N, r.c1, S2);
#pragma unroll
    for (int i = 0; i < D; ++i) Z[i] = zero[i] = 0;
    if constexpr (ST != 0) dn_from_moments<L, T, AT>(st.lm, T(1), zero, S2, tr, Z);
    else pass_dn_j<L, T, AT, ST>(g, T(1), zero, S2, tr, Z);
#pragma unroll
    for (int i = 0; i < D; ++i) st.BC[i] -= T(0.5) * Z[i];
  }
}

// Phase 2: the implicit inertial force (eq. (compo-constr) and the remark
// after eq. (deltaN)) as a fixed point on F, iterated until
// max_i |F_k - F_(k-1)| <= tol * rho.  F holds the starting guess on entry
// (0, or the previous step's converged F: the converged fixed point does not
// depend on it) and the converged F on exit; st keeps the equilibrium, dPi and
// F_tot of the last iteration for the output phase.  Each iteration uses
//   sum_a A_a N'_a = (1 - s) C + J s sum_a A_a f^eq_a + sum_a A_a dN_a
// so that no per-direction array is live inside the loop (s = 1/tau for BGK;
// for a general M, dN includes the stress term, whose population part Z is
// constant and sits in BC).  With A staged in LDS the last sum comes from the
// link moments, so an iteration walks the directions once (for X and dPi).
template <class L, class T, class AT, int ST>
__device__ __forceinline__ void collide_iterate(CellGeo<L, T, AT, ST>& gl, const Relax<T>& r, T tol, int max_iter,
                                                T* F, CollState<L, T, AT>& st, int min_iter = 1) {
  constexpr int D = L::D;
  const T k = T(1) - T(0.5) / r.tau;
  int it = 1;
  int done = 0;
  T& rho_l = st.rho;
  T prev = T(0);
  for (; it <= max_iter; ++it) {
    // Re-define the per-cell scalars each iteration (empty register
    // constraints, in place: the values do not change): quantities derived from
    // them (c.g.c per direction, rho w, widened g^{ij}) are then recomputed
    // instead of being kept live across iterations, which keeps the register
    // footprint and occupancy reasonable.
    pin_scalars<L, T, AT, ST>(gl, rho_l);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      st.Ft[i] = F[i] + rho_l * gl.ae(i);
      st.Ut[i] = st.U[i] + st.Ft[i] * st.half_inv_rho;
    }
    st.e = eq_coef<L, T, AT, ST>(gl, rho_l, st.U, st.Ut);
    T X[D], M[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      X[i] = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) M[i][j] = 0;
    }
    pass_feq<L, T, AT, ST, false>(gl, st.e, X, nullptr, M);
    st.trdpi = finish_dpi<L, T, AT, ST>(gl, M, st.Ut, rho_l, k, st.dpi);
    if (r.general) {   // wave-uniform: the f^eq part of the stress term, -c1 rho (T0 g + Ut Ut)
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
          const T v = r.c1 * rho_l * (T(L::T0) * gval(gl, i, j) + st.Ut[i] * st.Ut[j]);
          st.dpi[up<D>(i, j)] -= v;
          if (i == j) st.trdpi -= v;
        }
    }
    T Y[D];
    if constexpr (ST != 0) {
      dn_from_moments<L, T, AT>(st.lm, gl.j(), st.Ft, st.dpi, st.trdpi, Y);
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) Y[i] = 0;
      pass_dn<L, T, AT, ST>(gl, st.Ft, st.dpi, st.trdpi, Y);
    }
    T change = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const T Fn = (st.BC[i] - T(0.5) * (st.cJ * X[i] + Y[i])) * st.invJ;
      const T dd = Fn - F[i];
      change = fmax(change, dd < T(0) ? -dd : dd);
      F[i] = Fn;
    }
    if (change <= tol * rho_l && it >= min_iter) {
      done = 1;
      break;
    }
    // FP32 arithmetic: on coarse, strongly stretched meshes the change can
    // stall at the rounding level of the sums (the terms of eq.
    // (compo-constr) are far larger than F) just above the tolerance; an
    // iterate whose change no longer decreases and lies within 16 tolerances
    // is as close as this precision gets
    if constexpr (sizeof(T) == 4) {
      if (it > min_iter && change >= prev && change <= T(16) * tol * rho_l) {
        done = 1;
        break;
      }
    }
    prev = change;
  }
  st.iters = done ? it : max_iter + 1;
}

// Between phases 2 and 3: the equilibrium and the force part of dN take the
// newest F (the output of the last iteration), and dPi stays that of the last
// iteration.  The stopping rule bounds |F_k - F_(k-1)|; the distance of F_k
// from the fixed point is smaller than that of F_(k-1) by the contraction
// factor, so the output sits closer to the converged step for the same number
// of iterations (any convergent solver reaches the same N').
template <class L, class T, class AT, int ST>
__device__ __forceinline__ void collide_refresh(const CellGeo<L, T, AT, ST>& g, const T* F, CollState<L, T, AT>& st) {
#pragma unroll
  for (int i = 0; i < L::D; ++i) {
    st.Ft[i] = F[i] + st.rho * g.ae(i);
    st.Ut[i] = st.U[i] + st.Ft[i] * st.half_inv_rho;
  }
  st.e = eq_coef<L, T, AT, ST>(g, st.rho, st.U, st.Ut);
}

// Phase 3: N' of the last iteration (eqs. (lbe), (collide), (deltaN)); for a
// general M the population part c1 S2 / J of the stress term joins dPi here.
template <class L, class T, class AT, int ST, class NS>
__device__ __forceinline__ void collide_output(const CellGeo<L, T, AT, ST>& g, const NS* N, const Relax<T>& r,
                                               const CollState<L, T, AT>& st, T* Np) {
  if (r.general) {
    T dpi[nup<L::D>()];
    T tr = second_moment<L, T, NS>(N, r.c1 * st.invJ, dpi);
#pragma unroll
    for (int k = 0; k < nup<L::D>(); ++k) dpi[k] += st.dpi[k];
    tr += st.trdpi;
    pass_out<L, T, AT, ST, NS>(g, st.e, N, st.Ft, dpi, tr, r.s, Np);
  } else {
    pass_out<L, T, AT, ST, NS>(g, st.e, N, st.Ft, st.dpi, st.trdpi, r.s, Np);
  }
}

struct CollideOut {
  int iters;   // iterations used; max_iter + 1 when the cap was hit
};

// The whole collision of one cell with N held in registers throughout.
template <class L, class T, class AT, int ST, class NS>
__device__ __forceinline__ CollideOut collide(CellGeo<L, T, AT, ST>& g, const NS* N, const Relax<T>& r, T tol,
                                              int max_iter, T* Np, T* F, T* Ut_out, T* U_out, T& rho_out) {
  CollState<L, T, AT> st;
  collide_prepare<L, T, AT, ST, NS>(g, N, r, st);
  collide_iterate<L, T, AT, ST>(g, r, tol, max_iter, F, st);
  collide_refresh<L, T, AT, ST>(g, F, st);
  collide_output<L, T, AT, ST, NS>(g, N, r, st, Np);
#pragma unroll
  for (int i = 0; i < L::D; ++i) {
    Ut_out[i] = st.Ut[i];
    U_out[i] = st.U[i];
  }
  rho_out = st.rho;
  CollideOut o;
  o.iters = st.iters;
  return o;
}

// Consistent equilibrium (the library's reading for the initial state): find F
// such that with U = Ut - F_tot/(2 rho) the populations N = J f^eq(rho, U, Ut)
// have that F as their collision fixed point.  Omega = 0 there (f = f^eq at
// that Ut), so N' = N + dN and
//   J F = -1/2 sum_a [A_a (N_a + dN_a) + A_opp(a) N_a] = -1/2 [J X + Y + J Xo].
template <class L, class T, class AT, int ST>
__device__ __forceinline__ int consistent_equilibrium(const CellGeo<L, T, AT, ST>& g, T rho, const T* Ut, T tau, T tol,
                                                      int max_iter, T* N, T* F_out) {
  constexpr int D = L::D;
  const T k = T(1) - T(0.5) / tau;
  const T half_inv_rho = T(0.5) / rho;
  T F[D], U[D], Ft[D];
#pragma unroll
  for (int i = 0; i < D; ++i) F[i] = 0;
  int ok = 0;
  for (int it = 0; it < max_iter; ++it) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      Ft[i] = F[i] + rho * g.ae(i);
      U[i] = Ut[i] - Ft[i] * half_inv_rho;
    }
    const EqCoef<L, T> e = eq_coef<L, T, AT, ST>(g, rho, U, Ut);
    T X[D], Xo[D], M[D][D], Y[D], dpi[nup<D>()];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      X[i] = Xo[i] = Y[i] = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) M[i][j] = 0;
    }
    pass_feq<L, T, AT, ST, true>(g, e, X, Xo, M);
    const T trdpi = finish_dpi<L, T, AT, ST>(g, M, Ut, rho, k, dpi);
    pass_dn<L, T, AT, ST>(g, Ft, dpi, trdpi, Y);
    T change = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const T Fn = T(-0.5) * (X[i] + Xo[i] + Y[i] / g.j());
      const T dd = Fn - F[i];
      change = fmax(change, dd < T(0) ? -dd : dd);
      F[i] = Fn;
    }
    if (change <= tol * rho) {
      ok = 1;
      break;
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    Ft[i] = F[i] + rho * g.ae(i);
    U[i] = Ut[i] - Ft[i] * half_inv_rho;
    F_out[i] = F[i];
  }
  const EqCoef<L, T> e = eq_coef<L, T, AT, ST>(g, rho, U, Ut);
  T fe[L::Q];
  feq_all<L, T, AT, ST>(g, e, fe);
#pragma unroll
  for (int a = 0; a < L::Q; ++a) N[a] = g.j() * fe[a];
  return ok;
}

// Far-field populations f^eq(rho_inf, U_inf, U_inf) (multiply by J for N).
template <class L, class T, class AT, int ST>
__device__ __forceinline__ void feq_farfield(const CellGeo<L, T, AT, ST>& g, T rho_inf, const T* Uinf, T* fe) {
  const EqCoef<L, T> e = eq_coef<L, T, AT, ST>(g, rho_inf, Uinf, Uinf);
  feq_all<L, T, AT, ST>(g, e, fe);
}

}  // namespace vlbm

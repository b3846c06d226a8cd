// Core of the fused time step shared by the single-mesh and the batched
// kernels: pull advection (eq. (adv)) + collision (BGK, or a general matrix
// that satisfies eq. (matrix)) with the implicit inertial force (eqs. (lbe),
// (collide), (compo-constr), (delta-flux), (deltaN), (equilibrium)), one
// thread per cell, SoA populations.
#pragma once

#include <type_traits>

#include "dynamics.hpp"

namespace vlbm {

// Resident waves per SIMD that the register budget is held to: two where the
// LDS staging of A (55 KB per 256-thread block for D3Q19 FP32) allows two
// blocks per CU; three for D3Q19 with FP32 arithmetic, whose LDS holds three
// blocks once one direction stays in registers (CellGeo::KA).
template <class L, class S, class T> constexpr int step_min_waves() {
  return (L::Q == 19 && sizeof(S) == 4 && sizeof(T) == 4) ? 3 : 2;
}
#define VLBM_STEP_ATTR __attribute__((amdgpu_waves_per_eu(step_min_waves<L, S, T>(), 8)))

// P: population storage tag (PopCodec); S: geometry storage type; T: arithmetic type.
template <class P, class S, class T> struct StepArgs {
  Box box;
  const PopE<P>* __restrict__ in;
  PopE<P>* __restrict__ out;
  // shifted modes: the reference of every slot, [Q][cells]; the writer encodes
  // against its own slots, the reader decodes at the offset it gathers from
  const PopR<P>* __restrict__ rown;
  // re-basing step (else null): the outputs are re-based as the re-basing
  // kernel would re-base them after the step, the new references go here
  PopR<P>* __restrict__ rown_new;
  float scale, inv_scale;
  const S* __restrict__ geo;
  T tau, tau_g, tol, rho_inf;
  // relaxation rates from the host (kernel arguments, so no lane divides):
  // 1/tau, s = 1/tau_g and c1 = (s - 1/tau) / 2 (tau_g = tau for BGK)
  T inv_tau, relax_s, relax_c1;
  int general;                  // collision matrix other than BGK (tau_g != tau)
  int max_iter, min_iter;
  int stream_only;
  int has_force, has_ff;
  // [D][cells] the converged F per unit density F / rho of the last step in
  // (the starting guess is rho F / rho_prev: most of a step's change of F is
  // the density's, through the metric part of the equilibrium stress), that
  // of this step out: FP64 with FP64 storage, FP32 otherwise (a starting guess
  // only; the converged F does not depend on it)
  typename std::conditional<std::is_same<S, double>::value, double, float>::type* __restrict__ fcache;
  int* flags;
  // optional fixed-point statistics (null: off): [0] sum over cells of the
  // iterations, [1] sum over wavefronts of their largest count (the lanes of a
  // wavefront iterate together), [2] cells, [3] wavefronts
  unsigned long long* stats;
};

// Wavefront sum and maximum of the per-lane iteration counts, from ballots
// (which only see the active lanes: a ragged last wavefront has lanes that
// left early), added by the first active lane to the statistics.
__device__ __forceinline__ void add_iteration_stats(unsigned long long* stats, int iters) {
  const unsigned long long act = __ballot(1);
  unsigned long long sum = 0;
  int mx = 0;
  for (int k = 1;; ++k) {   // wave-uniform: ends at the largest count
    const unsigned long long m = __ballot(iters >= k);
    if (m == 0ull) break;
    sum += (unsigned long long)__popcll(m);
    mx = k;
  }
  const int lane = (int)(threadIdx.x & 63);
  if (lane == __ffsll((long long)act) - 1) {
    // kStatSlots copies of the four counters, chosen by block: one address
    // shared by every wave of a launch serialises their atomics
    unsigned long long* q = stats + 4 * (blockIdx.x & (kStatSlots - 1));
    atomicAdd(&q[0], sum);
    atomicAdd(&q[1], (unsigned long long)mx);
    atomicAdd(&q[2], (unsigned long long)__popcll(act));
    atomicAdd(&q[3], 1ull);
  }
}

// Streaming accesses: data that each step reads once (the packed geometry,
// the force cache) or writes once (the populations, the force cache) goes
// through non-temporal loads and stores, which keeps the caches for the
// gathered populations that neighbouring wavefronts share.  Measured on the
// 256x128x128 channel: FP32C 344 -> 312 us per step, FP16S 341 -> 308 us,
// FP32 493 -> 473 us.  FP64 words load the regular way: the FP64 kernel runs
// one wavefront per SIMD and waited longer on non-temporal loads (827 ->
// 887 us).
template <class X>
__device__ __forceinline__ X load_stream(const X* p) {
  if constexpr (std::is_same<X, float>::value) {
    return __builtin_nontemporal_load(p);
  } else {
    return *p;
  }
}
template <class X>
__device__ __forceinline__ void store_stream(X* p, X v) {
  if constexpr (std::is_same<X, float>::value || std::is_same<X, double>::value) {
    __builtin_nontemporal_store(v, p);
  } else if constexpr (sizeof(X) == 2) {
    unsigned short u;
    __builtin_memcpy(&u, &v, 2);
    __builtin_nontemporal_store(u, reinterpret_cast<unsigned short*>(p));
  } else {
    *p = v;
  }
}

// Word w of a SoA array: the wave-uniform base (w * nc) is formed in scalar
// registers, lanes carry only their 32-bit cell offset.
template <class X>
__device__ __forceinline__ const X* word(const X* __restrict__ base, int w, int nc) {
  return base + (size_t)w * (size_t)nc;
}
template <class X>
__device__ __forceinline__ X* word(X* __restrict__ base, int w, int nc) {
  return base + (size_t)w * (size_t)nc;
}

// Placement of a cell's coefficient of slot a >= 1, component i: the outgoing
// one (put_a) in registers or in this thread's LDS column (stride ST), the
// incoming one of a moving mesh (put_ain) in registers for the first KR
// directions when staged, after the outgoing ones in LDS otherwise.
template <class L, class S, class T, int ST>
__device__ __forceinline__ void put_a(CellGeo<L, T, S, ST>& g, S* lds, int a, int i, S v) {
  if constexpr (ST == 0) g.Areg[a][i] = v;
  else lds[((a - 1) * L::D + i) * ST] = v;
}
template <class L, class S, class T, int ST>
__device__ __forceinline__ void put_ain(CellGeo<L, T, S, ST>& g, S* lds, int a, int i, S v) {
  if constexpr (ST == 0) g.Ainreg[a][i] = v;
  else if (a <= CellGeo<L, T, S, ST>::KR) g.Ainreg[a - 1][i] = v;
  else lds[((L::Q - 1) * L::D + (a - 1 - CellGeo<L, T, S, ST>::KR) * L::D + i) * ST] = v;
}
// The zero coefficients of the rest direction (registers only).
template <class L, class S, class T, int ST>
__device__ __forceinline__ void zero_rest(CellGeo<L, T, S, ST>& g) {
  if constexpr (ST == 0) {
#pragma unroll
    for (int i = 0; i < L::D; ++i) {
      g.Areg[0][i] = S(0);
      if constexpr (L::MOVING) g.Ainreg[0][i] = S(0);
    }
  }
}

// Packed geometry of one cell (static meshes).  With ST > 0 the link
// coefficients are staged in LDS (this thread's column of lds, stride ST)
// instead of registers; only this thread reads its column.
template <class L, class S, class T, int ST>
__device__ __forceinline__ CellGeo<L, T, S, ST> load_pack(const S* __restrict__ geo, int nc, int cell, int has_force,
                                                          S* lds) {
  static_assert(!L::MOVING, "a moving mesh computes its coefficients (MovingGeo)");
  CellGeo<L, T, S, ST> g;
  // this cell's element of word 0 of its tile; word w is w * kGeoTile further
  const S* __restrict__ gw = geo + pack_index<L>(0, cell);
  g.J = load_stream(gw + Pack<L>::J * kGeoTile);
#pragma unroll
  for (int k = 0; k < nup<L::D>(); ++k) {
    g.gup[k] = load_stream(gw + (Pack<L>::GUP + k) * kGeoTile);
    if constexpr (CellGeo<L, T, S, ST>::LO) g.gup_lo[k] = load_stream(gw + (Pack<L>::GUPLO + k) * kGeoTile);
  }
#pragma unroll
  for (int a = 1; a < L::Q; ++a)
#pragma unroll
    for (int i = 0; i < L::D; ++i) {
      const S v = load_stream(gw + (Pack<L>::A + (a - 1) * L::D + i) * kGeoTile);
      constexpr int KA = CellGeo<L, T, S, ST>::KA;
      if constexpr (ST == 0) {
        g.Areg[a][i] = v;
      } else if constexpr (KA > 0) {
        if (a <= KA) g.Areg[a - 1][i] = v;
        else lds[((a - 1 - KA) * L::D + i) * ST] = v;
      } else {
        lds[((a - 1) * L::D + i) * ST] = v;
      }
    }
  if constexpr (ST == 0)
#pragma unroll
    for (int i = 0; i < L::D; ++i) g.Areg[0][i] = S(0);
  g.lds = lds;
  g.lofs = 0;
#pragma unroll
  for (int i = 0; i < L::D; ++i) g.aext[i] = has_force ? load_stream(gw + (Pack<L>::AEXT + i) * kGeoTile) : S(0);
  return g;
}

template <class L, class P, class S, class T, class NR, int al = 0>
__device__ __forceinline__ void gather_dirs(const StepArgs<P, S, T>& a, const LinkPlan& plan, int x, int y, int z,
                                            int cell, NR* N, DirMask<L>& ff) {
  if constexpr (al < L::Q) {
    using C = PopCodec<P>;
    const int nc = a.box.ncells;
    int src;
    // one-cell links resolve from the per-cell plan; longer ones (periodic
    // axes only) wrap their own coordinates
    int kind;
    if constexpr (L::SPEED == 1) kind = link_at<L, al>(plan, cell, src);
    else kind = link_source<L>(a.box, al, x, y, z, src);
    // slot al of src, or (bounced / far field: src = cell) slot opp(al) of the
    // cell, as an element offset from the pair's lower slot array: the base is
    // wave-uniform and the offset (< 2 nc <= 2^31) a 32-bit lane value
    constexpr int lo = opp(al) < al ? opp(al) : al;
    const unsigned e = (unsigned)src + (unsigned)nc * (kind == LINK_INTERIOR ? unsigned(al - lo) : unsigned(opp(al) - lo));
    const PopE<P> h = word(a.in, lo, nc)[e];
    // the slot's reference sits at the same offset of the reference array
    if constexpr (C::shifted) N[al] = C::template decode<NR>(h, word(a.rown, lo, nc)[e], a.inv_scale);
    else N[al] = h;
    ff |= DirMask<L>(kind == LINK_FARFIELD ? 1 : 0) << al;
    gather_dirs<L, P, S, T, NR, al + 1>(a, plan, x, y, z, cell, N, ff);
  }
}

// Pull N_a(q) = N'_a(q - c_a) (eq. (adv)).  Every load is unconditional and in
// bounds (a bounced or far-field link reads the cell's own opposite slot), so
// no lane diverges; far-field links then take J f^eq(rho_inf, U_inf, U_inf),
// evaluated only in the cells that have such a link.
// FF: 0 = no far-field links, 1 = far-field links, 2 = decided at run time
// (has_ff); a compile-time choice keeps the fill out of the control flow.
template <class L, class P, class S, class T, class NR, int ST, int FF = 2>
__device__ __forceinline__ void gather(const StepArgs<P, S, T>& a, const CellGeo<L, T, S, ST>& g, int x, int y,
                                       int z, int cell, NR* N) {
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  using C = PopCodec<P>;
  const int nc = a.box.ncells;
  LinkPlan plan{};
  if constexpr (L::SPEED == 1) plan = link_plan<L>(a.box, x, y, z);
  DirMask<L> ff = 0;
  gather_dirs<L, P, S, T, NR>(a, plan, x, y, z, cell, N, ff);
  // compile-time or wave-uniform, then only cells with a far-field link (a wave
  // without one skips the equilibrium)
  if ((FF == 1 || (FF == 2 && a.has_ff)) && ff != 0) {
    T Uinf[D];
#pragma unroll
    for (int i = 0; i < D; ++i) Uinf[i] = T(a.geo[pack_index<L>(Pack<L>::UINF + i, cell)]);
    T fe[Q];
    feq_farfield<L, T>(g, a.rho_inf, Uinf, fe);
#pragma unroll
    for (int al = 0; al < Q; ++al) N[al] = (ff >> al) & 1 ? NR(g.j() * fe[al]) : N[al];
  }
}

template <class L, class P, class S, class T, class V>
__device__ __forceinline__ void store_slot(const StepArgs<P, S, T>& a, int al, int cell, V v) {
  using C = PopCodec<P>;
  const int nc = a.box.ncells;
  if constexpr (C::shifted)
    store_stream(word(a.out, al, nc) + cell, C::template encode<T>(T(v), word(a.rown, al, nc)[cell], a.scale));
  else store_stream(word(a.out, al, nc) + cell, PopE<P>(v));
}

// Geometry source of a static mesh: the packed words (load_pack).
struct PackGeo {};

// Geometry source of a step on a moving mesh (time t to t + 1, FP64): each
// cell computes its link coefficients from g_i on the geometry boxes of the
// times t - 1, t and t + 1,
//   outgoing  A+^i_a(q, t) = [e_a(q + c_a, t + 1) - e_a(q, t)] . g^i(q, t)
//   incoming  A-^i_a(q, t) = [e_a(q, t) - e_a(q - c_a, t - 1)] . g^i(q, t)
// with e_a = c_a^j g_j, and takes J, g^{ij} and a_ext = G . g^i of time t from
// the real-cell arrays: no coefficient words go through HBM.
struct MovingGeo {
  const double* gprev;   // [d][d][nbox], word j * d + k: component k of g_j
  const double* gcur;
  const double* gnext;
  const double* J;       // time t, real cells: [cells], [d][d][cells], [d][d][cells]
  const double* gup;
  const double* gco;
  int nb[3], nbox, layers;
  double G[3];

  template <class L, class P, class S, class T, int ST>
  __device__ __forceinline__ CellGeo<L, T, S, ST> load(const StepArgs<P, S, T>& a, int x, int y, int z, int cell,
                                                       S* lds) const {
    static_assert(L::MOVING && std::is_same<S, double>::value, "moving meshes step in FP64");
    constexpr int D = L::D;
    const int nc = a.box.ncells;
    const double* __restrict__ gp = gprev;
    const double* __restrict__ gc = gcur;
    const double* __restrict__ gn = gnext;
    const double* __restrict__ gi_w = gco;
    CellGeo<L, T, S, ST> g;
    g.J = J[cell];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j) g.gup[up<D>(i, j)] = gup[(i * D + j) * nc + cell];
    const int b0 = (x + layers) + nb[0] * ((D > 1 ? y + layers : 0) + nb[1] * (D > 2 ? z + layers : 0));
    // g_j(q, t) and g^i(q, t) of this cell, read once for all links
    double gq[D * D], gi[D * D];
#pragma unroll
    for (int w = 0; w < D * D; ++w) {
      gq[w] = gc[(size_t)w * nbox + b0];
      gi[w] = gi_w[(size_t)w * nc + cell];
    }
#pragma unroll
    for (int al = 1; al < L::Q; ++al) {
      const int st = L::c(al, 0) + nb[0] * ((D > 1 ? L::c(al, 1) : 0) + nb[1] * (D > 2 ? L::c(al, 2) : 0));
      double e_cur[D], e_there[D], e_back[D], v[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        double sc = 0, sn = 0, sp = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const int cj = L::c(al, j);
          if (cj != 0) {
            sc += cj * gq[j * D + k];
            sn += cj * gn[(size_t)(j * D + k) * nbox + (b0 + st)];   // e_a(q + c_a, t + 1)
            sp += cj * gp[(size_t)(j * D + k) * nbox + (b0 - st)];   // e_a(q - c_a, t - 1)
          }
        }
        e_cur[k] = sc;
        e_there[k] = sn;
        e_back[k] = sp;
      }
#pragma unroll
      for (int k = 0; k < D; ++k) v[k] = e_there[k] - e_cur[k];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double r = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) r += v[k] * gi[i * D + k];
        put_a<L, S, T, ST>(g, lds, al, i, r);
      }
#pragma unroll
      for (int k = 0; k < D; ++k) v[k] = e_cur[k] - e_back[k];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double r = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) r += v[k] * gi[i * D + k];
        put_ain<L, S, T, ST>(g, lds, al, i, r);
      }
    }
    zero_rest<L, S, T, ST>(g);
    g.lds = lds;
    g.lofs = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double ae = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) ae += G[k] * gi[i * D + k];
      g.aext[i] = a.has_force ? ae : 0.0;
    }
    return g;
  }
};

// One cell of one mesh; BLOCK threads per workgroup share the LDS staging.
// GEN: general collision matrix (compiled separately, so that the BGK kernels
// carry none of its registers).  Src supplies the cell's geometry.
template <class L, class P, class S, class T, int BLOCK, int FF = 2, bool GEN = false, class Src = PackGeo>
__device__ __forceinline__ void step_cell(const StepArgs<P, S, T>& a, int cell, const Src& src = Src()) {
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  // registers hold populations in the storage type, decoded deviations in the
  // arithmetic type (FP32 for 16-bit storage, FP64 for FP32 deviations)
  using NR = typename std::conditional<PopCodec<P>::shifted, T, PopE<P>>::type;
  if (cell >= a.box.ncells) return;
  const int nc = a.box.ncells;
  int x, y, z;
  cell_coords(a.box, cell, x, y, z);
  // FP32 geometry stages A in LDS (55 KB per 256-thread block for D3Q19); so
  // do D3Q39 in FP64 (its 114 A words cannot live in registers) and a moving
  // 3-D mesh in FP64 (outgoing and incoming coefficients, 108 words, 48 of
  // them kept in registers)
  constexpr int ST = (sizeof(S) == 4 || L::Q > 21 || (L::MOVING && D == 3)) ? BLOCK : 0;
  __shared__ S sA[ST ? CellGeo<L, T, S, ST>::LDS_WORDS * BLOCK : 1];
  NR N[Q];
  // (the static path calls load_pack here directly: a wrapper around it was
  // measured to change the register allocation of the static kernels)
  CellGeo<L, T, S, ST> g;
  if constexpr (std::is_same<Src, PackGeo>::value)
    g = load_pack<L, S, T, ST>(a.geo, nc, cell, a.has_force, sA + (ST ? threadIdx.x : 0));
  else g = src.template load<L, P, S, T, ST>(a, x, y, z, cell, sA + (ST ? threadIdx.x : 0));
  // a wavefront without a far-field cell takes the gather compiled without the
  // far-field fill: with the fill in the same code, the compiler issues each
  // direction's loads only after the previous direction's data arrived
  // (measured on the O-grid, where three wavefronts in four have no far-field
  // cell: the FP32 step waited five times longer per wavefront than on the
  // channel)
  bool ffwave = false;
  if constexpr (FF == 2 && L::SPEED == 1) ffwave = a.has_ff && __ballot(on_farfield_face<L>(a.box, x, y, z)) != 0ull;
  if (ffwave) gather<L, P, S, T, NR, ST, FF>(a, g, x, y, z, cell, N);
  else gather<L, P, S, T, NR, ST, (FF == 2 ? 0 : FF)>(a, g, x, y, z, cell, N);
  if (a.stream_only) {
#pragma unroll
    for (int al = 0; al < Q; ++al) store_slot<L>(a, al, cell, N[al]);
    return;
  }
  T F[D];
#pragma unroll
  for (int i = 0; i < D; ++i) F[i] = load_stream(word(a.fcache, i, nc) + cell);
  CollState<L, T, S> st;
  Relax<T> rx;
  rx.tau = a.tau;
  rx.general = GEN ? 1 : 0;
  rx.s = GEN ? a.relax_s : a.inv_tau;
  rx.c1 = GEN ? a.relax_c1 : T(0);
  collide_prepare<L, T, S, ST, NR>(g, N, rx, st);
#pragma unroll
  for (int i = 0; i < D; ++i) F[i] *= st.rho;
  collide_iterate<L, T, S, ST>(g, rx, a.tol, a.max_iter, F, st, a.min_iter);
  if (st.iters > a.max_iter) atomicAdd(&a.flags[0], 1);
  if (a.stats) add_iteration_stats(a.stats, st.iters);   // wave-uniform
  collide_refresh<L, T, S, ST>(g, F, st);
  using FC = typename std::remove_cv<typename std::remove_reference<decltype(*a.fcache)>::type>::type;
#pragma unroll
  for (int i = 0; i < D; ++i) store_stream(word(a.fcache, i, nc) + cell, FC(T(2) * st.half_inv_rho * F[i]));
  // gather again (cache hits) rather than keeping N live across the fixed point
  // where registers are short: D3Q19 FP32 deviations (decoded into FP64
  // registers, 38 VGPRs that would cost its second wavefront per SIMD; they
  // re-read their references with them) and the general collision variants
  // with FP64 arithmetic.  Everywhere else the populations stay in registers:
  // D2Q9 FP32 deviations (three wavefronts per SIMD either way, measured 8 %
  // faster on the bump-channel batch), D2Q21 (two either way, 6 %), D3Q39
  // (one either way, 11 %), decoded 16-bit populations, and the FP64 ones in
  // accumulation registers (that kernel runs one wave per SIMD either way).
  constexpr bool regather =
      (std::is_same<P, F32Dev>::value && (L::Q == 19 || GEN)) || (!PopCodec<P>::shifted && sizeof(T) == 8 && GEN);
  if constexpr (regather) {
    // opaque copies of the coordinates: the source addresses are recomputed
    // here instead of being kept (or spilled) across the fixed point
    int xr = x, yr = y, zr = z, cr = cell;
    pin(xr);
    pin(yr);
    pin(zr);
    pin(cr);
    if (ffwave) gather<L, P, S, T, NR, ST, FF>(a, g, xr, yr, zr, cr, N);
    else gather<L, P, S, T, NR, ST, (FF == 2 ? 0 : FF)>(a, g, xr, yr, zr, cr, N);
  }
  T Np[Q];
  if constexpr (PopCodec<P>::shifted) {
    // the references of the written slots are loaded before the output
    // arithmetic, so their latency hides behind it
    PopR<P> ref[Q];
#pragma unroll
    for (int al = 0; al < Q; ++al) ref[al] = word(a.rown, al, nc)[cell];
    collide_output<L, T, S, ST, NR>(g, N, rx, st, Np);
    using C = PopCodec<P>;
    if (a.rown_new) {   // wave-uniform: the steps of rebase_cell on the written word
#pragma unroll
      for (int al = 0; al < Q; ++al) {
        const T n = C::template decode<T>(C::template encode<T>(T(Np[al]), ref[al], a.scale), ref[al], a.inv_scale);
        const PopR<P> r = C::template reference<T>(n);
        store_stream(word(a.rown_new, al, nc) + cell, r);
        store_stream(word(a.out, al, nc) + cell, C::template encode<T>(n, r, a.scale));
      }
    } else {
#pragma unroll
      for (int al = 0; al < Q; ++al)
        store_stream(word(a.out, al, nc) + cell, C::template encode<T>(T(Np[al]), ref[al], a.scale));
    }
  } else {
    collide_output<L, T, S, ST, NR>(g, N, rx, st, Np);
#pragma unroll
    for (int al = 0; al < Q; ++al) store_slot<L>(a, al, cell, Np[al]);
  }
}

// Kernel arguments of one simulation's step (current buffer parity).
template <class P, class S, class T>
inline StepArgs<P, S, T> make_step_args(const SimObj* s) {
  StepArgs<P, S, T> a;
  a.box = s->mesh->box;
  a.in = static_cast<const PopE<P>*>(s->pop[s->buf]);
  a.out = static_cast<PopE<P>*>(s->pop[s->buf ^ 1]);
  a.rown = static_cast<const PopR<P>*>(s->rown);
  a.rown_new = s->rebase_in_step ? static_cast<PopR<P>*>(s->rown_spare) : nullptr;
  a.scale = pop_scale(s->p.precision, s->mesh->report.max_J);
  a.inv_scale = 1.0f / a.scale;
  a.geo = static_cast<const S*>(s->geo);
  a.tau = T(s->p.tau);
  a.general = general_collision(s->p);
  a.tau_g = T(a.general ? s->p.tau_g : s->p.tau);
  a.inv_tau = T(1) / a.tau;
  a.relax_s = T(1) / a.tau_g;
  a.relax_c1 = T(0.5) * (a.relax_s - a.inv_tau);
  a.tol = T(s->p.fp_tol);
  a.rho_inf = T(s->p.rho_inf);
  a.max_iter = s->p.fp_max_iter;
  // FP32 arithmetic cannot resolve a warm-started first update below its own
  // roundoff: take at least two iterations there.
  a.min_iter = sizeof(T) == 4 ? 2 : 1;
  a.stream_only = s->p.stream_only;
  a.has_force = s->has_force || s->comp_A;   // the step reads the a_ext words
  a.has_ff = s->has_farfield;
  a.flags = s->flags + 2;   // the step kernel's own count of unconverged cell-steps
  a.stats = s->stats_on ? s->stats : nullptr;
  a.fcache = static_cast<decltype(a.fcache)>(s->fcache);
  return a;
}

}  // namespace vlbm

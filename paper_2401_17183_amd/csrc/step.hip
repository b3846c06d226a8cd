// The fused time step: pull advection (eq. (adv)) + BGK collision with the
// implicit inertial force (eqs. (lbe), (collide), (compo-constr), (delta-flux),
// (deltaN), (equilibrium)), one thread per cell, SoA populations, A/B buffers.
#include "dynamics.hpp"

namespace vlbm {
namespace {

constexpr int kBlock = 256;

// Two resident waves per SIMD: the LDS staging of A (55 KB per 256-thread
// block for D3Q19 FP32) allows two blocks per CU, and the register budget is
// held to that occupancy.
#ifndef VLBM_STEP_ATTR
#define VLBM_STEP_ATTR __attribute__((amdgpu_waves_per_eu(2, 8)))
#endif

// P: population storage type; S: geometry storage type; T: arithmetic type.
template <class P, class S, class T> struct StepArgs {
  Box box;
  const P* __restrict__ in;
  P* __restrict__ out;
  const P* __restrict__ rsrc;   // 16-bit modes: reference of each arriving link
  const P* __restrict__ rown;   // 16-bit modes: reference of each written slot
  float scale, inv_scale;
  const S* __restrict__ geo;
  T tau, tol, rho_inf;
  int max_iter, min_iter;
  int stream_only;
  int has_force, has_ff;
  T* __restrict__ fcache;       // [D][cells] starting guess in, converged F out
  int* flags;
};

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

// Packed geometry of one cell.  With ST > 0 the link coefficients are staged
// in LDS (this thread's column of lds, stride ST) instead of registers; only
// this thread reads its column.
template <class L, class S, class T, int ST>
__device__ __forceinline__ CellGeo<L, T, S, ST> load_pack(const S* __restrict__ geo, int nc, int cell, int has_force,
                                                          S* lds) {
  CellGeo<L, T, S, ST> g;
  g.J = word(geo, Pack<L>::J, nc)[cell];
#pragma unroll
  for (int k = 0; k < nup<L::D>(); ++k) g.gup[k] = word(geo, Pack<L>::GUP + k, nc)[cell];
#pragma unroll
  for (int a = 1; a < L::Q; ++a)
#pragma unroll
    for (int i = 0; i < L::D; ++i) {
      const S v = word(geo, Pack<L>::A + (a - 1) * L::D + i, nc)[cell];
      if constexpr (ST == 0) g.Areg[a][i] = v;
      else lds[((a - 1) * L::D + i) * ST] = v;
    }
  if constexpr (ST == 0)
#pragma unroll
    for (int i = 0; i < L::D; ++i) g.Areg[0][i] = S(0);
  g.lds = lds;
#pragma unroll
  for (int i = 0; i < L::D; ++i) g.aext[i] = has_force ? word(geo, Pack<L>::AEXT + i, nc)[cell] : S(0);
  return g;
}

// Pull N_a(q) = N'_a(q - c_a) (eq. (adv)).  Every load is unconditional and in
// bounds (a bounced or far-field link reads the cell's own opposite slot), so
// no lane diverges; far-field links then take J f^eq(rho_inf, U_inf, U_inf).
template <class L, class P, class S, class T, class NR, int ST>
__device__ __forceinline__ void gather(const StepArgs<P, S, T>& a, const CellGeo<L, T, S, ST>& g, int x, int y,
                                       int z, int cell, NR* N) {
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  using C = PopCodec<P>;
  const int nc = a.box.ncells;
  unsigned ff = 0;
#pragma unroll
  for (int al = 0; al < Q; ++al) {
    int src;
    const int kind = link_source<L>(a.box, al, x, y, z, src);
    const int dir = kind == LINK_INTERIOR ? al : opp(al);
    const P h = word(a.in, 0, nc)[(size_t)dir * nc + src];
    if constexpr (C::shifted) N[al] = C::template decode<NR>(h, word(a.rsrc, al, nc)[cell], a.inv_scale);
    else N[al] = h;
    ff |= (kind == LINK_FARFIELD ? 1u : 0u) << al;
  }
  if (a.has_ff) {   // wave-uniform
    T Uinf[D];
#pragma unroll
    for (int i = 0; i < D; ++i) Uinf[i] = T(word(a.geo, Pack<L>::UINF + i, nc)[cell]);
    T fe[Q];
    feq_farfield<L, T>(g, a.rho_inf, Uinf, fe);
#pragma unroll
    for (int al = 0; al < Q; ++al) N[al] = (ff >> al) & 1u ? NR(g.j() * fe[al]) : N[al];
  }
}

template <class L, class P, class S, class T, class V>
__device__ __forceinline__ void store_slot(const StepArgs<P, S, T>& a, int al, int cell, V v) {
  using C = PopCodec<P>;
  const int nc = a.box.ncells;
  if constexpr (C::shifted) word(a.out, al, nc)[cell] = C::template encode<T>(T(v), word(a.rown, al, nc)[cell], a.scale);
  else word(a.out, al, nc)[cell] = P(v);
}

template <class L, class P, class S, class T>
__device__ __forceinline__ void step_cell(const StepArgs<P, S, T>& a) {
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  // registers hold populations in the storage type, or FP32 for 16-bit storage
  using NR = typename std::conditional<PopCodec<P>::shifted, float, P>::type;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= a.box.ncells) return;
  const int nc = a.box.ncells;
  const int x = cell % a.box.n[0];
  const int r = cell / a.box.n[0];
  const int y = r % a.box.n[1];
  const int z = r / a.box.n[1];
  // FP32 geometry stages A in LDS (55 KB per 256-thread block for D3Q19)
  constexpr int ST = sizeof(S) == 4 ? kBlock : 0;
  __shared__ S sA[ST ? (Q - 1) * D * kBlock : 1];
  NR N[Q];
  const CellGeo<L, T, S, ST> g = load_pack<L, S, T, ST>(a.geo, nc, cell, a.has_force, sA + (ST ? threadIdx.x : 0));
  gather<L, P, S, T, NR, ST>(a, g, x, y, z, cell, N);
  if (a.stream_only) {
#pragma unroll
    for (int al = 0; al < Q; ++al) store_slot<L>(a, al, cell, N[al]);
    return;
  }
  T F[D];
#pragma unroll
  for (int i = 0; i < D; ++i) F[i] = word(a.fcache, i, nc)[cell];
  CollState<L, T> st;
  collide_prepare<L, T, S, ST, NR>(g, N, a.tau, st);
  collide_iterate<L, T, S, ST>(g, a.tau, a.tol, a.max_iter, F, st, a.min_iter);
  if (st.iters > a.max_iter) atomicAdd(&a.flags[0], 1);
#pragma unroll
  for (int i = 0; i < D; ++i) word(a.fcache, i, nc)[cell] = F[i];
  // gather again (cache hits) rather than keeping N live across the fixed point
  int xr = x;
  pin(xr);
  gather<L, P, S, T, NR, ST>(a, g, xr, y, z, cell, N);
  T Np[Q];
  collide_output<L, T, S, ST, NR>(g, N, a.tau, st, Np);
#pragma unroll
  for (int al = 0; al < Q; ++al) store_slot<L>(a, al, cell, Np[al]);
}

// FP32 geometry: two waves per SIMD (see VLBM_STEP_ATTR).
template <class L, class P, class S, class T>
__global__ __launch_bounds__(kBlock) VLBM_STEP_ATTR void k_step(StepArgs<P, S, T> a) {
  step_cell<L, P, S, T>(a);
}

// FP64 storage keeps A in registers and runs at the occupancy the compiler picks.
template <class L, class P, class S, class T>
__global__ __launch_bounds__(kBlock) void k_step64(StepArgs<P, S, T> a) {
  step_cell<L, P, S, T>(a);
}

// Pack FP64 geometry into the kernel precision: J, g^{ij} (upper), A (a >= 1),
// a_ext^i = G . g^i, U_inf^i = u_inf . g^i.
template <class L, class S>
__global__ __launch_bounds__(kBlock) void k_pack(Box box, const double* J, const double* gup, const double* gco,
                                                 const double* A, double G0, double G1, double G2, double u0,
                                                 double u1, double u2, int has_force, int has_ff, S* geo) {
  constexpr int D = L::D;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= box.ncells) return;
  const long nc = box.ncells;
  geo[Pack<L>::J * nc + cell] = S(J[cell]);
  for (int i = 0; i < D; ++i)
    for (int j = i; j < D; ++j) geo[(Pack<L>::GUP + up<D>(i, j)) * nc + cell] = S(gup[(i * D + j) * nc + cell]);
  for (int al = 1; al < L::Q; ++al)
    for (int i = 0; i < D; ++i) geo[(Pack<L>::A + (al - 1) * D + i) * nc + cell] = S(A[(al * D + i) * nc + cell]);
  const double G[3] = {G0, G1, G2};
  const double ui[3] = {u0, u1, u2};
  for (int i = 0; i < D; ++i) {
    double ae = 0, uc = 0;
    for (int k = 0; k < D; ++k) {
      ae += G[k] * gco[(i * D + k) * nc + cell];
      uc += ui[k] * gco[(i * D + k) * nc + cell];
    }
    if (has_force) geo[(Pack<L>::AEXT + i) * nc + cell] = S(ae);
    if (has_ff) geo[(Pack<L>::UINF + i) * nc + cell] = S(uc);
  }
}

template <class L, class P, class S, class T>
hipError_t step_typed(SimObj* s) {
  StepArgs<P, S, T> a;
  a.box = s->mesh->box;
  a.in = static_cast<const P*>(s->pop[s->buf]);
  a.out = static_cast<P*>(s->pop[s->buf ^ 1]);
  a.rsrc = static_cast<const P*>(s->rsrc);
  a.rown = static_cast<const P*>(s->rown);
  a.scale = pop_scale(s->p.precision);
  a.inv_scale = 1.0f / a.scale;
  a.geo = static_cast<const S*>(s->geo);
  a.tau = T(s->p.tau);
  a.tol = T(s->p.fp_tol);
  a.rho_inf = T(s->p.rho_inf);
  a.max_iter = s->p.fp_max_iter;
  // FP32 arithmetic cannot resolve a warm-started first update below its own
  // roundoff: take at least two iterations there.
  a.min_iter = sizeof(T) == 4 ? 2 : 1;
  a.stream_only = s->p.stream_only;
  a.has_force = s->has_force;
  a.has_ff = s->has_farfield;
  a.flags = s->flags;
  a.fcache = static_cast<T*>(s->fcache);
  const int nb = (a.box.ncells + kBlock - 1) / kBlock;
  if constexpr (sizeof(S) == 8)
    k_step64<L, P, S, T><<<nb, kBlock, 0, s->stream>>>(a);
  else
    k_step<L, P, S, T><<<nb, kBlock, 0, s->stream>>>(a);
  return hipGetLastError();
}

template <class L, class S>
hipError_t pack_typed(SimObj* s) {
  MeshObj* m = s->mesh;
  const int nb = (m->box.ncells + kBlock - 1) / kBlock;
  k_pack<L, S><<<nb, kBlock, 0, s->stream>>>(m->box, m->J, m->gup, m->gco, m->A, s->p.body_force[0],
                                              s->p.body_force[1], s->p.body_force[2], s->p.u_inf[0],
                                              s->p.u_inf[1], s->p.u_inf[2], s->has_force, s->has_farfield,
                                              static_cast<S*>(s->geo));
  return hipGetLastError();
}

template <class L>
hipError_t step_lattice(SimObj* s) {
  switch (s->p.precision) {
    case VLBM_FP64: return step_typed<L, double, double, double>(s);
    case VLBM_FP32: return step_typed<L, float, float, double>(s);
    case VLBM_FP16S: return step_typed<L, __half, float, float>(s);
    case VLBM_BF16S: return step_typed<L, __hip_bfloat16, float, float>(s);
    default: return step_typed<L, float, float, float>(s);
  }
}

}  // namespace

hipError_t launch_step(SimObj* s) {
  return s->mesh->lattice == VLBM_D2Q9 ? step_lattice<D2Q9>(s) : step_lattice<D3Q19>(s);
}

hipError_t launch_pack(SimObj* s) {
  const bool d2 = s->mesh->lattice == VLBM_D2Q9;
  if (storage_is_fp64(s->p.precision)) return d2 ? pack_typed<D2Q9, double>(s) : pack_typed<D3Q19, double>(s);
  return d2 ? pack_typed<D2Q9, float>(s) : pack_typed<D3Q19, float>(s);
}

}  // namespace vlbm

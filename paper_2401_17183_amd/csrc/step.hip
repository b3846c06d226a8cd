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

// S: storage type of populations and packed geometry; T: arithmetic type.
template <class S, class T> struct StepArgs {
  Box box;
  const S* __restrict__ in;
  S* __restrict__ out;
  const S* __restrict__ geo;
  T tau, tol, rho_inf;
  int max_iter;
  int stream_only;
  int has_force, has_ff;
  T* __restrict__ fcache;       // [D][cells] starting guess in, converged F out
  int min_iter;
  int* flags;
};

// A stays in registers in its storage type S and converts to T at each use.
// Word w of a SoA array: the wave-uniform base (w * nc) is formed in scalar
// registers, lanes carry only their 32-bit cell offset.
template <class S>
__device__ __forceinline__ const S* word(const S* __restrict__ base, int w, int nc) {
  return base + (size_t)w * (size_t)nc;
}
template <class S>
__device__ __forceinline__ S* word(S* __restrict__ base, int w, int nc) {
  return base + (size_t)w * (size_t)nc;
}

// With ST > 0 the link coefficients are staged in LDS (this thread's column
// of lds, stride ST) instead of registers; only this thread reads its column.
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
template <class L, class S, class T, int ST>
__device__ __forceinline__ void gather(const StepArgs<S, T>& a, const CellGeo<L, T, S, ST>& g, int x, int y, int z,
                                       int cell, S* N) {
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  const int nc = a.box.ncells;
  unsigned ff = 0;
#pragma unroll
  for (int al = 0; al < Q; ++al) {
    int src;
    const int kind = link_source<L>(a.box, al, x, y, z, src);
    const int dir = kind == LINK_INTERIOR ? al : opp(al);
    N[al] = word(a.in, 0, nc)[(size_t)dir * nc + src];
    ff |= (kind == LINK_FARFIELD ? 1u : 0u) << al;
  }
  if (a.has_ff) {   // wave-uniform
    T Uinf[D];
#pragma unroll
    for (int i = 0; i < D; ++i) Uinf[i] = T(word(a.geo, Pack<L>::UINF + i, nc)[cell]);
    T fe[Q];
    feq_farfield<L, T>(g, a.rho_inf, Uinf, fe);
#pragma unroll
    for (int al = 0; al < Q; ++al) N[al] = (ff >> al) & 1u ? S(g.j() * fe[al]) : N[al];
  }
}

template <class L, class S, class T>
__device__ __forceinline__ void step_cell(const StepArgs<S, T>& a) {
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= a.box.ncells) return;
  const int nc = a.box.ncells;
  const int x = cell % a.box.n[0];
  const int r = cell / a.box.n[0];
  const int y = r % a.box.n[1];
  const int z = r / a.box.n[1];
  // FP32 storage stages A in LDS (55 KB per 256-thread block for D3Q19)
  constexpr int ST = sizeof(S) == 4 ? kBlock : 0;
  __shared__ S sA[ST ? (Q - 1) * D * kBlock : 1];
  // pull advection: N_a(q) = N'_a(q - c_a); walls bounce back, far field imposes.
  S N[Q];
  const CellGeo<L, T, S, ST> g = load_pack<L, S, T, ST>(a.geo, nc, cell, a.has_force, sA + (ST ? threadIdx.x : 0));
  gather<L, S, T, ST>(a, g, x, y, z, cell, N);
  if (a.stream_only) {
#pragma unroll
    for (int al = 0; al < Q; ++al) word(a.out, al, nc)[cell] = N[al];
    return;
  }
  T F[D];
#pragma unroll
  for (int i = 0; i < D; ++i) F[i] = T(word(a.fcache, i, nc)[cell]);
  CollState<L, T> st;
  collide_prepare<L, T, S, ST, S>(g, N, a.tau, st);
  collide_iterate<L, T, S, ST>(g, a.tau, a.tol, a.max_iter, F, st, a.min_iter);
  if (st.iters > a.max_iter) atomicAdd(&a.flags[0], 1);
#pragma unroll
  for (int i = 0; i < D; ++i) word(a.fcache, i, nc)[cell] = F[i];
  // gather again (cache hits) rather than keeping N live across the fixed point
  int xr = x;
  pin(xr);
  gather<L, S, T, ST>(a, g, xr, y, z, cell, N);
  T Np[Q];
  collide_output<L, T, S, ST, S>(g, N, a.tau, st, Np);
#pragma unroll
  for (int al = 0; al < Q; ++al) word(a.out, al, nc)[cell] = S(Np[al]);
}

// FP32 storage: two waves per SIMD (see VLBM_STEP_ATTR).
template <class L, class S, class T>
__global__ __launch_bounds__(kBlock) VLBM_STEP_ATTR void k_step(StepArgs<S, T> a) {
  step_cell<L, S, T>(a);
}

// FP64 storage keeps A in registers and runs at the occupancy the compiler picks.
template <class L, class S, class T>
__global__ __launch_bounds__(kBlock) void k_step64(StepArgs<S, T> a) {
  step_cell<L, S, T>(a);
}

// Pack FP64 geometry into the kernel precision: J, g^{ij} (upper), A (a >= 1),
// a_ext^i = G . g^i, U_inf^i = u_inf . g^i.
template <class L, class T>
__global__ __launch_bounds__(kBlock) void k_pack(Box box, const double* J, const double* gup, const double* gco,
                                                 const double* A, double G0, double G1, double G2, double u0,
                                                 double u1, double u2, int has_force, int has_ff, T* geo) {
  constexpr int D = L::D;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= box.ncells) return;
  const long nc = box.ncells;
  geo[Pack<L>::J * nc + cell] = T(J[cell]);
  for (int i = 0; i < D; ++i)
    for (int j = i; j < D; ++j) geo[(Pack<L>::GUP + up<D>(i, j)) * nc + cell] = T(gup[(i * D + j) * nc + cell]);
  for (int al = 1; al < L::Q; ++al)
    for (int i = 0; i < D; ++i) geo[(Pack<L>::A + (al - 1) * D + i) * nc + cell] = T(A[(al * D + i) * nc + cell]);
  const double G[3] = {G0, G1, G2};
  const double ui[3] = {u0, u1, u2};
  for (int i = 0; i < D; ++i) {
    double ae = 0, uc = 0;
    for (int k = 0; k < D; ++k) {
      ae += G[k] * gco[(i * D + k) * nc + cell];
      uc += ui[k] * gco[(i * D + k) * nc + cell];
    }
    if (has_force) geo[(Pack<L>::AEXT + i) * nc + cell] = T(ae);
    if (has_ff) geo[(Pack<L>::UINF + i) * nc + cell] = T(uc);
  }
}

template <class L, class S, class T>
hipError_t step_typed(SimObj* s) {
  StepArgs<S, T> a;
  a.box = s->mesh->box;
  a.in = static_cast<const S*>(s->pop[s->buf]);
  a.out = static_cast<S*>(s->pop[s->buf ^ 1]);
  a.geo = static_cast<const S*>(s->geo);
  a.tau = T(s->p.tau);
  a.tol = T(s->p.fp_tol);
  a.rho_inf = T(s->p.rho_inf);
  a.max_iter = s->p.fp_max_iter;
  a.stream_only = s->p.stream_only;
  a.has_force = s->has_force;
  a.has_ff = s->has_farfield;
  a.flags = s->flags;
  a.fcache = static_cast<T*>(s->fcache);
  // FP32 arithmetic cannot resolve a warm-started first update below its own
  // roundoff: take at least two iterations there.
  a.min_iter = sizeof(T) == 4 ? 2 : 1;
  const int nb = (a.box.ncells + kBlock - 1) / kBlock;
  if constexpr (sizeof(S) == 8)
    k_step64<L, S, T><<<nb, kBlock, 0, s->stream>>>(a);
  else
    k_step<L, S, T><<<nb, kBlock, 0, s->stream>>>(a);
  return hipGetLastError();
}

template <class L, class T>
hipError_t pack_typed(SimObj* s) {
  MeshObj* m = s->mesh;
  const int nb = (m->box.ncells + kBlock - 1) / kBlock;
  k_pack<L, T><<<nb, kBlock, 0, s->stream>>>(m->box, m->J, m->gup, m->gco, m->A, s->p.body_force[0],
                                              s->p.body_force[1], s->p.body_force[2], s->p.u_inf[0],
                                              s->p.u_inf[1], s->p.u_inf[2], s->has_force, s->has_farfield,
                                              static_cast<T*>(s->geo));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(SimObj* s) {
  const bool d2 = s->mesh->lattice == VLBM_D2Q9;
  switch (s->p.precision) {
    case VLBM_FP64:
      return d2 ? step_typed<D2Q9, double, double>(s) : step_typed<D3Q19, double, double>(s);
    case VLBM_FP32:
      return d2 ? step_typed<D2Q9, float, double>(s) : step_typed<D3Q19, float, double>(s);
    default:
      return d2 ? step_typed<D2Q9, float, float>(s) : step_typed<D3Q19, float, float>(s);
  }
}

hipError_t launch_pack(SimObj* s) {
  const bool d2 = s->mesh->lattice == VLBM_D2Q9;
  if (storage_is_fp64(s->p.precision)) return d2 ? pack_typed<D2Q9, double>(s) : pack_typed<D3Q19, double>(s);
  return d2 ? pack_typed<D2Q9, float>(s) : pack_typed<D3Q19, float>(s);
}

}  // namespace vlbm

// The fused time step: pull advection (eq. (adv)) + BGK collision with the
// implicit inertial force (eqs. (lbe), (collide), (compo-constr), (delta-flux),
// (deltaN), (equilibrium)), one thread per cell, SoA populations, A/B buffers.
#include "dynamics.hpp"

namespace vlbm {
namespace {

constexpr int kBlock = 256;

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
  int* flags;
};

template <class L, class S, class T>
__device__ __forceinline__ CellGeo<L, T> load_pack(const S* __restrict__ geo, int nc, int cell, int has_force) {
  CellGeo<L, T> g;
  g.J = T(geo[(long)Pack<L>::J * nc + cell]);
#pragma unroll
  for (int k = 0; k < nup<L::D>(); ++k) g.gup[k] = T(geo[(long)(Pack<L>::GUP + k) * nc + cell]);
#pragma unroll
  for (int i = 0; i < L::D; ++i) g.A[0][i] = T(0);
#pragma unroll
  for (int a = 1; a < L::Q; ++a)
#pragma unroll
    for (int i = 0; i < L::D; ++i) g.A[a][i] = T(geo[(long)(Pack<L>::A + (a - 1) * L::D + i) * nc + cell]);
#pragma unroll
  for (int i = 0; i < L::D; ++i) g.aext[i] = has_force ? T(geo[(long)(Pack<L>::AEXT + i) * nc + cell]) : T(0);
  return g;
}

template <class L, class S, class T>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs<S, T> a) {
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= a.box.ncells) return;
  const int nc = a.box.ncells;
  const int x = cell % a.box.n[0];
  const int r = cell / a.box.n[0];
  const int y = r % a.box.n[1];
  const int z = r / a.box.n[1];
  // pull advection: N_a(q) = N'_a(q - c_a); walls bounce back, far field imposes
  T N[Q];
  unsigned ff = 0;
#pragma unroll
  for (int al = 0; al < Q; ++al) {
    int src;
    const int kind = link_source<L>(a.box, al, x, y, z, src);
    if (kind == LINK_INTERIOR) N[al] = T(a.in[(long)al * nc + src]);
    else if (kind == LINK_WALL) N[al] = T(a.in[(long)opp(al) * nc + cell]);
    else {
      N[al] = T(0);
      ff |= 1u << al;
    }
  }
  const CellGeo<L, T> g = load_pack<L, S, T>(a.geo, nc, cell, a.has_force);
  if (ff) {
    T Uinf[D];
#pragma unroll
    for (int i = 0; i < D; ++i) Uinf[i] = T(a.geo[(long)(Pack<L>::UINF + i) * nc + cell]);
    T fe[Q];
    feq_farfield<L, T>(g, a.rho_inf, Uinf, fe);
#pragma unroll
    for (int al = 0; al < Q; ++al)
      if (ff & (1u << al)) N[al] = g.J * fe[al];
  }
  if (a.stream_only) {
#pragma unroll
    for (int al = 0; al < Q; ++al) a.out[(long)al * nc + cell] = S(N[al]);
    return;
  }
  T Np[Q], F[D], Ut[D], U[D], rho;
  const CollideOut o = collide<L, T>(g, N, a.tau, a.tol, a.max_iter, Np, F, Ut, U, rho);
  if (o.iters > a.max_iter) atomicAdd(&a.flags[0], 1);
#pragma unroll
  for (int al = 0; al < Q; ++al) a.out[(long)al * nc + cell] = S(Np[al]);
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
  const int nb = (a.box.ncells + kBlock - 1) / kBlock;
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

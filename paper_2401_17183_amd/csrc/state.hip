// State kernels in FP64 on the FP64 geometry: initial state, population
// read/write, the output mapping (eq. (result)) and the audits.
#include <math.h>

#include "dynamics.hpp"

namespace vlbm {
namespace {

constexpr int kBlock = 256;
constexpr int kAuditWords = 13;

// S: population storage tag (PopCodec).
template <class S> struct StateArgs {
  Box box;
  const double* J;
  const double* gup;   // [d*d][cells]
  const double* gco;   // [d][d][cells]
  const double* g;     // [d][d][cells]
  const double* A;     // [Q][d][cells]
  double G[3], uinf[3];
  double rho_inf, tau, tau_g, tol;
  int general, max_iter;
  const PopE<S>* in;   // populations to gather from (N'(t-1))
  PopE<S>* out;        // populations to scatter into
  PopR<S>* rown;       // shifted modes: reference of each slot (same layout as the populations)
  float scale, inv_scale;
  const double* rho_in;
  const double* u_in;
  const double* N_in;
  double* rho_out;
  double* u_out;
  double* U_out;
  double* N_out;
  int* flag;
  double* u_prev;
  void* fcache;        // [d][cells], FP64 or FP32 (fc64)
  int fc64;
  int have_prev;
  double* partial;     // [blocks][kAuditWords]
  const double* Ain;   // moving mesh: incoming coefficients of the current state, [Q][d][cells] (else null)
};

template <class L, class S>
__device__ inline CellGeo<L, double> load_fp64(const StateArgs<S>& a, int cell, double* Uinf) {
  constexpr int D = L::D;
  const long nc = a.box.ncells;
  CellGeo<L, double> g;
  g.J = a.J[cell];
  for (int i = 0; i < D; ++i)
    for (int j = i; j < D; ++j) g.gup[up<D>(i, j)] = a.gup[(i * D + j) * nc + cell];
  // the collision takes the coefficients in pair form
#pragma unroll
  for (int i = 0; i < D; ++i) g.Areg[0][i] = 0;
#pragma unroll
  for (int al = 1; al < L::Q; al += 2)
#pragma unroll
    for (int i = 0; i < D; ++i)
      pair_form(a.A[(al * D + i) * nc + cell], a.A[((al + 1) * D + i) * nc + cell], g.Areg[al][i], g.Areg[al + 1][i]);
  for (int i = 0; i < D; ++i) {
    double ae = 0, uc = 0;
    for (int k = 0; k < D; ++k) {
      const double gc = a.gco[(i * D + k) * nc + cell];
      ae += a.G[k] * gc;
      uc += a.uinf[k] * gc;
    }
    g.aext[i] = ae;
    Uinf[i] = uc;
  }
  return g;
}

__device__ inline void cell_xyz(const Box& b, int cell, int& x, int& y, int& z) {
  x = cell % b.n[0];
  const int r = cell / b.n[0];
  y = r % b.n[1];
  z = r / b.n[1];
}

// Pull N_a(q) (eq. (adv)) in FP64; far-field links get J f^eq(rho_inf, U_inf, U_inf).
// wallmask receives the directions that bounced.
template <class L, class S>
__device__ inline void gather64(const StateArgs<S>& a, const CellGeo<L, double>& g, const double* Uinf, int cell,
                                int x, int y, int z, double* N, DirMask<L>& wallmask) {
  const long nc = a.box.ncells;
  DirMask<L> ff = 0;
  wallmask = 0;
#pragma unroll
  for (int al = 0; al < L::Q; ++al) {
    int src;
    const int kind = link_source<L>(a.box, al, x, y, z, src);
    const int dir = kind == LINK_INTERIOR ? al : opp(al);
    const long i = dir * nc + src;
    N[al] = PopCodec<S>::template decode<double>(a.in[i], a.rown ? a.rown[i] : PopR<S>(0), a.inv_scale);
    if (kind == LINK_WALL) wallmask |= DirMask<L>(1) << al;
    if (kind == LINK_FARFIELD) ff |= DirMask<L>(1) << al;
  }
  if (ff) {
    double fe[L::Q];
    feq_farfield<L, double>(g, a.rho_inf, Uinf, fe);
#pragma unroll
    for (int al = 0; al < L::Q; ++al)
      if ((ff >> al) & 1) N[al] = g.j() * fe[al];
  }
}

// Inverse of the pull: put N_a(q) where the next gather reads it.
template <class L, class S>
__device__ inline void unstream_store(const StateArgs<S>& a, int cell, int x, int y, int z, const double* N) {
  const long nc = a.box.ncells;
#pragma unroll
  for (int al = 0; al < L::Q; ++al) {
    int src;
    const int kind = link_source<L>(a.box, al, x, y, z, src);
    if (kind == LINK_FARFIELD) continue;
    const int dir = kind == LINK_INTERIOR ? al : opp(al);
    const long i = dir * nc + src;
    a.out[i] = PopCodec<S>::template encode<double>(N[al], a.rown ? a.rown[i] : PopR<S>(0), a.scale);
  }
}

template <class L, class S>
__global__ __launch_bounds__(kBlock) void k_init(StateArgs<S> a) {
  constexpr int D = L::D;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= a.box.ncells) return;
  const long nc = a.box.ncells;
  int x, y, z;
  cell_xyz(a.box, cell, x, y, z);
  double Uinf[D];
  CellGeo<L, double> g = load_fp64<L, S>(a, cell, Uinf);
  const double rho = a.rho_in ? a.rho_in[cell] : 1.0;
  double Ut[D];
  for (int i = 0; i < D; ++i) {
    double s = 0;
    if (a.u_in)
      for (int k = 0; k < D; ++k) s += a.u_in[k * nc + cell] * a.gco[(i * D + k) * nc + cell];
    Ut[i] = s;
  }
  double N[L::Q], F[D];
  if (!consistent_equilibrium<L, double>(g, rho, Ut, a.tau, a.tol, a.max_iter, N, F)) atomicAdd(a.flag, 1);
  unstream_store<L, S>(a, cell, x, y, z, N);
  // the step's force cache holds F per unit density
  for (int i = 0; i < D; ++i) {
    if (a.fc64) static_cast<double*>(a.fcache)[i * nc + cell] = F[i] / rho;
    else static_cast<float*>(a.fcache)[i * nc + cell] = (float)(F[i] / rho);
  }
}

template <class L, class S>
__global__ __launch_bounds__(kBlock) void k_set_pop(StateArgs<S> a) {
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= a.box.ncells) return;
  const long nc = a.box.ncells;
  int x, y, z;
  cell_xyz(a.box, cell, x, y, z);
  double N[L::Q];
#pragma unroll
  for (int al = 0; al < L::Q; ++al) N[al] = a.N_in[al * nc + cell];
  unstream_store<L, S>(a, cell, x, y, z, N);
}

template <class L, class S>
__global__ __launch_bounds__(kBlock) void k_get_pop(StateArgs<S> a) {
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= a.box.ncells) return;
  const long nc = a.box.ncells;
  int x, y, z;
  cell_xyz(a.box, cell, x, y, z);
  double Uinf[L::D];
  CellGeo<L, double> g = load_fp64<L, S>(a, cell, Uinf);
  double N[L::Q];
  DirMask<L> wm;
  gather64<L, S>(a, g, Uinf, cell, x, y, z, N, wm);
#pragma unroll
  for (int al = 0; al < L::Q; ++al) a.N_out[al * nc + cell] = N[al];
}

// Shifted-storage references: the post-collision rest state of every cell
// (rest consistent equilibrium, rho = 1, u = 0, then one collision), rounded to
// the reference type, is the first reference of the slots the cell writes.
template <class L, class S>
__global__ __launch_bounds__(kBlock) void k_refs_own(StateArgs<S> a) {
  constexpr int D = L::D;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= a.box.ncells) return;
  const long nc = a.box.ncells;
  double Uinf[D];
  CellGeo<L, double> g = load_fp64<L, S>(a, cell, Uinf);
  double Ut[D], N[L::Q], F[D];
  for (int i = 0; i < D; ++i) Ut[i] = 0;
  if (!consistent_equilibrium<L, double>(g, 1.0, Ut, a.tau, a.tol, a.max_iter, N, F)) atomicAdd(a.flag, 1);
  double Np[L::Q], U[D], rho;
  for (int i = 0; i < D; ++i) F[i] = 0;
  const CollideOut o = collide<L, double, double, 0, double>(g, N, make_relax<double>(a.tau, a.tau_g, a.general), a.tol,
                                                         a.max_iter, Np, F, Ut, U, rho);
  if (o.iters > a.max_iter) atomicAdd(a.flag, 1);
  for (int al = 0; al < L::Q; ++al) a.rown[al * nc + cell] = PopCodec<S>::template reference<double>(Np[al]);
}

// Re-basing of the references on the current state (rebase_cell): the
// reader decodes at the offset it gathers from, so nothing else changes.
template <class L, class S>
__global__ __launch_bounds__(kBlock) void k_rebase(StateArgs<S> a) {
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= a.box.ncells) return;
  rebase_cell<L, S>(const_cast<PopE<S>*>(a.in), a.rown, a.box.ncells, cell, a.scale, a.inv_scale);
}

// Output mapping: rho, u = Ut^i g_i (Euclidean), U^i (eq. (result) and the
// shifted velocity of eq. (continuity1)), from a dry run of the collision.
template <class L, class S>
__global__ __launch_bounds__(kBlock) void k_moments(StateArgs<S> a) {
  constexpr int D = L::D;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= a.box.ncells) return;
  const long nc = a.box.ncells;
  int x, y, z;
  cell_xyz(a.box, cell, x, y, z);
  double Uinf[D];
  CellGeo<L, double> g = load_fp64<L, S>(a, cell, Uinf);
  double N[L::Q];
  DirMask<L> wm;
  gather64<L, S>(a, g, Uinf, cell, x, y, z, N, wm);
  double Np[L::Q], F[D], Ut[D], U[D], rho;
  for (int i = 0; i < D; ++i) F[i] = 0;
  const CollideOut o = collide<L, double, double, 0, double>(g, N, make_relax<double>(a.tau, a.tau_g, a.general), a.tol,
                                                         a.max_iter, Np, F, Ut, U, rho);
  if (o.iters > a.max_iter) atomicAdd(a.flag, 1);
  a.rho_out[cell] = rho;
  for (int k = 0; k < D; ++k) {
    double s = 0;
    for (int i = 0; i < D; ++i) s += Ut[i] * a.g[(i * D + k) * nc + cell];
    a.u_out[k * nc + cell] = s;
  }
  if (a.U_out)
    for (int i = 0; i < D; ++i) a.U_out[i * nc + cell] = U[i];
}

// Audits of the current state: mass, mid-link momentum I, wall impulse of the
// previous step, residual, counts; block partials in a fixed order.
template <class L, class S>
__global__ __launch_bounds__(kBlock) void k_audit(StateArgs<S> a) {
  constexpr int D = L::D;
  constexpr int Q = L::Q;
  __shared__ double red[kAuditWords][kBlock];
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  double v[kAuditWords];
  for (int k = 0; k < kAuditWords; ++k) v[k] = 0;
  if (cell < a.box.ncells) {
    const long nc = a.box.ncells;
    int x, y, z;
    cell_xyz(a.box, cell, x, y, z);
    double Uinf[D];
    CellGeo<L, double> g = load_fp64<L, S>(a, cell, Uinf);
    double N[Q];
    DirMask<L> wm;
    gather64<L, S>(a, g, Uinf, cell, x, y, z, N, wm);
    double gi[D][D];
    for (int i = 0; i < D; ++i)
      for (int k = 0; k < D; ++k) gi[i][k] = a.g[(i * D + k) * nc + cell];
    double mass = 0, inner[D], wall[D], wallE[D];
    int nonfinite = 0, negative = 0;
    for (int i = 0; i < D; ++i) inner[i] = wall[i] = wallE[i] = 0;
#pragma unroll
    for (int al = 0; al < Q; ++al) {
      const double n = N[al];
      mass += n;
      if (!isfinite(n)) ++nonfinite;
      if (n < 0) ++negative;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const double ci = L::c(al, i);
        // incoming coefficient: the opposite outgoing one on a static mesh
        const double Ao = a.Ain ? a.Ain[(al * D + i) * nc + cell] : a.A[(opp(al) * D + i) * nc + cell];
        inner[i] += (ci - 0.5 * Ao) * n;
        if ((wm >> al) & 1) wall[i] += (2.0 * ci - Ao) * n;
      }
      if constexpr (L::SPEED > 1) {
        // a bounced long link arrives from another cell q_s: its departing
        // mid-link momentum g_i(q_s) (c^i - A^i_opp(q_s)/2) N replaces the
        // second copy of this cell's in the one-cell form 2 c - A_opp
        if ((wm >> al) & 1) {
          int src;
          (void)link_source<L>(a.box, al, x, y, z, src);
#pragma unroll
          for (int i = 0; i < D; ++i) {
            const double ci = L::c(al, i);
            const double ah = a.A[(opp(al) * D + i) * nc + cell];
            const double as = a.A[(opp(al) * D + i) * nc + src];
            wall[i] -= (ci - 0.5 * ah) * n;   // keep this cell's half only
#pragma unroll
            for (int k = 0; k < D; ++k) wallE[k] += a.g[(i * D + k) * nc + src] * (ci - 0.5 * as) * n;
          }
        }
      }
    }
    v[0] = mass;
    for (int k = 0; k < D; ++k) {
      double sI = 0, sW = wallE[k];
      for (int i = 0; i < D; ++i) {
        sI += gi[i][k] * inner[i];
        sW += gi[i][k] * wall[i];
      }
      v[1 + k] = sI;
      v[4 + k] = sW;
    }
    v[9] = nonfinite;
    v[10] = negative;
    if (!nonfinite) {
      double Np[Q], F[D], Ut[D], U[D], rho;
      for (int i = 0; i < D; ++i) F[i] = 0;
      const CollideOut o = collide<L, double, double, 0, double>(g, N, make_relax<double>(a.tau, a.tau_g, a.general), a.tol,
                                                         a.max_iter, Np, F, Ut, U, rho);
      v[11] = o.iters > a.max_iter ? 1.0 : 0.0;
      v[12] = o.iters;
      double du2 = 0, uu = 0;
      for (int k = 0; k < D; ++k) {
        double s = 0;
        for (int i = 0; i < D; ++i) s += Ut[i] * gi[i][k];
        if (a.have_prev) {
          const double dd = s - a.u_prev[k * nc + cell];
          du2 += dd * dd;
        }
        uu += s * s;
        a.u_prev[k * nc + cell] = s;
      }
      v[7] = du2;
      v[8] = uu;
    }
  }
  for (int k = 0; k < kAuditWords; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      for (int k = 0; k < 12; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
      red[12][threadIdx.x] = fmax(red[12][threadIdx.x], red[12][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < kAuditWords; ++k) a.partial[(long)blockIdx.x * kAuditWords + k] = red[k][0];
}

__global__ __launch_bounds__(kBlock) void k_audit_final(const double* partial, int nblocks, int64_t step,
                                                        double G0, double G1, double G2, int have_prev,
                                                        vlbm_audit* out) {
  __shared__ double red[kAuditWords][kBlock];
  double v[kAuditWords];
  for (int k = 0; k < kAuditWords; ++k) v[k] = 0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
    for (int k = 0; k < 12; ++k) v[k] += partial[(long)b * kAuditWords + k];
    v[12] = fmax(v[12], partial[(long)b * kAuditWords + 12]);
  }
  for (int k = 0; k < kAuditWords; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      for (int k = 0; k < 12; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
      red[12][threadIdx.x] = fmax(red[12][threadIdx.x], red[12][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    vlbm_audit r;
    r.step = step;
    r.mass = red[0][0];
    for (int k = 0; k < 3; ++k) {
      r.mom_I[k] = red[1 + k][0];
      r.wall_impulse[k] = red[4 + k][0];
    }
    r.force_impulse[0] = G0 * r.mass;
    r.force_impulse[1] = G1 * r.mass;
    r.force_impulse[2] = G2 * r.mass;
    r.residual = have_prev ? sqrt(red[7][0] / red[8][0]) : NAN;
    r.max_fp_iters = (int32_t)red[12][0];
    r.nonfinite = (int32_t)red[9][0];
    r.negative = (int32_t)red[10][0];
    r.unconverged = (int32_t)red[11][0];
    *out = r;
  }
}

template <class S>
StateArgs<S> make_args(SimObj* s) {
  MeshObj* m = s->mesh;
  StateArgs<S> a{};
  a.box = m->box;
  a.J = m->J;
  a.gup = m->gup;
  a.gco = m->gco;
  a.g = m->g;
  a.A = m->A;
  for (int k = 0; k < 3; ++k) {
    a.G[k] = s->p.body_force[k];
    a.uinf[k] = s->p.u_inf[k];
  }
  a.rho_inf = s->p.rho_inf;
  a.tau = s->p.tau;
  a.general = general_collision(s->p);
  a.tau_g = a.general ? s->p.tau_g : s->p.tau;
  // the FP64 dry run converges to FP64 roundoff whatever the storage precision
  a.tol = fmin(s->p.fp_tol, 1e-13);
  a.max_iter = s->p.fp_max_iter;
  a.in = static_cast<const PopE<S>*>(s->pop[s->buf]);
  a.out = static_cast<PopE<S>*>(s->pop[s->buf]);
  a.rown = static_cast<PopR<S>*>(s->rown);
  a.scale = pop_scale(s->p.precision, s->mesh->report.max_J);
  a.inv_scale = 1.0f / a.scale;
  a.flag = s->flags;
  a.fcache = s->fcache;
  a.fc64 = fcache_elem(s->p.precision) == 8;
  a.Ain = s->state_moving ? s->Ain : nullptr;
  return a;
}

template <class L, class S>
hipError_t dispatch(SimObj* s, int what, const double* r_in, const double* u_in, double* r_out, double* u_out,
                    double* U_out, double* N_out, const double* N_in, int slot) {
  StateArgs<S> a = make_args<S>(s);
  const int nb = (a.box.ncells + kBlock - 1) / kBlock;
  hipStream_t st = s->stream;
  switch (what) {
    case 0:
      a.rho_in = r_in;
      a.u_in = u_in;
      k_init<L, S><<<nb, kBlock, 0, st>>>(a);
      break;
    case 1:
      a.rho_out = r_out;
      a.u_out = u_out;
      a.U_out = U_out;
      k_moments<L, S><<<nb, kBlock, 0, st>>>(a);
      break;
    case 2:
      a.N_out = N_out;
      k_get_pop<L, S><<<nb, kBlock, 0, st>>>(a);
      break;
    case 3:
      a.N_in = N_in;
      k_set_pop<L, S><<<nb, kBlock, 0, st>>>(a);
      break;
    case 5:
      k_refs_own<L, S><<<nb, kBlock, 0, st>>>(a);
      break;
    case 6:
      k_rebase<L, S><<<nb, kBlock, 0, st>>>(a);
      break;
    case 4: {
      a.u_prev = s->u_prev;
      a.have_prev = s->have_u_prev;
      a.partial = s->audit_partial;
      k_audit<L, S><<<nb, kBlock, 0, st>>>(a);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      vlbm_audit* ring = static_cast<vlbm_audit*>(s->audit_ring);
      k_audit_final<<<1, kBlock, 0, st>>>(s->audit_partial, nb, s->t, s->p.body_force[0], s->p.body_force[1],
                                          s->p.body_force[2], s->have_u_prev, ring + slot);
      s->have_u_prev = 1;
      break;
    }
  }
  return hipGetLastError();
}

template <class L>
hipError_t dispatch_lattice(SimObj* s, int what, const double* r_in, const double* u_in, double* r_out,
                            double* u_out, double* U_out, double* N_out, const double* N_in, int slot) {
  switch (s->p.precision) {
    case VLBM_FP64: return dispatch<L, double>(s, what, r_in, u_in, r_out, u_out, U_out, N_out, N_in, slot);
    case VLBM_FP16S:
      if constexpr (L::SPEED == 1)
        return dispatch<L, __half>(s, what, r_in, u_in, r_out, u_out, U_out, N_out, N_in, slot);
      else
        return hipErrorInvalidValue;   // 16-bit storage is rejected for long-link lattices at init
    case VLBM_BF16S:
      if constexpr (L::SPEED == 1)
        return dispatch<L, __hip_bfloat16>(s, what, r_in, u_in, r_out, u_out, U_out, N_out, N_in, slot);
      else
        return hipErrorInvalidValue;
    case VLBM_FP32: return dispatch<L, F32Dev>(s, what, r_in, u_in, r_out, u_out, U_out, N_out, N_in, slot);
    default: return dispatch<L, float>(s, what, r_in, u_in, r_out, u_out, U_out, N_out, N_in, slot);
  }
}

hipError_t dispatch_any(SimObj* s, int what, const double* r_in, const double* u_in, double* r_out, double* u_out,
                        double* U_out, double* N_out, const double* N_in, int slot) {
  const hipError_t e = refresh_moving_state(s);   // the coefficients of a state the mesh moved into
  if (e != hipSuccess) return e;
  switch (s->mesh->lattice) {
    case VLBM_D2Q9: return dispatch_lattice<D2Q9>(s, what, r_in, u_in, r_out, u_out, U_out, N_out, N_in, slot);
    case VLBM_D3Q19: return dispatch_lattice<D3Q19>(s, what, r_in, u_in, r_out, u_out, U_out, N_out, N_in, slot);
    case VLBM_D2Q21: return dispatch_lattice<D2Q21>(s, what, r_in, u_in, r_out, u_out, U_out, N_out, N_in, slot);
    default: return dispatch_lattice<D3Q39>(s, what, r_in, u_in, r_out, u_out, U_out, N_out, N_in, slot);
  }
}

}  // namespace

int audit_partial_blocks(const MeshObj* m) { return (m->box.ncells + kBlock - 1) / kBlock; }
int audit_words() { return kAuditWords; }

hipError_t launch_init(SimObj* s, const double* rho, const double* u, int* /*dflag*/) {
  return dispatch_any(s, 0, rho, u, nullptr, nullptr, nullptr, nullptr, nullptr, 0);
}
hipError_t launch_moments(SimObj* s, double* rho, double* u, double* U, int* /*dflag*/) {
  return dispatch_any(s, 1, nullptr, nullptr, rho, u, U, nullptr, nullptr, 0);
}
hipError_t launch_get_pop(SimObj* s, double* N) {
  return dispatch_any(s, 2, nullptr, nullptr, nullptr, nullptr, nullptr, N, nullptr, 0);
}
hipError_t launch_set_pop(SimObj* s, const double* N) {
  return dispatch_any(s, 3, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, N, 0);
}
hipError_t launch_refs(SimObj* s) {
  return dispatch_any(s, 5, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0);
}
hipError_t launch_rebase(SimObj* s) {
  if (!storage_shifted(s->p.precision)) return hipSuccess;
  return dispatch_any(s, 6, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0);
}
hipError_t launch_audit(SimObj* s, int slot) {
  return dispatch_any(s, 4, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, slot);
}

}  // namespace vlbm

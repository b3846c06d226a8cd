// The fused time step: pull advection (eq. (adv)) + collision (eq. (collide))
// with the implicit inertial force (eqs. (lbe), (collide), (compo-constr), (delta-flux),
// (deltaN), (equilibrium)), one thread per cell, SoA populations, A/B buffers.
#include "stepcore.hpp"

namespace vlbm {
namespace {

constexpr int kBlock = 256;

// FP32 geometry: two or three waves per SIMD (see VLBM_STEP_ATTR).
// FF = 0 when the mesh has no far-field links, else 2 (wave-uniform run-time
// test, which keeps the far-field variant free of spills).
// GEN: general collision matrix (its own instantiation, always with FF = 2).
template <class L, class P, class S, class T, int FF, bool GEN, int BLOCK = kBlock>
__global__ __launch_bounds__(BLOCK) VLBM_STEP_ATTR void k_step(StepArgs<P, S, T> a) {
  step_cell<L, P, S, T, BLOCK, FF, GEN>(a, blockIdx.x * BLOCK + threadIdx.x);
}

// FP64 storage keeps A in registers and runs at the occupancy the compiler picks.
template <class L, class P, class S, class T, int FF, bool GEN, int BLOCK = kBlock>
__global__ __launch_bounds__(BLOCK) void k_step64(StepArgs<P, S, T> a) {
  step_cell<L, P, S, T, BLOCK, FF, GEN>(a, blockIdx.x * BLOCK + threadIdx.x);
}

// Threads per block: D3Q39 stages its 114 A words per cell in LDS, so its
// blocks are smaller: 128 threads with FP64 arithmetic on FP32 geometry (one
// wave per SIMD, no spills), 64 otherwise (measured faster for FP32
// arithmetic; FP64 geometry needs 58 KB of LDS per 64 threads).
template <class L, class S, class T> constexpr int block_for() {
  return L::Q > 21 ? ((sizeof(S) == 4 && sizeof(T) == 8) ? 128 : 64) : kBlock;
}

// Pack FP64 geometry into the kernel precision: J, g^{ij} (upper), the link
// coefficients in pair form (S = A_a + A_(a+1) in slot a, D = A_a - A_(a+1)
// in slot a + 1, odd a), a_ext^i = G . g^i, U_inf^i = u_inf . g^i.
//
// comp (FP32 words, FP64 arithmetic): a_ext also cancels the rounding of the
// coefficients.  The kernel's A_a is (fl32(S) + fl32(D)) / 2; with dA its
// difference from A, eq. (compo-constr) applied to a fluid at rest
// (N = N' = J rho f^eq(rho = 1, U = Ut = 0)) gives the extra force rho kappa,
//   kappa^i = -1/2 sum_a (dA^i_a + dA^i_opp(a)) f_a,
// and dA_a + dA_(a+1) = fl32(S) - S over each pair (f_a = f_(a+1) at rest), so
//   kappa^i = -sum_pairs (fl32(S^i) - S^i) f_a.
// The velocity-linear part of f^eq does not reach that sum (dA_a + dA_opp(a)
// is even in c_a, c_a . U odd), and the force enters every step as
// F + rho a_ext, so storing a_ext - kappa cancels the rounding up to second
// order in the velocity.  Without it the rounding acts as a spurious body
// force on strongly stretched meshes (a 20:1 O-grid).
template <class L, class S>
__global__ __launch_bounds__(kBlock) void k_pack(Box box, const double* J, const double* gup, const double* gco,
                                                 const double* A, double G0, double G1, double G2, double u0,
                                                 double u1, double u2, int has_force, int comp, int has_ff, S* geo) {
  constexpr int D = L::D;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= box.ncells) return;
  const long nc = box.ncells;
  geo[pack_index<L>(Pack<L>::J, cell)] = S(J[cell]);
  for (int i = 0; i < D; ++i)
    for (int j = i; j < D; ++j) {
      const double v = gup[(i * D + j) * nc + cell];
      const S hi = S(v);
      geo[pack_index<L>(Pack<L>::GUP + up<D>(i, j), cell)] = hi;
      geo[pack_index<L>(Pack<L>::GUPLO + up<D>(i, j), cell)] = S(v - double(hi));
    }
  for (int al = 1; al < L::Q; al += 2)
    for (int i = 0; i < D; ++i) {
      double sv, dv;
      pair_form(A[(al * D + i) * nc + cell], A[((al + 1) * D + i) * nc + cell], sv, dv);
      geo[pack_index<L>(Pack<L>::A + (al - 1) * D + i, cell)] = S(sv);
      geo[pack_index<L>(Pack<L>::A + al * D + i, cell)] = S(dv);
    }
  double kappa[D] = {};
  if constexpr (sizeof(S) < sizeof(double)) {
    if (comp) {
      CellGeo<L, double> g;
      for (int k = 0; k < nup<D>(); ++k) g.gup[k] = 0;
      for (int i = 0; i < D; ++i)
        for (int j = i; j < D; ++j) g.gup[up<D>(i, j)] = gup[(i * D + j) * nc + cell];
      const double rest[D] = {};
      double f[L::Q];
      feq_all<L, double, double, 0>(g, eq_coef<L, double, double, 0>(g, 1.0, rest, rest), f);
      for (int al = 1; al < L::Q; al += 2)
        for (int i = 0; i < D; ++i) {
          double sv, dv;
          pair_form(A[(al * D + i) * nc + cell], A[((al + 1) * D + i) * nc + cell], sv, dv);
          kappa[i] -= 0.5 * (double(S(sv)) - sv) * (f[al] + f[al + 1]);
        }
    }
  }
  const double G[3] = {G0, G1, G2};
  const double ui[3] = {u0, u1, u2};
  for (int i = 0; i < D; ++i) {
    double ae = 0, uc = 0;
    for (int k = 0; k < D; ++k) {
      ae += G[k] * gco[(i * D + k) * nc + cell];
      uc += ui[k] * gco[(i * D + k) * nc + cell];
    }
    if (has_force || comp) geo[pack_index<L>(Pack<L>::AEXT + i, cell)] = S(ae - kappa[i]);
    if (has_ff) geo[pack_index<L>(Pack<L>::UINF + i, cell)] = S(uc);
  }
}

template <class L, class P, class S, class T>
hipError_t step_typed(SimObj* s) {
  const StepArgs<P, S, T> a = make_step_args<P, S, T>(s);
  if constexpr (L::SPEED > 1) {   // periodic axes only: no far field
    constexpr int B = block_for<L, S, T>();
    const int nb = (a.box.ncells + B - 1) / B;
    if constexpr (sizeof(S) == 8) {
      if (a.general) k_step64<L, P, S, T, 0, true, B><<<nb, B, 0, s->stream>>>(a);
      else k_step64<L, P, S, T, 0, false, B><<<nb, B, 0, s->stream>>>(a);
    } else {
      if (a.general) k_step<L, P, S, T, 0, true, B><<<nb, B, 0, s->stream>>>(a);
      else k_step<L, P, S, T, 0, false, B><<<nb, B, 0, s->stream>>>(a);
    }
  } else {
    const int nb = (a.box.ncells + kBlock - 1) / kBlock;
    if constexpr (sizeof(S) == 8) {
      if (a.general) k_step64<L, P, S, T, 2, true><<<nb, kBlock, 0, s->stream>>>(a);
      else if (a.has_ff) k_step64<L, P, S, T, 2, false><<<nb, kBlock, 0, s->stream>>>(a);
      else k_step64<L, P, S, T, 0, false><<<nb, kBlock, 0, s->stream>>>(a);
    } else {
      if (a.general) k_step<L, P, S, T, 2, true><<<nb, kBlock, 0, s->stream>>>(a);
      else if (a.has_ff) k_step<L, P, S, T, 2, false><<<nb, kBlock, 0, s->stream>>>(a);
      else k_step<L, P, S, T, 0, false><<<nb, kBlock, 0, s->stream>>>(a);
    }
  }
  return hipGetLastError();
}

template <class L, class S>
hipError_t pack_typed(SimObj* s) {
  MeshObj* m = s->mesh;
  const int nb = (m->box.ncells + kBlock - 1) / kBlock;
  k_pack<L, S><<<nb, kBlock, 0, s->stream>>>(m->box, m->J, m->gup, m->gco, m->A, s->p.body_force[0],
                                              s->p.body_force[1], s->p.body_force[2], s->p.u_inf[0],
                                              s->p.u_inf[1], s->p.u_inf[2], s->has_force, s->comp_A, s->has_farfield,
                                              static_cast<S*>(s->geo));
  return hipGetLastError();
}

template <class L>
hipError_t step_lattice(SimObj* s) {
  switch (s->p.precision) {
    case VLBM_FP64: return step_typed<L, double, double, double>(s);
    case VLBM_FP32: return step_typed<L, F32Dev, float, double>(s);
    case VLBM_FP16S:
      if constexpr (L::SPEED == 1) return step_typed<L, __half, float, float>(s);
      else return hipErrorInvalidValue;   // rejected at init
    case VLBM_BF16S:
      if constexpr (L::SPEED == 1) return step_typed<L, __hip_bfloat16, float, float>(s);
      else return hipErrorInvalidValue;
    default: return step_typed<L, float, float, float>(s);
  }
}

}  // namespace


hipError_t launch_step(SimObj* s) {
  switch (s->mesh->lattice) {
    case VLBM_D2Q9: return step_lattice<D2Q9>(s);
    case VLBM_D3Q19: return step_lattice<D3Q19>(s);
    case VLBM_D2Q21: return step_lattice<D2Q21>(s);
    default: return step_lattice<D3Q39>(s);
  }
}

template <class S>
hipError_t pack_storage(SimObj* s) {
  switch (s->mesh->lattice) {
    case VLBM_D2Q9: return pack_typed<D2Q9, S>(s);
    case VLBM_D3Q19: return pack_typed<D3Q19, S>(s);
    case VLBM_D2Q21: return pack_typed<D2Q21, S>(s);
    default: return pack_typed<D3Q39, S>(s);
  }
}

hipError_t launch_pack(SimObj* s) {
  return storage_is_fp64(s->p.precision) ? pack_storage<double>(s) : pack_storage<float>(s);
}

}  // namespace vlbm

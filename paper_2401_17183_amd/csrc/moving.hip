// The fused time step on a moving mesh (time-varying coordinates): pull
// advection, collision and implicit inertial force as in the static step, with
// each cell's outgoing and incoming link coefficients computed from g_i on the
// geometry boxes of three times (MovingGeo).
#include "stepcore.hpp"

namespace vlbm {
namespace {

constexpr int kBlock = 256;

// One step on a moving mesh (FP64; periodic meshes): every cell computes the
// outgoing and incoming link coefficients of time t from g_i on the geometry
// boxes of t - 1, t and t + 1 (MovingGeo).
// Block order: one block per (chunk of BLOCK cells along x, row), blocks dealt
// to the XCDs in contiguous runs (xcd_grouped), the rows of a run taken in
// y-bands of kBand rows that sweep z, so that the neighbour rows whose g_i a
// cell reads were fetched by the same XCD shortly before (bands of 16 were
// measured 1.5 % faster than the plain order on the 256x128x128 box, 4, 32,
// 64 and 128 slower than 16).
constexpr int kBand = 16;

template <int BLOCK>
__device__ __forceinline__ int band_cell(const Box& box, int blk) {
  const int nxc = (box.n[0] + BLOCK - 1) / BLOCK;
  const int xc = blk % nxc, r = blk / nxc;
  const int n1 = box.n[1], n2 = box.n[2];
  const int band = r / (kBand * n2), rem = r - band * kBand * n2;
  const int hb = min(kBand, n1 - band * kBand);   // the last band may be narrower
  const int z = rem / hb, y = band * kBand + rem % hb;
  const int x = xc * BLOCK + threadIdx.x;
  return x < box.n[0] ? x + box.n[0] * (y + n1 * z) : -1;
}

template <int BLOCK>
int band_blocks(const Box& box) {
  return (box.n[0] + BLOCK - 1) / BLOCK * box.n[1] * box.n[2];
}

template <class L, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_step_moving(StepArgs<double, double, double> a, MovingGeo mg) {
  const int cell = band_cell<BLOCK>(a.box, xcd_grouped(blockIdx.x, gridDim.x));
  if (cell < 0) return;
  step_cell<Moving<L>, double, double, double, BLOCK, 0, false>(a, cell, mg);
}

template <class L, int B>
hipError_t step_moving_typed(SimObj* s, const MovingGeo& mg) {
  StepArgs<double, double, double> a = make_step_args<double, double, double>(s);
  a.geo = nullptr;
  const int nb = band_blocks<B>(a.box);
  k_step_moving<L, B><<<nb, B, 0, s->stream>>>(a, mg);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step_moving(SimObj* s, const double* gprev, const double* gcur, const double* gnext) {
  const MeshObj* m = s->mesh;
  MovingGeo mg;
  mg.gprev = gprev;
  mg.gcur = gcur;
  mg.gnext = gnext;
  mg.J = m->J;
  mg.gup = m->gup;
  mg.gco = m->gco;
  mg.layers = lattice_speed(m->lattice);
  mg.nbox = 1;
  for (int i = 0; i < 3; ++i) {
    mg.nb[i] = i < m->d ? m->box.n[i] + 2 * mg.layers : 1;
    mg.nbox *= mg.nb[i];
    mg.G[i] = s->p.body_force[i];
  }
  switch (m->lattice) {
    case VLBM_D2Q9: return step_moving_typed<D2Q9, kBlock>(s, mg);
    // 60 of the 108 coefficient words staged in LDS: 30,720 bytes per 64 threads
    case VLBM_D3Q19: return step_moving_typed<D3Q19, 64>(s, mg);
    default: return hipErrorInvalidValue;   // rejected by the caller
  }
}

}  // namespace vlbm

// FP64 geometry precompute on the device (Sec. 2.1): tangent vectors, volume,
// co-tangent vectors, inverse metric, and the link coefficients A (Theta of
// eq. (gamma) contracted with the link velocity), plus a diagnostics report;
// and the variant of the precompute that allocates nothing.
#include <math.h>

#include <mutex>

#include "common.hpp"

namespace vlbm {
namespace {

constexpr int kBlock = 256;

struct GeoArgs {
  Box box;
  int d;
  int m[3];           // coordinate extents
  int layers;         // box layers around the real cells: the lattice's longest link
  int ghost;          // ghost node layers per non-periodic face (layers + 1)
  int nb[3];          // box extents (n_i + 2 layers on axes < d, 1 otherwise)
  int nbox;
  double wrap[3][3];
  double inv2dx;
  const double* coords;
  double* gbox;       // [d][d][nbox]
  double* J;
  double* gup;        // [d*d][cells]
  double* gco;        // [d][d][cells]
  double* g;          // [d][d][cells]
  double* A;          // [Q][d][cells]
  int* flag;
  double* partial;    // [blocks][6]
};

// x(q) for q outside the real box: periodic axes wrap the index (any number of
// periods) and add the translation, non-periodic axes read the ghost node
// layers of the coordinate input.
template <int D>
__device__ inline void coord_at(const GeoArgs& a, const int* q, double* x) {
  int idx[3] = {0, 0, 0};
  double shift[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < D; ++i) {
    int qi = q[i];
    if (a.box.face[i][0] == VLBM_PERIODIC) {
      const int n = a.box.n[i];
      int s = 0;
      while (qi < 0) { qi += n; --s; }
      while (qi >= n) { qi -= n; ++s; }
      idx[i] = qi;
      shift[i] = (double)s;
    } else {
      idx[i] = qi + a.ghost;
    }
  }
  const long off = ((long)idx[2] * a.m[1] + idx[1]) * a.m[0] + idx[0];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    double v = a.coords[off * D + k];
#pragma unroll
    for (int i = 0; i < D; ++i) v += shift[i] * a.wrap[i][k];
    x[k] = v;
  }
}

// Pass 1 for one box cell b (real cells and `layers` layers around them) at
// index q, from its node x0 and the nodes xp[i] = x(q + e_i), xm[i] = x(q - e_i):
// D_{+-i} (eq. (distance)), beta_i and g_i (eq. (tangent)), J (eq. (jacobian)),
// g^i (eq. (covectors)), g^{ij} (eq. (inverse)).
template <int D>
__device__ __forceinline__ void basis_cell(const GeoArgs& a, int b, const int* q, const double* x0,
                                           const double (*xp)[3], const double (*xm)[3]) {
  constexpr int d = D;
  double gv[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  int bad = 0;
  #pragma unroll
  for (int i = 0; i < d; ++i) {
    double Dp[3], Dm[3], df[3];
    double np2 = 0, nm2 = 0, nd2 = 0;
    #pragma unroll
    for (int k = 0; k < d; ++k) {
      Dp[k] = xp[i][k] - x0[k];
      Dm[k] = xm[i][k] - x0[k];
      df[k] = Dp[k] - Dm[k];
      np2 += Dp[k] * Dp[k];
      nm2 += Dm[k] * Dm[k];
      nd2 += df[k] * df[k];
    }
    if (!(nd2 > 0.0)) {
      bad |= 1;
      nd2 = 1.0;
    }
    const double beta = (sqrt(np2) + sqrt(nm2)) / sqrt(nd2);
    #pragma unroll
    for (int k = 0; k < d; ++k) gv[i][k] = beta * df[k] * a.inv2dx;
  }
  double J;
  double gc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  if constexpr (d == 2) {
    J = gv[0][0] * gv[1][1] - gv[0][1] * gv[1][0];
    gc[0][0] = gv[1][1] / J;
    gc[0][1] = -gv[1][0] / J;
    gc[1][0] = -gv[0][1] / J;
    gc[1][1] = gv[0][0] / J;
  } else {
    double c12[3] = {gv[0][1] * gv[1][2] - gv[0][2] * gv[1][1], gv[0][2] * gv[1][0] - gv[0][0] * gv[1][2],
                     gv[0][0] * gv[1][1] - gv[0][1] * gv[1][0]};
    J = c12[0] * gv[2][0] + c12[1] * gv[2][1] + c12[2] * gv[2][2];
    const double c23[3] = {gv[1][1] * gv[2][2] - gv[1][2] * gv[2][1], gv[1][2] * gv[2][0] - gv[1][0] * gv[2][2],
                           gv[1][0] * gv[2][1] - gv[1][1] * gv[2][0]};
    const double c31[3] = {gv[2][1] * gv[0][2] - gv[2][2] * gv[0][1], gv[2][2] * gv[0][0] - gv[2][0] * gv[0][2],
                           gv[2][0] * gv[0][1] - gv[2][1] * gv[0][0]};
    #pragma unroll
    for (int k = 0; k < 3; ++k) {
      gc[0][k] = c23[k] / J;
      gc[1][k] = c31[k] / J;
      gc[2][k] = c12[k] / J;
    }
  }
  if (!(J > 0.0)) bad |= 2;
  if (bad) atomicOr(a.flag, bad);
  #pragma unroll
  for (int i = 0; i < d; ++i)
    #pragma unroll
    for (int k = 0; k < d; ++k) a.gbox[(long)(i * d + k) * a.nbox + b] = gv[i][k];
  // real cell?
  bool real = true;
  #pragma unroll
  for (int i = 0; i < d; ++i) real = real && q[i] >= 0 && q[i] < a.box.n[i];
  if (!real) return;
  const int cell = q[0] + a.box.n[0] * (q[1] + a.box.n[1] * q[2]);
  const long nc = a.box.ncells;
  a.J[cell] = J;
  #pragma unroll
  for (int i = 0; i < d; ++i)
    #pragma unroll
    for (int k = 0; k < d; ++k) {
      a.gco[(i * d + k) * nc + cell] = gc[i][k];
      if (a.g) a.g[(i * d + k) * nc + cell] = gv[i][k];   // null: left to the caller (moving steps)
    }
  #pragma unroll
  for (int i = 0; i < d; ++i)
    #pragma unroll
    for (int j = 0; j < d; ++j) {
      double s = 0;
      #pragma unroll
      for (int k = 0; k < d; ++k) s += gc[i][k] * gc[j][k];
      a.gup[(i * d + j) * nc + cell] = s;
    }
}

// Pass 1: one thread per box cell, each reading its 2d + 1 nodes; D = a.d
// (a compile-time dimension keeps the per-node arrays in registers: with the
// run-time one they went to scratch memory and the kernel took 1.8x as long).
template <int D>
__global__ __launch_bounds__(kBlock) void k_basis(GeoArgs a) {
  const int b = blockIdx.x * kBlock + threadIdx.x;
  if (b >= a.nbox) return;
  constexpr int d = D;
  int bq[3] = {b % a.nb[0], (b / a.nb[0]) % a.nb[1], b / (a.nb[0] * a.nb[1])};
  int q[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < d; ++i) q[i] = bq[i] - a.layers;
  double x0[3], xp[3][3], xm[3][3];
  coord_at<D>(a, q, x0);
#pragma unroll
  for (int i = 0; i < d; ++i) {
    int qp[3] = {q[0], q[1], q[2]};
    int qm[3] = {q[0], q[1], q[2]};
    qp[i] += 1;
    qm[i] -= 1;
    coord_at<D>(a, qp, xp[i]);
    coord_at<D>(a, qm, xm[i]);
  }
  basis_cell<D>(a, b, q, x0, xp, xm);
}


__device__ inline void sym_eig_range(int d, const double* G /* d*d */, double& lo, double& hi) {
  if (d == 2) {
    const double m = 0.5 * (G[0] + G[3]);
    const double h = 0.5 * (G[0] - G[3]);
    const double r = sqrt(h * h + G[1] * G[1]);
    lo = m - r;
    hi = m + r;
    return;
  }
  const double a00 = G[0], a11 = G[4], a22 = G[8], a01 = G[1], a02 = G[2], a12 = G[5];
  const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
  const double q = (a00 + a11 + a22) / 3.0;
  const double p2 = (a00 - q) * (a00 - q) + (a11 - q) * (a11 - q) + (a22 - q) * (a22 - q) + 2.0 * p1;
  if (p2 <= 0.0) {
    lo = hi = q;
    return;
  }
  const double p = sqrt(p2 / 6.0);
  const double b00 = (a00 - q) / p, b11 = (a11 - q) / p, b22 = (a22 - q) / p;
  const double b01 = a01 / p, b02 = a02 / p, b12 = a12 / p;
  double r = 0.5 * (b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) + b02 * (b01 * b12 - b11 * b02));
  r = fmin(1.0, fmax(-1.0, r));
  const double phi = acos(r) / 3.0;
  hi = q + 2.0 * p * cos(phi);
  lo = q + 2.0 * p * cos(phi + 2.0943951023931957);
}

// Pass 2: one thread per real cell: A^i_a = [e_a(q + c_a) - e_a(q)] . g^i(q)
// (eqs. (lattice), (gamma)) and the per-block diagnostics.
template <class L>
__global__ __launch_bounds__(kBlock) void k_links(GeoArgs a) {
  constexpr int D = L::D;
  __shared__ double red[6][kBlock];
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  double vmin_J = INFINITY, vmax_J = -INFINITY, vmin_e = INFINITY, vmax_e = -INFINITY, vrest = INFINITY, vA = 0;
  if (cell < a.box.ncells) {
    const long nc = a.box.ncells;
    const int x = cell % a.box.n[0];
    const int y = (cell / a.box.n[0]) % a.box.n[1];
    const int z = cell / (a.box.n[0] * a.box.n[1]);
    const int ly = a.layers;
    int bq[3] = {x + ly, y + (D > 1 ? ly : 0), z + (D > 2 ? ly : 0)};
    const int b0 = bq[0] + a.nb[0] * (bq[1] + a.nb[1] * bq[2]);
    double gco[D][D], g0[D][D];
    for (int i = 0; i < D; ++i)
      for (int k = 0; k < D; ++k) {
        gco[i][k] = a.gco[(i * D + k) * nc + cell];
        g0[i][k] = a.gbox[(long)(i * D + k) * a.nbox + b0];
      }
    for (int i = 0; i < D; ++i) a.A[(0 * D + i) * nc + cell] = 0.0;
#pragma unroll
    for (int al = 1; al < L::Q; ++al) {
      int bs[3] = {bq[0], bq[1], bq[2]};
      for (int i = 0; i < D; ++i) bs[i] += L::c(al, i);
      const int b1 = bs[0] + a.nb[0] * (bs[1] + a.nb[1] * bs[2]);
      double de[D];
      for (int k = 0; k < D; ++k) {
        double s = 0;
        for (int j = 0; j < D; ++j) {
          const int cj = L::c(al, j);
          if (cj == 0) continue;
          s += cj * (a.gbox[(long)(j * D + k) * a.nbox + b1] - g0[j][k]);
        }
        de[k] = s;
      }
      for (int i = 0; i < D; ++i) {
        double s = 0;
        for (int k = 0; k < D; ++k) s += de[k] * gco[i][k];
        a.A[(al * D + i) * nc + cell] = s;
        vA = fmax(vA, fabs(s));
      }
    }
    const double J = a.J[cell];
    vmin_J = vmax_J = J;
    double G[9];
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) G[i * D + j] = a.gup[(i * D + j) * nc + cell];
    sym_eig_range(D, G, vmin_e, vmax_e);
    double trg = 0;
    for (int i = 0; i < D; ++i) trg += G[i * D + i];
#pragma unroll
    for (int al = 0; al < L::Q; ++al) {
      double cgc = 0;
      int cc = 0;
      for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) cgc += L::c(al, i) * L::c(al, j) * G[i * D + j];
      for (int i = 0; i < D; ++i) cc += L::c(al, i) * L::c(al, i);
      const double ratio = 1.0 + 0.5 * (L::INV_T0 * (cgc - cc) - (trg - D));
      vrest = fmin(vrest, ratio);
    }
  }
  red[0][threadIdx.x] = vmin_J;
  red[1][threadIdx.x] = -vmax_J;
  red[2][threadIdx.x] = vmin_e;
  red[3][threadIdx.x] = -vmax_e;
  red[4][threadIdx.x] = vrest;
  red[5][threadIdx.x] = -vA;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 6; ++k) a.partial[blockIdx.x * 6 + k] = red[k][0];
}

}  // namespace

int geometry_partial_blocks(const MeshObj* m) { return (m->box.ncells + kBlock - 1) / kBlock; }

// Cells of the geometry box: the real cells and `layers` layers around them
// on the d axes (g_i is needed one link beyond every real cell).
size_t geometry_box_cells(const MeshObj* m) {
  const int layers = lattice_speed(m->lattice);
  size_t nbox = 1;
  for (int i = 0; i < m->d; ++i) nbox *= (size_t)(m->box.n[i] + 2 * layers);
  return nbox;
}

// Enqueue the two geometry passes on stream s.  Scratch: dflag (int, cleared
// by the caller), partial [nblocks_partial][6], gbox [d][d][box cells].
hipError_t launch_geometry(MeshObj* m, hipStream_t s, int* dflag, double* partial, int nblocks_partial,
                           double* gbox) {
  GeoArgs a;
  a.box = m->box;
  a.d = m->d;
  a.nbox = 1;
  a.layers = lattice_speed(m->lattice);
  a.ghost = a.layers + 1;
  for (int i = 0; i < 3; ++i) {
    a.m[i] = m->m[i];
    a.nb[i] = i < m->d ? m->box.n[i] + 2 * a.layers : 1;
    a.nbox *= a.nb[i];
    for (int k = 0; k < 3; ++k) a.wrap[i][k] = m->wrap[i][k];
  }
  a.inv2dx = 1.0 / (2.0 * m->dx);
  a.coords = m->coords;
  a.J = m->J;
  a.gup = m->gup;
  a.gco = m->gco;
  a.g = m->g;
  a.A = m->A;
  a.flag = dflag;
  a.partial = partial;
  a.gbox = gbox;
  if (a.d == 2) k_basis<2><<<(a.nbox + kBlock - 1) / kBlock, kBlock, 0, s>>>(a);
  else k_basis<3><<<(a.nbox + kBlock - 1) / kBlock, kBlock, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (m->lattice) {
    case VLBM_D2Q9: k_links<D2Q9><<<nblocks_partial, kBlock, 0, s>>>(a); break;
    case VLBM_D3Q19: k_links<D3Q19><<<nblocks_partial, kBlock, 0, s>>>(a); break;
    case VLBM_D2Q21: k_links<D2Q21><<<nblocks_partial, kBlock, 0, s>>>(a); break;
    default: k_links<D3Q39><<<nblocks_partial, kBlock, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

namespace {

// e_a = c_a^j g_j at box cell b, from g on a box ([d][d][nbox], word j * D + k
// holds component k of g_j); only the axes the link moves along are read.
template <class L>
__device__ __forceinline__ void e_at(const double* __restrict__ gb, int al, long b, int nbox, double* e) {
#pragma unroll
  for (int k = 0; k < L::D; ++k) {
    double v = 0;
#pragma unroll
    for (int j = 0; j < L::D; ++j) {
      const int cj = L::c(al, j);
      if (cj != 0) v += cj * gb[(long)(j * L::D + k) * nbox + b];
    }
    e[k] = v;
  }
}

// r^i = v . g^i with g^i in registers (gi[i * D + k] = component k of g^i).
template <int D>
__device__ __forceinline__ void project(const double* gi, const double* v, double* r) {
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double s = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) s += v[k] * gi[i * D + k];
    r[i] = s;
  }
}

// Index on the geometry box (`layers` layers around the real cells) of a real cell.
template <class L>
__device__ __forceinline__ long box_index(const int* nb, int layers, int cell, const Box& box) {
  const int x = cell % box.n[0];
  const int y = (cell / box.n[0]) % box.n[1];
  const int z = cell / (box.n[0] * box.n[1]);
  const int b0 = x + layers, b1 = y + (L::D > 1 ? layers : 0), b2 = z + (L::D > 2 ? layers : 0);
  return b0 + (long)nb[0] * (b1 + (long)nb[1] * b2);
}

// The coefficients of the state at time T on a mesh that moved into it, for
// the audits, the output mapping and a static step that follows (the mesh
// taken as momentarily at rest), from g_i on the boxes of T - 1 and T (and
// g_i(T) on the real cells, which the moving step's k_basis leaves out):
//   incoming  Ain^i_a(q) = [e_a(q, T) - e_a(q - c_a, T - 1)] . g^i(q, T)
//   outgoing  A^i_a(q)   = [e_a(q + c_a, T) - e_a(q, T)] . g^i(q, T)
struct StateLinkArgs {
  Box box;
  int nb[3], nbox, layers;
  const double *gprev, *gcur;              // [d][d][nbox], times T - 1 and T
  const double* gco;                       // g^i(T), real cells
  double* Ain;                             // [Q][d][cells]
  double* A;                               // [Q][d][cells]
  double* g;                               // g_i(T) on the real cells, [d][d][cells]
};

template <class L>
__global__ __launch_bounds__(kBlock) void k_links_state(StateLinkArgs a) {
  constexpr int D = L::D;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= a.box.ncells) return;
  const long nc = a.box.ncells;
  const double* __restrict__ gprev = a.gprev;
  const double* __restrict__ gcur = a.gcur;
  const double* __restrict__ gco = a.gco;
  double* __restrict__ Ain = a.Ain;
  double* __restrict__ A = a.A;
  const long b0 = box_index<L>(a.nb, a.layers, cell, a.box);
  double gq[D * D], gi[D * D];
#pragma unroll
  for (int w = 0; w < D * D; ++w) {
    gq[w] = gcur[(long)w * a.nbox + b0];
    gi[w] = gco[w * nc + cell];
    a.g[w * nc + cell] = gq[w];
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    Ain[i * nc + cell] = 0.0;
    A[i * nc + cell] = 0.0;
  }
#pragma unroll
  for (int al = 1; al < L::Q; ++al) {
    const int c0 = L::c(al, 0), c1 = D > 1 ? L::c(al, 1) : 0, c2 = D > 2 ? L::c(al, 2) : 0;
    const long st = c0 + (long)a.nb[0] * (c1 + (long)a.nb[1] * c2);
    double e_cur[3], e_there[3], e_back[3], v[3], r[3];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double s = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const int cj = L::c(al, j);
        if (cj != 0) s += cj * gq[j * D + k];
      }
      e_cur[k] = s;
    }
    e_at<L>(gprev, al, b0 - st, a.nbox, e_back);    // e_a(q - c_a, T - 1)
    e_at<L>(gcur, al, b0 + st, a.nbox, e_there);    // e_a(q + c_a, T)
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = e_cur[k] - e_back[k];
    project<D>(gi, v, r);
#pragma unroll
    for (int i = 0; i < D; ++i) Ain[(al * D + i) * nc + cell] = r[i];
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = e_there[k] - e_cur[k];
    project<D>(gi, v, r);
#pragma unroll
    for (int i = 0; i < D; ++i) A[(al * D + i) * nc + cell] = r[i];
  }
}

template <class Args>
void box_shape(const MeshObj* m, Args& a) {
  a.box = m->box;
  a.layers = lattice_speed(m->lattice);
  a.nbox = 1;
  for (int i = 0; i < 3; ++i) {
    a.nb[i] = i < m->d ? m->box.n[i] + 2 * a.layers : 1;
    a.nbox *= a.nb[i];
  }
}

}  // namespace

// g_i on the geometry box and J, g^{ij}, g^i, g_i on the real cells of the
// node positions `coords` (mesh layout) with periodic translations `wrap`,
// into the given arrays (pass 1 of the precompute; g may be null: the real-cell
// g_i are then not written); degenerate cells set bits of *dflag.
hipError_t launch_basis_of(const MeshObj* m, const double* coords, const double (*wrap)[3], double* gbox, double* J,
                           double* gup, double* gco, double* g, int* dflag, hipStream_t s) {
  GeoArgs a;
  a.box = m->box;
  a.d = m->d;
  a.nbox = 1;
  a.layers = lattice_speed(m->lattice);
  a.ghost = a.layers + 1;
  for (int i = 0; i < 3; ++i) {
    a.m[i] = m->m[i];
    a.nb[i] = i < m->d ? m->box.n[i] + 2 * a.layers : 1;
    a.nbox *= a.nb[i];
    for (int k = 0; k < 3; ++k) a.wrap[i][k] = wrap[i][k];
  }
  a.inv2dx = 1.0 / (2.0 * m->dx);
  a.coords = coords;
  a.J = J;
  a.gup = gup;
  a.gco = gco;
  a.g = g;
  a.A = nullptr;
  a.flag = dflag;
  a.partial = nullptr;
  a.gbox = gbox;
  if (a.d == 2) k_basis<2><<<(a.nbox + kBlock - 1) / kBlock, kBlock, 0, s>>>(a);
  else k_basis<3><<<(a.nbox + kBlock - 1) / kBlock, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t refresh_moving_state(SimObj* sim) {
  if (!sim->mv_state_stale) return hipSuccess;
  const MeshObj* m = sim->mesh;
  StateLinkArgs a;
  box_shape(m, a);
  // after a moving step the boxes rotate: [0] holds the previous time, [1] the current
  a.gprev = sim->mv_box[0];
  a.gcur = sim->mv_box[1];
  a.gco = m->gco;
  a.Ain = sim->Ain;
  a.A = m->A;
  a.g = m->g;
  const int nb = (m->box.ncells + kBlock - 1) / kBlock;
  switch (m->lattice) {
    case VLBM_D2Q9: k_links_state<D2Q9><<<nb, kBlock, 0, sim->stream>>>(a); break;
    case VLBM_D3Q19: k_links_state<D3Q19><<<nb, kBlock, 0, sim->stream>>>(a); break;
    default: return hipErrorInvalidValue;   // moving meshes are D2Q9 and D3Q19
  }
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) sim->mv_state_stale = 0;
  return e;
}

namespace {

// The precompute that allocates nothing keeps its scratch (degenerate-cell
// flag, per-block diagnostics and their reduction, the g_i box) in this
// device array.  Every GPU the library runs on holds its own copy until the
// process ends; host code reaches it through the per-device address from
// hipGetSymbolAddress, never through the name.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Address of this device's scratch (looked up once per device, with that
// device current).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

__global__ void k_clear_flag(int* flag) { *flag = 0; }

// Minimum of each of the 6 diagnostics over the per-block partials (one
// block; min is exact in any order, so this equals the host reduction).
__global__ __launch_bounds__(kBlock) void k_geo_final(const double* partial, int nblocks, double* out) {
  __shared__ double red[6][kBlock];
  double v[6];
  for (int k = 0; k < 6; ++k) v[k] = INFINITY;
  for (int b = threadIdx.x; b < nblocks; b += kBlock)
    for (int k = 0; k < 6; ++k) v[k] = fmin(v[k], partial[(size_t)b * 6 + k]);
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 6; ++k) out[k] = red[k][0];
}

}  // namespace

}  // namespace vlbm

extern "C" int vlbm_geometry_precompute_noalloc(vlbm_mesh mh, void* stream, vlbm_geom_report* rep) {
  using namespace vlbm;
  MeshObj* m = reinterpret_cast<MeshObj*>(mh);
  if (!m) return set_error(VLBM_ERR_ARG, "null mesh");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = geometry_partial_blocks(m);
  const size_t nbox = geometry_box_cells(m);
  // scratch layout (doubles): [0] flag word, [8, 14) reduced diagnostics,
  // [32, 32 + 6 nb) per-block partials, then the g_i box, 256-byte aligned
  const size_t part_off = 32;
  const size_t box_off = (part_off + (size_t)nb * 6 + 31) / 32 * 32;
  const size_t need = (box_off + (size_t)m->d * m->d * nbox) * sizeof(double);
  if (need > kScratchBytes)
    return set_error(VLBM_ERR_ARG,
                     "vlbm_geometry_precompute_noalloc: the mesh needs %zu bytes of scratch, more than its %zu "
                     "(use vlbm_geometry_precompute)",
                     need, kScratchBytes);
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return set_error(VLBM_ERR_DEVICE, "scratch address: %s", hipGetErrorString(e));
  double* sp = static_cast<double*>(base);
  int* dflag = reinterpret_cast<int*>(sp);
  double* reduced = sp + 8;
  double* partial = sp + part_off;
  double* gbox = sp + box_off;
  k_clear_flag<<<1, 1, 0, s>>>(dflag);
  e = hipGetLastError();
  if (e == hipSuccess) e = launch_geometry(m, s, dflag, partial, nb, gbox);
  if (e == hipSuccess) {
    k_geo_final<<<1, kBlock, 0, s>>>(partial, nb, reduced);
    e = hipGetLastError();
  }
  int flag = 0;
  double r[6];
  if (e == hipSuccess) e = hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(r, reduced, sizeof(r), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(VLBM_ERR_DEVICE, "geometry precompute: %s", hipGetErrorString(e));
  return finish_geometry(m, flag, r, rep);
}

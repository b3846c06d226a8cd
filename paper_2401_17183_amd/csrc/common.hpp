// Internal declarations shared by the HIP translation units of libvlbm.
// Not part of the public ABI (include/vlbm.h is).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/vlbm.h"

namespace vlbm {

// ---------------------------------------------------------------------------
// Lattices (Sec. 2.1, eq. (iso) and the D3Q19 set printed there; D2Q9 is its
// planar analogue).  Rest first, then opposite pairs (2k-1, 2k).  All lookups
// are constexpr so fully unrolled loops fold them into immediates.  Each
// lattice carries its T0 and the factors 1/T0, 1/(2 T0), 1/(6 T0^3) of the
// equilibrium and of dN, and SPEED, its longest link in cells per axis.
//
// D3Q39 and D2Q21 are sixth-order isotropic (eq. (iso) in full), T0 = 2/3:
// D3Q39 has the shells 0, (1,0,0), (1,1,1), (2,0,0), (2,2,0), (3,0,0) with
// weights 1/12, 1/12, 1/27, 2/135, 1/432, 1/1620; D2Q21 is its projection on
// the (x, y) plane (shells 0, (1,0), (1,1), (2,0), (2,2), (3,0) with weights
// 91/324, 1/12, 2/27, 7/360, 1/432, 1/1620).  Their links span up to three
// cells, so they run on periodic axes only.
// ---------------------------------------------------------------------------
struct D2Q9 {
  static constexpr bool MOVING = false;
  static constexpr int Q = 9;
  static constexpr int D = 2;
  static constexpr int ID = VLBM_D2Q9;
  static constexpr int SPEED = 1;
  static constexpr double T0 = 1.0 / 3.0, INV_T0 = 3.0, INV_2T0 = 1.5, INV_6T03 = 4.5;
  __host__ __device__ static constexpr int c(int a, int i) {
    constexpr int t[9][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                             {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
    return t[a][i];
  }
  __host__ __device__ static constexpr double w(int a) {
    return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

struct D3Q19 {
  static constexpr bool MOVING = false;
  static constexpr int Q = 19;
  static constexpr int D = 3;
  static constexpr int ID = VLBM_D3Q19;
  static constexpr int SPEED = 1;
  static constexpr double T0 = 1.0 / 3.0, INV_T0 = 3.0, INV_2T0 = 1.5, INV_6T03 = 4.5;
  __host__ __device__ static constexpr int c(int a, int i) {
    constexpr int t[19][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},
                              {0, 0, 1},   {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
                              {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1}};
    return t[a][i];
  }
  __host__ __device__ static constexpr double w(int a) {
    return a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

struct D2Q21 {
  static constexpr bool MOVING = false;
  static constexpr int Q = 21;
  static constexpr int D = 2;
  static constexpr int ID = VLBM_D2Q21;
  static constexpr int SPEED = 3;
  static constexpr double T0 = 2.0 / 3.0, INV_T0 = 1.5, INV_2T0 = 0.75, INV_6T03 = 0.5625;
  __host__ __device__ static constexpr int c(int a, int i) {
    constexpr int t[21][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},   {0, -1, 0}, {1, 1, 0},
                              {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},  {2, 0, 0},   {-2, 0, 0}, {0, 2, 0},
                              {0, -2, 0}, {2, 2, 0},  {-2, -2, 0}, {2, -2, 0},  {-2, 2, 0}, {3, 0, 0},
                              {-3, 0, 0}, {0, 3, 0},  {0, -3, 0}};
    return t[a][i];
  }
  __host__ __device__ static constexpr double w(int a) {
    return a == 0 ? 91.0 / 324.0
                  : a < 5 ? 1.0 / 12.0
                  : a < 9 ? 2.0 / 27.0
                  : a < 13 ? 7.0 / 360.0
                  : a < 17 ? 1.0 / 432.0
                  : 1.0 / 1620.0;
  }
};

struct D3Q39 {
  static constexpr bool MOVING = false;
  static constexpr int Q = 39;
  static constexpr int D = 3;
  static constexpr int ID = VLBM_D3Q39;
  static constexpr int SPEED = 3;
  static constexpr double T0 = 2.0 / 3.0, INV_T0 = 1.5, INV_2T0 = 0.75, INV_6T03 = 0.5625;
  __host__ __device__ static constexpr int c(int a, int i) {
    constexpr int t[39][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},
                              {0, 0, -1},  {1, 1, 1},   {-1, -1, -1}, {1, 1, -1},  {-1, -1, 1}, {1, -1, 1},
                              {-1, 1, -1}, {1, -1, -1}, {-1, 1, 1},  {2, 0, 0},   {-2, 0, 0},  {0, 2, 0},
                              {0, -2, 0},  {0, 0, 2},   {0, 0, -2},  {2, 2, 0},   {-2, -2, 0}, {2, -2, 0},
                              {-2, 2, 0},  {2, 0, 2},   {-2, 0, -2}, {2, 0, -2},  {-2, 0, 2},  {0, 2, 2},
                              {0, -2, -2}, {0, 2, -2},  {0, -2, 2},  {3, 0, 0},   {-3, 0, 0},  {0, 3, 0},
                              {0, -3, 0},  {0, 0, 3},   {0, 0, -3}};
    return t[a][i];
  }
  __host__ __device__ static constexpr double w(int a) {
    return a == 0 ? 1.0 / 12.0
                  : a < 7 ? 1.0 / 12.0
                  : a < 15 ? 1.0 / 27.0
                  : a < 21 ? 2.0 / 135.0
                  : a < 33 ? 1.0 / 432.0
                  : 1.0 / 1620.0;
  }
};

// A lattice on a mesh that moves in time: the same velocities and weights,
// and each cell carries incoming link coefficients of its own (the outgoing
// and incoming momentum changes of a hop then involve the mesh at different
// times) instead of the opposite direction's outgoing ones.
template <class B> struct Moving : B {
  static constexpr bool MOVING = true;
};

__host__ __device__ constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }

// Workgroups are dealt to the 8 XCDs in turn (block b to XCD b mod 8), each
// XCD with its own L2.  xcd_grouped(b, nb) renumbers the nb blocks of a grid
// so that each XCD receives one contiguous run of the logical order (a
// bijection of [0, nb)): neighbouring logical blocks share an L2.
__device__ __forceinline__ int xcd_grouped(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// One bit per direction (64 bits once Q exceeds 32).
template <class L> using DirMask = typename std::conditional<(L::Q > 32), unsigned long long, unsigned>::type;

// Longest link of a lattice id (cells per axis).
inline int lattice_speed(int lattice) { return lattice == VLBM_D2Q21 || lattice == VLBM_D3Q39 ? 3 : 1; }

// ---------------------------------------------------------------------------
// Population storage codecs, keyed by a storage tag P.  E is the stored element
// type and R the type of the per-slot reference.  FP64 and plain FP32 (the tag
// float) store N itself.  The shifted modes store a scaled deviation from a
// reference held in the 16-bit type at the slot: h = s (N - R), with R the
// post-collision state of the cell that wrote the slot, re-based on the state
// every few steps.  Writer and reader add back the same R, so R only has to be
// a representable number close to N:
//   __half / __hip_bfloat16   16-bit deviations (FP32 arithmetic),
//   F32Dev                    FP32 deviations from an FP16 reference, decoded
//                             exactly into the (FP64) arithmetic type; the
//                             rounding of the stored number is then relative
//                             to N - R, not to N.
// ---------------------------------------------------------------------------
struct F32Dev {};

template <class P> struct PopCodec {
  using E = P;
  using R = P;
  static constexpr bool shifted = false;
  template <class T> __device__ __forceinline__ static T decode(E h, R, float) { return T(h); }
  template <class T> __device__ __forceinline__ static E encode(T n, R, float) { return E(n); }
  template <class T> __device__ __forceinline__ static R reference(T n) { return R(n); }
};
template <> struct PopCodec<__half> {
  using E = __half;
  using R = __half;
  static constexpr bool shifted = true;
  template <class T> __device__ __forceinline__ static T decode(__half h, __half r, float inv_s) {
    return T(__half2float(r)) + T(__half2float(h)) * T(inv_s);
  }
  template <class T> __device__ __forceinline__ static __half encode(T n, __half r, float s) {
    return __float2half_rn(float((n - T(__half2float(r))) * T(s)));
  }
  template <class T> __device__ __forceinline__ static R reference(T n) { return __float2half_rn(float(n)); }
};
template <> struct PopCodec<__hip_bfloat16> {
  using E = __hip_bfloat16;
  using R = __hip_bfloat16;
  static constexpr bool shifted = true;
  template <class T> __device__ __forceinline__ static T decode(__hip_bfloat16 h, __hip_bfloat16 r, float inv_s) {
    return T(__bfloat162float(r)) + T(__bfloat162float(h)) * T(inv_s);
  }
  template <class T> __device__ __forceinline__ static __hip_bfloat16 encode(T n, __hip_bfloat16 r, float s) {
    return __float2bfloat16(float((n - T(__bfloat162float(r))) * T(s)));
  }
  template <class T> __device__ __forceinline__ static R reference(T n) { return __float2bfloat16(float(n)); }
};
template <> struct PopCodec<F32Dev> {
  using E = float;
  using R = __half;
  static constexpr bool shifted = true;
  // FP16 + FP32 -> FP64 is exact; the arithmetic type is FP64 for this storage
  template <class T> __device__ __forceinline__ static T decode(float h, __half r, float) {
    return T(__half2float(r)) + T(h);
  }
  template <class T> __device__ __forceinline__ static float encode(T n, __half r, float) {
    return float(n - T(__half2float(r)));
  }
  // FP16's range ends at 65504: a population beyond it keeps the largest
  // finite reference (the FP32 deviation carries the rest)
  template <class T> __device__ __forceinline__ static R reference(T n) {
    const float v = float(n);
    return __float2half_rn(fminf(fmaxf(v, -65504.0f), 65504.0f));
  }
};
template <class P> using PopE = typename PopCodec<P>::E;
template <class P> using PopR = typename PopCodec<P>::R;

// Re-basing of one cell's slots (shifted modes): every slot the cell wrote
// takes its own rounding to the reference type as its new reference and is
// re-encoded against it, so the stored deviations restart near zero.  Shared
// by the single-mesh and the batched re-basing kernels, so both give the same
// bits.
template <class L, class P>
__device__ __forceinline__ void rebase_cell(PopE<P>* __restrict__ pop, PopR<P>* __restrict__ rown, int nc, int cell,
                                            float scale, float inv_scale) {
  using C = PopCodec<P>;
  using T = typename std::conditional<std::is_same<P, F32Dev>::value, double, float>::type;
#pragma unroll
  for (int al = 0; al < L::Q; ++al) {
    const size_t i = (size_t)al * (size_t)nc + (size_t)cell;
    const T n = C::template decode<T>(pop[i], rown[i], inv_scale);
    const PopR<P> r = C::template reference<T>(n);
    rown[i] = r;
    pop[i] = C::template encode<T>(n, r, scale);
  }
}


// Number of stored g^{ij} words (upper triangle) and its index map.
template <int D> __host__ __device__ constexpr int nup() { return D * (D + 1) / 2; }
template <int D> __host__ __device__ constexpr int up(int i, int j) {
  // row-major upper triangle: D=2: 00,01,11; D=3: 00,01,02,11,12,22
  return (i <= j) ? (i * D - i * (i - 1) / 2 + (j - i)) : (j * D - j * (j - 1) / 2 + (i - j));
}

// ---------------------------------------------------------------------------
// Topology of the index box, passed by value to kernels.
// ---------------------------------------------------------------------------
struct Box {
  int n[3];        // real cells per axis (n[2] = 1 in 2-D)
  int face[3][2];  // VLBM_PERIODIC / VLBM_WALL / VLBM_FARFIELD
  int ncells;
  double inv_n[2]; // 1 / n[0], 1 / n[1] (cell_coords)
};

// (x, y, z) of a cell index without integer division: with c < 2^30 and
// n <= 2^20, (c + 1/2) / n lies at least 1/(2n) >= 2^-21 from an integer and
// the FP64 product (c + 1/2) * fl(1/n) is within 2^-22 of it, so its floor is
// the exact quotient.
__device__ __forceinline__ void cell_coords(const Box& b, int cell, int& x, int& y, int& z) {
  const int r = int(floor((double(cell) + 0.5) * b.inv_n[0]));
  x = cell - r * b.n[0];
  z = int(floor((double(r) + 0.5) * b.inv_n[1]));
  y = r - z * b.n[1];
}

// Kind of the source of a pulled link.
enum LinkKind { LINK_INTERIOR = 0, LINK_WALL = 1, LINK_FARFIELD = 2 };

// Source of direction a arriving at cell (x, y, z): N_a(q) = N'_a(q - c_a)
// (eq. (adv)).  Periodic axes wrap; a link that leaves through a far-field
// face is FARFIELD, otherwise through a wall face is WALL.  Written with
// selects only, so that a wavefront never diverges on it.
//
// A WALL link reads the opposite population of its bounce-back source: the
// cell itself for one-cell links.  A longer link (D2Q21, D3Q39: walls on one
// axis i only) follows its straight path reflected at the wall, half a cell
// beyond the last real cell: the source lies d cells from the wall with
// q_s^i = |c^i| - 1 - q^i (low face) or 2 n_i - 1 - |c^i| - q^i (high face),
// and q_s^j = q^j - c^j (|c^i| - 2 d - 1) / |c^i| on the other (periodic) axes.
template <class L>
__device__ __forceinline__ int link_source(const Box& b, int a, int x, int y, int z, int& src) {
  const int q0[3] = {x, y, z};
  int q[3] = {x, y, z};
  int wall = 0, far = 0, wax = 0;
#pragma unroll
  for (int i = 0; i < L::D; ++i) {
    const int ci = L::c(a, i);
    if (ci == 0) continue;                    // compile-time
    const int s = q[i] - ci;
    const int n = b.n[i];
    const int side = ci > 0 ? 0 : 1;          // compile-time: leaving through the low (0) or high (1) face
    const int out = ci > 0 ? (s < 0) : (s >= n);
    const int f = b.face[i][side];
    const int per = f == VLBM_PERIODIC;
    q[i] = out ? (per ? (ci > 0 ? s + n : s - n) : q[i]) : s;
    const int w = out & (f == VLBM_WALL);
    wall |= w;
    wax = w ? i : wax;
    far |= out & (f == VLBM_FARFIELD);
  }
  src = q[0] + b.n[0] * (q[1] + b.n[1] * q[2]);
  // non-periodic exits keep the own cell as source (the bounce-back slot)
  src = (wall | far) ? x + b.n[0] * (y + b.n[1] * z) : src;
  if constexpr (L::SPEED > 1) {
    // every non-zero component of a link of these lattices has the same
    // magnitude k, so the shift c^j (k - 2 d - 1) / k is sgn(c^j) (k - 2 d - 1)
    int qs[3] = {x, y, z};
    int dist = 0;
#pragma unroll
    for (int i = 0; i < L::D; ++i) {
      const int ci = L::c(a, i);
      if (ci == 0) continue;
      const int n = b.n[i];
      const int kk = ci > 0 ? ci : -ci;
      const int si = ci > 0 ? kk - 1 - q0[i] : 2 * n - 1 - kk - q0[i];
      const int here = i == wax;
      qs[i] = here ? si : qs[i];
      dist = here ? (ci > 0 ? si : n - 1 - si) : dist;
    }
#pragma unroll
    for (int j = 0; j < L::D; ++j) {
      const int cj = L::c(a, j);
      if (cj == 0) continue;
      const int k = cj > 0 ? cj : -cj;
      const int n = b.n[j];
      int s = q0[j] - (cj > 0 ? 1 : -1) * (k - 2 * dist - 1);
      s = s < 0 ? s + n : (s >= n ? s - n : s);
      qs[j] = j == wax ? qs[j] : s;
    }
    src = (wall & !far) ? qs[0] + b.n[0] * (qs[1] + b.n[1] * qs[2]) : src;
  }
  return far ? LINK_FARFIELD : (wall ? LINK_WALL : LINK_INTERIOR);
}

// The same rule prepared once per cell: along each axis the linear offset of
// the source for c^i = +1 (the neighbour at q^i - 1) and for c^i = -1 (at
// q^i + 1), with the periodic wrap applied, and bit i set in wall/far when that
// neighbour lies beyond a wall or far-field face.  link_at then resolves a
// direction with compile-time component tests only.
struct LinkPlan {
  int off_lo[3], off_hi[3];
  unsigned wall_lo, wall_hi, far_lo, far_hi;
};

// the cell lies on a far-field face (so some of its links come from beyond it)
template <class L>
__device__ __forceinline__ bool on_farfield_face(const Box& b, int x, int y, int z) {
  const int q[3] = {x, y, z};
  bool f = false;
#pragma unroll
  for (int i = 0; i < L::D; ++i)
    f = f || (q[i] == 0 && b.face[i][0] == VLBM_FARFIELD) || (q[i] == b.n[i] - 1 && b.face[i][1] == VLBM_FARFIELD);
  return f;
}

template <class L>
__device__ __forceinline__ LinkPlan link_plan(const Box& b, int x, int y, int z) {
  const int q[3] = {x, y, z};
  LinkPlan p;
  p.wall_lo = p.wall_hi = p.far_lo = p.far_hi = 0u;
  int stride = 1;
#pragma unroll
  for (int i = 0; i < L::D; ++i) {
    const int n = b.n[i];
    const int at_lo = q[i] == 0, at_hi = q[i] == n - 1;
    const int flo = b.face[i][0], fhi = b.face[i][1];
    p.off_lo[i] = at_lo ? (flo == VLBM_PERIODIC ? (n - 1) * stride : 0) : -stride;
    p.off_hi[i] = at_hi ? (fhi == VLBM_PERIODIC ? -(n - 1) * stride : 0) : stride;
    p.wall_lo |= (unsigned)(at_lo & (flo == VLBM_WALL)) << i;
    p.far_lo |= (unsigned)(at_lo & (flo == VLBM_FARFIELD)) << i;
    p.wall_hi |= (unsigned)(at_hi & (fhi == VLBM_WALL)) << i;
    p.far_hi |= (unsigned)(at_hi & (fhi == VLBM_FARFIELD)) << i;
    stride *= n;
  }
  return p;
}

// link_source for compile-time direction a from a prepared plan (cell = own index).
template <class L, int a>
__device__ __forceinline__ int link_at(const LinkPlan& p, int cell, int& src) {
  int off = 0;
  unsigned lo = 0u, hi = 0u;   // compile-time masks of the axes whose low / high neighbour is the source
#pragma unroll
  for (int i = 0; i < L::D; ++i) {
    const int ci = L::c(a, i);
    if (ci > 0) {
      off += p.off_lo[i];
      lo |= 1u << i;
    } else if (ci < 0) {
      off += p.off_hi[i];
      hi |= 1u << i;
    }
  }
  const unsigned far = (p.far_lo & lo) | (p.far_hi & hi);
  const unsigned wall = (p.wall_lo & lo) | (p.wall_hi & hi);
  src = (far | wall) ? cell : cell + off;
  return far ? LINK_FARFIELD : (wall ? LINK_WALL : LINK_INTERIOR);
}

// ---------------------------------------------------------------------------
// Host-side objects.
// ---------------------------------------------------------------------------
struct SimObj;

struct MeshObj {
  int users = 0;                 // simulations that hold the mesh
  SimObj* mover = nullptr;       // the simulation that moved the mesh (vlbm_step_moving), if any
  bool destroy_pending = false;  // vlbm_mesh_destroy was called while simulations held it
  int lattice;
  int d, Q;
  Box box;
  int m[3];          // coordinate array extents (with ghosts on non-periodic axes)
  double wrap[3][3];
  double dx;
  double* coords = nullptr;   // device [m3][m2][m1][d]
  // FP64 geometry (device), valid after precompute
  bool have_geometry = false;
  double* J = nullptr;        // [cells]
  double* gup = nullptr;      // [d*d][cells]
  double* gco = nullptr;      // [d][d][cells]  g^i components
  double* g = nullptr;        // [d][d][cells]  g_i components
  double* A = nullptr;        // [Q][d][cells]; after a moving step made on demand (refresh_moving_state)
  vlbm_geom_report report{};
};

// Geometry pack words for the step kernels (SoA, stride = ncells).  With FP32
// words and FP64 arithmetic g^{ij} is held as a pair hi + lo of FP32 words
// (hi = fl32(g), lo = fl32(g - hi), about 48 bits): g^{ij} sets the metric part
// of the equilibrium stress, which balances the inertial force of a resting
// fluid, and FP32 rounding of it alone acts as a spurious force (on slow flows
// it dominates the FP32-storage error); J and A in FP32 are harmless.  The lo
// words are read only by that combination (zero for FP64 words).
template <class L> struct Pack {
  static constexpr int J = 0;
  static constexpr int GUP = 1;
  // a >= 1: S^i = A^i_a + A^i_(a+1) (odd a) and D^i = A^i_(a-1) - A^i_a (even
  // a), the pair form (moving meshes have no pack: their step computes the
  // coefficients from g_i)
  static constexpr int A = GUP + nup<L::D>();
  static constexpr int AEXT = A + (L::Q - 1) * L::D;          // present if force
  static constexpr int UINF = AEXT + L::D;                    // present if far field
  static constexpr int GUPLO = UINF + L::D;                   // low words of g^{ij}
  static constexpr int WORDS = GUPLO + nup<L::D>();
};

// The packed geometry is tiled by wavefronts: the words of 64 consecutive
// cells are stored word by word, [cell / 64][word][cell % 64].  A wave reads
// 64 consecutive elements per word (as with one array per word), and all the
// words of its cells lie within immediate offsets of one per-lane address.
constexpr int kGeoTile = 64;
template <class L>
__host__ __device__ __forceinline__ size_t pack_index(int word, int cell) {
  const unsigned c = (unsigned)cell;
  return (size_t)(c / kGeoTile) * (Pack<L>::WORDS * kGeoTile) + (size_t)word * kGeoTile + (size_t)(c % kGeoTile);
}
// Elements of a packed geometry of nc cells (the last tile is whole).
inline size_t pack_elements(int words, size_t nc) {
  return (nc + kGeoTile - 1) / kGeoTile * kGeoTile * (size_t)words;
}

inline int pack_words(int lattice) {
  switch (lattice) {
    case VLBM_D2Q9: return Pack<D2Q9>::WORDS;
    case VLBM_D3Q19: return Pack<D3Q19>::WORDS;
    case VLBM_D2Q21: return Pack<D2Q21>::WORDS;
    default: return Pack<D3Q39>::WORDS;
  }
}

struct SimObj {
  MeshObj* mesh;
  vlbm_params p;
  hipStream_t stream;
  int64_t t = 0;
  int buf = 0;            // index of the buffer that holds N'(t-1)
  void* pop[2] = {nullptr, nullptr};
  size_t pop_bytes = 0;
  void* geo = nullptr;    // precision pack
  void* rown = nullptr;     // shifted modes: [Q][cells] 16-bit reference of each slot (read by the slot's
                            // writer and, at the same offset as the population, by its reader)
  void* rown_spare = nullptr;   // shifted modes: a second reference array; a re-basing step writes the new
                                // references there and the two are swapped after it
  int rebase_in_step = 0;       // the next step launch re-bases its outputs (into rown_spare)
  int batch_member = 0;         // owned by a batch, whose step arguments hold its reference array
  void* fcache = nullptr;   // [d][cells]: converged inertial force per unit density of the last step (fixed-point start),
                            // FP64 with FP64 storage, FP32 otherwise
  int has_force = 0, has_farfield = 0;
  int comp_A = 0;   // FP32 words, FP64 arithmetic: the a_ext words also cancel the rounding of A
  // audits
  void* audit_ring = nullptr;   // device vlbm_audit[cap]
  int audit_cap = 0;
  int64_t audit_head = 0, audit_tail = 0;
  double* audit_partial = nullptr;  // device scratch for block partials
  int audit_blocks = 0;
  double* u_prev = nullptr;     // device [d][cells]
  int have_u_prev = 0;
  int* flags = nullptr;         // device int[4]: 0 = unconverged cells of a dry run (init, moments),
                                //                2 = unconverged cell-steps of the step kernel
  unsigned long long* stats = nullptr;   // device [kStatSlots][4]: fixed-point statistics of the steps (when stats_on)
  int stats_on = 0;
  // moving mesh (vlbm_step_moving): g_i boxes of the times t - 1, t, t + 1,
  // the real-cell geometry of t + 1 and the incoming coefficients of the
  // current state (audits); allocated at the first moving step
  int moving = 0;
  int geo_stale = 0;              // the static pack no longer matches the mesh
  // the mesh moved in the last step: the state's incoming coefficients (Ain),
  // the mesh's outgoing ones of the new positions (mesh->A) and its real-cell
  // g_i (mesh->g) are made from the g_i boxes of the last two times when
  // first needed
  int mv_state_stale = 0;
  int state_moving = 0;           // the last step moved the mesh: the state reads Ain
  double* mv_box[3] = {nullptr, nullptr, nullptr};
  double *mv_J = nullptr, *mv_gup = nullptr, *mv_gco = nullptr;
  double* Ain = nullptr;          // [Q][d][cells], null on a static mesh
  // kernel timing (vlbm_kernel_timing): event pairs around the step and the
  // re-basing launches, resolved when read
  int timing_on = 0;
  void* timing = nullptr;   // host-side event pool (capi.hip)
};

// The general collision matrix is used when tau_g is set and differs from tau
// (tau_g = tau is BGK exactly).
inline int general_collision(const vlbm_params& p) { return p.tau_g != 0.0 && p.tau_g != p.tau ? 1 : 0; }

inline bool storage_is_fp64(int precision) { return precision == VLBM_FP64; }
inline bool storage_is_16(int precision) { return precision == VLBM_FP16S || precision == VLBM_BF16S; }
// modes whose slots hold deviations from a 16-bit per-slot reference
inline bool storage_shifted(int precision) { return storage_is_16(precision) || precision == VLBM_FP32; }
inline size_t pop_elem(int precision) {
  return precision == VLBM_FP64 ? 8 : (storage_is_16(precision) ? 2 : 4);
}
// Scale s of the stored FP16 deviations (N - reference) * s.  FP16 keeps its
// relative precision at any scale, but its range ends at 65504: deviations grow
// with the cell volume J, so the scale is the largest power of two up to 4096
// that keeps deviations up to 4 J_max representable.  BF16 shares FP32's
// exponent range and FP32 deviations need no scale.
inline float pop_scale(int precision, double max_J) {
  if (precision != VLBM_FP16S) return 1.0f;
  const double jm = max_J > 1e-30 ? max_J : 1e-30;
  const double cap = 65504.0 / (4.0 * jm);
  float s = 4096.0f;
  while (s > 1.0f / 1024.0f && s > cap) s *= 0.5f;
  return s;
}
// The force cache only seeds the fixed point (the converged F does not depend
// on it): FP32 except with FP64 storage.
inline size_t fcache_elem(int precision) { return precision == VLBM_FP64 ? 8 : 4; }
// Re-basing period of the references (steps; vlbm_params.rebase_every: 0 =
// default, < 0 = never).
// copies of the fixed-point statistics counters (by block), summed on the host
constexpr int kStatSlots = 64;
constexpr int kDefaultRebase = 10;
inline int rebase_period(const vlbm_params& p) { return p.rebase_every == 0 ? kDefaultRebase : p.rebase_every; }

// Kernel launchers (defined in the .hip files).
hipError_t launch_geometry(MeshObj* m, hipStream_t s, int* dflag, double* partial, int nblocks_partial,
                           double* gbox);
size_t geometry_box_cells(const MeshObj* m);
hipError_t launch_basis_of(const MeshObj* m, const double* coords, const double (*wrap)[3], double* gbox, double* J,
                           double* gup, double* gco, double* g, int* dflag, hipStream_t s);
// After a moving step: Ain of the state and mesh->A of the new positions, if
// not made since (geometry.hip); enqueued on the sim's stream.
hipError_t refresh_moving_state(SimObj* s);
// Allocates the mesh's FP64 geometry arrays (J, g^{ij}, g^i, g_i, A).
int alloc_mesh_geometry(MeshObj* m);
// Report of a geometry pass (capi.hip): flag of degenerate cells and the
// reduced diagnostics r[6]; sets the thread-local error on failure.
int finish_geometry(MeshObj* m, int flag, const double* r, vlbm_geom_report* rep);
int set_error(int code, const char* fmt, ...);
hipError_t launch_pack(SimObj* s);
hipError_t launch_init(SimObj* s, const double* rho, const double* u, int* dflag);
hipError_t launch_step(SimObj* s);
// one step on a moving mesh from g_i on the geometry boxes of the times
// t - 1, t and t + 1 and the mesh's real-cell geometry of t (step.hip)
hipError_t launch_step_moving(SimObj* s, const double* gprev, const double* gcur, const double* gnext);
hipError_t launch_moments(SimObj* s, double* rho, double* u, double* U, int* dflag);
hipError_t launch_get_pop(SimObj* s, double* N);
hipError_t launch_set_pop(SimObj* s, const double* N);
hipError_t launch_audit(SimObj* s, int slot);
hipError_t launch_refs(SimObj* s);
hipError_t launch_rebase(SimObj* s);     // shifted modes: references re-based on the current state

int geometry_partial_blocks(const MeshObj* m);

}  // namespace vlbm

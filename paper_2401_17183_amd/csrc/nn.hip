// Kernels of the convolutional surrogate (gfx950): implicit-GEMM 3x3
// convolutions on v_mfma_f32_16x16x32_bf16 with FP32 accumulation, and the
// small elementwise kernels of training (ReLU gradient, MSE, Adam, packing).
//
// Operand layout of the 16x16x32 BF16 MFMA used throughout: lane l supplies
// row (l % 16) of the 16x32 A operand and column (l % 16) of the 32x16 B
// operand, each as the 8 consecutive reduction indices 8 (l / 16) .. +7; it
// receives rows 4 (l / 16) + r, r = 0..3, of column (l % 16) of the 16x16
// result.
#include "nn.hpp"

namespace vlbm {
namespace nn {
namespace {

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));
typedef uint32_t u32x4 __attribute__((__vector_size__(4 * sizeof(uint32_t))));

constexpr int kThreads = 256;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ u32x4 ld16(const uint16_t* p) { return *reinterpret_cast<const u32x4*>(p); }

__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// Output pixel of a forward row: batch index and the top-left input corner.
struct RowF {
  int n, ih0, iw0;
  bool ok;
};

__device__ __forceinline__ RowF row_fwd(const Conv& c, int64_t m, int64_t M) {
  RowF r;
  r.ok = m < M;
  const int64_t mm = r.ok ? m : 0;
  const int ow = (int)(mm % c.OW);
  const int64_t t = mm / c.OW;
  const int oh = (int)(t % c.OH);
  r.n = (int)(t / c.OH);
  r.ih0 = oh * c.stride - 1;
  r.iw0 = ow * c.stride - 1;
  return r;
}

// The 8 input channels ch..ch+7 at tap (kh, kw) of a forward row (zero
// outside).  Branch-free: the load always happens, from the tensor's first
// element when the tap is outside, and the result is then selected.  Element
// offsets are 32-bit (check() bounds every tensor below 2^31 elements).
__device__ __forceinline__ u32x4 gather_fwd(const Conv& c, const uint16_t* x, const uint16_t* skip, const RowF& r,
                                            int kh, int kw, int ch, bool kok) {
  const int ih = r.ih0 + kh, iw = r.iw0 + kw;
  const u32x4 z = {0u, 0u, 0u, 0u};
  const bool valid = r.ok && kok && (unsigned)ih < (unsigned)c.H && (unsigned)iw < (unsigned)c.W;
  const bool prim = ch < c.cin;
  const int hs = c.up ? (c.H >> 1) : c.H, ws = c.up ? (c.W >> 1) : c.W;
  const int y = c.up ? (ih >> 1) : ih, xx = c.up ? (iw >> 1) : iw;
  const int offp = ((r.n * hs + y) * ws + xx) * c.cin + ch;
  const int offs = ((r.n * c.H + ih) * c.W + iw) * c.cskip + (ch - c.cin);
  const uint16_t* p = prim ? x + offp : skip + offs;
  const u32x4 v = ld16(valid ? p : x);
  return valid ? v : z;
}

// Input-gradient row: pixel (n, y, x) of the tensor whose gradient is formed;
// with sub4 it is a pixel of the half-resolution primary input and the four
// upsampled positions it feeds are folded into the reduction.
struct RowB {
  int n, y, x;
  bool ok;
};

__device__ __forceinline__ RowB row_bwd(int64_t m, int64_t M, int h, int w) {
  RowB r;
  r.ok = m < M;
  const int64_t mm = r.ok ? m : 0;
  r.x = (int)(mm % w);
  const int64_t t = mm / w;
  r.y = (int)(t % h);
  r.n = (int)(t / h);
  return r;
}

// gy channels co..co+7 at the output pixel that reads input (ih, iw) through
// tap (kh, kw); branch-free like gather_fwd (stride 1 or 2).
__device__ __forceinline__ u32x4 gather_bwd(const Conv& c, const uint16_t* gy, const RowB& r, int sub4, int sub,
                                            int kh, int kw, int co, bool kok) {
  const u32x4 z = {0u, 0u, 0u, 0u};
  const int ih = sub4 ? 2 * r.y + (sub >> 1) : r.y;
  const int iw = sub4 ? 2 * r.x + (sub & 1) : r.x;
  const int ohn = ih + 1 - kh, own = iw + 1 - kw;
  const int sm = c.stride - 1, sh = c.stride >> 1;   // stride 1 or 2
  const int oh = ohn >> sh, ow = own >> sh;
  const bool valid = r.ok && kok && ohn >= 0 && own >= 0 && ((ohn | own) & sm) == 0 && oh < c.OH && ow < c.OW;
  const int off = ((r.n * c.OH + oh) * c.OW + ow) * c.cout + co;
  const u32x4 v = ld16(valid ? gy + off : gy);
  return valid ? v : z;
}

struct Gemm {
  int64_t M;
  int ncols, K;
  const uint16_t* a0;
  const uint16_t* a1;
  const uint16_t* b;   // [rows][b_ld]
  int b_ld, b_row0;
  int sub4;            // backward only: fold the 2x2 upsampling
  int rh, rw;          // backward only: spatial size of the rows' tensor
  const float* bias;
  uint16_t* y16;
  float* y32;
  int out_ld;
};

// C[m][n] = sum_k A(m, k) B[n][k].  FWD: A = im2col of the layer input,
// B = W; epilogue bias + ReLU, BF16 and/or FP32 store.  BWD: A = the output
// gradient read through the transposed convolution, B = W^T; epilogue +=.
// Four waves stacked along m, each owning 32 rows x 16 TJ columns: one A
// gather (the costly, index-heavy operand) feeds 2 TJ MFMAs per K step.
template <bool FWD, int TJ>
__global__ __launch_bounds__(kThreads) void k_conv_gemm(Conv c, Gemm g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * 128 + wave * 32;
  const int n0 = blockIdx.y * (16 * TJ);
  const int l16 = lane & 15, kq = 8 * (lane >> 4);
  f32x4 acc[2][TJ];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  RowF rf[2];
  RowB rb[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int64_t m = m0 + 16 * i + l16;
    if constexpr (FWD) rf[i] = row_fwd(c, m, g.M);
    else rb[i] = row_bwd(m, g.M, g.rh, g.rw);
  }
  const int ct = c.ctot();
  const int kb = 9 * c.cout;   // backward: reduction indices per sub-position
  const u32x4 z = {0u, 0u, 0u, 0u};
  const uint16_t* brow[TJ];
  bool bok[TJ];
#pragma unroll
  for (int j = 0; j < TJ; ++j) {
    const int col = n0 + 16 * j + l16;
    bok[j] = col < g.ncols;
    brow[j] = g.b + (int64_t)(g.b_row0 + (bok[j] ? col : 0)) * g.b_ld;
  }
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    const int k = k0 + kq;
    const bool kok = k < g.K;
    u32x4 av[2];
    int kbk;   // column of B
    if constexpr (FWD) {
      const int tap = k / ct, ch = k - tap * ct;
      const int kh = (tap * 11) >> 5, kw = tap - 3 * kh;   // tap / 3 for tap < 9
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = gather_fwd(c, g.a0, g.a1, rf[i], kh, kw, ch, kok);
      kbk = k;
    } else {
      const int sub = g.sub4 ? k / kb : 0;
      const int rem = k - sub * kb;
      const int tap = rem / c.cout, co = rem - tap * c.cout;
      const int kh = (tap * 11) >> 5, kw = tap - 3 * kh;
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = gather_bwd(c, g.a0, rb[i], g.sub4, sub, kh, kw, co, kok);
      kbk = rem;
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const bool ok = kok && bok[j];
      const u32x4 v = ld16(brow[j] + (ok ? kbk : 0));
      const u32x4 bv = ok ? v : z;
#pragma unroll
      for (int i = 0; i < 2; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(av[i]), as_bf(bv), acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int col = n0 + 16 * j + l16;
      if (col >= g.ncols) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + 16 * i + 4 * (lane >> 4) + r;
        if (row >= g.M) continue;
        float v = acc[i][j][r];
        const int64_t o = row * g.out_ld + col;
        if constexpr (FWD) {
          v += g.bias ? g.bias[col] : 0.f;
          if (c.relu) v = v > 0.f ? v : 0.f;
          if (g.y16) g.y16[o] = f2bf(v);
          if (g.y32) g.y32[o] = v;
        } else {
          g.y32[o] += v;
        }
      }
    }
}

// Weight gradient: gw[co][t][ch] += sum_p gy[p][co] x(p + tap t)[ch] and
// gb[co] += sum_p gy[p][co], the sums over the N x OH x OW output pixels p.
// The MFMA reduction index must be contiguous in a lane's operand, so the
// pixels of one reduction step are grouped as 8 images x 4 positions: a lane
// supplies the 8 images of one output position.  A block stages, per box of
// PH x PW output positions of 8 images, the output gradient [co][position][8
// images] and the input halo of its 32-channel chunk [channel][halo
// position][8 images] in LDS; the shift of tap t is then a whole 16-byte
// step in the halo, so every fragment read is one aligned 16-byte LDS read
// for any tap and stride.  Staging loads 8 images x 8 channels as eight 16-byte
// loads and transposes them in registers (v_perm_b32) into eight 16-byte rows.
// A block owns CO = 16 CF output channels x the 9 taps x one 32-channel chunk
// (4 waves share the 18 (tap, 16-channel) column fragments), and a run of
// boxes; the bias is one more MFMA against a fragment of ones.  With a
// workspace each block writes its partial sums to slice blockIdx.x (weights at
// [co][9 ct], then the bias at [C_out 9 ct + co]) and the slices are summed in
// a fixed order (k_sum_slices, k_wgrad_reduce), so the result does not depend
// on scheduling; without one, the blocks add their sums with FP32 atomics.
struct WgradTile {
  const uint16_t* x;      // primary input (half resolution when up)
  const uint16_t* skip;   // skip input, channels [cin, ct)
  const uint16_t* gy;
  int N, H, W, cin, ct, up, OH, OW, cout;
  int tiles_w, tiles_h, units, per_block;
  float* part;            // slices of slice floats, or null
  int64_t slice;
  float* gw;
  float* gb;
};

__device__ __forceinline__ void transpose8(const u32x4 (&v)[8], int c, u32x4& out) {
  // row c of the 8 x 8 block: element c of each of the 8 vectors
  const uint32_t sel = (c & 1) ? 0x07060302u : 0x05040100u;
  const int d = c >> 1;
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = __builtin_amdgcn_perm(v[2 * k + 1][d], v[2 * k][d], sel);
}

template <int CF, int RS>
__global__ __launch_bounds__(kThreads) void k_wgrad_tile(WgradTile g) {
  constexpr int CO = 16 * CF;
  constexpr int PH = 4, PW = RS == 1 ? 8 : 4, P = PH * PW;
  constexpr int HH = RS * (PH - 1) + 3, HW = RS * (PW - 1) + 3, HP = HH * HW;
  constexpr int GS = P + 1;          // row strides in 16-byte units, odd: conflict-free fragment reads
  constexpr int XS = HP | 1;
  constexpr int NPAIR = 5;           // (tap, channel fragment) pairs per wave: 18 over 4 waves
  __shared__ __attribute__((aligned(16))) uint16_t sG[CO * GS * 8];
  __shared__ __attribute__((aligned(16))) uint16_t sX[32 * XS * 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  const int chunk = blockIdx.y, co0 = blockIdx.z * CO, ch0 = 32 * chunk;
  const int K = 9 * g.ct;
  const bool bias = wave == 3 && chunk == 0;
  const u32x4 z = {0u, 0u, 0u, 0u};
  const u32x4 ones = {0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u};
  f32x4 acc[NPAIR][CF], accb[CF];
#pragma unroll
  for (int i = 0; i < NPAIR; ++i)
#pragma unroll
    for (int f = 0; f < CF; ++f) acc[i][f] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int f = 0; f < CF; ++f) accb[f] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int hs = g.up ? g.H >> 1 : g.H, ws = g.up ? g.W >> 1 : g.W, c1 = g.ct - g.cin;

  const int u0 = blockIdx.x * g.per_block;
  const int u1 = u0 + g.per_block < g.units ? u0 + g.per_block : g.units;
  for (int u = u0; u < u1; ++u) {
    const int ow0 = (u % g.tiles_w) * PW;
    const int ut = u / g.tiles_w;
    const int oh0 = (ut % g.tiles_h) * PH;
    const int n0 = (ut / g.tiles_h) * 8;
    __syncthreads();   // the previous box's fragment reads are done
    for (int e = tid; e < P * CO / 8; e += kThreads) {
      const int pos = e / (CO / 8), cg = e % (CO / 8);
      const int oh = oh0 + pos / PW, ow = ow0 + pos % PW, co = co0 + 8 * cg;
      const bool ok = oh < g.OH && ow < g.OW && co < g.cout;
      u32x4 v[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int n = n0 + m;
        v[m] = (ok && n < g.N) ? ld16(g.gy + ((n * g.OH + oh) * g.OW + ow) * g.cout + co) : z;
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        u32x4 r;
        transpose8(v, c, r);
        *reinterpret_cast<u32x4*>(sG + ((8 * cg + c) * GS + pos) * 8) = r;
      }
    }
    for (int e = tid; e < HP * 4; e += kThreads) {
      const int hp = e >> 2, grp = e & 3;
      const int ih = RS * oh0 - 1 + hp / HW, iw = RS * ow0 - 1 + hp % HW, ch = ch0 + 8 * grp;
      const bool ok = (unsigned)ih < (unsigned)g.H && (unsigned)iw < (unsigned)g.W && ch < g.ct;
      u32x4 v[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int n = n0 + m;
        v[m] = z;
        if (ok && n < g.N) {
          if (ch < g.cin) {
            const int y = g.up ? ih >> 1 : ih, xx = g.up ? iw >> 1 : iw;
            v[m] = ld16(g.x + ((n * hs + y) * ws + xx) * g.cin + ch);
          } else {
            v[m] = ld16(g.skip + ((n * g.H + ih) * g.W + iw) * c1 + (ch - g.cin));
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        u32x4 r;
        transpose8(v, c, r);
        *reinterpret_cast<u32x4*>(sX + ((8 * grp + c) * XS + hp) * 8) = r;
      }
    }
    __syncthreads();
#pragma unroll 2
    for (int ks = 0; ks < P / 4; ++ks) {
      const int pos = 4 * ks + lg;   // this lane group's output position; its 8 images are the K slice
      const int ph = pos / PW, pw = pos % PW;
      u32x4 a[CF];
#pragma unroll
      for (int f = 0; f < CF; ++f) a[f] = *reinterpret_cast<const u32x4*>(sG + ((16 * f + l16) * GS + pos) * 8);
#pragma unroll
      for (int i = 0; i < NPAIR; ++i) {
        const int pr = wave + 4 * i;
        if (pr >= 18) continue;
        const int tap = pr >> 1, chf = pr & 1;
        const int hp = (RS * ph + tap / 3) * HW + RS * pw + tap % 3;
        const u32x4 b = *reinterpret_cast<const u32x4*>(sX + ((16 * chf + l16) * XS + hp) * 8);
#pragma unroll
        for (int f = 0; f < CF; ++f)
          acc[i][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a[f]), as_bf(b), acc[i][f], 0, 0, 0);
      }
      if (bias) {
#pragma unroll
        for (int f = 0; f < CF; ++f)
          accb[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a[f]), as_bf(ones), accb[f], 0, 0, 0);
      }
    }
  }
  float* part = g.part ? g.part + (int64_t)blockIdx.x * g.slice : nullptr;
#pragma unroll
  for (int i = 0; i < NPAIR; ++i) {
    const int pr = wave + 4 * i;
    if (pr >= 18) continue;
    const int tap = pr >> 1, ch = ch0 + 16 * (pr & 1) + l16;
    if (ch >= g.ct) continue;
#pragma unroll
    for (int f = 0; f < CF; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = co0 + 16 * f + 4 * lg + r;
        if (co >= g.cout) continue;
        const int64_t o = (int64_t)co * K + tap * g.ct + ch;
        if (part) part[o] = acc[i][f][r];
        else unsafeAtomicAdd(&g.gw[o], acc[i][f][r]);
      }
  }
  if (bias && l16 == 0) {
#pragma unroll
    for (int f = 0; f < CF; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = co0 + 16 * f + 4 * lg + r;
        if (co >= g.cout) continue;
        if (part) part[(int64_t)g.cout * K + co] = accb[f][r];
        else unsafeAtomicAdd(&g.gb[co], accb[f][r]);
      }
  }
}

// dst[g][e] = sum over z in [g G, min((g + 1) G, slices)) of src[z][e], in that
// order (slices of m elements).
__global__ void k_sum_slices(const float* __restrict__ src, float* dst, int64_t m, int slices, int G) {
  const int groups = (slices + G - 1) / G;
  const int64_t total = (int64_t)groups * m;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(i / m);
    const int64_t e = i - (int64_t)g * m;
    const int z1 = (g + 1) * G < slices ? (g + 1) * G : slices;
    float acc = 0.f;
#pragma unroll 8
    for (int z = g * G; z < z1; ++z) acc += src[z * m + e];
    dst[i] = acc;
  }
}

// gw[e] += sum over z of part[z][e] (e < n), gb[e - n] likewise (n <= e < m),
// in slice order; with assign, = instead of +=.
__global__ void k_wgrad_reduce(const float* __restrict__ part, float* gw, float* gb, int64_t n, int64_t m,
                               int slices, int assign) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    float acc = 0.f;
#pragma unroll 8
    for (int z = 0; z < slices; ++z) acc += part[z * m + e];
    if (e < n) gw[e] = assign ? acc : gw[e] + acc;
    else gb[e - n] = assign ? acc : gb[e - n] + acc;
  }
}

__global__ void k_pack_w(Conv c, const float* __restrict__ w, uint16_t* w16, uint16_t* wt16) {
  const int ct = c.ctot();
  const int64_t n = (int64_t)c.cout * 9 * ct;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ci = (int)(i % ct);
    const int64_t r = i / ct;
    const int tap = (int)(r % 9);
    const int co = (int)(r / 9);
    const uint16_t h = f2bf(w[i]);
    w16[i] = h;
    wt16[((int64_t)ci * 9 + tap) * c.cout + co] = h;
  }
}

// k_pack_w for several layers in one launch: blockIdx.y is the layer.
struct PackTable {
  int n;
  int64_t off[kMaxPackLayers];
  int cout[kMaxPackLayers], ct[kMaxPackLayers];
};

__global__ void k_pack_w_all(PackTable t, const float* __restrict__ params, uint16_t* w16, uint16_t* wt16) {
  const int l = blockIdx.y;
  const int64_t off = t.off[l];
  const int cout = t.cout[l], ct = t.ct[l];
  const int64_t n = (int64_t)cout * 9 * ct;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ci = (int)(i % ct);
    const int64_t r = i / ct;
    const int tap = (int)(r % 9);
    const int co = (int)(r / 9);
    const uint16_t h = f2bf(params[off + i]);
    w16[off + i] = h;
    wt16[off + ((int64_t)ci * 9 + tap) * cout + co] = h;
  }
}

__global__ void k_adam(float* p, const float* __restrict__ g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

__global__ void k_fill(float* p, int64_t n, float val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

__global__ void k_relu_grad(const float* __restrict__ g, const uint16_t* __restrict__ act, uint16_t* out, int64_t n,
                            int relu) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float v = g[i];
    out[i] = f2bf(relu ? (bf2f(act[i]) > 0.f ? v : 0.f) : v);
  }
}

__global__ void k_pack_input(const float* __restrict__ x, uint16_t* x16, int64_t pixels, int cin, int cpad) {
  const int64_t n = pixels * cpad;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ch = (int)(i % cpad);
    const int64_t p = i / cpad;
    x16[i] = ch < cin ? f2bf(x[p * cin + ch]) : (uint16_t)0;
  }
}

__global__ void k_unpack_output(const float* __restrict__ out, float* y, int64_t pixels, int cpad, int cout) {
  const int64_t n = pixels * cout;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ch = (int)(i % cout);
    y[i] = out[(i / cout) * cpad + ch];
  }
}

// Per-block sums of squared errors into part[blockIdx.x]; k_loss_sum adds the
// blocks in a fixed order, so the loss is bit-reproducible.
__global__ __launch_bounds__(kThreads) void k_mse(const float* __restrict__ out, const float* __restrict__ t,
                                                  float* gout, double* part, int64_t pixels, int cpad, int ct,
                                                  double inv_count) {
  __shared__ double red[kThreads / 64];
  double s = 0.0;
  const int64_t n = pixels * cpad;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ch = (int)(i % cpad);
    const int64_t p = i / cpad;
    float gv = 0.f;
    if (ch < ct) {
      const double d = (double)out[i] - (double)t[p * ct + ch];
      s += d * d;
      gv = (float)(2.0 * d * inv_count);
    }
    gout[i] = gv;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) b += red[w];
    part[blockIdx.x] = b;
  }
}

// *loss = inv_count * sum of part[0 .. nblocks): one wave, each lane summing a
// fixed strided subset in order, then a fixed butterfly across the lanes.
__global__ __launch_bounds__(64) void k_loss_sum(const double* __restrict__ part, int nblocks, double inv_count,
                                                 double* loss) {
  double s = 0.0;
#pragma unroll 16
  for (int i = threadIdx.x; i < nblocks; i += 64) s += part[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (threadIdx.x == 0) *loss = s * inv_count;
}

int grid_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

template <bool FWD>
hipError_t launch_gemm(const Conv& c, const Gemm& g, hipStream_t st) {
  if (g.M <= 0 || g.ncols <= 0) return hipSuccess;
  const unsigned gm = (unsigned)((g.M + 127) / 128);
  auto cols = [&](int w) { return (unsigned)((g.ncols + w - 1) / w); };
  // the widest column tile that still gives >= 1024 blocks (4 per CU): small
  // layers need the parallelism more than the operand reuse
  int tj = 8;
  while (tj > 1 && (g.ncols <= 8 * tj || (int64_t)gm * cols(16 * tj) < 1024)) tj >>= 1;
  switch (tj) {
    case 8: k_conv_gemm<FWD, 8><<<dim3(gm, cols(128)), kThreads, 0, st>>>(c, g); break;
    case 4: k_conv_gemm<FWD, 4><<<dim3(gm, cols(64)), kThreads, 0, st>>>(c, g); break;
    case 2: k_conv_gemm<FWD, 2><<<dim3(gm, cols(32)), kThreads, 0, st>>>(c, g); break;
    default: k_conv_gemm<FWD, 1><<<dim3(gm, cols(16)), kThreads, 0, st>>>(c, g); break;
  }
  return hipGetLastError();
}


// Convolutions as a spatial-tile implicit GEMM.  A block owns a box of TI
// images x TH rows x TW columns of the row grid (128 GEMM rows, four waves of
// 32) and NB = 16 TJ columns.  Per chunk of 32 reduction channels it stages in
// LDS the halo of the box, the input pixels its taps read, stored [pixel][32
// channels], and the chunk's weights of its taps, stored [tap][column][32
// channels]; tap t then reads a row's A fragment at a fixed offset (dy_t,
// dx_t) from the row's halo pixel.  The index arithmetic happens once per
// staged element instead of once per tap and K step, a staged input element
// serves every tap that sees it, and each 16-byte fragment read feeds 2 or TJ
// MFMAs.  Row pixel (ph, pw) of the box sits at halo pixel (rs ph, rs pw): rs
// is the stride of a forward convolution.
//
// Input gradients are the same product over the output gradient gy with
// B = W^T.  Stride 1: the taps mirrored (tap t reads W at tap 8 - t).  Stride
// 2: the pixels of one parity class (sy, sx) of the gradient's grid, each
// reached by 1, 2 or 4 taps at offsets 0 or 1 in gy, one launch per class, so
// no MFMA multiplies a structural zero.  A 2x-upsampled primary input: the rows
// are the 2x2 quads of the full-resolution grid, four consecutive rows per
// quad, which is exactly the four accumulator rows a lane holds; their sum is
// the half-resolution gradient.  The order of the FP32 sums differs from
// k_conv_gemm's; the products are the same.
constexpr int kMaxTaps = 9;
enum TileOut { kDirect = 0, kQuad = 1, kClass = 2 };

struct Tile {
  const uint16_t* src0;   // halo tensor, channels [0, c0)
  const uint16_t* src1;   // channels [c0, ct), full resolution (null when c0 == ct)
  int c0, ct, up;         // up: src0 is stored at half resolution
  int N, Hin, Win;        // full-resolution grid of the halo tensor
  int Ho, Wo;             // row grid
  int TI, TH, TW, tiles_w, tiles_h;
  int lh, lw;             // log2 TH, log2 TW
  int rs, org, HH, HW;    // halo pixel of row (ph, pw): (rs ph, rs pw); halo origin rs h0 + org
  float inv_hh, inv_hw;   // 1 / HH, 1 / HW: exact quotients of the (small) halo indices
  int ntaps, mirror;      // 3x3 taps: B tap t, or 8 - t when mirrored
  int tdy[kMaxTaps], tdx[kMaxTaps], tb[kMaxTaps];   // tap offsets in the halo; tap of B
  const uint16_t* b;      // B row of column j: b + (b_row0 + j) * b_ld, [9][ct]
  int b_ld, b_row0, ncols;
  int mode, sy, sx, oH, oW;   // kClass: row (y, x) is output pixel (2 y + sy, 2 x + sx) of oH x oW
  const float* bias;
  int relu;
  uint16_t* y16;
  float* y32;
  int out_ld;
  const uint16_t* act;    // input gradient with g16: g16 = bf16(y32 (act > 0)) (act_relu) or bf16(y32)
  int act_relu;
  uint16_t* g16;
  int assign;             // input gradient: y32 = the product instead of y32 += it
};

constexpr int kTileRows = 128;
// 16-byte halo items per thread: at most 384 halo pixels, or 640 for the
// halos of stride-2 forward boxes (2 TH + 1 rows of 2 TW + 1 pixels)
constexpr int kHaloItems = 6;
constexpr int kHaloItemsWide = 10;
constexpr size_t kTileLdsMax = 65536;

// NT: the taps, 9 for a 3x3 convolution (offsets t / 3, t % 3, unrolled at
// compile time), or the 1, 2 or 4 taps of a parity class (offsets from g)
template <bool FWD, int TJ, int HI, int NT>
__global__ __launch_bounds__(kThreads) void k_conv_tile(Tile g) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
  constexpr int NB = 16 * TJ;
  constexpr int BITEMS = NT * NB * 4;
  constexpr int BI = (BITEMS + kThreads - 1) / kThreads;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, kq = 8 * (lane >> 4), grp = tid & 3;
  const int HH = g.HH, HW = g.HW;
  const int halo = g.TI * HH * HW;
  uint16_t* sA = lds;
  uint16_t* sB = lds + halo * 32;
  int bt = blockIdx.x;
  const int w0 = (bt % g.tiles_w) * g.TW;
  bt /= g.tiles_w;
  const int h0 = (bt % g.tiles_h) * g.TH;
  const int n0 = (bt / g.tiles_h) * g.TI;
  const int col0 = blockIdx.y * NB;

  // box coordinates (i, ph, pw) of GEMM row `row` (TW, TH powers of two)
  auto pixel = [&](int row, int& i, int& ph, int& pw) {
    if (g.mode == kQuad) {
      const int q = row >> 2, r = row & 3;
      const int qt = q >> (g.lw - 1);
      pw = 2 * (q & ((g.TW >> 1) - 1)) + (r & 1);
      ph = 2 * (qt & ((g.TH >> 1) - 1)) + (r >> 1);
      i = qt >> (g.lh - 1);
    } else {
      const int rt = row >> g.lw;
      pw = row & (g.TW - 1);
      ph = rt & (g.TH - 1);
      i = rt >> g.lh;
    }
  };
  int abase[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    int i, ph, pw;
    pixel(wave * 32 + 16 * f + l16, i, ph, pw);
    abase[f] = ((i * HH + g.rs * ph) * HW + g.rs * pw) * 32 + kq;
  }
  // this thread's halo items: element offsets of their pixel in src0 and src1 (-1: zero padding)
  int off0[HI], off1[HI];
  {
    const int c1 = g.ct - g.c0;
    const int hs = g.up ? g.Hin >> 1 : g.Hin, ws = g.up ? g.Win >> 1 : g.Win;
    const int ih0 = g.rs * h0 + g.org, iw0 = g.rs * w0 + g.org;
#pragma unroll
    for (int k = 0; k < HI; ++k) {
      const int px = (tid + k * kThreads) >> 2;
      off0[k] = off1[k] = -1;
      if (px < halo) {
        // quotients by (px + 1/2) / HW in FP32: exact, px being far below 2^16
        const int ht = (int)(((float)px + 0.5f) * g.inv_hw), hw = px - ht * HW;
        const int i = (int)(((float)ht + 0.5f) * g.inv_hh), hh = ht - i * HH;
        const int n = n0 + i, ih = ih0 + hh, iw = iw0 + hw;
        if (n < g.N && (unsigned)ih < (unsigned)g.Hin && (unsigned)iw < (unsigned)g.Win) {
          const int y = g.up ? ih >> 1 : ih, x = g.up ? iw >> 1 : iw;
          off0[k] = ((n * hs + y) * ws + x) * g.c0;
          off1[k] = ((n * g.Hin + ih) * g.Win + iw) * c1;
        }
      }
    }
  }
  const u32x4 z = {0u, 0u, 0u, 0u};
  f32x4 acc[2][TJ];
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[f][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int nchunks = (g.ct + 31) >> 5;
  for (int c = 0; c < nchunks; ++c) {
    const int ch = 32 * c + 8 * grp;
    const bool chok = ch < g.ct;
    u32x4 hv[HI];
#pragma unroll
    for (int k = 0; k < HI; ++k) {
      hv[k] = z;
      if (chok && off0[k] >= 0) hv[k] = ch < g.c0 ? ld16(g.src0 + off0[k] + ch) : ld16(g.src1 + off1[k] + (ch - g.c0));
    }
    u32x4 bv[BI];
#pragma unroll
    for (int k = 0; k < BI; ++k) {
      const int e = tid + k * kThreads;
      const int t = e / (NB * 4), col = (e % (NB * 4)) >> 2;
      bv[k] = z;
      if (e < BITEMS && chok && col0 + col < g.ncols)
      {
        const int btap = NT == 9 ? (g.mirror ? 8 - t : t) : g.tb[t];
        bv[k] = ld16(g.b + (int64_t)(g.b_row0 + col0 + col) * g.b_ld + btap * g.ct + ch);
      }
    }
    __syncthreads();   // the previous chunk's fragment reads are done
#pragma unroll
    for (int k = 0; k < HI; ++k) {
      const int px = (tid + k * kThreads) >> 2;
      if (px < halo) *reinterpret_cast<u32x4*>(sA + px * 32 + 8 * grp) = hv[k];
    }
#pragma unroll
    for (int k = 0; k < BI; ++k) {
      const int e = tid + k * kThreads;
      if (e < BITEMS) *reinterpret_cast<u32x4*>(sB + (e >> 2) * 32 + 8 * grp) = bv[k];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int toff = NT == 9 ? ((t / 3) * HW + t % 3) * 32 : (g.tdy[t] * HW + g.tdx[t]) * 32;
      u32x4 a[2];
#pragma unroll
      for (int f = 0; f < 2; ++f) a[f] = *reinterpret_cast<const u32x4*>(sA + abase[f] + toff);
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const u32x4 b = *reinterpret_cast<const u32x4*>(sB + (t * NB + 16 * j + l16) * 32 + kq);
#pragma unroll
        for (int f = 0; f < 2; ++f)
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a[f]), as_bf(b), acc[f][j], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const int row = wave * 32 + 16 * f + 4 * (lane >> 4);
    // output offsets of the lane's 4 rows (-1: outside the grid); quad: of the quad, in [0]
    int64_t orow[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int i, ph, pw;
      pixel(row + r, i, ph, pw);
      const int n = n0 + i, oh = h0 + ph, ow = w0 + pw;
      orow[r] = -1;
      if (n < g.N && oh < g.Ho && ow < g.Wo) {
        if (g.mode == kQuad) orow[r] = ((int64_t)(n * (g.Ho >> 1) + (oh >> 1)) * (g.Wo >> 1) + (ow >> 1)) * g.out_ld;
        else if (g.mode == kClass) orow[r] = ((int64_t)(n * g.oH + 2 * oh + g.sy) * g.oW + 2 * ow + g.sx) * g.out_ld;
        else orow[r] = ((int64_t)(n * g.Ho + oh) * g.Wo + ow) * g.out_ld;
      }
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int col = col0 + 16 * j + l16;
      if (col >= g.ncols) continue;
      if (g.mode == kQuad) {   // row r = 0 is the quad's top-left pixel
        if (orow[0] >= 0) {
          const int64_t o = orow[0] + col;
          const float v = ((acc[f][j][0] + acc[f][j][1]) + acc[f][j][2]) + acc[f][j][3];
          const float y = g.assign ? v : g.y32[o] + v;
          g.y32[o] = y;
          if (g.g16) g.g16[o] = f2bf(g.act_relu ? (bf2f(g.act[o]) > 0.f ? y : 0.f) : y);
        }
        continue;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (orow[r] < 0) continue;
        const int64_t o = orow[r] + col;
        float v = acc[f][j][r];
        if constexpr (FWD) {
          v += g.bias ? g.bias[col] : 0.f;
          if (g.relu) v = v > 0.f ? v : 0.f;
          if (g.y16) g.y16[o] = f2bf(v);
          if (g.y32) g.y32[o] = v;
        } else {
          const float y = g.assign ? v : g.y32[o] + v;
          g.y32[o] = y;
          if (g.g16) g.g16[o] = f2bf(g.act_relu ? (bf2f(g.act[o]) > 0.f ? y : 0.f) : y);
        }
      }
    }
  }
}

// Box of the tile kernel for its row grid: TW and TH the powers of two
// covering the width (at most 16) and the height, TI images; halo sizes from
// the taps.  False when the halo would exceed `items` 16-byte items per thread.
bool pick_tile(Tile& t, int items = kHaloItems) {
  auto p2 = [](int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
  };
  if (t.Ho <= 0 || t.Wo <= 0 || t.ntaps <= 0) return false;
  t.TW = p2(t.Wo) < 16 ? p2(t.Wo) : 16;
  t.TH = p2(t.Ho) < kTileRows / t.TW ? p2(t.Ho) : kTileRows / t.TW;
  t.TI = kTileRows / (t.TW * t.TH);
  if (t.mode == kQuad && (t.TW < 2 || t.TH < 2 || t.Ho % 2 || t.Wo % 2)) return false;
  int my = 0, mx = 0;
  for (int k = 0; k < t.ntaps; ++k) {
    my = t.tdy[k] > my ? t.tdy[k] : my;
    mx = t.tdx[k] > mx ? t.tdx[k] : mx;
  }
  t.HH = t.rs * (t.TH - 1) + my + 1;
  t.HW = t.rs * (t.TW - 1) + mx + 1;
  if ((int64_t)t.TI * t.HH * t.HW * 4 > (int64_t)items * kThreads) return false;
  t.tiles_w = (t.Wo + t.TW - 1) / t.TW;
  t.tiles_h = (t.Ho + t.TH - 1) / t.TH;
  t.lw = 0;
  while ((1 << t.lw) < t.TW) ++t.lw;
  t.lh = 0;
  while ((1 << t.lh) < t.TH) ++t.lh;
  t.inv_hh = 1.f / (float)t.HH;
  t.inv_hw = 1.f / (float)t.HW;
  return true;
}

// the 9 taps of a 3x3 convolution, B tap t (forward) or 8 - t (mirrored)
void conv_taps(Tile& t, bool mirror) {
  t.ntaps = 9;
  t.mirror = mirror;
  for (int k = 0; k < 9; ++k) {
    t.tdy[k] = k / 3;
    t.tdx[k] = k % 3;
    t.tb[k] = mirror ? 8 - k : k;
  }
}

// Input gradient of a stride-2 convolution at the pixels of parity class
// (sy, sx): gradient pixel 2 y + sy is reached by gy row y + (sy + 1 - kh) / 2
// through the taps kh with sy + 1 - kh even (kh = 1 for sy = 0, kh = 0, 2 for
// sy = 1), likewise along x.
void class_taps(Tile& t, int sy, int sx) {
  int khs[2], dys[2], nh = 0, kws[2], dxs[2], nw = 0;
  for (int k = 0; k < 3; ++k) {
    if (((sy + 1 - k) & 1) == 0) {
      khs[nh] = k;
      dys[nh++] = (sy + 1 - k) / 2;
    }
    if (((sx + 1 - k) & 1) == 0) {
      kws[nw] = k;
      dxs[nw++] = (sx + 1 - k) / 2;
    }
  }
  t.ntaps = 0;
  for (int a = 0; a < nh; ++a)
    for (int b = 0; b < nw; ++b) {
      t.tdy[t.ntaps] = dys[a];
      t.tdx[t.ntaps] = dxs[b];
      t.tb[t.ntaps++] = 3 * khs[a] + kws[b];
    }
}

template <bool FWD>
hipError_t launch_tile(const Tile& t, hipStream_t st) {
  const int64_t tiles = (int64_t)((t.N + t.TI - 1) / t.TI) * t.tiles_h * t.tiles_w;
  if (tiles <= 0 || t.ncols <= 0) return hipSuccess;
  if (tiles >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const int halo = t.TI * t.HH * t.HW;
  auto lds_of = [&](int tj) { return (size_t)(halo * 32 + t.ntaps * 16 * tj * 32) * sizeof(uint16_t); };
  // the widest column tile that still gives >= 512 blocks and fits the LDS
  int tj = t.ncols > 32 ? 4 : (t.ncols > 16 ? 2 : 1);
  while (tj > 1 && (tiles * ((t.ncols + 16 * tj - 1) / (16 * tj)) < 512 || lds_of(tj) > kTileLdsMax)) tj >>= 1;
  if (lds_of(tj) > kTileLdsMax) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tiles, (unsigned)((t.ncols + 16 * tj - 1) / (16 * tj)));
  const size_t lds = lds_of(tj);
  const bool wide = halo * 4 > kHaloItems * kThreads;
#define VLBM_TILE(HI, NT)                                                                    \
  switch (tj) {                                                                            \
    case 4: k_conv_tile<FWD, 4, HI, NT><<<grid, kThreads, lds, st>>>(t); break;            \
    case 2: k_conv_tile<FWD, 2, HI, NT><<<grid, kThreads, lds, st>>>(t); break;            \
    default: k_conv_tile<FWD, 1, HI, NT><<<grid, kThreads, lds, st>>>(t); break;           \
  }
  if constexpr (FWD) {   // 3x3 taps; stride-2 boxes need the wide halo
    if (t.ntaps != 9) return hipErrorInvalidValue;
    if (wide) {
      VLBM_TILE(kHaloItemsWide, 9)
    } else {
      VLBM_TILE(kHaloItems, 9)
    }
  } else {               // mirrored 3x3 taps or the taps of one parity class
    if (wide) return hipErrorInvalidValue;
    switch (t.ntaps) {
      case 9: VLBM_TILE(kHaloItems, 9) break;
      case 4: VLBM_TILE(kHaloItems, 4) break;
      case 2: VLBM_TILE(kHaloItems, 2) break;
      case 1: VLBM_TILE(kHaloItems, 1) break;
      default: return hipErrorInvalidValue;
    }
  }
#undef VLBM_TILE
  return hipGetLastError();
}

}  // namespace

const char* check(const Conv& c) {
  if (c.N <= 0 || c.H <= 0 || c.W <= 0) return "batch and spatial sizes must be positive";
  if (c.cin <= 0 || c.cin % 8 || c.cskip < 0 || c.cskip % 8) return "channel counts must be multiples of 8";
  if (c.cout <= 0 || c.cout % 8) return "output channels must be a positive multiple of 8";
  if (c.stride != 1 && c.stride != 2) return "stride must be 1 or 2";
  if (c.up && (c.H % 2 || c.W % 2 || c.stride != 1)) return "upsampled inputs need even sizes and stride 1";
  if (c.OH != (c.H + c.stride - 1) / c.stride || c.OW != (c.W + c.stride - 1) / c.stride) return "bad output size";
  const int64_t cmax = c.cin > c.cskip ? (c.cin > c.cout ? c.cin : c.cout) : (c.cskip > c.cout ? c.cskip : c.cout);
  if ((int64_t)c.N * c.H * c.W * cmax >= (int64_t)1 << 31) return "tensors must hold fewer than 2^31 elements";
  return nullptr;
}

hipError_t conv_forward(const Conv& c, const uint16_t* x, const uint16_t* skip, const uint16_t* w,
                        const float* bias, uint16_t* y16, float* y32, hipStream_t st) {
  {
    Tile t{};
    t.src0 = x;
    t.src1 = skip;
    t.c0 = c.cin;
    t.ct = c.ctot();
    t.up = c.up;
    t.N = c.N;
    t.Hin = c.H;
    t.Win = c.W;
    t.Ho = c.OH;
    t.Wo = c.OW;
    t.rs = c.stride;
    t.org = -1;
    conv_taps(t, false);
    t.b = w;
    t.b_ld = 9 * c.ctot();
    t.ncols = c.cout;
    t.bias = bias;
    t.relu = c.relu;
    t.y16 = y16;
    t.y32 = y32;
    t.out_ld = c.cout;
    if (pick_tile(t, c.stride == 2 ? kHaloItemsWide : kHaloItems)) return launch_tile<true>(t, st);
  }
  Gemm g{};
  g.M = c.out_pixels();
  g.ncols = c.cout;
  g.K = 9 * c.ctot();
  g.a0 = x;
  g.a1 = skip;
  g.b = w;
  g.b_ld = g.K;
  g.bias = bias;
  g.y16 = y16;
  g.y32 = y32;
  g.out_ld = c.cout;
  return launch_gemm<true>(c, g, st);
}

hipError_t conv_backward_data(const Conv& c, const uint16_t* gy, const uint16_t* wt, float* gx, float* gskip,
                              hipStream_t st, const uint16_t* act, int act_relu, uint16_t* g16, int assign_gx,
                              int assign_gskip) {
  const int kb = 9 * c.cout;
  const int64_t gx_count = (int64_t)c.N * (c.up ? (c.H / 2) * (c.W / 2) : c.H * c.W) * c.cin;
  if (!gx) g16 = nullptr;
  // the product over gy with B = W^T, rows on the gradient's grid
  auto base = [&](float* out, int row0, int ncols, Tile& t) {
    t = Tile{};
    t.src0 = gy;
    t.c0 = t.ct = c.cout;
    t.N = c.N;
    t.Hin = c.OH;
    t.Win = c.OW;
    t.b = wt;
    t.b_ld = kb;
    t.b_row0 = row0;
    t.ncols = ncols;
    t.y32 = out;
    t.out_ld = ncols;
    t.rs = 1;
  };
  Tile t;
  if (gx && c.stride == 1) {
    base(gx, 0, c.cin, t);
    t.Ho = c.H;
    t.Wo = c.W;
    t.org = -1;
    t.mode = c.up ? kQuad : kDirect;
    t.act = act;
    t.act_relu = act_relu;
    t.g16 = g16;
    t.assign = assign_gx;
    conv_taps(t, true);
    if (pick_tile(t)) {
      hipError_t e = launch_tile<false>(t, st);
      if (e != hipSuccess) return e;
      gx = nullptr;
      g16 = nullptr;
    }
  } else if (gx) {   // stride 2 (never upsampled): one launch per parity class of the gradient's pixels
    bool ok = true, empty[4];
    Tile ts[4];
    for (int k = 0; k < 4 && ok; ++k) {
      base(gx, 0, c.cin, ts[k]);
      ts[k].mode = kClass;
      ts[k].sy = k >> 1;
      ts[k].sx = k & 1;
      ts[k].oH = c.H;
      ts[k].oW = c.W;
      ts[k].Ho = (c.H - ts[k].sy + 1) / 2;
      ts[k].Wo = (c.W - ts[k].sx + 1) / 2;
      ts[k].org = 0;
      ts[k].act = act;
      ts[k].act_relu = act_relu;
      ts[k].g16 = g16;
      ts[k].assign = assign_gx;   // the parity classes write disjoint pixels
      class_taps(ts[k], ts[k].sy, ts[k].sx);
      empty[k] = ts[k].Ho <= 0 || ts[k].Wo <= 0;
      ok = empty[k] || pick_tile(ts[k]);
    }
    if (ok) {
      for (int k = 0; k < 4; ++k) {
        if (empty[k]) continue;
        hipError_t e = launch_tile<false>(ts[k], st);
        if (e != hipSuccess) return e;
      }
      gx = nullptr;
      g16 = nullptr;
    }
  }
  if (gskip && c.cskip > 0) {
    base(gskip, c.cin, c.cskip, t);
    t.Ho = c.H;
    t.Wo = c.W;
    t.org = -1;
    t.assign = assign_gskip;
    conv_taps(t, true);
    if (pick_tile(t)) {
      hipError_t e = launch_tile<false>(t, st);
      if (e != hipSuccess) return e;
      gskip = nullptr;
    }
  }
  if (gx) {
    if (assign_gx) {
      hipError_t e = fill(gx, gx_count, 0.f, st);
      if (e != hipSuccess) return e;
    }
    Gemm g{};
    g.sub4 = c.up;
    g.rh = c.up ? c.H / 2 : c.H;
    g.rw = c.up ? c.W / 2 : c.W;
    g.M = (int64_t)c.N * g.rh * g.rw;
    g.ncols = c.cin;
    g.K = c.up ? 4 * kb : kb;
    g.a0 = gy;
    g.b = wt;
    g.b_ld = kb;
    g.b_row0 = 0;
    g.y32 = gx;
    g.out_ld = c.cin;
    hipError_t e = launch_gemm<false>(c, g, st);
    if (e != hipSuccess) return e;
    if (g16) {
      e = relu_grad(gx, act, g16, gx_count, act_relu, st);
      if (e != hipSuccess) return e;
    }
  }
  if (gskip && c.cskip > 0) {
    if (assign_gskip) {
      hipError_t e = fill(gskip, c.in_pixels() * c.cskip, 0.f, st);
      if (e != hipSuccess) return e;
    }
    Gemm g{};
    g.sub4 = 0;
    g.rh = c.H;
    g.rw = c.W;
    g.M = c.in_pixels();
    g.ncols = c.cskip;
    g.K = kb;
    g.a0 = gy;
    g.b = wt;
    g.b_ld = kb;
    g.b_row0 = c.cin;
    g.y32 = gskip;
    g.out_ld = c.cskip;
    return launch_gemm<false>(c, g, st);
  }
  return hipSuccess;
}

namespace {
// Launch shape of k_wgrad_tile.  The number of slices is at most
// wgrad_max_slices(c), which does not depend on the batch size.
constexpr int kWgradBlocks = 512;
struct WgradShape {
  int cf, rs, cotiles, chunks;
  int64_t cap;
};
WgradShape wgrad_shape(const Conv& c) {
  WgradShape w;
  w.cf = c.cout > 32 ? 4 : (c.cout > 16 ? 2 : 1);
  w.rs = c.stride;
  w.cotiles = (c.cout + 16 * w.cf - 1) / (16 * w.cf);
  w.chunks = (c.ctot() + 31) / 32;
  const int64_t per = (int64_t)w.cotiles * w.chunks;
  w.cap = kWgradBlocks / per > 1 ? kWgradBlocks / per : 1;
  return w;
}
}  // namespace

// Slices summed per thread in each level of the ordered reduction.
constexpr int kSliceGroup = 32;

// Workspace floats for `slices` slices of m elements: the slices, then the
// group sums of the levels needed to bring them down to kSliceGroup.
int64_t reduce_workspace(int64_t slices, int64_t m) {
  int64_t total = slices * m;
  for (int64_t s = slices; s > kSliceGroup; s = (s + kSliceGroup - 1) / kSliceGroup)
    total += (s + kSliceGroup - 1) / kSliceGroup * m;
  return total;
}

int64_t conv_backward_weight_workspace(const Conv& c) {
  return reduce_workspace(wgrad_shape(c).cap, (int64_t)c.cout * (9 * c.ctot() + 1));
}

hipError_t conv_backward_weight(const Conv& c, const uint16_t* x, const uint16_t* skip, const uint16_t* gy,
                                float* gw, float* gb, hipStream_t st, float* work, int64_t work_floats, int assign) {
  const WgradShape w = wgrad_shape(c);
  WgradTile t{};
  t.x = x;
  t.skip = skip;
  t.gy = gy;
  t.N = c.N;
  t.H = c.H;
  t.W = c.W;
  t.cin = c.cin;
  t.ct = c.ctot();
  t.up = c.up;
  t.OH = c.OH;
  t.OW = c.OW;
  t.cout = c.cout;
  const int ph = 4, pw = w.rs == 1 ? 8 : 4;
  t.tiles_w = (c.OW + pw - 1) / pw;
  t.tiles_h = (c.OH + ph - 1) / ph;
  const int64_t units = (int64_t)((c.N + 7) / 8) * t.tiles_h * t.tiles_w;
  if (units <= 0) return hipSuccess;
  if (units >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  t.units = (int)units;
  t.per_block = (int)((units + w.cap - 1) / w.cap);
  const int64_t splits = (units + t.per_block - 1) / t.per_block;
  const int64_t n = (int64_t)c.cout * 9 * t.ct, m = n + c.cout;
  const bool ordered = work && work_floats >= reduce_workspace(splits, m);
  t.part = ordered ? work : nullptr;
  if (assign && !ordered) {   // the atomic path adds
    hipError_t e = fill(gw, n, 0.f, st);
    if (e == hipSuccess) e = fill(gb, c.cout, 0.f, st);
    if (e != hipSuccess) return e;
  }
  t.slice = m;
  t.gw = gw;
  t.gb = gb;
  const dim3 grid((unsigned)splits, (unsigned)w.chunks, (unsigned)w.cotiles);
#define VLBM_WGRAD(CF)                                                                        \
  if (w.rs == 1) k_wgrad_tile<CF, 1><<<grid, kThreads, 0, st>>>(t);                          \
  else k_wgrad_tile<CF, 2><<<grid, kThreads, 0, st>>>(t);
  switch (w.cf) {
    case 4: VLBM_WGRAD(4) break;
    case 2: VLBM_WGRAD(2) break;
    default: VLBM_WGRAD(1) break;
  }
#undef VLBM_WGRAD
  if (ordered) {
    // groups of kSliceGroup consecutive slices, level by level, then the sum
    // of the remaining slices into gw and gb: a fixed order at every level
    float* src = work;
    int64_t slices = splits;
    while (slices > kSliceGroup) {
      float* dst = src + slices * m;
      const int64_t groups = (slices + kSliceGroup - 1) / kSliceGroup;
      k_sum_slices<<<grid_for(groups * m), kThreads, 0, st>>>(src, dst, m, (int)slices, kSliceGroup);
      src = dst;
      slices = groups;
    }
    k_wgrad_reduce<<<grid_for(m), kThreads, 0, st>>>(src, gw, gb, n, m, (int)slices, assign);
  }
  return hipGetLastError();
}

hipError_t pack_weights(const Conv& c, const float* w, uint16_t* w16, uint16_t* wt16, hipStream_t st) {
  k_pack_w<<<grid_for((int64_t)c.cout * 9 * c.ctot()), kThreads, 0, st>>>(c, w, w16, wt16);
  return hipGetLastError();
}

hipError_t pack_weights_all(int nlayers, const Conv* convs, const int64_t* w_off, const float* params, uint16_t* w16,
                            uint16_t* wt16, hipStream_t st) {
  if (nlayers <= 0) return hipSuccess;
  if (nlayers > kMaxPackLayers) return hipErrorInvalidValue;
  PackTable t{};
  t.n = nlayers;
  int64_t most = 0;
  for (int l = 0; l < nlayers; ++l) {
    t.off[l] = w_off[l];
    t.cout[l] = convs[l].cout;
    t.ct[l] = convs[l].ctot();
    const int64_t n = (int64_t)t.cout[l] * 9 * t.ct[l];
    most = n > most ? n : most;
  }
  const int64_t bx = (most + kThreads - 1) / kThreads;
  k_pack_w_all<<<dim3((unsigned)(bx < 1024 ? bx : 1024), (unsigned)nlayers), kThreads, 0, st>>>(t, params, w16, wt16);
  return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t st) {
  k_adam<<<grid_for(n), kThreads, 0, st>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t fill(float* p, int64_t n, float v, hipStream_t st) {
  k_fill<<<grid_for(n), kThreads, 0, st>>>(p, n, v);
  return hipGetLastError();
}

hipError_t relu_grad(const float* g, const uint16_t* act, uint16_t* out16, int64_t n, int relu, hipStream_t st) {
  k_relu_grad<<<grid_for(n), kThreads, 0, st>>>(g, act, out16, n, relu);
  return hipGetLastError();
}

hipError_t pack_input(const float* x, uint16_t* x16, int64_t pixels, int cin, int cpad, hipStream_t st) {
  k_pack_input<<<grid_for(pixels * cpad), kThreads, 0, st>>>(x, x16, pixels, cin, cpad);
  return hipGetLastError();
}

hipError_t unpack_output(const float* out, float* y, int64_t pixels, int cpad, int cout, hipStream_t st) {
  k_unpack_output<<<grid_for(pixels * cout), kThreads, 0, st>>>(out, y, pixels, cpad, cout);
  return hipGetLastError();
}

hipError_t mse(const float* out, const float* t, float* gout, double* loss, int64_t pixels, int cpad, int ct,
               double* part, hipStream_t st) {
  const double inv = 1.0 / ((double)pixels * ct);
  const int nb = grid_for(pixels * cpad);
  if (nb > kMseBlocks) return hipErrorInvalidValue;   // grid_for caps at 4096 blocks
  k_mse<<<nb, kThreads, 0, st>>>(out, t, gout, part, pixels, cpad, ct, inv);
  k_loss_sum<<<1, 64, 0, st>>>(part, nb, inv, loss);
  return hipGetLastError();
}

}  // namespace nn
}  // namespace vlbm

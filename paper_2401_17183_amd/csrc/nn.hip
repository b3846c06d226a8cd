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

// Weight gradient: gw[co][k] += sum_m gy[m][co] A(m, k), gb[co] += sum_m gy[m][co].
// A 64 (co) x 64 (k) tile per block; 32 output pixels per step are staged in LDS
// transposed (pixel index fastest) so that each MFMA operand fragment is one
// 16-byte LDS read; blocks split the pixel range (blockIdx.z).  With a
// workspace, each split stores its partial tile in slice z of part (weights at
// [co][k], then the bias at [C_out * K + co]) and the slices are summed in a
// fixed order (k_sum_slices, k_wgrad_reduce), so the result does not depend on
// scheduling; without one, the splits add their tiles with FP32 atomics.
constexpr int kLd = 40;   // LDS row length in 16-bit words (80 B, keeps 16 B alignment)

__global__ __launch_bounds__(kThreads) void k_wgrad(Conv c, const uint16_t* __restrict__ x,
                                                    const uint16_t* __restrict__ skip,
                                                    const uint16_t* __restrict__ gy, float* gw, float* gb,
                                                    int chunks_per_block, float* part) {
  __shared__ __attribute__((aligned(16))) uint16_t sG[64 * kLd];
  __shared__ __attribute__((aligned(16))) uint16_t sA[64 * kLd];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int ct = c.ctot();
  const int K = 9 * ct;
  const int k0 = blockIdx.x * 64, co0 = blockIdx.y * 64;
  const int64_t M = c.out_pixels();
  const int64_t chunk0 = (int64_t)blockIdx.z * chunks_per_block;
  const int ml = t & 31, grp = t >> 5;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, kq = 8 * (lane >> 4);
  const u32x4 z = {0u, 0u, 0u, 0u};
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  const int co = co0 + 8 * grp;
  const int k = k0 + 8 * grp;
  const int tap = k / ct, ch = k - tap * ct;
  const int kh = tap / 3, kw = tap - 3 * kh;
  for (int cc = 0; cc < chunks_per_block; ++cc) {
    const int64_t m = (chunk0 + cc) * 32 + ml;
    const u32x4 gv = (m < M && co < c.cout) ? ld16(gy + m * c.cout + co) : z;
    const RowF r = row_fwd(c, m, M);
    const u32x4 av = gather_fwd(c, x, skip, r, kh, kw, ch, k < K);
    __syncthreads();   // the previous step's fragment reads are done
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sG[(8 * grp + 2 * j) * kLd + ml] = (uint16_t)(gv[j] & 0xffffu);
      sG[(8 * grp + 2 * j + 1) * kLd + ml] = (uint16_t)(gv[j] >> 16);
      sA[(8 * grp + 2 * j) * kLd + ml] = (uint16_t)(av[j] & 0xffffu);
      sA[(8 * grp + 2 * j + 1) * kLd + ml] = (uint16_t)(av[j] >> 16);
    }
    __syncthreads();
    if (blockIdx.x == 0 && t < 64) {
#pragma unroll 8
      for (int q = 0; q < 32; ++q) bsum += bf2f(sG[t * kLd + q]);
    }
    u32x4 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const u32x4*>(&sG[(wm * 32 + 16 * i + l16) * kLd + kq]);
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const u32x4*>(&sA[(wn * 32 + 16 * j + l16) * kLd + kq]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a[i]), as_bf(b[j]), acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int kk = k0 + wn * 32 + 16 * j + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = co0 + wm * 32 + 16 * i + 4 * (lane >> 4) + r;
        if (o < c.cout && kk < K) {
          if (part) part[(int64_t)blockIdx.z * ((int64_t)c.cout * (K + 1)) + (int64_t)o * K + kk] = acc[i][j][r];
          else unsafeAtomicAdd(&gw[(int64_t)o * K + kk], acc[i][j][r]);
        }
      }
    }
  if (blockIdx.x == 0 && t < 64 && co0 + t < c.cout) {
    if (part) part[(int64_t)blockIdx.z * ((int64_t)c.cout * (K + 1)) + (int64_t)c.cout * K + co0 + t] = bsum;
    else unsafeAtomicAdd(&gb[co0 + t], bsum);
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
    for (int z = g * G; z < z1; ++z) acc += src[z * m + e];
    dst[i] = acc;
  }
}

// gw[e] += sum over z of part[z][e] (e < n), gb[e - n] likewise (n <= e < m),
// in slice order.
__global__ void k_wgrad_reduce(const float* __restrict__ part, float* gw, float* gb, int64_t n, int64_t m,
                               int slices) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int z = 0; z < slices; ++z) acc += part[z * m + e];
    if (e < n) gw[e] += acc;
    else gb[e - n] += acc;
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
                              hipStream_t st) {
  const int kb = 9 * c.cout;
  if (gx) {
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
  }
  if (gskip && c.cskip > 0) {
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
// Launch shape of k_wgrad: pixel chunks per block and the number of splits.
// splits <= want for every batch size (it depends on the tile counts only).
struct WgradShape {
  int K, kt, ctl;
  int64_t want, cpb, splits;
};
WgradShape wgrad_shape(const Conv& c) {
  WgradShape w;
  w.K = 9 * c.ctot();
  w.kt = (w.K + 63) / 64;
  w.ctl = (c.cout + 63) / 64;
  const int64_t chunks = (c.out_pixels() + 31) / 32;
  w.want = (2048 + (int64_t)w.kt * w.ctl - 1) / ((int64_t)w.kt * w.ctl);
  const int64_t s = w.want < chunks ? (w.want > 0 ? w.want : 1) : chunks;
  w.cpb = (chunks + s - 1) / s;
  w.splits = (chunks + w.cpb - 1) / w.cpb;
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
  const WgradShape w = wgrad_shape(c);
  return reduce_workspace(w.want > 0 ? w.want : 1, (int64_t)c.cout * (w.K + 1));
}

hipError_t conv_backward_weight(const Conv& c, const uint16_t* x, const uint16_t* skip, const uint16_t* gy,
                                float* gw, float* gb, hipStream_t st, float* work, int64_t work_floats) {
  const WgradShape w = wgrad_shape(c);
  const int64_t n = (int64_t)c.cout * w.K, m = n + c.cout;
  const bool ordered = work && work_floats >= reduce_workspace(w.splits, m);
  dim3 grid((unsigned)w.kt, (unsigned)w.ctl, (unsigned)w.splits);
  k_wgrad<<<grid, kThreads, 0, st>>>(c, x, skip, gy, gw, gb, (int)w.cpb, ordered ? work : nullptr);
  if (ordered) {
    // groups of kSliceGroup consecutive slices, level by level, then the sum
    // of the remaining slices into gw and gb: a fixed order at every level
    float* src = work;
    int64_t slices = w.splits;
    while (slices > kSliceGroup) {
      float* dst = src + slices * m;
      const int64_t groups = (slices + kSliceGroup - 1) / kSliceGroup;
      k_sum_slices<<<grid_for(groups * m), kThreads, 0, st>>>(src, dst, m, (int)slices, kSliceGroup);
      src = dst;
      slices = groups;
    }
    k_wgrad_reduce<<<grid_for(m), kThreads, 0, st>>>(src, gw, gb, n, m, (int)slices);
  }
  return hipGetLastError();
}

hipError_t pack_weights(const Conv& c, const float* w, uint16_t* w16, uint16_t* wt16, hipStream_t st) {
  k_pack_w<<<grid_for((int64_t)c.cout * 9 * c.ctot()), kThreads, 0, st>>>(c, w, w16, wt16);
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

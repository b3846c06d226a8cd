// STREAM-style HBM kernels (read-only, write-only, copy) that measure the
// bandwidth a plain streaming kernel achieves on this device: the practical
// ceiling the step kernel's achieved bandwidth is compared with.  Each kernel
// walks 16-byte elements in a grid-stride loop with four independent accesses
// in flight per lane; the non-temporal variants use streaming loads and
// stores.  Several grid sizes are tried and the best is reported.
#include <algorithm>

#include "common.hpp"

namespace vlbm {
int set_error(int code, const char* fmt, ...);
}

namespace {

using vlbm::set_error;

constexpr int kThreads = 256;

// 16-byte element as a native vector type (what the non-temporal builtins take)
typedef float v4f __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ v4f ld(const v4f* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ void st(v4f* p, v4f v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Read-only: the lane sums are written only when `sink` is set (never, at run
// time), which keeps the loads alive.
template <bool NT>
__global__ __launch_bounds__(kThreads) void k_read(const v4f* __restrict__ a, size_t n, int sink,
                                                   float* __restrict__ out) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  v4f s0 = {0.f, 0.f, 0.f, 0.f}, s1 = s0, s2 = s0, s3 = s0;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const v4f x0 = ld<NT>(a + i), x1 = ld<NT>(a + i + stride), x2 = ld<NT>(a + i + 2 * stride),
                 x3 = ld<NT>(a + i + 3 * stride);
    s0 += x0;
    s1 += x1;
    s2 += x2;
    s3 += x3;
  }
  for (; i < n; i += stride) {
    s0 += ld<NT>(a + i);
  }
  if (sink) out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s0.x + s1.y + s2.z + s3.w;
}

template <bool NT>
__global__ __launch_bounds__(kThreads) void k_write(v4f* __restrict__ b, size_t n, float v) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const v4f x = {v, v, v, v};
  for (; i + 3 * stride < n; i += 4 * stride) {
    st<NT>(b + i, x);
    st<NT>(b + i + stride, x);
    st<NT>(b + i + 2 * stride, x);
    st<NT>(b + i + 3 * stride, x);
  }
  for (; i < n; i += stride) st<NT>(b + i, x);
}

template <bool NT>
__global__ __launch_bounds__(kThreads) void k_copy(const v4f* __restrict__ a, v4f* __restrict__ b, size_t n) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const v4f x0 = ld<NT>(a + i), x1 = ld<NT>(a + i + stride), x2 = ld<NT>(a + i + 2 * stride),
                 x3 = ld<NT>(a + i + 3 * stride);
    st<NT>(b + i, x0);
    st<NT>(b + i + stride, x1);
    st<NT>(b + i + 2 * stride, x2);
    st<NT>(b + i + 3 * stride, x3);
  }
  for (; i < n; i += stride) st<NT>(b + i, ld<NT>(a + i));
}

template <bool NT>
hipError_t launch(int kind, int grid, const v4f* a, v4f* b, size_t n, float* sink_out, hipStream_t s) {
  if (kind == 0) k_read<NT><<<grid, kThreads, 0, s>>>(a, n, 0, sink_out);
  else if (kind == 1) k_write<NT><<<grid, kThreads, 0, s>>>(b, n, 1.0f);
  else k_copy<NT><<<grid, kThreads, 0, s>>>(a, b, n);
  return hipGetLastError();
}

}  // namespace

extern "C" int vlbm_membench(int kind, int nontemporal, size_t bytes, int reps, void* stream, double* gbps,
                             int* best_grid) {
  if (kind < 0 || kind > 2 || reps <= 0 || !gbps || bytes < (1u << 20))
    return set_error(VLBM_ERR_ARG, "vlbm_membench: kind 0..2, reps > 0, bytes >= 1 MiB, gbps not null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t n = bytes / sizeof(v4f);
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  v4f *a = nullptr, *b = nullptr;
  float* sink = nullptr;
  // grid-stride launches of 4..32 blocks per CU, and (write, copy) one
  // element per lane; the read kernel's (never written) sink covers its grids
  const int grids[5] = {cus * 4, cus * 8, cus * 16, cus * 32, (int)std::min<size_t>((n + kThreads - 1) / kThreads, 1u << 30)};
  const int ngrids = kind == 0 ? 4 : 5;
  const size_t sink_elems = (size_t)cus * 32 * kThreads;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = VLBM_OK;
  auto bail = [&](int code, const char* what, hipError_t e) {
    rc = set_error(code, "vlbm_membench: %s: %s", what, hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipMalloc((void**)&a, n * sizeof(v4f))) != hipSuccess) bail(VLBM_ERR_NOMEM, "allocation", e);
  else if ((e = hipMalloc((void**)&b, n * sizeof(v4f))) != hipSuccess) bail(VLBM_ERR_NOMEM, "allocation", e);
  else if ((e = hipMalloc((void**)&sink, sink_elems * sizeof(float))) != hipSuccess) bail(VLBM_ERR_NOMEM, "allocation", e);
  else if ((e = hipMemsetAsync(a, 0, n * sizeof(v4f), s)) != hipSuccess) bail(VLBM_ERR_DEVICE, "fill", e);
  else if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    bail(VLBM_ERR_DEVICE, "events", e);
  double best = 0.0;
  int bg = 0;
  const double moved = (kind == 2 ? 2.0 : 1.0) * (double)(n * sizeof(v4f));
  for (int gi = 0; gi < ngrids && rc == VLBM_OK; ++gi) {
    const int g = grids[gi];
    auto run = [&]() { return nontemporal ? launch<true>(kind, g, a, b, n, sink, s) : launch<false>(kind, g, a, b, n, sink, s); };
    if ((e = run()) != hipSuccess) { bail(VLBM_ERR_DEVICE, "warm-up launch", e); break; }
    if ((e = hipEventRecord(e0, s)) != hipSuccess) { bail(VLBM_ERR_DEVICE, "event", e); break; }
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = run();
    if (e != hipSuccess) { bail(VLBM_ERR_DEVICE, "launch", e); break; }
    float ms = 0.f;
    if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
        (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
      bail(VLBM_ERR_DEVICE, "timing", e);
      break;
    }
    const double gb = moved * reps / (ms * 1e-3) / 1e9;
    if (gb > best) {
      best = gb;
      bg = g;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (sink) (void)hipFree(sink);
  if (rc) return rc;
  *gbps = best;
  if (best_grid) *best_grid = bg;
  set_error(VLBM_OK, "%s", "");
  return VLBM_OK;
}

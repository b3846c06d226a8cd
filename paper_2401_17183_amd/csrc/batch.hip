// Batched time stepping of many independent meshes: one launch advances every
// member mesh by one step.  The work list is a table of (mesh, first cell)
// tiles of BLOCK cells over all members, largest meshes first; a persistent
// grid of blocks strides over it.  The kernel boundary is the only barrier
// between steps (no cross-workgroup waiting), and n steps replay a captured
// hipGraph of such launches.  The launch shape (BLOCK, blocks per CU) is
// chosen by a small measured search, cached in a text file.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "batch.hpp"
#include "stepcore.hpp"

namespace vlbm {

namespace {

// FF = 0 when no member has far-field links, else 2 (per-member run-time test).
// GEN: some member uses a general collision matrix; members stepped with
// the BGK matrix then take the same arithmetic with tau_g = tau (c1 = 0).
// With one block per tile the tile order is regrouped (xcd_grouped) so that
// consecutive tiles (which share halo rows) run on one XCD and its L2.

template <class L, class P, class S, class T, int BLOCK, int FF, bool GEN>
__global__ __launch_bounds__(BLOCK) VLBM_STEP_ATTR void k_batch(const StepArgs<P, S, T>* __restrict__ args,
                                                                const Tile* __restrict__ tiles, int ntiles,
                                                                int parity) {
  const int first = (int)gridDim.x == ntiles ? xcd_grouped(blockIdx.x, ntiles) : (int)blockIdx.x;
  for (int t = first; t < ntiles; t += gridDim.x) {
    const Tile tl = tiles[t];
    const StepArgs<P, S, T> a = args[2 * tl.mesh + parity];
    step_cell<L, P, S, T, BLOCK, FF, GEN>(a, tl.first + threadIdx.x);
  }
}

// Re-basing of every active member's references (rebase_cell, as for a single
// mesh), over the same tile table; args of the parity whose input buffer holds
// the state just written.
template <class L, class P, class S, class T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batch_rebase(const StepArgs<P, S, T>* __restrict__ args,
                                                        const Tile* __restrict__ tiles, int ntiles, int parity) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile tl = tiles[t];
    const StepArgs<P, S, T> a = args[2 * tl.mesh + parity];
    const int cell = tl.first + threadIdx.x;
    if (cell < a.box.ncells)
      rebase_cell<L, P>(const_cast<PopE<P>*>(a.in), const_cast<PopR<P>*>(a.rown), a.box.ncells, cell, a.scale,
                        a.inv_scale);
  }
}

__global__ void k_gather(const double* const* __restrict__ src, double* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = *src[i];
}

}  // namespace

namespace {

template <class P, class S, class T>
hipError_t upload_args(BatchObj* b) {
  std::vector<StepArgs<P, S, T>> h(2 * b->members.size());
  for (size_t m = 0; m < b->members.size(); ++m) {
    SimObj* s = b->members[m];
    const int buf = s->buf;
    for (int par = 0; par < 2; ++par) {
      s->buf = par;
      h[2 * m + par] = make_step_args<P, S, T>(s);
    }
    s->buf = buf;
  }
  if (!b->d_args) {
    hipError_t e = hipMalloc(&b->d_args, sizeof(StepArgs<P, S, T>) * h.size());
    if (e != hipSuccess) return e;
  }
  return hipMemcpy(b->d_args, h.data(), sizeof(StepArgs<P, S, T>) * h.size(), hipMemcpyHostToDevice);
}

hipError_t build_tiles(BatchObj* b) {
  std::vector<int> order;
  for (size_t i = 0; i < b->members.size(); ++i)
    if (b->active.empty() || b->active[i]) order.push_back((int)i);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return b->members[x]->mesh->box.ncells > b->members[y]->mesh->box.ncells;
  });
  std::vector<Tile> tiles;
  for (int m : order) {
    const int nc = b->members[m]->mesh->box.ncells;
    for (int c = 0; c < nc; c += b->block) tiles.push_back(Tile{m, c});
  }
  b->ntiles = (int)tiles.size();
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  b->d_tiles = nullptr;
  if (tiles.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)&b->d_tiles, sizeof(Tile) * tiles.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(b->d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice);
}

template <class L, class P, class S, class T, int BLOCK>
hipError_t launch_batch_typed(BatchObj* b, int parity) {
  const int grid = b->grid_per_cu > 0 ? std::min(b->ntiles, b->grid_per_cu * b->cus) : b->ntiles;
  const StepArgs<P, S, T>* args = static_cast<const StepArgs<P, S, T>*>(b->d_args);
  if (b->any_general)
    k_batch<L, P, S, T, BLOCK, 2, true><<<grid, BLOCK, 0, b->stream>>>(args, b->d_tiles, b->ntiles, parity);
  else if (b->any_ff)
    k_batch<L, P, S, T, BLOCK, 2, false><<<grid, BLOCK, 0, b->stream>>>(args, b->d_tiles, b->ntiles, parity);
  else
    k_batch<L, P, S, T, BLOCK, 0, false><<<grid, BLOCK, 0, b->stream>>>(args, b->d_tiles, b->ntiles, parity);
  return hipGetLastError();
}

template <class L, class P, class S, class T, int BLOCK>
hipError_t launch_rebase_typed(BatchObj* b, int parity) {
  if constexpr (!PopCodec<P>::shifted) {
    return hipSuccess;
  } else {
    const int grid = b->grid_per_cu > 0 ? std::min(b->ntiles, b->grid_per_cu * b->cus) : b->ntiles;
    const StepArgs<P, S, T>* args = static_cast<const StepArgs<P, S, T>*>(b->d_args);
    k_batch_rebase<L, P, S, T, BLOCK><<<grid, BLOCK, 0, b->stream>>>(args, b->d_tiles, b->ntiles, parity);
    return hipGetLastError();
  }
}

// what: 0 = step with the given parity, 1 = re-base the buffer of that parity
template <class L, class P, class S, class T>
hipError_t launch_batch_block(BatchObj* b, int parity, int what) {
  switch (b->block) {
    case 64: return what ? launch_rebase_typed<L, P, S, T, 64>(b, parity) : launch_batch_typed<L, P, S, T, 64>(b, parity);
    case 128:
      return what ? launch_rebase_typed<L, P, S, T, 128>(b, parity) : launch_batch_typed<L, P, S, T, 128>(b, parity);
    default:
      return what ? launch_rebase_typed<L, P, S, T, 256>(b, parity) : launch_batch_typed<L, P, S, T, 256>(b, parity);
  }
}

template <class L>
hipError_t launch_batch_lattice(BatchObj* b, int parity, int what) {
  switch (b->precision) {
    case VLBM_FP64: return launch_batch_block<L, double, double, double>(b, parity, what);
    case VLBM_FP32: return launch_batch_block<L, F32Dev, float, double>(b, parity, what);
    default: return launch_batch_block<L, float, float, float>(b, parity, what);
  }
}

template <class L>
hipError_t upload_lattice(BatchObj* b) {
  switch (b->precision) {
    case VLBM_FP64: return upload_args<double, double, double>(b);
    case VLBM_FP32: return upload_args<F32Dev, float, double>(b);
    default: return upload_args<float, float, float>(b);
  }
}

}  // namespace

hipError_t batch_launch(BatchObj* b, int parity) {
  if (b->ntiles == 0) return hipSuccess;   // no active member
  return b->lattice == VLBM_D2Q9 ? launch_batch_lattice<D2Q9>(b, parity, 0) : launch_batch_lattice<D3Q19>(b, parity, 0);
}

hipError_t batch_rebase(BatchObj* b, int parity) {
  if (b->ntiles == 0 || b->rebase <= 0) return hipSuccess;
  return b->lattice == VLBM_D2Q9 ? launch_batch_lattice<D2Q9>(b, parity, 1) : launch_batch_lattice<D3Q19>(b, parity, 1);
}

hipError_t batch_upload(BatchObj* b) {
  hipError_t e = b->lattice == VLBM_D2Q9 ? upload_lattice<D2Q9>(b) : upload_lattice<D3Q19>(b);
  if (e != hipSuccess) return e;
  return build_tiles(b);
}

hipError_t batch_gather(BatchObj* b, const double* const* src, double* dst, int n) {
  if (n <= 0) return hipSuccess;
  k_gather<<<(n + 255) / 256, 256, 0, b->stream>>>(src, dst, n);
  return hipGetLastError();
}

void batch_drop_graphs(BatchObj* b) {
  for (int p = 0; p < 2; ++p)
    if (b->exec[p]) {
      (void)hipGraphExecDestroy(b->exec[p]);
      b->exec[p] = nullptr;
    }
}

// Capture graph_steps consecutive steps (parities alternate) starting at parity p,
// at a step count that is a multiple of the re-basing period (graph_steps is
// one too): the references are re-based after the steps that reach a multiple
// of it, as for a single mesh.
hipError_t batch_capture(BatchObj* b, int p, bool per_member) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t le = hipSuccess;
  for (int k = 0; k < b->graph_steps && le == hipSuccess; ++k) {
    const int par = (p + k) & 1;
    if (!per_member) {
      le = batch_launch(b, par);
    } else {
      for (size_t m = 0; m < b->members.size(); ++m) {
        if (!b->active[m]) continue;
        SimObj* s = b->members[m];
        const int keep = s->buf;
        s->buf = par;
        le = launch_step(s);
        s->buf = keep;
        if (le != hipSuccess) break;
      }
    }
    if (le == hipSuccess && b->rebase > 0 && (k + 1) % b->rebase == 0) le = batch_rebase(b, par ^ 1);
  }
  e = hipStreamEndCapture(b->stream, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return le;
  }
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(&b->exec[p], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

}  // namespace vlbm

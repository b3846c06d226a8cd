// Host-side batch object shared by batch.hip and the C API.
#pragma once

#include <vector>

#include "common.hpp"

namespace vlbm {

struct Tile {
  int mesh;
  int first;
};

struct BatchObj {
  std::vector<SimObj*> members;
  std::vector<char> active;          // per member: stepped by vlbm_batch_step (all by default)
  int lattice = 0, precision = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* d_args = nullptr;      // StepArgs [count][2 parities]
  Tile* d_tiles = nullptr;
  int ntiles = 0;
  int block = 256, grid_per_cu = 4, cus = 256;
  int mode = 0;                // VLBM_BATCH_*
  hipGraphExec_t exec[2] = {nullptr, nullptr};   // per starting parity
  int graph_steps = 32;         // steps per captured graph: even, and a multiple of rebase
  int rebase = 0;               // shifted storage: re-basing period of the references (0: none)
  int64_t t = 0;
  int64_t total_cells = 0;
  bool any_ff = false;               // some member has far-field links
  bool any_general = false;          // some member uses a general collision matrix
  const double** d_rsrc = nullptr;   // per member: address of its latest audit's residual
  double* d_resid = nullptr;         // gathered residuals [count]
};

hipError_t batch_launch(BatchObj* b, int parity);
// shifted storage: re-base every active member's buffer of parity `parity`
hipError_t batch_rebase(BatchObj* b, int parity);
hipError_t batch_upload(BatchObj* b);
hipError_t batch_capture(BatchObj* b, int p, bool per_member);
void batch_drop_graphs(BatchObj* b);
// dst[i] = *src[i] for i < n, on the batch stream
hipError_t batch_gather(BatchObj* b, const double* const* src, double* dst, int n);

}  // namespace vlbm

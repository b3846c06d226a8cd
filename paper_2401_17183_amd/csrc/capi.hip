// Host side of the C ABI declared in include/vlbm.h: handle objects, argument
// validation, error strings, the launch sequence of each call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "common.hpp"

namespace vlbm {
int audit_partial_blocks(const MeshObj* m);
int audit_words();
}  // namespace vlbm

#include "batch.hpp"

#include <string>
#include <utility>
#include <vector>

using namespace vlbm;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int ok() {
  g_err[0] = 0;
  return VLBM_OK;
}

}  // namespace

namespace vlbm {
// Error reporting shared with the other translation units of the C ABI:
// records the message in the thread-local error string and returns `code`.
int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}
}  // namespace vlbm

namespace {

#define HIP_TRY(expr)                                                                          \
  do {                                                                                          \
    hipError_t _e = (expr);                                                                     \
    if (_e != hipSuccess) return fail(VLBM_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

template <class T> int dev_alloc(T** p, size_t bytes) {
  if (hipMalloc((void**)p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(VLBM_ERR_NOMEM, "device allocation of %zu bytes failed", bytes);
  }
  return VLBM_OK;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

size_t storage_bytes(int precision) { return pop_elem(precision); }
size_t geometry_bytes(int precision) { return precision == VLBM_FP64 ? 8 : 4; }

constexpr uint64_t kMagic = 0x314d42564c4d4956ull;  // checkpoint tag

struct CkptHeader {
  uint64_t magic;
  int32_t lattice, precision;
  int64_t ncells, Q, t;
  int64_t bytes;
};

// Event pairs recorded around kernel launches while a sim's timing is on:
// kind 0 = step, 1 = re-basing, 2 = g_i of the next node positions (moving
// steps).  Events are reused across reads.
constexpr int kTimingKinds = 3;
struct EventPool {
  std::vector<hipEvent_t> ev;      // 2 per recorded launch
  std::vector<int> kind;
  size_t used = 0;                 // launches recorded since the last read
  ~EventPool() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  hipError_t begin(hipStream_t s, int k) {
    if (2 * used + 2 > ev.size()) {
      for (int i = 0; i < 2; ++i) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        ev.push_back(e);
      }
      kind.push_back(k);
    }
    kind[used] = k;
    return hipEventRecord(ev[2 * used], s);
  }
  hipError_t end(hipStream_t s) { return hipEventRecord(ev[2 * used++ + 1], s); }
};

}  // namespace

extern "C" {

const char* vlbm_last_error(void) { return g_err; }

extern "C++" {
template <class L>
static void lattice_table(int32_t* Q, int32_t* d, int32_t* c, double* w) {
  *Q = L::Q;
  *d = L::D;
  for (int a = 0; a < L::Q; ++a) {
    for (int i = 0; i < L::D; ++i)
      if (c) c[a * L::D + i] = L::c(a, i);
    if (w) w[a] = L::w(a);
  }
}
}

int vlbm_lattice_info(int lattice, int32_t* Q, int32_t* d, int32_t* c, double* w) {
  if (!Q || !d) return fail(VLBM_ERR_ARG, "vlbm_lattice_info: null output");
  switch (lattice) {
    case VLBM_D2Q9: lattice_table<D2Q9>(Q, d, c, w); break;
    case VLBM_D3Q19: lattice_table<D3Q19>(Q, d, c, w); break;
    case VLBM_D2Q21: lattice_table<D2Q21>(Q, d, c, w); break;
    case VLBM_D3Q39: lattice_table<D3Q39>(Q, d, c, w); break;
    default: return fail(VLBM_ERR_ARG, "unknown lattice %d", lattice);
  }
  return ok();
}

int vlbm_mesh_create(int lattice, const int64_t n[3], const double* coords, const vlbm_topology* topo, double dx,
                     vlbm_mesh* out) {
  if (!n || !coords || !topo || !out) return fail(VLBM_ERR_ARG, "vlbm_mesh_create: null argument");
  *out = nullptr;
  if (lattice < VLBM_D2Q9 || lattice > VLBM_D3Q39) return fail(VLBM_ERR_ARG, "unknown lattice %d", lattice);
  if (!(dx > 0.0) || !isfinite(dx)) return fail(VLBM_ERR_ARG, "dx must be positive and finite");
  const int d = (lattice == VLBM_D2Q9 || lattice == VLBM_D2Q21) ? 2 : 3;
  const int speed = lattice_speed(lattice);
  if (d == 2 && n[2] != 1) return fail(VLBM_ERR_ARG, "a 2-D lattice needs n[2] == 1");
  int64_t nc = 1;
  for (int i = 0; i < d; ++i) {
    if (n[i] < 1 || n[i] > (1 << 20)) return fail(VLBM_ERR_ARG, "n[%d] = %lld out of range", i, (long long)n[i]);
    nc *= n[i];
  }
  if (nc > (int64_t)0x3fffffff) return fail(VLBM_ERR_ARG, "too many cells (%lld)", (long long)nc);
  MeshObj* m = new (std::nothrow) MeshObj();
  if (!m) return fail(VLBM_ERR_NOMEM, "host allocation failed");
  m->lattice = lattice;
  m->d = d;
  m->Q = lattice == VLBM_D2Q9 ? 9 : lattice == VLBM_D3Q19 ? 19 : lattice == VLBM_D2Q21 ? 21 : 39;
  const int ghost = speed + 1;   // ghost node layers per non-periodic face
  int wall_axes = 0;
  m->dx = dx;
  size_t ncoord = (size_t)d;
  for (int i = 0; i < 3; ++i) {
    const bool active = i < d;
    m->box.n[i] = active ? (int)n[i] : 1;
    for (int f = 0; f < 2; ++f) m->box.face[i][f] = active ? topo->face[i][f] : VLBM_PERIODIC;
    if (active) {
      const int lo = topo->face[i][0], hi = topo->face[i][1];
      if (lo < 0 || lo > 2 || hi < 0 || hi > 2) {
        delete m;
        return fail(VLBM_ERR_ARG, "axis %d: unknown face kind", i);
      }
      if ((lo == VLBM_PERIODIC) != (hi == VLBM_PERIODIC)) {
        delete m;
        return fail(VLBM_ERR_ARG, "axis %d must be periodic on both faces or on neither", i);
      }
      if (lo == VLBM_PERIODIC && n[i] < 2) {
        delete m;
        return fail(VLBM_ERR_ARG, "periodic axis %d needs at least 2 cells", i);
      }
      // links longer than one cell: walls on one axis at most, no far field
      if (speed > 1 && (lo == VLBM_FARFIELD || hi == VLBM_FARFIELD)) {
        delete m;
        return fail(VLBM_ERR_UNSUPPORTED, "axis %d: far-field faces are built for one-cell links only", i);
      }
      if (speed > 1 && lo == VLBM_WALL && ++wall_axes > 1) {
        delete m;
        return fail(VLBM_ERR_UNSUPPORTED, "this lattice takes walls on one axis at most");
      }
      if (n[i] < speed) {
        delete m;
        return fail(VLBM_ERR_ARG, "axis %d needs at least %d cells for this lattice", i, speed);
      }
    }
    m->m[i] = !active ? 1 : (m->box.face[i][0] == VLBM_PERIODIC ? (int)n[i] : (int)n[i] + 2 * ghost);
    ncoord *= m->m[i];
    for (int k = 0; k < 3; ++k) m->wrap[i][k] = (active && k < d) ? topo->wrap[i][k] : 0.0;
  }
  m->box.ncells = (int)nc;
  m->box.inv_n[0] = 1.0 / m->box.n[0];
  m->box.inv_n[1] = 1.0 / m->box.n[1];
  int rc = dev_alloc(&m->coords, ncoord * sizeof(double));
  if (rc) {
    delete m;
    return rc;
  }
  // device or host coordinates: the direction follows from the pointer
  if (hipMemcpy(m->coords, coords, ncoord * sizeof(double), hipMemcpyDefault) != hipSuccess) {
    dev_free(m->coords);
    delete m;
    return fail(VLBM_ERR_DEVICE, "copy of coordinates failed");
  }
  if ((rc = alloc_mesh_geometry(m))) {
    vlbm_mesh_destroy(reinterpret_cast<vlbm_mesh>(m));
    return rc;
  }
  *out = reinterpret_cast<vlbm_mesh>(m);
  return ok();
}

static void release_mesh(MeshObj* m) {
  dev_free(m->coords);
  dev_free(m->J);
  dev_free(m->gup);
  dev_free(m->gco);
  dev_free(m->g);
  dev_free(m->A);
  delete m;
}

int vlbm_mesh_destroy(vlbm_mesh mh) {
  MeshObj* m = reinterpret_cast<MeshObj*>(mh);
  if (!m) return ok();
  // simulations still hold the mesh: it is released with the last of them
  if (m->users > 0) {
    m->destroy_pending = true;
    return ok();
  }
  release_mesh(m);
  return ok();
}


}  // extern "C"

namespace vlbm {

int alloc_mesh_geometry(MeshObj* m) {
  const size_t nc = m->box.ncells;
  const int d = m->d;
  int rc;
  if ((rc = dev_alloc(&m->J, nc * sizeof(double)))) return rc;
  if ((rc = dev_alloc(&m->gup, nc * d * d * sizeof(double)))) return rc;
  if ((rc = dev_alloc(&m->gco, nc * d * d * sizeof(double)))) return rc;
  if ((rc = dev_alloc(&m->g, nc * d * d * sizeof(double)))) return rc;
  if ((rc = dev_alloc(&m->A, nc * m->Q * d * sizeof(double)))) return rc;
  return VLBM_OK;
}

// The report of a geometry pass from its flag and its (already reduced or
// per-block) diagnostics: r[6] = min J, -max J, min eig, -max eig, min rest
// f^eq/w, -max |A|.
int finish_geometry(MeshObj* m, int flag, const double* r, vlbm_geom_report* rep) {
  if (flag) {
    m->have_geometry = false;
    return fail(VLBM_ERR_MESH, "degenerate mesh:%s%s", (flag & 1) ? " beta undefined (D_i == D_-i)" : "",
                (flag & 2) ? " J <= 0 (reorder axes for a positive handedness)" : "");
  }
  m->report.min_J = r[0];
  m->report.max_J = -r[1];
  m->report.min_gup_eig = r[2];
  m->report.max_gup_eig = -r[3];
  m->report.min_rest_feq_over_w = r[4];
  m->report.max_abs_A = -r[5];
  m->have_geometry = true;
  if (rep) *rep = m->report;
  return ok();
}

}  // namespace vlbm

extern "C" {

int vlbm_geometry_precompute(vlbm_mesh mh, void* stream, vlbm_geom_report* rep) {
  MeshObj* m = reinterpret_cast<MeshObj*>(mh);
  if (!m) return fail(VLBM_ERR_ARG, "null mesh");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = geometry_partial_blocks(m);
  const size_t nbox = geometry_box_cells(m);
  int* dflag = nullptr;
  double* partial = nullptr;
  double* gbox = nullptr;
  int rc;
  auto release = [&]() {
    dev_free(dflag);
    dev_free(partial);
    dev_free(gbox);
  };
  if ((rc = dev_alloc(&dflag, sizeof(int))) || (rc = dev_alloc(&partial, (size_t)nb * 6 * sizeof(double))) ||
      (rc = dev_alloc(&gbox, sizeof(double) * m->d * m->d * nbox))) {
    release();
    return rc;
  }
  hipError_t e = hipMemsetAsync(dflag, 0, sizeof(int), s);
  if (e == hipSuccess) e = launch_geometry(m, s, dflag, partial, nb, gbox);
  int flag = 0;
  std::vector<double> hp((size_t)nb * 6);
  if (e == hipSuccess) e = hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), partial, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release();
  if (e != hipSuccess) return fail(VLBM_ERR_DEVICE, "geometry precompute: %s", hipGetErrorString(e));
  double r[6];
  for (int k = 0; k < 6; ++k) r[k] = INFINITY;
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < 6; ++k) r[k] = fmin(r[k], hp[b * 6 + k]);
  return finish_geometry(m, flag, r, rep);
}

int vlbm_geometry_fields(vlbm_mesh mh, double* J, double* gup, double* A, double* g) {
  MeshObj* m = reinterpret_cast<MeshObj*>(mh);
  if (!m) return fail(VLBM_ERR_ARG, "null mesh");
  if (!m->have_geometry) return fail(VLBM_ERR_STATE, "geometry not precomputed");
  const size_t nc = m->box.ncells;
  const int d = m->d;
  if (m->mover) {   // a moved mesh: its coefficients of the current positions, on the mover's stream
    HIP_TRY(refresh_moving_state(m->mover));
    HIP_TRY(hipStreamSynchronize(m->mover->stream));
  }
  if (J) HIP_TRY(hipMemcpy(J, m->J, nc * sizeof(double), hipMemcpyDeviceToDevice));
  if (gup) HIP_TRY(hipMemcpy(gup, m->gup, nc * d * d * sizeof(double), hipMemcpyDeviceToDevice));
  if (A) HIP_TRY(hipMemcpy(A, m->A, nc * m->Q * d * sizeof(double), hipMemcpyDeviceToDevice));
  if (g) HIP_TRY(hipMemcpy(g, m->g, nc * d * d * sizeof(double), hipMemcpyDeviceToDevice));
  return ok();
}

static void free_sim(SimObj* s) {
  MeshObj* mesh = s->mesh;
  if (mesh && mesh->mover == s) {
    // the mesh outlives the simulation that moved it: its outgoing coefficients
    // of the current positions are made before the boxes they come from go
    if (refresh_moving_state(s) == hipSuccess) (void)hipStreamSynchronize(s->stream);
    mesh->mover = nullptr;
  }
  for (double* b : s->mv_box) dev_free(b);
  dev_free(s->mv_J);
  dev_free(s->mv_gup);
  dev_free(s->mv_gco);
  dev_free(s->Ain);
  dev_free(s->pop[0]);
  dev_free(s->pop[1]);
  dev_free(s->geo);
  dev_free(s->fcache);
  dev_free(s->rown);
  dev_free(s->rown_spare);
  dev_free(s->audit_ring);
  dev_free(s->audit_partial);
  dev_free(s->u_prev);
  dev_free(s->flags);
  dev_free(s->stats);
  delete static_cast<EventPool*>(s->timing);
  delete s;
  // the last simulation of a mesh whose destruction was asked for releases it
  if (mesh && --mesh->users == 0 && mesh->destroy_pending) release_mesh(mesh);
}

int vlbm_sim_destroy(vlbm_sim sh) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (s) free_sim(s);
  return ok();
}


}  // extern "C"

static int create_sim(MeshObj* m, const vlbm_params* p, const double* rho, const double* u, hipStream_t stream,
                      SimObj** out) {
  if (!m || !p || !out) return fail(VLBM_ERR_ARG, "vlbm_init: null argument");
  *out = nullptr;
  if (!m->have_geometry) return fail(VLBM_ERR_STATE, "vlbm_init before vlbm_geometry_precompute");
  if (!(p->tau > 0.5) || !isfinite(p->tau)) return fail(VLBM_ERR_ARG, "tau must exceed 1/2 (got %g)", p->tau);
  if (p->tau_g != 0.0 && (!(p->tau_g > 0.5) || !isfinite(p->tau_g)))
    return fail(VLBM_ERR_ARG, "tau_g must be 0 (BGK) or exceed 1/2 (got %g)", p->tau_g);
  if (p->precision < VLBM_FP64 || p->precision > VLBM_FP32C)
    return fail(VLBM_ERR_UNSUPPORTED, "precision %d is not built", p->precision);
  if (p->audit_every < 0) return fail(VLBM_ERR_ARG, "audit_every must be >= 0");
  if (lattice_speed(m->lattice) > 1 && storage_is_16(p->precision))
    return fail(VLBM_ERR_UNSUPPORTED, "16-bit storage is built for D2Q9 and D3Q19");
  SimObj* s = new (std::nothrow) SimObj();
  if (!s) return fail(VLBM_ERR_NOMEM, "host allocation failed");
  s->mesh = m;
  m->users++;
  s->p = *p;
  if (s->p.fp_max_iter <= 0) s->p.fp_max_iter = 50;
  if (s->p.fp_tol < 0)
    s->p.fp_tol = s->p.precision == VLBM_FP64 ? 1e-14 : (s->p.precision == VLBM_FP32 ? 1e-10 : 1e-7);
  // (FP16S / BF16S use FP32 arithmetic, like FP32C)
  s->stream = stream;
  const int d = m->d;
  for (int k = 0; k < d; ++k)
    if (p->body_force[k] != 0.0) s->has_force = 1;
  s->comp_A = s->p.precision == VLBM_FP32;
  for (int i = 0; i < d; ++i)
    for (int f = 0; f < 2; ++f)
      if (m->box.face[i][f] == VLBM_FARFIELD) s->has_farfield = 1;
  const size_t nc = m->box.ncells;
  const size_t sb = storage_bytes(s->p.precision);
  s->pop_bytes = nc * m->Q * sb;
  int rc;
  auto bail = [&](int code) {
    free_sim(s);
    return code;
  };
  if ((rc = dev_alloc(&s->pop[0], s->pop_bytes))) return bail(rc);
  if ((rc = dev_alloc(&s->pop[1], s->pop_bytes))) return bail(rc);
  const int words = pack_words(m->lattice);
  if ((rc = dev_alloc(&s->geo, pack_elements(words, nc) * geometry_bytes(s->p.precision)))) return bail(rc);
  if (storage_shifted(s->p.precision))   // 16-bit references
    if ((rc = dev_alloc(&s->rown, nc * m->Q * 2))) return bail(rc);
    if ((rc = dev_alloc(&s->rown_spare, nc * m->Q * 2))) return bail(rc);
  if ((rc = dev_alloc(&s->fcache, nc * d * fcache_elem(s->p.precision)))) return bail(rc);
  s->audit_cap = 4096;
  if ((rc = dev_alloc(&s->audit_ring, sizeof(vlbm_audit) * s->audit_cap))) return bail(rc);
  s->audit_blocks = audit_partial_blocks(m);
  if ((rc = dev_alloc(&s->audit_partial, sizeof(double) * s->audit_blocks * audit_words()))) return bail(rc);
  if ((rc = dev_alloc(&s->u_prev, sizeof(double) * nc * d))) return bail(rc);
  if ((rc = dev_alloc(&s->flags, sizeof(int) * 4))) return bail(rc);
  if ((rc = dev_alloc(&s->stats, sizeof(unsigned long long) * 4 * kStatSlots))) return bail(rc);
  hipError_t e = hipMemsetAsync(s->flags, 0, sizeof(int) * 4, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->stats, 0, sizeof(unsigned long long) * 4 * kStatSlots, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->pop[0], 0, s->pop_bytes, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->pop[1], 0, s->pop_bytes, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->fcache, 0, nc * d * fcache_elem(s->p.precision), s->stream);
  if (e == hipSuccess) e = launch_pack(s);
  if (e == hipSuccess && storage_shifted(s->p.precision)) e = launch_refs(s);
  if (e == hipSuccess) e = launch_init(s, rho, u, s->flags);
  int hflag = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hflag, s->flags, sizeof(int), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    fail(VLBM_ERR_DEVICE, "vlbm_init: %s", hipGetErrorString(e));
    return bail(VLBM_ERR_DEVICE);
  }
  if (hflag) {
    fail(VLBM_ERR_NOCONVERGE, "initial-state fixed point did not converge in %d cells", hflag);
    return bail(VLBM_ERR_NOCONVERGE);
  }
  (void)hipMemsetAsync(s->flags, 0, sizeof(int) * 4, s->stream);
  s->buf = 0;
  s->t = 0;
  *out = s;
  return ok();
}

extern "C" {

int vlbm_init(vlbm_mesh mh, const vlbm_params* p, const double* rho, const double* u, void* stream, vlbm_sim* out) {
  if (!out) return fail(VLBM_ERR_ARG, "vlbm_init: null argument");
  SimObj* s = nullptr;
  const int rc = create_sim(reinterpret_cast<MeshObj*>(mh), p, rho, u, static_cast<hipStream_t>(stream), &s);
  *out = reinterpret_cast<vlbm_sim>(s);
  return rc;
}

int vlbm_reinit(vlbm_sim sh, const double* rho, const double* u) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s) return fail(VLBM_ERR_ARG, "null sim");
  const size_t nc = s->mesh->box.ncells;
  HIP_TRY(hipMemsetAsync(s->flags, 0, sizeof(int) * 4, s->stream));
  HIP_TRY(hipMemsetAsync(s->pop[0], 0, s->pop_bytes, s->stream));
  HIP_TRY(hipMemsetAsync(s->pop[1], 0, s->pop_bytes, s->stream));
  s->buf = 0;
  HIP_TRY(launch_init(s, rho, u, s->flags));
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, s->flags, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  (void)nc;
  if (hflag) return fail(VLBM_ERR_NOCONVERGE, "initial-state fixed point did not converge in %d cells", hflag);
  HIP_TRY(hipMemsetAsync(s->flags, 0, sizeof(int) * 4, s->stream));
  s->t = 0;
  s->have_u_prev = 0;
  return ok();
}

int vlbm_audit_now(vlbm_sim sh) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s) return fail(VLBM_ERR_ARG, "null sim");
  const int slot = (int)(s->audit_head % s->audit_cap);
  HIP_TRY(launch_audit(s, slot));
  s->audit_head++;
  if (s->audit_head - s->audit_tail > s->audit_cap) s->audit_tail = s->audit_head - s->audit_cap;
  return ok();
}

int vlbm_step(vlbm_sim sh, int64_t nsteps) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s) return fail(VLBM_ERR_ARG, "null sim");
  if (nsteps < 0) return fail(VLBM_ERR_ARG, "nsteps < 0");
  if (s->geo_stale) {   // the mesh moved (vlbm_step_moving): re-pack its current geometry
    HIP_TRY(refresh_moving_state(s));
    HIP_TRY(launch_pack(s));
    s->geo_stale = 0;
  }
  const int rebase = rebase_period(s->p);
  EventPool* ep = s->timing_on ? static_cast<EventPool*>(s->timing) : nullptr;
  for (int64_t k = 0; k < nsteps; ++k) {
    // the step that reaches a multiple of the re-basing period re-bases its
    // own outputs (new references into the spare array, swapped in after it);
    // a stream-only step, and a batch member (whose batch keeps its reference
    // array in its step arguments), leave that to the re-basing kernel
    const bool due = rebase > 0 && storage_shifted(s->p.precision) && (s->t + 1) % rebase == 0;
    s->rebase_in_step = due && !s->p.stream_only && !s->batch_member;
    if (ep) HIP_TRY(ep->begin(s->stream, 0));
    const hipError_t le = launch_step(s);
    const bool fused = s->rebase_in_step;
    s->rebase_in_step = 0;
    HIP_TRY(le);
    if (ep) HIP_TRY(ep->end(s->stream));
    if (fused) std::swap(s->rown, s->rown_spare);
    s->buf ^= 1;
    s->t++;
    s->state_moving = 0;   // a static step: the state's incoming coefficients are the opposite outgoing ones
    if (due && !fused) {
      if (ep) HIP_TRY(ep->begin(s->stream, 1));
      HIP_TRY(launch_rebase(s));
      if (ep) HIP_TRY(ep->end(s->stream));
    }
    if (s->p.audit_every > 0 && s->t % s->p.audit_every == 0) {
      int rc = vlbm_audit_now(sh);
      if (rc) return rc;
    }
  }
  return ok();
}

// Count of cell-steps whose fixed point hit its cap since the last report
// (flags[2]); reset once read.  Synchronises the stream.
static int take_step_unconverged(SimObj* s, int* count) {
  HIP_TRY(hipMemcpyAsync(count, s->flags + 2, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (*count) HIP_TRY(hipMemsetAsync(s->flags + 2, 0, sizeof(int), s->stream));
  return VLBM_OK;
}

int vlbm_sync(vlbm_sim sh) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s) return fail(VLBM_ERR_ARG, "null sim");
  int n = 0;
  const int rc = take_step_unconverged(s, &n);
  if (rc) return rc;
  if (s->moving) {   // degenerate cells met by the geometry of a moving step
    int bad = 0;
    HIP_TRY(hipMemcpy(&bad, s->flags + 1, sizeof(int), hipMemcpyDeviceToHost));
    if (bad) {
      HIP_TRY(hipMemset(s->flags + 1, 0, sizeof(int)));
      return fail(VLBM_ERR_MESH, "the moving mesh became degenerate:%s%s",
                  (bad & 1) ? " beta undefined (D_i == D_-i)" : "", (bad & 2) ? " J <= 0" : "");
    }
  }
  if (n) return fail(VLBM_ERR_NOCONVERGE, "fixed point hit its cap in %d cell-steps", n);
  return ok();
}

int vlbm_step_moving(vlbm_sim sh, const double* coords_next, const double* wrap_next) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s || !coords_next) return fail(VLBM_ERR_ARG, "vlbm_step_moving: null argument");
  MeshObj* m = s->mesh;
  if (s->p.precision != VLBM_FP64)
    return fail(VLBM_ERR_UNSUPPORTED, "moving meshes are built for FP64 storage and arithmetic");
  if (m->lattice != VLBM_D2Q9 && m->lattice != VLBM_D3Q19)
    return fail(VLBM_ERR_UNSUPPORTED, "moving meshes are built for D2Q9 and D3Q19");
  for (int i = 0; i < m->d; ++i)
    if (m->box.face[i][0] != VLBM_PERIODIC)
      return fail(VLBM_ERR_UNSUPPORTED, "moving meshes are built for periodic axes only");
  if (general_collision(s->p) || s->p.stream_only)
    return fail(VLBM_ERR_UNSUPPORTED, "moving meshes are built for the BGK collision");
  if (m->users != 1) return fail(VLBM_ERR_STATE, "the mesh is shared by %d simulations; moving it would change them all",
                                 m->users);
  const size_t nc = m->box.ncells;
  const int d = m->d;
  const size_t nbox = geometry_box_cells(m);
  int rc;
  if (!s->moving) {   // first moving step: the mesh was at rest before it (the box of t - 1 is that of t)
    for (double*& b : s->mv_box)
      if ((rc = dev_alloc(&b, sizeof(double) * d * d * nbox))) return rc;
    if ((rc = dev_alloc(&s->mv_J, nc * sizeof(double))) || (rc = dev_alloc(&s->mv_gup, nc * d * d * sizeof(double))) ||
        (rc = dev_alloc(&s->mv_gco, nc * d * d * sizeof(double))) ||
        (rc = dev_alloc(&s->Ain, nc * m->Q * d * sizeof(double))))
      return rc;
    HIP_TRY(hipMemsetAsync(s->flags + 1, 0, sizeof(int), s->stream));
    // g_i of the current mesh on its box (into the t box; the real-cell arrays
    // it also writes are the next-time scratch), then t - 1 = t
    HIP_TRY(launch_basis_of(m, m->coords, m->wrap, s->mv_box[1], s->mv_J, s->mv_gup, s->mv_gco, nullptr,
                            s->flags + 1, s->stream));
    HIP_TRY(hipMemcpyAsync(s->mv_box[0], s->mv_box[1], sizeof(double) * d * d * nbox, hipMemcpyDeviceToDevice,
                           s->stream));
    s->moving = 1;
    m->mover = s;
  }
  double wrap[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) wrap[i][k] = (wrap_next && i < d && k < d) ? wrap_next[i * 3 + k] : m->wrap[i][k];
  EventPool* ep = s->timing_on ? static_cast<EventPool*>(s->timing) : nullptr;
  // geometry of t + 1
  if (ep) HIP_TRY(ep->begin(s->stream, 2));
  HIP_TRY(launch_basis_of(m, coords_next, wrap, s->mv_box[2], s->mv_J, s->mv_gup, s->mv_gco, nullptr, s->flags + 1,
                          s->stream));
  if (ep) HIP_TRY(ep->end(s->stream));
  // the step at t, its link coefficients computed from the boxes of t - 1, t, t + 1
  if (ep) HIP_TRY(ep->begin(s->stream, 0));
  HIP_TRY(launch_step_moving(s, s->mv_box[0], s->mv_box[1], s->mv_box[2]));
  if (ep) HIP_TRY(ep->end(s->stream));
  s->buf ^= 1;
  s->t++;
  // the mesh is now at t + 1: its coordinates, translations and geometry
  const size_t ncoord = (size_t)m->m[0] * m->m[1] * m->m[2] * d;
  HIP_TRY(hipMemcpyAsync(m->coords, coords_next, ncoord * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) m->wrap[i][k] = wrap[i][k];
  std::swap(m->J, s->mv_J);
  std::swap(m->gup, s->mv_gup);
  std::swap(m->gco, s->mv_gco);
  double* oldest = s->mv_box[0];
  s->mv_box[0] = s->mv_box[1];
  s->mv_box[1] = s->mv_box[2];
  s->mv_box[2] = oldest;
  s->geo_stale = 1;
  s->mv_state_stale = 1;   // Ain and mesh->A of t + 1: made when first needed
  s->state_moving = 1;
  if (s->p.audit_every > 0 && s->t % s->p.audit_every == 0) {
    const int arc = vlbm_audit_now(sh);
    if (arc) return arc;
  }
  return ok();
}

int vlbm_step_stats(vlbm_sim sh, int enable, uint64_t* out) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s) return fail(VLBM_ERR_ARG, "null sim");
  if (out) {
    unsigned long long h[4 * kStatSlots];
    HIP_TRY(hipMemcpyAsync(h, s->stats, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipMemsetAsync(s->stats, 0, sizeof(h), s->stream));
    for (int k = 0; k < 4; ++k) {
      out[k] = 0;
      for (int q = 0; q < kStatSlots; ++q) out[k] += h[4 * q + k];
    }
  }
  s->stats_on = enable ? 1 : 0;
  return ok();
}

int vlbm_kernel_timing(vlbm_sim sh, int enable, double* out) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s) return fail(VLBM_ERR_ARG, "null sim");
  if (!s->timing) {
    s->timing = new (std::nothrow) EventPool();
    if (!s->timing) return fail(VLBM_ERR_NOMEM, "host allocation failed");
  }
  EventPool* ep = static_cast<EventPool*>(s->timing);
  if (out) {
    for (int k = 0; k < 2 * kTimingKinds; ++k) out[k] = 0.0;
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (size_t i = 0; i < ep->used; ++i) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ep->ev[2 * i], ep->ev[2 * i + 1]));
      out[2 * ep->kind[i]] += ms;
      out[2 * ep->kind[i] + 1] += 1.0;
    }
  }
  if (out || !enable) ep->used = 0;
  s->timing_on = enable ? 1 : 0;
  return ok();
}

int vlbm_set_fixed_point(vlbm_sim sh, int32_t max_iter, double tol) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s) return fail(VLBM_ERR_ARG, "null sim");
  s->p.fp_max_iter = max_iter > 0 ? max_iter : 50;
  s->p.fp_tol = tol >= 0 ? tol : (s->p.precision == VLBM_FP64 ? 1e-14 : (s->p.precision == VLBM_FP32 ? 1e-10 : 1e-7));
  return ok();
}

int vlbm_moments(vlbm_sim sh, double* rho, double* u, double* U) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s || !rho || !u) return fail(VLBM_ERR_ARG, "vlbm_moments: null argument");
  int steps_unconv = 0;
  int rc = take_step_unconverged(s, &steps_unconv);
  if (rc) return rc;
  HIP_TRY(hipMemsetAsync(s->flags, 0, sizeof(int), s->stream));
  HIP_TRY(launch_moments(s, rho, u, U, s->flags));
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, s->flags, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (hflag) return fail(VLBM_ERR_NOCONVERGE, "fixed point did not converge in %d cells", hflag);
  if (steps_unconv)
    return fail(VLBM_ERR_NOCONVERGE, "fixed point hit its cap in %d cell-steps of the steps taken", steps_unconv);
  return ok();
}

int vlbm_populations(vlbm_sim sh, double* N) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s || !N) return fail(VLBM_ERR_ARG, "vlbm_populations: null argument");
  HIP_TRY(launch_get_pop(s, N));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return ok();
}

int vlbm_set_populations(vlbm_sim sh, const double* N) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s || !N) return fail(VLBM_ERR_ARG, "vlbm_set_populations: null argument");
  HIP_TRY(launch_set_pop(s, N));
  HIP_TRY(hipMemsetAsync(s->fcache, 0, (size_t)s->mesh->box.ncells * s->mesh->d * fcache_elem(s->p.precision),
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return ok();
}

int vlbm_audits(vlbm_sim sh, vlbm_audit* out, int cap, int* n_out) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s || !n_out || (cap > 0 && !out)) return fail(VLBM_ERR_ARG, "vlbm_audits: null argument");
  *n_out = 0;
  HIP_TRY(hipStreamSynchronize(s->stream));
  int n = 0;
  bool bad = false;
  vlbm_audit* ring = static_cast<vlbm_audit*>(s->audit_ring);
  while (n < cap && s->audit_tail < s->audit_head) {
    const int slot = (int)(s->audit_tail % s->audit_cap);
    HIP_TRY(hipMemcpy(out + n, ring + slot, sizeof(vlbm_audit), hipMemcpyDeviceToHost));
    if (out[n].nonfinite) bad = true;
    ++n;
    s->audit_tail++;
  }
  *n_out = n;
  if (bad) return fail(VLBM_ERR_NONFINITE, "non-finite populations detected");
  return ok();
}

// Shifted modes: the checkpoint also holds the slots' references (re-based
// during the run, so they are part of the state).
static size_t ref_bytes(const SimObj* s) {
  return storage_shifted(s->p.precision) ? (size_t)s->mesh->box.ncells * s->mesh->Q * 2 : 0;
}

int vlbm_save(vlbm_sim sh, void* buf, size_t cap, size_t* used) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s || !used) return fail(VLBM_ERR_ARG, "vlbm_save: null argument");
  const size_t fbytes = (size_t)s->mesh->box.ncells * s->mesh->d * fcache_elem(s->p.precision);
  const size_t rbytes = ref_bytes(s);
  const size_t need = sizeof(CkptHeader) + s->pop_bytes + fbytes + rbytes;
  *used = need;
  if (!buf) return ok();
  if (cap < need) return fail(VLBM_ERR_ARG, "buffer too small: need %zu bytes", need);
  CkptHeader h{kMagic, s->mesh->lattice, s->p.precision, s->mesh->box.ncells, s->mesh->Q, s->t,
               (int64_t)s->pop_bytes};
  memcpy(buf, &h, sizeof(h));
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemcpy(static_cast<char*>(buf) + sizeof(h), s->pop[s->buf], s->pop_bytes, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(static_cast<char*>(buf) + sizeof(h) + s->pop_bytes, s->fcache, fbytes, hipMemcpyDeviceToHost));
  if (rbytes)
    HIP_TRY(hipMemcpy(static_cast<char*>(buf) + sizeof(h) + s->pop_bytes + fbytes, s->rown, rbytes,
                      hipMemcpyDeviceToHost));
  return ok();
}

int vlbm_restore(vlbm_sim sh, const void* buf, size_t size) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s || !buf) return fail(VLBM_ERR_ARG, "vlbm_restore: null argument");
  if (size < sizeof(CkptHeader)) return fail(VLBM_ERR_ARG, "checkpoint too small");
  const size_t fbytes = (size_t)s->mesh->box.ncells * s->mesh->d * fcache_elem(s->p.precision);
  const size_t rbytes = ref_bytes(s);
  CkptHeader h;
  memcpy(&h, buf, sizeof(h));
  if (h.magic != kMagic || h.lattice != s->mesh->lattice || h.precision != s->p.precision ||
      h.ncells != s->mesh->box.ncells || h.Q != s->mesh->Q || h.bytes != (int64_t)s->pop_bytes ||
      size != sizeof(h) + s->pop_bytes + fbytes + rbytes)
    return fail(VLBM_ERR_ARG, "checkpoint does not match this simulation");
  HIP_TRY(hipStreamSynchronize(s->stream));
  HIP_TRY(hipMemcpy(s->pop[s->buf], static_cast<const char*>(buf) + sizeof(h), s->pop_bytes,
                    hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(s->fcache, static_cast<const char*>(buf) + sizeof(h) + s->pop_bytes, fbytes,
                    hipMemcpyHostToDevice));
  if (rbytes)
    HIP_TRY(hipMemcpy(s->rown, static_cast<const char*>(buf) + sizeof(h) + s->pop_bytes + fbytes, rbytes,
                      hipMemcpyHostToDevice));
  s->t = h.t;
  s->have_u_prev = 0;
  return ok();
}

int vlbm_sim_step_count(vlbm_sim sh, int64_t* t) {
  SimObj* s = reinterpret_cast<SimObj*>(sh);
  if (!s || !t) return fail(VLBM_ERR_ARG, "null argument");
  *t = s->t;
  return ok();
}


/* ---------------------------- batches of meshes ---------------------------- */

static int batch_cus() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus > 0 ? cus : 256;
}

int vlbm_batch_create(const vlbm_mesh* meshes, const vlbm_params* params, int count, void* stream, vlbm_batch* out) {
  if (!meshes || !params || !out || count <= 0) return fail(VLBM_ERR_ARG, "vlbm_batch_create: bad argument");
  *out = nullptr;
  if (!meshes[0]) return fail(VLBM_ERR_ARG, "vlbm_batch_create: null mesh");
  const int lat = reinterpret_cast<MeshObj*>(meshes[0])->lattice;
  const int prec = params[0].precision;
  if (prec != VLBM_FP64 && prec != VLBM_FP32 && prec != VLBM_FP32C)
    return fail(VLBM_ERR_UNSUPPORTED, "batches are built for FP64, FP32 and FP32C");
  if (lat != VLBM_D2Q9 && lat != VLBM_D3Q19) return fail(VLBM_ERR_UNSUPPORTED, "batches are built for D2Q9 and D3Q19");
  BatchObj* b = new (std::nothrow) BatchObj();
  if (!b) return fail(VLBM_ERR_NOMEM, "host allocation failed");
  b->lattice = lat;
  b->precision = prec;
  b->cus = batch_cus();
  if (stream) {
    b->stream = static_cast<hipStream_t>(stream);
  } else if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return fail(VLBM_ERR_DEVICE, "stream creation failed");
  } else {
    b->own_stream = true;
  }
  auto bail = [&](int rc) {
    vlbm_batch_destroy(reinterpret_cast<vlbm_batch>(b));
    return rc;
  };
  for (int i = 0; i < count; ++i) {
    MeshObj* m = reinterpret_cast<MeshObj*>(meshes[i]);
    if (!m || m->lattice != lat || params[i].precision != prec) {
      fail(VLBM_ERR_ARG, "member %d: every member needs the same lattice and precision", i);
      return bail(VLBM_ERR_ARG);
    }
    SimObj* s = nullptr;
    const int rc = create_sim(m, &params[i], nullptr, nullptr, b->stream, &s);
    if (rc) return bail(rc);
    s->batch_member = 1;
    b->members.push_back(s);
    const int rb = storage_shifted(prec) ? rebase_period(s->p) : 0;
    if (i == 0) {
      b->rebase = rb > 0 ? rb : 0;
    } else if ((rb > 0 ? rb : 0) != b->rebase) {
      fail(VLBM_ERR_ARG, "member %d: every member needs the same re-basing period", i);
      return bail(VLBM_ERR_ARG);
    }
    b->total_cells += m->box.ncells;
    b->any_ff = b->any_ff || s->has_farfield;
    b->any_general = b->any_general || general_collision(s->p);
  }
  // graphs hold an even number of steps (parity) that is a multiple of the
  // re-basing period, at least 32
  if (b->rebase > 0) {
    int gs = b->rebase % 2 ? 2 * b->rebase : b->rebase;
    b->graph_steps = gs * ((32 + gs - 1) / gs);
  }
  b->active.assign(b->members.size(), 1);
  if (batch_upload(b) != hipSuccess) {
    fail(VLBM_ERR_DEVICE, "batch upload failed");
    return bail(VLBM_ERR_DEVICE);
  }
  *out = reinterpret_cast<vlbm_batch>(b);
  return ok();
}

int vlbm_batch_destroy(vlbm_batch bh) {
  BatchObj* b = reinterpret_cast<BatchObj*>(bh);
  if (!b) return VLBM_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  batch_drop_graphs(b);
  for (SimObj* s : b->members) free_sim(s);
  dev_free(b->d_args);
  dev_free(b->d_tiles);
  dev_free(b->d_rsrc);
  dev_free(b->d_resid);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return VLBM_OK;
}

int vlbm_batch_residuals(vlbm_batch bh, double* residual) {
  BatchObj* b = reinterpret_cast<BatchObj*>(bh);
  if (!b || !residual) return fail(VLBM_ERR_ARG, "vlbm_batch_residuals: null argument");
  const int n = (int)b->members.size();
  if (!b->d_rsrc) {
    if (dev_alloc(&b->d_rsrc, sizeof(double*) * n) || dev_alloc(&b->d_resid, sizeof(double) * n))
      return VLBM_ERR_NOMEM;
  }
  std::vector<const double*> src(n);
  for (int i = 0; i < n; ++i) {
    SimObj* s = b->members[i];
    if (!b->active[i] && s->audit_head > 0) {   // retired: its last residual
      const int last = (int)((s->audit_head - 1) % s->audit_cap);
      src[i] = &static_cast<const vlbm_audit*>(s->audit_ring)[last].residual;
      continue;
    }
    const int slot = (int)(s->audit_head % s->audit_cap);
    HIP_TRY(launch_audit(s, slot));
    s->audit_head++;
    if (s->audit_head - s->audit_tail > s->audit_cap) s->audit_tail = s->audit_head - s->audit_cap;
    src[i] = &static_cast<const vlbm_audit*>(s->audit_ring)[slot].residual;
  }
  HIP_TRY(hipMemcpyAsync(b->d_rsrc, src.data(), sizeof(double*) * n, hipMemcpyHostToDevice, b->stream));
  HIP_TRY(batch_gather(b, b->d_rsrc, b->d_resid, n));
  HIP_TRY(hipMemcpyAsync(residual, b->d_resid, sizeof(double) * n, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return ok();
}

int vlbm_batch_member(vlbm_batch bh, int i, vlbm_sim* out) {
  BatchObj* b = reinterpret_cast<BatchObj*>(bh);
  if (!b || !out || i < 0 || i >= (int)b->members.size()) return fail(VLBM_ERR_ARG, "vlbm_batch_member: bad argument");
  *out = reinterpret_cast<vlbm_sim>(b->members[i]);
  return ok();
}

int vlbm_batch_info(vlbm_batch bh, int* count, int64_t* cells, void** stream, int* block, int* grid_per_cu) {
  BatchObj* b = reinterpret_cast<BatchObj*>(bh);
  if (!b) return fail(VLBM_ERR_ARG, "null batch");
  if (count) *count = (int)b->members.size();
  if (cells) *cells = b->total_cells;
  if (stream) *stream = b->stream;
  if (block) *block = b->block;
  if (grid_per_cu) *grid_per_cu = b->grid_per_cu;
  return ok();
}

int vlbm_batch_set_mode(vlbm_batch bh, int mode) {
  BatchObj* b = reinterpret_cast<BatchObj*>(bh);
  if (!b || mode < 0 || mode > 3) return fail(VLBM_ERR_ARG, "vlbm_batch_set_mode: bad argument");
  HIP_TRY(hipStreamSynchronize(b->stream));
  batch_drop_graphs(b);
  b->mode = mode;
  return ok();
}

int vlbm_batch_config(vlbm_batch bh, int block, int grid_per_cu) {
  BatchObj* b = reinterpret_cast<BatchObj*>(bh);
  if (!b || (block != 64 && block != 128 && block != 256) || grid_per_cu < 0)
    return fail(VLBM_ERR_ARG, "vlbm_batch_config: block must be 64, 128 or 256 and grid_per_cu >= 0");
  HIP_TRY(hipStreamSynchronize(b->stream));
  batch_drop_graphs(b);
  const bool rebuild = block != b->block;
  b->block = block;
  b->grid_per_cu = grid_per_cu;
  if (rebuild && batch_upload(b) != hipSuccess) return fail(VLBM_ERR_DEVICE, "batch upload failed");
  return ok();
}

// One step of every active member; `t` is the members' step count before it.
// The references are re-based after a step that reaches a multiple of the
// re-basing period, as vlbm_step does for a single mesh.
static int batch_one_step_eager(BatchObj* b, int parity, bool per_member, int64_t t) {
  if (!per_member) {
    HIP_TRY(batch_launch(b, parity));
  } else {
    for (size_t m = 0; m < b->members.size(); ++m)
      if (b->active[m]) HIP_TRY(launch_step(b->members[m]));
  }
  if (b->rebase > 0 && (t + 1) % b->rebase == 0) HIP_TRY(batch_rebase(b, parity ^ 1));
  return VLBM_OK;
}

static void batch_advance(BatchObj* b, int64_t k) {
  for (size_t m = 0; m < b->members.size(); ++m) {
    if (!b->active[m]) continue;
    SimObj* s = b->members[m];
    s->t += k;
    if (k & 1) s->buf ^= 1;
  }
  b->t += k;
}

// The first active member (its step count and buffer parity are the batch's),
// or nullptr when every member is retired.
static SimObj* batch_lead(const BatchObj* b) {
  for (size_t m = 0; m < b->members.size(); ++m)
    if (b->active[m]) return b->members[m];
  return nullptr;
}

int vlbm_batch_step(vlbm_batch bh, int64_t nsteps) {
  BatchObj* b = reinterpret_cast<BatchObj*>(bh);
  if (!b || nsteps < 0) return fail(VLBM_ERR_ARG, "vlbm_batch_step: bad argument");
  SimObj* lead = batch_lead(b);
  if (!lead) return ok();   // every member retired: nothing to step
  for (size_t m = 0; m < b->members.size(); ++m)
    if (b->active[m] && (b->members[m]->buf != lead->buf || b->members[m]->t != lead->t))
      return fail(VLBM_ERR_STATE, "batch members were stepped individually; they must share one step count");
  const bool per_member = b->mode >= VLBM_BATCH_EAGER;
  const bool graphs = b->mode == VLBM_BATCH_PERSISTENT_GRAPH || b->mode == VLBM_BATCH_EAGER_GRAPH;
  int64_t done = 0;
  if (graphs) {
    // graphs start at a multiple of the re-basing period
    while (b->rebase > 0 && done < nsteps && lead->t % b->rebase != 0) {
      const int rc = batch_one_step_eager(b, lead->buf, per_member, lead->t);
      if (rc) return rc;
      batch_advance(b, 1);
      ++done;
    }
    while (nsteps - done >= b->graph_steps) {
      const int par = lead->buf;
      if (!b->exec[par]) {
        hipError_t e = batch_capture(b, par, per_member);
        if (e != hipSuccess) return fail(VLBM_ERR_DEVICE, "graph capture: %s", hipGetErrorString(e));
      }
      HIP_TRY(hipGraphLaunch(b->exec[par], b->stream));
      batch_advance(b, b->graph_steps);
      done += b->graph_steps;
    }
  }
  for (; done < nsteps; ++done) {
    const int rc = batch_one_step_eager(b, lead->buf, per_member, lead->t);
    if (rc) return rc;
    batch_advance(b, 1);
  }
  return ok();
}

int vlbm_batch_set_active(vlbm_batch bh, const int32_t* active) {
  BatchObj* b = reinterpret_cast<BatchObj*>(bh);
  if (!b) return fail(VLBM_ERR_ARG, "null batch");
  const size_t n = b->members.size();
  std::vector<char> next(n, 1);
  if (active)
    for (size_t m = 0; m < n; ++m) next[m] = active[m] != 0;
  // the members stepped together must share their step count and parity
  const SimObj* lead = nullptr;
  for (size_t m = 0; m < n; ++m) {
    if (!next[m]) continue;
    const SimObj* s = b->members[m];
    if (!lead) lead = s;
    else if (s->t != lead->t || s->buf != lead->buf)
      return fail(VLBM_ERR_STATE, "member %zu is at step %lld, the others at %lld: they cannot step together", m,
                  (long long)s->t, (long long)lead->t);
  }
  if (next == b->active) return ok();
  HIP_TRY(hipStreamSynchronize(b->stream));
  batch_drop_graphs(b);
  b->active = next;
  if (batch_upload(b) != hipSuccess) return fail(VLBM_ERR_DEVICE, "batch upload failed");
  return ok();
}

int vlbm_batch_sync(vlbm_batch bh) {
  BatchObj* b = reinterpret_cast<BatchObj*>(bh);
  if (!b) return fail(VLBM_ERR_ARG, "null batch");
  HIP_TRY(hipStreamSynchronize(b->stream));
  int unconv = 0;
  for (SimObj* s : b->members) {
    int h = 0;
    const int rc = take_step_unconverged(s, &h);
    if (rc) return rc;
    unconv += h;
  }
  if (unconv) return fail(VLBM_ERR_NOCONVERGE, "fixed point hit its cap in %d cell-steps", unconv);
  return ok();
}

// Measured search over the launch shape of the batched kernel.  The state is
// snapshotted and restored, so tuning leaves the simulation where it was.
int vlbm_batch_autotune(vlbm_batch bh, int trial_steps, const char* cache_path, int* block_out, int* grid_out) {
  BatchObj* b = reinterpret_cast<BatchObj*>(bh);
  if (!b || trial_steps <= 0) return fail(VLBM_ERR_ARG, "vlbm_batch_autotune: bad argument");
  char key[256];
  snprintf(key, sizeof(key), "gfx950 lattice=%d precision=%d cells=%lld meshes=%d", b->lattice, b->precision,
           (long long)b->total_cells, (int)b->members.size());
  if (cache_path) {
    FILE* f = fopen(cache_path, "r");
    if (f) {
      char line[512];
      while (fgets(line, sizeof(line), f)) {
        int bl = 0, gp = 0;
        char* sep = strstr(line, " | ");
        if (sep && (size_t)(sep - line) == strlen(key) && strncmp(line, key, strlen(key)) == 0 &&
            sscanf(sep + 3, "block=%d grid_per_cu=%d", &bl, &gp) == 2) {
          fclose(f);
          const int rc = vlbm_batch_config(bh, bl, gp);
          if (block_out) *block_out = bl;
          if (grid_out) *grid_out = gp;
          return rc;
        }
      }
      fclose(f);
    }
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  // Snapshot every member's state (populations of the current parity, force
  // cache, step count); the trials below advance the members.
  struct Snap {
    void* mem;
    int buf;
    int64_t t;
  };
  std::vector<Snap> snap;
  auto fc_bytes = [](const SimObj* s) {
    return s->fcache ? (size_t)s->mesh->box.ncells * s->mesh->d * fcache_elem(s->p.precision) : (size_t)0;
  };
  auto rf_bytes = [](const SimObj* s) { return ref_bytes(s); };
  auto drop = [&]() {
    for (Snap& x : snap) dev_free(x.mem);
    snap.clear();
  };
  for (SimObj* s : b->members) {
    void* p = nullptr;
    const size_t fb = fc_bytes(s), rb = rf_bytes(s);
    if (dev_alloc((char**)&p, s->pop_bytes + fb + rb)) {
      drop();
      return VLBM_ERR_NOMEM;
    }
    snap.push_back(Snap{p, s->buf, s->t});
    hipError_t e = hipMemcpyAsync(p, s->pop[s->buf], s->pop_bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess && fb)
      e = hipMemcpyAsync(static_cast<char*>(p) + s->pop_bytes, s->fcache, fb, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess && rb)
      e = hipMemcpyAsync(static_cast<char*>(p) + s->pop_bytes + fb, s->rown, rb, hipMemcpyDeviceToDevice,
                         b->stream);
    if (e != hipSuccess) {
      drop();
      return fail(VLBM_ERR_DEVICE, "autotune snapshot: %s", hipGetErrorString(e));
    }
  }
  const int keep_mode = b->mode;
  b->mode = VLBM_BATCH_PERSISTENT;
  const int blocks[3] = {64, 128, 256};
  const int grids[5] = {1, 2, 4, 8, 0};
  float best = 1e30f;
  int bb = b->block, bg = b->grid_per_cu;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = VLBM_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = fail(VLBM_ERR_DEVICE, "autotune: event creation failed");
  for (int bl : blocks)
    for (int gp : grids) {
      if (rc) break;
      rc = vlbm_batch_config(bh, bl, gp);
      if (!rc) rc = vlbm_batch_step(bh, 2);
      if (!rc && hipEventRecord(e0, b->stream) != hipSuccess) rc = fail(VLBM_ERR_DEVICE, "autotune: event");
      if (!rc) rc = vlbm_batch_step(bh, trial_steps);
      float ms = 0;
      if (!rc && (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(VLBM_ERR_DEVICE, "autotune: timing");
      if (!rc && ms < best) {
        best = ms;
        bb = bl;
        bg = gp;
      }
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  // restore the snapshot whatever happened in the trials
  (void)hipStreamSynchronize(b->stream);
  for (size_t i = 0; i < b->members.size(); ++i) {
    SimObj* s = b->members[i];
    const size_t fb = fc_bytes(s), rb = rf_bytes(s);
    s->buf = snap[i].buf;
    s->t = snap[i].t;
    hipError_t e = hipMemcpyAsync(s->pop[s->buf], snap[i].mem, s->pop_bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess && fb)
      e = hipMemcpyAsync(s->fcache, static_cast<char*>(snap[i].mem) + s->pop_bytes, fb, hipMemcpyDeviceToDevice,
                         b->stream);
    if (e == hipSuccess && rb)
      e = hipMemcpyAsync(s->rown, static_cast<char*>(snap[i].mem) + s->pop_bytes + fb, rb, hipMemcpyDeviceToDevice,
                         b->stream);
    if (e != hipSuccess && !rc) rc = fail(VLBM_ERR_DEVICE, "autotune restore: %s", hipGetErrorString(e));
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess && !rc) rc = fail(VLBM_ERR_DEVICE, "autotune restore");
  drop();
  b->t = b->members.empty() ? 0 : b->members[0]->t;
  b->mode = keep_mode;
  if (rc) return rc;
  rc = vlbm_batch_config(bh, bb, bg);
  if (rc) return rc;
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%s | block=%d grid_per_cu=%d ms_per_step=%.6f\n", key, bb, bg, best / trial_steps);
      fclose(f);
    }
  }
  if (block_out) *block_out = bb;
  if (grid_out) *grid_out = bg;
  return ok();
}

}  // extern "C"

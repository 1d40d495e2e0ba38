// The C interface declared in include/tetct.h.
#include <algorithm>
#include <cstring>

#include "common.h"
#include "kernels.h"

namespace tct {
extern thread_local std::string g_err;

namespace {

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

tct_status need_device(const tct_mesh* m) {
  if (!m) {
    set_error("null mesh");
    return TCT_E_ARG;
  }
  if (m->host_only) {
    set_error("mesh was created with TCT_MESH_HOST_ONLY");
    return TCT_E_ARG;
  }
  return TCT_OK;
}

tct_status check_pair(const tct_mesh* m, const tct_geom* g) {
  tct_status st = need_device(m);
  if (st != TCT_OK) return st;
  if (!g) {
    set_error("null geometry");
    return TCT_E_ARG;
  }
  if (g->device != m->device) {
    set_error("mesh and geometry live on different devices");
    return TCT_E_ARG;
  }
  return check_geometry(m, g);
}

}  // namespace

int default_tile_u() { return 8; }

}  // namespace tct

using namespace tct;

extern "C" {

const char* tct_last_error(void) { return g_err.c_str(); }

const char* tct_version(void) { return "tetct 0.1 gfx950"; }

tct_status tct_mesh_create(const float* verts, int32_t nv, const int32_t* tets, int32_t nt, const int32_t* nbrs,
                           uint32_t flags, int device, tct_mesh** out) {
  if (!out) {
    set_error("tct_mesh_create: null output handle");
    return TCT_E_ARG;
  }
  *out = nullptr;
  if (flags & TCT_MESH_HOST_ONLY) return mesh_build(verts, nv, tets, nt, nbrs, flags, device, out);
  DeviceGuard dg(device);
  if (!dg.ok) {
    set_error("tct_mesh_create: cannot select the device");
    return TCT_E_HIP;
  }
  return mesh_build(verts, nv, tets, nt, nbrs, flags, device, out);
}

tct_status tct_mesh_counts(const tct_mesh* m, int32_t* nv, int32_t* nt, int32_t* nboundary, int64_t* device_bytes) {
  if (!m) {
    set_error("null mesh");
    return TCT_E_ARG;
  }
  if (nv) *nv = m->nv;
  if (nt) *nt = m->nt;
  if (nboundary) *nboundary = m->nb;
  if (device_bytes) *device_bytes = m->device_bytes;
  return TCT_OK;
}

tct_status tct_mesh_boundary(const tct_mesh* m, float* xyz, int32_t* owner) {
  if (!m) {
    set_error("null mesh");
    return TCT_E_ARG;
  }
  if (xyz) std::memcpy(xyz, m->bface_xyz.data(), sizeof(float) * m->bface_xyz.size());
  if (owner) std::memcpy(owner, m->bface_owner.data(), sizeof(int32_t) * m->bface_owner.size());
  return TCT_OK;
}

tct_status tct_mesh_rstar(const tct_mesh* m, int32_t* nnodes, int32_t* nlist, int32_t* height, float* box,
                          int32_t* link, int32_t* list) {
  if (!m) {
    set_error("null mesh");
    return TCT_E_ARG;
  }
  if (!m->has_rstar) {
    set_error("tct_mesh_rstar: mesh created without TCT_MESH_RSTAR");
    return TCT_E_ARG;
  }
  if (nnodes) *nnodes = (int32_t)m->rstar_nodes.size();
  if (nlist) *nlist = (int32_t)m->rstar_list.size();
  if (height) *height = m->rstar_height;
  for (size_t i = 0; i < m->rstar_nodes.size(); ++i) {
    const tct::BvhNode& nd = m->rstar_nodes[i];
    if (box)
      for (int k = 0; k < 3; ++k) {
        box[6 * i + k] = nd.lo[k];
        box[6 * i + 3 + k] = nd.hi[k];
      }
    if (link) {
      link[2 * i] = nd.skip;
      link[2 * i + 1] = nd.leaf;
    }
  }
  if (list) std::memcpy(list, m->rstar_list.data(), sizeof(int32_t) * m->rstar_list.size());
  return TCT_OK;
}

tct_status tct_mesh_permutation(const tct_mesh* m, int32_t* internal_to_user) {
  if (!m || !internal_to_user) {
    set_error("null argument");
    return TCT_E_ARG;
  }
  std::memcpy(internal_to_user, m->perm.data(), sizeof(int32_t) * m->perm.size());
  return TCT_OK;
}

tct_status tct_mesh_neighbors(const tct_mesh* m, int32_t* nbrs) {
  if (!m || !nbrs) {
    set_error("null argument");
    return TCT_E_ARG;
  }
  std::memcpy(nbrs, m->user_nbrs.data(), sizeof(int32_t) * m->user_nbrs.size());
  return TCT_OK;
}

tct_status tct_mesh_to_internal(const tct_mesh* m, const float* x_user, float* x_internal, tct_stream s) {
  tct_status st = need_device(m);
  if (st != TCT_OK) return st;
  if (!x_user || !x_internal || x_user == x_internal) {
    set_error("tct_mesh_to_internal: null or aliased arrays");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  return launch_permute(x_user, x_internal, m->d_perm, m->nt, 0, (hipStream_t)s);
}

tct_status tct_mesh_to_user(const tct_mesh* m, const float* x_internal, float* x_user, tct_stream s) {
  tct_status st = need_device(m);
  if (st != TCT_OK) return st;
  if (!x_user || !x_internal || x_user == x_internal) {
    set_error("tct_mesh_to_user: null or aliased arrays");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  return launch_permute(x_internal, x_user, m->d_perm, m->nt, 1, (hipStream_t)s);
}

tct_status tct_stats_read(const tct_mesh* m, tct_stats* out, int reset) {
  tct_status st = need_device(m);
  if (st != TCT_OK) return st;
  if (!out) {
    set_error("null stats output");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  unsigned long long h[kNumCounters];
  TCT_HIP(hipDeviceSynchronize());
  TCT_HIP(hipMemcpy(h, m->d_counters, sizeof(h), hipMemcpyDeviceToHost));
  out->rays = (int64_t)h[kRays];
  out->segments = (int64_t)h[kSegments];
  out->zero_len = (int64_t)h[kZeroLen];
  out->fp64_stage = (int64_t)h[kFp64Stage];
  out->exact_stage = (int64_t)h[kExactStage];
  out->perturbed_ties = (int64_t)h[kPerturbed];
  out->failed = (int64_t)h[kFailed];
  out->grazing_fp64 = (int64_t)h[kGrazing];
  if (reset) {
    unsigned long long z[kNumCounters] = {0};
    TCT_HIP(hipMemcpy(m->d_counters, z, sizeof(z), hipMemcpyHostToDevice));
  }
  if (out->failed > 0) {
    set_error("walk failures were counted");
    return TCT_E_WALK;
  }
  return TCT_OK;
}

void tct_mesh_destroy(tct_mesh* m) {
  if (!m) return;
  if (!m->host_only) {
    DeviceGuard dg(m->device);
    mesh_free_device(m);
  }
  delete m;
}

tct_status tct_geom_create(const tct_cone* cone, const double* angles_rad, int32_t na, int device, tct_geom** out) {
  if (!out) {
    set_error("tct_geom_create: null output handle");
    return TCT_E_ARG;
  }
  DeviceGuard dg(device);
  if (!dg.ok) {
    set_error("tct_geom_create: cannot select the device");
    return TCT_E_HIP;
  }
  return geom_build(cone, angles_rad, na, device, out);
}

int64_t tct_geom_nrays(const tct_geom* g) { return g ? g->nrays() : 0; }

tct_status tct_geom_frame(const tct_geom* g, float* S, float* D, float* U, float* V, float* u, float* v) {
  if (!g) {
    set_error("null geometry");
    return TCT_E_ARG;
  }
  for (int a = 0; a < g->na; ++a)
    for (int k = 0; k < 3; ++k) {
      const float* f = &g->frame[12 * (size_t)a];
      if (S) S[3 * a + k] = f[k];
      if (D) D[3 * a + k] = f[3 + k];
      if (U) U[3 * a + k] = f[6 + k];
      if (V) V[3 * a + k] = f[9 + k];
    }
  if (u) std::memcpy(u, g->ut.data(), 4 * g->ut.size());
  if (v) std::memcpy(v, g->vt.data(), 4 * g->vt.size());
  return TCT_OK;
}

void tct_geom_destroy(tct_geom* g) {
  if (!g) return;
  DeviceGuard dg(g->device);
  if (g->d_frame) (void)hipFree(g->d_frame);
  if (g->d_ut) (void)hipFree(g->d_ut);
  if (g->d_vt) (void)hipFree(g->d_vt);
  delete g;
}

tct_status tct_entry(const tct_mesh* m, const tct_geom* g, int32_t* entry, tct_stream s) {
  tct_status st = check_pair(m, g);
  if (st != TCT_OK) return st;
  if (!entry) {
    set_error("tct_entry: null output");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  return launch_pixel_walk(kModeEntry, m, g, 0, g->na, nullptr, nullptr, nullptr, entry, nullptr, default_tile_u(),
                           (hipStream_t)s);
}

tct_status tct_entry_rstar(const tct_mesh* m, const tct_geom* g, int32_t* entry, tct_stream s) {
  tct_status st = check_pair(m, g);
  if (st != TCT_OK) return st;
  if (!entry) {
    set_error("tct_entry_rstar: null output");
    return TCT_E_ARG;
  }
  if (!m->has_rstar) {
    set_error("tct_entry_rstar: mesh created without TCT_MESH_RSTAR");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  return launch_pixel_walk(kModeEntryRstar, m, g, 0, g->na, nullptr, nullptr, nullptr, entry, nullptr,
                           default_tile_u(), (hipStream_t)s);
}

tct_status tct_entry_raster(const tct_mesh* m, const tct_geom* g, int32_t* entry, tct_stream s) {
  tct_status st = check_pair(m, g);
  if (st != TCT_OK) return st;
  if (!entry) {
    set_error("tct_entry_raster: null output");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  return entry_raster(m, g, entry, (hipStream_t)s);
}

namespace {
tct_status check_range(const tct_geom* g, const tct_range* r) {
  if (!r || r->a0 < 0 || r->na < 0 || r->a0 + r->na > g->na) {
    set_error("tct_range: angles out of range");
    return TCT_E_ARG;
  }
  if (r->tile_u != 4 && r->tile_u != 8 && r->tile_u != 16 && r->tile_u != 32 && r->tile_u != 64) {
    set_error("tct_range: tile_u must be 4, 8, 16, 32 or 64");
    return TCT_E_ARG;
  }
  return TCT_OK;
}
}  // namespace

tct_status tct_forward_range(const tct_mesh* m, const tct_geom* g, const float* x, float* proj, const int32_t* entry,
                             const tct_range* r, tct_stream s) {
  tct_status st = check_pair(m, g);
  if (st != TCT_OK) return st;
  if ((st = check_range(g, r)) != TCT_OK) return st;
  if (!x || !proj) {
    set_error("tct_forward_range: null input or output");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  return launch_pixel_walk(kModeForward, m, g, r->a0, r->na, entry, x, proj, nullptr, nullptr, r->tile_u,
                           (hipStream_t)s);
}

tct_status tct_backproject_range(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int mode,
                                 int accumulate, const int32_t* entry, const tct_range* r, tct_stream s) {
  tct_status st = check_pair(m, g);
  if (st != TCT_OK) return st;
  if ((st = check_range(g, r)) != TCT_OK) return st;
  if (!proj || !xhat) {
    set_error("tct_backproject_range: null input or output");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  if (mode == TCT_BP_GATHER)
    return backproject_gather(m, g, proj, xhat, accumulate, entry, r->tile_u, r->a0, r->na, (hipStream_t)s);
  if (mode == TCT_BP_SHADOW) return backproject_shadow(m, g, proj, xhat, accumulate, r->a0, r->na, (hipStream_t)s);
  if (mode == TCT_BP_FIXED)
    return backproject_fixed(m, g, proj, xhat, accumulate, entry, r->tile_u, r->a0, r->na, (hipStream_t)s);
  if (mode != TCT_BP_ATOMIC && mode != TCT_BP_ATOMIC_DIRECT) {
    set_error("tct_backproject_range: unknown mode");
    return TCT_E_ARG;
  }
  if (!accumulate) {
    st = launch_fill(xhat, m->nt, 0.f, (hipStream_t)s);
    if (st != TCT_OK) return st;
  }
  return launch_pixel_walk(kModeBackAtomic, m, g, r->a0, r->na, entry, proj, xhat, nullptr, nullptr, r->tile_u,
                           (hipStream_t)s, mode == TCT_BP_ATOMIC);
}

tct_status tct_forward(const tct_mesh* m, const tct_geom* g, const float* x, float* proj, const int32_t* entry,
                       tct_stream s) {
  tct_status st = check_pair(m, g);
  if (st != TCT_OK) return st;
  if (!x || !proj) {
    set_error("tct_forward: null input or output");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  return launch_pixel_walk(kModeForward, m, g, 0, g->na, entry, x, proj, nullptr, nullptr, default_tile_u(),
                           (hipStream_t)s);
}

tct_status tct_backproject(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int mode,
                           int accumulate, const int32_t* entry, tct_stream s) {
  tct_status st = check_pair(m, g);
  if (st != TCT_OK) return st;
  if (!proj || !xhat) {
    set_error("tct_backproject: null input or output");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  if (mode == TCT_BP_GATHER)
    return backproject_gather(m, g, proj, xhat, accumulate, entry, default_tile_u(), 0, g->na, (hipStream_t)s);
  if (mode == TCT_BP_SHADOW) return backproject_shadow(m, g, proj, xhat, accumulate, 0, g->na, (hipStream_t)s);
  if (mode == TCT_BP_FIXED)
    return backproject_fixed(m, g, proj, xhat, accumulate, entry, default_tile_u(), 0, g->na, (hipStream_t)s);
  if (mode != TCT_BP_ATOMIC && mode != TCT_BP_ATOMIC_DIRECT) {
    set_error("tct_backproject: unknown mode");
    return TCT_E_ARG;
  }
  return backproject_atomic(m, g, proj, xhat, accumulate, entry, default_tile_u(), mode == TCT_BP_ATOMIC,
                            (hipStream_t)s);
}

tct_status tct_backproject_fixed_noalloc(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat,
                                         int accumulate, const int32_t* entry, tct_stream s) {
  tct_status st = check_pair(m, g);
  if (st != TCT_OK) return st;
  if (!proj || !xhat) {
    set_error("tct_backproject_fixed_noalloc: null input or output");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  return backproject_fixed_noalloc(m, g, proj, xhat, accumulate, entry, default_tile_u(), (hipStream_t)s);
}

tct_status tct_forward_paper(const tct_mesh* m, const tct_geom* g, const float* x, float* proj, const int32_t* entry,
                             int precision, tct_paper_stats* stats, tct_stream s) {
  tct_status st = check_pair(m, g);
  if (st != TCT_OK) return st;
  if (!x || !proj || !entry) {
    set_error("tct_forward_paper: null input, output or entry cache");
    return TCT_E_ARG;
  }
  if (precision != 32 && precision != 64) {
    set_error("tct_forward_paper: precision must be 32 or 64");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  return forward_paper(m, g, x, proj, entry, precision, stats, (hipStream_t)s);
}

namespace {
tct_status trace_common(const tct_mesh* m, const tct_geom* g, const int64_t* ids, const float* S, const float* P,
                        const float* U, const float* V, int32_t n, int64_t* offsets, int32_t* tets, float* lens,
                        int64_t cap, int64_t* needed, hipStream_t s) {
  if (n < 0 || !offsets || (cap > 0 && (!tets || !lens))) {
    set_error("tct_trace: bad arguments");
    return TCT_E_ARG;
  }
  if (n == 0) {
    int64_t z = 0;
    TCT_HIP(hipMemcpyAsync(offsets, &z, 8, hipMemcpyHostToDevice, s));
    TCT_HIP(hipStreamSynchronize(s));
    if (needed) *needed = 0;
    return TCT_OK;
  }
  int64_t* counts = nullptr;
  TCT_HIP(hipMallocAsync((void**)&counts, sizeof(int64_t) * (size_t)n, s));
  tct_status st = launch_list_walk(kModeCountAll, m, g, ids, S, P, U, V, n, counts, nullptr, nullptr, nullptr, s);
  std::vector<int64_t> h(n), off(n + 1);
  if (st == TCT_OK) {
    if (hipMemcpyAsync(h.data(), counts, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = hip_fail(hipGetLastError(), "tct_trace: count copy");
  }
  (void)hipFreeAsync(counts, s);
  if (st != TCT_OK) return st;
  off[0] = 0;
  for (int32_t i = 0; i < n; ++i) off[i + 1] = off[i] + h[i];
  TCT_HIP(hipMemcpyAsync(offsets, off.data(), sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice, s));
  if (needed) *needed = off[n];
  if (off[n] > cap) {
    TCT_HIP(hipStreamSynchronize(s));
    set_error("tct_trace: output capacity too small");
    return TCT_E_CAPACITY;
  }
  st = launch_list_walk(kModeTrace, m, g, ids, S, P, U, V, n, nullptr, offsets, tets, lens, s);
  if (st != TCT_OK) return st;
  TCT_HIP(hipStreamSynchronize(s));
  return TCT_OK;
}
}  // namespace

tct_status tct_trace(const tct_mesh* m, const tct_geom* g, const int64_t* ray_ids, int32_t nrays, int64_t* offsets,
                     int32_t* tets, float* lengths, int64_t cap, int64_t* needed, tct_stream s) {
  tct_status st = check_pair(m, g);
  if (st != TCT_OK) return st;
  if (!ray_ids && nrays > 0) {
    set_error("tct_trace: null ray ids");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  return trace_common(m, g, ray_ids, nullptr, nullptr, nullptr, nullptr, nrays, offsets, tets, lengths, cap, needed,
                      (hipStream_t)s);
}

tct_status tct_trace_rays(const tct_mesh* m, const float* S, const float* P, const float* U, const float* V,
                          int32_t n, int64_t* offsets, int32_t* tets, float* lengths, int64_t cap, int64_t* needed,
                          tct_stream s) {
  tct_status st = need_device(m);
  if (st != TCT_OK) return st;
  if (n > 0 && (!S || !P || !U || !V)) {
    set_error("tct_trace_rays: null ray arrays");
    return TCT_E_ARG;
  }
  DeviceGuard dg(m->device);
  return trace_common(m, nullptr, nullptr, S, P, U, V, n, offsets, tets, lengths, cap, needed, (hipStream_t)s);
}

tct_status tct_dot(const float* a, const float* b, int64_t n, double* result, double* workspace, tct_stream s) {
  if (!a || !b || !result || !workspace || n < 0) {
    set_error("tct_dot: bad arguments");
    return TCT_E_ARG;
  }
  return blas_dot(a, b, n, result, workspace, (hipStream_t)s);
}

tct_status tct_axpy_ratio(float* y, const float* x, int64_t n, const double* num, const double* den, double sign,
                          tct_stream s) {
  if (!y || !x || !num || !den || n < 0) {
    set_error("tct_axpy_ratio: bad arguments");
    return TCT_E_ARG;
  }
  return blas_axpy_ratio(y, x, n, num, den, sign, (hipStream_t)s);
}

tct_status tct_xpay_ratio(float* p, const float* x, int64_t n, const double* num, const double* den, tct_stream s) {
  if (!p || !x || !num || !den || n < 0) {
    set_error("tct_xpay_ratio: bad arguments");
    return TCT_E_ARG;
  }
  return blas_xpay_ratio(p, x, n, num, den, (hipStream_t)s);
}

tct_status tct_axpby(float* y, const float* x, int64_t n, float a, float b, tct_stream s) {
  if (!y || !x || n < 0) {
    set_error("tct_axpby: bad arguments");
    return TCT_E_ARG;
  }
  return blas_axpby(y, x, n, a, b, (hipStream_t)s);
}

tct_status tct_mul(float* y, const float* a, const float* b, int64_t n, tct_stream s) {
  if (!y || !a || !b || n < 0) {
    set_error("tct_mul: bad arguments");
    return TCT_E_ARG;
  }
  return blas_mul(y, a, b, n, (hipStream_t)s);
}

tct_status tct_recip(float* y, const float* a, int64_t n, float eps, tct_stream s) {
  if (!y || !a || n < 0) {
    set_error("tct_recip: bad arguments");
    return TCT_E_ARG;
  }
  return blas_recip(y, a, n, eps, (hipStream_t)s);
}

tct_status tct_copy_f64(double* dst, const double* src, int32_t n, tct_stream s) {
  if (!dst || !src || n < 0) {
    set_error("tct_copy_f64: bad arguments");
    return TCT_E_ARG;
  }
  return blas_copy_f64(dst, src, n, (hipStream_t)s);
}

tct_status tct_vecset_create(int32_t n, float* const* ptrs, const int64_t* lens, int device, tct_vecset** out) {
  if (!out || n < 0 || (n > 0 && (!ptrs || !lens))) {
    set_error("tct_vecset_create: bad arguments");
    return TCT_E_ARG;
  }
  *out = nullptr;
  for (int k = 0; k < n; ++k)
    if (!ptrs[k] || lens[k] < 0) {
      set_error("tct_vecset_create: null vector or negative length");
      return TCT_E_ARG;
    }
  DeviceGuard dg(device);
  tct_vecset* v = new tct_vecset();
  v->device = device;
  v->n = n;
  v->ptrs.assign(ptrs, ptrs + n);
  v->lens.assign(lens, lens + n);
  size_t np = sizeof(float*) * (size_t)std::max(n, 1), nl = sizeof(int64_t) * (size_t)std::max(n, 1);
  if (hipMalloc((void**)&v->d_ptrs, np) != hipSuccess || hipMalloc((void**)&v->d_lens, nl) != hipSuccess ||
      (n > 0 && (hipMemcpy(v->d_ptrs, ptrs, sizeof(float*) * n, hipMemcpyHostToDevice) != hipSuccess ||
                 hipMemcpy(v->d_lens, lens, sizeof(int64_t) * n, hipMemcpyHostToDevice) != hipSuccess))) {
    if (v->d_ptrs) (void)hipFree(v->d_ptrs);
    if (v->d_lens) (void)hipFree(v->d_lens);
    delete v;
    set_error("tct_vecset_create: device allocation failed");
    return TCT_E_NOMEM;
  }
  *out = v;
  return TCT_OK;
}

void tct_vecset_destroy(tct_vecset* v) {
  if (!v) return;
  DeviceGuard dg(v->device);
  if (v->d_ptrs) (void)hipFree(v->d_ptrs);
  if (v->d_lens) (void)hipFree(v->d_lens);
  delete v;
}

namespace {
tct_status check_sets(const tct_vecset* a, const tct_vecset* b, const char* what) {
  if (!a || !b || a->n != b->n || a->device != b->device) {
    set_error(std::string(what) + ": vector sets differ in count or device");
    return TCT_E_ARG;
  }
  for (int k = 0; k < a->n; ++k)
    if (a->lens[k] != b->lens[k]) {
      set_error(std::string(what) + ": vector lengths differ at " + std::to_string(k));
      return TCT_E_ARG;
    }
  return TCT_OK;
}
}  // namespace

tct_status tct_vecset_dot(const tct_vecset* a, const tct_vecset* b, double* results, double* workspace,
                          tct_stream s) {
  tct_status st = check_sets(a, b, "tct_vecset_dot");
  if (st != TCT_OK) return st;
  if (!results || !workspace) {
    set_error("tct_vecset_dot: null output");
    return TCT_E_ARG;
  }
  DeviceGuard dg(a->device);
  return vecset_dot(a, b, results, workspace, (hipStream_t)s);
}

tct_status tct_vecset_axpy_ratio(const tct_vecset* y, const tct_vecset* x, const double* num, const double* den,
                                 double sign, tct_stream s) {
  tct_status st = check_sets(y, x, "tct_vecset_axpy_ratio");
  if (st != TCT_OK) return st;
  if (!num || !den) {
    set_error("tct_vecset_axpy_ratio: null scalars");
    return TCT_E_ARG;
  }
  DeviceGuard dg(y->device);
  return vecset_axpy_ratio(y, x, num, den, sign, (hipStream_t)s);
}

tct_status tct_vecset_xpay_ratio(const tct_vecset* p, const tct_vecset* x, const double* num, const double* den,
                                 tct_stream s) {
  tct_status st = check_sets(p, x, "tct_vecset_xpay_ratio");
  if (st != TCT_OK) return st;
  if (!num || !den) {
    set_error("tct_vecset_xpay_ratio: null scalars");
    return TCT_E_ARG;
  }
  DeviceGuard dg(p->device);
  return vecset_xpay_ratio(p, x, num, den, (hipStream_t)s);
}

tct_status tct_vecset_fill(const tct_vecset* y, float value, tct_stream s) {
  if (!y) {
    set_error("tct_vecset_fill: null set");
    return TCT_E_ARG;
  }
  DeviceGuard dg(y->device);
  return vecset_fill(y, value, (hipStream_t)s);
}

tct_status tct_batch_create(const tct_mesh* const* meshes, const tct_geom* const* geoms, int32_t n,
                            const int32_t* tile_u, int32_t* const* entries, tct_batch** out) {
  if (!out || !meshes || !geoms || n <= 0) {
    set_error("tct_batch_create: bad arguments");
    return TCT_E_ARG;
  }
  *out = nullptr;
  for (int k = 0; k < n; ++k) {
    tct_status st = check_pair(meshes[k], geoms[k]);
    if (st != TCT_OK) return st;
    if (meshes[k]->device != meshes[0]->device) {
      set_error("tct_batch_create: problems on different devices");
      return TCT_E_ARG;
    }
    if (tile_u) {
      int t = tile_u[k];
      if (t != 4 && t != 8 && t != 16 && t != 32 && t != 64) {
        set_error("tct_batch_create: tile_u must be 4, 8, 16, 32 or 64");
        return TCT_E_ARG;
      }
    }
  }
  DeviceGuard dg(meshes[0]->device);
  return batch_build(meshes, geoms, n, tile_u, entries, out);
}

namespace {
tct_status check_batch_sets(const tct_batch* b, const tct_vecset* xs, const tct_vecset* ps) {
  if (!b || !xs || !ps || xs->n != b->n || ps->n != b->n || xs->device != b->device || ps->device != b->device) {
    set_error("batch: vector sets do not match the batch");
    return TCT_E_ARG;
  }
  for (int k = 0; k < b->n; ++k)
    if (xs->lens[k] != b->meshes[k]->nt || ps->lens[k] != b->geoms[k]->nrays()) {
      set_error("batch: vector " + std::to_string(k) + " has the wrong length");
      return TCT_E_ARG;
    }
  return TCT_OK;
}
}  // namespace

tct_status tct_batch_forward(tct_batch* b, const tct_vecset* x, const tct_vecset* proj, tct_stream s) {
  tct_status st = check_batch_sets(b, x, proj);
  if (st != TCT_OK) return st;
  DeviceGuard dg(b->device);
  return batch_walk(b, kModeForward, x, proj, (hipStream_t)s);
}

tct_status tct_batch_backproject(tct_batch* b, const tct_vecset* proj, const tct_vecset* xhat, int accumulate,
                                 tct_stream s) {
  tct_status st = check_batch_sets(b, xhat, proj);
  if (st != TCT_OK) return st;
  DeviceGuard dg(b->device);
  if (!accumulate) {
    st = vecset_fill(xhat, 0.f, (hipStream_t)s);
    if (st != TCT_OK) return st;
  }
  return batch_walk(b, kModeBackAtomic, proj, xhat, (hipStream_t)s);
}

tct_status tct_batch_set_queue_chunk(tct_batch* b, int32_t blocks_per_fetch) {
  if (!b || blocks_per_fetch < 1 || blocks_per_fetch > 64) {
    set_error("tct_batch_set_queue_chunk: blocks per fetch must be 1..64");
    return TCT_E_ARG;
  }
  b->queue_chunk = blocks_per_fetch;
  return TCT_OK;
}

int64_t tct_batch_items(const tct_batch* b) { return b ? b->total_items : 0; }

void tct_batch_destroy(tct_batch* b) {
  if (!b) return;
  DeviceGuard dg(b->device);
  batch_free(b);
}

}  // extern "C"

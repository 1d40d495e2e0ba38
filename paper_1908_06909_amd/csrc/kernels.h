// Kernel launchers (walk.hip, gather.hip, shadow.hip, paper_mode.hip) used by the C interface.
#pragma once

#include "common.h"

namespace tct {

enum WalkMode {
  kModeEntry = 0,
  kModeForward = 1,
  kModeBackAtomic = 2,
  kModeCountAll = 3,
  kModeTrace = 5,
  kModeGatherFill = 6,
  kModeBackDirect = 7,  // backprojection with one global atomic per segment
  kModeEntryRstar = 8,  // entry search through the R*-tree
  kModeBackFixed = 9,   // backprojection through the block table into 64-bit fixed-point sums (reproducible)
};

// Explicit per-tetrahedron lists (TCT_BP_GATHER): records of one chunk of
// angles, each the exact fixed-point sum m 2^-scale over the rays of one
// wavefront and one window of steps that cross tetrahedron `tet` with
// positive length (scale: the wavefront's, a power of two).  One 16-byte
// record, written and moved with single 16-byte accesses.
struct alignas(16) GatherRecord {
  long long m;
  int32_t tet;
  int32_t scale;
};
// The fill walk's output: counts[tet] counts the tetrahedron's records.
// Each workgroup writes its records into one of kGatherGroups regions of
// rec (gcap records each; the region a hash of the block index),
// positions handed out by that region's cursor, so no single counter
// serialises the whole launch; cursor[g] counts all of the
// region's records, also those beyond gcap, which are not written.
constexpr int kGatherGroups = 64;
struct GatherOut {
  GatherRecord* rec;
  int32_t* counts;
  unsigned long long* cursor;  // [kGatherGroups]
  int64_t gcap;
};

tct_status launch_pixel_walk(int mode, const tct_mesh* m, const tct_geom* g, int a0, int na_chunk,
                             const int32_t* entry, const float* in, float* out_f32, int32_t* out_i32,
                             const GatherOut* gather, int tile_u, hipStream_t s, int lds_table = 0,
                             unsigned long long* acc64 = nullptr, const int* scale_exp = nullptr);

tct_status backproject_atomic(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int accumulate,
                              const int32_t* entry, int tile_u, int lds_table, hipStream_t s);

tct_status launch_list_walk(int mode, const tct_mesh* m, const tct_geom* g, const int64_t* ids, const float* S,
                            const float* P, const float* U, const float* V, int32_t n, int64_t* counts,
                            const int64_t* offsets, int32_t* tets, float* lens, hipStream_t s);

tct_status launch_fill(float* p, int64_t n, float v, hipStream_t s);
// Wavefronts of a pixel-walk launch over na_chunk angles (four per block).
int64_t pixel_walk_waves(const tct_geom* g, int na_chunk, int tile_u);
tct_status entry_raster(const tct_mesh* m, const tct_geom* g, int32_t* entry, hipStream_t s);
tct_status launch_permute(const float* in, float* out, const int32_t* perm, int n, int scatter, hipStream_t s);

tct_status backproject_fixed(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int accumulate,
                             const int32_t* entry, int tile_u, int a_begin, int a_count, hipStream_t s);
tct_status backproject_fixed_noalloc(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat,
                                     int accumulate, const int32_t* entry, int tile_u, hipStream_t s);

tct_status backproject_gather(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int accumulate,
                              const int32_t* entry, int tile_u, int a_begin, int a_count, hipStream_t s);

tct_status backproject_shadow(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int accumulate,
                              int a_begin, int a_count, hipStream_t s);

tct_status forward_paper(const tct_mesh* m, const tct_geom* g, const float* x, float* proj, const int32_t* entry,
                         int precision, tct_paper_stats* stats, hipStream_t s);

tct_status batch_build(const tct_mesh* const* meshes, const tct_geom* const* geoms, int32_t n, const int32_t* tile_u,
                       int32_t* const* entries, tct_batch** out);
void batch_free(tct_batch* b);
tct_status batch_walk(tct_batch* b, int mode, const tct_vecset* in, const tct_vecset* out, hipStream_t s);

tct_status vecset_dot(const tct_vecset* a, const tct_vecset* b, double* results, double* workspace, hipStream_t s);
tct_status vecset_axpy_ratio(const tct_vecset* y, const tct_vecset* x, const double* num, const double* den,
                             double sign, hipStream_t s);
tct_status vecset_xpay_ratio(const tct_vecset* p, const tct_vecset* x, const double* num, const double* den,
                             hipStream_t s);
tct_status vecset_fill(const tct_vecset* y, float v, hipStream_t s);

tct_status exclusive_scan_counts(const int32_t* in, int64_t* out, int64_t n, int64_t* sums, hipStream_t s);

// Host-side builders (mesh.cpp).
tct_status mesh_build(const float* verts, int32_t nv, const int32_t* tets, int32_t nt, const int32_t* nbrs,
                      uint32_t flags, int device, tct_mesh** out);
void mesh_free_device(tct_mesh* m);
tct_status geom_build(const tct_cone* cone, const double* angles, int32_t na, int device, tct_geom** out);
tct_status check_geometry(const tct_mesh* m, const tct_geom* g);

int default_tile_u();

tct_status blas_dot(const float* a, const float* b, int64_t n, double* result, double* workspace, hipStream_t s);
tct_status blas_axpy_ratio(float* y, const float* x, int64_t n, const double* num, const double* den, double sign,
                           hipStream_t s);
tct_status blas_xpay_ratio(float* p, const float* x, int64_t n, const double* num, const double* den, hipStream_t s);
tct_status blas_axpby(float* y, const float* x, int64_t n, float a, float b, hipStream_t s);
tct_status blas_mul(float* y, const float* a, const float* b, int64_t n, hipStream_t s);
tct_status blas_recip(float* y, const float* a, int64_t n, float eps, hipStream_t s);
tct_status blas_copy_f64(double* dst, const double* src, int n, hipStream_t s);

}  // namespace tct

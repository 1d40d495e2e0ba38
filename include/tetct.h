/*
 * tetct: tetrahedral-mesh cone-beam CT projector for AMD Instinct MI355X (gfx950).
 *
 * The operator is the linear CT model A x = b of Biguri et al.,
 * "Numerically robust tetrahedron-based tomographic forward and backward
 * projectors on parallel architectures" (Section II-A, Eq. 1): the entry
 * a_ij of A is the length of ray j inside tetrahedron i, x holds one
 * attenuation value per tetrahedron and b one value per detector pixel and
 * angle.  A is never stored; each call recomputes a_ij by walking every ray
 * through the mesh (Section II-A, matrix-free operator; Section II-D,
 * Algorithm 2).
 *
 * Conventions shared by every call
 *   - Plain C99.  All functions return tct_status (0 = success) unless noted.
 *     On error, tct_last_error() gives a message (thread-local, valid until the
 *     next call on the same thread).  No exceptions cross this interface and
 *     nothing calls exit().
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the device the handle was created for.  Device arrays
 *     are caller-owned unless stated: the library never frees them.
 *   - float is IEEE-754 binary32, double binary64, ids are int32 (-1 = none).
 *   - Face k of a tetrahedron is the face opposite its vertex k; neighbour k
 *     is the tetrahedron across face k (the paper's element graph, Section
 *     II-B, Fig. 1: nD+1 nodes and nD+1 ordered neighbours per element).
 *   - tct_stream is a hipStream_t (NULL = the default stream).  Compute calls
 *     are asynchronous on that stream; argument errors are reported
 *     synchronously before anything is enqueued.
 *   - Tetrahedron-indexed device arrays (x, xhat) use the library's
 *     *internal* order (a spatial reordering made at mesh creation).
 *     tct_mesh_to_internal / tct_mesh_to_user convert; tct_mesh_permutation
 *     exports the map.
 *   - Rays: ray id r = (a * nv + j) * nu + i for angle a, detector row j and
 *     column i; projections are laid out proj[a][j][i] (float, i fastest).
 *     Ray r runs from the source point S to the pixel centre P (Algorithm 2's
 *     R1, R2).  a_ij is computed for t in [0, 1] along S + t (P - S); the
 *     whole mesh must lie strictly between the source and the detector plane
 *     (checked: TCT_E_GEOM).  Rays that miss the mesh give 0.
 *   - Ties (rays through vertices, along edges, inside face planes) are
 *     resolved as the limit of the ray translated by eps*U + eps^2*V,
 *     eps -> 0+, U and V the detector axes of the ray's angle: every ray then
 *     has one well-defined sequence of visited tetrahedra, zero-length
 *     passages included (Fig. 3), and lengths that add up to its chord.
 */
#ifndef TETCT_H
#define TETCT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* tct_stream; /* hipStream_t */
typedef struct tct_mesh tct_mesh;
typedef struct tct_geom tct_geom;
typedef struct tct_batch tct_batch;
typedef struct tct_vecset tct_vecset;

typedef enum {
  TCT_OK = 0,
  TCT_E_ARG = -1,              /* bad argument (null pointer, size, id out of range) */
  TCT_E_MESH_DEGENERATE = -2,  /* a tetrahedron has zero volume */
  TCT_E_MESH_NONMANIFOLD = -3, /* a face shared by >2 tetrahedra, or an open/inconsistent boundary */
  TCT_E_MESH_NONCONVEX = -4,   /* the hull is not convex (the method requires it, Section II-D) */
  TCT_E_MESH_DISCONNECTED = -5,/* the boundary surface has more than one component */
  TCT_E_GEOM = -6,             /* the mesh is not strictly between source and detector */
  TCT_E_NOMEM = -7,            /* device or host allocation failed */
  TCT_E_HIP = -8,              /* a HIP runtime call failed */
  TCT_E_WALK = -9,             /* device walk failures were counted (see tct_stats) */
  TCT_E_CAPACITY = -10         /* an output buffer is too small (required size reported) */
} tct_status;

/* Circular cone-beam geometry (the paper's experiments, Section III-A: cone
 * beam, circular trajectory, equidistant angles).  Rotation is about +z.  For
 * angle theta: source S = dso (cos, sin, 0); detector centre
 * D = -(dsd - dso) (cos, sin, 0); U = (-sin, cos, 0); V = (0, 0, 1).  Pixel
 * centres: u_i = (i - (nu-1)/2) du + off_u, v_j = (j - (nv-1)/2) dv + off_v,
 * P = D + u_i U + v_j V.  cos/sin are evaluated in double and replaced by the
 * exact 0/+-1 within 1e-12 of a quarter turn; every vector is then rounded to
 * float, and P is formed in float as fl(fl(D + fl(u U)) + fl(v V)) without
 * fused multiply-add. */
typedef struct {
  double dso, dsd;
  int32_t nu, nv;
  double du, dv, off_u, off_v;
} tct_cone;

/* Device-side counters accumulated by every walk on a mesh since the last
 * reset.  segments counts visited tetrahedra (zero-length passages
 * included); fp64_stage counts sign tests the float32 filter could not
 * certify; exact_stage those the float64 filter could not certify either;
 * perturbed_ties those decided by the eps*U / eps^2*V terms; failed counts
 * rays that stopped without leaving the mesh (should stay 0); grazing_fp64
 * counts exit crossings recomputed in float64 because the face was nearly
 * parallel to the ray. */
typedef struct {
  int64_t rays, segments, zero_len, fp64_stage, exact_stage, perturbed_ties, failed, grazing_fp64;
} tct_stats;

/* ---------------------------------------------------------------- mesh */

/* Flags for tct_mesh_create. */
#define TCT_MESH_NO_REORDER 1u /* keep the user's tetrahedron order as the internal order */
#define TCT_MESH_HOST_ONLY 2u  /* build and validate on the host only; no device upload (compute calls fail) */
#define TCT_MESH_RSTAR 4u      /* also build the R*-tree over the boundary faces (tct_entry_rstar) */

/* Build a mesh from nodes and elements (Section II-B).
 *   verts  host float [nv][3]  node coordinates
 *   tets   host int32 [nt][4]  node ids of each tetrahedron, any orientation
 *   nbrs   host int32 [nt][4]  neighbour across face k, -1 on the boundary, or
 *                              NULL to compute them; when given they are checked
 *   device HIP device ordinal
 * Inputs are copied; the caller may free them on return.  Validation:
 * ids in range, non-zero volume (exact), each face shared by at most two
 * tetrahedra, a closed, connected, convex boundary (exact tests at every
 * boundary edge).  Tetrahedra are reordered along a Morton curve of their
 * centroids unless TCT_MESH_NO_REORDER.  Builds the boundary-face list
 * (Section II-B) and a bounding-volume hierarchy over it (entry search,
 * Section II-E).  On error *out is set to NULL. */
tct_status tct_mesh_create(const float* verts, int32_t nv, const int32_t* tets, int32_t nt, const int32_t* nbrs,
                           uint32_t flags, int device, tct_mesh** out);

/* Boundary faces in entry-id order (the ids tct_entry returns).
 *   xyz    host float [nboundary][3][3]  vertices, ordered so that (p1 - p0) x (p2 - p0) points out of the mesh
 *   owner  host int32 [nboundary]        user id of the tetrahedron the face belongs to
 * Either pointer may be NULL. */
tct_status tct_mesh_boundary(const tct_mesh* m, float* xyz, int32_t* owner);

/* The R*-tree built with TCT_MESH_RSTAR (Section II-E: nodes of 4 to 10
 * entries; R* insertion rules with forced reinsertion), flattened in
 * depth-first preorder: an interior node's first child is the next node,
 * skip is the node after its subtree (-1 at the end).
 *   nnodes, nlist, height  host int32 out: node count, leaf-list length, levels (leaves included)
 *   box    host float [nnodes][6]  lo xyz, hi xyz (face boxes padded outward)
 *   link   host int32 [nnodes][2]  skip, leaf field (-1 interior; else first * 16 + count into list)
 *   list   host int32 [nlist]      boundary-face ids of the leaves
 * Call with NULL arrays to get the sizes.  TCT_E_ARG if the mesh has no R*-tree. */
tct_status tct_mesh_rstar(const tct_mesh* m, int32_t* nnodes, int32_t* nlist, int32_t* height, float* box,
                          int32_t* link, int32_t* list);

/* Sizes of the element graph (Section II-B: nodes, elements and the boundary
 * elements the entry search starts from): node count, tetrahedron count,
 * boundary faces, device bytes held.  Any pointer may be NULL; TCT_E_ARG for a
 * null mesh. */
tct_status tct_mesh_counts(const tct_mesh* m, int32_t* nv, int32_t* nt, int32_t* nboundary, int64_t* device_bytes);

/* The element order of the internal layout (not in the paper: the library
 * reorders the elements of Section II-B along a Morton curve so that
 * neighbours across faces sit close in memory).
 *   internal_to_user  host int32 [nt], caller-owned: user id of each internal tetrahedron
 * TCT_E_ARG for a null mesh or output. */
tct_status tct_mesh_permutation(const tct_mesh* m, int32_t* internal_to_user);

/* The ordered neighbour list of Section II-B (Fig. 1) as the library built or
 * checked it: host int32 [nt][4], caller-owned, the neighbour (user ids, -1 on
 * the boundary) across face k of each user tetrahedron, faces numbered by the
 * user's vertex order.  TCT_E_ARG for a null mesh or output. */
tct_status tct_mesh_neighbors(const tct_mesh* m, int32_t* nbrs);

/* Per-element values (x of Eq. 2, xhat of Eq. 3) between the user's element
 * order and the internal one: device float [nt] each, caller-owned, not
 * aliased; x_internal[i] = x_user[perm[i]]  /  x_user[perm[i]] = x_internal[i]
 * with perm from tct_mesh_permutation.  Asynchronous on s; TCT_E_ARG for null
 * pointers or a host-only mesh. */
tct_status tct_mesh_to_internal(const tct_mesh* m, const float* x_user, float* x_internal, tct_stream s);
tct_status tct_mesh_to_user(const tct_mesh* m, const float* x_internal, float* x_user, tct_stream s);

/* Walk counters since the last reset (see tct_stats).  The paper requires that
 * no ray halts or loops inside the mesh (Section II-C, the failure cases of
 * Fig. 3); `failed` counts rays that did, so a caller can detect them.
 *   out    host, filled (may be NULL)
 *   reset  non-zero: zero the counters after reading
 * Synchronises the device.  Returns TCT_E_WALK when failed > 0 (the counters
 * are still written); TCT_E_ARG for a null or host-only mesh. */
tct_status tct_stats_read(const tct_mesh* m, tct_stats* out, int reset);

/* Frees the mesh and its device memory (NULL is a no-op).  No call using the
 * mesh may still be running on any stream. */
void tct_mesh_destroy(tct_mesh* m);

/* ---------------------------------------------------------------- geometry */

/* Circular cone-beam geometry with the given source angles (Section III-A:
 * cone beam on a circular trajectory; the rays of Algorithm 2 run from the
 * source R1 to each pixel centre R2).
 *   cone        host, see tct_cone
 *   angles_rad  host double [na], any values (the experiments use equidistant ones)
 *   device      HIP device ordinal; frames and pixel tables are copied there
 * The host arrays are copied; the handle owns its device memory until
 * tct_geom_destroy.  TCT_E_ARG unless na, nu, nv >= 1 and 0 < dso < dsd, or
 * for 2^40 rays or more; TCT_E_HIP / TCT_E_NOMEM when the upload fails.  Whether a mesh lies between source and detector is
 * checked when both are used together (TCT_E_GEOM). */
tct_status tct_geom_create(const tct_cone* cone, const double* angles_rad, int32_t na, int device, tct_geom** out);

/* Number of rays na * nv * nu (one per pixel and angle, Section III-A); 0 for NULL. */
int64_t tct_geom_nrays(const tct_geom* g);

/* The float32 frames the kernels build rays from (Section III-A geometry, the
 * rounding rule of tct_cone): host float S, D, U, V [na][3] and the pixel-centre
 * tables u [nu], v [nv], caller-owned; any pointer may be NULL. */
tct_status tct_geom_frame(const tct_geom* g, float* S, float* D, float* U, float* V, float* u, float* v);

/* Frees the geometry and its device memory (NULL is a no-op). */
void tct_geom_destroy(tct_geom* g);

/* ---------------------------------------------------------------- operators */

/* Entry faces (Section II-E: the boundary element each ray enters by).
 * entry: device int32 [nrays], boundary-face index or -1 for a miss.  The
 * array can be passed to the operators below to skip the search (it depends
 * only on the mesh and the geometry). */
tct_status tct_entry(const tct_mesh* m, const tct_geom* g, int32_t* entry, tct_stream s);

/* The same entry faces found through the R*-tree of Section II-E instead of
 * the bounding-volume hierarchy (the mesh must be created with
 * TCT_MESH_RSTAR, else TCT_E_ARG).  The result is identical: the exact entry
 * test admits one face per ray. */
tct_status tct_entry_rstar(const tct_mesh* m, const tct_geom* g, int32_t* entry, tct_stream s);

/* The same entry faces found by projecting the boundary instead of searching
 * a tree (Section II-E defines the entry face; the search structure is this
 * library's).  For each angle, every boundary face whose plane has the
 * source on its outer side is projected onto the detector plane in double
 * precision, and the pixels inside the bounding box of the projection,
 * widened by a twentieth of the pitch, are tested with the exact entry test
 * on their float32 rays.  The result is identical to tct_entry's: the exact
 * test admits one face per ray of a convex mesh.
 *   entry: device int32 [nrays], every element written (-1 for a miss)
 * Errors: TCT_E_ARG for a null output or a mesh/geometry device mismatch. */
tct_status tct_entry_raster(const tct_mesh* m, const tct_geom* g, int32_t* entry, tct_stream s);

/* Forward projection b_j = sum_i a_ij x_i (Eq. 2).
 *   x     device float [nt], internal order
 *   proj  device float [na][nv][nu], overwritten
 *   entry device int32 [nrays] from tct_entry, or NULL to search in-kernel */
tct_status tct_forward(const tct_mesh* m, const tct_geom* g, const float* x, float* proj, const int32_t* entry,
                       tct_stream s);

#define TCT_BP_ATOMIC 0        /* ray-driven float32 scatter (Section II-F); each wavefront (an 8x8-pixel tile)
                                  first sums its segments per tetrahedron in on-chip memory over windows of
                                  steps (64-bit fixed point scaled to the wavefront's largest |y_j| |P_j - S|:
                                  every term is kept to 2^-51 of it), then adds one float atomic per distinct
                                  tetrahedron to xhat */
#define TCT_BP_GATHER 1        /* deterministic: explicit per-tetrahedron lists of the wavefronts' exact
                                  fixed-point partial sums (one per wavefront and window of steps that crosses
                                  the tetrahedron), each list added exactly as 128-bit integers, so the sum does
                                  not depend on the order of the list */
#define TCT_BP_ATOMIC_DIRECT 2 /* one float32 atomic add to xhat per segment, as in the paper */
#define TCT_BP_FIXED 4         /* reproducible ray-driven scatter: the atomic walk with every term rounded to
                                  a multiple of 2^-s, one s per launch (terms stay below 2^K in magnitude,
                                  K = min(50, 62 - ceil(log2 rays))), so all sums are exact integers and the
                                  result is the same bits on every run; terms far below the launch's largest
                                  |y_j| |P_j - S| lose relative precision (quantum 2^-K times the power of
                                  two above it) */
#define TCT_BP_SHADOW 3        /* deterministic, element-driven: each tetrahedron enumerates the pixels of
                                  its detector shadow per angle, keeps the rays that cross it (the walk's
                                  exact predicate) and sums length x y_j in float64 in a fixed order
                                  (ray order, except elements with exact ties: per angle, then a fixed
                                  tree over angles) */

/* Backprojection xhat_i = sum_j a_ij y_j (Eq. 3 with the detector index on y).
 *   proj  device float [na][nv][nu]
 *   xhat  device float [nt], internal order; overwritten unless accumulate != 0
 *   mode  TCT_BP_ATOMIC, TCT_BP_ATOMIC_DIRECT, TCT_BP_GATHER or TCT_BP_SHADOW.
 *         The atomic modes sum in a run-dependent order.  GATHER and SHADOW give
 *         bitwise-identical results run to run.  GATHER allocates stream-ordered
 *         scratch and synchronises the stream once per angle chunk; SHADOW does
 *         not use `entry`, never synchronises, and allocates stream-ordered
 *         float64 partial sums only when the mesh has too few elements to fill
 *         the device (then angles are split into chunks summed in order). */
tct_status tct_backproject(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int mode,
                           int accumulate, const int32_t* entry, tct_stream s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * reproducible scatter of tct_backproject(mode = TCT_BP_FIXED), same arguments
 * and the same bits, without any allocation.  Its scratch (8 bytes per
 * tetrahedron plus 256) is a static device array sized for
 * TCT_NOALLOC_MAX_TETS tetrahedra (32 MiB), held by each GPU the library runs
 * on until the process ends; the first call on a device looks its address
 * up.  Every call on one GPU shares that array and clears what it needs at
 * its start, so calls that overlap in time on one GPU (several streams or
 * threads) race and give wrong results.  The caller still passes inputs and
 * outputs.
 *   Errors: TCT_E_ARG for null arguments, a mesh/geometry device mismatch or a
 *   mesh of more than TCT_NOALLOC_MAX_TETS tetrahedra; TCT_E_HIP when the
 *   scratch address cannot be looked up or a launch fails.  Asynchronous on s. */
#define TCT_NOALLOC_MAX_TETS 4194304
tct_status tct_backproject_fixed_noalloc(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat,
                                         int accumulate, const int32_t* entry, tct_stream s);

/* Launch options: the angles [a0, a0 + na) to process (projection arrays keep
 * their full [na_total][nv][nu] layout; other angles are not touched) and the
 * wavefront pixel tile width tile_u in {4, 8, 16, 32, 64} (tile height
 * 64 / tile_u; a 256-thread block covers 2 x 2 tiles).  The paper tuned its
 * pixel block shape per GPU and recommends re-tuning elsewhere (Section II-F). */
typedef struct {
  int32_t a0, na;
  int32_t tile_u;
} tct_range;

/* tct_forward / tct_backproject restricted to an angle range with a tile shape
 * (subset iterations such as OS-SART, and tile autotuning). */
tct_status tct_forward_range(const tct_mesh* m, const tct_geom* g, const float* x, float* proj, const int32_t* entry,
                             const tct_range* r, tct_stream s);
tct_status tct_backproject_range(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int mode,
                                 int accumulate, const int32_t* entry, const tct_range* r, tct_stream s);

/* Paper-faithful forward projection (Algorithms 1 and 2, Section II): the
 * Moller-Trumbore test with the safety parameter eps (from 1e-9, x10 per
 * failure to find two faces, halted past 1) on the four faces of each
 * tetrahedron, stepping across the face with the larger parameter, in
 * float32 (precision 32) or float64 (64) arithmetic.  For comparison with the
 * exact walk (the paper's single versus double precision experiment, Section
 * III-C); rays that halt or exceed 16384 steps keep their partial sums.
 *   x          device float [nt], internal order
 *   proj       device float [na][nv][nu], overwritten
 *   entry      device int32 [nrays] from tct_entry (required)
 *   stats      host, filled when not NULL (then the stream is synchronised) */
typedef struct {
  int64_t rays;         /* rays that entered the mesh */
  int64_t steps;        /* tetrahedra visited */
  int64_t escalations;  /* eps increases */
  int64_t halted;       /* rays stopped because eps passed 1 */
  int64_t looped;       /* rays stopped at the step cap */
} tct_paper_stats;

tct_status tct_forward_paper(const tct_mesh* m, const tct_geom* g, const float* x, float* proj, const int32_t* entry,
                             int precision, tct_paper_stats* stats, tct_stream s);

/* Visited tetrahedra of selected rays, zero-length passages included, in CSR
 * form: row j of the system matrix (Section II-A, Eq. 1: a_ij = length of ray j
 * inside tetrahedron i) in visiting order, the sequence Algorithm 2 walks
 * (zero-length passages through edges and vertices, Fig. 3, included).
 *   ray_ids  device int64 [nrays]
 *   offsets  device int64 [nrays + 1]   written: ray k owns [offsets[k], offsets[k+1])
 *   tets     device int32 [cap]          user ids
 *   lengths  device float [cap]
 * Synchronises the stream.  If the total exceeds cap, returns TCT_E_CAPACITY
 * with offsets filled and *needed set. */
tct_status tct_trace(const tct_mesh* m, const tct_geom* g, const int64_t* ray_ids, int32_t nrays, int64_t* offsets,
                     int32_t* tets, float* lengths, int64_t cap, int64_t* needed, tct_stream s);

/* Same for caller-given rays (Algorithm 2's R1 = S, R2 = P, not tied to a
 * detector): device float [n][3] arrays S, P (endpoints) and
 * U, V (tie-breaking axes; {P - S, U, V} must be a basis, else the ray is
 * counted as failed and gets an empty path). */
tct_status tct_trace_rays(const tct_mesh* m, const float* S, const float* P, const float* U, const float* V,
                          int32_t n, int64_t* offsets, int32_t* tets, float* lengths, int64_t cap, int64_t* needed,
                          tct_stream s);

/* ---------------------------------------------------------------- solver vectors
 * Building blocks for iterative reconstruction with A and A^T (the paper names
 * SART and CGLS as consumers of the projector, Section II-A; it reconstructs
 * with OS-SART, Section III-A).  All arrays are device memory of n floats;
 * scalars passed as `const double*` are device pointers, so an iteration
 * needs no host round trip and can be captured in a graph. */

#define TCT_DOT_WORKSPACE 512 /* doubles of workspace tct_dot needs */

/* result[0] (device double) = sum_i a_i b_i, accumulated in double in a fixed
 * order (bitwise reproducible).  workspace: device double [TCT_DOT_WORKSPACE]. */
tct_status tct_dot(const float* a, const float* b, int64_t n, double* result, double* workspace, tct_stream s);

/* y += sign * (num[0] / den[0]) * x; a zero denominator gives a zero step. */
tct_status tct_axpy_ratio(float* y, const float* x, int64_t n, const double* num, const double* den, double sign,
                          tct_stream s);

/* p = x + (num[0] / den[0]) * p; a zero denominator gives p = x. */
tct_status tct_xpay_ratio(float* p, const float* x, int64_t n, const double* num, const double* den, tct_stream s);

/* y = a * x + b * y (host scalars). */
tct_status tct_axpby(float* y, const float* x, int64_t n, float a, float b, tct_stream s);

/* y = a .* b (elementwise; y may alias a or b). */
tct_status tct_mul(float* y, const float* a, const float* b, int64_t n, tct_stream s);

/* y = (a > eps) ? 1 / a : 0 (elementwise; y may alias a). */
tct_status tct_recip(float* y, const float* a, int64_t n, float eps, tct_stream s);

/* dst[0..n) = src[0..n) for device doubles (solver scalars). */
tct_status tct_copy_f64(double* dst, const double* src, int32_t n, tct_stream s);

/* ---------------------------------------------------------------- batches
 * Many independent problems (each its own mesh and geometry) processed by one
 * persistent launch that pulls pixel blocks of every problem from a device
 * work counter, most expensive problems first.  Vector arguments are
 * "vector sets": tables of device pointers built once, so a batched call
 * takes no host data and can be captured in a graph. */

/* n device float arrays (ptrs[k] of lens[k] elements) on `device`.  The
 * table is copied; the arrays stay caller-owned and must outlive the set. */
tct_status tct_vecset_create(int32_t n, float* const* ptrs, const int64_t* lens, int device, tct_vecset** out);
void tct_vecset_destroy(tct_vecset* v);

#define TCT_VECSET_DOT_WORKSPACE 256 /* doubles of workspace per vector for tct_vecset_dot */

/* results[k] (device double [n]) = a_k . b_k, float64, fixed order (reproducible).
 * workspace: device double [n * TCT_VECSET_DOT_WORKSPACE]. */
tct_status tct_vecset_dot(const tct_vecset* a, const tct_vecset* b, double* results, double* workspace,
                          tct_stream s);
/* y_k += sign * (num[k] / den[k]) * x_k   (num, den: device double [n]) */
tct_status tct_vecset_axpy_ratio(const tct_vecset* y, const tct_vecset* x, const double* num, const double* den,
                                 double sign, tct_stream s);
/* p_k = x_k + (num[k] / den[k]) * p_k */
tct_status tct_vecset_xpay_ratio(const tct_vecset* p, const tct_vecset* x, const double* num, const double* den,
                                 tct_stream s);
/* y_k[:] = value */
tct_status tct_vecset_fill(const tct_vecset* y, float value, tct_stream s);

/* A batch of n (mesh, geometry) problems on one device.  tile_u: host int32 [n]
 * wavefront tile widths (NULL = 8).  entries: host array of n device entry
 * caches from tct_entry / tct_entry_raster; for NULL (or NULL elements) the
 * batch computes its own caches by boundary projection (device memory it
 * frees in tct_batch_destroy; synchronises the device).  The
 * handles must outlive the batch.  The launches take pixel blocks from eight
 * device work lists, one per die of the chip, each holding one contiguous
 * run of every problem's blocks (most expensive problem first); a workgroup
 * takes from its own die's list, then from the others'.  A batch is
 * stream-exclusive: its list counters are reset by each call. */
tct_status tct_batch_create(const tct_mesh* const* meshes, const tct_geom* const* geoms, int32_t n,
                            const int32_t* tile_u, int32_t* const* entries, tct_batch** out);
/* proj_k = A_k x_k for every problem (x: nt_k floats, internal order; proj: rays_k floats). */
tct_status tct_batch_forward(tct_batch* b, const tct_vecset* x, const tct_vecset* proj, tct_stream s);
/* xhat_k (+)= A_k^T proj_k for every problem (atomic mode with on-chip pre-summing). */
tct_status tct_batch_backproject(tct_batch* b, const tct_vecset* proj, const tct_vecset* xhat, int accumulate,
                                 tct_stream s);
/* Total pixel blocks (work-list items) of the batch. */
int64_t tct_batch_items(const tct_batch* b);
/* Pixel blocks a workgroup of the persistent batched launch takes from a
 * work list per fetch (1..64, default 1; else TCT_E_ARG).  The pixel block
 * shape follows the paper's thread-block tuning (Section II-F); the queue
 * granularity is the batched launch's second tuned knob.  Applies to later
 * tct_batch_forward / tct_batch_backproject calls. */
tct_status tct_batch_set_queue_chunk(tct_batch* b, int32_t blocks_per_fetch);
void tct_batch_destroy(tct_batch* b);

/* ---------------------------------------------------------------- misc */

const char* tct_last_error(void);
const char* tct_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TETCT_H */

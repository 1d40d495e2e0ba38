// Deterministic backprojection: xhat_i = sum_j a_ij y_j (Eq. 3) over explicit
// per-tetrahedron lists, summed exactly, so the result is bitwise
// reproducible.
//
// The paper scatters with atomics (Section II-F), having found a variant
// that kept the rays' contributions apart slower on its GPU; the atomic path
// (walk.hip) is the fast one here too.  This path trades some speed for
// reproducibility.  Per chunk of angles:
//   1. fill walk: every wavefront sums its segments per tetrahedron over a
//      window of steps in its LDS table, exactly, in 64-bit fixed point with
//      the wavefront's own power-of-two scale, and at the end of each window
//      writes one record (tetrahedron, scale, integer sum) per tetrahedron
//      it met, counting the records of each tetrahedron;
//   2. exclusive scan of the counts -> each tetrahedron's list;
//   3. scatter of the records into their tetrahedron's list (the order
//      inside a list depends on timing);
//   4. one wavefront per tetrahedron adds its list exactly: every record is
//      brought to the list's finest scale (or, when the list's scales are
//      more than 36 powers of two apart, to 36 above its coarsest, the finer
//      records truncated there), summed as 128-bit integers, and the sum is
//      converted to float64 once, so the result does not depend on the
//      order; chunks are added in angle order.
// The records are some fourteen times fewer than the segments (the
// wavefront's 64 rays cross each tetrahedron together).
#include "common.h"
#include "kernels.h"

namespace tct {

namespace {

__global__ void zero_f64_kernel(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void zero_i32_kernel(int32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void zero_u64_small_kernel(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// Records into their tetrahedron's list: list t is [off[t], off[t] + counts
// of t); cur[t] (zeroed) hands out its positions.  One 16-byte load and one
// 16-byte store per record.  blockIdx.y is the record region (its first
// nrec[y] records are written, region size gcap).
__global__ void scatter_records_kernel(const GatherRecord* rec, const unsigned long long* nrec, int64_t gcap,
                                       const int64_t* off, int32_t* cur, GatherRecord* list) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nrec[blockIdx.y]) return;
  const GatherRecord x = rec[(int64_t)blockIdx.y * gcap + i];
  const int64_t p = off[x.tet] + atomicAdd(cur + x.tet, 1);
  list[p] = x;
}

// 128-bit two's complement integers for exact sums.
struct I128 {
  unsigned long long lo;
  long long hi;
};

__device__ __forceinline__ I128 i128_add(I128 a, I128 b) {
  I128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1 : 0);
  return r;
}

// m 2^k exactly for 0 <= k <= 36 (|m| < 2^60, so |m 2^k| < 2^96 and up to 2^30
// of them add up below 2^127), floor(m 2^k) for k < 0.
__device__ __forceinline__ I128 i128_scaled(long long m, int k) {
  I128 r;
  if (k > 0) {
    r.lo = (unsigned long long)m << k;
    r.hi = m >> (64 - k);
  } else {
    const long long v = k < 0 ? (k > -64 ? m >> -k : (m < 0 ? -1 : 0)) : m;
    r.lo = (unsigned long long)v;
    r.hi = v >> 63;
  }
  return r;
}

// One wavefront per tetrahedron: its list summed exactly (see step 4).
constexpr int kSumWaves = 4;
constexpr int kMaxScaleSpread = 36;

__global__ __launch_bounds__(64 * kSumWaves) void exact_sum_kernel(const int64_t* off, const GatherRecord* list,
                                                                   double* acc, int nt) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * kSumWaves + (threadIdx.x >> 6);
  if (t >= nt) return;
  const int64_t b = off[t], e = off[t + 1];
  if (b == e) return;
  int smin = 1 << 30, smax = -(1 << 30);
  for (int64_t i = b + lane; i < e; i += 64) {
    const int sc = list[i].scale;
    smin = min(smin, sc);
    smax = max(smax, sc);
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    smin = min(smin, __shfl_xor(smin, o, 64));
    smax = max(smax, __shfl_xor(smax, o, 64));
  }
  const int sref = min(smax, smin + kMaxScaleSpread);
  I128 s{0ull, 0ll};
  for (int64_t i = b + lane; i < e; i += 64) {
    const GatherRecord x = list[i];
    s = i128_add(s, i128_scaled(x.m, sref - x.scale));
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    I128 x;
    x.lo = ((unsigned long long)(unsigned)__shfl_xor((int)(s.lo >> 32), o, 64) << 32) |
           (unsigned)__shfl_xor((int)s.lo, o, 64);
    x.hi = (long long)(((unsigned long long)(unsigned)__shfl_xor((int)(s.hi >> 32), o, 64) << 32) |
                       (unsigned)__shfl_xor((int)s.hi, o, 64));
    s = i128_add(s, x);
  }
  if (lane == 0) acc[t] += ldexp((double)s.hi, 64 - sref) + ldexp((double)s.lo, -sref);
}

__global__ void finish_kernel(const double* acc, float* xhat, int nt, int accumulate) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  xhat[t] = accumulate ? (float)((double)xhat[t] + acc[t]) : (float)acc[t];
}

template <typename T>
struct AsyncBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s;
  explicit AsyncBuf(hipStream_t st) : s(st) {}
  hipError_t ensure(size_t need) {
    if (need <= n) return hipSuccess;
    if (p) (void)hipFreeAsync(p, s);
    p = nullptr;
    n = 0;
    hipError_t e = hipMallocAsync((void**)&p, std::max<size_t>(need, 1) * sizeof(T), s);
    if (e == hipSuccess) n = need;
    return e;
  }
  ~AsyncBuf() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

unsigned grid_of(int64_t n, int per_block) { return (unsigned)std::max<int64_t>(1, (n + per_block - 1) / per_block); }

}  // namespace

// Exclusive scan of n int32 counts into n + 1 int64 offsets (out[n] = the
// total), in three launches: per-block sums of kScanItems counts, a scan of
// those sums by one block, then each block's own scan from its offset.
namespace {
constexpr int kScanItems = 2048;  // counts per block (256 threads x 8)

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* total) {
  __shared__ int64_t s_w[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[w] = x;
  __syncthreads();
  int64_t before = 0;
  for (int k = 0; k < w; ++k) before += s_w[k];
  *total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
  __syncthreads();
  return before + x - v;
}

__global__ __launch_bounds__(256) void scan_sums_kernel(const int32_t* in, int64_t n, int64_t* sums) {
  const int64_t i0 = (int64_t)blockIdx.x * kScanItems + threadIdx.x * 8;
  int64_t v = 0;
  for (int u = 0; u < 8; ++u)
    if (i0 + u < n) v += in[i0 + u];
  int64_t total;
  (void)block_exclusive_scan(v, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block scans the block sums in place (exclusive) and writes the total.
__global__ __launch_bounds__(256) void scan_top_kernel(int64_t* sums, int64_t nb, int64_t* total_out) {
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += 256) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < nb ? sums[i] : 0;
    int64_t total;
    const int64_t ex = block_exclusive_scan(v, &total);
    if (i < nb) sums[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(256) void scan_out_kernel(const int32_t* in, int64_t n, const int64_t* sums,
                                                       int64_t* out) {
  const int64_t i0 = (int64_t)blockIdx.x * kScanItems + threadIdx.x * 8;
  int64_t c[8], v = 0;
  for (int u = 0; u < 8; ++u) {
    c[u] = i0 + u < n ? in[i0 + u] : 0;
    v += c[u];
  }
  int64_t total;
  int64_t x = sums[blockIdx.x] + block_exclusive_scan(v, &total);
  for (int u = 0; u < 8; ++u) {
    if (i0 + u < n) out[i0 + u] = x;
    x += c[u];
  }
}
}  // namespace

tct_status exclusive_scan_counts(const int32_t* in, int64_t* out, int64_t n, int64_t* sums, hipStream_t s) {
  const int64_t nb = std::max<int64_t>(1, (n + kScanItems - 1) / kScanItems);
  hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)nb), dim3(256), 0, s, in, n, sums);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(256), 0, s, sums, nb, out + n);
  hipLaunchKernelGGL(scan_out_kernel, dim3((unsigned)nb), dim3(256), 0, s, in, n, (const int64_t*)sums, out);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status backproject_gather(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int accumulate,
                              const int32_t* entry, int tile_u, int a_begin, int a_count, hipStream_t s) {
  const int nt = m->nt;
  const int64_t rays_per_angle = (int64_t)g->cone.nu * g->cone.nv;
  // Records per chunk: a budget of 2^28 (8 GB of records and lists); the
  // first chunk is sized from a guess of 16 records per ray and later ones
  // from the records per angle seen so far.
  const int64_t kBudget = (int64_t)1 << 28;
  AsyncBuf<double> acc(s);
  AsyncBuf<int32_t> counts(s);
  AsyncBuf<GatherRecord> rec(s), list(s);
  AsyncBuf<int64_t> scan_sums(s), offsets(s);
  AsyncBuf<unsigned long long> cursor(s);
  TCT_HIP(acc.ensure(nt));
  TCT_HIP(counts.ensure(nt));
  TCT_HIP(scan_sums.ensure((size_t)nt / kScanItems + 1));
  TCT_HIP(offsets.ensure((size_t)nt + 1));
  TCT_HIP(cursor.ensure(kGatherGroups));
  hipLaunchKernelGGL(zero_f64_kernel, dim3(grid_of(nt, 256)), dim3(256), 0, s, acc.p, (int64_t)nt);
  TCT_HIP(hipGetLastError());
  double rec_per_angle = 16.0 * (double)rays_per_angle;
  const int a_end = a_begin + a_count;
  int a0 = a_begin;
  while (a0 < a_end) {
    int na_c = (int)std::max<double>(1.0, std::min<double>(a_end - a0, std::floor(kBudget / rec_per_angle)));
    // Per region: an even share of the expected records, with room for the
    // regions' spread.
    int64_t gcap = std::max<int64_t>(256, (int64_t)(rec_per_angle * na_c * 1.25) / kGatherGroups);
    int64_t total = 0, most = 0;
    unsigned long long need[kGatherGroups];
    for (;;) {
      TCT_HIP(rec.ensure((size_t)gcap * kGatherGroups));
      hipLaunchKernelGGL(zero_i32_kernel, dim3(grid_of(nt, 256)), dim3(256), 0, s, counts.p, (int64_t)nt);
      hipLaunchKernelGGL(zero_u64_small_kernel, dim3(1), dim3(kGatherGroups), 0, s, cursor.p, kGatherGroups);
      TCT_HIP(hipGetLastError());
      const GatherOut go{rec.p, counts.p, cursor.p, gcap};
      tct_status st = launch_pixel_walk(kModeGatherFill, m, g, a0, na_c, entry, proj, nullptr, nullptr, &go, tile_u,
                                        s);
      if (st != TCT_OK) return st;
      TCT_HIP(hipMemcpyAsync(need, cursor.p, sizeof(need), hipMemcpyDeviceToHost, s));
      TCT_HIP(hipStreamSynchronize(s));
      total = 0;
      most = 0;
      for (int k = 0; k < kGatherGroups; ++k) {
        total += (int64_t)need[k];
        most = std::max<int64_t>(most, (int64_t)need[k]);
      }
      if (most <= gcap) break;
      gcap = most + most / 8;  // every record fits on the second pass
    }
    rec_per_angle = std::max(1.0, (double)total / na_c);
    if (total > 0) {
      TCT_HIP(list.ensure(total));
      tct_status st = exclusive_scan_counts(counts.p, offsets.p, nt, scan_sums.p, s);
      if (st != TCT_OK) return st;
      hipLaunchKernelGGL(zero_i32_kernel, dim3(grid_of(nt, 256)), dim3(256), 0, s, counts.p, (int64_t)nt);
      hipLaunchKernelGGL(scatter_records_kernel, dim3(grid_of(most, 256), kGatherGroups), dim3(256), 0, s, rec.p,
                         (const unsigned long long*)cursor.p, gcap, offsets.p, counts.p, list.p);
      hipLaunchKernelGGL(exact_sum_kernel, dim3(grid_of(nt, kSumWaves)), dim3(64 * kSumWaves), 0, s, offsets.p,
                         list.p, acc.p, nt);
      TCT_HIP(hipGetLastError());
    }
    a0 += na_c;
  }
  hipLaunchKernelGGL(finish_kernel, dim3(grid_of(nt, 256)), dim3(256), 0, s, acc.p, xhat, nt, accumulate);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

}  // namespace tct

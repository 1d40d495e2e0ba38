// Deterministic backprojection: xhat_i = sum_j a_ij y_j (Eq. 3) summed per
// tetrahedron in a fixed order, so the result is bitwise reproducible.
//
// The paper scatters with atomics (Section II-F), having found a variant
// that kept the rays' contributions apart slower on its GPU; the atomic path
// (walk.hip) is the fast one here too.  This path trades speed for
// reproducibility.  Per chunk of angles:
//   1. count walk: positive-length visits per ray, reduced to the longest
//      list of each wavefront;
//   2. exclusive scan -> each wavefront's slot range (64 x its longest list);
//   3. fill walk: (tetrahedron, a_ij y_j) pairs, segment k of lane l at
//      base + 64 k + l, so each step stores 64 consecutive words; shorter
//      lists padded with key nt;
//   4. stable LSD radix sort by tetrahedron (slot order kept within a key);
//   5. run boundaries from the sorted keys; one wavefront per tetrahedron
//      sums its run in float64 (lane l takes elements l, l+64, ... in order,
//      then a fixed butterfly), added to a float64 accumulator; chunks are
//      added in angle order.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "common.h"
#include "kernels.h"

namespace tct {

namespace {

__global__ void zero_f64_kernel(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void zero_i64_kernel(int64_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Run boundaries of the sorted keys: [run[2 t], run[2 t + 1]) holds
// tetrahedron t (both zero when it has no segment); padding keys (>= nt)
// are skipped.
// Each thread takes kRunItems consecutive keys.
constexpr int kRunItems = 8;

__global__ void run_bounds_kernel(const int32_t* keys, int64_t n, int nt, int64_t* run) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRunItems;
  if (i0 >= n) return;
  int prev = i0 > 0 ? keys[i0 - 1] : -1;
#pragma unroll
  for (int u = 0; u < kRunItems; ++u) {
    const int64_t i = i0 + u;
    if (i >= n) break;
    const int k = keys[i];
    const int next = i + 1 < n ? keys[i + 1] : -1;
    if (k < nt) {
      if (prev != k) run[2 * (int64_t)k] = i;
      if (next != k) run[2 * (int64_t)k + 1] = i + 1;
    }
    prev = k;
  }
}

// One wavefront per tetrahedron.
__global__ __launch_bounds__(256) void segment_sum_kernel(const int64_t* run, const float* vals, double* acc,
                                                          int nt) {
  int t = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  int lane = threadIdx.x & 63;
  if (t >= nt) return;
  const int64_t b = run[2 * (int64_t)t], e = run[2 * (int64_t)t + 1];
  if (b == e) return;
  double s = 0.0;
  for (int64_t i = b + lane; i < e; i += 64) s += (double)vals[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) acc[t] += s;
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

int key_bits(int nt) {
  int b = 1;
  while ((1ll << b) < (long long)nt) ++b;
  return b;
}

}  // namespace

tct_status exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total_host, hipStream_t s) {
  // out has n + 1 entries; out[n] is the total.
  size_t tmp_bytes = 0;
  TCT_HIP(rocprim::inclusive_scan(nullptr, tmp_bytes, in, out + 1, (size_t)n, rocprim::plus<int64_t>(), s));
  AsyncBuf<char> tmp(s);
  TCT_HIP(tmp.ensure(tmp_bytes));
  int64_t zero = 0;
  TCT_HIP(hipMemcpyAsync(out, &zero, sizeof(int64_t), hipMemcpyHostToDevice, s));
  TCT_HIP(rocprim::inclusive_scan(tmp.p, tmp_bytes, in, out + 1, (size_t)n, rocprim::plus<int64_t>(), s));
  if (total_host) {
    TCT_HIP(hipMemcpyAsync(total_host, out + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TCT_HIP(hipStreamSynchronize(s));
  }
  return TCT_OK;
}

tct_status backproject_gather(const tct_mesh* m, const tct_geom* g, const float* proj, float* xhat, int accumulate,
                              const int32_t* entry, int tile_u, int a_begin, int a_count, hipStream_t s) {
  const int64_t rays_per_angle = (int64_t)g->cone.nu * g->cone.nv;
  // Chunk of angles: about 4M rays, at least one angle.
  int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(a_count, ((int64_t)1 << 22) / rays_per_angle));
  AsyncBuf<double> acc(s);
  AsyncBuf<int64_t> counts(s), offsets(s);
  AsyncBuf<int32_t> keys(s), keys_sorted(s);
  AsyncBuf<float> vals(s), vals_sorted(s);
  AsyncBuf<char> sort_tmp(s);
  AsyncBuf<int64_t> run(s);
  TCT_HIP(acc.ensure(m->nt));
  TCT_HIP(run.ensure(2 * (size_t)m->nt));
  hipLaunchKernelGGL(zero_f64_kernel, dim3((m->nt + 255) / 256), dim3(256), 0, s, acc.p, (int64_t)m->nt);
  TCT_HIP(hipGetLastError());
  const int bits = key_bits(m->nt + 1);  // padding key nt included
  const int a_end = a_begin + a_count;
  for (int a0 = a_begin; a0 < a_end; a0 += chunk) {
    int na_c = std::min(chunk, a_end - a0);
    const int64_t nw = pixel_walk_waves(g, na_c, tile_u);
    TCT_HIP(counts.ensure(nw));
    TCT_HIP(offsets.ensure(nw + 1));
    tct_status st = launch_pixel_walk(kModeCountPos, m, g, a0, na_c, entry, proj, nullptr, nullptr, counts.p,
                                      nullptr, nullptr, nullptr, tile_u, s);
    if (st != TCT_OK) return st;
    int64_t total = 0;
    st = exclusive_scan_i64(counts.p, offsets.p, nw, &total, s);
    if (st != TCT_OK) return st;
    if (total == 0) continue;
    TCT_HIP(keys.ensure(total));
    TCT_HIP(vals.ensure(total));
    TCT_HIP(keys_sorted.ensure(total));
    TCT_HIP(vals_sorted.ensure(total));
    st = launch_pixel_walk(kModeGatherFill, m, g, a0, na_c, entry, proj, nullptr, nullptr, nullptr, offsets.p, keys.p,
                           vals.p, tile_u, s);
    if (st != TCT_OK) return st;
    size_t tmp_bytes = 0;
    TCT_HIP(rocprim::radix_sort_pairs(nullptr, tmp_bytes, keys.p, keys_sorted.p, vals.p, vals_sorted.p,
                                      (size_t)total, 0, bits, s));
    TCT_HIP(sort_tmp.ensure(tmp_bytes));
    TCT_HIP(rocprim::radix_sort_pairs(sort_tmp.p, tmp_bytes, keys.p, keys_sorted.p, vals.p, vals_sorted.p,
                                      (size_t)total, 0, bits, s));
    const int64_t nrun = 2 * (int64_t)m->nt;
    hipLaunchKernelGGL(zero_i64_kernel, dim3((unsigned)((nrun + 255) / 256)), dim3(256), 0, s, run.p, nrun);
    const int64_t run_threads = (total + kRunItems - 1) / kRunItems;
    hipLaunchKernelGGL(run_bounds_kernel, dim3((unsigned)((run_threads + 255) / 256)), dim3(256), 0, s,
                       keys_sorted.p, total, m->nt, run.p);
    int64_t threads = (int64_t)m->nt * 64;
    hipLaunchKernelGGL(segment_sum_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, run.p,
                       vals_sorted.p, acc.p, m->nt);
    TCT_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(finish_kernel, dim3((m->nt + 255) / 256), dim3(256), 0, s, acc.p, xhat, m->nt, accumulate);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

}  // namespace tct

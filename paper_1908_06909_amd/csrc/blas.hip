// Vector kernels for the iterative solvers that consume A and A^T (the paper
// names SART and CGLS, Section II-A).  Scalars that feed later steps (step
// sizes gamma / delta) stay on the device, so a solver iteration needs no host
// synchronisation and can be captured in a graph.  Dot products are
// deterministic: fixed grid, float64 partial sums, summed in block order.
#include "common.h"
#include "kernels.h"

namespace tct {

namespace {

constexpr int kDotBlocks = TCT_DOT_WORKSPACE;
constexpr int kDotThreads = 256;

__global__ __launch_bounds__(kDotThreads) void dot_partial_kernel(const float* a, const float* b, int64_t n,
                                                                  double* partial) {
  __shared__ double sh[kDotThreads];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDotThreads)
    s += (double)a[i] * (double)b[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kDotThreads) void dot_final_kernel(const double* partial, int np, double* result) {
  __shared__ double sh[kDotThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kDotThreads) s += partial[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) result[0] = sh[0];
}

__device__ __forceinline__ double safe_ratio(const double* num, const double* den) {
  double d = den[0];
  return d != 0.0 ? num[0] / d : 0.0;
}

// y += sign * (num / den) * x
__global__ void axpy_ratio_kernel(float* y, const float* x, int64_t n, const double* num, const double* den,
                                  double sign) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float a = (float)(sign * safe_ratio(num, den));
  y[i] += a * x[i];
}

// p = s + (num / den) * p
__global__ void xpay_ratio_kernel(float* p, const float* s, int64_t n, const double* num, const double* den) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float b = (float)safe_ratio(num, den);
  p[i] = s[i] + b * p[i];
}

// y = a * x + b * y
__global__ void axpby_kernel(float* y, const float* x, int64_t n, float a, float b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = a * x[i] + b * y[i];
}

// y = a .* b
__global__ void mul_kernel(float* y, const float* a, const float* b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = a[i] * b[i];
}

// y = a > eps ? 1 / a : 0
__global__ void recip_kernel(float* y, const float* a, int64_t n, float eps) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float v = a[i];
  y[i] = v > eps ? 1.0f / v : 0.0f;
}

__global__ void copy_f64_kernel(double* dst, const double* src, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// ---- vector sets: one launch over n vectors; block (p, c) handles chunk c of vector p.
constexpr int kSetChunks = TCT_VECSET_DOT_WORKSPACE;

__device__ __forceinline__ void chunk_range(int64_t len, int c, int64_t* b, int64_t* e) {
  *b = len * c / kSetChunks;
  *e = len * (c + 1) / kSetChunks;
}

__global__ __launch_bounds__(kDotThreads) void vs_dot_partial_kernel(float* const* A, float* const* B,
                                                                     const int64_t* lens, double* ws) {
  __shared__ double sh[kDotThreads];
  int p = blockIdx.y, c = blockIdx.x;
  int64_t b, e;
  chunk_range(lens[p], c, &b, &e);
  const float* a = A[p];
  const float* bb = B[p];
  double s = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += kDotThreads) s += (double)a[i] * (double)bb[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) ws[(size_t)p * kSetChunks + c] = sh[0];
}

__global__ __launch_bounds__(kDotThreads) void vs_dot_final_kernel(const double* ws, double* results) {
  __shared__ double sh[kDotThreads];
  int p = blockIdx.x;
  double s = 0.0;
  for (int c = threadIdx.x; c < kSetChunks; c += kDotThreads) s += ws[(size_t)p * kSetChunks + c];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) results[p] = sh[0];
}

__global__ __launch_bounds__(256) void vs_axpy_ratio_kernel(float* const* Y, float* const* X, const int64_t* lens,
                                                            const double* num, const double* den, double sign) {
  int p = blockIdx.y, c = blockIdx.x;
  int64_t b, e;
  chunk_range(lens[p], c, &b, &e);
  float a = (float)(sign * safe_ratio(num + p, den + p));
  float* y = Y[p];
  const float* x = X[p];
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) y[i] += a * x[i];
}

__global__ __launch_bounds__(256) void vs_xpay_ratio_kernel(float* const* Pp, float* const* X, const int64_t* lens,
                                                            const double* num, const double* den) {
  int p = blockIdx.y, c = blockIdx.x;
  int64_t b, e;
  chunk_range(lens[p], c, &b, &e);
  float beta = (float)safe_ratio(num + p, den + p);
  float* q = Pp[p];
  const float* x = X[p];
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) q[i] = x[i] + beta * q[i];
}

__global__ __launch_bounds__(256) void vs_fill_kernel(float* const* Y, const int64_t* lens, float v) {
  int p = blockIdx.y, c = blockIdx.x;
  int64_t b, e;
  chunk_range(lens[p], c, &b, &e);
  float* y = Y[p];
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) y[i] = v;
}

}  // namespace

tct_status blas_dot(const float* a, const float* b, int64_t n, double* result, double* workspace, hipStream_t s) {
  int grid = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (n + kDotThreads - 1) / kDotThreads));
  hipLaunchKernelGGL(dot_partial_kernel, dim3(grid), dim3(kDotThreads), 0, s, a, b, n, workspace);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kDotThreads), 0, s, workspace, grid, result);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status blas_axpy_ratio(float* y, const float* x, int64_t n, const double* num, const double* den, double sign,
                           hipStream_t s) {
  if (n <= 0) return TCT_OK;
  hipLaunchKernelGGL(axpy_ratio_kernel, dim3(blocks_for(n)), dim3(256), 0, s, y, x, n, num, den, sign);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status blas_xpay_ratio(float* p, const float* x, int64_t n, const double* num, const double* den,
                           hipStream_t s) {
  if (n <= 0) return TCT_OK;
  hipLaunchKernelGGL(xpay_ratio_kernel, dim3(blocks_for(n)), dim3(256), 0, s, p, x, n, num, den);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status blas_axpby(float* y, const float* x, int64_t n, float a, float b, hipStream_t s) {
  if (n <= 0) return TCT_OK;
  hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for(n)), dim3(256), 0, s, y, x, n, a, b);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status blas_mul(float* y, const float* a, const float* b, int64_t n, hipStream_t s) {
  if (n <= 0) return TCT_OK;
  hipLaunchKernelGGL(mul_kernel, dim3(blocks_for(n)), dim3(256), 0, s, y, a, b, n);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status blas_recip(float* y, const float* a, int64_t n, float eps, hipStream_t s) {
  if (n <= 0) return TCT_OK;
  hipLaunchKernelGGL(recip_kernel, dim3(blocks_for(n)), dim3(256), 0, s, y, a, n, eps);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status blas_copy_f64(double* dst, const double* src, int n, hipStream_t s) {
  if (n <= 0) return TCT_OK;
  hipLaunchKernelGGL(copy_f64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, dst, src, n);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status vecset_dot(const tct_vecset* a, const tct_vecset* b, double* results, double* workspace, hipStream_t s) {
  if (a->n <= 0) return TCT_OK;
  hipLaunchKernelGGL(vs_dot_partial_kernel, dim3(kSetChunks, a->n), dim3(kDotThreads), 0, s, a->d_ptrs, b->d_ptrs,
                     a->d_lens, workspace);
  hipLaunchKernelGGL(vs_dot_final_kernel, dim3(a->n), dim3(kDotThreads), 0, s, workspace, results);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status vecset_axpy_ratio(const tct_vecset* y, const tct_vecset* x, const double* num, const double* den,
                             double sign, hipStream_t s) {
  if (y->n <= 0) return TCT_OK;
  hipLaunchKernelGGL(vs_axpy_ratio_kernel, dim3(kSetChunks, y->n), dim3(256), 0, s, y->d_ptrs, x->d_ptrs, y->d_lens,
                     num, den, sign);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status vecset_xpay_ratio(const tct_vecset* p, const tct_vecset* x, const double* num, const double* den,
                             hipStream_t s) {
  if (p->n <= 0) return TCT_OK;
  hipLaunchKernelGGL(vs_xpay_ratio_kernel, dim3(kSetChunks, p->n), dim3(256), 0, s, p->d_ptrs, x->d_ptrs, p->d_lens,
                     num, den);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

tct_status vecset_fill(const tct_vecset* y, float v, hipStream_t s) {
  if (y->n <= 0) return TCT_OK;
  hipLaunchKernelGGL(vs_fill_kernel, dim3(kSetChunks, y->n), dim3(256), 0, s, y->d_ptrs, y->d_lens, v);
  TCT_HIP(hipGetLastError());
  return TCT_OK;
}

}  // namespace tct

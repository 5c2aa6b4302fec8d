// Device kernels of the GMRES / flexible GMRES Arnoldi process (FP64): block
// dot products V^T w, fused classical Gram-Schmidt updates w -= V h with the
// dot products of the re-orthogonalisation pass, and fixed-order two-stage
// reductions (deterministic results for a fixed grid).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stig {

constexpr int KRY_BLOCK = 256;
constexpr int KRY_GRID = 1024;   // partial sums per dot product
constexpr int KRY_MAXV = 33;     // basis vectors per call (restart <= 32) + w.w

// Block-wide sums of the per-thread values vals[i] for the active slots
// (i < nv, plus slot KRY_MAXV-1 if with_norm); written to
// partial[i * gridDim.x + blockIdx.x].  Register arrays are only indexed with
// compile-time constants.
__device__ inline void block_reduce_store(const double (&vals)[KRY_MAXV], int nv, int with_norm,
                                          double *red, double *__restrict__ partial) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < KRY_MAXV; ++i) {
    bool active = (i < nv) || (i == KRY_MAXV - 1 && with_norm);
    if (active) {
      double s = vals[i];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) red[wave * KRY_MAXV + i] = s;
    }
  }
  __syncthreads();
  int i = threadIdx.x;
  if (i < KRY_MAXV && ((i < nv) || (i == KRY_MAXV - 1 && with_norm))) {
    double s = 0.0;
    for (int w = 0; w < KRY_BLOCK / 64; ++w) s += red[w * KRY_MAXV + i];
    partial[(int64_t)i * gridDim.x + blockIdx.x] = s;
  }
}

// partial[i * gridDim.x + block] = this block's share of V_i . w (i < nv) and,
// if with_norm, slot KRY_MAXV-1 = w . w.  V_i = V + i * ldv.
__global__ void __launch_bounds__(KRY_BLOCK)
krylov_dots(const double *__restrict__ V, int64_t ldv, int nv, const double *__restrict__ w,
            int64_t N, int with_norm, double *__restrict__ partial) {
  __shared__ double red[(KRY_BLOCK / 64) * KRY_MAXV];
  double acc[KRY_MAXV];
#pragma unroll
  for (int i = 0; i < KRY_MAXV; ++i) acc[i] = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x) {
    double we = w[e];
#pragma unroll
    for (int i = 0; i < KRY_MAXV - 1; ++i)
      if (i < nv) acc[i] += V[i * ldv + e] * we;
    acc[KRY_MAXV - 1] += we * we;
  }
  block_reduce_store(acc, nv, with_norm, red, partial);
}

// w += sign * sum_i coef[i] V_i (coef in device memory); then, if with_dots,
// partial dots V_i . w_new and w_new . w_new as in krylov_dots (with_norm = 1).
__global__ void __launch_bounds__(KRY_BLOCK)
krylov_update(const double *__restrict__ V, int64_t ldv, int nv, const double *__restrict__ coef,
              double sign, double *__restrict__ w, int64_t N, int with_dots,
              double *__restrict__ partial) {
  __shared__ double red[(KRY_BLOCK / 64) * KRY_MAXV];
  __shared__ double cs[KRY_MAXV];
  if (threadIdx.x < KRY_MAXV) cs[threadIdx.x] = (threadIdx.x < nv) ? sign * coef[threadIdx.x] : 0.0;
  __syncthreads();
  double acc[KRY_MAXV];
#pragma unroll
  for (int i = 0; i < KRY_MAXV; ++i) acc[i] = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v[KRY_MAXV - 1];
    double we = w[e];
#pragma unroll
    for (int i = 0; i < KRY_MAXV - 1; ++i) {
      v[i] = (i < nv) ? V[i * ldv + e] : 0.0;
      we += cs[i] * v[i];
    }
    w[e] = we;
    if (with_dots) {
#pragma unroll
      for (int i = 0; i < KRY_MAXV - 1; ++i) acc[i] += v[i] * we;
      acc[KRY_MAXV - 1] += we * we;
    }
  }
  if (!with_dots) return;
  block_reduce_store(acc, nv, 1, red, partial);
}

// out[i] = sum_b partial[i * nparts + b], fixed order; one block per i.
__global__ void __launch_bounds__(KRY_BLOCK)
reduce_partials(const double *__restrict__ partial, int nparts, double *__restrict__ out) {
  __shared__ double red[KRY_BLOCK / 64];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) s += partial[(int64_t)i * nparts + b];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < KRY_BLOCK / 64; ++w) t += red[w];
    out[i] = t;
  }
}

// out = a * x + b * y  (y may be null -> out = a * x)
__global__ void axpby(const double *__restrict__ x, const double *__restrict__ y,
                      double *__restrict__ out, double a, double b, int64_t N) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = y ? a * x[e] + b * y[e] : a * x[e];
}

// out = 1 / sqrt(D) elementwise (geometry-aware scaling)
__global__ void rsqrt_copy(const double *__restrict__ D, double *__restrict__ out, int64_t N) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = 1.0 / sqrt(D[e]);
}

}  // namespace stig

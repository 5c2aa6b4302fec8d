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

// Streaming loops take KRY_UNROLL elements per thread per trip (grid-stride
// apart), so each thread has that many independent loads of every vector in
// flight.  Kernels are instantiated for basis sizes up to NV (4, 8, 12, 16, 24,
// 32) so that register arrays and redundant loads stay as small as the call
// needs; large bases have enough loads in flight with one element per trip.
constexpr int KRY_UNROLL = 4;
template <int NV>
constexpr int kry_unroll() {
  return NV <= 4 ? KRY_UNROLL : (NV <= 8 ? 2 : 1);
}

// Block-wide sums of the per-thread values vals[i] for the active slots
// (i < nv, plus the norm slot vals[NV] if with_norm); slot i goes to
// partial[i * gridDim.x + blockIdx.x] and the norm to slot KRY_MAXV-1.
// Register arrays are only indexed with compile-time constants.
template <int NV>
__device__ inline void block_reduce_store(const double (&vals)[NV + 1], int nv, int with_norm,
                                          double *red, double *__restrict__ partial) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i <= NV; ++i) {
    bool active = (i < nv) || (i == NV && with_norm);
    if (active) {
      double s = vals[i];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) red[wave * (NV + 1) + i] = s;
    }
  }
  __syncthreads();
  int i = threadIdx.x;
  if (i <= NV && ((i < nv) || (i == NV && with_norm))) {
    double s = 0.0;
    for (int w = 0; w < KRY_BLOCK / 64; ++w) s += red[w * (NV + 1) + i];
    const int slot = i == NV ? KRY_MAXV - 1 : i;
    partial[(int64_t)slot * gridDim.x + blockIdx.x] = s;
  }
}

// partial[i * gridDim.x + block] = this block's share of V_i . w (i < nv) and,
// if with_norm, slot KRY_MAXV-1 = w . w.  V_i = V + i * ldv.
template <int NV>
__global__ void __launch_bounds__(KRY_BLOCK)
krylov_dots(const double *__restrict__ V, int64_t ldv, int nv, const double *__restrict__ w,
            int64_t N, int with_norm, double *__restrict__ partial) {
  __shared__ double red[(KRY_BLOCK / 64) * (NV + 1)];
  double acc[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
  constexpr int U = kry_unroll<NV>();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < N;
       e0 += U * stride) {
    double we[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + u * stride;
      we[u] = e < N ? w[e] : 0.0;
    }
    // branch-free: every slot loads (slots past nv re-read V_0, a cache hit,
    // and are never stored), so all loads of a trip are in flight together
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double *vi = V + (i < nv ? i : 0) * ldv;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = e0 + u * stride;
        acc[i] += (e < N ? vi[e] : 0.0) * we[u];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc[NV] += we[u] * we[u];
  }
  block_reduce_store<NV>(acc, nv, with_norm, red, partial);
}

// w_new = w + sign * sum_i coef[i] V_i (coef in device memory; w == nullptr
// reads as zero), written as dst = scale * w_new (dst may be w); then, if with_dots, partial dots
// V_i . w_new and w_new . w_new as in krylov_dots (with_norm = 1), from the
// V_i[e] values the update loaded.
template <int NV>
__global__ void __launch_bounds__(KRY_BLOCK)
krylov_update(const double *__restrict__ V, int64_t ldv, int nv, const double *__restrict__ coef,
              double sign, const double *w, double *dst, double scale, int64_t N, int with_dots,
              double *__restrict__ partial) {
  __shared__ double red[(KRY_BLOCK / 64) * (NV + 1)];
  __shared__ double cs[NV];
  if (threadIdx.x < NV) cs[threadIdx.x] = ((int)threadIdx.x < nv) ? sign * coef[threadIdx.x] : 0.0;
  __syncthreads();
  double acc[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
  constexpr int U = kry_unroll<NV>();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < N;
       e0 += U * stride) {
    double we[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + u * stride;
      we[u] = (w && e < N) ? w[e] : 0.0;
    }
    // the basis entries stay in registers for the dot products below (for large
    // bases a second read would miss the caches)
    // (branch-free as in krylov_dots: slots past nv have coefficient 0)
    double vv[NV][U];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double *vi = V + (i < nv ? i : 0) * ldv;
      const double c = cs[i];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = e0 + u * stride;
        vv[i][u] = e < N ? vi[e] : 0.0;
        we[u] += c * vv[i][u];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + u * stride;
      if (e < N) dst[e] = scale * we[u];
    }
    if (with_dots) {
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int u = 0; u < U; ++u) acc[i] += vv[i][u] * we[u];
#pragma unroll
      for (int u = 0; u < U; ++u) acc[NV] += we[u] * we[u];
    }
  }
  if (!with_dots) return;
  block_reduce_store<NV>(acc, nv, 1, red, partial);
}

// ---- delayed re-orthogonalisation (classical Gram-Schmidt, second pass
// lagged by one Arnoldi step): two passes over the basis per step.
// Slots of the one-pass products: Q^T u at [0, KRY_MAXV), Q^T w at
// [KRY_MAXV, 2 KRY_MAXV), then u.u, u.w, w.w.
constexpr int KRY_D2 = 2 * KRY_MAXV + 3;

// partial[slot * gridDim.x + block]: this block's shares of Q_i . u, Q_i . w
// (i < nq, Q_i = Q + i * ldv), u . u, u . w and w . w, from one read of each
// (NV = 0: no basis, the first step of a cycle).
template <int NV>
__global__ void __launch_bounds__(KRY_BLOCK)
krylov_dots2(const double *__restrict__ Q, int64_t ldv, int nq, const double *__restrict__ u,
             const double *__restrict__ w, int64_t N, double *__restrict__ partial) {
  constexpr int A = 2 * NV + 3;
  __shared__ double red[(KRY_BLOCK / 64) * A];
  double acc[A];
#pragma unroll
  for (int i = 0; i < A; ++i) acc[i] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const double ue = u[e], we = w[e];
    // branch-free: slots past nq re-read Q_0 (a cache hit) and are never stored
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double q = Q[(int64_t)(i < nq ? i : 0) * ldv + e];
      acc[i] += q * ue;
      acc[NV + i] += q * we;
    }
    acc[2 * NV] += ue * ue;
    acc[2 * NV + 1] += ue * we;
    acc[2 * NV + 2] += we * we;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < A; ++i) {
    const bool active = i >= 2 * NV || (i < NV ? i : i - NV) < nq;
    if (active) {
      double v = acc[i];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) red[wave * A + i] = v;
    }
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i < A && (i >= 2 * NV || (i < NV ? i : i - NV) < nq)) {
    double v = 0.0;
    for (int wv = 0; wv < KRY_BLOCK / 64; ++wv) v += red[wv * A + i];
    const int slot = i < NV ? i : (i < 2 * NV ? KRY_MAXV + (i - NV) : 2 * KRY_MAXV + (i - 2 * NV));
    partial[(int64_t)slot * gridDim.x + blockIdx.x] = v;
  }
}

// The second pass of a step, from one read of Q, u and w:
//   v = (u - sum_i s_i Q_i) * rv                       (written over u)
//   x = (w - a u - sum_i (t_i - a s_i) Q_i) * rx       (into x)
// with s, t in device memory (the reduced one-pass products; s may be a later
// re-orthogonalisation's); with_norm: shares of x . x in slot KRY_MAXV-1.
// write_v = 0 leaves u untouched; x = nullptr computes the norm only.
template <int NV>
__global__ void __launch_bounds__(KRY_BLOCK)
krylov_update2(const double *__restrict__ Q, int64_t ldv, int nq, const double *__restrict__ s,
               const double *__restrict__ t, double *u, const double *__restrict__ w,
               double *__restrict__ x, double a, double rv, double rx, int64_t N, int write_v,
               int with_norm, double *__restrict__ partial) {
  __shared__ double red[KRY_BLOCK / 64];
  __shared__ double cs[NV > 0 ? NV : 1], ct[NV > 0 ? NV : 1];
  if (threadIdx.x < NV) {
    const int i = threadIdx.x;
    cs[i] = i < nq ? s[i] : 0.0;
    ct[i] = i < nq ? t[i] - a * s[i] : 0.0;
  }
  __syncthreads();
  double nx = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const double ue = u[e], we = w[e];
    double pv = 0.0, px = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double q = Q[(int64_t)(i < nq ? i : 0) * ldv + e];
      pv += cs[i] * q;
      px += ct[i] * q;
    }
    const double xv = (we - a * ue - px) * rx;
    if (x) x[e] = xv;
    if (write_v) u[e] = (ue - pv) * rv;
    nx += xv * xv;
  }
  if (!with_norm) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) nx += __shfl_xor(nx, off, 64);
  if (lane == 0) red[wave] = nx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int wv = 0; wv < KRY_BLOCK / 64; ++wv) v += red[wv];
    partial[(int64_t)(KRY_MAXV - 1) * gridDim.x + blockIdx.x] = v;
  }
}

// r = f - Ax and this block's share of r . r in slot KRY_MAXV-1 of partial.
__global__ void __launch_bounds__(KRY_BLOCK)
residual_norm(const double *__restrict__ f, const double *__restrict__ Ax, double *__restrict__ r,
              int64_t N, double *__restrict__ partial) {
  __shared__ double red[(KRY_BLOCK / 64) * 2];
  double acc[2] = {0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < N;
       e0 += KRY_UNROLL * stride) {
    double fv[KRY_UNROLL], av[KRY_UNROLL];
#pragma unroll
    for (int u = 0; u < KRY_UNROLL; ++u) {
      const int64_t e = e0 + u * stride;
      fv[u] = e < N ? f[e] : 0.0;
      av[u] = e < N ? Ax[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < KRY_UNROLL; ++u) {
      const int64_t e = e0 + u * stride;
      const double rv = fv[u] - av[u];
      if (e < N) r[e] = rv;
      acc[1] += rv * rv;
    }
  }
  block_reduce_store<1>(acc, 0, 1, red, partial);
}

// Shares of x . x (slot 0) and y . y (slot KRY_MAXV-1) in one pass.
__global__ void __launch_bounds__(KRY_BLOCK)
two_norms(const double *__restrict__ x, const double *__restrict__ y, int64_t N,
          double *__restrict__ partial) {
  __shared__ double red[(KRY_BLOCK / 64) * 2];
  double acc[2] = {0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < N;
       e0 += KRY_UNROLL * stride) {
    double xv[KRY_UNROLL], yv[KRY_UNROLL];
#pragma unroll
    for (int u = 0; u < KRY_UNROLL; ++u) {
      const int64_t e = e0 + u * stride;
      xv[u] = e < N ? x[e] : 0.0;
      yv[u] = e < N ? y[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < KRY_UNROLL; ++u) {
      acc[0] += xv[u] * xv[u];
      acc[1] += yv[u] * yv[u];
    }
  }
  block_reduce_store<1>(acc, 1, 1, red, partial);
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

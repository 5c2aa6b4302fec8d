// Device kernels of the FP64 system matvec (Section 4.5): banded mode products
// for the matrix-free Kronecker form of eq. syst_mat, and a CSR product for the
// explicit form.
//
// Sum factorisation of A x = gamma (W_t (x) M_s) x + nu (M_t (x) K_s) x with
// K_s = sum_l (M ... K_l ... M) (eq. space_univ_par_mat) runs one pass per axis,
// carrying two tensors: a = x x_1 M_1 ... x_l M_l (mass chain) and
// b = the stiffness part of directions 1..l.  Each pass computes
//     out1 = in1 x_k Ba,          out2 = in2 x_k Bb + in1 x_k Bc
// (out1 / in2 optional), which gives a and b for the next axis; the time pass
// uses Bb = nu M_t, Bc = gamma W_t and writes only out2 = A x.
// Band storage: B[j*(2P+1) + P + m] = B[j][j+m], zero outside the matrix.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels_fd.h"

namespace stig {

// Axis with inner stride > 1: one thread per column (o, i), sliding a register
// window of 2P+1 entries along the axis, so each input entry is read once and
// loads are coalesced across i.
template <int P>
__global__ void band_pass_strided(const double *__restrict__ in1, const double *__restrict__ in2,
                                  double *__restrict__ out1, double *__restrict__ out2,
                                  const double *__restrict__ Ba, const double *__restrict__ Bb,
                                  const double *__restrict__ Bc, int n, int64_t inner,
                                  int64_t total_cols) {
  constexpr int B = 2 * P + 1;
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= total_cols) return;
  int64_t o = c / inner, i = c - o * inner;
  int64_t base = o * (int64_t)n * inner + i;
  double w1[B], w2[B];
#pragma unroll
  for (int m = 0; m < B; ++m) {
    int j = m - P;  // window holds entries j-P .. j+P for j = 0
    w1[m] = (j >= 0 && j < n) ? in1[base + (int64_t)j * inner] : 0.0;
    w2[m] = (in2 && j >= 0 && j < n) ? in2[base + (int64_t)j * inner] : 0.0;
  }
  cptr<double> cBa = as_const(Ba), cBb = as_const(Bb), cBc = as_const(Bc);
  for (int j = 0; j < n; ++j) {
    cptr<double> ra = cBa + (size_t)j * B;
    cptr<double> rb = cBb + (size_t)j * B;
    cptr<double> rc = cBc + (size_t)j * B;
    int64_t a = base + (int64_t)j * inner;
    if (out1) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < B; ++m) s += ra[m] * w1[m];
      out1[a] = s;
    }
    if (out2) {
      double s = 0.0;
      if (in2) {
#pragma unroll
        for (int m = 0; m < B; ++m) s += rb[m] * w2[m];
      }
#pragma unroll
      for (int m = 0; m < B; ++m) s += rc[m] * w1[m];
      out2[a] = s;
    }
#pragma unroll
    for (int m = 0; m < B - 1; ++m) {
      w1[m] = w1[m + 1];
      w2[m] = w2[m + 1];
    }
    int jn = j + P + 1;
    w1[B - 1] = (jn < n) ? in1[base + (int64_t)jn * inner] : 0.0;
    w2[B - 1] = (in2 && jn < n) ? in2[base + (int64_t)jn * inner] : 0.0;
  }
}

// Contiguous axis (inner == 1): one thread per output entry; the 2P+1 reads
// of neighbouring entries hit the same cache lines as the neighbouring threads.
template <int P>
__global__ void band_pass_contig(const double *__restrict__ in1, const double *__restrict__ in2,
                                 double *__restrict__ out1, double *__restrict__ out2,
                                 const double *__restrict__ Ba, const double *__restrict__ Bb,
                                 const double *__restrict__ Bc, int n, int64_t total) {
  constexpr int B = 2 * P + 1;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int64_t row = e / n;
  int j = (int)(e - row * n);
  const double *x1 = in1 + row * n;
  const double *x2 = in2 ? in2 + row * n : nullptr;
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int m = 0; m < B; ++m) {
    int jj = j + m - P;
    if (jj < 0 || jj >= n) continue;
    double v1 = x1[jj];
    if (out1) s1 += Ba[(size_t)j * B + m] * v1;
    if (out2) {
      s2 += Bc[(size_t)j * B + m] * v1;
      if (x2) s2 += Bb[(size_t)j * B + m] * x2[jj];
    }
  }
  if (out1) out1[e] = s1;
  if (out2) out2[e] = s2;
}

// Weighted sum along t: out[rhs][s] = sum_t w[t] * in[rhs][t][s] (ns spatial entries).
__global__ void time_weighted_sum(const double *__restrict__ in, double *__restrict__ out,
                                  const double *__restrict__ w, int nt, int64_t ns, int nrhs) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ns * nrhs) return;
  int64_t rhs = g / ns, s = g - rhs * ns;
  const double *x = in + rhs * ns * nt + s;
  double acc = 0.0;
  for (int t = 0; t < nt; ++t) acc += w[t] * x[(int64_t)t * ns];
  out[g] = acc;
}

// Outer product along t: out[rhs][t][s] = wa[t] * a[rhs][s] + wb[t] * b[rhs][s].
__global__ void time_outer2(const double *__restrict__ a, const double *__restrict__ b,
                            const double *__restrict__ wa, const double *__restrict__ wb,
                            double *__restrict__ out, int nt, int64_t ns, int nrhs) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ns * nrhs) return;
  int64_t rhs = g / ns, s = g - rhs * ns;
  double av = a[g], bv = b[g];
  double *o = out + rhs * ns * nt + s;
  for (int t = 0; t < nt; ++t) o[(int64_t)t * ns] = wa[t] * av + wb[t] * bv;
}

// Entries of A = W (x) M_s + Mt (x) K_s as CSR, one thread per row (t, s):
// for each time neighbour t' in the band and each entry (s, s') of the spatial
// pattern, column t' * ns + s' and value W[t][t'] M_s[s][s'] + Mt[t][t'] K_s[s][s'].
// Time bands as rows of 2P+1 coefficients (zero outside the matrix).
__global__ void kron_csr_fill(const int64_t *__restrict__ rowptr, int32_t *__restrict__ col,
                              double *__restrict__ val, const int64_t *__restrict__ rp2,
                              const int32_t *__restrict__ col2, const double *__restrict__ m2,
                              const double *__restrict__ k2, const double *__restrict__ wb,
                              const double *__restrict__ mb, int P, int nt, int64_t ns) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ns * nt) return;
  int64_t t = r / ns, s = r - t * ns;
  int64_t k = rowptr[r];
  const int B = 2 * P + 1;
  for (int64_t tp = t - P; tp <= t + P; ++tp) {
    if (tp < 0 || tp >= nt) continue;
    double wv = wb[t * B + (tp - t) + P], mv = mb[t * B + (tp - t) + P];
    for (int64_t e = rp2[s]; e < rp2[s + 1]; ++e) {
      col[k] = (int32_t)(tp * ns + col2[e]);
      val[k] = wv * m2[e] + mv * k2[e];
      ++k;
    }
  }
}

// y = A x for a CSR matrix (int64 row pointers, int32 columns).  One wavefront
// per row: rows of the space-time quarter-annulus operator hold ~700 entries.
__global__ void csr_spmv(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                         const double *__restrict__ val, const double *__restrict__ x,
                         double *__restrict__ y, int64_t nrows) {
  const int lane = threadIdx.x & 63;
  const int64_t wstride = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; row < nrows;
       row += wstride) {
    int64_t b = rowptr[row], e = rowptr[row + 1];
    double s = 0.0;
    for (int64_t k = b + lane; k < e; k += 64) s += val[k] * x[col[k]];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) y[row] = s;
  }
}

}  // namespace stig

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

// Axis with inner stride > 1: one thread per column (o, i) and chunk of jc
// entries along the axis (blockIdx.y), sliding a register window of 2P+1
// entries, so each input entry is read once per chunk (plus a 2P halo) and
// loads are coalesced across i.  Chunks (CH) only split the axis when there are
// too few columns to fill the device; CH false is the one-chunk form (jc unused).
template <int P, bool CH>
__global__ void band_pass_strided(const double *__restrict__ in1, const double *__restrict__ in2,
                                  double *__restrict__ out1, double *__restrict__ out2,
                                  const double *__restrict__ Ba, const double *__restrict__ Bb,
                                  const double *__restrict__ Bc, int n, int64_t inner,
                                  int64_t total_cols, int jc) {
  constexpr int B = 2 * P + 1;
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j0 = CH ? (int)blockIdx.y * jc : 0;
  const int j1 = CH ? (j0 + jc < n ? j0 + jc : n) : n;
  if (c >= total_cols || j0 >= n) return;
  int64_t o = c / inner, i = c - o * inner;
  int64_t base = o * (int64_t)n * inner + i;
  double w1[B], w2[B];
#pragma unroll
  for (int m = 0; m < B; ++m) {
    int j = j0 + m - P;  // window holds entries j-P .. j+P for j = j0
    w1[m] = (j >= 0 && j < n) ? in1[base + (int64_t)j * inner] : 0.0;
    w2[m] = (in2 && j >= 0 && j < n) ? in2[base + (int64_t)j * inner] : 0.0;
  }
  cptr<double> cBa = as_const(Ba), cBb = as_const(Bb), cBc = as_const(Bc);
  for (int j = j0; j < j1; ++j) {
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

// The last pass of the matvec fused with the residual: for each spatial
// column (stride inner along t) and chunk of jc time levels (blockIdx.y),
// r = f - (sum_m Bb[j][m] b[j+m-P] + Bc[j][m] a[j+m-P]) and this block's share
// of r . r in partial[blockIdx.y * gridDim.x + blockIdx.x] (fixed-order block
// reduction).
template <int P, bool CH>
__global__ void __launch_bounds__(256)
time_pass_residual(const double *__restrict__ a, const double *__restrict__ b,
                   const double *__restrict__ f, double *__restrict__ r,
                   const double *__restrict__ Bb, const double *__restrict__ Bc, int n,
                   int64_t inner, int64_t total_cols, int jc, double *__restrict__ partial) {
  constexpr int B = 2 * P + 1;
  __shared__ double red[4];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j0 = CH ? (int)blockIdx.y * jc : 0;
  const int j1 = CH ? (j0 + jc < n ? j0 + jc : n) : n;
  double acc = 0.0;
  if (c < total_cols) {
    const int64_t o = c / inner, i = c - o * inner;
    const int64_t base = o * (int64_t)n * inner + i;
    double wa[B], wb[B];
#pragma unroll
    for (int m = 0; m < B; ++m) {
      const int j = j0 + m - P;
      wa[m] = (j >= 0 && j < n) ? a[base + (int64_t)j * inner] : 0.0;
      wb[m] = (j >= 0 && j < n) ? b[base + (int64_t)j * inner] : 0.0;
    }
    cptr<double> cBb = as_const(Bb), cBc = as_const(Bc);
    for (int j = j0; j < j1; ++j) {
      cptr<double> rb = cBb + (size_t)j * B;
      cptr<double> rc = cBc + (size_t)j * B;
      const int64_t e = base + (int64_t)j * inner;
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < B; ++m) s += rb[m] * wb[m] + rc[m] * wa[m];
      const double rv = f[e] - s;
      r[e] = rv;
      acc += rv * rv;
#pragma unroll
      for (int m = 0; m < B - 1; ++m) {
        wa[m] = wa[m + 1];
        wb[m] = wb[m + 1];
      }
      const int jn = j + P + 1;
      wa[B - 1] = (jn < n) ? a[base + (int64_t)jn * inner] : 0.0;
      wb[B - 1] = (jn < n) ? b[base + (int64_t)jn * inner] : 0.0;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    partial[CH ? (int64_t)blockIdx.y * gridDim.x + blockIdx.x : (int64_t)blockIdx.x] =
        red[0] + red[1] + red[2] + red[3];
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

// Outer product along t: out[rhs][t][s] = wa[t] * a[rhs][s] + wb[t] * b[rhs][s],
// or f[rhs][t][s] minus it when f is given (f may be out).
__global__ void time_outer2(const double *__restrict__ a, const double *__restrict__ b,
                            const double *__restrict__ wa, const double *__restrict__ wb,
                            const double *f, double *out, int nt, int64_t ns, int nrhs) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ns * nrhs) return;
  int64_t rhs = g / ns, s = g - rhs * ns;
  double av = a[g], bv = b[g];
  double *o = out + rhs * ns * nt + s;
  if (f) {
    const double *fi = f + rhs * ns * nt + s;
    for (int t = 0; t < nt; ++t) o[(int64_t)t * ns] = fi[(int64_t)t * ns] - (wa[t] * av + wb[t] * bv);
  } else {
    for (int t = 0; t < nt; ++t) o[(int64_t)t * ns] = wa[t] * av + wb[t] * bv;
  }
}

// Space-time CSR of W (x) M_s + M_t (x) K_s from the spatial CSR (rp2, col2,
// m2, k2) and the time bands (wb, mb: rows of 2P+1, entry P + d at column
// t + d).  Row r = t ns + s holds, for each time neighbour tp = t-P .. t+P in
// range (ascending), the spatial row s shifted by tp ns.  One wavefront per
// row: its lanes write consecutive entries.
__global__ void kron_csr_fill(const int64_t *__restrict__ rowptr, int32_t *__restrict__ col,
                              double *__restrict__ val, const int64_t *__restrict__ rp2,
                              const int32_t *__restrict__ col2, const double *__restrict__ m2,
                              const double *__restrict__ k2, const double *__restrict__ wb,
                              const double *__restrict__ mb, int P, int nt, int64_t ns) {
  const int lane = threadIdx.x & 63;
  const int64_t wstride = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int B = 2 * P + 1;
  for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < ns * nt;
       r += wstride) {
    const int64_t t = r / ns, s = r - t * ns;
    const int64_t e0 = rp2[s], L = rp2[s + 1] - e0;
    const int64_t tlo = t - P < 0 ? 0 : t - P, thi = t + P < nt ? t + P : nt - 1;
    int64_t k = rowptr[r];
    for (int64_t tp = tlo; tp <= thi; ++tp, k += L) {
      const double wv = wb[t * B + (tp - t) + P], mv = mb[t * B + (tp - t) + P];
      for (int64_t e = lane; e < L; e += 64) {
        col[k + e] = (int32_t)(tp * ns + col2[e0 + e]);
        val[k + e] = wv * m2[e0 + e] + mv * k2[e0 + e];
      }
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

// Spatial part of the matvec with general sparse spatial factors (Section 4.5:
// only the spatial and time factors of A are stored): for every slice s of
// ns entries (one time level of one right-hand side),
//     a[s][i] = sum_k Me[k][i] x[s][ce[k][i]],   b[s][i] = sum_k Ke[k][i] x[s][ce[k][i]].
// M_s and K_s share one pattern, stored padded and column-major: entry k of
// row i at k * ns + i (padding: column i, value 0), with the width a multiple
// of KU, so the loads of a wavefront's rows are coalesced.  A thread owns row i
// for TT consecutive slices: each matrix entry is loaded once per TT slices,
// and neighbouring rows read neighbouring columns of x.  The entries are taken
// KU at a time, the next group's loaded while the current group's KU x TT
// gathers of x are in flight.  Blocks are numbered so that the slice chunks of
// one row block run on one XCD (blocks are dispatched round-robin over the 8
// XCDs): its rows' matrix entries come from HBM once into that XCD's L2.
constexpr int ELL_KU = 2;  // the padded width is a multiple of this

template <int TT, int KU>
__global__ void __launch_bounds__(256)
spatial_ell_pair(const double *__restrict__ x, double *__restrict__ a, double *__restrict__ b,
                 const int32_t *__restrict__ ce, const double *__restrict__ me,
                 const double *__restrict__ ke, int width, int64_t ns, int64_t nslices,
                 int nchunks) {
  const unsigned nb = gridDim.x, q = nb / 8, rem = nb % 8, xcd = blockIdx.x % 8;
  const unsigned g = xcd * q + (xcd < rem ? xcd : rem) + blockIdx.x / 8;
  const int64_t i = (int64_t)(g / nchunks) * blockDim.x + threadIdx.x;
  const int64_t s0 = (int64_t)(g % nchunks) * TT;
  if (i >= ns || s0 >= nslices) return;
  const int nt = (int)(nslices - s0 < TT ? nslices - s0 : TT);
  const double *xs = x + s0 * ns;
  double sa[TT], sb[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) sa[t] = sb[t] = 0.0;
  int cn[KU];
  double mn[KU], kn[KU];
#pragma unroll
  for (int u = 0; u < KU; ++u) {
    cn[u] = ce[(int64_t)u * ns + i];
    mn[u] = me[(int64_t)u * ns + i];
    kn[u] = ke[(int64_t)u * ns + i];
  }
  for (int k0 = 0; k0 < width; k0 += KU) {
    int c[KU];
    double mv[KU], kv[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      c[u] = cn[u];
      mv[u] = mn[u];
      kv[u] = kn[u];
    }
    if (k0 + KU < width) {
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int64_t e = (int64_t)(k0 + KU + u) * ns + i;
        cn[u] = ce[e];
        mn[u] = me[e];
        kn[u] = ke[e];
      }
    }
    if (nt == TT) {
#pragma unroll
      for (int u = 0; u < KU; ++u)
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          const double xv = xs[(int64_t)t * ns + c[u]];
          sa[t] += mv[u] * xv;
          sb[t] += kv[u] * xv;
        }
    } else {
#pragma unroll
      for (int u = 0; u < KU; ++u)
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          if (t < nt) {
            const double xv = xs[(int64_t)t * ns + c[u]];
            sa[t] += mv[u] * xv;
            sb[t] += kv[u] * xv;
          }
        }
    }
  }
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    if (t < nt) {
      a[(s0 + t) * ns + i] = sa[t];
      b[(s0 + t) * ns + i] = sb[t];
    }
  }
}

// The same product with M_s and K_s stored by diagonals: diagonal k holds the
// entries at offset offs[k] = col - row, row i's at k * ns + i (zero where the
// row has none, e.g. near the boundary of a tensor-product pattern).  The
// column of every lane is i + offs[k] with a uniform offset, so no column
// indices are loaded and a wavefront's gathers stay contiguous.  Padding
// entries have value 0 and a column clamped into [0, ns).
template <int TT, int KU>
__global__ void __launch_bounds__(256)
spatial_dia_pair(const double *__restrict__ x, double *__restrict__ a, double *__restrict__ b,
                 const int32_t *__restrict__ offs, const double *__restrict__ me,
                 const double *__restrict__ ke, int ndiag, int64_t ns, int64_t nslices,
                 int nchunks) {
  const unsigned nb = gridDim.x, q = nb / 8, rem = nb % 8, xcd = blockIdx.x % 8;
  const unsigned g = xcd * q + (xcd < rem ? xcd : rem) + blockIdx.x / 8;
  const int64_t i = (int64_t)(g / nchunks) * blockDim.x + threadIdx.x;
  const int64_t s0 = (int64_t)(g % nchunks) * TT;
  if (i >= ns || s0 >= nslices) return;
  const int nt = (int)(nslices - s0 < TT ? nslices - s0 : TT);
  const double *xs = x + s0 * ns;
  cptr<int32_t> co = as_const(offs);
  double sa[TT], sb[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) sa[t] = sb[t] = 0.0;
  for (int k0 = 0; k0 < ndiag; k0 += KU) {
    int64_t c[KU];
    double mv[KU], kv[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int64_t e = (int64_t)(k0 + u) * ns + i;
      mv[u] = me[e];
      kv[u] = ke[e];
      const int64_t cc = i + co[k0 + u];
      c[u] = cc < 0 ? 0 : (cc >= ns ? ns - 1 : cc);
    }
    if (nt == TT) {
#pragma unroll
      for (int u = 0; u < KU; ++u)
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          const double xv = xs[(int64_t)t * ns + c[u]];
          sa[t] += mv[u] * xv;
          sb[t] += kv[u] * xv;
        }
    } else {
#pragma unroll
      for (int u = 0; u < KU; ++u)
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          if (t < nt) {
            const double xv = xs[(int64_t)t * ns + c[u]];
            sa[t] += mv[u] * xv;
            sb[t] += kv[u] * xv;
          }
        }
    }
  }
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    if (t < nt) {
      a[(s0 + t) * ns + i] = sa[t];
      b[(s0 + t) * ns + i] = sb[t];
    }
  }
}

// The diagonal form with x staged in LDS, for patterns whose offsets span
// little: a block's rows [i0, i0 + 256) read columns [i0 + omin, i0 + 255 +
// omax] only, so the block copies that range of its TT slices to LDS with
// coalesced loads and gathers from there (the gathers of the global form are
// bound by the L1 access rate).  Dynamic LDS: TT * span doubles.
template <int TT, int KU>
__global__ void __launch_bounds__(256)
spatial_dia_lds(const double *__restrict__ x, double *__restrict__ a, double *__restrict__ b,
                const int32_t *__restrict__ offs, const double *__restrict__ me,
                const double *__restrict__ ke, int ndiag, int64_t ns, int64_t nslices, int nchunks,
                int omin, int span) {
  extern __shared__ __align__(16) unsigned char smem[];
  double *xl = reinterpret_cast<double *>(smem);  // [TT][span]
  const unsigned nb = gridDim.x, q = nb / 8, rem = nb % 8, xcd = blockIdx.x % 8;
  const unsigned g = xcd * q + (xcd < rem ? xcd : rem) + blockIdx.x / 8;
  const int64_t i0 = (int64_t)(g / nchunks) * blockDim.x;
  const int64_t i = i0 + threadIdx.x;
  const int64_t s0 = (int64_t)(g % nchunks) * TT;
  const int nt = (int)(nslices - s0 < TT ? nslices - s0 : TT);
  // staged columns [cb, cb + span), clamped to the matrix
  int64_t cb = i0 + omin;
  if (cb < 0) cb = 0;
  const double *xs = x + s0 * ns;
  constexpr int FU = 8;
  for (int e0 = threadIdx.x; e0 < TT * span; e0 += 256 * FU) {
    double v[FU];
#pragma unroll
    for (int u = 0; u < FU; ++u) {
      const int e = e0 + u * 256;
      const int t = e / span, j = e - t * span;
      const int64_t col = cb + j;
      const bool ok = e < TT * span && t < nt && col < ns;
      v[u] = xs[ok ? (int64_t)t * ns + col : 0];
    }
#pragma unroll
    for (int u = 0; u < FU; ++u) {
      const int e = e0 + u * 256;
      if (e < TT * span) xl[e] = v[u];
    }
  }
  __syncthreads();
  if (i >= ns) return;
  cptr<int32_t> co = as_const(offs);
  double sa[TT], sb[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) sa[t] = sb[t] = 0.0;
  for (int k0 = 0; k0 < ndiag; k0 += KU) {
    int c[KU];
    double mv[KU], kv[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int64_t e = (int64_t)(k0 + u) * ns + i;
      mv[u] = me[e];
      kv[u] = ke[e];
      int64_t cc = i + co[k0 + u];
      cc = cc < 0 ? 0 : (cc >= ns ? ns - 1 : cc);
      c[u] = (int)(cc - cb);
    }
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        const double xv = xl[t * span + c[u]];
        sa[t] += mv[u] * xv;
        sb[t] += kv[u] * xv;
      }
  }
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    if (t < nt) {
      a[(s0 + t) * ns + i] = sa[t];
      b[(s0 + t) * ns + i] = sb[t];
    }
  }
}

// The diagonal form for wide patterns whose offsets come in runs of
// consecutive values (a tensor-product pattern: runs of 2p+1 along x_1).  For
// run g (first offset goff[g], length glen[g] <= ELL_RUN_MAX, first diagonal
// gdiag[g]) a wavefront loads the window x[i0w + goff[g] .. i0w + goff[g] + 63 +
// glen[g] - 1] of each of its TT slices once into its own LDS and every lane
// reads its glen[g] shifted values from there, instead of one L1-bound gather
// per diagonal.  Diagonals are summed in the same order as spatial_dia_pair.
// Window indices are clamped into [0, ns): such entries only meet zero values.
constexpr int ELL_RUN_MAX = 32;

template <int TT>
__global__ void __launch_bounds__(256)
spatial_dia_runs(const double *__restrict__ x, double *__restrict__ a, double *__restrict__ b,
                 const int32_t *__restrict__ runs, const double *__restrict__ me,
                 const double *__restrict__ ke, int nruns, int64_t ns, int64_t nslices,
                 int nchunks) {
  __shared__ double win[4][TT][64 + ELL_RUN_MAX];
  const unsigned nb = gridDim.x, q = nb / 8, rem = nb % 8, xcd = blockIdx.x % 8;
  const unsigned g = xcd * q + (xcd < rem ? xcd : rem) + blockIdx.x / 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0w = (int64_t)(g / nchunks) * blockDim.x + wave * 64;
  const int64_t i = i0w + lane;
  const int64_t s0 = (int64_t)(g % nchunks) * TT;
  const int nt = (int)(nslices - s0 < TT ? nslices - s0 : TT);
  if (i0w >= ns) return;  // whole wavefront past the rows (no block barrier below)
  const bool valid = i < ns;
  const int64_t iv = valid ? i : 0;
  const double *xs = x + s0 * ns;
  cptr<int32_t> cr = as_const(runs);  // [nruns][3]: first offset, length, first diagonal
  double sa[TT], sb[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) sa[t] = sb[t] = 0.0;
  auto clampc = [&](int64_t c) { return c < 0 ? (int64_t)0 : (c >= ns ? ns - 1 : c); };
  for (int r = 0; r < nruns; ++r) {
    const int o = cr[3 * r], len = cr[3 * r + 1], k0 = cr[3 * r + 2];
    const int64_t c0 = clampc(i0w + o + lane), c1 = clampc(i0w + o + 64 + lane);
    double w0[TT], w1[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      const int tt = t < nt ? t : 0;
      w0[t] = xs[(int64_t)tt * ns + c0];
      w1[t] = lane < len - 1 ? xs[(int64_t)tt * ns + c1] : 0.0;
    }
    // the previous run's reads of the window are done before it is overwritten
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      win[wave][t][lane] = w0[t];
      if (lane < ELL_RUN_MAX) win[wave][t][64 + lane] = w1[t];
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int d = 0; d < len; ++d) {
      const int64_t e = (int64_t)(k0 + d) * ns + iv;
      const double mv = me[e], kv = ke[e];
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        const double xv = win[wave][t][lane + d];
        sa[t] += mv * xv;
        sb[t] += kv * xv;
      }
    }
  }
  if (!valid) return;
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    if (t < nt) {
      a[(s0 + t) * ns + i] = sa[t];
      b[(s0 + t) * ns + i] = sb[t];
    }
  }
}

// Spatial part of the matvec in one pass over each (rhs, t) slice (d = 2, 3):
//   a = x x_1 M_1 x_2 M_2 x_3 M_3,   b = x x_1 K_1 x_2 M_2 x_3 M_3
//       + x x_1 M_1 x_2 K_2 x_3 M_3 + x x_1 M_1 x_2 M_2 x_3 K_3
// (for d = 2 the third factors are the identity and zero).  A block owns R
// rows y (all x) of one slice and a chunk of planes z, and streams along z.
// Thread (yy, xx) keeps one column: its rows of the x band and of the y band
// live in registers.  Per input plane it moves its window rows yy and yy + R
// (the y halo of P rows on each side needs R >= 2P) to LDS, forms their x
// products (M_1, K_1), and after one barrier the y products of its own row,
// which enter a register window of 2P + 1 planes; the z products (scalar
// band loads, z is uniform) give a and b.  The LDS tiles are double-buffered
// so one barrier per plane suffices, and input planes are loaded SPF planes
// ahead of their LDS store into registers.  One read of x (plus halos, mostly L2 hits) and one
// write of a and b: about 24 bytes per unknown, against 88 for three separate
// axis passes.  Bands (device, [n][2P+1], entry m of row i at column
// i + m - P, zero outside): M0, K0 (x), M1, K1 (y), M2, K2 (z).
constexpr int STENCIL_SPF = 1;  // input planes in flight per thread
constexpr int STENCIL_ZC = 24;  // most output planes per block (2P halo planes are recomputed)

template <int P>
__device__ __forceinline__ int stencil_ldx(int nx) {
  return nx + 2 * P;  // x rows with P zero columns on each side
}

constexpr int STENCIL_THREADS = 512;  // at most R * nx threads per block

template <int P>
__global__ void __launch_bounds__(STENCIL_THREADS) __attribute__((amdgpu_waves_per_eu(P <= 3 ? 4 : 2)))
spatial_stencil(const double *__restrict__ x, double *__restrict__ a, double *__restrict__ b,
                const double *__restrict__ M0, const double *__restrict__ K0,
                const double *__restrict__ M1, const double *__restrict__ K1,
                const double *__restrict__ M2, const double *__restrict__ K2, int nx, int ny,
                int nz, int R, int ZC, int64_t slices) {
  constexpr int B = 2 * P + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  const int rows = R + 2 * P, ldx = stencil_ldx<P>(nx);
  // [2][rows][ldx] input rows, [2][rows][nx] M_1 and K_1 products
  double *xin = reinterpret_cast<double *>(smem);
  double *xu = xin + 2 * rows * ldx;
  double *xv = xu + 2 * rows * nx;
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * rows * ldx; e += blockDim.x) xin[e] = 0.0;  // zero x pads
  const int ntiles = (ny + R - 1) / R, nchunks = (nz + ZC - 1) / ZC;
  // Blocks go to the 8 XCDs round-robin (block b to XCD b % 8); each XCD takes a
  // contiguous run of tiles instead, y tiles fastest, so that tiles next to
  // each other run on one XCD at the same time and their halo rows hit its L2.
  const int64_t nb = gridDim.x, q = nb / 8, rem = nb % 8, xcd = blockIdx.x % 8;
  int64_t blk = xcd * q + min(xcd, rem) + blockIdx.x / 8;
  const int y0 = (int)(blk % ntiles) * R;
  blk /= ntiles;
  const int chunk = (int)(blk % nchunks);
  const int64_t slice = blk / nchunks;
  if (slice >= slices) return;  // whole block: no barrier is skipped by part of it
  const int z0 = chunk * ZC, z1 = min(nz, z0 + ZC);  // outputs z0 .. z1-1
  const int64_t plane = (int64_t)nx * ny;
  const double *xs = x + slice * plane * nz;
  double *as = a + slice * plane * nz, *bs = b + slice * plane * nz;
  const bool act = tid < R * nx;
  const int yy = act ? tid / nx : 0, xx = act ? tid - yy * nx : 0;
  const int y = y0 + yy;
  const bool out_ok = act && y < ny;
  const bool two = act && yy + R < rows;  // second window row yy + R
  // window rows yy, yy + R are the global rows y0 - P + yy, y0 - P + yy + R
  const int ya = y0 - P + yy, yb = ya + R;
  const bool oka = act && ya >= 0 && ya < ny, okb = two && yb >= 0 && yb < ny;
  double bxm[B], bxk[B], bym[B], byk[B];
#pragma unroll
  for (int m = 0; m < B; ++m) {
    bxm[m] = M0[xx * B + m];
    bxk[m] = K0[xx * B + m];
    bym[m] = out_ok ? M1[y * B + m] : 0.0;
    byk[m] = out_ok ? K1[y * B + m] : 0.0;
  }
  cptr<double> mz = as_const(M2), kz = as_const(K2);
  double Aw[B], Bw[B];
#pragma unroll
  for (int m = 0; m < B; ++m) Aw[m] = Bw[m] = 0.0;
  // input planes z0 - P .. z1 + P - 1
  const int zfirst = z0 - P, zlast = z1 + P;
  double ra[STENCIL_SPF], rb[STENCIL_SPF];
  auto gload = [&](int zin, double &va, double &vb) {
    const bool zok = zin >= 0 && zin < nz;
    const int64_t base = (int64_t)(zok ? zin : 0) * plane + xx;
    const double u = xs[base + (int64_t)(oka ? ya : 0) * nx];
    const double v = xs[base + (int64_t)(okb ? yb : 0) * nx];
    va = (zok && oka) ? u : 0.0;
    vb = (zok && okb) ? v : 0.0;
  };
#pragma unroll
  for (int k = 0; k < STENCIL_SPF; ++k) gload(zfirst + k, ra[k], rb[k]);
  // pushes the oldest loaded plane into LDS buffer `buf` and loads plane `znext`
  auto push = [&](int buf, int znext) {
    double *xi = xin + buf * rows * ldx + P;
    if (act) xi[yy * ldx + xx] = ra[0];
    if (two) xi[(yy + R) * ldx + xx] = rb[0];
#pragma unroll
    for (int k = 0; k + 1 < STENCIL_SPF; ++k) {
      ra[k] = ra[k + 1];
      rb[k] = rb[k + 1];
    }
    gload(znext, ra[STENCIL_SPF - 1], rb[STENCIL_SPF - 1]);
  };
  __syncthreads();  // x pads are zero before the first row store
  push(0, zfirst + STENCIL_SPF);
  __syncthreads();
  // x products (M_1, K_1) of window rows yy and yy + R of the plane in buffer buf
  auto xpass_store = [&](int buf, double *u, double *v) {
    const double *xi = xin + buf * rows * ldx + P;
    if (act) {
      double su = 0.0, sv = 0.0, tu = 0.0, tv = 0.0;
      const double *r0 = xi + yy * ldx + xx - P, *r1 = r0 + R * ldx;
#pragma unroll
      for (int m = 0; m < B; ++m) {
        const double c0 = r0[m];
        su = fma(bxm[m], c0, su);
        sv = fma(bxk[m], c0, sv);
      }
      u[yy * nx + xx] = su;
      v[yy * nx + xx] = sv;
      if (two) {
#pragma unroll
        for (int m = 0; m < B; ++m) {
          const double c1 = r1[m];
          tu = fma(bxm[m], c1, tu);
          tv = fma(bxk[m], c1, tv);
        }
        u[(yy + R) * nx + xx] = tu;
        v[(yy + R) * nx + xx] = tv;
      }
    }
  };
  // Plane j = zin - zfirst goes to window slot j % B: the plane loop is
  // unrolled B times, so every slot index is a compile-time constant and the
  // window needs no register moves.  The output of plane zin - P reads the
  // planes j - 2P .. j, i.e. slots (ph + 1 + m) % B for m = 0 .. 2P.
  for (int base = 0; zfirst + base < zlast; base += B) {
#pragma unroll
    for (int ph = 0; ph < B; ++ph) {
      const int zin = zfirst + base + ph;
      if (zin < zlast) {  // block-uniform: every thread takes the same barriers
        const int buf = (base + ph) & 1;
        double *u = xu + buf * rows * nx, *v = xv + buf * rows * nx;
        xpass_store(buf, u, v);
        // plane zin + 1 into the other buffer (its previous plane's x products
        // are done: they preceded the last barrier); one barrier per plane
        push(buf ^ 1, zin + 1 + STENCIL_SPF);
        __syncthreads();
        // y products of this thread's row -> window slot ph
        double An = 0.0, Bn = 0.0;
#pragma unroll
        for (int m = 0; m < B; ++m) {
          const double uu = u[(yy + m) * nx + xx], vv = v[(yy + m) * nx + xx];
          An = fma(bym[m], uu, An);
          Bn = fma(bym[m], vv, Bn);
          Bn = fma(byk[m], uu, Bn);
        }
        Aw[ph] = An;
        Bw[ph] = Bn;
        const int z = zin - P;
        if (z >= z0 && out_ok) {
          double sa = 0.0, sb = 0.0;
#pragma unroll
          for (int m = 0; m < B; ++m) {
            const int sl = (ph + 1 + m) % B;
            const double cm = mz[z * B + m], ck = kz[z * B + m];
            sa = fma(cm, Aw[sl], sa);
            sb = fma(ck, Aw[sl], sb);
            sb = fma(cm, Bw[sl], sb);
          }
          const int64_t o = (int64_t)z * plane + (int64_t)y * nx + xx;
          as[o] = sa;
          bs[o] = sb;
        }
      }
    }
  }
}
}  // namespace stig

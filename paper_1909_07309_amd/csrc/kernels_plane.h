// Fused mode products along the two fastest axes of the unknown tensor.
//
// With x (mode 1) fastest and y (mode 2) next, the tensor is a stack of n x n
// planes X_o[y][x].  The two mode products X x_1 Op_x x_2 Op_y of Section 2.3
// act on each plane as
//     Y_o = Op_y X_o Op_x^T,
// so one pass over memory does both (steps 2 and 4 of Algorithm 1 need them on
// every time slice and every z index).  The plane stays in LDS, the
// intermediate Z = X_o Op_x^T never leaves registers.
//
// MFMA mapping (one wave per 16-column strip x' = 16w .. 16w+15 of the output):
//  * product 1, Z[y][x'] = sum_x X[y][x] Op_x[x'][x]: A operand = the plane
//    (rows y, read from LDS), B operand = Op_x^T for the strip (registers, loaded
//    once per block); one accumulator tile per 16 rows of y.
//  * product 2, Y[y'][x'] = sum_y Op_y[y'][y] Z[y][x']: B operand = Z taken
//    straight from the accumulators of product 1.  Lane (c, g) of a wave holds
//    Z[16T + out_row(g, v)][16w + c]; the contraction over y is summed in the
//    order in which the lanes already hold it (k slot (s, g, u) <-> y =
//    16T + out_row(g, v)), and the A operand (Op_y, from LDS) is read in that
//    same order.  No transpose, no LDS round trip for Z.
//  * n = 16q + 1 (the workload sizes 65 and 49): the last row / column of the
//    plane, of Op_x and of Op_y are handled on the vector ALU: the k = 16q
//    terms as rank-one initialisations of the accumulators, the output row and
//    column 16q by short dot products reduced across the four k-slices.
#pragma once

#include "kernels_fd.h"

namespace stig {

constexpr int PLANE_MAX_N = 80;

// Vector-ALU view of operand elements and accumulators.
template <typename TC> struct PlaneVal;
template <> struct PlaneVal<double> {
  typedef double vt;
  __device__ static inline double get(double a, int) { return a; }
  __device__ static inline double of(double e) { return e; }
  __device__ static inline double to_elem(double x) { return x; }
};
template <> struct PlaneVal<float> {
  typedef float vt;
  __device__ static inline float get(float a, int) { return a; }
  __device__ static inline float of(float e) { return e; }
  __device__ static inline float to_elem(float x) { return x; }
};
template <> struct PlaneVal<bf16> {
  typedef float vt;
  __device__ static inline float get(v4s a, int u) { return bf16_bits_to_float((uint16_t)a[u]); }
  __device__ static inline float of(uint16_t e) { return bf16_bits_to_float(e); }
  __device__ static inline uint16_t to_elem(float x) { return float_to_bf16_bits(x); }
};

// Y_o = Op_y X_o Op_x^T for o = 0 .. planes-1, X_o = in + o*in_stride (row y, x
// fastest), Y_o = out + o*out_stride (strides >= n*n; padding left untouched).
// Op_x, Op_y: n x n row-major, compute precision.  NC = n at compile time (65 or
// 49), or 0 for any n <= PLANE_MAX_N taken from the argument (zero padded to 80).
// Block = 64 * (NMAX / 16) threads; dynamic LDS = (2 * NR + 1) * ld elements.
// Persistent: block b handles planes b, b + gridDim.x, ..., the next plane is
// loaded into registers while the current one is multiplied.
template <typename Tin, typename Tout, typename TC, int NC>
__global__ void __launch_bounds__(64 * ((NC ? NC : PLANE_MAX_N) / 16), 2)
mode_gemm_plane(const Tin *__restrict__ in, Tout *__restrict__ out,
                const typename Mfma<TC>::elem *__restrict__ opx,
                const typename Mfma<TC>::elem *__restrict__ opy, int n_arg, int64_t planes,
                int64_t in_stride, int64_t out_stride) {
  typedef Mfma<TC> MF;
  typedef typename MF::elem E;
  typedef PlaneVal<TC> PV;
  typedef typename PV::vt VT;
  constexpr int NMAX = NC ? NC : PLANE_MAX_N;
  constexpr int Q = NMAX / 16, R = NMAX % 16;
  static_assert(R <= 1, "compile-time plane size must be 16q or 16q + 1");
  constexpr int NT = 64 * Q;
  constexpr int KPL = MF::KPL, KSTEP = MF::KSTEP;
  constexpr int KS = 16 * Q / KSTEP;  // MFMA k steps over y (or x) < 16q
  constexpr int SPT = 16 / KSTEP;     // k steps per 16-row accumulator tile
  constexpr int NR = 16 * Q + R;      // LDS rows; columns 0 .. NR-1 are read
  constexpr int PER = (NMAX * NMAX + NT - 1) / NT;
  const int n = NC ? NC : n_arg;
  const int nn = n * n;
  const int ld = lds_ld<TC>(NR);
  extern __shared__ __align__(16) unsigned char smem[];
  E *xs = reinterpret_cast<E *>(smem);  // current plane [NR][ld]
  E *ys = xs + NR * ld;                 // Op_y [NR][ld]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;

  for (int e = tid; e < NR * ld; e += NT) {
    int j = e / ld, k = e - j * ld;
    bool ok = j < n && k < n;
    E v = opy[ok ? j * n + k : 0];
    ys[e] = ok ? v : MF::zero();
    xs[e] = MF::zero();
  }
  // B operand of product 1 for this wave's strip: Op_x[16w + c][k]
  E bx[KS][KPL];
#pragma unroll
  for (int s = 0; s < KS; ++s)
#pragma unroll
    for (int u = 0; u < KPL; ++u) {
      int k = s * KSTEP + g * KPL + u, j = 16 * w + c;
      bool ok = j < n && k < n;
      E v = opx[ok ? j * n + k : 0];
      bx[s][u] = ok ? v : MF::zero();
    }
  // fringe of Op_x: column 16q of the strip's rows (registers) and row 16q
  // (LDS row NR of the Op_y buffer, read in k-slice order)
  VT bxf = 0, oxff = 0;
  if constexpr (R != 0) {
    bxf = PV::of(opx[(16 * w + c) * n + 16 * Q]);
    oxff = PV::of(opx[16 * Q * n + 16 * Q]);
    for (int k = tid; k < NR; k += NT) ys[NR * ld + k] = opx[16 * Q * n + k];
  }
  const E *oxf = ys + NR * ld;

  Tin pre[PER];
  auto gload = [&](int64_t p) {
    const bool pv = p < planes;
    const Tin *src = in + (pv ? p : 0) * in_stride;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      int e = tid + i * NT;
      pre[i] = src[(pv && e < nn) ? e : 0];
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      int e = tid + i * NT;
      if (e < nn) {
        int y = e / n, x = e - y * n;
        xs[y * ld + x] = MF::from_f64(Conv<Tin>::to_f64(pre[i]));
      }
    }
  };
  auto xor_sum = [](VT x) {
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
  };

  int64_t p = blockIdx.x;
  gload(p);
  __syncthreads();  // zero fill done before the first plane lands
  lstore();
  __syncthreads();
  for (; p < planes; p += gridDim.x) {
    gload(p + gridDim.x);
    // ---- product 1: Z = X Op_x^T, rows y < 16q, this wave's 16 columns
    typename MF::acc acc1[Q];
    VT zp[Q];  // partial sums of Z[16T + c][16q] over this lane's k-slice
#pragma unroll
    for (int T = 0; T < Q; ++T) {
      zp[T] = 0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc1[T][v] = 0;
        if constexpr (R != 0) acc1[T][v] = PV::of(xs[(16 * T + MF::out_row(g, v)) * ld + 16 * Q]) * bxf;
      }
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      typename MF::frag b = MF::make(bx[s]);
      VT of[KPL];
      if constexpr (R != 0) {
#pragma unroll
        for (int u = 0; u < KPL; ++u) of[u] = PV::of(oxf[s * KSTEP + g * KPL + u]);
      }
#pragma unroll
      for (int T = 0; T < Q; ++T) {
        typename MF::frag a = MF::load(xs + (16 * T + c) * ld + s * KSTEP + g * KPL);
        acc1[T] = MF::mma(a, b, acc1[T]);
        if constexpr (R != 0) {
#pragma unroll
          for (int u = 0; u < KPL; ++u) zp[T] += PV::get(a, u) * of[u];
        }
      }
    }
    // ---- fringe of product 1: row 16q of Z (zr, this lane's column), column
    // 16q of Z (zp[T] -> Z[16T + c][16q]), corner Z[16q][16q] (zcc)
    VT zr = 0, zcc = 0;
    if constexpr (R != 0) {
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int u = 0; u < KPL; ++u) {
          VT xv = PV::of(xs[16 * Q * ld + s * KSTEP + g * KPL + u]);
          zr += xv * PV::of(bx[s][u]);
          zcc += xv * PV::of(oxf[s * KSTEP + g * KPL + u]);
        }
      VT x64 = PV::of(xs[16 * Q * ld + 16 * Q]);
      zr = xor_sum(zr) + x64 * bxf;
      zcc = xor_sum(zcc) + x64 * oxff;
#pragma unroll
      for (int T = 0; T < Q; ++T) zp[T] = xor_sum(zp[T]) + PV::of(xs[(16 * T + c) * ld + 16 * Q]) * oxff;
    }
    __syncthreads();  // every wave is done with this plane
    lstore();         // next plane into LDS (waits for its loads)

    // ---- product 2: Y = Op_y Z
    typename MF::acc acc2[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc2[t][v] = 0;
        if constexpr (R != 0) acc2[t][v] = PV::of(ys[(16 * t + MF::out_row(g, v)) * ld + 16 * Q]) * zr;
      }
    VT yr = 0, yc = 0, ycc = 0;  // output row 16q, column 16q, corner (partials)
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int T = s / SPT, v0 = (s % SPT) * KPL;
      E be[KPL];
#pragma unroll
      for (int u = 0; u < KPL; ++u) be[u] = PV::to_elem(acc1[T][v0 + u]);
      typename MF::frag b = MF::make(be);
      const int kcol = 16 * T + MF::out_row(g, v0);  // y of slot u is kcol + u
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        typename MF::frag a = MF::load(ys + (16 * t + c) * ld + kcol);
        acc2[t] = MF::mma(a, b, acc2[t]);
      }
      if constexpr (R != 0) {
#pragma unroll
        for (int u = 0; u < KPL; ++u) {
          VT oy = PV::of(ys[16 * Q * ld + kcol + u]);
          VT zc = __shfl(zp[T], MF::out_row(g, v0 + u), 64);  // Z[kcol + u][16q]
          yr += oy * PV::of(be[u]);
          yc += PV::of(ys[(16 * w + c) * ld + kcol + u]) * zc;
          ycc += oy * zc;
        }
      }
    }
    Tout *dst = out + p * out_stride;
#pragma unroll
    for (int t = 0; t < Q; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int yy = 16 * t + MF::out_row(g, v), xx = 16 * w + c;
        if (NC != 0 || (yy < n && xx < n))
          dst[yy * n + xx] = Conv<Tout>::from_f64((double)acc2[t][v]);
      }
    if constexpr (R != 0) {
      VT oyy = PV::of(ys[16 * Q * ld + 16 * Q]);
      yr = xor_sum(yr) + oyy * zr;
      yc = xor_sum(yc) + PV::of(ys[(16 * w + c) * ld + 16 * Q]) * zcc;
      ycc = xor_sum(ycc) + oyy * zcc;
      if (g == 0) {
        dst[16 * Q * n + 16 * w + c] = Conv<Tout>::from_f64((double)yr);
        dst[(16 * w + c) * n + 16 * Q] = Conv<Tout>::from_f64((double)yc);
      }
      if (tid == 0) dst[16 * Q * n + 16 * Q] = Conv<Tout>::from_f64((double)ycc);
    }
    __syncthreads();  // the next plane is in LDS
  }
}

}  // namespace stig

// Mode products with a parity-split eigenbasis.
//
// When a 1D pencil (K_l, M_l) is persymmetric (J K J = K, J M J = M for the
// reversal J, as for uniform open knot vectors), its eigenvectors can be taken
// even or odd: U[n-1-x][k] = +-U[x][k].  With the even modes first (NE of
// them) and the odd modes after (M of them), n = 2M + ODD, NE = M + ODD, a
// mode product splits into two half-size products around a butterfly:
//   forward (Y = U^T X along the axis):
//     e[x] = X[x] + X[n-1-x], o[x] = X[x] - X[n-1-x]  (x < M), e[M] = X[M] (ODD)
//     Y[0 .. NE) = Ue^T e,  Y[NE .. n) = Uo^T o
//   backward (X = U Y):
//     E = Ue Y[0 .. NE), O = Uo Y[NE .. n)
//     X[x] = E[x] + O[x], X[n-1-x] = E[x] - O[x]  (x < M), X[M] = E[M] (ODD)
// where Ue (NE x NE) and Uo (M x M) are the rows x < NE, resp. x < M, of the
// even and odd eigenvectors.  Half the multiply-adds of the dense product.
#pragma once

#include "kernels_fd.h"

namespace stig {

// Y = X x_k U^T (FWD) or X x_k U (!FWD) along one axis (layout as mode_gemm:
// columns c = (o, i), entries at o*n*inner + k*inner + i), with the split
// operator: opE (NE x NE) and opO (M x M) row-major, rows = output index of
// the half product, columns = contraction index (FWD: Ue^T, Uo^T; !FWD: Ue, Uo).
// M is a multiple of 16.  Each wave streams 16-column strips; the operators
// sit in LDS; the B operand (the butterflied or split input) is loaded straight
// into registers in the MFMA layout, one strip ahead.
// Dynamic LDS: (NE + M) * lds_ld<TC>(NE) elements.
constexpr int SYM_THREADS = 256;

template <typename Tin, typename Tout, typename TC, int M, bool ODD, bool FWD>
__global__ void __launch_bounds__(SYM_THREADS)
mode_gemm_sym(const Tin *__restrict__ in, Tout *__restrict__ out,
              const typename Mfma<TC>::elem *__restrict__ opE,
              const typename Mfma<TC>::elem *__restrict__ opO, int64_t inner,
              int64_t total_cols) {
  typedef Mfma<TC> MF;
  typedef typename MF::elem E;
  static_assert(M % 16 == 0, "half size must be a multiple of 16");
  constexpr int NE = M + (ODD ? 1 : 0), N = 2 * M + (ODD ? 1 : 0);
  constexpr int Q = M / 16, KS = M / MF::KSTEP, KPL = MF::KPL;
  extern __shared__ __align__(16) unsigned char smem[];
  const int ld = lds_ld<TC>(NE);
  E *le = reinterpret_cast<E *>(smem);  // [NE][ld]
  E *lo = le + NE * ld;                 // [M][ld]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < NE * NE; e += SYM_THREADS) {
    int j = e / NE, k = e - j * NE;
    le[j * ld + k] = opE[e];
  }
  for (int e = tid; e < M * M; e += SYM_THREADS) {
    int j = e / M, k = e - j * M;
    lo[j * ld + k] = opO[e];
  }
  __syncthreads();

  const int64_t nstrips = (total_cols + 15) >> 4;
  const int64_t slab = (int64_t)N * inner;
  const uint32_t uinner = (uint32_t)inner;
  const int col = lane & 15, kg = lane >> 4;
  const int64_t wstride = (int64_t)gridDim.x * (SYM_THREADS / 64);
  auto locate = [&](int64_t c, int64_t &base, int64_t &step) {
    if (inner == 1) {
      base = c * N;
      step = 1;
    } else {
      uint32_t o = (uint32_t)c / uinner, i = (uint32_t)c - o * uinner;
      base = (int64_t)o * slab + i;
      step = inner;
    }
  };
  struct Frags {
    E e[KS][KPL], o[KS][KPL];
    double m;  // ODD: the middle entry (contraction index M of the even half)
  };
  // B operands of one strip (branch-free loads)
  auto load_b = [&](int64_t strip, Frags &f) {
    const int64_t c = strip * 16 + col;
    const bool cvalid = strip < nstrips && c < total_cols;
    int64_t base, step;
    locate(cvalid ? c : 0, base, step);
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int u = 0; u < KPL; ++u) {
        const int k = s * MF::KSTEP + kg * KPL + u;  // < M
        double a, b;
        if (FWD) {
          a = Conv<Tin>::to_f64(in[cvalid ? base + (int64_t)k * step : 0]);
          b = Conv<Tin>::to_f64(in[cvalid ? base + (int64_t)(N - 1 - k) * step : 0]);
          f.e[s][u] = MF::from_f64(a + b);
          f.o[s][u] = MF::from_f64(a - b);
        } else {
          a = Conv<Tin>::to_f64(in[cvalid ? base + (int64_t)k * step : 0]);
          b = Conv<Tin>::to_f64(in[cvalid ? base + (int64_t)(NE + k) * step : 0]);
          f.e[s][u] = MF::from_f64(a);
          f.o[s][u] = MF::from_f64(b);
        }
      }
    f.m = 0.0;
    if (ODD) f.m = MF::to_f64(MF::from_f64(Conv<Tin>::to_f64(in[cvalid ? base + (int64_t)M * step : 0])));
  };
  auto process = [&](int64_t strip, const Frags &f) {
    const int64_t c = strip * 16 + col;
    const bool cvalid = c < total_cols;
    int64_t base, step;
    locate(cvalid ? c : 0, base, step);
    typename MF::acc ae[Q], ao[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ao[t][v] = 0;
        // contraction index M of the even half: rank-one start
        ae[t][v] = ODD ? (typename MF::acc_elem)(MF::to_f64(le[(16 * t + MF::out_row(kg, v)) * ld + M]) * f.m)
                       : (typename MF::acc_elem)0;
      }
    const E *abe = le + col * ld + kg * KPL, *abo = lo + col * ld + kg * KPL;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      typename MF::frag bfe = MF::make(f.e[s]), bfo = MF::make(f.o[s]);
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        ae[t] = MF::mma(MF::load(abe + 16 * t * ld + s * MF::KSTEP), bfe, ae[t]);
        ao[t] = MF::mma(MF::load(abo + 16 * t * ld + s * MF::KSTEP), bfo, ao[t]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // ODD: row M of the even half on the vector ALU
    double fr = 0.0;
    if (ODD) {
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int u = 0; u < KPL; ++u)
          fr += MF::to_f64(le[M * ld + s * MF::KSTEP + kg * KPL + u]) * MF::to_f64(f.e[s][u]);
      fr += __shfl_xor(fr, 16, 64);
      fr += __shfl_xor(fr, 32, 64);
      fr += MF::to_f64(le[M * ld + M]) * f.m;
    }
    if (cvalid) {
#pragma unroll
      for (int t = 0; t < Q; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = 16 * t + MF::out_row(kg, v);  // < M
          const double ve = (double)ae[t][v], vo = (double)ao[t][v];
          if (FWD) {
            out[base + (int64_t)j * step] = Conv<Tout>::from_f64(ve);
            out[base + (int64_t)(NE + j) * step] = Conv<Tout>::from_f64(vo);
          } else {
            out[base + (int64_t)j * step] = Conv<Tout>::from_f64(ve + vo);
            out[base + (int64_t)(N - 1 - j) * step] = Conv<Tout>::from_f64(ve - vo);
          }
        }
      if (ODD && kg == 0) out[base + (int64_t)M * step] = Conv<Tout>::from_f64(fr);
    }
  };
  int64_t strip = (int64_t)blockIdx.x * (SYM_THREADS / 64) + wave;
  Frags fnext;
  load_b(strip, fnext);
  for (; strip < nstrips; strip += wstride) {
    Frags f = fnext;
    load_b(strip + wstride, fnext);
    process(strip, f);
  }
}

}  // namespace stig

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

// CG adjacent columns of one storage type as one aligned vector access.
template <typename T, int CG>
struct alignas(sizeof(T) * CG) ColPack {
  T v[CG];
};

// Y = X x_k U^T (FWD) or X x_k U (!FWD) along one axis (layout as mode_gemm:
// columns c = (o, i), entries at o*n*inner + k*inner + i), with the split
// operator: opE (NE x NE) and opO (M x M) row-major, rows = output index of
// the half product, columns = contraction index (FWD: Ue^T, Uo^T; !FWD: Ue, Uo).
// M is a multiple of 16.  Each wave streams strips of 16 CG columns; the
// operators sit in LDS; the B operand (the butterflied or split input) is
// loaded straight into registers in the MFMA layout, one strip ahead.
// Column groups: lane l % 16 owns the CG adjacent columns 16 CG s + CG (l % 16)
// .. + CG - 1 of strip s and feeds them to CG separate MFMA tiles that share
// each A fragment; its loads and stores are CG-element vectors (8 bytes for
// FP32 pairs instead of 4).  Columns are independent,
// so the permuted column order within a strip changes nothing.  CG > 1 needs
// inner % CG == 0 and inner > 1 (the CG columns are then contiguous).
// Dynamic LDS: (NE + M) * lds_ld<TC>(NE) elements.
constexpr int SYM_THREADS = 256;

template <typename Tin, typename Tout, typename TC, int M, bool ODD, bool FWD, int CG>
__global__ void __launch_bounds__(SYM_THREADS)
mode_gemm_sym(const Tin *__restrict__ in, Tout *__restrict__ out,
              const typename Mfma<TC>::elem *__restrict__ opE,
              const typename Mfma<TC>::elem *__restrict__ opO, int64_t inner,
              int64_t total_cols) {
  typedef Mfma<TC> MF;
  typedef typename MF::elem E;
  typedef ColPack<Tin, CG> PIn;
  typedef ColPack<Tout, CG> POut;
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

  const int64_t nstrips = (total_cols + 16 * CG - 1) / (16 * CG);
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
  auto vload = [&](int64_t idx) { return *reinterpret_cast<const PIn *>(in + idx); };
  auto vstore = [&](int64_t idx, const double (&v)[CG]) {
    POut pk;
#pragma unroll
    for (int g = 0; g < CG; ++g) pk.v[g] = Conv<Tout>::from_f64(v[g]);
    *reinterpret_cast<POut *>(out + idx) = pk;
  };
  // value u of a B fragment (KPL values per lane)
  auto felem = [&](const typename MF::frag &f, int u) -> double {
    if constexpr (KPL == 1) return MF::to_f64(f);
    else return MF::to_f64((E)(uint16_t)f[u]);
  };
  struct Frags {
    typename MF::frag e[CG][KS], o[CG][KS];
    double m[CG];  // ODD: the middle entry (contraction index M of the even half)
  };
  // B operands of one strip (branch-free loads)
  auto load_b = [&](int64_t strip, Frags &f) {
    const int64_t c = (strip * 16 + col) * CG;
    const bool cvalid = strip < nstrips && c < total_cols;
    int64_t base, step;
    locate(cvalid ? c : 0, base, step);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      E te[CG][KPL], to[CG][KPL];
#pragma unroll
      for (int u = 0; u < KPL; ++u) {
        const int k = s * MF::KSTEP + kg * KPL + u;  // < M
        const PIn a = vload(cvalid ? base + (int64_t)k * step : 0);
        const PIn b = vload(cvalid ? base + (int64_t)(FWD ? N - 1 - k : NE + k) * step : 0);
#pragma unroll
        for (int g = 0; g < CG; ++g) {
          const double x = Conv<Tin>::to_f64(a.v[g]), y = Conv<Tin>::to_f64(b.v[g]);
          te[g][u] = MF::from_f64(FWD ? x + y : x);
          to[g][u] = MF::from_f64(FWD ? x - y : y);
        }
      }
#pragma unroll
      for (int g = 0; g < CG; ++g) {
        f.e[g][s] = MF::make(te[g]);
        f.o[g][s] = MF::make(to[g]);
      }
    }
#pragma unroll
    for (int g = 0; g < CG; ++g) f.m[g] = 0.0;
    if (ODD) {
      const PIn mm = vload(cvalid ? base + (int64_t)M * step : 0);
#pragma unroll
      for (int g = 0; g < CG; ++g) f.m[g] = MF::to_f64(MF::from_f64(Conv<Tin>::to_f64(mm.v[g])));
    }
  };
  auto process = [&](int64_t strip, const Frags &f) {
    const int64_t c = (strip * 16 + col) * CG;
    const bool cvalid = c < total_cols;
    int64_t base, step;
    locate(cvalid ? c : 0, base, step);
    typename MF::acc ae[CG][Q], ao[CG][Q];
#pragma unroll
    for (int t = 0; t < Q; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // contraction index M of the even half: rank-one start
        const double cm = ODD ? MF::to_f64(le[(16 * t + MF::out_row(kg, v)) * ld + M]) : 0.0;
#pragma unroll
        for (int g = 0; g < CG; ++g) {
          ao[g][t][v] = 0;
          ae[g][t][v] = ODD ? (typename MF::acc_elem)(cm * f.m[g]) : (typename MF::acc_elem)0;
        }
      }
    const E *abe = le + col * ld + kg * KPL, *abo = lo + col * ld + kg * KPL;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        const typename MF::frag fe = MF::load(abe + 16 * t * ld + s * MF::KSTEP);
        const typename MF::frag fo = MF::load(abo + 16 * t * ld + s * MF::KSTEP);
#pragma unroll
        for (int g = 0; g < CG; ++g) {
          ae[g][t] = MF::mma(fe, f.e[g][s], ae[g][t]);
          ao[g][t] = MF::mma(fo, f.o[g][s], ao[g][t]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // ODD: row M of the even half on the vector ALU
    double fr[CG];
#pragma unroll
    for (int g = 0; g < CG; ++g) fr[g] = 0.0;
    if (ODD) {
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int u = 0; u < KPL; ++u) {
          const double w = MF::to_f64(le[M * ld + s * MF::KSTEP + kg * KPL + u]);
#pragma unroll
          for (int g = 0; g < CG; ++g) fr[g] += w * felem(f.e[g][s], u);
        }
      const double wm = MF::to_f64(le[M * ld + M]);
#pragma unroll
      for (int g = 0; g < CG; ++g) {
        fr[g] += __shfl_xor(fr[g], 16, 64);
        fr[g] += __shfl_xor(fr[g], 32, 64);
        fr[g] += wm * f.m[g];
      }
    }
    if (cvalid) {
#pragma unroll
      for (int t = 0; t < Q; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = 16 * t + MF::out_row(kg, v);  // < M
          double lo_[CG], hi_[CG];
#pragma unroll
          for (int g = 0; g < CG; ++g) {
            const double ve = (double)ae[g][t][v], vo = (double)ao[g][t][v];
            lo_[g] = FWD ? ve : ve + vo;
            hi_[g] = FWD ? vo : ve - vo;
          }
          vstore(base + (int64_t)j * step, lo_);
          vstore(base + (int64_t)(FWD ? NE + j : N - 1 - j) * step, hi_);
        }
      if (ODD && kg == 0) vstore(base + (int64_t)M * step, fr);
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

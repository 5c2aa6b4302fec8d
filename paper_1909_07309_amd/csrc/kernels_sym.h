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
// loaded straight into registers in the MFMA layout, the next strip's k steps
// one by one under the current strip's products.
// Column groups: lane l % 16 owns the CG adjacent columns 16 CG s + CG (l % 16)
// .. + CG - 1 of strip s and feeds them to CG separate MFMA tiles that share
// each A fragment; its loads and stores are CG-element vectors (8 bytes for
// FP32 pairs instead of 4).  Columns are independent,
// so the permuted column order within a strip changes nothing.  CG > 1 needs
// inner % CG == 0 and inner > 1 (the CG columns are then contiguous).
// Dynamic LDS: (NE + M) * lds_ld<TC>(NE) elements.
constexpr int SYM_THREADS = 256;

// waves per SIMD the registers are sized for: 3 (168 registers), FP32 with
// column pairs 2
template <typename TC, int CG> __host__ __device__ constexpr int sym_waves() {
  return sizeof(typename Mfma<TC>::elem) == 4 && CG > 1 ? 2 : 3;
}
template <typename Tin, typename Tout, typename TC, int M, bool ODD, bool FWD, int CG>
__global__ void __launch_bounds__(SYM_THREADS, (sym_waves<TC, CG>()))
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
  // The B operand of a strip stays in registers as the raw entries (both
  // mirror entries per contraction index), one slot per k step; the butterfly
  // is formed when the slot is used.  Slot s takes the next strip's k step s
  // as soon as the MFMAs of step s have read it, so the next strip's loads run
  // under this strip's products with one set of registers (a second full set,
  // double buffering, costs a wave per SIMD).
  PIn ra[KS][KPL], rb[KS][KPL];  // entries k and its mirror (FWD) / partner (!FWD)
  PIn rm;                         // ODD: the middle entry M
  struct Col {
    int64_t base, step;
    bool valid;
  };
  auto column = [&](int64_t strip) {
    const int64_t c = (strip * 16 + col) * CG;
    Col r;
    r.valid = strip < nstrips && c < total_cols;
    locate(r.valid ? c : 0, r.base, r.step);
    return r;
  };
  auto issue = [&](const Col &L, int s) {
#pragma unroll
    for (int u = 0; u < KPL; ++u) {
      const int k = s * MF::KSTEP + kg * KPL + u;  // < M
      ra[s][u] = vload(L.base + (int64_t)k * L.step);
      rb[s][u] = vload(L.base + (int64_t)(FWD ? N - 1 - k : NE + k) * L.step);
    }
  };
  // fragments of k step s for column group g: even and odd halves
  auto frags = [&](int s, int g, typename MF::frag &fe, typename MF::frag &fo) {
    E te[KPL], to[KPL];
#pragma unroll
    for (int u = 0; u < KPL; ++u) {
      const double x = Conv<Tin>::to_f64(ra[s][u].v[g]), y = Conv<Tin>::to_f64(rb[s][u].v[g]);
      te[u] = MF::from_f64(FWD ? x + y : x);
      to[u] = MF::from_f64(FWD ? x - y : y);
    }
    fe = MF::make(te);
    fo = MF::make(to);
  };
  auto process = [&](const Col &cc, const Col &nx) {
    double fm[CG];  // ODD: the middle entry, as the operand type rounds it
#pragma unroll
    for (int g = 0; g < CG; ++g) fm[g] = ODD ? MF::to_f64(MF::from_f64(Conv<Tin>::to_f64(rm.v[g]))) : 0.0;
    if (ODD) rm = vload(nx.base + (int64_t)M * nx.step);
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
          ae[g][t][v] = ODD ? (typename MF::acc_elem)(cm * fm[g]) : (typename MF::acc_elem)0;
        }
      }
    const E *abe = le + col * ld + kg * KPL, *abo = lo + col * ld + kg * KPL;
    // ODD: row M of the even half on the vector ALU, accumulated in the same
    // k steps from the same operand values
    double fr[CG];
#pragma unroll
    for (int g = 0; g < CG; ++g) fr[g] = 0.0;
    // A fragments one k step ahead, read before the previous step's MFMAs
    typename MF::frag ane[Q], ano[Q];
    auto afr = [&](int s) {
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        ane[t] = MF::load(abe + 16 * t * ld + s * MF::KSTEP);
        ano[t] = MF::load(abo + 16 * t * ld + s * MF::KSTEP);
      }
    };
    afr(0);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      typename MF::frag fe[Q], fo[Q];
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        fe[t] = ane[t];
        fo[t] = ano[t];
      }
      double w[KPL];
      if (ODD) {
#pragma unroll
        for (int u = 0; u < KPL; ++u) w[u] = MF::to_f64(le[M * ld + s * MF::KSTEP + kg * KPL + u]);
      }
      if (s + 1 < KS) afr(s + 1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int g = 0; g < CG; ++g) {
        typename MF::frag be, bo;
        frags(s, g, be, bo);
#pragma unroll
        for (int t = 0; t < Q; ++t) {
          ae[g][t] = MF::mma(fe[t], be, ae[g][t]);
          ao[g][t] = MF::mma(fo[t], bo, ao[g][t]);
        }
        if (ODD) {
#pragma unroll
          for (int u = 0; u < KPL; ++u) fr[g] += w[u] * felem(be, u);
        }
      }
      issue(nx, s);  // past the last strip: column 0 again, never used
      __builtin_amdgcn_sched_barrier(0);
    }
    if (ODD) {
      const double wm = MF::to_f64(le[M * ld + M]);
#pragma unroll
      for (int g = 0; g < CG; ++g) {
        fr[g] += __shfl_xor(fr[g], 16, 64);
        fr[g] += __shfl_xor(fr[g], 32, 64);
        fr[g] += wm * fm[g];
      }
    }
    if (cc.valid) {
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
          vstore(cc.base + (int64_t)j * cc.step, lo_);
          vstore(cc.base + (int64_t)(FWD ? NE + j : N - 1 - j) * cc.step, hi_);
        }
      if (ODD && kg == 0) vstore(cc.base + (int64_t)M * cc.step, fr);
    }
  };
  int64_t strip = (int64_t)blockIdx.x * (SYM_THREADS / 64) + wave;
  Col cur = column(strip);
  // the first strip's loads go out before the operator copy, so the two overlap
#pragma unroll
  for (int s = 0; s < KS; ++s) issue(cur, s);
  if (ODD) rm = vload(cur.base + (int64_t)M * cur.step);
  for (int e = tid; e < NE * NE; e += SYM_THREADS) {
    int j = e / NE, k = e - j * NE;
    le[j * ld + k] = opE[e];
  }
  for (int e = tid; e < M * M; e += SYM_THREADS) {
    int j = e / M, k = e - j * M;
    lo[j * ld + k] = opO[e];
  }
  __syncthreads();
  for (; strip < nstrips; strip += wstride) {
    const Col nx = column(strip + wstride);
    process(cur, nx);
    cur = nx;
  }
}

}  // namespace stig

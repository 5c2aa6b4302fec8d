// Fused x/y mode products with parity-split eigenbases in both directions.
//
// With n = 2M + ODD, NE = M + ODD, and the even modes of a direction before
// its odd ones (see kernels_sym.h), the two-sided product of an n x n plane
// decouples into four quadrants after a two-dimensional butterfly:
//   forward  Y_ab = (U^a_y)^T B_ab U^b_x,  a, b in {even, odd},
//            B_ab[y][x] = X[y][x] +-_b X[y][n-1-x] +-_a X[n-1-y][x] +-_ab X[n-1-y][n-1-x]
//            (half coordinates y, x; on the middle row / column the mirror image
//            is the point itself and is counted once),
//   backward Z_ab = U^a_y Y_ab (U^b_x)^T, then X at the four mirror points is
//            the signed sum of the four Z_ab at the half coordinates.
// Each of the four waves of a block transforms one quadrant (sizes NE or M per
// side): half the multiply-adds of the dense fused plane kernel.  The plane is
// loaded orbit by orbit (the four mirror points of a half coordinate) so that
// the butterfly happens in registers on the way into LDS.
#pragma once

#include "kernels_plane.h"

namespace stig {

// One quadrant: Out = OpY In OpX^T with In (16Q+RY) x (16Q+RX), OpX
// (16Q+RX)^2 and OpY (16Q+RY)^2 in LDS (leading dimensions ldi, ldo, ldo).
// store(row, col, value) receives every output entry.
template <typename TC, int Q, int RY, int RX, typename StoreF>
__device__ inline void quad_transform(const typename Mfma<TC>::elem *in, int ldi,
                                      const typename Mfma<TC>::elem *opx,
                                      const typename Mfma<TC>::elem *opy, int ldo, int c, int g,
                                      StoreF store) {
  typedef Mfma<TC> MF;
  typedef typename MF::elem E;
  typedef PlaneVal<TC> PV;
  typedef typename PV::vt VT;
  constexpr int KSTEP = MF::KSTEP, KPL = MF::KPL, KS = 16 * Q / KSTEP, SPT = 16 / KSTEP;
  auto xor_sum = [](VT x) {
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
  };
  const E *oxrow = opx + 16 * Q * ldo;  // RX: row 16Q of OpX
  VT bxf[Q];                            // RX: column 16Q of OpX, rows 16j + c
  VT oxff = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) bxf[j] = 0;
  if constexpr (RX != 0) {
#pragma unroll
    for (int j = 0; j < Q; ++j) bxf[j] = PV::of(opx[(16 * j + c) * ldo + 16 * Q]);
    oxff = PV::of(oxrow[16 * Q]);
  }
  // ---- product 1, every strip: Z[y][16j + c] for y < 16Q
  typename MF::acc acc1[Q][Q];  // [strip j][row tile T]
  VT zp[Q];                     // RX: partial sums of Z[16T + c][16Q]
#pragma unroll
  for (int T = 0; T < Q; ++T) {
    zp[T] = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc1[j][T][v] = 0;
        if constexpr (RX != 0)  // contraction index 16Q: rank-one start
          acc1[j][T][v] = PV::of(in[(16 * T + MF::out_row(g, v)) * ldi + 16 * Q]) * bxf[j];
      }
  }
  // fringe sums of product 1, accumulated in the same k steps from the same
  // operand values: row 16Q of Z (zr, RY), column 16Q (zp, RX), corner (zc2)
  VT zr[Q], zcc = 0, zc2 = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) zr[j] = 0;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    VT of[KPL], xv[KPL];
    if constexpr (RX != 0) {
#pragma unroll
      for (int u = 0; u < KPL; ++u) of[u] = PV::of(oxrow[s * KSTEP + g * KPL + u]);
    }
    if constexpr (RY != 0) {
#pragma unroll
      for (int u = 0; u < KPL; ++u) xv[u] = PV::of(in[16 * Q * ldi + s * KSTEP + g * KPL + u]);
    }
    typename MF::frag bq[Q];  // B fragments of OpX rows 16j + c
#pragma unroll
    for (int j = 0; j < Q; ++j) bq[j] = MF::load(opx + (16 * j + c) * ldo + s * KSTEP + g * KPL);
#pragma unroll
    for (int T = 0; T < Q; ++T) {
      typename MF::frag a = MF::load(in + (16 * T + c) * ldi + s * KSTEP + g * KPL);
#pragma unroll
      for (int j = 0; j < Q; ++j) acc1[j][T] = MF::mma(a, bq[j], acc1[j][T]);
      if constexpr (RX != 0) {
#pragma unroll
        for (int u = 0; u < KPL; ++u) zp[T] += PV::get(a, u) * of[u];
      }
    }
    if constexpr (RY != 0) {
#pragma unroll
      for (int u = 0; u < KPL; ++u) {
#pragma unroll
        for (int j = 0; j < Q; ++j) zr[j] += xv[u] * PV::get(bq[j], u);
        if constexpr (RX != 0) zc2 += xv[u] * of[u];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if constexpr (RY != 0) {
#pragma unroll
    for (int j = 0; j < Q; ++j) zr[j] = xor_sum(zr[j]);
    if constexpr (RX != 0) {
      const VT x64 = PV::of(in[16 * Q * ldi + 16 * Q]);
#pragma unroll
      for (int j = 0; j < Q; ++j) zr[j] += x64 * bxf[j];
      if constexpr (RX != 0) zcc = xor_sum(zc2) + x64 * oxff;
    }
  }
  if constexpr (RX != 0) {
#pragma unroll
    for (int T = 0; T < Q; ++T) zp[T] = xor_sum(zp[T]) + PV::of(in[(16 * T + c) * ldi + 16 * Q]) * oxff;
  }
  // ---- product 2, all strips at once: Out = OpY Z (each OpY fragment read once
  // per k step serves every strip; Q*Q independent accumulator chains)
  VT yc[Q], ycc = 0;  // RX: output column 16Q (rows 16t + c), corner
#pragma unroll
  for (int t = 0; t < Q; ++t) yc[t] = 0;
  typename MF::acc acc2[Q][Q];  // [strip j][row tile t]
  VT yr[Q];                     // RY: output row 16Q of strip j
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    yr[j] = 0;
#pragma unroll
    for (int t = 0; t < Q; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc2[j][t][v] = 0;
        if constexpr (RY != 0)
          acc2[j][t][v] = PV::of(opy[(16 * t + MF::out_row(g, v)) * ldo + 16 * Q]) * zr[j];
      }
  }
  // RX: Z[y][16Q] at the contraction indices of a k step, gathered across
  // lanes one step ahead (the shuffle's latency runs under a step's MFMAs)
  VT zcn[KPL];
  auto zc_of = [&](int s) {
#pragma unroll
    for (int u = 0; u < KPL; ++u)
      zcn[u] = __shfl(zp[s / SPT], MF::out_row(g, (s % SPT) * KPL + u), 64);
  };
  if constexpr (RX != 0) zc_of(0);
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int T = s / SPT, v0 = (s % SPT) * KPL;
    const int kcol = 16 * T + MF::out_row(g, v0);  // contraction index of slot u: kcol + u
    typename MF::frag a[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) a[t] = MF::load(opy + (16 * t + c) * ldo + kcol);
    VT zc[KPL];
    if constexpr (RX != 0) {
#pragma unroll
      for (int u = 0; u < KPL; ++u) zc[u] = zcn[u];
      if (s + 1 < KS) zc_of(s + 1);
#pragma unroll
      for (int t = 0; t < Q; ++t)
#pragma unroll
        for (int u = 0; u < KPL; ++u) yc[t] += PV::get(a[t], u) * zc[u];
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      E be[KPL];
#pragma unroll
      for (int u = 0; u < KPL; ++u) be[u] = PV::to_elem(acc1[j][T][v0 + u]);
      typename MF::frag b = MF::make(be);
#pragma unroll
      for (int t = 0; t < Q; ++t) acc2[j][t] = MF::mma(a[t], b, acc2[j][t]);
      if constexpr (RY != 0) {
#pragma unroll
        for (int u = 0; u < KPL; ++u) yr[j] += PV::of(opy[16 * Q * ldo + kcol + u]) * PV::of(be[u]);
      }
    }
    if constexpr (RY != 0 && RX != 0) {
#pragma unroll
      for (int u = 0; u < KPL; ++u) ycc += PV::of(opy[16 * Q * ldo + kcol + u]) * zc[u];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
#pragma unroll
    for (int t = 0; t < Q; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) store(16 * t + MF::out_row(g, v), 16 * j + c, (VT)acc2[j][t][v]);
    if constexpr (RY != 0) {
      const VT r = xor_sum(yr[j]) + PV::of(opy[16 * Q * ldo + 16 * Q]) * zr[j];
      if (g == 0) store(16 * Q, 16 * j + c, r);
    }
  }
  if constexpr (RX != 0) {
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      VT y = xor_sum(yc[t]);
      if constexpr (RY != 0) y += PV::of(opy[(16 * t + c) * ldo + 16 * Q]) * zcc;
      if (g == 0) store(16 * t + c, 16 * Q, y);
    }
    if constexpr (RY != 0) {
      ycc = xor_sum(ycc) + PV::of(opy[16 * Q * ldo + 16 * Q]) * zcc;
      if (g == 0 && c == 0) store(16 * Q, 16 * Q, ycc);
    }
  }
}

// One 16-column strip j of a quadrant: Out[.][16j + c'] = (OpY In OpX^T)
// for c' < 16, with In (16Q+RY) x (16Q+RX), OpX (16Q+RX)^2 and OpY (16Q+RY)^2
// in LDS (leading dimensions ldi, ldo, ldo).  The strips of a quadrant are
// independent: product 2 of strip j only needs strip j of Z = In OpX^T.
// RY / RX: the quadrant's y / x size is 16Q + 1 (contraction index 16Q on
// the vector ALU, as rank-one starts).  The fringe row 16Q of the output
// (RY) is computed by every strip for its own columns; OWN: this strip also
// computes the fringe column 16Q (of Z and of the output) and, with RY, the
// corner.  store(row, col, value) receives every output entry of the strip,
// after before_store() (called once, when the strip no longer reads `in`).
template <typename TC, int Q, int RY, int RX, bool OWN, typename StoreF, typename SyncF>
__device__ inline void quad_strip(const typename Mfma<TC>::elem *in, int ldi,
                                  const typename Mfma<TC>::elem *opx,
                                  const typename Mfma<TC>::elem *opy, int ldo, int c, int g, int j,
                                  StoreF store, SyncF before_store) {
  typedef Mfma<TC> MF;
  typedef PlaneVal<TC> PV;
  typedef typename PV::vt VT;
  static_assert(!OWN || RX, "the fringe column exists only with RX");
  constexpr int KSTEP = MF::KSTEP, KPL = MF::KPL, KS = 16 * Q / KSTEP, SPT = 16 / KSTEP;
  auto xor_sum = [](VT x) {
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
  };
  const typename MF::elem *oxrow = opx + 16 * Q * ldo;  // RX: row 16Q of OpX
  const typename MF::elem *oxj = opx + (16 * j + c) * ldo;  // OpX row 16j + c
  VT bxf = 0, oxff = 0;  // RX: OpX[16j + c][16Q], OpX[16Q][16Q]
  if constexpr (RX != 0) {
    bxf = PV::of(oxj[16 * Q]);
    oxff = PV::of(oxrow[16 * Q]);
  }
  // ---- product 1: Z[y][16j + c] for y < 16Q
  typename MF::acc acc1[Q];  // [row tile T]
  VT zp[Q];                  // OWN: partial sums of Z[16T + c][16Q]
#pragma unroll
  for (int T = 0; T < Q; ++T) {
    zp[T] = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      acc1[T][v] = 0;
      if constexpr (RX != 0)  // contraction index 16Q: rank-one start
        acc1[T][v] = PV::of(in[(16 * T + MF::out_row(g, v)) * ldi + 16 * Q]) * bxf;
    }
  }
  // fragments of k step s (B: OpX row 16j + c, A: input rows 16T + c), read
  // one step ahead, before the previous step's MFMAs (the fences keep them
  // there), so the LDS latency runs under those MFMAs
  typename MF::frag bqn, aqn[Q];
  auto frags1 = [&](int s) {
    bqn = MF::load(oxj + s * KSTEP + g * KPL);
#pragma unroll
    for (int T = 0; T < Q; ++T) aqn[T] = MF::load(in + (16 * T + c) * ldi + s * KSTEP + g * KPL);
  };
  frags1(0);
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    typename MF::frag bq = bqn, aq[Q];
#pragma unroll
    for (int T = 0; T < Q; ++T) aq[T] = aqn[T];
    VT of[KPL];
    if constexpr (OWN) {
#pragma unroll
      for (int u = 0; u < KPL; ++u) of[u] = PV::of(oxrow[s * KSTEP + g * KPL + u]);
    }
    if (s + 1 < KS) frags1(s + 1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int T = 0; T < Q; ++T) {
      acc1[T] = MF::mma(aq[T], bq, acc1[T]);
      if constexpr (OWN) {
#pragma unroll
        for (int u = 0; u < KPL; ++u) zp[T] += PV::get(aq[T], u) * of[u];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  // fringe of product 1: row 16Q of Z for this strip (zr, RY), column 16Q
  // (zp, OWN), corner (zcc, OWN and RY)
  VT zr = 0, zcc = 0;
  if constexpr (RY != 0) {
    VT zc2 = 0;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int u = 0; u < KPL; ++u) {
        const VT xv = PV::of(in[16 * Q * ldi + s * KSTEP + g * KPL + u]);
        zr += xv * PV::of(oxj[s * KSTEP + g * KPL + u]);
        if constexpr (OWN) zc2 += xv * PV::of(oxrow[s * KSTEP + g * KPL + u]);
      }
    zr = xor_sum(zr);
    if constexpr (RX != 0) {
      const VT x64 = PV::of(in[16 * Q * ldi + 16 * Q]);
      zr += x64 * bxf;
      if constexpr (OWN) zcc = xor_sum(zc2) + x64 * oxff;
    }
  }
  if constexpr (OWN) {
#pragma unroll
    for (int T = 0; T < Q; ++T) zp[T] = xor_sum(zp[T]) + PV::of(in[(16 * T + c) * ldi + 16 * Q]) * oxff;
  }
  // ---- product 2: Out = OpY Z for the strip
  VT yc[Q], ycc = 0;  // OWN: output column 16Q (rows 16t + c), corner
#pragma unroll
  for (int t = 0; t < Q; ++t) yc[t] = 0;
  typename MF::acc acc2[Q];  // [row tile t]
  VT yr = 0;                 // RY: output row 16Q of the strip
#pragma unroll
  for (int t = 0; t < Q; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      acc2[t][v] = 0;
      if constexpr (RY != 0)
        acc2[t][v] = PV::of(opy[(16 * t + MF::out_row(g, v)) * ldo + 16 * Q]) * zr;
    }
  // A fragments of OpY (and, RY, its row 16Q) one k step ahead, as in product 1
  typename MF::frag an[Q];
  VT oyn[KPL];
  auto frags2 = [&](int s) {
    const int kc = 16 * (s / SPT) + MF::out_row(g, (s % SPT) * KPL);
#pragma unroll
    for (int t = 0; t < Q; ++t) an[t] = MF::load(opy + (16 * t + c) * ldo + kc);
    if constexpr (RY != 0) {
#pragma unroll
      for (int u = 0; u < KPL; ++u) oyn[u] = PV::of(opy[16 * Q * ldo + kc + u]);
    }
  };
  frags2(0);
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int T = s / SPT, v0 = (s % SPT) * KPL;
    typename MF::frag a[Q];
    VT oyr[KPL];  // RY: OpY row 16Q at the contraction indices of this step
#pragma unroll
    for (int t = 0; t < Q; ++t) a[t] = an[t];
#pragma unroll
    for (int u = 0; u < KPL; ++u) oyr[u] = RY != 0 ? oyn[u] : VT(0);
    if (s + 1 < KS) frags2(s + 1);
    __builtin_amdgcn_sched_barrier(0);
    VT zc[KPL];
    if constexpr (OWN) {
#pragma unroll
      for (int u = 0; u < KPL; ++u) zc[u] = __shfl(zp[T], MF::out_row(g, v0 + u), 64);
#pragma unroll
      for (int t = 0; t < Q; ++t)
#pragma unroll
        for (int u = 0; u < KPL; ++u) yc[t] += PV::get(a[t], u) * zc[u];
    }
    typename MF::elem be[KPL];
#pragma unroll
    for (int u = 0; u < KPL; ++u) be[u] = PV::to_elem(acc1[T][v0 + u]);
    typename MF::frag b = MF::make(be);
#pragma unroll
    for (int t = 0; t < Q; ++t) acc2[t] = MF::mma(a[t], b, acc2[t]);
    if constexpr (RY != 0) {
#pragma unroll
      for (int u = 0; u < KPL; ++u) yr += oyr[u] * PV::of(be[u]);
    }
    if constexpr (RY != 0 && OWN) {
#pragma unroll
      for (int u = 0; u < KPL; ++u) ycc += oyr[u] * zc[u];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  before_store();
#pragma unroll
  for (int t = 0; t < Q; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) store(16 * t + MF::out_row(g, v), 16 * j + c, (VT)acc2[t][v]);
  if constexpr (RY != 0) {
    const VT r = xor_sum(yr) + PV::of(opy[16 * Q * ldo + 16 * Q]) * zr;
    if (g == 0) store(16 * Q, 16 * j + c, r);
  }
  if constexpr (OWN) {
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      VT y = xor_sum(yc[t]);
      if constexpr (RY != 0) y += PV::of(opy[(16 * t + c) * ldo + 16 * Q]) * zcc;
      if (g == 0) store(16 * t + c, 16 * Q, y);
    }
    if constexpr (RY != 0) {
      ycc = xor_sum(ycc) + PV::of(opy[16 * Q * ldo + 16 * Q]) * zcc;
      if (g == 0 && c == 0) store(16 * Q, 16 * Q, ycc);
    }
  }
}

// LDS leading dimensions: quadrant columns start at 0 (even) and PS_COLO (odd,
// rounded up so that bf16 fragments stay 8-byte aligned).
template <int M, bool ODD> struct PlaneSymDims {
  static constexpr int NE = M + (ODD ? 1 : 0), N = 2 * M + (ODD ? 1 : 0);
  static constexpr int COLO = (NE + 3) / 4 * 4;
};
template <typename TC, int M, bool ODD> __host__ __device__ constexpr int plane_sym_ldp() {
  return lds_pad<TC>(PlaneSymDims<M, ODD>::COLO + M);
}
template <typename TC, int M, bool ODD> __host__ __device__ constexpr int plane_sym_ldo() {
  return lds_pad<TC>((PlaneSymDims<M, ODD>::NE + 3) / 4 * 4);
}
// LDS layout of mode_gemm_plane_sym: plane, OpY halves, OpX halves and, for
// the backward pass when the accumulator is wider than the element, an
// accumulator-precision copy of the quadrant results (16-byte aligned).
template <typename TC, int M, bool ODD> __host__ __device__ constexpr size_t plane_sym_zoff() {
  typedef PlaneSymDims<M, ODD> D;
  return ((size_t)(D::N * plane_sym_ldp<TC, M, ODD>() + 2 * D::N * plane_sym_ldo<TC, M, ODD>()) *
              sizeof(typename Mfma<TC>::elem) + 15) / 16 * 16;
}
template <typename TC, int M, bool ODD, bool FWD> __host__ __device__ constexpr size_t plane_sym_lds() {
  typedef PlaneSymDims<M, ODD> D;
  return plane_sym_zoff<TC, M, ODD>() +
         ((!FWD && sizeof(typename Mfma<TC>::acc_elem) != sizeof(typename Mfma<TC>::elem))
              ? (size_t)D::N * plane_sym_ldp<TC, M, ODD>() * sizeof(typename Mfma<TC>::acc_elem)
              : 0);
}

// FWD: out = modal planes (even modes first along both axes) of the physical
// planes in `in`; !FWD: the reverse.  Plane o starts at in + o*in_stride and
// out + o*out_stride (strides >= n*n; padding is neither read nor written).  opx*/opy*: half operators of directions
// x and y (FWD: rows of U^T; !FWD: rows of U), even (NE x NE) and odd (M x M).
// Block = 4 WQ waves: WQ per quadrant, each transforming Q / WQ of its
// 16-column strips (Q = M / 16); registers sized for two blocks per CU
// (2 WQ waves per SIMD); persistent over planes, the next plane's loads in
// flight while the current one is transformed.  WQ = Q (one strip per wave)
// in FP32 and BF16; in FP64 one wave per quadrant (a strip per wave needs more
// than the 128 registers of four waves per SIMD: measured slower, spilling).
template <typename TC, int M> __host__ __device__ constexpr int plane_sym_wq() {
  return sizeof(typename Mfma<TC>::elem) == 8 ? 1 : M / 16;
}
template <typename TC, int M> __host__ __device__ constexpr int plane_sym_threads() {
  return 64 * 4 * plane_sym_wq<TC, M>();
}
template <typename Tin, typename Tout, typename TC, int M, bool ODD, bool FWD>
__global__ void __launch_bounds__((plane_sym_threads<TC, M>()), (2 * plane_sym_wq<TC, M>()))
mode_gemm_plane_sym(const Tin *__restrict__ in, Tout *__restrict__ out,
                    const typename Mfma<TC>::elem *__restrict__ opxE,
                    const typename Mfma<TC>::elem *__restrict__ opxO,
                    const typename Mfma<TC>::elem *__restrict__ opyE,
                    const typename Mfma<TC>::elem *__restrict__ opyO, int64_t planes,
                    int64_t in_stride, int64_t out_stride) {
  typedef Mfma<TC> MF;
  typedef typename MF::elem E;
  typedef PlaneVal<TC> PV;
  typedef typename PV::vt VT;
  typedef typename MF::acc_elem AE;
  typedef PlaneSymDims<M, ODD> D;
  constexpr int NE = D::NE, N = D::N, COLO = D::COLO, Q = M / 16;
  constexpr int KSTEP = MF::KSTEP, KPL = MF::KPL, KS = 16 * Q / KSTEP;
  constexpr int LDP = plane_sym_ldp<TC, M, ODD>(), LDO = plane_sym_ldo<TC, M, ODD>();
  constexpr int NT = plane_sym_threads<TC, M>(), WQ = plane_sym_wq<TC, M>();
  constexpr int NORB = NE * NE;                  // orbits (forward loads)
  constexpr int PER = FWD ? (NORB + NT - 1) / NT : (N * N + NT - 1) / NT;
  constexpr int NLD = FWD ? 4 : 1;               // loads per item
  static_assert(M % 16 == 0, "half size must be a multiple of 16");
  extern __shared__ __align__(16) unsigned char smem[];
  E *pl = reinterpret_cast<E *>(smem);           // [N][LDP] quadrant layout
  E *oy = pl + N * LDP;                          // OpY even [NE][LDO], then odd [M][LDO]
  E *ox = oy + N * LDO;                          // OpX likewise
  AE *zb = (!FWD && sizeof(AE) != sizeof(E)) ? reinterpret_cast<AE *>(smem + plane_sym_zoff<TC, M, ODD>())
                                             : reinterpret_cast<AE *>(pl);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int quad = w / WQ, js = w % WQ;  // quadrant and strip of this wave
  const int qa = quad >> 1, qb = quad & 1;  // quadrant: y parity, x parity (0 even)

  for (int e = tid; e < NE * NE; e += NT) {
    oy[(e / NE) * LDO + e % NE] = opyE[e];
    ox[(e / NE) * LDO + e % NE] = opxE[e];
  }
  for (int e = tid; e < M * M; e += NT) {
    oy[(NE + e / M) * LDO + e % M] = opyO[e];
    ox[(NE + e / M) * LDO + e % M] = opxO[e];
  }

  // ---- plane loads: FWD orbit by orbit (four mirror points), !FWD plain
  Tin pre[PER][NLD];
  auto gload = [&](int64_t p) {
    const bool pv = p < planes;
    const Tin *src = in + (pv ? p : 0) * in_stride;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      if (FWD) {
        const bool ok = pv && e < NORB;
        const int yh = ok ? e / NE : 0, xh = ok ? e - (e / NE) * NE : 0;
        const int y2 = N - 1 - yh, x2 = N - 1 - xh;
        pre[i][0] = src[yh * N + xh];
        pre[i][NLD > 1 ? 1 : 0] = src[yh * N + x2];
        pre[i][NLD > 2 ? 2 : 0] = src[y2 * N + xh];
        pre[i][NLD > 3 ? 3 : 0] = src[y2 * N + x2];
      } else {
        pre[i][0] = src[(pv && e < N * N) ? e : 0];
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      if (FWD) {
        if (e < NORB) {
          const int yh = e / NE, xh = e - yh * NE;
          const bool xm = ODD && xh == M, ym = ODD && yh == M;  // middle column / row
          const double a = Conv<Tin>::to_f64(pre[i][0]), b = Conv<Tin>::to_f64(pre[i][NLD > 1 ? 1 : 0]);
          const double cc = Conv<Tin>::to_f64(pre[i][NLD > 2 ? 2 : 0]);
          const double d = Conv<Tin>::to_f64(pre[i][NLD > 3 ? 3 : 0]);
          const double e1 = xm ? a : a + b, o1 = a - b;   // row yh
          const double e2 = xm ? cc : cc + d, o2 = cc - d;  // row N-1-yh
          pl[yh * LDP + xh] = MF::from_f64(ym ? e1 : e1 + e2);
          if (!xm) pl[yh * LDP + COLO + xh] = MF::from_f64(ym ? o1 : o1 + o2);
          if (!ym) pl[(NE + yh) * LDP + xh] = MF::from_f64(e1 - e2);
          if (!xm && !ym) pl[(NE + yh) * LDP + COLO + xh] = MF::from_f64(o1 - o2);
        }
      } else if (e < N * N) {
        const int ky = e / N, kx = e - ky * N;
        pl[ky * LDP + (kx < NE ? kx : COLO + kx - NE)] = MF::from_f64(Conv<Tin>::to_f64(pre[i][0]));
      }
    }
  };

  int64_t p = blockIdx.x;
  gload(p);
  __syncthreads();  // operators in LDS
  lstore();
  __syncthreads();
  for (; p < planes; p += gridDim.x) {
    gload(p + gridDim.x);
    const E *inq = pl + (qa ? NE : 0) * LDP + (qb ? COLO : 0);
    const E *opyq = oy + (qa ? NE : 0) * LDO, *opxq = ox + (qb ? NE : 0) * LDO;
    Tout *dst = out + p * out_stride;
    const int r0 = qa ? NE : 0, c0 = qb ? NE : 0, cl0 = qb ? COLO : 0;
    auto store = [&](int row, int col, VT v) {
      if (FWD) dst[(r0 + row) * N + c0 + col] = Conv<Tout>::from_f64((double)v);
      else zb[(r0 + row) * LDP + cl0 + col] = (AE)v;
    };
    if constexpr (WQ == 1) {
      // wave-uniform: each wave transforms its own quadrant, which it alone
      // reads and (backward) overwrites
      constexpr int F = ODD ? 1 : 0;
      switch (quad) {
        case 0: quad_transform<TC, Q, F, F>(inq, LDP, opxq, opyq, LDO, c, g, store); break;
        case 1: quad_transform<TC, Q, F, 0>(inq, LDP, opxq, opyq, LDO, c, g, store); break;
        case 2: quad_transform<TC, Q, 0, F>(inq, LDP, opxq, opyq, LDO, c, g, store); break;
        default: quad_transform<TC, Q, 0, 0>(inq, LDP, opxq, opyq, LDO, c, g, store); break;
      }
    } else {
      // the backward results overwrite the plane in LDS when they have its
      // type: every strip of the quadrant has to be done reading it first
      auto before_store = [&]() {
        if constexpr (!FWD)
          if ((void *)zb == (void *)pl) __syncthreads();
      };
      // wave-uniform: the quadrant's fringe sizes, and the fringe column for strip 0
      constexpr int F = ODD ? 1 : 0;
      switch (quad * 2 + (js == 0 ? 1 : 0)) {
        case 1: quad_strip<TC, Q, F, F, ODD>(inq, LDP, opxq, opyq, LDO, c, g, js, store, before_store); break;
        case 0: quad_strip<TC, Q, F, F, false>(inq, LDP, opxq, opyq, LDO, c, g, js, store, before_store); break;
        case 2:
        case 3: quad_strip<TC, Q, F, 0, false>(inq, LDP, opxq, opyq, LDO, c, g, js, store, before_store); break;
        case 5: quad_strip<TC, Q, 0, F, ODD>(inq, LDP, opxq, opyq, LDO, c, g, js, store, before_store); break;
        case 4: quad_strip<TC, Q, 0, F, false>(inq, LDP, opxq, opyq, LDO, c, g, js, store, before_store); break;
        default: quad_strip<TC, Q, 0, 0, false>(inq, LDP, opxq, opyq, LDO, c, g, js, store, before_store); break;
      }
    }
    __syncthreads();  // every quadrant done
    if (!FWD) {
      // X at the four mirror points of each half coordinate, two half
      // coordinates per trip, branch-free: the LDS reads past the middle row /
      // column stay inside the allocation and are replaced by zeros, and on the
      // middle row / column the mirror point is the point itself, so its
      // second store writes the same value again
      constexpr int PB = (NORB + NT - 1) / NT;
#pragma unroll 1
      for (int i0 = 0; i0 < PB; i0 += 2)
#pragma unroll
      for (int i = i0; i < i0 + 2; ++i) {
        const int e = tid + i * NT;
        if (i < PB && e < NORB) {
          const int yh = e / NE, xh = e - yh * NE;
          const bool xm = ODD && xh == M, ym = ODD && yh == M;
          const double zee = (double)zb[yh * LDP + xh];
          double zeo = (double)zb[yh * LDP + COLO + xh];
          double zoe = (double)zb[(NE + yh) * LDP + xh];
          double zoo = (double)zb[(NE + yh) * LDP + COLO + xh];
          if (xm) zeo = 0.0;
          if (ym) zoe = 0.0;
          if (xm || ym) zoo = 0.0;
          const int y2 = N - 1 - yh, x2 = N - 1 - xh;
          dst[yh * N + xh] = Conv<Tout>::from_f64((zee + zoe) + (zeo + zoo));
          dst[yh * N + x2] = Conv<Tout>::from_f64((zee + zoe) - (zeo + zoo));
          dst[y2 * N + xh] = Conv<Tout>::from_f64((zee - zoe) + (zeo - zoo));
          dst[y2 * N + x2] = Conv<Tout>::from_f64((zee - zoe) - (zeo - zoo));
        }
      }
      if ((void *)zb == (void *)pl) __syncthreads();  // the results alias the plane
    }
    lstore();         // next plane into LDS (waits for its loads)
    __syncthreads();  // ... visible to every wave
  }
}

}  // namespace stig

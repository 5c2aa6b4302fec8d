// Step 3 of Algorithm 1 in the paper's own form: the time pencil diagonalized
// by the real block form of its arrowhead factorization (Section 4.2.2,
// eq. time_eig_2), the middle factor solved by block LU (eq. block_LU).
//
// With U^T M_t U = I and D = U^T W_t U = [[B, g], [h^T, sigma]], B block
// diagonal (a zero 1 x 1 block and 2 x 2 blocks [[0, d], [-d, 0]]),
// (gamma W_t + nu lambda M_t)^{-1} r = U (gamma D + nu lambda I)^{-1} U^T r.
// One kernel does, for 16 spatial indices k per wave and step:
//   x~ = U^T r            (MFMA, along t)
//   per k: block LU of the arrowhead: each 2 x 2 block H = gamma [[0,d],[-d,0]]
//   + nu lambda_k I is inverted in closed form, the Schur complement
//   s = gamma sigma + nu lambda - sum gamma^2 h^T H^{-1} g is a sum over the
//   blocks (in-lane, then across the four k-slices), q_n = (x~_n - sum gamma
//   h^T H^{-1} x~) / s, q_block = H^{-1} (x~ - gamma g q_n)
//   y = U q               (MFMA, B operand straight from the accumulators)
// Time modes are stored so that both members of a 2 x 2 block sit in one lane:
// rows r and r + 16 of the 32-row group r / 32; the zero mode is row 32 Q,
// the last (arrow) mode row 32 Q + 1, n_t = 32 Q + 2.
#pragma once

#include "kernels_fd.h"
#include "kernels_plane.h"

namespace stig {

constexpr int ARROW_THREADS = 256;

// tf: U^T in mode order (n_t x n_t row-major, rows = modes), tb: U (rows = t,
// columns = modes); dd[r] = d of the block of mode r, gv[r] / hv[r] = arrow
// column / row entry of mode r (r < n_t - 1), sigma = corner.  Layout of in /
// out: [rhs][t][ns], one system per spatial index k < ns.
template <typename Tio, typename TC, int Q>
__global__ void __launch_bounds__(ARROW_THREADS, 2)
time_arrow_solve(const Tio *__restrict__ in, Tio *__restrict__ out,
                 const double *__restrict__ lam, const typename Mfma<TC>::elem *__restrict__ tf,
                 const typename Mfma<TC>::elem *__restrict__ tb,
                 const typename PlaneVal<TC>::vt *__restrict__ tabs, typename PlaneVal<TC>::vt gamma,
                 typename PlaneVal<TC>::vt nu, int64_t ns, int64_t total_cols) {
  typedef Mfma<TC> MF;
  typedef typename MF::elem E;
  typedef PlaneVal<TC> PV;
  typedef typename PV::vt VT;
  constexpr int NT = 32 * Q + 2, NM = 32 * Q;  // systems' size, modes in 2 x 2 blocks
  constexpr int TILES = 2 * Q, KPL = MF::KPL, KSTEP = MF::KSTEP, KS = NM / KSTEP;
  constexpr int SPT = 16 / KSTEP;
  extern __shared__ __align__(16) unsigned char smem[];
  const int ld = lds_pad<TC>(NT);
  E *lf = reinterpret_cast<E *>(smem);  // U^T [NT][ld]
  E *lb = lf + NT * ld;                 // U   [NT][ld]
  VT *ltab = reinterpret_cast<VT *>(smem + (((size_t)2 * NT * ld * sizeof(E) + 15) / 16 * 16));
  VT *ldd = ltab, *lgv = ltab + NT, *lhv = ltab + 2 * NT;  // [NT] each
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < NT * NT; e += ARROW_THREADS) {
    const int i = e / NT, j = e - i * NT;
    lf[i * ld + j] = tf[e];
    lb[i * ld + j] = tb[e];
  }
  for (int e = tid; e < 3 * NT + 1; e += ARROW_THREADS) ltab[e] = tabs[e];
  __syncthreads();
  const VT sigma = ltab[3 * NT];

  const int col = lane & 15, g = lane >> 4;
  const int64_t nstrips = (total_cols + 15) >> 4;
  const int64_t wstride = (int64_t)gridDim.x * (ARROW_THREADS / 64);
  auto xor_sum = [](VT x) {
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
  };
  struct Frags {
    E b[KS][KPL];
    VT f0, f1;  // rows NM, NM + 1 of the strip's column (every lane)
  };
  auto base_of = [&](int64_t c) {
    const int64_t rhs = c / ns, k = c - rhs * ns;
    return rhs * ns * NT + k;
  };
  auto load = [&](int64_t strip, Frags &f) {
    const int64_t c = strip * 16 + col;
    const bool ok = strip < nstrips && c < total_cols;
    const int64_t base = base_of(ok ? c : 0);
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int u = 0; u < KPL; ++u) {
        const int t = s * KSTEP + g * KPL + u;
        f.b[s][u] = MF::from_f64(Conv<Tio>::to_f64(in[base + (int64_t)t * ns]));
      }
    f.f0 = PV::of(MF::from_f64(Conv<Tio>::to_f64(in[base + (int64_t)NM * ns])));
    f.f1 = PV::of(MF::from_f64(Conv<Tio>::to_f64(in[base + (int64_t)(NM + 1) * ns])));
  };
  // one strip; the next strip's loads go out once this strip's operands are
  // consumed (after the first product), so the two never share registers
  auto process = [&](int64_t strip, const Frags &f, Frags &fnext, int64_t next) {
    const int64_t c = strip * 16 + col;
    const bool cvalid = c < total_cols;
    const int64_t base = base_of(cvalid ? c : 0);
    const int64_t k = cvalid ? c % ns : 0;
    const VT nul = nu * (VT)lam[k];
    // ---- x~ = U^T r: tiles of modes 0..NM-1 on MFMA, modes NM, NM+1 on the ALU
    typename MF::acc acc[TILES];
#pragma unroll
    for (int T = 0; T < TILES; ++T)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * T + MF::out_row(g, v);
        acc[T][v] = PV::of(lf[r * ld + NM]) * f.f0 + PV::of(lf[r * ld + NM + 1]) * f.f1;
      }
    VT xz = 0, xa = 0;  // zero mode, arrow mode (partial over this lane's k-slice)
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      typename MF::frag b = MF::make(f.b[s]);
#pragma unroll
      for (int T = 0; T < TILES; ++T)
        acc[T] = MF::mma(MF::load(lf + (16 * T + col) * ld + s * KSTEP + g * KPL), b, acc[T]);
#pragma unroll
      for (int u = 0; u < KPL; ++u) {
        const int t = s * KSTEP + g * KPL + u;
        xz += PV::of(lf[NM * ld + t]) * PV::of(f.b[s][u]);
        xa += PV::of(lf[(NM + 1) * ld + t]) * PV::of(f.b[s][u]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    xz = xor_sum(xz) + PV::of(lf[NM * ld + NM]) * f.f0 + PV::of(lf[NM * ld + NM + 1]) * f.f1;
    xa = xor_sum(xa) + PV::of(lf[(NM + 1) * ld + NM]) * f.f0 + PV::of(lf[(NM + 1) * ld + NM + 1]) * f.f1;
    load(next, fnext);
    // ---- block LU of gamma D + nu lambda I (reciprocals: hardware estimate
    // refined by Newton steps, as for the banded pivots)
    VT sp = 0, yp = 0;
    VT tg[TILES / 2][4][2];  // H^{-1} g of each block, kept for the back substitution
#pragma unroll
    for (int T = 0; T < TILES; T += 2)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r1 = 16 * T + MF::out_row(g, v), r2 = r1 + 16;
        const VT gd = gamma * ldd[r1], inv = recip(nul * nul + gd * gd);
        const VT x1 = (VT)acc[T][v], x2 = (VT)acc[T + 1][v];
        const VT g1 = lgv[r1], g2 = lgv[r2], h1 = lhv[r1], h2 = lhv[r2];
        const VT u1 = (nul * x1 - gd * x2) * inv, u2 = (gd * x1 + nul * x2) * inv;  // H^{-1} x
        const VT t1 = (nul * g1 - gd * g2) * inv, t2 = (gd * g1 + nul * g2) * inv;  // H^{-1} g
        sp += h1 * t1 + h2 * t2;
        yp += h1 * u1 + h2 * u2;
        acc[T][v] = u1;
        acc[T + 1][v] = u2;
        tg[T / 2][v][0] = t1;
        tg[T / 2][v][1] = t2;
      }
    sp = xor_sum(sp);
    yp = xor_sum(yp);
    const VT gz = lgv[NM], hz = lhv[NM], rnul = recip(nul);
    const VT sch = gamma * sigma + nul - gamma * gamma * (sp + hz * gz * rnul);
    const VT qn = (xa - gamma * (yp + hz * xz * rnul)) * recip(sch);
    const VT qz = (xz - gamma * gz * qn) * rnul;
#pragma unroll
    for (int T = 0; T < TILES; T += 2)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[T][v] = (VT)acc[T][v] - gamma * qn * tg[T / 2][v][0];
        acc[T + 1][v] = (VT)acc[T + 1][v] - gamma * qn * tg[T / 2][v][1];
      }
    // ---- y = U q: B operand from the accumulators (contraction over modes in
    // the order the lanes hold them), modes NM, NM+1 as a rank-two start
    typename MF::acc acc2[TILES];
#pragma unroll
    for (int t = 0; t < TILES; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + MF::out_row(g, v);
        acc2[t][v] = PV::of(lb[row * ld + NM]) * qz + PV::of(lb[row * ld + NM + 1]) * qn;
      }
    VT y0 = 0, y1 = 0;  // output rows NM, NM+1
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int T = s / SPT, v0 = (s % SPT) * KPL;
      E be[KPL];
#pragma unroll
      for (int u = 0; u < KPL; ++u) be[u] = PV::to_elem((VT)acc[T][v0 + u]);
      typename MF::frag b = MF::make(be);
      const int kcol = 16 * T + MF::out_row(g, v0);
#pragma unroll
      for (int t = 0; t < TILES; ++t)
        acc2[t] = MF::mma(MF::load(lb + (16 * t + col) * ld + kcol), b, acc2[t]);
#pragma unroll
      for (int u = 0; u < KPL; ++u) {
        y0 += PV::of(lb[NM * ld + kcol + u]) * PV::of(be[u]);
        y1 += PV::of(lb[(NM + 1) * ld + kcol + u]) * PV::of(be[u]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    y0 = xor_sum(y0) + PV::of(lb[NM * ld + NM]) * qz + PV::of(lb[NM * ld + NM + 1]) * qn;
    y1 = xor_sum(y1) + PV::of(lb[(NM + 1) * ld + NM]) * qz + PV::of(lb[(NM + 1) * ld + NM + 1]) * qn;
    if (cvalid) {
#pragma unroll
      for (int t = 0; t < TILES; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + MF::out_row(g, v);
          out[base + (int64_t)row * ns] = Conv<Tio>::from_f64((double)acc2[t][v]);
        }
      if (g == 0) {
        out[base + (int64_t)NM * ns] = Conv<Tio>::from_f64((double)y0);
        out[base + (int64_t)(NM + 1) * ns] = Conv<Tio>::from_f64((double)y1);
      }
    }
  };
  int64_t strip = (int64_t)blockIdx.x * (ARROW_THREADS / 64) + wave;
  Frags fnext;
  load(strip, fnext);
  for (; strip < nstrips; strip += wstride) {
    Frags f = fnext;
    process(strip, f, fnext, strip + wstride);
  }
}

// ---------------------------------------------- any n_t: the middle factor
// Step 3 in the arrowhead form for any n_t, as three passes: x~ = U^T r along t
// (a mode product on MFMA), this kernel, then y = U q along t.  (Fusing this
// step into the second product's operand load was measured slower in every
// precision: it leaves one wave per SIMD.)  Mode order: the 2 x 2 blocks
// (2j, 2j + 1) first, then the zero mode (position n - 2) when the skew part
// has odd size (nz = 1), the arrow mode n - 1 last.  For each system k (column c = rhs * ns + k of x,
// layout [rhs][mode][ns]) the arrowhead middle factor gamma D + nu lam_k I
// (eq. block_LU) is solved in place: q_B = H^{-1} (x_B - gamma g q_n),
// q_n = (x_n - gamma h^T H^{-1} x_B) / (gamma sigma + nu lam_k
//       - gamma^2 h^T H^{-1} g),
// H = gamma B + nu lam_k I block diagonal with closed-form 2 x 2 inverses.
// tab: d of each mode's block (at both positions of the block), g[n], h[n]
// (arrow column / row), sigma, i.e. [d | g | h | sigma].
// L lanes per system: a wave covers CW = 64 / L consecutive columns, lane
// c + CW l (l < L) takes column c and every L-th block, and the two sums are
// reduced across the L lanes of a column.  Two passes over the modes (the
// second re-reads x, from L2), so nothing is held per mode.
template <typename TC, int L>
__global__ void __launch_bounds__(256)
time_arrow_middle(TC *__restrict__ x, const double *__restrict__ lam, const TC *__restrict__ tab,
                  TC gamma, TC nu, int n, int nz, int64_t ns, int64_t cols) {
  static_assert(L == 1 || L == 2 || L == 4 || L == 8 || L == 16, "lanes per system");
  constexpr int CW = 64 / L;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int grp = lane / CW;
  const int64_t c = wave * CW + (lane % CW);
  const bool valid = c < cols;
  const int64_t cc = valid ? c : 0;
  const int64_t rhs = cc / ns, k = cc - rhs * ns;
  TC *xc = x + rhs * ns * n + k;
  const TC nul = nu * (TC)lam[k];
  const int nb = (n - 1 - nz) / 2;  // 2 x 2 blocks
  const TC *dd = tab, *gv = tab + n, *hv = tab + 2 * n;
  auto lsum = [](TC v) {
#pragma unroll
    for (int off = CW; off < 64; off *= 2) v += __shfl_xor(v, off, 64);
    return v;
  };
  // pass 1: sums h^T H^{-1} g and h^T H^{-1} x (unrolled: the loads of several
  // blocks in flight)
  TC sp = 0, yp = 0;
#pragma unroll 8
  for (int j = grp; j < nb; j += L) {
    const int a = 2 * j;
    const TC x1 = xc[(int64_t)a * ns], x2 = xc[(int64_t)(a + 1) * ns];
    const TC gd = gamma * dd[a], inv = recip(nul * nul + gd * gd);
    const TC g1 = gv[a], g2 = gv[a + 1], h1 = hv[a], h2 = hv[a + 1];
    sp += (h1 * (nul * g1 - gd * g2) + h2 * (gd * g1 + nul * g2)) * inv;
    yp += (h1 * (nul * x1 - gd * x2) + h2 * (gd * x1 + nul * x2)) * inv;
  }
  sp = lsum(sp);
  yp = lsum(yp);
  const TC rnul = recip(nul);
  TC xz = 0;
  if (nz) {
    xz = xc[(int64_t)(n - 2) * ns];
    sp += hv[n - 2] * gv[n - 2] * rnul;
    yp += hv[n - 2] * xz * rnul;
  }
  const TC xn = xc[(int64_t)(n - 1) * ns];
  const TC sch = gamma * tab[3 * n] + nul - gamma * gamma * sp;
  const TC qn = (xn - gamma * yp) * recip(sch);
  // pass 2: q_B = H^{-1} (x_B - gamma g q_n)
#pragma unroll 8
  for (int j = grp; j < nb; j += L) {
    const int a = 2 * j;
    const TC g1 = gv[a], g2 = gv[a + 1];
    const TC x1 = xc[(int64_t)a * ns] - gamma * g1 * qn, x2 = xc[(int64_t)(a + 1) * ns] - gamma * g2 * qn;
    const TC gd = gamma * dd[a], inv = recip(nul * nul + gd * gd);
    if (valid) {
      xc[(int64_t)a * ns] = (nul * x1 - gd * x2) * inv;
      xc[(int64_t)(a + 1) * ns] = (gd * x1 + nul * x2) * inv;
    }
  }
  if (valid && grp == 0) {
    if (nz) xc[(int64_t)(n - 2) * ns] = (xz - gamma * gv[n - 2] * qn) * rnul;
    xc[(int64_t)(n - 1) * ns] = qn;
  }
}

// The same solve with each block taking CB = 256 / G consecutive columns and
// G threads per column (thread tid: column tid % CB, group tid / CB, blocks
// j = group + G i).  A half-wave (FP64, CB = 32) or a wave (FP32, CB = 64)
// then reads and writes whole 256-byte runs of a mode row, and a thread keeps
// its JM >= ceil(nb / G) blocks and their reciprocals in registers between the
// two passes, so x is read once (nb >= 1; JM is the smallest of the compiled
// counts that covers nb, so few iterations run idle).  The table goes to LDS first (its loads in
// flight with those of x; read from global memory inside the loops, each
// step's table loads took a round trip of their own).  The group sums are
// reduced through LDS in a fixed order, and the two modes after the blocks come
// from group 0 through LDS too (no thread reads a row that another writes).
template <typename TC, int G, int JM>
__global__ void __launch_bounds__(256)
time_arrow_middle_reg(TC *__restrict__ x, const double *__restrict__ lam,
                      const TC *__restrict__ tab, TC gamma, TC nu, int n, int nz, int64_t ns,
                      int64_t cols) {
  constexpr int CB = 256 / G;
  constexpr int NT = 3 * (2 * G * JM + 2) + 1;  // table entries at the largest n
  static_assert(CB * G == 256 && CB % 32 == 0, "columns per block");
  __shared__ TC red[2][G][CB];
  __shared__ TC last[2][CB];
  __shared__ TC tl[NT];
  const int tid = threadIdx.x, cl = tid % CB, grp = tid / CB;
  const int64_t c = (int64_t)blockIdx.x * CB + cl;
  const bool valid = c < cols;
  const int64_t cc = valid ? c : 0;
  const int64_t rhs = cc / ns, k = cc - rhs * ns;
  TC *xc = x + rhs * ns * n + k;
  const int nb = (n - 1 - nz) / 2, ntab = 3 * n + 1;
  TC tv[(NT + 255) / 256];
#pragma unroll
  for (int u = 0; u < (NT + 255) / 256; ++u) {
    const int e = tid + 256 * u;
    tv[u] = tab[e < ntab ? e : 0];
  }
  TC xr[JM][2], ir[JM];
#pragma unroll
  for (int i = 0; i < JM; ++i) {
    const int j = grp + G * i, a = j < nb ? 2 * j : 0;  // nb >= 1: rows 0, 1 exist
    xr[i][0] = xc[(int64_t)a * ns];
    xr[i][1] = xc[(int64_t)(a + 1) * ns];
    ir[i] = 0;
  }
  TC xz = 0, xn = 0;
  if (grp == 0) {
    if (nz) xz = xc[(int64_t)(n - 2) * ns];
    xn = xc[(int64_t)(n - 1) * ns];
  }
  const TC nul = nu * (TC)lam[k];
#pragma unroll
  for (int u = 0; u < (NT + 255) / 256; ++u) {
    const int e = tid + 256 * u;
    if (e < ntab) tl[e] = tv[u];
  }
  __syncthreads();
  const TC *dd = tl, *gv = tl + n, *hv = tl + 2 * n;
  // pass 1: this group's share of h^T H^{-1} g and h^T H^{-1} x
  TC sp = 0, yp = 0;
#pragma unroll
  for (int i = 0; i < JM; ++i) {
    const int j = grp + G * i;
    const bool ok = j < nb;
    const int a = ok ? 2 * j : 0;
    const TC gd = gamma * dd[a], inv = recip(nul * nul + gd * gd);
    const TC g1 = gv[a], g2 = gv[a + 1], h1 = hv[a], h2 = hv[a + 1];
    const TC x1 = xr[i][0], x2 = xr[i][1];
    const TC s1 = (h1 * (nul * g1 - gd * g2) + h2 * (gd * g1 + nul * g2)) * inv;
    const TC y1 = (h1 * (nul * x1 - gd * x2) + h2 * (gd * x1 + nul * x2)) * inv;
    sp += ok ? s1 : (TC)0;
    yp += ok ? y1 : (TC)0;
    ir[i] = inv;
  }
  red[0][grp][cl] = sp;
  red[1][grp][cl] = yp;
  if (grp == 0) {
    last[0][cl] = xz;
    last[1][cl] = xn;
  }
  __syncthreads();
  sp = 0;
  yp = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    sp += red[0][g][cl];
    yp += red[1][g][cl];
  }
  xz = last[0][cl];
  xn = last[1][cl];
  const TC rnul = recip(nul);
  if (nz) {
    sp += hv[n - 2] * gv[n - 2] * rnul;
    yp += hv[n - 2] * xz * rnul;
  }
  const TC sch = gamma * tl[3 * n] + nul - gamma * gamma * sp;
  const TC qn = (xn - gamma * yp) * recip(sch);
  // pass 2: q_B = H^{-1} (x_B - gamma g q_n) from the registers
  if (!valid) return;
#pragma unroll
  for (int i = 0; i < JM; ++i) {
    const int j = grp + G * i;
    const bool ok = j < nb;
    const int a = ok ? 2 * j : 0;
    const TC gd = gamma * dd[a], inv = ir[i];
    const TC x1 = xr[i][0] - gamma * gv[a] * qn, x2 = xr[i][1] - gamma * gv[a + 1] * qn;
    if (ok) {
      xc[(int64_t)a * ns] = (nul * x1 - gd * x2) * inv;
      xc[(int64_t)(a + 1) * ns] = (gd * x1 + nul * x2) * inv;
    }
  }
  if (grp == 0) {
    if (nz) xc[(int64_t)(n - 2) * ns] = (xz - gamma * gv[n - 2] * qn) * rnul;
    xc[(int64_t)(n - 1) * ns] = qn;
  }
}

}  // namespace stig

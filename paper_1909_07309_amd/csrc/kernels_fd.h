// Device kernels of the fast-diagonalization apply (steps 2-4 of Algorithm 1,
// Section 4.4, with the time pencil kept banded).
//
//  * mode_gemm: one mode-k product Y = X x_k Op (Section 2.3) of the unknown
//    tensor with a small dense square matrix (U_l or U_l^T), on MFMA.
//  * time_band_solve: one banded shifted system (gamma W_t + nu lambda_k M_t)
//    per spatial eigen-index k, Gaussian elimination without pivoting.
//
// The tensor is viewed as [outer][n][inner] around the contracted axis: a
// "column" c in [0, outer*inner) is the pencil (o, i) = (c / inner, c % inner)
// whose n entries sit at o*n*inner + k*inner + i.  A mode product is then the
// GEMM Y[:, c] = Op * X[:, c] over all columns.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stig {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

// bf16 stored as its 16 raw bits.
struct bf16 {
  uint16_t bits;
};

// Round to nearest even; NaN stays NaN (quiet bit forced), +-Inf stays Inf.
// Branch-free so that conversions do not split the surrounding load batches.
__device__ __host__ inline uint16_t float_to_bf16_bits(float f) {
  union { float f; uint32_t u; } v;
  v.f = f;
  uint32_t u = v.u;
  uint32_t rounded = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  uint32_t special = (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
  bool nonfinite = (u & 0x7f800000u) == 0x7f800000u;
  return (uint16_t)(nonfinite ? special : rounded);
}
__device__ __host__ inline float bf16_bits_to_float(uint16_t b) {
  union { float f; uint32_t u; } v;
  v.u = ((uint32_t)b) << 16;
  return v.f;
}

// Conversions between storage types and compute types.
template <typename T> struct Conv;
template <> struct Conv<double> {
  __device__ static inline double to_f64(double x) { return x; }
  __device__ static inline float to_f32(double x) { return (float)x; }
  __device__ static inline double from_f64(double x) { return x; }
  __device__ static inline double from_f32(float x) { return (double)x; }
};
template <> struct Conv<float> {
  __device__ static inline double to_f64(float x) { return (double)x; }
  __device__ static inline float to_f32(float x) { return x; }
  __device__ static inline float from_f64(double x) { return (float)x; }
  __device__ static inline float from_f32(float x) { return x; }
};
template <> struct Conv<bf16> {
  __device__ static inline double to_f64(bf16 x) { return (double)bf16_bits_to_float(x.bits); }
  __device__ static inline float to_f32(bf16 x) { return bf16_bits_to_float(x.bits); }
  __device__ static inline bf16 from_f64(double x) { return bf16{float_to_bf16_bits((float)x)}; }
  __device__ static inline bf16 from_f32(float x) { return bf16{float_to_bf16_bits(x)}; }
};

// ------------------------------------------------------------- MFMA traits
// Each trait describes one 16x16 output tile instruction D = A(16xK) B(Kx16) + D.
// Lane l of a wave holds A rows (l % 16), B columns (l % 16), and the k-slice
// (l / 16) * KPL .. + KPL-1 of the current K step.  Accumulator value v of lane l
// is D[out_row(l / 16, v)][l % 16]: rows 4*(l/16) + v for the FP32-accumulating
// instructions, rows (l/16) + 4*v for the FP64 one (checked on gfx950 by a
// lane-layout probe of the builtins).
template <typename TC> struct Mfma;

template <> struct Mfma<double> {
  static constexpr int KSTEP = 4, KPL = 1;
  typedef double elem;   // LDS element
  typedef double frag;   // per-lane operand
  typedef v4d acc;
  typedef double acc_elem;
  __device__ static inline frag load(const elem *p) { return *p; }
  __device__ static inline acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int g, int v) { return g + 4 * v; }
  __device__ static inline frag make(const elem *v) { return v[0]; }
  __device__ static inline double to_f64(elem x) { return x; }
  __device__ static inline elem from_f64(double x) { return x; }
  __device__ static inline elem zero() { return 0.0; }
};

template <> struct Mfma<float> {
  static constexpr int KSTEP = 4, KPL = 1;
  typedef float elem;
  typedef float frag;
  typedef v4f acc;
  typedef float acc_elem;
  __device__ static inline frag load(const elem *p) { return *p; }
  __device__ static inline acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int g, int v) { return 4 * g + v; }
  __device__ static inline frag make(const elem *v) { return v[0]; }
  __device__ static inline double to_f64(elem x) { return (double)x; }
  __device__ static inline elem from_f64(double x) { return (float)x; }
  __device__ static inline elem zero() { return 0.0f; }
};

template <> struct Mfma<bf16> {
  static constexpr int KSTEP = 16, KPL = 4;
  typedef uint16_t elem;
  typedef v4s frag;
  typedef v4f acc;
  typedef float acc_elem;
  __device__ static inline frag load(const elem *p) {
    return *reinterpret_cast<const v4s *>(p);  // 8-byte aligned by construction
  }
  __device__ static inline acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int g, int v) { return 4 * g + v; }
  __device__ static inline frag make(const elem *v) {
    frag r;
    r[0] = (short)v[0];
    r[1] = (short)v[1];
    r[2] = (short)v[2];
    r[3] = (short)v[3];
    return r;
  }
  __device__ static inline double to_f64(elem x) { return (double)bf16_bits_to_float(x); }
  __device__ static inline elem from_f64(double x) { return float_to_bf16_bits((float)x); }
  __device__ static inline elem zero() { return 0; }
};

__host__ __device__ constexpr inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

// Read-only coefficient tables (band rows, shifts) are read through the constant
// address space: uniform indices then compile to scalar loads instead of vector
// loads that the kernel would have to wait on row by row.
template <typename T> using cptr = const __attribute__((address_space(4))) T *;
template <typename T> __device__ inline cptr<T> as_const(const T *p) { return (cptr<T>)p; }

// LDS row stride (in elements) of at least mn elements for MFMA operand tiles.
// A wave reads rows c = lane % 16 at k-slice g = lane / 16, i.e. elements
// c * ld + g * KPL.  Measured on gfx950 (bank-conflict counter), such reads
// are conflict-free when the stride is 2 x odd elements for 8-byte (FP64) and
// 4-byte (FP32) reads, and 8 x odd elements for the 8-byte reads of four BF16
// values (which also keeps BF16 fragments 8-byte aligned).
template <typename TC> __host__ __device__ constexpr int lds_pad(int mn) {
  constexpr int q = sizeof(typename Mfma<TC>::elem) == 2 ? 8 : 2;
  int k = (mn + q - 1) / q;
  if (k % 2 == 0) ++k;
  return k * q;
}

// Leading dimension of an LDS tile holding k = 0 .. kpad-1 per column.
template <typename TC> __host__ __device__ inline int lds_ld(int n) {
  return lds_pad<TC>(round_up(n, Mfma<TC>::KSTEP));
}

constexpr int GEMM_TILE_COLS = 64;

// Y[:, c] = Op * X[:, c] for all columns c (see header comment).
// Op: n x n row-major in compute precision (device).
// Block = JB waves (JB = blockDim.x / 64); blockIdx.y selects the group of JB
// 16-row output tiles, wave w owns output rows 16*(JB*blockIdx.y + w) .. +15.
// Dynamic LDS: (GEMM_TILE_COLS + 16*JB) * ld elements.
// in_scale / out_scale: optional per-entry factors (length nscale, index taken
// modulo nscale) multiplied in on load / on store.
template <typename Tin, typename Tout, typename TC>
__global__ void mode_gemm(const Tin *__restrict__ in, Tout *__restrict__ out,
                          const typename Mfma<TC>::elem *__restrict__ Op, int n, int64_t inner,
                          int64_t total_cols, const double *__restrict__ in_scale,
                          const double *__restrict__ out_scale, int64_t nscale) {
  typedef Mfma<TC> MF;
  typedef typename MF::elem E;
  extern __shared__ __align__(16) unsigned char smem[];
  const int ld = lds_ld<TC>(n);
  const int kpad = round_up(n, MF::KSTEP);
  const int JB = blockDim.x >> 6;
  const int row0 = blockIdx.y * JB * 16;                 // first output row of this block
  E *opl = reinterpret_cast<E *>(smem);                  // [16*JB][ld]
  E *tile = opl + (size_t)16 * JB * ld;                  // [GEMM_TILE_COLS][ld]
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6;

  // rows row0 .. row0+16*JB-1 of Op -> LDS once per block, zero padded.
  for (int e = tid; e < 16 * JB * kpad; e += nthr) {
    int jl = e / kpad, k = e - jl * kpad, j = row0 + jl;
    opl[(size_t)jl * ld + k] = (j < n && k < n) ? Op[(size_t)j * n + k] : MF::zero();
  }

  const int64_t ntiles = (total_cols + GEMM_TILE_COLS - 1) / GEMM_TILE_COLS;
  const int64_t slab = (int64_t)n * inner;
  const uint32_t uinner = (uint32_t)inner;  // host guarantees total_cols < 2^31
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t c0 = t * GEMM_TILE_COLS;
    __syncthreads();  // previous tile fully consumed; Op visible
    // ---- load the X tile (converted) into tile[col][k]
    if (inner == 1) {
      // the tile's columns are contiguous rows of length n in memory
      for (int e = tid; e < GEMM_TILE_COLS * kpad; e += nthr) {
        int col = e / kpad, k = e - col * kpad;
        int64_t c = c0 + col;
        bool ok = c < total_cols && k < n;
        int64_t a = ok ? c * n + k : 0;
        double x = Conv<Tin>::to_f64(in[a]);
        if (in_scale) x *= in_scale[a % nscale];
        tile[(size_t)col * ld + k] = ok ? MF::from_f64(x) : MF::zero();
      }
    } else {
      // nthr is a multiple of 64, so each thread always touches the same column
      const int col = tid & (GEMM_TILE_COLS - 1);
      const int64_t c = c0 + col;
      const bool valid = c < total_cols;
      int64_t base = 0;
      if (valid) {
        uint32_t o = (uint32_t)c / uinner, i = (uint32_t)c - o * uinner;
        base = (int64_t)o * slab + i;
      }
      for (int k = tid / GEMM_TILE_COLS; k < kpad; k += nthr / GEMM_TILE_COLS) {
        bool ok = valid && k < n;
        int64_t a = ok ? base + (int64_t)k * inner : 0;
        double x = Conv<Tin>::to_f64(in[a]);
        if (in_scale) x *= in_scale[a % nscale];
        tile[(size_t)col * ld + k] = ok ? MF::from_f64(x) : MF::zero();
      }
    }
    __syncthreads();
    // ---- MFMA: wave owns output rows row0+16*wave .. +15, all tile columns
    typename MF::acc acc[GEMM_TILE_COLS / 16];
#pragma unroll
    for (int ct = 0; ct < GEMM_TILE_COLS / 16; ++ct)
      for (int v = 0; v < 4; ++v) acc[ct][v] = 0;
    const E *arow = opl + (size_t)(wave * 16 + (lane & 15)) * ld + (lane >> 4) * MF::KPL;
    const E *bcol = tile + (size_t)(lane & 15) * ld + (lane >> 4) * MF::KPL;
    for (int k0 = 0; k0 < kpad; k0 += MF::KSTEP) {
      typename MF::frag a = MF::load(arow + k0);
#pragma unroll
      for (int ct = 0; ct < GEMM_TILE_COLS / 16; ++ct) {
        typename MF::frag b = MF::load(bcol + (size_t)ct * 16 * ld + k0);
        acc[ct] = MF::mma(a, b, acc[ct]);
      }
    }
    // ---- accumulators -> global, rows j < n; lane holds column (lane & 15) of
    // each 16-column tile ct and rows row0 + 16*wave + out_row(lane>>4, v).
#pragma unroll
    for (int ct = 0; ct < GEMM_TILE_COLS / 16; ++ct) {
      int64_t c = c0 + ct * 16 + (lane & 15);
      if (c >= total_cols) continue;
      int64_t base, step;
      if (inner == 1) {
        base = c * n;
        step = 1;
      } else {
        uint32_t o = (uint32_t)c / uinner, i = (uint32_t)c - o * uinner;
        base = (int64_t)o * slab + i;
        step = inner;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int j = row0 + wave * 16 + MF::out_row(lane >> 4, v);
        if (j < n) {
          int64_t a = base + (int64_t)j * step;
          double y = (double)acc[ct][v];
          if (out_scale) y *= out_scale[a % nscale];
          out[a] = Conv<Tout>::from_f64(y);
        }
      }
    }
  }
}

// ------------------------------------------------ mode GEMM, streaming form
// Same contract as mode_gemm, for n <= GEMM2_MAX_N.  No tile staging and no
// block barriers in the main loop: every wave streams its own 16-column strips.
//  * Op (n x n, zero padded to kpad columns) is copied to LDS once per block;
//  * a wave loads the B operand X[k][c0..c0+15] for all k straight from global
//    memory in the MFMA operand layout (lane: column lane & 15, k-slice lane >> 4),
//    multiplies it by the n/16 full 16-row tiles of Op (A operand from LDS),
//  * and computes the n % 16 fringe rows on the vector ALU from the same B
//    registers, reduced across the four k-slices with cross-lane shuffles.
// Latency is hidden by occupancy (many independent waves per SIMD) and by the
// next strip's loads, issued under the current strip's products.
// Dynamic LDS: 16 * ceil(n/16) * ld elements.
constexpr int GEMM2_MAX_N = 79;
constexpr int GEMM2_THREADS = 256;

// NC = n as a compile-time constant (0: n taken from the argument).  With NC
// fixed, the MFMA chain has no runtime guards, so the accumulators stay in
// place instead of being copied at every branch.
// SC: 1 = in_scale, 2 = out_scale (length nscale, index taken modulo nscale):
// per-entry factors multiplied in on load (1) or on store (2); a column's
// entries lie in one period of nscale, so the modulo is taken once per column.
// Separate instantiations keep each one's registers to its own path.  SC 0:
// both null.
// RS > 1: the full 16-row tiles are split into RS parts, one per block of a
// group of RS consecutive blocks (numbered so that a group shares an XCD), and
// each block holds only its part of Op (plus the fringe rows, computed by the
// last part) in LDS: smaller blocks, more of them per CU, shorter MFMA chains.
// The grid is then a multiple of RS.
template <typename Tin, typename Tout, typename TC, int NC, int SC, int RS = 1>
__global__ void __launch_bounds__(GEMM2_THREADS, 2)
mode_gemm_small(const Tin *__restrict__ in, Tout *__restrict__ out,
                const typename Mfma<TC>::elem *__restrict__ Op, int n_arg, int64_t inner,
                int64_t total_cols, const double *__restrict__ in_scale,
                const double *__restrict__ out_scale, int64_t nscale) {
  typedef Mfma<TC> MF;
  typedef typename MF::elem E;
  constexpr int NMAX = NC ? NC : GEMM2_MAX_N;
  constexpr int KSMAX = (NMAX + MF::KSTEP - 1) / MF::KSTEP;
  constexpr int QALL = NMAX / 16;
  static_assert(QALL % RS == 0, "row tiles must split evenly");
  constexpr int QMAX = QALL / RS;  // full row tiles of this block
  const int n = NC ? NC : n_arg;
  extern __shared__ __align__(16) unsigned char smem[];
  // Op tile in LDS, sized for NMAX (the runtime-n variant reads the full NMAX
  // range unguarded; every entry with j >= n or k >= n is zero).  Local row j
  // is Op row row0 + j below 16 QMAX, fringe row 16 QALL + (j - 16 QMAX) above.
  constexpr int NROWS = RS == 1 ? (NMAX + 15) / 16 * 16 : 16 * QMAX + (NMAX - 16 * QALL);
  unsigned gb = blockIdx.x;
  if (RS > 1) {
    const unsigned nb = gridDim.x, q8 = nb / 8, r8 = nb % 8, xcd = blockIdx.x % 8;
    gb = xcd * q8 + (xcd < r8 ? xcd : r8) + blockIdx.x / 8;
  }
  const int part = RS > 1 ? (int)(gb % RS) : 0;
  const bool lastp = part == RS - 1;
  const int row0 = 16 * QMAX * part;
  const int64_t sblk = RS > 1 ? (int64_t)(gb / RS) : (int64_t)blockIdx.x;
  const int64_t nsblk = RS > 1 ? (int64_t)(gridDim.x / RS) : (int64_t)gridDim.x;
  constexpr int KPADM = KSMAX * MF::KSTEP;
  const int ld = lds_ld<TC>(NMAX);
  E *opl = reinterpret_cast<E *>(smem);  // [NROWS][ld]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t nstrips = (total_cols + 15) >> 4;
  const int64_t slab = (int64_t)n * inner;
  const uint32_t uinner = (uint32_t)inner;
  const int col = lane & 15, kg = lane >> 4;
  const int64_t wstride = nsblk * (GEMM2_THREADS / 64);
  // column c -> (base address, stride along the contracted axis)
  auto locate = [&](int64_t c, int64_t &base, int64_t &step) {
    if (inner == 1) {
      base = c * n;
      step = 1;
    } else {
      uint32_t o = (uint32_t)c / uinner, i = (uint32_t)c - o * uinner;
      base = (int64_t)o * slab + i;
      step = inner;
    }
  };
  struct Col {
    int64_t base, step, sb;  // first entry, stride along k, offset in the factors
    bool valid;
  };
  auto column = [&](int64_t strip) {
    const int64_t c = strip * 16 + col;
    Col r;
    r.valid = strip < nstrips && c < total_cols;
    locate(r.valid ? c : 0, r.base, r.step);
    r.sb = SC != 0 ? r.base % nscale : 0;
    return r;
  };
  // The B operand of one strip stays in registers as raw input values (and, SC
  // 1, input factors), one slot per k step.  ROLL: slot s takes the next
  // strip's k step s as soon as the MFMAs of step s have read it, so the next
  // strip's loads run under this strip's products with one set of registers (a
  // second full set, double buffering, halves the waves per SIMD at n = 130,
  // 131).  The runtime-n form (fringe rows accumulated after the products)
  // loads each strip after the previous one's stores and converts it to
  // operands at once, and so do the BF16 forms with a wider input type (their
  // raw values take 2-4 times the operand registers), the scaled forms whose
  // input is wider than the accumulator or whose operands are BF16, and the
  // FP64 input-scaled form (rolled, they spill: 36.0 against 32.0 us for the
  // FP64 n = 130 product at 16,900 columns of 131).
  constexpr bool ROLL =
      NC != 0 && (SC == 0 ? (MF::KPL == 1 || sizeof(Tin) == sizeof(E))
                          : (MF::KPL == 1 && sizeof(Tin) <= sizeof(typename MF::acc_elem) &&
                             !(SC == 1 && sizeof(E) == 8)));
  constexpr bool SCI = SC == 1;
  Tin raw[KSMAX][MF::KPL];
  double rsc[SCI ? KSMAX : 1][MF::KPL];
  E bv[ROLL ? 1 : KSMAX][MF::KPL];  // !ROLL: the strip's operands
  auto prepare = [&]() {
    if constexpr (!ROLL) {
#pragma unroll
      for (int s = 0; s < KSMAX; ++s)
#pragma unroll
        for (int u = 0; u < MF::KPL; ++u) {
          const int k = s * MF::KSTEP + kg * MF::KPL + u;
          double x = Conv<Tin>::to_f64(raw[s][u]);
          if constexpr (SCI) x *= rsc[s][u];
          bv[s][u] = k < n ? MF::from_f64(x) : MF::zero();
        }
    }
  };
  auto issue = [&](const Col &L, int s) {
#pragma unroll
    for (int u = 0; u < MF::KPL; ++u) {
      const int k = s * MF::KSTEP + kg * MF::KPL + u;
      const int64_t off = k < n ? (int64_t)k * L.step : 0;  // padding: a valid address
      raw[s][u] = in[L.base + off];
      if constexpr (SCI) rsc[s][u] = in_scale[L.sb + off];
    }
  };
  int64_t strip = sblk * (GEMM2_THREADS / 64) + wave;
  Col cur = column(strip);
  // ROLL, unscaled: the first strip's loads go out before the operator copy,
  // so the two overlap (the scaled forms have no registers to spare there)
  if constexpr (ROLL && SC == 0) {
#pragma unroll
    for (int s = 0; s < KSMAX; ++s) issue(cur, s);
  }
  // operator copy: all of a thread's loads in flight at once (one round trip
  // for the block's share at n = 130, 131 in FP64)
  constexpr int FILL = NROWS * KPADM;
  constexpr int FU0 = (FILL + GEMM2_THREADS - 1) / GEMM2_THREADS, FU = FU0 < 24 ? FU0 : 24;
  for (int e0 = tid; e0 < FILL; e0 += GEMM2_THREADS * FU) {
    E v[FU];
#pragma unroll
    for (int u = 0; u < FU; ++u) {
      const int e = e0 + u * GEMM2_THREADS;
      const int j = e / KPADM, k = e - j * KPADM;
      const int gj = j < 16 * QMAX ? row0 + j : 16 * QALL + (j - 16 * QMAX);
      const bool ok = e < FILL && gj < n && k < n;
      v[u] = Op[ok ? (size_t)gj * n + k : 0];
      if (!ok) v[u] = MF::zero();
    }
#pragma unroll
    for (int u = 0; u < FU; ++u) {
      const int e = e0 + u * GEMM2_THREADS;
      const int j = e / KPADM, k = e - j * KPADM;
      if (e < FILL) opl[(size_t)j * ld + k] = v[u];
    }
  }
  __syncthreads();
  if constexpr (ROLL && SC != 0) {
#pragma unroll
    for (int s = 0; s < KSMAX; ++s) issue(cur, s);
  }

  constexpr int NFR = NMAX - 16 * QALL;  // fringe rows (vector ALU, last part)
  auto operand = [&](int s, E (&be)[MF::KPL]) {
#pragma unroll
    for (int u = 0; u < MF::KPL; ++u) {
      if constexpr (ROLL) {
        const int k = s * MF::KSTEP + kg * MF::KPL + u;
        double x = Conv<Tin>::to_f64(raw[s][u]);
        if constexpr (SCI) x *= rsc[s][u];
        be[u] = k < n ? MF::from_f64(x) : MF::zero();
      } else {
        be[u] = bv[s][u];
      }
    }
  };
  // One strip: full row tiles on MFMA (the Op fragments of k step s+1 are read
  // from LDS while the MFMAs of step s run), the fringe rows on the vector ALU
  // from the same operand values (every part computes them, the last stores
  // them: no branches in the loop), then the stores.
  auto process = [&](const Col &c, const Col &nx) {
    // output factors (SC 2): all of the lane's in flight at once; ROLL: before
    // the next strip's loads, so that the stores wait only for them
    double osc[SC == 2 ? QMAX : 1][4], osf[NFR > 0 ? NFR : 1];
    auto load_out_factors = [&]() {
      if constexpr (SC == 2) {
#pragma unroll
        for (int t = 0; t < QMAX; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int j = row0 + 16 * t + MF::out_row(kg, v);
            osc[t][v] = out_scale[c.sb + (j < n ? (int64_t)j * c.step : 0)];
          }
#pragma unroll
        for (int q = 0; q < NFR; ++q) {
          const int j = 16 * QALL + q;
          osf[q] = out_scale[c.sb + (j < n ? (int64_t)j * c.step : 0)];
        }
      }
    };
    if constexpr (ROLL) load_out_factors();
    typename MF::acc acc[QMAX];
#pragma unroll
    for (int t = 0; t < QMAX; ++t)
      for (int v = 0; v < 4; ++v) acc[t][v] = 0;
    const E *abase = opl + (size_t)col * ld + kg * MF::KPL;
    const E *fbase = opl + (size_t)16 * QMAX * ld + kg * MF::KPL;  // fringe rows
    typename MF::frag acur[QMAX], anext[QMAX];
#pragma unroll
    for (int t = 0; t < QMAX; ++t) anext[t] = MF::load(abase + (size_t)16 * t * ld);
    double fr[NFR > 0 ? NFR : 1] = {};
#pragma unroll
    for (int s = 0; s < KSMAX; ++s) {
#pragma unroll
      for (int t = 0; t < QMAX; ++t) acur[t] = anext[t];
      // this step's fringe-row values, then the next step's A fragments:
      // issued ahead of this step's MFMAs (the fence keeps them there), so
      // both reads have those MFMAs to arrive
      E fo[ROLL && NFR > 0 ? NFR : 1][MF::KPL];
      if constexpr (ROLL) {
#pragma unroll
        for (int q = 0; q < NFR; ++q)
#pragma unroll
          for (int u = 0; u < MF::KPL; ++u) fo[q][u] = fbase[(size_t)q * ld + s * MF::KSTEP + u];
      }
      if (s + 1 < KSMAX) {
#pragma unroll
        for (int t = 0; t < QMAX; ++t)
          anext[t] = MF::load(abase + (size_t)16 * t * ld + (s + 1) * MF::KSTEP);
      }
      __builtin_amdgcn_sched_barrier(0);
      E be[MF::KPL];
      operand(s, be);
      typename MF::frag b = MF::make(be);
#pragma unroll
      for (int t = 0; t < QMAX; ++t) acc[t] = MF::mma(acur[t], b, acc[t]);
      if constexpr (ROLL) {
        __builtin_amdgcn_sched_barrier(0);  // fringe products after the MFMAs
#pragma unroll
        for (int q = 0; q < NFR; ++q)
#pragma unroll
          for (int u = 0; u < MF::KPL; ++u) fr[q] += MF::to_f64(fo[q][u]) * MF::to_f64(be[u]);
        issue(nx, s);  // past the last strip: column 0 again, never used
      }
      // one k step of lookahead only: without this fence the scheduler hoists
      // every LDS read of the loop and the register count quadruples
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (!ROLL) {
#pragma unroll
      for (int q = 0; q < NFR; ++q) {
        if (!lastp) break;
        double sum = 0.0;
#pragma unroll
        for (int s = 0; s < KSMAX; ++s) {
          E be[MF::KPL];
          operand(s, be);
#pragma unroll
          for (int u = 0; u < MF::KPL; ++u)
            sum += MF::to_f64(fbase[(size_t)q * ld + s * MF::KSTEP + u]) * MF::to_f64(be[u]);
        }
        fr[q] = sum;
      }
    }
#pragma unroll
    for (int q = 0; q < NFR; ++q) {
      fr[q] += __shfl_xor(fr[q], 16, 64);
      fr[q] += __shfl_xor(fr[q], 32, 64);
    }
    if (!c.valid) return;
    double yv[QMAX][4];
#pragma unroll
    for (int t = 0; t < QMAX; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) yv[t][v] = (double)acc[t][v];
    if constexpr (SC == 2) {
      if constexpr (!ROLL) load_out_factors();
#pragma unroll
      for (int t = 0; t < QMAX; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) yv[t][v] *= osc[t][v];
#pragma unroll
      for (int q = 0; q < NFR; ++q) fr[q] *= osf[q];
    }
#pragma unroll
    for (int t = 0; t < QMAX; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int j = row0 + 16 * t + MF::out_row(kg, v);
        if (j < n) out[c.base + (int64_t)j * c.step] = Conv<Tout>::from_f64(yv[t][v]);
      }
#pragma unroll
    for (int q = 0; q < NFR; ++q) {
      int j = 16 * QALL + q;
      if (lastp && kg == 0 && j < n) out[c.base + (int64_t)j * c.step] = Conv<Tout>::from_f64(fr[q]);
    }
  };
  // Tail split (streaming forms without input scaling): when the strips
  // beyond the last full round of waves are no more than the block groups (on
  // the 128-element annulus, 33 of 1,057 strips along t and 41 of 1,065 along
  // x, with 512 waves per row part), the waves run only the full rounds, and
  // block group g then takes tail strip g with the NW waves of each block
  // splitting the k steps; the partial sums meet in LDS (the operator's space,
  // after a barrier) and are added in wave order.  Otherwise a third round ran
  // a full strip on a few waves.  FP64 operands only: with FP32 operands
  // (shorter MFMA chains) the split tail measured slower than that round.
  constexpr bool TSPLIT = ROLL && SC != 1 && sizeof(E) == 8;
  constexpr int NW = GEMM2_THREADS / 64;                // waves per block
  constexpr int NV = QMAX * 4 + (NFR > 0 ? NFR : 0);  // partial sums per lane
  typedef typename MF::acc_elem AE;
  const int64_t full = TSPLIT ? nstrips / wstride * wstride : nstrips;
  const int64_t ntail = nstrips - full;
  const bool split = TSPLIT && ntail > 0 && ntail <= nsblk &&
                     (size_t)NROWS * ld * sizeof(E) >= (size_t)NW * NV * 64 * sizeof(AE);
  const int64_t lim = split ? full : nstrips;
  auto tail = [&](int64_t tstrip) {
    const Col tc = column(tstrip);
    constexpr int KQ = (KSMAX + NW - 1) / NW;  // k steps per wave
    const int s0 = wave * KQ;
#pragma unroll
    for (int s = 0; s < KSMAX; ++s)
      if (s >= s0 && s < s0 + KQ) issue(tc, s);
    typename MF::acc acc[QMAX];
#pragma unroll
    for (int t = 0; t < QMAX; ++t)
      for (int v = 0; v < 4; ++v) acc[t][v] = 0;
    double fr[NFR > 0 ? NFR : 1] = {};
    const E *abase = opl + (size_t)col * ld + kg * MF::KPL;
    const E *fbase = opl + (size_t)16 * QMAX * ld + kg * MF::KPL;
#pragma unroll
    for (int s = 0; s < KSMAX; ++s) {
      if (s < s0 || s >= s0 + KQ) continue;
      E be[MF::KPL];
      operand(s, be);
      typename MF::frag b = MF::make(be);
#pragma unroll
      for (int t = 0; t < QMAX; ++t)
        acc[t] = MF::mma(MF::load(abase + (size_t)16 * t * ld + s * MF::KSTEP), b, acc[t]);
#pragma unroll
      for (int q = 0; q < NFR; ++q)
#pragma unroll
        for (int u = 0; u < MF::KPL; ++u)
          fr[q] += MF::to_f64(fbase[(size_t)q * ld + s * MF::KSTEP + u]) * MF::to_f64(be[u]);
    }
#pragma unroll
    for (int q = 0; q < NFR; ++q) {
      fr[q] += __shfl_xor(fr[q], 16, 64);
      fr[q] += __shfl_xor(fr[q], 32, 64);
    }
    __syncthreads();  // every wave is done with Op: its space takes the partial sums
    AE *red = reinterpret_cast<AE *>(smem);  // [NW][NV][64]
#pragma unroll
    for (int t = 0; t < QMAX; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[((size_t)wave * NV + 4 * t + v) * 64 + lane] = acc[t][v];
#pragma unroll
    for (int q = 0; q < NFR; ++q) red[((size_t)wave * NV + 4 * QMAX + q) * 64 + lane] = (AE)fr[q];
    __syncthreads();
    if (wave != 0 || !tc.valid) return;
    auto total = [&](int i) {
      AE v = red[(size_t)i * 64 + lane];
#pragma unroll
      for (int w = 1; w < NW; ++w) v += red[((size_t)w * NV + i) * 64 + lane];
      return (double)v;
    };
#pragma unroll
    for (int t = 0; t < QMAX; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = row0 + 16 * t + MF::out_row(kg, v);
        double y = total(4 * t + v);
        if constexpr (SC == 2) y *= out_scale[tc.sb + (j < n ? (int64_t)j * tc.step : 0)];
        if (j < n) out[tc.base + (int64_t)j * tc.step] = Conv<Tout>::from_f64(y);
      }
#pragma unroll
    for (int q = 0; q < NFR; ++q) {
      const int j = 16 * QALL + q;
      double y = total(4 * QMAX + q);
      if constexpr (SC == 2) y *= out_scale[tc.sb + (j < n ? (int64_t)j * tc.step : 0)];
      if (lastp && kg == 0 && j < n) out[tc.base + (int64_t)j * tc.step] = Conv<Tout>::from_f64(y);
    }
  };
  for (; strip < lim; strip += wstride) {
    if constexpr (ROLL) {
      const Col nx = column(strip + wstride < lim ? strip + wstride : nstrips);
      process(cur, nx);
      cur = nx;
    } else {
      cur = column(strip);
#pragma unroll
      for (int s = 0; s < KSMAX; ++s) issue(cur, s);
      prepare();
      process(cur, cur);
    }
  }
  if constexpr (TSPLIT) {
    if (split && sblk < ntail) tail(full + sblk);  // the same for a whole block
  }
}

// ---------------------------------------------------------- time solves
// For each spatial eigen-index k (and right-hand side), solve
//   (gamma W + nu lam_k M) q = r   along t (stride ns between consecutive t),
// with banded W, M given as rows of 2P+1 coefficients: wb[i*(2P+1) + P + m] =
// W[i][i+m] (zero outside the matrix).  Elimination without pivoting: the
// symmetric part of the matrix is (gamma/2) e_n e_n^T + nu lam_k M, positive
// definite, so every pivot is positive; a non-positive pivot sets *flag.
// Scratch (compute type, [rhs][t][P+1][ns]): the U row entries u[i][i+1..i+P-1],
// the reciprocal pivot and the forward-substituted y_i.  u[i][i+P] equals the
// untouched matrix entry and is recomputed.
template <typename Tio, typename TC, int P>
__global__ void time_band_solve(const Tio *__restrict__ in, Tio *__restrict__ out,
                                const double *__restrict__ lam, const TC *__restrict__ wb,
                                const TC *__restrict__ mb, TC gamma, TC nu, int nt, int64_t ns,
                                int nrhs, TC *__restrict__ scratch, int *__restrict__ flag) {
  constexpr int B = 2 * P + 1;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ns * nrhs) return;
  int64_t rhs = g / ns, k = g - rhs * ns;
  const Tio *r = in + rhs * ns * nt + k;
  Tio *q = out + rhs * ns * nt + k;
  TC *sc = scratch + rhs * ns * nt * (P + 1) + k;
  const TC lk = (TC)lam[k];
  cptr<TC> wbc = as_const(wb), mbc = as_const(mb);
  // rolling state of the previous P rows: U entries (c = 1..P), reciprocal pivot, y
  TC pu[P][P + 1];   // pu[dist-1][c] = u[i-dist][i-dist+c], c = 1..P (index 0 unused)
  TC prp[P], py[P];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    prp[a] = 0;
    py[a] = 0;
#pragma unroll
    for (int c = 0; c <= P; ++c) pu[a][c] = 0;
  }
  bool bad = false;
  for (int i = 0; i < nt; ++i) {
    TC row[B];
#pragma unroll
    for (int m = 0; m < B; ++m) row[m] = gamma * wbc[i * B + m] + nu * lk * mbc[i * B + m];
    TC y = Conv<Tio>::to_f64(r[(int64_t)i * ns]);
    // eliminate with rows j = i-P .. i-1 (increasing j): dist = P .. 1
#pragma unroll
    for (int dist = P; dist >= 1; --dist) {
      if (i - dist >= 0) {
        TC l = row[P - dist] * prp[dist - 1];
#pragma unroll
        for (int c = 1; c <= P; ++c) row[P - dist + c] -= l * pu[dist - 1][c];
        y -= l * py[dist - 1];
      }
    }
    TC piv = row[P];
    if (!(piv > (TC)0)) bad = true;
    TC rp = (TC)1 / piv;
    // shift state
#pragma unroll
    for (int a = P - 1; a >= 1; --a) {
      prp[a] = prp[a - 1];
      py[a] = py[a - 1];
#pragma unroll
      for (int c = 1; c <= P; ++c) pu[a][c] = pu[a - 1][c];
    }
    prp[0] = rp;
    py[0] = y;
#pragma unroll
    for (int c = 1; c <= P; ++c) pu[0][c] = row[P + c];
    TC *s = sc + (int64_t)i * (P + 1) * ns;
#pragma unroll
    for (int c = 1; c < P; ++c) s[(int64_t)(c - 1) * ns] = row[P + c];
    s[(int64_t)(P - 1) * ns] = rp;
    s[(int64_t)P * ns] = y;
  }
  if (bad) *flag = 1;
  // back substitution, rolling last P solution values
  TC qn[P];
#pragma unroll
  for (int a = 0; a < P; ++a) qn[a] = 0;  // qn[c-1] = q[i+c]
  for (int i = nt - 1; i >= 0; --i) {
    const TC *s = sc + (int64_t)i * (P + 1) * ns;
    TC acc = s[(int64_t)P * ns];
#pragma unroll
    for (int c = 1; c < P; ++c) acc -= s[(int64_t)(c - 1) * ns] * qn[c - 1];
    // outermost superdiagonal: untouched entry
    TC uP = gamma * wbc[i * B + 2 * P] + nu * lk * mbc[i * B + 2 * P];
    acc -= uP * qn[P - 1];
    TC qi = acc * s[(int64_t)(P - 1) * ns];
#pragma unroll
    for (int a = P - 1; a >= 1; --a) qn[a] = qn[a - 1];
    qn[0] = qi;
    q[(int64_t)i * ns] = Conv<Tio>::from_f64((double)qi);
  }
}


// ----------------------------------------------- time solves, register form
// Same systems as time_band_solve for a compile-time number of rows NT and
// bandwidth P, with no scratch memory: each lane keeps only a checkpoint of the
// elimination state (the previous P rows of the U factor) every C rows.  Back
// substitution walks the segments backwards, refactoring each segment from its
// checkpoint (the same arithmetic in the same order, so the U entries are
// bit-identical to the forward sweep) and substituting.  HBM traffic is the
// compulsory read of r and write of q (plus, with YREG false, one write and one
// read of the forward-substituted values through the output buffer).
template <typename TC, int P> struct ElimState {
  TC rp[P];          // rp[d-1] = 1 / u[i-d][i-d]
  TC u[P][P + 1];    // u[d-1][c] = u[i-d][i-d+c], c = 1 .. P (index 0 unused)
};

// 1/x for the pivots: hardware reciprocal refined by two Newton steps
// (r <- r (2 - x r)), accurate to a few ulp; pivots are positive and far from
// the range limits.
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * (2.0 - x * r);
  r = r * (2.0 - x * r);
  return r;
}
__device__ inline float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  r = r * (2.0f - x * r);
  return r;
}

// Band coefficients of one row (W and M entries at offsets -P..P).
template <typename TC, int P> struct RowCoef {
  TC w[2 * P + 1], m[2 * P + 1];
};
template <typename TC, int P>
__device__ inline void load_coef(RowCoef<TC, P> &c, cptr<TC> wb, cptr<TC> mb, int i) {
#pragma unroll
  for (int k = 0; k < 2 * P + 1; ++k) {
    c.w[k] = wb[i * (2 * P + 1) + k];
    c.m[k] = mb[i * (2 * P + 1) + k];
  }
}

// Factor row i (coefficients cf) against the state of rows i-P..i-1.  Returns
// the eliminated row (row[P] = pivot, row[P+c] = u[i][i+c]) and multipliers.
// The outermost superdiagonal u[j][j+P] of an earlier row j is the untouched
// matrix entry, carried in the state.
template <typename TC, int P>
__device__ inline void factor_row(int i, const ElimState<TC, P> &st, const RowCoef<TC, P> &cf,
                                  TC gamma, TC nul, TC (&row)[2 * P + 1], TC (&l)[P]) {
  constexpr int B = 2 * P + 1;
#pragma unroll
  for (int m = 0; m < B; ++m) row[m] = gamma * cf.w[m] + nul * cf.m[m];
#pragma unroll
  for (int dist = P; dist >= 1; --dist) {
    l[dist - 1] = 0;
    if (i - dist >= 0) {
      TC lv = row[P - dist] * st.rp[dist - 1];
      l[dist - 1] = lv;
#pragma unroll
      for (int c = 1; c <= P; ++c) row[P - dist + c] -= lv * st.u[dist - 1][c];
    }
  }
}

template <typename TC, int P>
__device__ inline void push_row(ElimState<TC, P> &st, const TC (&row)[2 * P + 1], TC rp) {
#pragma unroll
  for (int a = P - 1; a >= 1; --a) {
    st.rp[a] = st.rp[a - 1];
#pragma unroll
    for (int c = 1; c <= P; ++c) st.u[a][c] = st.u[a - 1][c];
  }
  st.rp[0] = rp;
#pragma unroll
  for (int c = 1; c <= P; ++c) st.u[0][c] = row[P + c];
}

template <typename Tio, typename TC, int NT, int P, int C, bool YREG>
__global__ void __launch_bounds__(256)
time_band_solve_reg(const Tio *__restrict__ in, Tio *__restrict__ out, const double *__restrict__ lam,
                    const TC *__restrict__ wb, const TC *__restrict__ mb, TC gamma, TC nu, int64_t ns,
                    int nrhs, TC *__restrict__ ysc, int *__restrict__ flag) {
  // YREG: forward-substituted values stay in registers; otherwise they go to
  // ysc ([rhs][t][k], compute type; may alias `out` when Tio == TC) and are
  // read back segment by segment by the backward sweep.
  constexpr int NSEG = (NT + C - 1) / C;
  constexpr int NY = YREG ? NT : 1;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ns * nrhs) return;
  int64_t rhs = g / ns, k = g - rhs * ns;
  const Tio *r = in + rhs * ns * NT + k;
  Tio *q = out + rhs * ns * NT + k;
  TC *ys = ysc + rhs * ns * NT + k;
  const TC nul = nu * (TC)lam[k];
  const cptr<TC> wbc = as_const(wb), mbc = as_const(mb);
  // all right-hand-side loads up front (YREG) or one segment ahead (otherwise)
  TC y[NY];
  if (YREG) {
#pragma unroll
    for (int i = 0; i < NY; ++i) y[i] = (TC)Conv<Tio>::to_f64(r[(int64_t)i * ns]);
  }
  constexpr int CR = YREG ? 1 : C;
  TC rseg[CR], rnext[CR];
  if (!YREG) {
#pragma unroll
    for (int u = 0; u < CR; ++u) rnext[u] = (TC)Conv<Tio>::to_f64(r[(int64_t)(u < NT ? u : 0) * ns]);
  }
  TC yp[P];
#pragma unroll
  for (int a = 0; a < P; ++a) yp[a] = 0;
  ElimState<TC, P> st;
#pragma unroll
  for (int a = 0; a < P; ++a) {
    st.rp[a] = 0;
#pragma unroll
    for (int c = 0; c <= P; ++c) st.u[a][c] = 0;
  }
  ElimState<TC, P> ck[NSEG];
  bool bad = false;
  RowCoef<TC, P> cf, cfn;
  load_coef<TC, P>(cfn, wbc, mbc, 0);
  // forward sweep: factor and forward-substitute, checkpoint every C rows
#pragma unroll
  for (int sg = 0; sg < NSEG; ++sg) {
    const int i0 = sg * C;
    const int i1 = (i0 + C < NT) ? i0 + C : NT;
    ck[sg] = st;
    if (!YREG) {
#pragma unroll
      for (int u = 0; u < CR; ++u) rseg[u] = rnext[u];
      if (sg + 1 < NSEG) {
#pragma unroll
        for (int u = 0; u < CR; ++u) {
          int i = i1 + u;
          rnext[u] = (TC)Conv<Tio>::to_f64(r[(int64_t)(i < NT ? i : 0) * ns]);
        }
      }
    }
#pragma unroll
    for (int i = i0; i < i1; ++i) {
      cf = cfn;
      if (i + 1 < NT) load_coef<TC, P>(cfn, wbc, mbc, i + 1);  // next row's coefficients
      TC row[2 * P + 1], l[P];
      factor_row<TC, P>(i, st, cf, gamma, nul, row, l);
      if (YREG) {
#pragma unroll
        for (int dist = P; dist >= 1; --dist)
          if (i - dist >= 0) y[YREG ? i : 0] -= l[dist - 1] * y[YREG && i >= dist ? i - dist : 0];
      } else {
        TC yi = rseg[YREG ? 0 : i - i0];
#pragma unroll
        for (int dist = P; dist >= 1; --dist)
          if (i - dist >= 0) yi -= l[dist - 1] * yp[dist - 1];
#pragma unroll
        for (int a = P - 1; a >= 1; --a) yp[a] = yp[a - 1];
        yp[0] = yi;
        ys[(int64_t)i * ns] = yi;
      }
      if (!(row[P] > (TC)0)) bad = true;
      push_row<TC, P>(st, row, recip(row[P]));
      // one row at a time: stops the scheduler from computing every row's
      // entries up front (hundreds of live registers)
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (bad) *flag = 1;
  // backward sweep over segments.  nul and the band pointers pass through an
  // empty asm so the compiler cannot reuse the forward sweep's rows (which
  // would keep the whole U factor live); the recomputed values are bit-identical.
  TC nul2 = nul;
  asm volatile("" : "+v"(nul2));
  const TC *wb2p = wb, *mb2p = mb;
  asm volatile("" : "+s"(wb2p), "+s"(mb2p));
  const cptr<TC> wb2 = as_const(wb2p), mb2 = as_const(mb2p);
  TC qn[P];  // qn[c-1] = q[i+c]
#pragma unroll
  for (int a = 0; a < P; ++a) qn[a] = 0;
#pragma unroll
  for (int sgi = NSEG - 1; sgi >= 0; --sgi) {
    const int i0 = sgi * C;
    const int i1 = (i0 + C < NT) ? i0 + C : NT;
    TC su[C][P + 1];  // su[i-i0][0] = 1/pivot, su[i-i0][c] = u[i][i+c] (c = 1..P)
    TC yseg[YREG ? 1 : C];
    if (!YREG) {  // this segment's forward-substituted values
#pragma unroll
      for (int i = i0; i < i1; ++i) yseg[YREG ? 0 : i - i0] = ys[(int64_t)i * ns];
    }
    ElimState<TC, P> s2 = ck[sgi];
    load_coef<TC, P>(cfn, wb2, mb2, i0);
#pragma unroll
    for (int i = i0; i < i1; ++i) {
      cf = cfn;
      if (i + 1 < i1) load_coef<TC, P>(cfn, wb2, mb2, i + 1);
      TC row[2 * P + 1], l[P];
      factor_row<TC, P>(i, s2, cf, gamma, nul2, row, l);
      TC rp = recip(row[P]);
      su[i - i0][0] = rp;
#pragma unroll
      for (int c = 1; c <= P; ++c) su[i - i0][c] = row[P + c];
      push_row<TC, P>(s2, row, rp);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = i1 - 1; i >= i0; --i) {
      TC acc = YREG ? y[YREG ? i : 0] : yseg[YREG ? 0 : i - i0];
#pragma unroll
      for (int c = 1; c <= P; ++c) acc -= su[i - i0][c] * qn[c - 1];
      TC qi = acc * su[i - i0][0];
#pragma unroll
      for (int a = P - 1; a >= 1; --a) qn[a] = qn[a - 1];
      qn[0] = qi;
      q[(int64_t)i * ns] = Conv<Tio>::from_f64((double)qi);
    }
  }
}


// ------------------------------------- time solves, right-looking register form
// Same systems and contract as time_band_solve_reg, eliminated right-looking:
// the elimination state at pivot i is the P x P window S[a][b] = entry
// (i+a, i+b) of the partially eliminated matrix (rows i .. i+P-1 after the
// pivots before i).  Entries of those rows further right are still the
// original matrix entries, so S is the whole state: P*P values per checkpoint
// instead of the previous P rows of U.  Pivot i gives the U row u[i][i+b]
// = S[0][b] (b < P), u[i][i+P] = original entry, and multipliers
// l_a = S[a][0] / u[i][i] for the P rows below it.
//
// The matrix entries pivot i needs (column i+P of rows i..i+P-1, row i+P up
// to the diagonal) come from a step record: rec[i*RS + e] (W) and
// rec[i*RS + RH + e] (M), e = 0..2P, stored contiguously so that one pivot
// costs two scalar loads.
template <int P> struct StepRec {
  static constexpr int RH = (2 * P + 1 + 3) / 4 * 4;  // W half (padded)
  static constexpr int RS = 2 * RH;                   // record stride
};

// Segments of the backward sweep.  While segment s is substituted the lane
// holds the checkpoints of segments 1..s (P*P values each) and P+1 values per
// row of segment s (1/pivot, u[i][i+1..i+P-1], y_i); segment lengths shrink
// with s so that this total is about the same for every segment.
template <int NT, int P, int NSEG> struct SegPlan {
  static constexpr int start(int s) {
    if (s <= 0) return 0;
    if (s >= NSEG) return NT;
    double B = ((P + 1.0) * NT + P * P * NSEG * (NSEG - 1) / 2.0) / NSEG;
    double acc = 0;
    for (int t = 0; t < s; ++t) acc += (B - P * P * t) / (P + 1.0);
    int v = (int)(acc + 0.5);
    return v < NT ? v : NT;
  }
  static constexpr int len(int s) { return start(s + 1) - start(s); }
  static constexpr int maxlen() {
    int m = 0;
    for (int s = 0; s < NSEG; ++s) m = len(s) > m ? len(s) : m;
    return m;
  }
};

template <typename TC, int P> struct Window {
  TC s[P][P];
};

// One step record in registers (scalar registers: the address is uniform).
template <typename TC, int P> struct StepVals {
  TC w[2 * P + 1], m[2 * P + 1];
};
template <typename TC, int NT, int P>
__device__ inline void load_step(StepVals<TC, P> &v, cptr<TC> rec, int i) {
#pragma unroll
  for (int e = 0; e < 2 * P + 1; ++e) {
    v.w[e] = (i < NT) ? rec[i * StepRec<P>::RS + e] : (TC)0;
    v.m[e] = (i < NT) ? rec[i * StepRec<P>::RS + StepRec<P>::RH + e] : (TC)0;
  }
}

// Window at pivot 0: the leading P x P block (band layout wb/mb).
template <typename TC, int NT, int P>
__device__ inline void first_window(Window<TC, P> &S, cptr<TC> wb, cptr<TC> mb, TC gamma, TC nul) {
#pragma unroll
  for (int a = 0; a < P; ++a)
#pragma unroll
    for (int b = 0; b < P; ++b) {
      const int o = a * (2 * P + 1) + P + (b - a);
      S.s[a][b] = (a < NT && b < NT) ? gamma * wb[o] + nul * mb[o] : (TC)0;
    }
}

// Eliminate pivot i with its step record sv: returns 1/pivot, the U row
// (u[1..P-1]; u[i][i+P] is step entry 0) and the multipliers l[1..P] (rows
// i+1 .. i+P); advances S to pivot i+1.
template <typename TC, int NT, int P>
__device__ inline void pivot_step(int i, Window<TC, P> &S, const StepVals<TC, P> &sv, TC gamma,
                                  TC nul, TC &rp, TC (&u)[P + 1], TC (&l)[P + 1]) {
  const bool inner = i + P < NT;  // row i+P exists
  auto entry = [&](int e) { return inner ? gamma * sv.w[e] + nul * sv.m[e] : (TC)0; };
  rp = recip(S.s[0][0]);
#pragma unroll
  for (int b = 1; b < P; ++b) u[b] = S.s[0][b];
  u[P] = entry(0);
#pragma unroll
  for (int a = 1; a < P; ++a) l[a] = S.s[a][0] * rp;
  l[P] = entry(P) * rp;
  Window<TC, P> S2;
#pragma unroll
  for (int a = 1; a < P; ++a) {
#pragma unroll
    for (int b = 1; b < P; ++b) S2.s[a - 1][b - 1] = S.s[a][b] - l[a] * u[b];
    S2.s[a - 1][P - 1] = entry(a) - l[a] * u[P];
  }
#pragma unroll
  for (int b = 1; b <= P; ++b) S2.s[P - 1][b - 1] = entry(P + b) - l[P] * u[b];
  S = S2;
}

// rec: step records (see StepRec); wb, mb: band rows (first window only).
// YREC false: the forward-substituted values go to ysc ([rhs][t][k], compute
// type; may alias out when Tio == TC) and are read back segment by segment.
// YREC true: nothing is stored; the right-hand-side window is checkpointed with
// S and the backward sweep redoes the forward substitution of each segment
// from the input (read a second time, shortly after the first).
// LROWS (YREC only): the first LROWS right-hand-side rows, which the backward
// sweep reads again last, are kept in LDS (LROWS * 256 values per block)
// instead of being read from HBM a second time.
template <typename Tio, typename TC, int NT, int P, int NSEG, bool YREC, int LROWS>
__global__ void __launch_bounds__(256, sizeof(TC) == 8 ? 2 : (YREC ? 3 : 4))
time_band_solve_rl(const Tio *__restrict__ in, Tio *__restrict__ out, const double *__restrict__ lam,
                   const TC *__restrict__ rec, const TC *__restrict__ wb, const TC *__restrict__ mb,
                   TC gamma_arg, TC nu, int64_t ns, int nrhs, TC *__restrict__ ysc,
                   int *__restrict__ flag) {
  static_assert(YREC || LROWS == 0, "the LDS copy serves the recomputed substitution");
  __shared__ TC rstash[LROWS > 0 ? LROWS * 256 : 1];
  typedef SegPlan<NT, P, NSEG> SP;
  constexpr int LMAX = SP::maxlen();
  // right-hand-side prefetch distance (rows)
  constexpr int DP = sizeof(TC) == 8 ? 8 : 16;  // measured: FP64 no gain past 8
  constexpr int D = NT - P < DP ? NT - P : DP;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ns * nrhs) return;
  int64_t rhs = g / ns, k = g - rhs * ns;
  const Tio *r = in + rhs * ns * NT + k;
  Tio *q = out + rhs * ns * NT + k;
  TC *ys = YREC ? nullptr : ysc + rhs * ns * NT + k;
  // gamma and nu*lambda_k live in vector registers, so that each matrix entry
  // is one multiply and one fma with a single scalar operand each
  TC gamma = gamma_arg, nul = nu * (TC)lam[k];
  asm volatile("" : "+v"(gamma));
  const cptr<TC> recc = as_const(rec), wbc = as_const(wb), mbc = as_const(mb);
  auto rload = [&](const Tio *base, int i) {
    return (TC)Conv<Tio>::to_f64(base[(int64_t)(i < NT ? i : 0) * ns]);
  };
  // the backward sweep's second read of the input: the LDS copy for the first
  // LROWS rows, else a relaxed atomic load, which the compiler does not merge
  // with the first read (merging would keep every input value live across the
  // whole forward sweep)
  const int tx = threadIdx.x;
  auto stash = [&](int i, TC v) {
    if (LROWS > 0 && i < LROWS) rstash[(LROWS > 0 ? i : 0) * 256 + tx] = v;
  };
  auto rload_again = [&](int i) {
    if (LROWS > 0 && i < LROWS) return rstash[(LROWS > 0 ? i : 0) * 256 + tx];
    const Tio *p = r + (int64_t)(i < NT ? i : 0) * ns;
    Tio v;
    __atomic_load(p, &v, __ATOMIC_RELAXED);
    return (TC)Conv<Tio>::to_f64(v);
  };

  // ---- forward sweep: factor, forward-substitute, checkpoint at segment
  // starts.  The right-hand side of row i+P enters the window at pivot i; it
  // is loaded D rows ahead.
  Window<TC, P> S;
  first_window<TC, NT, P>(S, wbc, mbc, gamma, nul);
  TC rw[P], rq[D > 0 ? D : 1];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    rw[a] = rload(r, a);
    if (YREC) stash(a, rw[a]);
  }
#pragma unroll
  for (int j = 0; j < D; ++j) rq[j] = rload(r, P + j);
  Window<TC, P> ck[NSEG];
  TC ckr[YREC ? NSEG : 1][P];
  // pivot check without a per-row mask: smallest pivot, and a sum that turns
  // NaN if any pivot is NaN or infinite
  TC pmin = S.s[0][0], pnan = 0;
  StepVals<TC, P> sv, svn;
  load_step<TC, NT, P>(svn, recc, 0);
#pragma unroll
  for (int i = 0; i < NT; ++i) {
#pragma unroll
    for (int sg = 1; sg < NSEG; ++sg)
      if (i == SP::start(sg)) {
        ck[sg] = S;
        if (YREC) {
#pragma unroll
          for (int a = 0; a < P; ++a) ckr[YREC ? sg : 0][a] = rw[a];
        }
      }
    sv = svn;
    if (i + 1 < NT) load_step<TC, NT, P>(svn, recc, i + 1);  // next pivot's entries
    pmin = __builtin_fmin(pmin, S.s[0][0]);
    pnan = S.s[0][0] * (TC)0 + pnan;
    TC rp, uu[P + 1], l[P + 1];
    pivot_step<TC, NT, P>(i, S, sv, gamma, nul, rp, uu, l);
    const TC yi = rw[0];
    if (!YREC) ys[(int64_t)i * ns] = yi;
    TC rin = 0;
    if (i + P < NT && D > 0) {
      rin = rq[i % D];
      if (i + P + D < NT) rq[i % D] = rload(r, i + P + D);
      if (YREC) stash(i + P, rin);
    }
#pragma unroll
    for (int a = 1; a < P; ++a) rw[a - 1] = rw[a] - l[a] * yi;
    rw[P - 1] = rin - l[P] * yi;
    // the window is needed only at checkpoints when nothing is stored: pin it
    // here so that the substitution is not postponed (which would keep every
    // multiplier live until the backward sweep)
#pragma unroll
    for (int a = 0; a < P; ++a) asm volatile("" : "+v"(rw[a]));
    // one pivot at a time: keeps the scheduler from hoisting every row's
    // coefficient arithmetic (hundreds of live registers)
    __builtin_amdgcn_sched_barrier(0);
  }
  if (!(pmin > (TC)0) || !(pnan == (TC)0)) *flag = 1;

  // ---- backward sweep over segments: refactor the segment from its
  // checkpoint (same arithmetic, bit-identical U and y), then substitute.
  // gamma, nul and the pointers pass through an empty asm so that the compiler
  // cannot reuse the forward sweep's values (that would keep all of U live).
  TC gamma2 = gamma, nul2 = nul;
  asm volatile("" : "+v"(gamma2), "+v"(nul2));
  const TC *rec2p = rec, *wb2p = wb, *mb2p = mb;
  asm volatile("" : "+s"(rec2p), "+s"(wb2p), "+s"(mb2p));
  const cptr<TC> rec2 = as_const(rec2p), wb2 = as_const(wb2p), mb2 = as_const(mb2p);
  TC qn[P];  // qn[b-1] = q[i+b]
#pragma unroll
  for (int a = 0; a < P; ++a) qn[a] = 0;
#pragma unroll
  for (int sgi = NSEG - 1; sgi >= 0; --sgi) {
    const int i0 = SP::start(sgi), i1 = SP::start(sgi + 1);
    // YREC: right-hand sides entering the window in this segment (rows
    // i0+P .. i1-1+P) and, for the first segment, rows 0 .. P-1; otherwise
    // the stored forward-substituted values
    TC yseg[LMAX];
    TC rw2[P];
    if (YREC) {
#pragma unroll
      for (int i = i0; i < i1; ++i) yseg[i - i0] = (i + P < NT) ? rload_again(i + P) : (TC)0;
      if (sgi == 0) {
#pragma unroll
        for (int a = 0; a < P; ++a) rw2[a] = rload_again(a);
      } else {
#pragma unroll
        for (int a = 0; a < P; ++a) rw2[a] = ckr[YREC ? sgi : 0][a];
      }
    } else {
#pragma unroll
      for (int i = i0; i < i1; ++i) yseg[i - i0] = ys[(int64_t)i * ns];
    }
    Window<TC, P> S2;
    if (sgi == 0) first_window<TC, NT, P>(S2, wb2, mb2, gamma2, nul2);
    else S2 = ck[sgi];
    TC su[LMAX][P];  // su[i-i0][0] = 1/pivot, su[i-i0][b] = u[i][i+b], b = 1..P-1
    StepVals<TC, P> sv2, sv2n;
    load_step<TC, NT, P>(sv2n, rec2, i0);
#pragma unroll
    for (int i = i0; i < i1; ++i) {
      sv2 = sv2n;
      if (i + 1 < i1) load_step<TC, NT, P>(sv2n, rec2, i + 1);
      TC rp, uu[P + 1], l[P + 1];
      pivot_step<TC, NT, P>(i, S2, sv2, gamma2, nul2, rp, uu, l);
      su[i - i0][0] = rp;
#pragma unroll
      for (int b = 1; b < P; ++b) su[i - i0][b] = uu[b];
      if (YREC) {  // forward substitution again: y_i replaces r_{i+P} in yseg
        const TC yi = rw2[0];
        const TC rin = yseg[i - i0];
#pragma unroll
        for (int a = 1; a < P; ++a) rw2[a - 1] = rw2[a] - l[a] * yi;
        rw2[P - 1] = rin - l[P] * yi;
        yseg[i - i0] = yi;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = i1 - 1; i >= i0; --i) {
      TC acc = yseg[i - i0];
#pragma unroll
      for (int b = 1; b < P; ++b) acc -= su[i - i0][b] * qn[b - 1];
      // u[i][i+P] is the untouched matrix entry (step entry 0)
      if (i + P < NT)
        acc -= (gamma2 * rec2[i * StepRec<P>::RS] + nul2 * rec2[i * StepRec<P>::RS + StepRec<P>::RH]) *
               qn[P - 1];
      TC qi = acc * su[i - i0][0];
#pragma unroll
      for (int a = P - 1; a >= 1; --a) qn[a] = qn[a - 1];
      qn[0] = qi;
      q[(int64_t)i * ns] = Conv<Tio>::from_f64((double)qi);
    }
  }
}
}  // namespace stig

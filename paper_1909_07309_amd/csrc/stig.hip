// libstig: C ABI over the HIP kernels of the fast-diagonalization apply, the
// Kronecker / CSR matvec and (flexible) GMRES.  See include/stig.h for the
// contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <type_traits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/stig.h"
#include "kernels_fd.h"
#include "kernels_krylov.h"
#include "kernels_matvec.h"
#include "kernels_plane.h"
#include "kernels_sym.h"
#include "kernels_plane_sym.h"
#include "kernels_arrow.h"
#include "stig_internal.h"

using namespace stig;

namespace {

thread_local std::string g_last_error;

stig_status fail(stig_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(STIG_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));        \
  } while (0)

#define STIG_TRY(expr)                \
  do {                                \
    stig_status _s = (expr);          \
    if (_s < 0) return _s;            \
  } while (0)

constexpr int MAX_P = 5;
constexpr size_t GEMM_LDS_LIMIT = 160 * 1024;
constexpr int64_t GEMM2_GRID = 1024;  // persistent blocks of the small-n GEMM
constexpr int KRY_MAXB = 64;          // right-hand sides in one lockstep GMRES cycle
constexpr size_t WS_ALIGN = 256;      // alignment of the workspace and of its views

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  stig_status ensure(size_t need) {
    if (need <= bytes) return STIG_OK;
    if (p) {
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    if (hipMalloc(&p, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(STIG_ENOMEM, "hipMalloc of " + std::to_string(need) + " bytes failed");
    }
    bytes = need;
    return STIG_OK;
  }
  template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

// A view of caller-owned memory (the workspace, or the static scratch array):
// never allocated or freed here.  ensure() only checks that the view is large
// enough, so every use states the bytes it needs.
struct Span {
  void *p = nullptr;
  size_t bytes = 0;
  void set(char *base, size_t off, size_t n) {
    p = base ? base + off : nullptr;
    bytes = base ? n : 0;
  }
  stig_status ensure(size_t need) const {
    if (need <= bytes && (p || need == 0)) return STIG_OK;
    return fail(STIG_EINVAL, "workspace view of " + std::to_string(bytes) + " bytes, " +
                                 std::to_string(need) + " needed (stig_workspace_bytes)");
  }
  template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

template <typename T> stig_status upload(DevBuf &b, const std::vector<T> &v, hipStream_t s) {
  STIG_TRY(b.ensure(v.size() * sizeof(T)));
  HIP_TRY(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return STIG_OK;
}

}  // namespace

struct stig_plan {
  int d = 0;
  int n[3] = {1, 1, 1};
  int nt = 0, ps = 0, pt = 0;
  int64_t Ns = 0, N = 0;
  hipStream_t stream = nullptr;
  int device = 0;     // the plan's device (current at stig_plan_create)
  int num_cu = 256;  // compute units of the plan's device
  bool ready = false;
  double gamma = 1.0, nu = 1.0;
  // eigenvectors: [l] -> U_l and U_l^T in FP64, FP32, BF16 (row-major n x n)
  DevBuf U64[3], UT64[3], U32[3], UT32[3], U16[3], UT16[3];
  // parity-split eigenbasis (persymmetric pencils): half operators per
  // precision [0 f64, 1 f32, 2 bf16] and direction, forward (rows of U^T) and
  // backward (rows of U), even (NE x NE) and odd (M x M) halves
  bool split[3] = {false, false, false};
  DevBuf hFE[3][3], hFO[3][3], hBE[3][3], hBO[3][3];
  DevBuf lam;            // Ns doubles: lambda_k = sum_l lambda_{l,i_l}
  // lam in the padded plane layout of the fused x/y passes, one table per
  // storage size of the intermediates (8, 4, 2 bytes: plane stride lamp_ps[i])
  DevBuf lamp[3];
  int64_t lamp_ps[3] = {0, 0, 0};
  DevBuf tW64, tWT64, tM64, tW32, tWT32, tM32;  // time bands (unscaled)
  DevBuf tR64[2], tR32[2];  // step records of [W; M] and [W^T; M] (right-looking solve)
  // arrowhead form of the time pencil (n_t = 32 q + 2): U^T and U in mode order
  // per precision [f64, f32, bf16], tables [d | g | h | sigma] plain / transposed
  bool arrow_ok = false;     // the fused kernel's tables (n_t = 32 q + 2, one zero mode)
  DevBuf aTf[3], aTb[3], aTab64[2], aTab32[2];
  // the same factorization for any n_t (three-pass form): U^T (rows = modes)
  // and U (rows = t) in natural mode order per precision, the middle-factor
  // tables [d | g | h | sigma] plain / transposed, the zero-mode count
  bool arrow_gen = false;
  int arrow_nz = 0;
  DevBuf aGf[3], aGb[3], aGtab64[2], aGtab32[2];
  std::vector<double> hWt, hMt;  // host copies of the time factors (arrowhead setup)
  DevBuf tgW, tgWT, tnM;  // time bands scaled by gamma / nu (matvec)
  DevBuf sK[3], sM[3];    // spatial bands (matvec, mass apply)
  DevBuf sId, sZero;      // one-row identity / zero band (third direction of a 2D stencil)
  DevBuf dmh;             // D^{-1/2}, N doubles (optional)
  // host copies of the diagonals of the 1D factors (geometry scaling)
  std::vector<double> dK1[3], dM1[3], dWt, dMt;
  bool has_dmh = false;
  bool plane_fusion = true;  // fused x/y products in the FD apply
  int time_kernel = 0;        // 0 right-looking, 1 left-looking register form, 2 generic
  bool parity_split = true;   // half-size mode products where the basis is split
  bool time_recompute = true; // right-looking: redo the forward substitution backward
  const int64_t *csr_rowptr = nullptr;
  const int32_t *csr_col = nullptr;
  const double *csr_val = nullptr;
  int64_t csr_nnz = 0;
  // sparse spatial factors M_s, K_s ([0] as given, [1] transposed): by diagonals
  // (ell_dia, offsets in ellC) or padded column-major rows (columns in ellC)
  int ell_w[2] = {0, 0};
  bool ell_dia[2] = {false, false};
  int ell_omin[2] = {0, 0}, ell_omax[2] = {0, 0};  // offset range (diagonal form)
  int ell_nruns[2] = {0, 0};  // runs of consecutive offsets (diagonal form)
  DevBuf ellR[2];             // [run][3]: first offset, length, first diagonal
  DevBuf ellC[2], ellM[2], ellK[2];
  // small buffers owned by the plan (setup): reduction partials, coefficient
  // slots (4 KRY_MAXV doubles per right-hand side, KRY_MAXB of them), breakdown flag
  DevBuf partial, small, flag;
  // caller-owned workspace (stig_set_workspace) and the views of it that one
  // call uses: apply intermediates s0/s1 and time scratch; matvec / mass /
  // lifting intermediates m0..m3, lift0/lift1 and the lifting weights; the
  // Krylov bases.  The views are laid out by bind_workspace at each call.
  char *ws = nullptr;
  size_t ws_bytes = 0;
  Span s0, s1, tscr, m0, m1, m2, m3, lift0, lift1, liftw, V, Z, AZ, tmp;
  // pinned host staging of the small Krylov transfers (setup): 4 coefficient
  // slots of KRY_MAXV doubles per right-hand side, then the breakdown flag
  double *pin = nullptr;
  size_t pin_n = 0;  // doubles in the pinned area
  // optional per-kernel timing with HIP events on the plan's stream
  bool prof = false;
  struct Pending {
    int kind;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
  double prof_ms[STIG_NUM_KERNEL_KINDS] = {0};
  double prof_bytes[STIG_NUM_KERNEL_KINDS] = {0};
  long long prof_count[STIG_NUM_KERNEL_KINDS] = {0};
  ~stig_plan() {
    for (auto &q : pending) {
      (void)hipEventDestroy(q.a);
      (void)hipEventDestroy(q.b);
    }
    for (auto e : free_events) (void)hipEventDestroy(e);
    if (pin) (void)hipHostFree(pin);
  }
};

namespace {

// ------------------------------------------------------------------ helpers

stig_status check_plan(const stig_plan *p, bool need_ready) {
  if (!p) return fail(STIG_EINVAL, "null plan");
  if (need_ready && !p->ready) return fail(STIG_ESTATE, "stig_setup_1d_pencils has not been called");
  return STIG_OK;
}

hipEvent_t take_event(stig_plan *p) {
  if (!p->free_events.empty()) {
    hipEvent_t e = p->free_events.back();
    p->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Bracket one kernel launch with events when profiling is on.
struct ProfScope {
  stig_plan *p;
  int kind;
  double bytes;
  hipEvent_t a = nullptr;
  ProfScope(stig_plan *p_, int kind_, double bytes_) : p(p_), kind(kind_), bytes(bytes_) {
    if (p->prof) {
      a = take_event(p);
      if (a) (void)hipEventRecord(a, p->stream);
    }
  }
  ~ProfScope() {
    if (p->prof && a) {
      hipEvent_t b = take_event(p);
      if (b) {
        (void)hipEventRecord(b, p->stream);
        p->pending.push_back({kind, bytes, a, b});
      } else {
        p->free_events.push_back(a);
      }
    }
  }
};

stig_status prof_collect(stig_plan *p) {
  if (p->pending.empty()) return STIG_OK;
  HIP_TRY(hipStreamSynchronize(p->stream));
  for (auto &q : p->pending) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, q.a, q.b));
    p->prof_ms[q.kind] += ms;
    p->prof_bytes[q.kind] += q.bytes;
    p->prof_count[q.kind] += 1;
    p->free_events.push_back(q.a);
    p->free_events.push_back(q.b);
  }
  p->pending.clear();
  return STIG_OK;
}

// band[j*(2P+1) + P + m] = A[j][j+m]; error if A has entries outside the band.
stig_status extract_band(const double *A, int n, int P, std::vector<double> &band,
                         const char *name) {
  band.assign((size_t)n * (2 * P + 1), 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = A[(size_t)i * n + j];
      if (std::abs(i - j) > P) {
        if (v != 0.0)
          return fail(STIG_EINVAL, std::string(name) + " has an entry outside its bandwidth");
        continue;
      }
      band[(size_t)i * (2 * P + 1) + P + (j - i)] = v;
    }
  return STIG_OK;
}

// Step records of the right-looking time elimination (StepRec): for pivot i,
// entry e < P is A[i+e][i+P] and entry P+b (b = 0..P) is A[i+P][i+b], zero
// where row i+P does not exist; W entries, then M entries at offset RH.
std::vector<double> step_records(const std::vector<double> &wband, const std::vector<double> &mband,
                                 int n, int P) {
  const int B = 2 * P + 1, RH = (B + 3) / 4 * 4, RS = 2 * RH;
  std::vector<double> rec((size_t)n * RS, 0.0);
  for (int i = 0; i < n; ++i) {
    if (i + P >= n) continue;
    for (int part = 0; part < 2; ++part) {
      const std::vector<double> &band = part ? mband : wband;
      double *o = rec.data() + (size_t)i * RS + part * RH;
      for (int e = 0; e < P; ++e) o[e] = band[(size_t)(i + e) * B + P + (P - e)];
      for (int b = 0; b <= P; ++b) o[P + b] = band[(size_t)(i + P) * B + P + (b - P)];
    }
  }
  return rec;
}

template <typename T> std::vector<T> convert(const std::vector<double> &v);
template <> std::vector<double> convert(const std::vector<double> &v) { return v; }
template <> std::vector<float> convert(const std::vector<double> &v) {
  return std::vector<float>(v.begin(), v.end());
}
template <> std::vector<uint16_t> convert(const std::vector<double> &v) {
  std::vector<uint16_t> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = float_to_bf16_bits((float)v[i]);
  return o;
}

// Largest n_t of the three-pass arrowhead form (its mode products stage U in LDS).
constexpr int ARROW_GEN_MAX_NT = 200;

// Arrowhead form of the time pencil (Section 4.2.2, eq. time_eig_2).  For any
// n_t <= ARROW_GEN_MAX_NT (when `general`): U^T / U in natural mode order and the
// middle-factor tables of the three-pass form (arrow_gen).  For n_t = 32 q + 2
// with a zero mode: the fused kernel's tables (kernels_arrow.h), U^T / U in its
// mode order (arrow_ok).  Both for W_t and (transposed systems) W_t^T, whose
// form is D^T: d -> -d, arrow column and row exchanged.  A pencil without the
// block structure leaves both false.
stig_status setup_arrowhead(stig_plan *p, bool general) {
  p->arrow_ok = false;
  p->arrow_gen = false;
  const int n = p->nt;
  const bool fused_shape = n >= 34 && (n - 2) % 32 == 0;
  general = general && n <= ARROW_GEN_MAX_NT;
  if (!fused_shape && !general) return STIG_OK;
  if ((int)p->hWt.size() != n * n || (int)p->hMt.size() != n * n) return STIG_OK;
  const double *Wt = p->hWt.data(), *Mt = p->hMt.data();
  std::vector<double> U((size_t)n * n), D((size_t)n * n);
  int nz = 0;
  if (!time_arrowhead(n, Wt, Mt, 1e-10, U.data(), D.data(), &nz)) return STIG_OK;
  if (general) {
    // mode order of the three-pass form: blocks (2j, 2j + 1) first (natural
    // modes nz + 2j, nz + 2j + 1), the zero mode at n - 2 (natural 0) when
    // nz = 1, the arrow mode n - 1 last; perm[position] = natural mode
    std::vector<int> perm(n);
    for (int q = 0; q < n - 1 - nz; ++q) perm[q] = nz + q;
    if (nz) perm[n - 2] = 0;
    perm[n - 1] = n - 1;
    std::vector<double> gf((size_t)n * n), gb((size_t)n * n);
    for (int r = 0; r < n; ++r)
      for (int t = 0; t < n; ++t) {
        gf[(size_t)r * n + t] = U[(size_t)t * n + perm[r]];
        gb[(size_t)t * n + r] = U[(size_t)t * n + perm[r]];
      }
    STIG_TRY(upload(p->aGf[0], gf, p->stream));
    STIG_TRY(upload(p->aGb[0], gb, p->stream));
    STIG_TRY(upload(p->aGf[1], convert<float>(gf), p->stream));
    STIG_TRY(upload(p->aGb[1], convert<float>(gb), p->stream));
    STIG_TRY(upload(p->aGf[2], convert<uint16_t>(gf), p->stream));
    STIG_TRY(upload(p->aGb[2], convert<uint16_t>(gb), p->stream));
    for (int tr = 0; tr < 2; ++tr) {
      std::vector<double> tab((size_t)3 * n + 1, 0.0);
      for (int q = 0; q + 1 < n - 1 - nz; q += 2) {
        const int a = perm[q];
        const double d = D[(size_t)a * n + a + 1];
        tab[q] = tab[q + 1] = tr ? -d : d;
      }
      for (int q = 0; q < n - 1; ++q) {
        const int r = perm[q];
        const double gcol = D[(size_t)r * n + (n - 1)], hrow = D[(size_t)(n - 1) * n + r];
        tab[n + q] = tr ? hrow : gcol;
        tab[2 * n + q] = tr ? gcol : hrow;
      }
      tab[3 * n] = D[(size_t)(n - 1) * n + (n - 1)];
      STIG_TRY(upload(p->aGtab64[tr], tab, p->stream));
      STIG_TRY(upload(p->aGtab32[tr], convert<float>(tab), p->stream));
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->arrow_nz = nz;
    p->arrow_gen = true;
  }
  if (!fused_shape || nz != 1) return STIG_OK;
  const int NM = n - 2;  // modes in 2 x 2 blocks
  // mode order: block j -> rows 32 (j/16) + j%16 and that + 16; zero mode NM;
  // last mode NM + 1.  perm[r] = natural index (zero mode 0, block j: 1 + 2j, 2 + 2j).
  std::vector<int> perm(n);
  for (int j = 0; j < NM / 2; ++j) {
    const int r1 = 32 * (j / 16) + j % 16;
    perm[r1] = 1 + 2 * j;
    perm[r1 + 16] = 2 + 2 * j;
  }
  perm[NM] = 0;
  perm[NM + 1] = n - 1;
  std::vector<double> tf((size_t)n * n), tb((size_t)n * n);
  for (int r = 0; r < n; ++r)
    for (int t = 0; t < n; ++t) {
      tf[(size_t)r * n + t] = U[(size_t)t * n + perm[r]];
      tb[(size_t)t * n + r] = U[(size_t)t * n + perm[r]];
    }
  for (int tr = 0; tr < 2; ++tr) {
    std::vector<double> tab((size_t)3 * n + 1, 0.0);
    for (int r = 0; r < NM; ++r) {
      const int a = perm[r] - ((perm[r] - 1) % 2);  // first member of the block
      const double d = D[(size_t)a * n + a + 1];
      tab[r] = tr ? -d : d;
    }
    for (int r = 0; r <= NM; ++r) {
      const double gcol = D[(size_t)perm[r] * n + (n - 1)], hrow = D[(size_t)(n - 1) * n + perm[r]];
      tab[n + r] = tr ? hrow : gcol;
      tab[2 * n + r] = tr ? gcol : hrow;
    }
    tab[3 * n] = D[(size_t)(n - 1) * n + (n - 1)];
    STIG_TRY(upload(p->aTab64[tr], tab, p->stream));
    STIG_TRY(upload(p->aTab32[tr], convert<float>(tab), p->stream));
  }
  STIG_TRY(upload(p->aTf[0], tf, p->stream));
  STIG_TRY(upload(p->aTb[0], tb, p->stream));
  STIG_TRY(upload(p->aTf[1], convert<float>(tf), p->stream));
  STIG_TRY(upload(p->aTb[1], convert<float>(tb), p->stream));
  STIG_TRY(upload(p->aTf[2], convert<uint16_t>(tf), p->stream));
  STIG_TRY(upload(p->aTb[2], convert<uint16_t>(tb), p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->arrow_ok = true;
  return STIG_OK;
}

inline unsigned grid_for(int64_t work, int block, int64_t cap = 1 << 20) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ------------------------------------------------------------ mode GEMM launch

template <typename Tin, typename Tout, typename TC>
stig_status launch_mode_gemm(stig_plan *p, const Tin *in, Tout *out,
                             const typename Mfma<TC>::elem *op, int n, int64_t inner,
                             int64_t total_cols, const double *in_scale,
                             const double *out_scale) {
  typedef typename Mfma<TC>::elem E;
  if (total_cols >= ((int64_t)1 << 31)) return fail(STIG_EINVAL, "tensor too large for one launch");
  // streaming kernel: compile-time sizes of the workloads' spatial directions
  // (65, 49: cube; 32: extruded annulus; 130: annulus; scaled: 32, 130) and of
  // the annulus time axes (131 and 33, arrowhead form), runtime n up to
  // GEMM2_MAX_N otherwise
  const bool sc = in_scale || out_scale;
  const int nc = sc ? ((n == 32 || n == 130) ? n : 0)
                    : ((n == 65 || n == 49 || n == 32 || n == 130 || n == 131 || n == 33) ? n : 0);
  // the streaming kernel scales either its input or its output; both at once
  // take the tiled kernel
  if ((nc != 0 || n <= GEMM2_MAX_N) && !(in_scale && out_scale)) {
    // LDS as sized inside mode_gemm_small: the compile-time n, else GEMM2_MAX_N;
    // n = 130 splits its 8 full row tiles over 4 blocks in FP64 (rows: 32 + 2
    // fringe) and over 2 in FP32 / BF16 (64 + 2), the faster split for each
    constexpr int RS130 = sizeof(E) == 8 ? 4 : 2;
    const int nm = nc ? nc : GEMM2_MAX_N;
    const int rs = (nc == 130 || nc == 131) ? RS130 : 1;
    const int rows = rs == 1 ? round_up(nm, 16) : 16 * (nm / 16 / rs) + nm % 16;
    size_t lds = (size_t)rows * lds_ld<TC>(nm) * sizeof(E);
    if (lds > GEMM_LDS_LIMIT) return fail(STIG_EINVAL, "mode size too large for LDS");
    int64_t nstrips = (total_cols + 15) / 16;
    ProfScope ps(p, STIG_K_MODE_GEMM, (double)total_cols * n * (sizeof(Tin) + sizeof(Tout)));
    static size_t configured[13] = {};  // per kernel of this type triple
    static int per_cu[13] = {};         // resident blocks per CU at that LDS size
    static size_t per_cu_lds[13] = {};
    auto go = [&](auto kern, int slot) -> stig_status {
      if (lds > 65536 && lds > configured[slot]) {
        HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds));
        configured[slot] = lds;
      }
      if (per_cu_lds[slot] != lds) {
        int nb = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, GEMM2_THREADS, lds));
        per_cu[slot] = std::max(nb, 1);
        per_cu_lds[slot] = lds;
      }
      // persistent: no more block groups than are resident at once, so the
      // strips beyond one round are prefetched by running waves instead of
      // starting new blocks (which would fill Op into LDS again)
      const int64_t resident = std::max<int64_t>(1, (int64_t)per_cu[slot] * p->num_cu / rs);
      const unsigned grid =
          (unsigned)std::min<int64_t>(std::min<int64_t>((nstrips + 3) / 4, GEMM2_GRID), resident) * rs;
      hipLaunchKernelGGL(kern, dim3(grid), dim3(GEMM2_THREADS), lds, p->stream, in, out, op, n,
                         inner, total_cols, in_scale, out_scale, p->N);
      HIP_TRY(hipGetLastError());
      return STIG_OK;
    };
    if (in_scale) {
      if (nc == 32) return go(mode_gemm_small<Tin, Tout, TC, 32, 1>, 5);
      if (nc == 130) return go(mode_gemm_small<Tin, Tout, TC, 130, 1, RS130>, 6);
      return go(mode_gemm_small<Tin, Tout, TC, 0, 1>, 7);
    }
    if (out_scale) {
      if (nc == 32) return go(mode_gemm_small<Tin, Tout, TC, 32, 2>, 9);
      if (nc == 130) return go(mode_gemm_small<Tin, Tout, TC, 130, 2, RS130>, 10);
      return go(mode_gemm_small<Tin, Tout, TC, 0, 2>, 11);
    }
    if (nc == 65) return go(mode_gemm_small<Tin, Tout, TC, 65, 0>, 0);
    if (nc == 49) return go(mode_gemm_small<Tin, Tout, TC, 49, 0>, 1);
    if (nc == 32) return go(mode_gemm_small<Tin, Tout, TC, 32, 0>, 2);
    if (nc == 130) return go(mode_gemm_small<Tin, Tout, TC, 130, 0, RS130>, 3);
    if (nc == 131) return go(mode_gemm_small<Tin, Tout, TC, 131, 0, RS130>, 8);
    if (nc == 33) return go(mode_gemm_small<Tin, Tout, TC, 33, 0>, 12);
    return go(mode_gemm_small<Tin, Tout, TC, 0, 0>, 4);
  }
  const int jt = (n + 15) / 16;
  const int ld = lds_ld<TC>(n);
  // as many 16-row output tiles per block as fit in LDS (all of them when possible,
  // so each input tile is read from HBM once)
  int JB = jt;
  auto lds_of = [&](int jb) { return (size_t)(16 * jb + GEMM_TILE_COLS) * ld * sizeof(E); };
  while (JB > 1 && lds_of(JB) > GEMM_LDS_LIMIT) JB = (JB + 1) / 2;
  size_t lds = lds_of(JB);
  if (lds > GEMM_LDS_LIMIT) return fail(STIG_EINVAL, "mode size too large for LDS");
  const int groups = (jt + JB - 1) / JB;
  auto kern = mode_gemm<Tin, Tout, TC>;
  static size_t configured = 0;  // per instantiation
  if (lds > 65536 && lds > configured) {
    HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    configured = lds;
  }
  int64_t ntiles = (total_cols + GEMM_TILE_COLS - 1) / GEMM_TILE_COLS;
  unsigned grid = (unsigned)std::min<int64_t>(ntiles, 4096);
  ProfScope ps(p, STIG_K_MODE_GEMM, (double)total_cols * n * (sizeof(Tin) + sizeof(Tout)));
  hipLaunchKernelGGL(kern, dim3(grid, groups), dim3(64 * JB), lds, p->stream, in, out, op, n, inner,
                     total_cols, in_scale, out_scale, p->N);
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

// Fused x/y products of every plane: Y_o = Op_y X_o Op_x^T (n_x = n_y = n).
template <typename Tin, typename Tout, typename TC, int NC>
stig_status launch_plane_nc(stig_plan *p, const Tin *in, Tout *out,
                            const typename Mfma<TC>::elem *opx,
                            const typename Mfma<TC>::elem *opy, int n, int64_t planes,
                            int64_t in_stride, int64_t out_stride) {
  typedef typename Mfma<TC>::elem E;
  constexpr int NMAX = NC ? NC : PLANE_MAX_N;
  constexpr int NR = NMAX / 16 * 16 + NMAX % 16;
  constexpr int threads = 64 * (NMAX / 16);
  const size_t lds = (size_t)(2 * NR + 1) * lds_ld<TC>(NR) * sizeof(E);
  auto kern = mode_gemm_plane<Tin, Tout, TC, NC>;
  static int per_cu = 0;  // per instantiation: resident blocks per CU
  if (per_cu == 0) {
    if (lds > 65536)
      HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
    int nb = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, threads, lds));
    per_cu = std::max(nb, 1);
  }
  // persistent blocks, every block with the same number of planes (+-1)
  int64_t grid = std::min<int64_t>(planes, (int64_t)per_cu * p->num_cu);
  int64_t per = (planes + grid - 1) / grid;
  grid = (planes + per - 1) / per;
  ProfScope ps(p, STIG_K_PLANE_GEMM, (double)planes * n * n * (sizeof(Tin) + sizeof(Tout)));
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, p->stream, in, out, opx, opy,
                     n, planes, in_stride, out_stride);
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

template <typename Tin, typename Tout, typename TC>
stig_status launch_plane(stig_plan *p, const Tin *in, Tout *out,
                         const typename Mfma<TC>::elem *opx, const typename Mfma<TC>::elem *opy,
                         int n, int64_t planes, int64_t in_stride, int64_t out_stride) {
  if (n < 1 || n > PLANE_MAX_N) return fail(STIG_EINVAL, "plane size out of range");
  if (planes < 1) return STIG_OK;
  if (n == 65)
    return launch_plane_nc<Tin, Tout, TC, 65>(p, in, out, opx, opy, n, planes, in_stride, out_stride);
  if (n == 49)
    return launch_plane_nc<Tin, Tout, TC, 49>(p, in, out, opx, opy, n, planes, in_stride, out_stride);
  return launch_plane_nc<Tin, Tout, TC, 0>(p, in, out, opx, opy, n, planes, in_stride, out_stride);
}

// Half-size mode product along direction l with the parity-split operators.
template <typename TC> struct PrecIdx;
template <> struct PrecIdx<double> { static constexpr int v = 0; };
template <> struct PrecIdx<float> { static constexpr int v = 1; };
template <> struct PrecIdx<bf16> { static constexpr int v = 2; };

inline bool sym_size_ok(int n) { return n == 32 || n == 33 || n == 64 || n == 65; }

template <typename Tin, typename Tout, typename TC, int M, bool ODD, bool FWD, int CG>
stig_status launch_sym_m(stig_plan *p, const Tin *in, Tout *out, int l, int64_t inner,
                         int64_t total_cols) {
  typedef typename Mfma<TC>::elem E;
  constexpr int NE = M + (ODD ? 1 : 0);
  const int pi = PrecIdx<TC>::v;
  const E *oe = (FWD ? p->hFE[pi][l] : p->hBE[pi][l]).template as<E>();
  const E *oo = (FWD ? p->hFO[pi][l] : p->hBO[pi][l]).template as<E>();
  const size_t lds = (size_t)(NE + M) * lds_ld<TC>(NE) * sizeof(E);
  const int64_t nstrips = (total_cols + 16 * CG - 1) / (16 * CG);
  const unsigned grid = (unsigned)std::min<int64_t>((nstrips + 3) / 4, GEMM2_GRID);
  const int n = 2 * M + (ODD ? 1 : 0);
  ProfScope ps(p, STIG_K_MODE_GEMM, (double)total_cols * n * (sizeof(Tin) + sizeof(Tout)));
  hipLaunchKernelGGL((mode_gemm_sym<Tin, Tout, TC, M, ODD, FWD, CG>), dim3(grid), dim3(SYM_THREADS),
                     lds, p->stream, in, out, oe, oo, inner, total_cols);
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

// Column pairs (8-byte accesses) for FP32 storage between intermediates, where
// the two columns of a pair are contiguous (inner even).  Measured on the
// 65^3 x 66 cube: 36 us per FP32 pass against 38 us with single columns; for
// BF16, groups of 2 or 4 columns were slower (37-40 us against 27 us) because
// of the extra fragment and accumulator registers.
template <typename Tin, typename Tout, typename TC, int M, bool ODD, bool FWD>
stig_status launch_sym_cg(stig_plan *p, const Tin *in, Tout *out, int l, int64_t inner,
                          int64_t total_cols) {
  constexpr int CG = (std::is_same<Tin, Tout>::value && sizeof(Tin) == 4) ? 2 : 1;
  if (CG > 1 && inner > 1 && inner % CG == 0)
    return launch_sym_m<Tin, Tout, TC, M, ODD, FWD, CG>(p, in, out, l, inner, total_cols);
  return launch_sym_m<Tin, Tout, TC, M, ODD, FWD, 1>(p, in, out, l, inner, total_cols);
}

template <typename Tin, typename Tout, typename TC, bool FWD>
stig_status launch_sym(stig_plan *p, const Tin *in, Tout *out, int l, int64_t inner,
                       int64_t total_cols) {
  if (total_cols >= ((int64_t)1 << 31)) return fail(STIG_EINVAL, "tensor too large for one launch");
  switch (p->n[l]) {
    case 32: return launch_sym_cg<Tin, Tout, TC, 16, false, FWD>(p, in, out, l, inner, total_cols);
    case 33: return launch_sym_cg<Tin, Tout, TC, 16, true, FWD>(p, in, out, l, inner, total_cols);
    case 64: return launch_sym_cg<Tin, Tout, TC, 32, false, FWD>(p, in, out, l, inner, total_cols);
    case 65: return launch_sym_cg<Tin, Tout, TC, 32, true, FWD>(p, in, out, l, inner, total_cols);
  }
  return fail(STIG_EINVAL, "no split kernel for this size");
}

// Fused x/y products with parity-split bases in both directions (n_x = n_y).
template <typename Tin, typename Tout, typename TC, int M, bool ODD, bool FWD>
stig_status launch_plane_sym_m(stig_plan *p, const Tin *in, Tout *out, int64_t planes,
                               int64_t in_stride, int64_t out_stride) {
  typedef typename Mfma<TC>::elem E;
  const int pi = PrecIdx<TC>::v;
  auto op = [&](DevBuf (&b)[3][3], int l) { return b[pi][l].template as<E>(); };
  const E *xE = FWD ? op(p->hFE, 0) : op(p->hBE, 0), *xO = FWD ? op(p->hFO, 0) : op(p->hBO, 0);
  const E *yE = FWD ? op(p->hFE, 1) : op(p->hBE, 1), *yO = FWD ? op(p->hFO, 1) : op(p->hBO, 1);
  const size_t lds = plane_sym_lds<TC, M, ODD, FWD>();
  auto kern = mode_gemm_plane_sym<Tin, Tout, TC, M, ODD, FWD>;
  static int per_cu = 0;  // per instantiation: resident blocks per CU
  if (per_cu == 0) {
    if (lds > 65536)
      HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
    int nb = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, (plane_sym_threads<TC, M>()), lds));
    per_cu = std::max(nb, 1);
  }
  int64_t grid = std::min<int64_t>(planes, (int64_t)per_cu * p->num_cu);
  int64_t per = (planes + grid - 1) / grid;
  grid = (planes + per - 1) / per;
  const int n = 2 * M + (ODD ? 1 : 0);
  ProfScope ps(p, STIG_K_PLANE_GEMM, (double)planes * n * n * (sizeof(Tin) + sizeof(Tout)));
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3((plane_sym_threads<TC, M>())), lds, p->stream, in, out,
                     xE, xO, yE, yO,
                     planes, in_stride, out_stride);
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

template <typename Tin, typename Tout, typename TC, bool FWD>
stig_status launch_plane_sym(stig_plan *p, const Tin *in, Tout *out, int64_t planes,
                             int64_t in_stride, int64_t out_stride) {
  if (planes < 1) return STIG_OK;
  switch (p->n[0]) {
    case 32: return launch_plane_sym_m<Tin, Tout, TC, 16, false, FWD>(p, in, out, planes, in_stride, out_stride);
    case 33: return launch_plane_sym_m<Tin, Tout, TC, 16, true, FWD>(p, in, out, planes, in_stride, out_stride);
    case 64: return launch_plane_sym_m<Tin, Tout, TC, 32, false, FWD>(p, in, out, planes, in_stride, out_stride);
    case 65: return launch_plane_sym_m<Tin, Tout, TC, 32, true, FWD>(p, in, out, planes, in_stride, out_stride);
  }
  return fail(STIG_EINVAL, "no split plane kernel for this size");
}

// Layout of the shifted time systems: ns spatial indices per time row (the
// row stride), lam[k] the shift of system k.
struct TimeView {
  int64_t ns;
  const double *lam;
};

template <typename Tio, typename TC, int P>
stig_status launch_time_p(stig_plan *p, const Tio *in, Tio *out, int nrhs, int transpose, TimeView tv) {
  const TC *wb, *mb;
  if (std::is_same<TC, double>::value) {
    wb = (const TC *)(transpose ? p->tWT64.p : p->tW64.p);
    mb = (const TC *)p->tM64.p;
  } else {
    wb = (const TC *)(transpose ? p->tWT32.p : p->tW32.p);
    mb = (const TC *)p->tM32.p;
  }
  int64_t work = tv.ns * nrhs;
  ProfScope ps(p, STIG_K_TIME_SOLVE, (double)work * p->nt * 2 * sizeof(Tio));
  hipLaunchKernelGGL((time_band_solve<Tio, TC, P>), dim3(grid_for(work, 256)), dim3(256), 0,
                     p->stream, in, out, tv.lam, wb, mb, (TC)p->gamma, (TC)p->nu,
                     p->nt, tv.ns, nrhs, p->tscr.as<TC>(), p->flag.as<int>());
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

template <typename Tio, typename TC, int NT, int P, int C>
stig_status launch_time_reg(stig_plan *p, const Tio *in, Tio *out, int nrhs, int transpose,
                            TimeView tv) {
  // FP64 keeps the forward-substituted values in the output buffer (registers
  // would spill); FP32 keeps them in registers.
  constexpr bool YREG = !std::is_same<TC, double>::value;
  TC *ysc = nullptr;
  if (!YREG) {
    if (std::is_same<Tio, TC>::value) ysc = (TC *)out;
    else {
      STIG_TRY(p->tscr.ensure((size_t)tv.ns * p->nt * nrhs * sizeof(TC)));
      ysc = p->tscr.as<TC>();
    }
  }
  const TC *wb, *mb;
  if (std::is_same<TC, double>::value) {
    wb = (const TC *)(transpose ? p->tWT64.p : p->tW64.p);
    mb = (const TC *)p->tM64.p;
  } else {
    wb = (const TC *)(transpose ? p->tWT32.p : p->tW32.p);
    mb = (const TC *)p->tM32.p;
  }
  int64_t work = tv.ns * nrhs;
  ProfScope ps(p, STIG_K_TIME_SOLVE, (double)work * p->nt * 2 * sizeof(Tio));
  hipLaunchKernelGGL((time_band_solve_reg<Tio, TC, NT, P, C, YREG>), dim3(grid_for(work, 256)),
                     dim3(256), 0, p->stream, in, out, tv.lam, wb, mb, (TC)p->gamma,
                     (TC)p->nu, tv.ns, nrhs, ysc, p->flag.as<int>());
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

template <typename Tio, typename TC, int NT, int P, int NSEG, bool YREC, int LROWS>
stig_status launch_time_rl(stig_plan *p, const Tio *in, Tio *out, int nrhs, int transpose,
                           TimeView tv) {
  // forward-substituted values (YREC false): in the output buffer when it has
  // the compute type, else in compute-type scratch
  TC *ysc = nullptr;
  if (!YREC) {
    if (std::is_same<Tio, TC>::value) ysc = (TC *)out;
    else {
      STIG_TRY(p->tscr.ensure((size_t)tv.ns * p->nt * nrhs * sizeof(TC)));
      ysc = p->tscr.as<TC>();
    }
  }
  const TC *wb, *mb;
  if (std::is_same<TC, double>::value) {
    wb = (const TC *)(transpose ? p->tWT64.p : p->tW64.p);
    mb = (const TC *)p->tM64.p;
  } else {
    wb = (const TC *)(transpose ? p->tWT32.p : p->tW32.p);
    mb = (const TC *)p->tM32.p;
  }
  int64_t work = tv.ns * nrhs;
  ProfScope ps(p, STIG_K_TIME_SOLVE, (double)work * p->nt * 2 * sizeof(Tio));
  const TC *rec = std::is_same<TC, double>::value ? (const TC *)p->tR64[transpose ? 1 : 0].p
                                                  : (const TC *)p->tR32[transpose ? 1 : 0].p;
  hipLaunchKernelGGL((time_band_solve_rl<Tio, TC, NT, P, NSEG, YREC, LROWS>), dim3(grid_for(work, 256)),
                     dim3(256), 0, p->stream, in, out, tv.lam, rec, wb, mb,
                     (TC)p->gamma, (TC)p->nu, tv.ns, nrhs, ysc, p->flag.as<int>());
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

template <typename Tio, typename TC, int NT, int P, int NSEG>
stig_status launch_time_rl2(stig_plan *p, const Tio *in, Tio *out, int nrhs, int transpose,
                            TimeView tv) {
  // rows of the input kept in LDS for the second read: 64 KB per block in FP64
  // (two blocks per CU), 30 KB in FP32 (five blocks per CU)
  constexpr int LR = std::is_same<TC, double>::value ? 32 : 30;
  constexpr int LROWS = LR < NT ? LR : NT;
  if (p->time_recompute)
    return launch_time_rl<Tio, TC, NT, P, NSEG, true, LROWS>(p, in, out, nrhs, transpose, tv);
  return launch_time_rl<Tio, TC, NT, P, NSEG, false, 0>(p, in, out, nrhs, transpose, tv);
}

// MFMA type of the arrowhead transforms: that of the apply's GEMMs, i.e. the
// storage type of the intermediates (FP64, FP32 or BF16).
template <typename Tio, typename TC> struct TimeArrowType { typedef Tio type; };

// Step 3 in the arrowhead form (time_kernel 4); n_t = 32 Q + 2.
template <typename Tio, typename TC, int Q>
stig_status launch_time_arrow_q(stig_plan *p, const Tio *in, Tio *out, int nrhs, int transpose,
                                TimeView tv) {
  typedef typename Mfma<TC>::elem E;
  typedef typename PlaneVal<TC>::vt VT;
  constexpr int NT = 32 * Q + 2;
  const int pi = PrecIdx<TC>::v;
  const VT *tabs = std::is_same<VT, double>::value ? (const VT *)p->aTab64[transpose ? 1 : 0].p
                                                   : (const VT *)p->aTab32[transpose ? 1 : 0].p;
  const size_t lds = ((size_t)2 * NT * lds_pad<TC>(NT) * sizeof(E) + 15) / 16 * 16 +
                     (size_t)(3 * NT + 1) * sizeof(VT);
  auto kern = time_arrow_solve<Tio, TC, Q>;
  static int per_cu = 0;  // per instantiation: resident blocks per CU
  if (per_cu == 0) {
    if (lds > 65536)
      HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
    int nb = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, ARROW_THREADS, lds));
    per_cu = std::max(nb, 1);
  }
  const int64_t cols = tv.ns * nrhs;
  if (cols >= ((int64_t)1 << 31)) return fail(STIG_EINVAL, "tensor too large for one launch");
  const int64_t nstrips = (cols + 15) / 16;
  const unsigned grid = (unsigned)std::min<int64_t>((nstrips + 3) / 4, (int64_t)per_cu * p->num_cu);
  ProfScope ps(p, STIG_K_TIME_SOLVE, (double)cols * NT * 2 * sizeof(Tio));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(ARROW_THREADS), lds, p->stream, in, out, tv.lam,
                     p->aTf[pi].as<E>(), p->aTb[pi].as<E>(), tabs, (VT)p->gamma, (VT)p->nu, tv.ns,
                     cols);
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

template <typename Tio, typename TC>
stig_status launch_time_arrow(stig_plan *p, const Tio *in, Tio *out, int nrhs, int transpose,
                              TimeView tv) {
  if (p->nt == 66) return launch_time_arrow_q<Tio, TC, 2>(p, in, out, nrhs, transpose, tv);
  if (p->nt == 34) return launch_time_arrow_q<Tio, TC, 1>(p, in, out, nrhs, transpose, tv);
  return fail(STIG_EINVAL, "no arrowhead kernel for this n_t");
}

template <typename Tio, typename TC>
stig_status launch_time_banded(stig_plan *p, const Tio *in, Tio *out, int nrhs, int transpose,
                               TimeView tv);

// Step 3 in the three-pass arrowhead form (any n_t): x~ = U^T r along t into
// the time scratch (compute type TC), the middle factor in place, s = U q.
// GM: MFMA type of the two products (that of the apply's mode products).
template <typename Tio, typename TC, typename GM>
stig_status launch_time_arrow_gen(stig_plan *p, const Tio *in, Tio *out, int nrhs, int transpose,
                                  TimeView tv) {
  typedef typename Mfma<GM>::elem E;
  const int pi = PrecIdx<GM>::v;
  const int64_t cols = tv.ns * nrhs;
  STIG_TRY(p->tscr.ensure((size_t)cols * p->nt * sizeof(TC)));
  TC *mid = p->tscr.as<TC>();
  STIG_TRY((launch_mode_gemm<Tio, TC, GM>(p, in, mid, p->aGf[pi].as<E>(), p->nt, tv.ns, cols,
                                          nullptr, nullptr)));
  const TC *tab = std::is_same<TC, double>::value
                      ? (const TC *)p->aGtab64[transpose ? 1 : 0].p
                      : (const TC *)p->aGtab32[transpose ? 1 : 0].p;
  {
    ProfScope ps(p, STIG_K_TIME_SOLVE, (double)cols * p->nt * 3 * sizeof(TC));
    // register form: 8 threads per system in FP64, 4 in FP32, with up to 16 or
    // up to 72 / 68 blocks of the middle factor (n_t up to 34, up to 146 / 138);
    // beyond, the two-pass form with 8 / 4 lanes per system.  At 16,900
    // systems of 131 modes: FP64 12.0 us (two-pass: 17.1), FP32 9.9 us (11.7;
    // 11.8 with 8 threads); at 32,768 of 33 modes (the short count): 5.6 and
    // 4.2 us (two-pass: 7.4 and 5.3; the long count there: 8.0 and 5.5)
    constexpr int G = sizeof(TC) == 8 ? 8 : 4, JM = sizeof(TC) == 8 ? 9 : 17;
    constexpr int JS = 16 / G;
    constexpr int CB = 256 / G;
    const int nb = (p->nt - 1 - p->arrow_nz) / 2;
    const int64_t blocks = (cols + CB - 1) / CB;
    if (nb >= 1 && nb <= G * JM && blocks > ((int64_t)1 << 30))
      return fail(STIG_EINVAL, "too many time systems");
    if (nb >= 1 && nb <= G * JS) {
      hipLaunchKernelGGL((time_arrow_middle_reg<TC, G, JS>), dim3((unsigned)blocks), dim3(256), 0,
                         p->stream, mid, tv.lam, tab, (TC)p->gamma, (TC)p->nu, p->nt,
                         p->arrow_nz, tv.ns, cols);
    } else if (nb >= 1 && nb <= G * JM) {
      hipLaunchKernelGGL((time_arrow_middle_reg<TC, G, JM>), dim3((unsigned)blocks), dim3(256), 0,
                         p->stream, mid, tv.lam, tab, (TC)p->gamma, (TC)p->nu, p->nt,
                         p->arrow_nz, tv.ns, cols);
    } else {
      constexpr int L = G;
      const int64_t waves = (cols + 64 / L - 1) / (64 / L);
      if (waves * 64 > ((int64_t)1 << 20) * 256) return fail(STIG_EINVAL, "too many time systems");
      hipLaunchKernelGGL((time_arrow_middle<TC, L>), dim3(grid_for(waves * 64, 256)), dim3(256), 0,
                         p->stream, mid, tv.lam, tab, (TC)p->gamma, (TC)p->nu, p->nt,
                         p->arrow_nz, tv.ns, cols);
    }
    HIP_TRY(hipGetLastError());
  }
  return launch_mode_gemm<TC, Tio, GM>(p, mid, out, p->aGb[pi].as<E>(), p->nt, tv.ns, cols,
                                       nullptr, nullptr);
}

// (n_t, p_t) shapes with register-resident time kernels
bool time_reg_shape(const stig_plan *p) {
  return (p->nt == 66 && p->pt == 3) || (p->nt == 50 && p->pt == 3) || (p->nt == 9 && p->pt == 2);
}
bool time_arrow_shape(const stig_plan *p) {
  return p->time_kernel == 4 && p->arrow_ok && (p->nt == 66 || p->nt == 34);
}
// Fewer shifted systems than this (N_s times the right-hand sides of a call)
// leave the banded elimination, one lane per system, short of waves (below one
// wavefront per SIMD at four waves each), and a long time axis makes each lane's
// chain long: the default (time kernel 0) then takes the arrowhead three-pass
// form, whose mode products parallelise over the time axis too, where its
// products have a compile-time streaming kernel (n_t = 131, 33; measured
// faster there: 0.20 vs 0.25 ms per FP64 apply on the 128-element annulus,
// 0.066 vs 0.073 ms on the extruded one, n_t = 33 with 32,768 systems, which
// took 0.115 ms while its products ran the runtime-n kernel).
constexpr int64_t ARROW_AUTO_SYSTEMS = 262144;
bool arrow_auto_nt(int nt) { return nt == 131 || nt == 33; }

// the three-pass arrowhead form: chosen (time kernel 4, other n_t than the
// fused kernel's) or taken by the default
bool time_arrow_gen(const stig_plan *p, int64_t systems) {
  if (!p->arrow_gen || time_arrow_shape(p)) return false;
  if (p->time_kernel == 4) return true;
  return p->time_kernel == 0 && !time_reg_shape(p) && arrow_auto_nt(p->nt) &&
         systems < ARROW_AUTO_SYSTEMS;
}

// Compute-type entries of scratch the time solve of `ns` systems per time row
// and nrhs right-hand sides needs, for the kernel launch_time picks: none for
// the arrowhead and register-resident kernels (they keep the forward-
// substituted values in registers, or in the output when it has the compute
// type), one tensor for the right-looking kernel that stores them in a
// different type, P + 1 tensors for the generic kernel.
int64_t time_scratch_elems(const stig_plan *p, int64_t ns, int nrhs, bool tc_f64, bool io_is_tc) {
  const int64_t sys = ns * p->nt * nrhs;
  if (time_arrow_shape(p)) return 0;
  if (time_arrow_gen(p, ns * nrhs)) return sys;  // x~ / q between the two products
  if (time_reg_shape(p)) {
    if (p->time_kernel == 1) return (tc_f64 && !io_is_tc) ? sys : 0;
    if (p->time_kernel == 0) return (p->time_recompute || io_is_tc) ? 0 : sys;
  }
  return (int64_t)(p->pt + 1) * sys;
}

template <typename Tio, typename TC>
stig_status launch_time(stig_plan *p, const Tio *in, Tio *out, int nrhs, int transpose,
                        TimeView tv) {
  if (time_arrow_shape(p))
    return launch_time_arrow<Tio, typename TimeArrowType<Tio, TC>::type>(p, in, out, nrhs,
                                                                         transpose, tv);
  if (time_arrow_gen(p, tv.ns * nrhs))
    return launch_time_arrow_gen<Tio, TC, typename TimeArrowType<Tio, TC>::type>(p, in, out, nrhs,
                                                                                transpose, tv);
  if (p->time_kernel == 4) return fail(STIG_ESTATE, "no arrowhead factorization of the time pencil");
  return launch_time_banded<Tio, TC>(p, in, out, nrhs, transpose, tv);
}

// The banded eliminations: register-resident kernels for the workload shapes
// (n_t, p_t) under time kernels 0 and 1, the generic kernel otherwise.
template <typename Tio, typename TC>
stig_status launch_time_banded(stig_plan *p, const Tio *in, Tio *out, int nrhs, int transpose,
                               TimeView tv) {
  if (p->time_kernel == 1) {
    if (p->nt == 66 && p->pt == 3) return launch_time_reg<Tio, TC, 66, 3, 11>(p, in, out, nrhs, transpose, tv);
    if (p->nt == 50 && p->pt == 3) return launch_time_reg<Tio, TC, 50, 3, 10>(p, in, out, nrhs, transpose, tv);
    if (p->nt == 9 && p->pt == 2) return launch_time_reg<Tio, TC, 9, 2, 3>(p, in, out, nrhs, transpose, tv);
  } else if (p->time_kernel == 0) {
    if (p->nt == 66 && p->pt == 3) return launch_time_rl2<Tio, TC, 66, 3, 7>(p, in, out, nrhs, transpose, tv);
    if (p->nt == 50 && p->pt == 3) return launch_time_rl2<Tio, TC, 50, 3, 6>(p, in, out, nrhs, transpose, tv);
    if (p->nt == 9 && p->pt == 2) return launch_time_rl2<Tio, TC, 9, 2, 2>(p, in, out, nrhs, transpose, tv);
  }
  STIG_TRY(p->tscr.ensure((size_t)(p->pt + 1) * tv.ns * p->nt * nrhs * sizeof(TC)));
  switch (p->pt) {
    case 1: return launch_time_p<Tio, TC, 1>(p, in, out, nrhs, transpose, tv);
    case 2: return launch_time_p<Tio, TC, 2>(p, in, out, nrhs, transpose, tv);
    case 3: return launch_time_p<Tio, TC, 3>(p, in, out, nrhs, transpose, tv);
    case 4: return launch_time_p<Tio, TC, 4>(p, in, out, nrhs, transpose, tv);
    case 5: return launch_time_p<Tio, TC, 5>(p, in, out, nrhs, transpose, tv);
  }
  return fail(STIG_EINVAL, "unsupported time degree");
}
template <typename Tio, typename TC>
stig_status launch_time(stig_plan *p, const Tio *in, Tio *out, int nrhs, int transpose) {
  return launch_time<Tio, TC>(p, in, out, nrhs, transpose, TimeView{p->Ns, p->lam.as<double>()});
}

// Shifts for a padded plane layout: lamp[z * ps + i] = lam[z * nn + i] for i < nn;
// padding entries repeat the first shift of their z index (valid systems whose
// results are never read).
__global__ void pad_shifts(const double *__restrict__ lam, double *__restrict__ lamp, int64_t nn,
                           int64_t ps, int64_t nz) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nz * ps;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = k / ps, i = k - z * ps;
    lamp[k] = lam[z * nn + (i < nn ? i : 0)];
  }
}

// The fused x/y passes of the apply run when modes 1 and 2 have the same size
// n <= PLANE_MAX_N and no diagonal scaling is set.
bool apply_fuses(const stig_plan *p) {
  return p->d >= 2 && p->n[0] == p->n[1] && p->n[0] <= PLANE_MAX_N && !p->has_dmh &&
         p->plane_fusion;
}
// x/y plane stride of the fused passes' intermediates for a storage size of
// ss bytes: n_1 n_2 rounded up to 128 bytes
int64_t padded_plane(const stig_plan *p, size_t ss) {
  const int64_t nn = (int64_t)p->n[0] * p->n[1], q = 128 / (int64_t)ss;
  return (nn + q - 1) / q * q;
}
// spatial indices per time row of the apply's intermediates
int64_t apply_row(const stig_plan *p, size_t ss) {
  if (!apply_fuses(p)) return p->Ns;
  return padded_plane(p, ss) * (p->d == 3 ? p->n[2] : 1);
}

// Typed access to the eigenvector copies of one precision.
template <typename TC> struct OpSet;
template <> struct OpSet<double> {
  static const double *U(stig_plan *p, int l) { return p->U64[l].as<double>(); }
  static const double *UT(stig_plan *p, int l) { return p->UT64[l].as<double>(); }
};
template <> struct OpSet<float> {
  static const float *U(stig_plan *p, int l) { return p->U32[l].as<float>(); }
  static const float *UT(stig_plan *p, int l) { return p->UT32[l].as<float>(); }
};
template <> struct OpSet<bf16> {
  static const uint16_t *U(stig_plan *p, int l) { return p->U16[l].as<uint16_t>(); }
  static const uint16_t *UT(stig_plan *p, int l) { return p->UT16[l].as<uint16_t>(); }
};

template <typename TC> struct TimeCompute { typedef float type; };
template <> struct TimeCompute<double> { typedef double type; };

// Steps 2-4 of Algorithm 1 with storage type S for the intermediates and compute
// type TC for the GEMMs.  Modes 1 and 2 go through the fused plane kernel when
// they have the same size n <= PLANE_MAX_N and no diagonal scaling is set;
// the other mode products use the half-size kernels where the basis is
// parity-split, else the dense ones.
template <typename S, typename TC>
stig_status run_apply(stig_plan *p, const double *r, double *s, int nrhs, int transpose) {
  const double *scale = p->has_dmh ? p->dmh.as<double>() : nullptr;
  const bool fuse = apply_fuses(p);
  auto use_sym = [&](int l) { return p->parity_split && p->split[l] && sym_size_ok(p->n[l]) && !scale; };
  // Intermediates between the fused plane passes: planes padded to a multiple
  // of 128 bytes, so that the strided passes (mode 3, time) read and write
  // whole cache lines.
  const int64_t nn = p->d >= 2 ? (int64_t)p->n[0] * p->n[1] : p->n[0];
  const int64_t ps = fuse ? padded_plane(p, sizeof(S)) : nn;
  const int64_t nz = p->d == 3 ? p->n[2] : 1;
  const int64_t ns = apply_row(p, sizeof(S));      // spatial indices per time row
  const int64_t tot = ns * p->nt * nrhs;           // entries of one intermediate tensor
  const int64_t planes = (int64_t)nrhs * p->nt * nz;
  STIG_TRY(p->s0.ensure(tot * sizeof(S)));
  STIG_TRY(p->s1.ensure(tot * sizeof(S)));
  STIG_TRY(p->tscr.ensure(time_scratch_elems(p, ns, nrhs, sizeof(typename TimeCompute<TC>::type) == 8,
                                             std::is_same<S, typename TimeCompute<TC>::type>::value) *
                          sizeof(typename TimeCompute<TC>::type)));
  S *buf[2] = {p->s0.as<S>(), p->s1.as<S>()};
  int cur = 0;
  TimeView tv{p->Ns, p->lam.as<double>()};
  if (ps != nn) {
    const int li = sizeof(S) == 8 ? 0 : sizeof(S) == 4 ? 1 : 2;
    if (p->lamp_ps[li] != ps) return fail(STIG_ESTATE, "padded shift table missing");
    tv = TimeView{ns, p->lamp[li].as<double>()};
  }
  // one mode product, forward (U_l^T) or backward (U_l)
  auto mode = [&](auto tin, auto tout, int l, bool fwd, int64_t inner) -> stig_status {
    typedef typename std::remove_const<typename std::remove_pointer<decltype(tin)>::type>::type Ti;
    typedef typename std::remove_pointer<decltype(tout)>::type To;
    const int64_t cols = tot / p->n[l];
    if (use_sym(l))
      return fwd ? launch_sym<Ti, To, TC, true>(p, tin, tout, l, inner, cols)
                 : launch_sym<Ti, To, TC, false>(p, tin, tout, l, inner, cols);
    const bool first = fwd && l == p->d - 1, last = !fwd && l == p->d - 1;
    return launch_mode_gemm<Ti, To, TC>(p, tin, tout, fwd ? OpSet<TC>::UT(p, l) : OpSet<TC>::U(p, l),
                                        p->n[l], inner, cols, first ? scale : nullptr,
                                        last ? scale : nullptr);
  };
  if (scale) {
    // D^{-1/2} on both sides: the products run from the slowest spatial axis
    // to the fastest and back, so the two scaled ones (first and last) stride
    // over whole rows (coalesced loads of values and factors) instead of
    // running along the contiguous axis.  The mode products commute.
    int64_t in_l[3] = {1, 1, 1};
    for (int l = 1; l < p->d; ++l) in_l[l] = in_l[l - 1] * p->n[l - 1];
    for (int l = p->d - 1; l >= 0; --l) {
      if (l == p->d - 1) STIG_TRY(mode(r, buf[cur], l, true, in_l[l]));
      else STIG_TRY(mode((const S *)buf[cur ^ 1], buf[cur], l, true, in_l[l]));
      cur ^= 1;
    }
    STIG_TRY((launch_time<S, typename TimeCompute<TC>::type>(p, buf[cur ^ 1], buf[cur], nrhs,
                                                              transpose, tv)));
    cur ^= 1;
    for (int l = 0; l < p->d; ++l) {
      if (l == p->d - 1) STIG_TRY(mode((const S *)buf[cur ^ 1], s, l, false, in_l[l]));
      else {
        STIG_TRY(mode((const S *)buf[cur ^ 1], buf[cur], l, false, in_l[l]));
        cur ^= 1;
      }
    }
    return STIG_OK;
  }
  // step 2: forward spatial transform, X x_l U_l^T for l = 1..d
  const bool fuse_sym = fuse && use_sym(0) && use_sym(1);
  int64_t inner = 1;
  int l0 = 0;
  if (fuse) {
    if (fuse_sym)
      STIG_TRY((launch_plane_sym<double, S, TC, true>(p, r, buf[cur], planes, nn, ps)));
    else
      STIG_TRY((launch_plane<double, S, TC>(p, r, buf[cur], OpSet<TC>::UT(p, 0), OpSet<TC>::UT(p, 1),
                                             p->n[0], planes, nn, ps)));
    cur ^= 1;
    inner = ps;
    l0 = 2;
  }
  for (int l = l0; l < p->d; ++l) {
    if (l == 0) STIG_TRY(mode(r, buf[cur], l, true, inner));
    else STIG_TRY(mode((const S *)buf[cur ^ 1], buf[cur], l, true, inner));
    cur ^= 1;
    inner *= p->n[l];
  }
  // step 3: shifted time systems
  STIG_TRY((launch_time<S, typename TimeCompute<TC>::type>(p, buf[cur ^ 1], buf[cur], nrhs,
                                                            transpose, tv)));
  cur ^= 1;
  // step 4: back transform, x_l U_l for l = d..1
  for (int l = p->d - 1; l >= l0; --l) {
    inner /= p->n[l];
    if (l == 0) STIG_TRY(mode((const S *)buf[cur ^ 1], s, l, false, inner));
    else {
      STIG_TRY(mode((const S *)buf[cur ^ 1], buf[cur], l, false, inner));
      cur ^= 1;
    }
  }
  if (fuse) {
    if (fuse_sym)
      STIG_TRY((launch_plane_sym<S, double, TC, false>(p, buf[cur ^ 1], s, planes, ps, nn)));
    else
      STIG_TRY((launch_plane<S, double, TC>(p, buf[cur ^ 1], s, OpSet<TC>::U(p, 0), OpSet<TC>::U(p, 1),
                                             p->n[0], planes, ps, nn)));
  }
  return STIG_OK;
}

// --------------------------------------------------------------- band passes

// Chunks along a strided axis of length n with `cols` columns: split only when
// the columns alone give fewer than 4096 wavefronts, into chunks of at least
// 2 (2P + 1) entries (the 2P halo entries are read twice).
int axis_chunks(int64_t cols, int n, int P) {
  const int64_t waves = (cols + 63) / 64;
  if (waves >= 4096) return 1;
  const int want = (int)((4096 + waves - 1) / waves);
  const int most = std::max(1, n / (2 * (2 * P + 1)));
  const int ch = std::min(want, most);
  const int jc = (n + ch - 1) / ch;
  return (n + jc - 1) / jc;
}

template <int P>
stig_status band_pass_p(stig_plan *p, const double *in1, const double *in2, double *out1,
                        double *out2, const double *Ba, const double *Bb, const double *Bc, int n,
                        int64_t inner, int64_t total) {
  ProfScope ps(p, STIG_K_BAND_PASS,
               (double)total * 8 * ((in1 ? 1 : 0) + (in2 ? 1 : 0) + (out1 ? 1 : 0) + (out2 ? 1 : 0)));
  if (inner == 1) {
    hipLaunchKernelGGL(band_pass_contig<P>, dim3(grid_for(total, 256)), dim3(256), 0, p->stream,
                       in1, in2, out1, out2, Ba, Bb, Bc, n, total);
  } else {
    const int64_t cols = total / n;
    const int ch = axis_chunks(cols, n, P), jc = (n + ch - 1) / ch;
    if (ch > 1)
      hipLaunchKernelGGL((band_pass_strided<P, true>), dim3(grid_for(cols, 256), ch), dim3(256), 0,
                         p->stream, in1, in2, out1, out2, Ba, Bb, Bc, n, inner, cols, jc);
    else
      hipLaunchKernelGGL((band_pass_strided<P, false>), dim3(grid_for(cols, 256)), dim3(256), 0,
                         p->stream, in1, in2, out1, out2, Ba, Bb, Bc, n, inner, cols, n);
  }
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

stig_status band_pass(stig_plan *p, int P, const double *in1, const double *in2, double *out1,
                      double *out2, const double *Ba, const double *Bb, const double *Bc, int n,
                      int64_t inner, int64_t total) {
  switch (P) {
    case 1: return band_pass_p<1>(p, in1, in2, out1, out2, Ba, Bb, Bc, n, inner, total);
    case 2: return band_pass_p<2>(p, in1, in2, out1, out2, Ba, Bb, Bc, n, inner, total);
    case 3: return band_pass_p<3>(p, in1, in2, out1, out2, Ba, Bb, Bc, n, inner, total);
    case 4: return band_pass_p<4>(p, in1, in2, out1, out2, Ba, Bb, Bc, n, inner, total);
    case 5: return band_pass_p<5>(p, in1, in2, out1, out2, Ba, Bb, Bc, n, inner, total);
  }
  return fail(STIG_EINVAL, "unsupported degree");
}

// Spatial passes over a tensor of `tot` entries whose spatial part is the
// fastest d axes.  mass_only: out_a = x (x) M_1 .. M_d.  Otherwise a = mass
// chain, b = stiffness sum; returns pointers to the final (a, b).
stig_status spatial_chain(stig_plan *p, const double *x, int64_t tot, bool with_stiff,
                          const double **a_out, const double **b_out, Span *bufs[4]) {
  const double *a = x, *b = nullptr;
  int slot = 0;
  int64_t inner = 1;
  for (int l = 0; l < p->d; ++l) {
    double *oa = bufs[slot]->as<double>();
    double *ob = with_stiff ? bufs[slot + 1]->as<double>() : nullptr;
    STIG_TRY(band_pass(p, p->ps, a, b, oa, ob, p->sM[l].as<double>(), p->sM[l].as<double>(),
                       p->sK[l].as<double>(), p->n[l], inner, tot));
    a = oa;
    b = ob;
    slot ^= 2;
    inner *= p->n[l];
  }
  *a_out = a;
  *b_out = b;
  return STIG_OK;
}

template <int P>
stig_status launch_stencil_p(stig_plan *p, const double *x, double *a, double *b, int nrhs) {
  const int nx = p->n[0], ny = p->n[1], nz = p->d == 3 ? p->n[2] : 1;
  // R rows per block (R >= 2P: each thread holds two of the R + 2P window rows)
  const int rmax = std::max(2 * P, std::min(8, STENCIL_THREADS / nx));
  const int R = std::max(2 * P, (ny + (ny + rmax - 1) / rmax - 1) / ((ny + rmax - 1) / rmax));
  if (R * nx > STENCIL_THREADS) return fail(STIG_EINVAL, "plane too wide for the stencil pass");
  const int threads = (R * nx + 63) / 64 * 64;
  // z chunks of at most STENCIL_ZC planes per block, of balanced lengths
  const int nch = (nz + STENCIL_ZC - 1) / STENCIL_ZC, ZC = (nz + nch - 1) / nch;
  const size_t lds = (size_t)2 * (R + 2 * P) * (2 * nx + nx + 2 * P) * sizeof(double);
  if (lds > GEMM_LDS_LIMIT) return fail(STIG_EINVAL, "plane too wide for the stencil pass");
  auto kern = spatial_stencil<P>;
  static size_t configured = 0;
  if (lds > 65536 && lds > configured) {
    HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    configured = lds;
  }
  const int64_t slices = (int64_t)p->nt * nrhs;
  const int64_t blocks = slices * ((ny + R - 1) / R) * ((nz + ZC - 1) / ZC);
  // third direction: the z bands, or identity / zero for d = 2
  const double *M2 = p->d == 3 ? p->sM[2].as<double>() : p->sId.as<double>();
  const double *K2 = p->d == 3 ? p->sK[2].as<double>() : p->sZero.as<double>();
  ProfScope ps(p, STIG_K_BAND_PASS, (double)p->N * nrhs * 24);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(threads), lds, p->stream, x, a, b,
                     p->sM[0].as<double>(), p->sK[0].as<double>(), p->sM[1].as<double>(),
                     p->sK[1].as<double>(), M2, K2, nx, ny, nz, R, ZC, slices);
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

// The stencil pass holds R >= 2P full rows of x per block of at most
// STENCIL_THREADS threads; wider planes take the per-axis passes.
bool stencil_fits(const stig_plan *p) {
  return p->d >= 2 && p->ps >= 1 && p->ps <= 5 &&
         std::max(2 * p->ps, std::min(8, STENCIL_THREADS / p->n[0])) * p->n[0] <= STENCIL_THREADS;
}

stig_status launch_stencil(stig_plan *p, const double *x, double *a, double *b, int nrhs) {
  if (p->d == 2 && (p->sId.bytes == 0 || p->sZero.bytes == 0))
    return fail(STIG_ESTATE, "stencil bands missing");
  switch (p->ps) {
    case 1: return launch_stencil_p<1>(p, x, a, b, nrhs);
    case 2: return launch_stencil_p<2>(p, x, a, b, nrhs);
    case 3: return launch_stencil_p<3>(p, x, a, b, nrhs);
    case 4: return launch_stencil_p<4>(p, x, a, b, nrhs);
    case 5: return launch_stencil_p<5>(p, x, a, b, nrhs);
  }
  return fail(STIG_EINVAL, "unsupported degree");
}

// a = M_s x, b = K_s x per slice with the sparse spatial factors (transposed
// factors for the adjoint product)
stig_status launch_spatial_ell(stig_plan *p, const double *x, double *a, double *b, int nrhs,
                               int transpose) {
  constexpr int TT = 8;
  const int q = transpose ? 1 : 0;
  const int64_t slices = (int64_t)p->nt * nrhs;
  const int64_t chunks = (slices + TT - 1) / TT, rblocks = (p->Ns + 255) / 256;
  if (chunks * rblocks >= ((int64_t)1 << 31))
    return fail(STIG_EINVAL, "too many blocks for the sparse spatial pass");
  ProfScope ps(p, STIG_K_CSR,
               (double)p->N * nrhs * 24 + (double)p->ell_w[q] * p->Ns * (p->ell_dia[q] ? 16 : 20));
  // diagonal form: offsets in runs of consecutive values (one window load per
  // run and wavefront), else a narrow column span staged in LDS (4 slices per
  // block), else plain gathers
  constexpr int TL = 4;
  const int64_t span = 256 + (int64_t)p->ell_omax[q] - p->ell_omin[q];
  if (p->ell_dia[q] && 2 * p->ell_nruns[q] <= p->ell_w[q]) {
    hipLaunchKernelGGL((spatial_dia_runs<TT>), dim3((unsigned)(chunks * rblocks)), dim3(256), 0,
                       p->stream, x, a, b, p->ellR[q].as<int32_t>(), p->ellM[q].as<double>(),
                       p->ellK[q].as<double>(), p->ell_nruns[q], p->Ns, slices, (int)chunks);
  } else if (p->ell_dia[q] && span * TL * (int64_t)sizeof(double) <= 48 * 1024) {
    const int64_t lch = (slices + TL - 1) / TL;
    if (lch * rblocks >= ((int64_t)1 << 31))
      return fail(STIG_EINVAL, "too many blocks for the sparse spatial pass");
    hipLaunchKernelGGL((spatial_dia_lds<TL, ELL_KU>), dim3((unsigned)(lch * rblocks)), dim3(256),
                       (size_t)(span * TL * sizeof(double)), p->stream, x, a, b,
                       p->ellC[q].as<int32_t>(), p->ellM[q].as<double>(), p->ellK[q].as<double>(),
                       p->ell_w[q], p->Ns, slices, (int)lch, p->ell_omin[q], (int)span);
  } else if (p->ell_dia[q])
    hipLaunchKernelGGL((spatial_dia_pair<TT, ELL_KU>), dim3((unsigned)(chunks * rblocks)),
                       dim3(256), 0, p->stream, x, a, b, p->ellC[q].as<int32_t>(),
                       p->ellM[q].as<double>(), p->ellK[q].as<double>(), p->ell_w[q], p->Ns,
                       slices, (int)chunks);
  else
    hipLaunchKernelGGL((spatial_ell_pair<TT, ELL_KU>), dim3((unsigned)(chunks * rblocks)),
                       dim3(256), 0, p->stream, x, a, b, p->ellC[q].as<int32_t>(),
                       p->ellM[q].as<double>(), p->ellK[q].as<double>(), p->ell_w[q], p->Ns,
                       slices, (int)chunks);
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

// spatial part of the banded matvec: a = x (x) M_s, b = x (x) K_s (all d axes),
// from the sparse spatial factors when they are set
stig_status matvec_spatial(stig_plan *p, const double *x, int nrhs, int transpose,
                           const double **a, const double **b) {
  const int64_t tot = p->N * nrhs;
  if (p->ell_w[0] > 0) {
    STIG_TRY(p->m0.ensure(tot * sizeof(double)));
    STIG_TRY(p->m1.ensure(tot * sizeof(double)));
    STIG_TRY(launch_spatial_ell(p, x, p->m0.as<double>(), p->m1.as<double>(), nrhs, transpose));
    *a = p->m0.as<double>();
    *b = p->m1.as<double>();
    return STIG_OK;
  }
  if (stencil_fits(p)) {
    // spatial part in one stencil pass per (rhs, t) slice
    STIG_TRY(p->m0.ensure(tot * sizeof(double)));
    STIG_TRY(p->m1.ensure(tot * sizeof(double)));
    STIG_TRY(launch_stencil(p, x, p->m0.as<double>(), p->m1.as<double>(), nrhs));
    *a = p->m0.as<double>();
    *b = p->m1.as<double>();
    return STIG_OK;
  }
  Span *bufs[4] = {&p->m0, &p->m1, &p->m2, &p->m3};
  for (auto *bb : bufs) STIG_TRY(bb->ensure(tot * sizeof(double)));
  return spatial_chain(p, x, tot, true, a, b, bufs);
}

// blocks along the spatial columns and chunks along t of the fused residual pass
void residual_grid(const stig_plan *p, int64_t *blocks, int *chunks) {
  *blocks = (p->Ns + 255) / 256;
  *chunks = axis_chunks(p->Ns, p->nt, p->pt);
}

template <int P>
stig_status launch_time_residual(stig_plan *p, const double *a, const double *b, const double *f,
                                 double *r, int transpose, double *partial, int64_t blocks,
                                 int chunks) {
  const double *gW = transpose ? p->tgWT.as<double>() : p->tgW.as<double>();
  const int jc = (p->nt + chunks - 1) / chunks;
  ProfScope ps(p, STIG_K_BAND_PASS, (double)p->N * 8 * 4);
  if (chunks > 1)
    hipLaunchKernelGGL((time_pass_residual<P, true>), dim3((unsigned)blocks, chunks), dim3(256), 0,
                       p->stream, a, b, f, r, p->tnM.as<double>(), gW, p->nt, p->Ns, p->Ns, jc,
                       partial);
  else
    hipLaunchKernelGGL((time_pass_residual<P, false>), dim3((unsigned)blocks), dim3(256), 0,
                       p->stream, a, b, f, r, p->tnM.as<double>(), gW, p->nt, p->Ns, p->Ns, jc,
                       partial);
  HIP_TRY(hipGetLastError());
  return STIG_OK;
}

// r = f - A x for one right-hand side on the banded (Kronecker) form, with the
// last pass fused with the residual and this grid's partial sums of r . r in
// partial[0 .. *nparts).  Returns STIG_EINVAL (nothing launched) on the CSR form.
stig_status run_residual_banded(stig_plan *p, const double *f, const double *x, double *r,
                                int transpose, double *partial, int64_t partial_cap,
                                int64_t *nparts) {
  if (p->csr_rowptr) return fail(STIG_EINVAL, "no banded form");
  int64_t blocks;
  int ch;
  residual_grid(p, &blocks, &ch);
  if (blocks * ch > partial_cap) return fail(STIG_EINVAL, "residual partials do not fit");
  const double *a, *b;
  STIG_TRY(matvec_spatial(p, x, 1, transpose, &a, &b));
  *nparts = blocks * ch;
  switch (p->pt) {
    case 1: return launch_time_residual<1>(p, a, b, f, r, transpose, partial, blocks, ch);
    case 2: return launch_time_residual<2>(p, a, b, f, r, transpose, partial, blocks, ch);
    case 3: return launch_time_residual<3>(p, a, b, f, r, transpose, partial, blocks, ch);
    case 4: return launch_time_residual<4>(p, a, b, f, r, transpose, partial, blocks, ch);
    case 5: return launch_time_residual<5>(p, a, b, f, r, transpose, partial, blocks, ch);
  }
  return fail(STIG_EINVAL, "unsupported degree");
}

stig_status run_matvec(stig_plan *p, const double *x, double *y, int nrhs, int transpose) {
  const int64_t tot = p->N * nrhs;
  if (p->csr_rowptr) {
    if (transpose) return fail(STIG_EINVAL, "transposed product not supported on the CSR form");
    for (int r = 0; r < nrhs; ++r) {
      ProfScope ps(p, STIG_K_CSR, (double)p->csr_nnz * 12 + (double)p->N * 24);
      hipLaunchKernelGGL(csr_spmv, dim3(grid_for(p->N * 64, 256)), dim3(256), 0, p->stream,
                         p->csr_rowptr, p->csr_col, p->csr_val, x + r * p->N, y + r * p->N, p->N);
      HIP_TRY(hipGetLastError());
    }
    return STIG_OK;
  }
  const double *a, *b;
  STIG_TRY(matvec_spatial(p, x, nrhs, transpose, &a, &b));
  // time pass: y = nu (b x_t M_t) + gamma (a x_t W_t)
  const double *gW = transpose ? p->tgWT.as<double>() : p->tgW.as<double>();
  STIG_TRY(band_pass(p, p->pt, a, b, nullptr, y, nullptr, p->tnM.as<double>(), gW, p->nt, p->Ns,
                     tot));
  return STIG_OK;
}

// --------------------------------------------------------------- workspace

// What one call uses the operator part of the workspace for.
enum { WS_APPLY = 1, WS_MATVEC = 2, WS_MASS = 4, WS_LIFT = 8, WS_ALL = 15 };

inline size_t ws_round(size_t b) { return (b + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }
inline size_t store_size(stig_prec prec) { return prec == STIG_FP64 ? 8 : prec == STIG_FP32 ? 4 : 2; }
inline size_t time_size(stig_prec prec) { return prec == STIG_FP64 ? 8 : 4; }

// double intermediates of the spatial part of one matvec: the sparse spatial
// factors and the fused stencil write a and b, the per-axis passes ping-pong
// two pairs; the CSR form needs none
int matvec_bufs(const stig_plan *p) {
  if (p->csr_rowptr) return 0;
  return (p->ell_w[0] > 0 || stencil_fits(p)) ? 2 : 4;
}

// Byte offsets of the views of one call.  The operator views (apply, matvec,
// mass, lifting) all start at offset 0: one call runs one of them at a time.
// The Krylov bases follow them.
struct WsLayout {
  size_t s0 = 0, s1 = 0, tscr = 0;        // apply: two intermediates, time scratch
  size_t m = 0;                           // one matvec / mass intermediate
  size_t lm = 0, lw = 0;                  // lifting: one spatial intermediate, weights
  size_t op = 0;                          // operator part
  size_t v = 0, z = 0, vec = 0;           // Krylov: V, Z and AZ, one vector block (tmp)
  size_t total = 0;
};

WsLayout ws_layout(const stig_plan *p, int nrhs, stig_prec prec, int what, int nb, int m) {
  WsLayout L;
  const size_t ss = store_size(prec), ts = time_size(prec);
  if (what & WS_APPLY) {
    const int64_t ns = apply_row(p, ss);
    L.s0 = L.s1 = ws_round((size_t)ns * p->nt * nrhs * ss);
    L.tscr = ws_round((size_t)time_scratch_elems(p, ns, nrhs, ts == 8, ss == ts) * ts);
    L.op = std::max(L.op, L.s0 + L.s1 + L.tscr);
  }
  L.m = ws_round((size_t)p->N * nrhs * sizeof(double));
  if (what & WS_MATVEC) L.op = std::max(L.op, (size_t)matvec_bufs(p) * L.m);
  if (what & WS_MASS) L.op = std::max(L.op, 2 * L.m);
  if (what & WS_LIFT) {
    L.lm = ws_round((size_t)p->Ns * nrhs * sizeof(double));
    L.lw = ws_round((size_t)2 * p->nt * sizeof(double));
    L.op = std::max(L.op, 6 * L.lm + L.lw);
  }
  if (nb > 0) {
    L.vec = ws_round((size_t)nb * p->N * sizeof(double));
    L.v = ws_round((size_t)(m + 1) * nb * p->N * sizeof(double));
    L.z = ws_round((size_t)m * nb * p->N * sizeof(double));
  }
  L.total = L.op + L.v + 2 * L.z + L.vec;
  return L;
}

// Lay the views of one call over the caller's workspace.
void lay_views(stig_plan *p, const WsLayout &L, char *b, int what, int nb);

stig_status bind_workspace(stig_plan *p, int nrhs, stig_prec prec, int what, int nb = 0,
                           int m = 0) {
  const WsLayout L = ws_layout(p, nrhs, prec, what, nb, m);
  if (L.total > 0 && !p->ws)
    return fail(STIG_ESTATE, "no workspace: give one of stig_workspace_bytes bytes to "
                             "stig_set_workspace (" + std::to_string(L.total) + " bytes needed)");
  if (L.total > p->ws_bytes)
    return fail(STIG_EINVAL, "workspace of " + std::to_string(p->ws_bytes) + " bytes, " +
                                 std::to_string(L.total) + " needed (stig_workspace_bytes)");
  lay_views(p, L, p->ws, what, nb);
  return STIG_OK;
}

// The views of layout L over the memory at b.
void lay_views(stig_plan *p, const WsLayout &L, char *b, int what, int nb) {
  p->s0.set(b, 0, L.s0);
  p->s1.set(b, L.s0, L.s1);
  p->tscr.set(b, L.s0 + L.s1, L.tscr);
  if (what & WS_LIFT) {
    p->m0.set(b, 0, L.lm);
    p->m1.set(b, L.lm, L.lm);
    p->m2.set(b, 2 * L.lm, L.lm);
    p->m3.set(b, 3 * L.lm, L.lm);
    p->lift0.set(b, 4 * L.lm, L.lm);
    p->lift1.set(b, 5 * L.lm, L.lm);
    p->liftw.set(b, 6 * L.lm, L.lw);
  } else {
    const int nm = (what & WS_MATVEC) ? std::max(matvec_bufs(p), (what & WS_MASS) ? 2 : 0)
                                      : ((what & WS_MASS) ? 2 : 0);
    Span *ms[4] = {&p->m0, &p->m1, &p->m2, &p->m3};
    for (int i = 0; i < 4; ++i) ms[i]->set(i < nm ? b : nullptr, (size_t)i * L.m, L.m);
    p->lift0 = p->lift1 = p->liftw = Span{};
  }
  size_t o = L.op;
  p->V.set(nb ? b : nullptr, o, L.v);
  o += L.v;
  p->Z.set(nb ? b : nullptr, o, L.z);
  o += L.z;
  p->AZ.set(nb ? b : nullptr, o, L.z);
  o += L.z;
  p->tmp.set(nb ? b : nullptr, o, L.vec);
}

// ------------------------------------------- allocation-free apply (static scratch)

// Device scratch of the allocation-free apply, one copy per GPU, held until the
// process ends.  Host code must not pass `scratch` itself to a kernel (that is a
// host-side stand-in): it uses the device address from hipGetSymbolAddress,
// looked up once per device.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)128 << 20;
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];
std::mutex g_scratch_mutex;
void *g_scratch_ptr[MAX_DEVICES] = {nullptr};

// Device address of this device's scratch array (looked up on first use).
stig_status static_scratch(int dev, char **out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(STIG_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(STIG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<char *>(g_scratch_ptr[dev]);
  return STIG_OK;
}

// ------------------------------------------------------------------- GMRES

struct Krylov {
  stig_plan *p;
  int64_t ld = 0;   // distance between consecutive basis vectors (0: N)
  int64_t off = 0;  // offset of this right-hand side's slot regions in the small buffer
  double *partial() { return p->partial.as<double>(); }
  double *small() { return p->small.as<double>(); }
  int64_t ldv() const { return ld ? ld : p->N; }
  // out[0..KRY_MAXV) of the small buffer region `slot`
  double *slot(int k) { return small() + off + k * KRY_MAXV; }

  // reduce the per-block partial sums into slot region `out_slot`
  stig_status reduce(int out_slot) {
    hipLaunchKernelGGL(reduce_partials, dim3(KRY_MAXV), dim3(KRY_BLOCK), 0, p->stream, partial(),
                       KRY_GRID, slot(out_slot));
    HIP_TRY(hipGetLastError());
    return STIG_OK;
  }
  template <int NV>
  void launch_dots(const double *V, int nv, const double *w, int with_norm) {
    hipLaunchKernelGGL(krylov_dots<NV>, dim3(KRY_GRID), dim3(KRY_BLOCK), 0, p->stream, V, ldv(),
                       nv, w, p->N, with_norm, partial());
  }
  template <int NV>
  void launch_update(const double *V, int nv, const double *coef, double sign, const double *w,
                     double *dst, double scale, int with_dots) {
    hipLaunchKernelGGL(krylov_update<NV>, dim3(KRY_GRID), dim3(KRY_BLOCK), 0, p->stream, V, ldv(),
                       nv, coef, sign, w, dst, scale, p->N, with_dots, partial());
  }
  stig_status dots(const double *V, int nv, const double *w, int with_norm, int out_slot) {
    if (nv > KRY_MAXV - 1) return fail(STIG_EINVAL, "too many basis vectors");
    ProfScope ps(p, STIG_K_KRYLOV, (double)(nv + 1) * p->N * 8);
    if (nv <= 4) launch_dots<4>(V, nv, w, with_norm);
    else if (nv <= 8) launch_dots<8>(V, nv, w, with_norm);
    else if (nv <= 12) launch_dots<12>(V, nv, w, with_norm);
    else if (nv <= 16) launch_dots<16>(V, nv, w, with_norm);
    else if (nv <= 24) launch_dots<24>(V, nv, w, with_norm);
    else launch_dots<32>(V, nv, w, with_norm);
    HIP_TRY(hipGetLastError());
    return reduce(out_slot);
  }
  // dst (default w) = scale * (w + sign * V coef); with_dots: V^T w_new and
  // ||w_new||^2 into slot region out_slot
  // (w == nullptr with dst given: w reads as zero)
  stig_status update(const double *V, int nv, const double *coef, double sign, double *w,
                     int with_dots, int out_slot, double *dst = nullptr, double scale = 1.0) {
    if (nv > KRY_MAXV - 1) return fail(STIG_EINVAL, "too many basis vectors");
    if (!dst) dst = w;
    if (!dst) return fail(STIG_EINVAL, "update without a destination");
    ProfScope ps(p, STIG_K_KRYLOV, (double)(nv + 2) * p->N * 8);
    if (nv <= 4) launch_update<4>(V, nv, coef, sign, w, dst, scale, with_dots);
    else if (nv <= 8) launch_update<8>(V, nv, coef, sign, w, dst, scale, with_dots);
    else if (nv <= 12) launch_update<12>(V, nv, coef, sign, w, dst, scale, with_dots);
    else if (nv <= 16) launch_update<16>(V, nv, coef, sign, w, dst, scale, with_dots);
    else if (nv <= 24) launch_update<24>(V, nv, coef, sign, w, dst, scale, with_dots);
    else launch_update<32>(V, nv, coef, sign, w, dst, scale, with_dots);
    HIP_TRY(hipGetLastError());
    return with_dots ? reduce(out_slot) : STIG_OK;
  }
  // one pass of delayed re-orthogonalisation: Q^T u, Q^T w (nq basis vectors
  // Q_i = Q + i ldv), u.u, u.w, w.w into slot regions 0, 1 and the first
  // three entries of 2 (no synchronisation)
  template <int NV>
  void launch_dots2(const double *Q, int nq, const double *u, const double *w) {
    hipLaunchKernelGGL(krylov_dots2<NV>, dim3(KRY_GRID), dim3(KRY_BLOCK), 0, p->stream, Q, ldv(),
                       nq, u, w, p->N, partial());
  }
  stig_status dots2(const double *Q, int nq, const double *u, const double *w) {
    if (nq > KRY_MAXV - 1) return fail(STIG_EINVAL, "too many basis vectors");
    ProfScope ps(p, STIG_K_KRYLOV, (double)(nq + 2) * p->N * 8);
    if (nq == 0) launch_dots2<0>(Q, nq, u, w);
    else if (nq <= 4) launch_dots2<4>(Q, nq, u, w);
    else if (nq <= 8) launch_dots2<8>(Q, nq, u, w);
    else if (nq <= 12) launch_dots2<12>(Q, nq, u, w);
    else if (nq <= 16) launch_dots2<16>(Q, nq, u, w);
    else if (nq <= 24) launch_dots2<24>(Q, nq, u, w);
    else launch_dots2<32>(Q, nq, u, w);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(reduce_partials, dim3(KRY_D2), dim3(KRY_BLOCK), 0, p->stream, partial(),
                       KRY_GRID, slot(0));
    HIP_TRY(hipGetLastError());
    return STIG_OK;
  }
  // the second pass: v = (u - Q s) rv over u (write_v), x = (w - a u - Q (t - a s)) rx;
  // with_norm: x.x into slot region 3, entry KRY_MAXV-1 (no synchronisation)
  template <int NV>
  void launch_update2(const double *Q, int nq, const double *sv, const double *tv, double *u,
                      const double *w, double *x, double a, double rv, double rx, int write_v,
                      int with_norm) {
    hipLaunchKernelGGL(krylov_update2<NV>, dim3(KRY_GRID), dim3(KRY_BLOCK), 0, p->stream, Q, ldv(),
                       nq, sv, tv, u, w, x, a, rv, rx, p->N, write_v, with_norm, partial());
  }
  stig_status update2(const double *Q, int nq, const double *sv, const double *tv, double *u,
                      const double *w, double *x, double a, double rv, double rx, int write_v,
                      int with_norm) {
    if (nq > KRY_MAXV - 1) return fail(STIG_EINVAL, "too many basis vectors");
    ProfScope ps(p, STIG_K_KRYLOV, (double)(nq + 3 + write_v) * p->N * 8);
    if (nq == 0) launch_update2<0>(Q, nq, sv, tv, u, w, x, a, rv, rx, write_v, with_norm);
    else if (nq <= 4) launch_update2<4>(Q, nq, sv, tv, u, w, x, a, rv, rx, write_v, with_norm);
    else if (nq <= 8) launch_update2<8>(Q, nq, sv, tv, u, w, x, a, rv, rx, write_v, with_norm);
    else if (nq <= 12) launch_update2<12>(Q, nq, sv, tv, u, w, x, a, rv, rx, write_v, with_norm);
    else if (nq <= 16) launch_update2<16>(Q, nq, sv, tv, u, w, x, a, rv, rx, write_v, with_norm);
    else if (nq <= 24) launch_update2<24>(Q, nq, sv, tv, u, w, x, a, rv, rx, write_v, with_norm);
    else launch_update2<32>(Q, nq, sv, tv, u, w, x, a, rv, rx, write_v, with_norm);
    HIP_TRY(hipGetLastError());
    return with_norm ? reduce(3) : STIG_OK;
  }
  // host value of slot `k`'s entry i (synchronises)
  stig_status fetch(int k, int i, double *out) {
    HIP_TRY(hipMemcpyAsync(p->pin + 3 * KRY_MAXV, slot(k) + i, sizeof(double),
                           hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    *out = p->pin[3 * KRY_MAXV];
    return STIG_OK;
  }
  // r = f - A u; host value of ||r||_2 (synchronises).  On the banded form the
  // last pass of the product writes r and its partial norms directly.
  stig_status residual_of(const double *f, const double *u, double *r, double *tmp,
                          int transpose, double *norm) {
    const int64_t cap = (int64_t)(p->partial.bytes / sizeof(double));
    int64_t rblocks;
    int rch;
    residual_grid(p, &rblocks, &rch);
    if (!p->csr_rowptr && rblocks * rch <= cap) {
      int64_t nparts = 0;
      STIG_TRY(run_residual_banded(p, f, u, r, transpose, partial(), cap, &nparts));
      hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(KRY_BLOCK), 0, p->stream, partial(),
                         (int)nparts, slot(3));
      HIP_TRY(hipGetLastError());
      double v;
      STIG_TRY(fetch(3, 0, &v));
      *norm = std::sqrt(v);
      return STIG_OK;
    }
    STIG_TRY(run_matvec(p, u, tmp, 1, transpose));
    return residual(f, tmp, r, norm);
  }
  // ||x||^2, ||y||^2 into slot 3 entries 0 and KRY_MAXV-1 (no synchronisation)
  stig_status norms_async(const double *x, const double *y) {
    ProfScope ps(p, STIG_K_KRYLOV, 2.0 * p->N * 8);
    hipLaunchKernelGGL(two_norms, dim3(KRY_GRID), dim3(KRY_BLOCK), 0, p->stream, x, y, p->N,
                       partial());
    HIP_TRY(hipGetLastError());
    return reduce(3);
  }
  // r = f - Ax with ||r||^2 in slot 3 entry KRY_MAXV-1 (no synchronisation)
  stig_status residual_async(const double *f, const double *Ax, double *r) {
    ProfScope ps(p, STIG_K_KRYLOV, 3.0 * p->N * 8);
    hipLaunchKernelGGL(residual_norm, dim3(KRY_GRID), dim3(KRY_BLOCK), 0, p->stream, f, Ax, r,
                       p->N, partial());
    HIP_TRY(hipGetLastError());
    return reduce(3);
  }
  // r = f - Ax; host value of ||r||_2 (synchronises)
  stig_status residual(const double *f, const double *Ax, double *r, double *norm) {
    ProfScope ps(p, STIG_K_KRYLOV, 3.0 * p->N * 8);
    hipLaunchKernelGGL(residual_norm, dim3(KRY_GRID), dim3(KRY_BLOCK), 0, p->stream, f, Ax, r,
                       p->N, partial());
    HIP_TRY(hipGetLastError());
    STIG_TRY(reduce(3));
    double v;
    STIG_TRY(fetch(3, KRY_MAXV - 1, &v));
    *norm = std::sqrt(v);
    return STIG_OK;
  }
  // host values of ||x||_2 and ||y||_2 from one pass (synchronises)
  stig_status norms(const double *x, const double *y, double *nx, double *ny) {
    ProfScope ps(p, STIG_K_KRYLOV, 2.0 * p->N * 8);
    hipLaunchKernelGGL(two_norms, dim3(KRY_GRID), dim3(KRY_BLOCK), 0, p->stream, x, y, p->N,
                       partial());
    HIP_TRY(hipGetLastError());
    STIG_TRY(reduce(3));
    double *v = p->pin + 3 * KRY_MAXV;
    HIP_TRY(hipMemcpyAsync(v, slot(3), KRY_MAXV * sizeof(double), hipMemcpyDeviceToHost,
                           p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    *nx = std::sqrt(v[0]);
    *ny = std::sqrt(v[KRY_MAXV - 1]);
    return STIG_OK;
  }
  stig_status axpby(const double *x, const double *y, double *out, double a, double b) {
    hipLaunchKernelGGL(stig::axpby, dim3(grid_for(p->N, 256, 8192)), dim3(256), 0, p->stream, x,
                       y, out, a, b, p->N);
    HIP_TRY(hipGetLastError());
    return STIG_OK;
  }
};

stig_status apply_dispatch(stig_plan *p, const double *r, double *s, int nrhs, int transpose,
                           stig_prec prec) {
  switch (prec) {
    case STIG_FP64: return run_apply<double, double>(p, r, s, nrhs, transpose);
    case STIG_FP32: return run_apply<float, float>(p, r, s, nrhs, transpose);
    case STIG_BF16: return run_apply<bf16, bf16>(p, r, s, nrhs, transpose);
  }
  return fail(STIG_EINVAL, "unknown precision");
}

// pinned staging area of the plan (allocated by the setup)
stig_status ensure_pinned(stig_plan *p, size_t n) {
  if (p->pin && p->pin_n >= n) return STIG_OK;
  if (p->pin) (void)hipHostFree(p->pin);
  p->pin = nullptr;
  p->pin_n = 0;
  if (hipHostMalloc((void **)&p->pin, n * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    p->pin = nullptr;
    return fail(STIG_ENOMEM, "pinned host staging buffer");
  }
  p->pin_n = n;
  return STIG_OK;
}
// the breakdown flag's copy: the last double of the pinned area
int *pinned_flag(stig_plan *p) { return reinterpret_cast<int *>(p->pin + p->pin_n - 1); }

// reports (and clears) the breakdown flag whose copy is in the pinned area
stig_status flag_result(stig_plan *p, int f) {
  if (f) {
    int z = 0;
    HIP_TRY(hipMemcpy(p->flag.p, &z, sizeof(int), hipMemcpyHostToDevice));
    return fail(STIG_EBREAKDOWN, "non-positive pivot in a shifted time system");
  }
  return STIG_OK;
}

stig_status check_flag(stig_plan *p) {
  int f = 0;
  HIP_TRY(hipMemcpyAsync(&f, p->flag.p, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (f) {
    int z = 0;
    HIP_TRY(hipMemcpy(p->flag.p, &z, sizeof(int), hipMemcpyHostToDevice));
    return fail(STIG_EBREAKDOWN, "non-positive pivot in a shifted time system");
  }
  return STIG_OK;
}

// Host side of one right-hand side's Arnoldi process with delayed
// re-orthogonalisation.  The Hessenberg matrix is kept un-rotated: column j is
// provisional after step j (its subdiagonal entry is the norm of the once-
// orthogonalised w_j) and final after step j + 1, which re-orthogonalises the
// next basis vector and corrects the column; the least-squares problem is
// re-solved by Givens rotations from scratch at every step (k <= 32).
struct ArnoldiHost {
  int m = 0;
  double beta = 0.0;
  std::vector<double> H;  // (m + 1) x m, row-major
  double &h(int i, int j) { return H[(size_t)i * m + j]; }
  void reset(int m_, double beta_) {
    m = m_;
    beta = beta_;
    H.assign((size_t)(m + 1) * m, 0.0);
  }
  // min || beta e_0 - H_k y || over the first k columns: the residual norm, and
  // y (host, k entries) when asked
  double solve(int k, double *y) const {
    std::vector<double> R((size_t)(k + 1) * k), g(k + 1, 0.0);
    for (int i = 0; i <= k; ++i)
      for (int c = 0; c < k; ++c) R[(size_t)i * k + c] = H[(size_t)i * m + c];
    g[0] = beta;
    for (int c = 0; c < k; ++c) {
      const double a = R[(size_t)c * k + c], b = R[(size_t)(c + 1) * k + c];
      const double rr = std::hypot(a, b);
      const double cs = rr == 0.0 ? 1.0 : a / rr, sn = rr == 0.0 ? 0.0 : b / rr;
      for (int q = c; q < k; ++q) {
        const double x = R[(size_t)c * k + q], z = R[(size_t)(c + 1) * k + q];
        R[(size_t)c * k + q] = cs * x + sn * z;
        R[(size_t)(c + 1) * k + q] = -sn * x + cs * z;
      }
      const double g0 = g[c];
      g[c] = cs * g0;
      g[c + 1] = -sn * g0;
    }
    if (y)
      for (int q = k - 1; q >= 0; --q) {
        double acc = g[q];
        for (int c = q + 1; c < k; ++c) acc -= R[(size_t)q * k + c] * y[c];
        y[q] = acc / R[(size_t)q * k + q];
      }
    return std::fabs(g[k]);
  }
};

// One Arnoldi step's host arithmetic after the one-pass products of
// krylov_dots2: hs = [Q^T u (KRY_MAXV) | Q^T w (KRY_MAXV) | u.u, u.w, w.w].
// Re-orthogonalising u_j = w'_{j-1} / nrm_prev against Q = [v_0 .. v_{j-1}]
// (u_j = Q s + rho v_j) finalises column j - 1; w_j = A z_j is then split as
// Q t + v_j h_jj + w'_j, the provisional column j.  s2 (optional) is the
// product of an explicit re-orthogonalisation pass of u_j (then u.u is that
// pass's norm and s the first pass's).
// ||w'||^2 = w.w - ||t||^2 - h_jj^2 carries an absolute rounding error of a few
// eps w.w: below this fraction of w.w the norm is taken from w' itself (one more
// round trip); above it its relative error is below 1e-7, and the next step's
// re-orthogonalisation absorbs any error of the scaling.
constexpr double KRY_CANCEL = 1e-8;

struct StepHost {
  double rho = 1.0, hjj = 0.0, nrm2 = 0.0, ww = 0.0;
};
bool arnoldi_step(ArnoldiHost &ah, int j, const double *hs, const double *s2, double uu2,
                  double nrm_prev, StepHost &out) {
  const double *sv = hs, *tv = hs + KRY_MAXV;
  const double uu = s2 ? uu2 : hs[2 * KRY_MAXV], uw = hs[2 * KRY_MAXV + 1];
  const double ww = hs[2 * KRY_MAXV + 2];
  double ss = 0.0, stt = 0.0, tt = 0.0;
  for (int i = 0; i < j; ++i) {
    const double st = s2 ? sv[i] + s2[i] : sv[i];  // total component of u_j along v_i
    const double sr = s2 ? s2[i] : sv[i];           // what remains to remove from u in memory
    ss += sr * sr;
    stt += st * tv[i];
    tt += tv[i] * tv[i];
  }
  double rho = 1.0;
  if (j > 0) {
    const double rho2 = uu - ss;
    rho = rho2 > 0.0 ? std::sqrt(rho2) : 0.0;
    for (int i = 0; i < j; ++i) ah.h(i, j - 1) += nrm_prev * (s2 ? sv[i] + s2[i] : sv[i]);
    ah.h(j, j - 1) = nrm_prev * rho;
  }
  out.rho = rho;
  out.ww = ww;
  if (rho == 0.0) return false;  // u_j in span(Q): the Krylov space is invariant
  for (int i = 0; i < j; ++i) ah.h(i, j) = tv[i];
  out.hjj = (uw - stt) / rho;
  ah.h(j, j) = out.hjj;
  out.nrm2 = ww - tt - out.hjj * out.hjj;
  return true;
}

// One right-hand side: restarted (F)GMRES with right preconditioning.  Both
// variants keep the preconditioned basis Z (m vectors): for a fixed linear
// preconditioner u += Z y equals u += P^{-1} (V y), and it saves one
// preconditioner apply per cycle; flexible GMRES needs Z anyway.  The Arnoldi
// process is classical Gram-Schmidt with delayed re-orthogonalisation (the
// second pass of step j is done at step j + 1, together with the first pass of
// w_{j+1}): one reduction and two passes over the basis per step.  z_j is
// P^{-1} u_j of the once-orthogonalised u_j; A z_j = w_j is expressed in the
// final basis, so A Z = V H holds with the corrected columns.
stig_status gmres_one(stig_plan *p, const double *f, double *u, int m, double rtol, int maxit,
                      int flexible, int transpose, stig_prec prec, stig_info *info) {
  (void)flexible;
  const int64_t N = p->N;
  Krylov K{p};
  STIG_TRY(p->V.ensure((size_t)(m + 1) * N * sizeof(double)));
  STIG_TRY(p->Z.ensure((size_t)m * N * sizeof(double)));
  STIG_TRY(p->AZ.ensure((size_t)m * N * sizeof(double)));
  STIG_TRY(p->tmp.ensure(N * sizeof(double)));
  double *V = p->V.as<double>(), *Z = p->Z.as<double>(), *AZ = p->AZ.as<double>(),
         *tmp = p->tmp.as<double>();
  std::vector<double> y(m);
  double *hs = p->pin;

  double fnorm, unorm;
  STIG_TRY(K.norms(f, u, &fnorm, &unorm));
  if (!std::isfinite(fnorm)) return fail(STIG_ENONFINITE, "non-finite right-hand side norm");
  if (!std::isfinite(unorm)) return fail(STIG_ENONFINITE, "non-finite initial guess");
  info->iters = 0;
  info->restarts = 0;
  info->relres_true = 0.0;
  info->relres_est = 0.0;
  if (fnorm == 0.0) {
    HIP_TRY(hipMemsetAsync(u, 0, N * sizeof(double), p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return STIG_OK;
  }
  // r0 = f - A u (= f for a zero initial guess, without a product)
  double beta;
  const double *r = V;
  if (unorm == 0.0) {
    r = f;
    beta = fnorm;
  } else {
    STIG_TRY(K.residual_of(f, u, V, tmp, transpose, &beta));
  }
  if (!std::isfinite(beta)) return fail(STIG_ENONFINITE, "non-finite initial residual");
  info->relres_true = beta / fnorm;
  info->relres_est = info->relres_true;
  int cycle = 0;
  ArnoldiHost ah;
  // pinned layout: [one-pass products (KRY_D2) | explicit pass region (KRY_MAXV)]
  auto fetch_products = [&]() -> stig_status {
    HIP_TRY(hipMemcpyAsync(hs, K.slot(0), KRY_D2 * sizeof(double), hipMemcpyDeviceToHost,
                           p->stream));
    HIP_TRY(hipMemcpyAsync(pinned_flag(p), p->flag.p, sizeof(int), hipMemcpyDeviceToHost,
                           p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return flag_result(p, *pinned_flag(p));
  };
  double *hx = hs + 3 * KRY_MAXV;  // region 3 copy
  while (beta / fnorm > rtol && info->iters < maxit) {
    if (cycle++ > 0) info->restarts++;
    STIG_TRY(K.axpby(r, nullptr, V, 1.0 / beta, 0.0));  // u_0 = v_0 = r / beta
    r = V;
    ah.reset(m, beta);
    int k = 0;
    bool stop = false;       // estimate at rtol, breakdown or iteration budget spent
    double nrm_prev = 1.0;   // u_j = w'_{j-1} / nrm_prev
    for (int j = 0; j < m; ++j) {
      double *uj = V + (int64_t)j * N;
      double *zj = Z + (int64_t)j * N, *azj = AZ + (int64_t)j * N;
      STIG_TRY(apply_dispatch(p, uj, zj, 1, transpose, prec));
      STIG_TRY(run_matvec(p, zj, azj, 1, transpose));  // w_j = A z_j, kept for the cycle's residual
      STIG_TRY(K.dots2(V, j, uj, azj));
      STIG_TRY(fetch_products());
      info->iters++;
      // u_j far from orthogonal to Q (s.s > 3/4 u.u): one explicit pass
      // u_j -= Q s with Q^T u_j and u_j . u_j (region 3) before v_j is formed
      const double *s_dev = K.slot(0);
      const double *s2 = nullptr;
      double uu2 = 0.0;
      if (j > 0) {
        double ss = 0.0;
        for (int i = 0; i < j; ++i) ss += hs[i] * hs[i];
        if (!(hs[2 * KRY_MAXV] - ss > 0.25 * hs[2 * KRY_MAXV])) {
          STIG_TRY(K.update(V, j, K.slot(0), -1.0, uj, 1, 3));
          HIP_TRY(hipMemcpyAsync(hx, K.slot(3), KRY_MAXV * sizeof(double), hipMemcpyDeviceToHost,
                                 p->stream));
          HIP_TRY(hipStreamSynchronize(p->stream));
          s2 = hx;
          uu2 = hx[KRY_MAXV - 1];
          s_dev = K.slot(3);
        }
      }
      StepHost st;
      const bool alive = arnoldi_step(ah, j, hs, s2, uu2, nrm_prev, st);
      if (!alive) {  // u_j lies in the span of the basis: the solution is in it
        k = j;
        stop = true;
        break;
      }
      if (!std::isfinite(st.hjj) || !std::isfinite(st.nrm2))
        return fail(STIG_ENONFINITE, "non-finite value in the Arnoldi process");
      const double a = st.hjj / st.rho;
      double *unext = V + (int64_t)(j + 1) * N;
      if (!(st.nrm2 > KRY_CANCEL * st.ww)) {
        // w_j nearly in the span (the norm by Pythagoras would be lost to
        // rounding): the norm of w'_j from w'_j itself (one more round trip;
        // the vector is written below only if the cycle goes on)
        STIG_TRY(K.update2(V, j, s_dev, K.slot(1), uj, azj, nullptr, a, 1.0 / st.rho, 1.0, 0, 1));
        double xx;
        STIG_TRY(K.fetch(3, KRY_MAXV - 1, &xx));
        ah.h(j + 1, j) = std::sqrt(xx);
      } else {
        ah.h(j + 1, j) = std::sqrt(st.nrm2);
      }
      nrm_prev = ah.h(j + 1, j);
      k = j + 1;
      double colnorm = 0.0;
      for (int i = 0; i <= j; ++i) colnorm += ah.h(i, j) * ah.h(i, j);
      const double hnext = ah.h(j + 1, j);
      if (!std::isfinite(hnext) || !std::isfinite(colnorm))
        return fail(STIG_ENONFINITE, "non-finite value in the Arnoldi process");
      info->relres_est = ah.solve(k, nullptr) / fnorm;
      const bool breakdown = hnext <= 1e-14 * std::sqrt(colnorm + hnext * hnext);
      stop = info->relres_est <= rtol || breakdown || info->iters >= maxit;
      if (stop || j + 1 == m) break;
      // the step's second pass: v_j over u_j, u_{j+1} = w'_j / nrm
      STIG_TRY(K.update2(V, j, s_dev, K.slot(1), uj, azj, unext, a, 1.0 / st.rho,
                         1.0 / nrm_prev, j > 0, 0));
    }
    if (k == 0) break;  // nothing to add (cannot happen with beta > 0)
    ah.solve(k, y.data());
    // y and y / beta to the device (the pinned area is not written again
    // before the next synchronisation)
    for (int i = 0; i < k; ++i) {
      hs[2 * KRY_MAXV + i] = y[i];
      hs[3 * KRY_MAXV + i] = y[i] / beta;
    }
    HIP_TRY(hipMemcpyAsync(K.slot(3), hs + 2 * KRY_MAXV, k * sizeof(double),
                           hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(K.slot(2), hs + 3 * KRY_MAXV, k * sizeof(double),
                           hipMemcpyHostToDevice, p->stream));
    // u += Z y (u = Z y while u is the zero initial guess)
    if (cycle == 1 && unorm == 0.0) STIG_TRY(K.update(Z, k, K.slot(3), 1.0, nullptr, 0, 0, u));
    else STIG_TRY(K.update(Z, k, K.slot(3), 1.0, u, 0, 0));
    if (stop) {
      // the cycle that may end the solve: a fresh residual r = f - A u (one
      // product of A), written over v_0; the solve restarts from it if it is
      // still above rtol
      STIG_TRY(K.residual_of(f, u, V, tmp, transpose, &beta));
    } else {
      // a full cycle without convergence: the next cycle's residual from this
      // cycle's products of A, r = r_0 - sum_i y_i A z_i = beta (v_0 - AZ y / beta),
      // written over v_0, with its norm
      STIG_TRY(K.update(AZ, k, K.slot(2), -1.0, V, 1, 3, V, beta));
      double nsq;
      STIG_TRY(K.fetch(3, KRY_MAXV - 1, &nsq));
      beta *= std::sqrt(nsq);
    }
    if (!std::isfinite(beta)) return fail(STIG_ENONFINITE, "non-finite residual");
    info->relres_true = beta / fnorm;
  }
  STIG_TRY(check_flag(p));
  return info->relres_true <= rtol ? STIG_OK : STIG_NOT_CONVERGED;
}

// First restart cycle of (F)GMRES for nb right-hand sides in lockstep: step j
// applies the preconditioner and A to the j-th basis vectors of all of them in
// one batched call (basis vectors stored [j][rhs][N]), runs each one's
// Gram-Schmidt passes (delayed re-orthogonalisation, as gmres_one), and
// synchronises once for all.  A right-hand side whose estimate reaches rtol
// (or that breaks down) freezes; its later basis slots are zeroed so the
// batched calls stay finite.  At the end every solution is updated and its
// fresh residual computed (one batched product); done[r] tells which reached
// rtol.  The iteration is the same as gmres_one's first cycle for each
// right-hand side.
stig_status gmres_batch(stig_plan *p, const double *f, double *u, int nb, int m, double rtol,
                        int maxit, int transpose, stig_prec prec, stig_info *infos, bool *done) {
  const int64_t N = p->N, ld = (int64_t)nb * N;
  constexpr int S4 = 4 * KRY_MAXV;  // small-buffer doubles per right-hand side
  STIG_TRY(p->V.ensure((size_t)(m + 1) * ld * sizeof(double)));
  STIG_TRY(p->Z.ensure((size_t)m * ld * sizeof(double)));
  STIG_TRY(p->AZ.ensure((size_t)m * ld * sizeof(double)));
  STIG_TRY(p->tmp.ensure((size_t)ld * sizeof(double)));
  if (nb > KRY_MAXB || p->small.bytes < (size_t)nb * S4 * sizeof(double) ||
      p->pin_n < (size_t)nb * S4 + 1)
    return fail(STIG_EINVAL, "too many right-hand sides in one lockstep cycle");
  double *V = p->V.as<double>(), *Z = p->Z.as<double>(), *AZ = p->AZ.as<double>(),
         *tmp = p->tmp.as<double>(), *hs = p->pin;
  std::vector<Krylov> K;
  for (int r = 0; r < nb; ++r) K.push_back(Krylov{p, ld, (int64_t)r * S4});
  auto fetch_all = [&](bool with_flag) -> stig_status {
    HIP_TRY(hipMemcpyAsync(hs, p->small.p, (size_t)nb * S4 * sizeof(double),
                           hipMemcpyDeviceToHost, p->stream));
    if (with_flag)
      HIP_TRY(hipMemcpyAsync(pinned_flag(p), p->flag.p, sizeof(int), hipMemcpyDeviceToHost,
                             p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return with_flag ? flag_result(p, *pinned_flag(p)) : STIG_OK;
  };
  // ||f||, ||u|| of every right-hand side in one round trip
  for (int r = 0; r < nb; ++r) STIG_TRY(K[r].norms_async(f + r * N, u + r * N));
  STIG_TRY(fetch_all(false));
  std::vector<double> fnorm(nb), unorm(nb), beta(nb, 0.0), nrm_prev(nb, 1.0);
  for (int r = 0; r < nb; ++r) {
    fnorm[r] = std::sqrt(hs[r * S4 + 3 * KRY_MAXV]);
    unorm[r] = std::sqrt(hs[r * S4 + 3 * KRY_MAXV + KRY_MAXV - 1]);
    if (!std::isfinite(fnorm[r])) return fail(STIG_ENONFINITE, "non-finite right-hand side norm");
    if (!std::isfinite(unorm[r])) return fail(STIG_ENONFINITE, "non-finite initial guess");
  }
  std::vector<char> active(nb, 0);
  std::vector<int> kk(nb, 0);
  std::vector<ArnoldiHost> ah(nb);
  for (int r = 0; r < nb; ++r) {
    infos[r] = stig_info{0, 0, 0.0, 0.0, 0.0};
    done[r] = false;
    double *v0 = V + r * N;
    if (fnorm[r] == 0.0) {
      HIP_TRY(hipMemsetAsync(u + r * N, 0, N * sizeof(double), p->stream));
      HIP_TRY(hipMemsetAsync(v0, 0, N * sizeof(double), p->stream));
      done[r] = true;
      continue;
    }
    if (unorm[r] == 0.0) {
      beta[r] = fnorm[r];
      STIG_TRY(K[r].axpby(f + r * N, nullptr, v0, 1.0 / beta[r], 0.0));
    } else {
      STIG_TRY(K[r].residual_of(f + r * N, u + r * N, v0, tmp, transpose, &beta[r]));
      if (!std::isfinite(beta[r])) return fail(STIG_ENONFINITE, "non-finite initial residual");
      if (beta[r] / fnorm[r] <= rtol) {  // already converged: keep u
        infos[r].relres_true = infos[r].relres_est = beta[r] / fnorm[r];
        HIP_TRY(hipMemsetAsync(v0, 0, N * sizeof(double), p->stream));
        done[r] = true;
        continue;
      }
      STIG_TRY(K[r].axpby(v0, nullptr, v0, 1.0 / beta[r], 0.0));
    }
    infos[r].relres_true = infos[r].relres_est = beta[r] / fnorm[r];
    active[r] = 1;
    ah[r].reset(m, beta[r]);
  }
  auto any_active = [&]() {
    for (int r = 0; r < nb; ++r)
      if (active[r]) return true;
    return false;
  };
  for (int j = 0; j < m && any_active(); ++j) {
    STIG_TRY(apply_dispatch(p, V + j * ld, Z + j * ld, nb, transpose, prec));
    STIG_TRY(run_matvec(p, Z + j * ld, AZ + j * ld, nb, transpose));
    for (int r = 0; r < nb; ++r)
      if (active[r]) STIG_TRY(K[r].dots2(V + r * N, j, V + j * ld + r * N, AZ + j * ld + r * N));
    STIG_TRY(fetch_all(true));
    for (int r = 0; r < nb; ++r) {
      if (!active[r]) continue;
      const double *h = hs + r * S4;
      double *uj = V + j * ld + r * N, *azj = AZ + j * ld + r * N;
      double *unext = V + (j + 1) * ld + r * N;
      infos[r].iters++;
      const double *s_dev = K[r].slot(0);
      const double *s2 = nullptr;
      double uu2 = 0.0;
      std::vector<double> s2h;
      if (j > 0) {
        double ss = 0.0;
        for (int i = 0; i < j; ++i) ss += h[i] * h[i];
        if (!(h[2 * KRY_MAXV] - ss > 0.25 * h[2 * KRY_MAXV])) {
          STIG_TRY(K[r].update(V + r * N, j, K[r].slot(0), -1.0, uj, 1, 3));
          s2h.resize(KRY_MAXV);
          HIP_TRY(hipMemcpyAsync(s2h.data(), K[r].slot(3), KRY_MAXV * sizeof(double),
                                 hipMemcpyDeviceToHost, p->stream));
          HIP_TRY(hipStreamSynchronize(p->stream));
          s2 = s2h.data();
          uu2 = s2h[KRY_MAXV - 1];
          s_dev = K[r].slot(3);
        }
      }
      StepHost st;
      if (!arnoldi_step(ah[r], j, h, s2, uu2, nrm_prev[r], st)) {
        kk[r] = j;
        active[r] = 0;
        continue;
      }
      if (!std::isfinite(st.hjj) || !std::isfinite(st.nrm2))
        return fail(STIG_ENONFINITE, "non-finite value in the Arnoldi process");
      const double a = st.hjj / st.rho;
      if (!(st.nrm2 > KRY_CANCEL * st.ww)) {
        STIG_TRY(K[r].update2(V + r * N, j, s_dev, K[r].slot(1), uj, azj, nullptr, a,
                              1.0 / st.rho, 1.0, 0, 1));
        double xx;
        STIG_TRY(K[r].fetch(3, KRY_MAXV - 1, &xx));
        ah[r].h(j + 1, j) = std::sqrt(xx);
      } else {
        ah[r].h(j + 1, j) = std::sqrt(st.nrm2);
      }
      nrm_prev[r] = ah[r].h(j + 1, j);
      kk[r] = j + 1;
      double colnorm = 0.0;
      for (int i = 0; i <= j; ++i) colnorm += ah[r].h(i, j) * ah[r].h(i, j);
      const double hnext = ah[r].h(j + 1, j);
      if (!std::isfinite(hnext) || !std::isfinite(colnorm))
        return fail(STIG_ENONFINITE, "non-finite value in the Arnoldi process");
      infos[r].relres_est = ah[r].solve(kk[r], nullptr) / fnorm[r];
      const bool breakdown = hnext <= 1e-14 * std::sqrt(colnorm + hnext * hnext);
      if (infos[r].relres_est <= rtol || breakdown || infos[r].iters >= maxit || j + 1 == m) {
        active[r] = 0;
        continue;
      }
      STIG_TRY(K[r].update2(V + r * N, j, s_dev, K[r].slot(1), uj, azj, unext, a, 1.0 / st.rho,
                            1.0 / nrm_prev[r], j > 0, 0));
    }
    // frozen right-hand sides: zero basis vector for the next batched step
    if (j + 1 < m)
      for (int r = 0; r < nb; ++r)
        if (!active[r])
          HIP_TRY(hipMemsetAsync(V + (j + 1) * ld + r * N, 0, N * sizeof(double), p->stream));
  }
  // solutions, then their fresh residuals (one batched product, one round trip)
  for (int r = 0; r < nb; ++r) {
    if (kk[r] == 0) continue;
    std::vector<double> y(kk[r]);
    ah[r].solve(kk[r], y.data());
    double *stage = hs + r * S4 + 2 * KRY_MAXV;  // not written again before the next round trip
    for (int i = 0; i < kk[r]; ++i) stage[i] = y[i];
    HIP_TRY(hipMemcpyAsync(K[r].slot(3), stage, kk[r] * sizeof(double), hipMemcpyHostToDevice,
                           p->stream));
    if (unorm[r] == 0.0) STIG_TRY(K[r].update(Z + r * N, kk[r], K[r].slot(3), 1.0, nullptr, 0, 0, u + r * N));
    else STIG_TRY(K[r].update(Z + r * N, kk[r], K[r].slot(3), 1.0, u + r * N, 0, 0));
  }
  STIG_TRY(run_matvec(p, u, tmp, nb, transpose));
  for (int r = 0; r < nb; ++r)
    if (kk[r] > 0) STIG_TRY(K[r].residual_async(f + r * N, tmp + r * N, V + r * N));
  STIG_TRY(fetch_all(true));
  for (int r = 0; r < nb; ++r) {
    if (kk[r] == 0) continue;
    const double bt = std::sqrt(hs[r * S4 + 3 * KRY_MAXV + KRY_MAXV - 1]);
    if (!std::isfinite(bt)) return fail(STIG_ENONFINITE, "non-finite residual");
    infos[r].relres_true = bt / fnorm[r];
    done[r] = infos[r].relres_true <= rtol;
  }
  return STIG_OK;
}

}  // namespace

// =================================================================== C ABI

extern "C" {

const char *stig_status_string(stig_status s) {
  switch (s) {
    case STIG_OK: return "ok";
    case STIG_NOT_CONVERGED: return "not converged";
    case STIG_EINVAL: return "invalid argument";
    case STIG_ENOMEM: return "out of device memory";
    case STIG_EHIP: return "HIP runtime error";
    case STIG_EBREAKDOWN: return "breakdown (non-positive pivot)";
    case STIG_ENONFINITE: return "non-finite value";
    case STIG_ESTATE: return "plan not set up";
  }
  return "unknown status";
}

const char *stig_last_error(void) { return g_last_error.c_str(); }

stig_status stig_plan_create(stig_plan **out, int d, const int *n_s, int n_t, int p_s, int p_t,
                             void *stream) {
  if (!out) return fail(STIG_EINVAL, "null output pointer");
  *out = nullptr;
  if (d < 1 || d > 3 || !n_s) return fail(STIG_EINVAL, "d must be 1..3 with n_s given");
  if (n_t < 2 || n_t > 1024) return fail(STIG_EINVAL, "n_t out of range");
  if (p_s < 1 || p_s > MAX_P || p_t < 1 || p_t > MAX_P)
    return fail(STIG_EINVAL, "spline degree must be 1..5");
  stig_plan *p = new stig_plan;
  p->d = d;
  p->Ns = 1;
  for (int l = 0; l < d; ++l) {
    if (n_s[l] < 1 || n_s[l] > 200) {
      delete p;
      return fail(STIG_EINVAL, "n_s out of range");
    }
    p->n[l] = n_s[l];
    p->Ns *= n_s[l];
  }
  p->nt = n_t;
  p->ps = p_s;
  p->pt = p_t;
  p->N = p->Ns * n_t;
  p->stream = (hipStream_t)stream;
  int dev = 0, cu = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    p->device = dev;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
      p->num_cu = cu;
  }
  (void)hipGetLastError();
  *out = p;
  return STIG_OK;
}

void stig_plan_destroy(stig_plan *plan) { delete plan; }

stig_status stig_set_option(stig_plan *plan, int option, int value) {
  STIG_TRY(check_plan(plan, false));
  switch (option) {
    case STIG_OPT_PLANE_FUSION:
      if (value != 0 && value != 1) return fail(STIG_EINVAL, "plane fusion takes 0 or 1");
      plan->plane_fusion = value != 0;
      return STIG_OK;
    case STIG_OPT_PARITY_SPLIT:
      if (value != 0 && value != 1) return fail(STIG_EINVAL, "parity split takes 0 or 1");
      plan->parity_split = value != 0;
      return STIG_OK;
    case STIG_OPT_TIME_KERNEL:
      if (value < 0 || value > 4) return fail(STIG_EINVAL, "time kernel takes 0 .. 4");
      if (value == 4 && plan->nt > ARROW_GEN_MAX_NT && (plan->nt - 2) % 32 != 0)
        return fail(STIG_EINVAL, "the arrowhead time kernel needs n_t <= 200 or n_t = 32 q + 2");
      if (value == 4 && plan->ready && !plan->arrow_ok && !plan->arrow_gen) {
        // factor the set-up time pencil now (host work and uploads)
        STIG_TRY(setup_arrowhead(plan, true));
        if (!plan->arrow_ok && !plan->arrow_gen)
          return fail(STIG_EINVAL, "the time pencil has no arrowhead factorization");
      }
      plan->time_kernel = value == 3 ? 0 : value;
      plan->time_recompute = value != 3;
      return STIG_OK;
  }
  return fail(STIG_EINVAL, "unknown option");
}

stig_status stig_set_stream(stig_plan *plan, void *stream) {
  STIG_TRY(check_plan(plan, false));
  plan->stream = (hipStream_t)stream;
  return STIG_OK;
}

stig_status stig_setup_1d_pencils(stig_plan *p, const double *const *K1d, const double *const *M1d,
                                  const double *Wt, const double *Mt, double gamma, double nu) {
  STIG_TRY(check_plan(p, false));
  if (!K1d || !M1d || !Wt || !Mt) return fail(STIG_EINVAL, "null matrix pointer");
  if (!(gamma >= 0.0) || !(nu >= 0.0) || !std::isfinite(gamma) || !std::isfinite(nu))
    return fail(STIG_EINVAL, "gamma and nu must be finite and non-negative");
  p->ready = false;
  p->gamma = gamma;
  p->nu = nu;
  for (auto &v : p->lamp_ps) v = 0;  // padded shifts are rebuilt from the new ones
  hipStream_t s = p->stream;
  std::vector<std::vector<double>> lams(p->d);
  for (int l = 0; l < p->d; ++l) {
    int n = p->n[l];
    if (!K1d[l] || !M1d[l]) return fail(STIG_EINVAL, "null spatial factor");
    std::vector<double> U((size_t)n * n), UT((size_t)n * n);
    lams[l].resize(n);
    // persymmetric pencil (uniform knots): even / odd eigenbasis, which the
    // half-size mode products use; otherwise the plain generalized eigenbasis
    const bool sp = n >= 2 && persymmetric(n, K1d[l], 1e-13) && persymmetric(n, M1d[l], 1e-13);
    if (!(sp ? split_eig(n, K1d[l], M1d[l], U.data(), lams[l].data())
             : sym_eig(n, K1d[l], M1d[l], U.data(), lams[l].data())))
      return fail(STIG_EBREAKDOWN, "spatial mass matrix is not positive definite");
    p->split[l] = sp;
    if (sp) {
      const int m = n / 2, ne = n - m;
      std::vector<double> fe((size_t)ne * ne), fo((size_t)m * m), be((size_t)ne * ne), bo((size_t)m * m);
      for (int j = 0; j < ne; ++j)
        for (int x = 0; x < ne; ++x) {
          fe[(size_t)j * ne + x] = U[(size_t)x * n + j];
          be[(size_t)x * ne + j] = U[(size_t)x * n + j];
        }
      for (int j = 0; j < m; ++j)
        for (int x = 0; x < m; ++x) {
          fo[(size_t)j * m + x] = U[(size_t)x * n + ne + j];
          bo[(size_t)x * m + j] = U[(size_t)x * n + ne + j];
        }
      STIG_TRY(upload(p->hFE[0][l], fe, s));
      STIG_TRY(upload(p->hFO[0][l], fo, s));
      STIG_TRY(upload(p->hBE[0][l], be, s));
      STIG_TRY(upload(p->hBO[0][l], bo, s));
      STIG_TRY(upload(p->hFE[1][l], convert<float>(fe), s));
      STIG_TRY(upload(p->hFO[1][l], convert<float>(fo), s));
      STIG_TRY(upload(p->hBE[1][l], convert<float>(be), s));
      STIG_TRY(upload(p->hBO[1][l], convert<float>(bo), s));
      STIG_TRY(upload(p->hFE[2][l], convert<uint16_t>(fe), s));
      STIG_TRY(upload(p->hFO[2][l], convert<uint16_t>(fo), s));
      STIG_TRY(upload(p->hBE[2][l], convert<uint16_t>(be), s));
      STIG_TRY(upload(p->hBO[2][l], convert<uint16_t>(bo), s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) UT[(size_t)i * n + j] = U[(size_t)j * n + i];
    STIG_TRY(upload(p->U64[l], U, s));
    STIG_TRY(upload(p->UT64[l], UT, s));
    STIG_TRY(upload(p->U32[l], convert<float>(U), s));
    STIG_TRY(upload(p->UT32[l], convert<float>(UT), s));
    STIG_TRY(upload(p->U16[l], convert<uint16_t>(U), s));
    STIG_TRY(upload(p->UT16[l], convert<uint16_t>(UT), s));
    std::vector<double> kb, mb;
    STIG_TRY(extract_band(K1d[l], n, p->ps, kb, "spatial stiffness"));
    STIG_TRY(extract_band(M1d[l], n, p->ps, mb, "spatial mass"));
    STIG_TRY(upload(p->sK[l], kb, s));
    STIG_TRY(upload(p->sM[l], mb, s));
    p->dK1[l].resize(n);
    p->dM1[l].resize(n);
    for (int i = 0; i < n; ++i) {
      p->dK1[l][i] = K1d[l][(size_t)i * n + i];
      p->dM1[l][i] = M1d[l][(size_t)i * n + i];
    }
    HIP_TRY(hipStreamSynchronize(s));  // host vectors go out of scope
  }
  // lambda_k = sum_l lambda_{l, i_l}, k = i_1 + n_1 (i_2 + n_2 i_3)
  std::vector<double> lk(p->Ns);
  for (int64_t k = 0; k < p->Ns; ++k) {
    int64_t r = k;
    double v = 0.0;
    for (int l = 0; l < p->d; ++l) {
      v += lams[l][r % p->n[l]];
      r /= p->n[l];
    }
    lk[k] = v;
  }
  STIG_TRY(upload(p->lam, lk, s));
  // the shifts in the padded plane layouts of the fused x/y passes (one per
  // storage size of the intermediates); padding entries repeat the first shift
  // of their z index (valid systems whose results are never read)
  if (p->d >= 2 && p->n[0] == p->n[1] && p->n[0] <= PLANE_MAX_N) {
    const int64_t nn = (int64_t)p->n[0] * p->n[1], nz = p->d == 3 ? p->n[2] : 1;
    const size_t sizes[3] = {8, 4, 2};
    for (int i = 0; i < 3; ++i) {
      const int64_t ps = padded_plane(p, sizes[i]);
      if (ps == nn) continue;
      STIG_TRY(p->lamp[i].ensure((size_t)nz * ps * sizeof(double)));
      hipLaunchKernelGGL(pad_shifts, dim3(grid_for(nz * ps, 256, 4096)), dim3(256), 0, s,
                         p->lam.as<double>(), p->lamp[i].as<double>(), nn, ps, nz);
      HIP_TRY(hipGetLastError());
      p->lamp_ps[i] = ps;
    }
  }
  {
    std::vector<double> id(2 * p->ps + 1, 0.0), zero(2 * p->ps + 1, 0.0);
    id[p->ps] = 1.0;
    STIG_TRY(upload(p->sId, id, s));
    STIG_TRY(upload(p->sZero, zero, s));
  }
  int nt = p->nt, P = p->pt;
  std::vector<double> WT((size_t)nt * nt);
  for (int i = 0; i < nt; ++i)
    for (int j = 0; j < nt; ++j) WT[(size_t)i * nt + j] = Wt[(size_t)j * nt + i];
  std::vector<double> wb, wtb, mb;
  STIG_TRY(extract_band(Wt, nt, P, wb, "W_t"));
  STIG_TRY(extract_band(WT.data(), nt, P, wtb, "W_t"));
  STIG_TRY(extract_band(Mt, nt, P, mb, "M_t"));
  p->dWt.resize(nt);
  p->dMt.resize(nt);
  for (int i = 0; i < nt; ++i) {
    p->dWt[i] = Wt[(size_t)i * nt + i];
    p->dMt[i] = Mt[(size_t)i * nt + i];
  }
  STIG_TRY(upload(p->tW64, wb, s));
  STIG_TRY(upload(p->tWT64, wtb, s));
  STIG_TRY(upload(p->tM64, mb, s));
  STIG_TRY(upload(p->tW32, convert<float>(wb), s));
  STIG_TRY(upload(p->tWT32, convert<float>(wtb), s));
  STIG_TRY(upload(p->tM32, convert<float>(mb), s));
  for (int tr = 0; tr < 2; ++tr) {
    std::vector<double> rec = step_records(tr ? wtb : wb, mb, nt, P);
    STIG_TRY(upload(p->tR64[tr], rec, s));
    STIG_TRY(upload(p->tR32[tr], convert<float>(rec), s));
  }
  p->hWt.assign(Wt, Wt + (size_t)nt * nt);
  p->hMt.assign(Mt, Mt + (size_t)nt * nt);
  // the general arrowhead form where it can run: chosen, or a default for shapes
  // without a register-resident banded kernel
  STIG_TRY(setup_arrowhead(p, p->time_kernel == 4 || arrow_auto_nt(nt)));
  if (p->time_kernel == 4 && !p->arrow_ok && !p->arrow_gen)
    return fail(STIG_EBREAKDOWN, "arrowhead factorization of the time pencil not reached "
                                 "(time kernel 4 selected)");
  std::vector<double> gw(wb), gwt(wtb), nm(mb);
  for (auto &v : gw) v *= gamma;
  for (auto &v : gwt) v *= gamma;
  for (auto &v : nm) v *= nu;
  STIG_TRY(upload(p->tgW, gw, s));
  STIG_TRY(upload(p->tgWT, gwt, s));
  STIG_TRY(upload(p->tnM, nm, s));
  STIG_TRY(p->flag.ensure(sizeof(int)));
  HIP_TRY(hipMemsetAsync(p->flag.p, 0, sizeof(int), s));
  STIG_TRY(p->partial.ensure((size_t)KRY_D2 * KRY_GRID * sizeof(double)));
  STIG_TRY(p->small.ensure((size_t)KRY_MAXB * 4 * KRY_MAXV * sizeof(double)));
  STIG_TRY(ensure_pinned(p, (size_t)KRY_MAXB * 4 * KRY_MAXV + 1));
  HIP_TRY(hipStreamSynchronize(s));
  // pivot check: one FP64 time pass on a zero input factors every shifted
  // system (its own temporaries: no workspace is needed for setup)
  {
    DevBuf zin, zout, zscr;
    STIG_TRY(zin.ensure(p->N * sizeof(double)));
    STIG_TRY(zout.ensure(p->N * sizeof(double)));
    // the banded elimination checks its pivots (whatever form the apply uses)
    const bool reg = time_reg_shape(p) && (p->time_kernel == 0 || p->time_kernel == 1);
    const size_t scr = reg ? 0 : (size_t)(p->pt + 1) * p->N * sizeof(double);
    if (scr) STIG_TRY(zscr.ensure(scr));
    const Span keep = p->tscr;
    p->tscr.p = zscr.p;
    p->tscr.bytes = scr;
    HIP_TRY(hipMemsetAsync(zin.p, 0, p->N * sizeof(double), s));
    const stig_status st = launch_time_banded<double, double>(
        p, zin.as<double>(), zout.as<double>(), 1, 0, TimeView{p->Ns, p->lam.as<double>()});
    p->tscr = keep;
    STIG_TRY(st);
    HIP_TRY(hipStreamSynchronize(s));
    STIG_TRY(check_flag(p));
  }
  p->ready = true;
  return STIG_OK;
}

stig_status stig_set_diag_scaling(stig_plan *p, const double *D) {
  STIG_TRY(check_plan(p, false));
  if (!D) {
    p->has_dmh = false;
    return STIG_OK;
  }
  STIG_TRY(p->dmh.ensure(p->N * sizeof(double)));
  hipLaunchKernelGGL(rsqrt_copy, dim3(grid_for(p->N, 256, 8192)), dim3(256), 0, p->stream, D,
                     p->dmh.as<double>(), p->N);
  HIP_TRY(hipGetLastError());
  p->has_dmh = true;
  return STIG_OK;
}

stig_status stig_set_diag_scaling_kron(stig_plan *p, const double *dMs, const double *dKs) {
  STIG_TRY(check_plan(p, true));
  if (!dMs || !dKs) return fail(STIG_EINVAL, "null diagonal");
  std::vector<double> D((size_t)p->N);
  for (int64_t s = 0; s < p->Ns; ++s) {
    // diagonals of M-tilde_s = (x)_l M_l and K-tilde_s = sum_l (.. K_l ..)
    double dm = 1.0, dk = 0.0;
    int64_t r = s;
    int idx[3] = {0, 0, 0};
    for (int l = 0; l < p->d; ++l) {
      idx[l] = (int)(r % p->n[l]);
      r /= p->n[l];
    }
    for (int l = 0; l < p->d; ++l) dm *= p->dM1[l][idx[l]];
    for (int l = 0; l < p->d; ++l) {
      double term = p->dK1[l][idx[l]];
      for (int m = 0; m < p->d; ++m)
        if (m != l) term *= p->dM1[m][idx[m]];
      dk += term;
    }
    for (int t = 0; t < p->nt; ++t) {
      double num = p->gamma * p->dWt[t] * dMs[s] + p->nu * p->dMt[t] * dKs[s];
      double den = p->gamma * p->dWt[t] * dm + p->nu * p->dMt[t] * dk;
      if (!(num > 0.0) || !(den > 0.0))
        return fail(STIG_EBREAKDOWN, "non-positive diagonal in the geometry scaling");
      D[(size_t)t * p->Ns + s] = num / den;
    }
  }
  DevBuf Dd;
  STIG_TRY(upload(Dd, D, p->stream));
  STIG_TRY(stig_set_diag_scaling(p, Dd.as<double>()));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return STIG_OK;
}

stig_status stig_assemble_2d(int n_el, int p, int nq, const double *c11, const double *c22,
                             const double *c33, int64_t *rowptr, int32_t *col, double *valK,
                             double *valM, int64_t *nnz) {
  if (n_el < 1 || p < 1 || p > 16 || nq < 1 || !nnz) return fail(STIG_EINVAL, "bad 2D assembly");
  if (rowptr && (!col || !valK || !valM || !c11 || !c22 || !c33))
    return fail(STIG_EINVAL, "null 2D assembly array");
  *nnz = assemble_2d(n_el, p, nq, c11, c22, c33, rowptr, col, valK, valM);
  return STIG_OK;
}

stig_status stig_separate_2d(int n1, int n2, const double *C11, const double *C22,
                             const double *C33, double *phi1, double *phi2, double *Phi1,
                             double *Phi2) {
  if (n1 < 1 || n2 < 1 || !C11 || !C22 || !C33 || !phi1 || !phi2 || !Phi1 || !Phi2)
    return fail(STIG_EINVAL, "bad separation arguments");
  for (int64_t i = 0; i < (int64_t)n1 * n2; ++i)
    if (!(C11[i] > 0) || !(C22[i] > 0) || !(C33[i] > 0))
      return fail(STIG_EINVAL, "coefficients must be positive");
  separate_2d(n1, n2, C11, C22, C33, phi1, phi2, Phi1, Phi2);
  return STIG_OK;
}

stig_status stig_assemble_3d(int n_el, int p, int nq, const double *c11, const double *c22,
                             const double *c33, const double *c00, int64_t *rowptr, int32_t *col,
                             double *valK, double *valM, int64_t *nnz) {
  if (n_el < 1 || p < 1 || p > 16 || nq < 1 || !nnz || n_el + p - 2 < 1)
    return fail(STIG_EINVAL, "bad 3D assembly");
  const int64_t n = n_el + p - 2;
  if (n * n * n >= ((int64_t)1 << 31)) return fail(STIG_EINVAL, "3D space too large for int32 columns");
  if (rowptr && (!col || !valK || !valM || !c11 || !c22 || !c33 || !c00))
    return fail(STIG_EINVAL, "null 3D assembly array");
  *nnz = assemble_3d(n_el, p, nq, c11, c22, c33, c00, rowptr, col, valK, valM);
  return STIG_OK;
}

stig_status stig_separate_3d(int n1, int n2, int n3, const double *C11, const double *C22,
                             const double *C33, const double *C00, double *phi1, double *phi2,
                             double *phi3, double *Phi1, double *Phi2, double *Phi3) {
  if (n1 < 1 || n2 < 1 || n3 < 1 || !C11 || !C22 || !C33 || !C00 || !phi1 || !phi2 || !phi3 ||
      !Phi1 || !Phi2 || !Phi3)
    return fail(STIG_EINVAL, "bad separation arguments");
  for (int64_t i = 0; i < (int64_t)n1 * n2 * n3; ++i)
    if (!(C11[i] > 0) || !(C22[i] > 0) || !(C33[i] > 0) || !(C00[i] > 0))
      return fail(STIG_EINVAL, "coefficients must be positive");
  separate_3d(n1, n2, n3, C11, C22, C33, C00, phi1, phi2, phi3, Phi1, Phi2, Phi3);
  return STIG_OK;
}

stig_status stig_kron_csr_rowptr(int n_t, int p_t, int64_t ns, const int64_t *rowptr2d,
                                 int64_t *rowptr) {
  if (n_t < 1 || p_t < 0 || ns < 1 || !rowptr2d || !rowptr) return fail(STIG_EINVAL, "bad rowptr");
  rowptr[0] = 0;
  int64_t k = 0;
  for (int t = 0; t < n_t; ++t) {
    int nb = std::min(n_t - 1, t + p_t) - std::max(0, t - p_t) + 1;
    for (int64_t s = 0; s < ns; ++s) {
      k += (int64_t)nb * (rowptr2d[s + 1] - rowptr2d[s]);
      rowptr[(int64_t)t * ns + s + 1] = k;
    }
  }
  return STIG_OK;
}

stig_status stig_kron_csr_fill(stig_plan *p, const int64_t *rowptr, int32_t *col, double *val,
                               const int64_t *rowptr2d, const int32_t *col2d, const double *valM2d,
                               const double *valK2d, const double *Wt, const double *Mt) {
  STIG_TRY(check_plan(p, false));
  if (!rowptr || !col || !val || !rowptr2d || !col2d || !valM2d || !valK2d || !Wt || !Mt)
    return fail(STIG_EINVAL, "null CSR build argument");
  if (p->N >= ((int64_t)1 << 31)) return fail(STIG_EINVAL, "int32 columns cannot index N");
  std::vector<double> wb, mb;
  STIG_TRY(extract_band(Wt, p->nt, p->pt, wb, "W_t"));
  STIG_TRY(extract_band(Mt, p->nt, p->pt, mb, "M_t"));
  DevBuf dw, dm;
  STIG_TRY(upload(dw, wb, p->stream));
  STIG_TRY(upload(dm, mb, p->stream));
  hipLaunchKernelGGL(kron_csr_fill, dim3(grid_for(p->N * 64, 256)), dim3(256), 0, p->stream, rowptr,
                     col, val, rowptr2d, col2d, valM2d, valK2d, dw.as<double>(), dm.as<double>(),
                     p->pt, p->nt, p->Ns);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(p->stream));
  return STIG_OK;
}

stig_status stig_set_A_csr(stig_plan *p, const int64_t *rowptr, const int32_t *col,
                           const double *val, int64_t nnz) {
  STIG_TRY(check_plan(p, false));
  if (!rowptr) {
    p->csr_rowptr = nullptr;
    return STIG_OK;
  }
  if (!col || !val || nnz < 0) return fail(STIG_EINVAL, "bad CSR arrays");
  p->ell_w[0] = p->ell_w[1] = 0;
  p->csr_rowptr = rowptr;
  p->csr_col = col;
  p->csr_val = val;
  p->csr_nnz = nnz;
  return STIG_OK;
}

stig_status stig_set_spatial_factors(stig_plan *p, const int64_t *rowptr, const int32_t *col,
                                     const double *valM, const double *valK) {
  STIG_TRY(check_plan(p, false));
  if (!rowptr) {
    p->ell_w[0] = p->ell_w[1] = 0;
    for (int q = 0; q < 2; ++q) {
      p->ellC[q].release();
      p->ellM[q].release();
      p->ellK[q].release();
      p->ellR[q].release();
      p->ell_nruns[q] = 0;
    }
    return STIG_OK;
  }
  if (!col || !valM || !valK) return fail(STIG_EINVAL, "null spatial factor array");
  std::vector<int32_t> ce[2];
  std::vector<double> me[2], ke[2];
  int w[2];
  bool dia[2];
  for (int q = 0; q < 2; ++q) {
    // by diagonals when there are at most 5/4 as many as entries in the longest row
    const int wr = spatial_ell(p->Ns, rowptr, col, valM, valK, q == 1, ELL_KU, nullptr, nullptr,
                               nullptr);
    if (wr < 0) return fail(STIG_EINVAL, "spatial factors: bad row pointers or columns");
    const int nd = spatial_dia(p->Ns, rowptr, col, valM, valK, q == 1, ELL_KU, wr + wr / 4,
                               &ce[q], &me[q], &ke[q]);
    dia[q] = nd > 0;
    w[q] = dia[q] ? nd
                  : spatial_ell(p->Ns, rowptr, col, valM, valK, q == 1, ELL_KU, &ce[q], &me[q],
                                &ke[q]);
  }
  p->ell_w[0] = p->ell_w[1] = 0;
  for (int q = 0; q < 2; ++q) {
    STIG_TRY(upload(p->ellC[q], ce[q], p->stream));
    STIG_TRY(upload(p->ellM[q], me[q], p->stream));
    STIG_TRY(upload(p->ellK[q], ke[q], p->stream));
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->ell_w[0] = w[0];
  p->ell_w[1] = w[1];
  p->ell_dia[0] = dia[0];
  p->ell_dia[1] = dia[1];
  for (int q = 0; q < 2; ++q) {
    p->ell_omin[q] = dia[q] ? ce[q].front() : 0;  // offsets ascending
    p->ell_omax[q] = dia[q] ? ce[q].back() : 0;
    p->ell_nruns[q] = 0;
    if (!dia[q]) continue;
    // maximal runs of consecutive offsets, at most ELL_RUN_MAX diagonals each
    std::vector<int32_t> runs;
    for (int k = 0; k < w[q]; ++k) {
      const int nr = (int)runs.size() / 3;
      if (nr > 0 && ce[q][k] == ce[q][k - 1] + 1 && runs[3 * (nr - 1) + 1] < ELL_RUN_MAX) {
        ++runs[3 * (nr - 1) + 1];
      } else {
        runs.push_back(ce[q][k]);
        runs.push_back(1);
        runs.push_back(k);
      }
    }
    STIG_TRY(upload(p->ellR[q], runs, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->ell_nruns[q] = (int)runs.size() / 3;
  }
  p->csr_rowptr = nullptr;
  return STIG_OK;
}

stig_status stig_apply_Pinv(stig_plan *p, const double *r, double *s, int nrhs, int transpose,
                            stig_prec prec) {
  STIG_TRY(check_plan(p, true));
  if (!r || !s || nrhs < 1) return fail(STIG_EINVAL, "bad apply arguments");
  if (r == s) return fail(STIG_EINVAL, "r and s must not overlap");
  if (prec != STIG_FP64 && prec != STIG_FP32 && prec != STIG_BF16)
    return fail(STIG_EINVAL, "unknown precision");
  STIG_TRY(bind_workspace(p, nrhs, prec, WS_APPLY));
  return apply_dispatch(p, r, s, nrhs, transpose ? 1 : 0, prec);
}

stig_status stig_apply_Pinv_noalloc(stig_plan *p, const double *r, double *s, int nrhs,
                                    int transpose, stig_prec prec) {
  STIG_TRY(check_plan(p, true));
  if (!r || !s || nrhs < 1) return fail(STIG_EINVAL, "bad apply arguments");
  if (r == s) return fail(STIG_EINVAL, "r and s must not overlap");
  if (prec != STIG_FP64 && prec != STIG_FP32 && prec != STIG_BF16)
    return fail(STIG_EINVAL, "unknown precision");
  const WsLayout L = ws_layout(p, nrhs, prec, WS_APPLY, 0, 0);
  if (L.total > STATIC_SCRATCH_BYTES)
    return fail(STIG_EINVAL, "the allocation-free apply needs " + std::to_string(L.total) +
                                 " bytes of scratch; its static scratch holds " +
                                 std::to_string(STATIC_SCRATCH_BYTES) +
                                 " (use stig_apply_Pinv with a workspace)");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) return fail(STIG_EINVAL, "the plan's device is not the current device");
  char *base = nullptr;
  STIG_TRY(static_scratch(dev, &base));
  lay_views(p, L, base, WS_APPLY, 0);
  return apply_dispatch(p, r, s, nrhs, transpose ? 1 : 0, prec);
}

stig_status stig_matvec_A(stig_plan *p, const double *x, double *y, int nrhs, int transpose) {
  STIG_TRY(check_plan(p, true));
  if (!x || !y || nrhs < 1 || x == y) return fail(STIG_EINVAL, "bad matvec arguments");
  STIG_TRY(bind_workspace(p, nrhs, STIG_FP64, WS_MATVEC));
  return run_matvec(p, x, y, nrhs, transpose ? 1 : 0);
}

size_t stig_workspace_bytes(const stig_plan *p, int restart, int flexible, stig_prec prec,
                            int nrhs) {
  (void)flexible;  // GMRES and FGMRES keep the same vectors
  if (!p || nrhs < 1 || restart < 0 || restart > KRY_MAXV - 1) return 0;
  if (prec != STIG_FP64 && prec != STIG_FP32 && prec != STIG_BF16) return 0;
  size_t need = ws_layout(p, nrhs, prec, WS_ALL, 0, 0).total;
  if (restart > 0) {
    const int nb = std::min(nrhs, KRY_MAXB);
    need = std::max(need, ws_layout(p, nb, prec, WS_APPLY | WS_MATVEC, nb, restart).total);
  }
  return need;
}

stig_status stig_set_workspace(stig_plan *p, void *ws, size_t bytes) {
  STIG_TRY(check_plan(p, false));
  if (ws && (reinterpret_cast<uintptr_t>(ws) % WS_ALIGN))
    return fail(STIG_EINVAL, "workspace must be aligned to 256 bytes");
  p->ws = static_cast<char *>(ws);
  p->ws_bytes = ws ? bytes : 0;
  return STIG_OK;
}

stig_status stig_apply_mass(stig_plan *p, const double *z, double *y, int nrhs) {
  STIG_TRY(check_plan(p, true));
  if (!z || !y || nrhs < 1 || z == y) return fail(STIG_EINVAL, "bad mass-apply arguments");
  const int64_t tot = p->N * nrhs;
  STIG_TRY(bind_workspace(p, nrhs, STIG_FP64, WS_MASS));
  // the mass chain alternates between slots 0 and 2
  Span *bufs[4] = {&p->m0, nullptr, &p->m1, nullptr};
  STIG_TRY(p->m0.ensure(tot * sizeof(double)));
  STIG_TRY(p->m1.ensure(tot * sizeof(double)));
  const double *a, *b;
  STIG_TRY(spatial_chain(p, z, tot, false, &a, &b, bufs));
  return band_pass(p, p->pt, a, nullptr, y, nullptr, p->tM64.as<double>(), nullptr, nullptr, p->nt,
                   p->Ns, tot);
}

stig_status stig_lift_adjoint(stig_plan *p, const double *a_col, const double *b_col,
                              const double *lam, double *g, int nrhs) {
  STIG_TRY(check_plan(p, true));
  if (!a_col || !b_col || !lam || !g || nrhs < 1) return fail(STIG_EINVAL, "bad lift arguments");
  const int64_t ts = p->Ns * nrhs;
  STIG_TRY(bind_workspace(p, nrhs, STIG_FP64, WS_LIFT));
  double *wa = p->liftw.as<double>(), *wbv = wa + p->nt;
  HIP_TRY(hipMemcpyAsync(wa, a_col, p->nt * sizeof(double), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(wbv, b_col, p->nt * sizeof(double), hipMemcpyHostToDevice, p->stream));
  hipLaunchKernelGGL(time_weighted_sum, dim3(grid_for(ts, 256)), dim3(256), 0, p->stream, lam,
                     p->lift0.as<double>(), wa, p->nt, p->Ns, nrhs);
  hipLaunchKernelGGL(time_weighted_sum, dim3(grid_for(ts, 256)), dim3(256), 0, p->stream, lam,
                     p->lift1.as<double>(), wbv, p->nt, p->Ns, nrhs);
  HIP_TRY(hipGetLastError());
  Span *bufs[4] = {&p->m0, &p->m1, &p->m2, &p->m3};
  const double *ma, *dummy, *sa, *sb;
  STIG_TRY(spatial_chain(p, p->lift0.as<double>(), ts, false, &ma, &dummy, bufs));
  // keep the mass result: copy it to g scaled, before the buffers are reused
  hipLaunchKernelGGL(stig::axpby, dim3(grid_for(ts, 256, 8192)), dim3(256), 0, p->stream, ma,
                     nullptr, g, -p->gamma, 0.0, ts);
  HIP_TRY(hipGetLastError());
  STIG_TRY(spatial_chain(p, p->lift1.as<double>(), ts, true, &sa, &sb, bufs));
  hipLaunchKernelGGL(stig::axpby, dim3(grid_for(ts, 256, 8192)), dim3(256), 0, p->stream, g, sb,
                     g, 1.0, -p->nu, ts);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(p->stream));  // the host weights are read by the copies above
  return STIG_OK;
}

stig_status stig_lift_apply(stig_plan *p, const double *a_col, const double *b_col,
                            const double *c0, const double *f, double *y, int nrhs) {
  STIG_TRY(check_plan(p, true));
  if (!a_col || !b_col || !c0 || !y || nrhs < 1) return fail(STIG_EINVAL, "bad lift arguments");
  const int64_t ts = p->Ns * nrhs;
  std::vector<double> ab(2 * (size_t)p->nt);
  for (int t = 0; t < p->nt; ++t) {
    ab[t] = p->gamma * a_col[t];
    ab[p->nt + t] = p->nu * b_col[t];
  }
  STIG_TRY(bind_workspace(p, nrhs, STIG_FP64, WS_LIFT));
  double *wa = p->liftw.as<double>(), *wbv = wa + p->nt;
  HIP_TRY(hipMemcpyAsync(wa, ab.data(), 2 * p->nt * sizeof(double), hipMemcpyHostToDevice,
                         p->stream));
  Span *bufs[4] = {&p->m0, &p->m1, &p->m2, &p->m3};
  const double *ma, *dummy, *sa, *sb;
  STIG_TRY(spatial_chain(p, c0, ts, false, &ma, &dummy, bufs));
  // keep M_s c0 aside before the buffers are reused by the stiffness chain
  hipLaunchKernelGGL(stig::axpby, dim3(grid_for(ts, 256, 8192)), dim3(256), 0, p->stream, ma,
                     nullptr, p->lift0.as<double>(), 1.0, 0.0, ts);
  HIP_TRY(hipGetLastError());
  STIG_TRY(spatial_chain(p, c0, ts, true, &sa, &sb, bufs));
  hipLaunchKernelGGL(time_outer2, dim3(grid_for(ts, 256)), dim3(256), 0, p->stream,
                     p->lift0.as<double>(), sb, wa, wbv, f, y, p->nt, p->Ns, nrhs);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(p->stream));  // ab is read by the copy above
  return STIG_OK;
}

stig_status stig_gmres_solve(stig_plan *p, const double *f, double *u, int nrhs, int restart,
                             double rtol, int maxit, int flexible, int transpose, stig_prec prec,
                             stig_info *info) {
  STIG_TRY(check_plan(p, true));
  if (!f || !u || nrhs < 1 || f == u) return fail(STIG_EINVAL, "bad solve arguments");
  if (restart < 1 || restart > KRY_MAXV - 1) return fail(STIG_EINVAL, "restart must be 1..32");
  if (!(rtol > 0.0) || maxit < 1) return fail(STIG_EINVAL, "rtol must be > 0 and maxit >= 1");
  if (prec != STIG_FP64 && !flexible)
    return fail(STIG_EINVAL, "a low-precision preconditioner needs flexible GMRES");
  auto t0 = std::chrono::steady_clock::now();
  stig_info worst{0, 0, 0.0, 0.0, 0.0};
  stig_status result = STIG_OK;
  auto merge = [&](const stig_info &one) {
    worst.iters = std::max(worst.iters, one.iters);
    worst.restarts = std::max(worst.restarts, one.restarts);
    worst.relres_true = std::max(worst.relres_true, one.relres_true);
    worst.relres_est = std::max(worst.relres_est, one.relres_est);
  };
  // Batches: the first restart cycle of up to nb right-hand sides in lockstep,
  // nb the largest count (at most KRY_MAXB) whose bases, products and
  // intermediates fit the workspace; right-hand sides it leaves above rtol
  // continue one by one from their current iterate.
  int nb = std::min(nrhs, KRY_MAXB);
  while (nb > 1 &&
         ws_layout(p, nb, prec, WS_APPLY | WS_MATVEC, nb, restart).total > p->ws_bytes)
    --nb;
  STIG_TRY(bind_workspace(p, nb, prec, WS_APPLY | WS_MATVEC, nb, restart));
  for (int r0 = 0; r0 < nrhs; r0 += nb) {
    const int cnt = std::min(nb, nrhs - r0);
    std::vector<stig_info> first(cnt, stig_info{0, 0, 0.0, 0.0, 0.0});
    std::vector<char> dn(cnt, 0);
    if (cnt > 1) {
      std::unique_ptr<bool[]> d(new bool[cnt]);
      STIG_TRY(gmres_batch(p, f + r0 * p->N, u + r0 * p->N, cnt, restart, rtol, maxit,
                           transpose ? 1 : 0, prec, first.data(), d.get()));
      for (int i = 0; i < cnt; ++i) dn[i] = d[i];
    }
    for (int i = 0; i < cnt; ++i) {
      const int r = r0 + i;
      if (dn[i]) {
        merge(first[i]);
        continue;
      }
      const int used = first[i].iters;
      if (cnt > 1 && used >= maxit) {  // budget spent in the batched cycle
        result = STIG_NOT_CONVERGED;
        merge(first[i]);
        continue;
      }
      stig_info one{0, 0, 0.0, 0.0, 0.0};
      stig_status st = gmres_one(p, f + r * p->N, u + r * p->N, restart, rtol, maxit - used,
                                 flexible, transpose ? 1 : 0, prec, &one);
      if (st < 0) return st;
      if (st == STIG_NOT_CONVERGED) result = st;
      one.iters += used;
      if (cnt > 1 && used > 0) one.restarts += 1;
      merge(one);
    }
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  worst.t_solve_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = worst;
  return result;
}

stig_status stig_profile_enable(stig_plan *p, int on) {
  STIG_TRY(check_plan(p, false));
  if (!on) STIG_TRY(prof_collect(p));
  p->prof = on != 0;
  return STIG_OK;
}

stig_status stig_profile_reset(stig_plan *p) {
  STIG_TRY(check_plan(p, false));
  STIG_TRY(prof_collect(p));
  for (int k = 0; k < STIG_NUM_KERNEL_KINDS; ++k) {
    p->prof_ms[k] = 0.0;
    p->prof_bytes[k] = 0.0;
    p->prof_count[k] = 0;
  }
  return STIG_OK;
}

stig_status stig_profile_get(stig_plan *p, int kind, double *total_ms, double *bytes,
                             long long *launches) {
  STIG_TRY(check_plan(p, false));
  if (kind < 0 || kind >= STIG_NUM_KERNEL_KINDS) return fail(STIG_EINVAL, "bad kernel kind");
  STIG_TRY(prof_collect(p));
  if (total_ms) *total_ms = p->prof_ms[kind];
  if (bytes) *bytes = p->prof_bytes[kind];
  if (launches) *launches = p->prof_count[kind];
  return STIG_OK;
}

size_t stig_plan_device_bytes(const stig_plan *p) {
  if (!p) return 0;
  size_t t = 0;
  const DevBuf *bs[] = {&p->lam, &p->lamp[0], &p->lamp[1], &p->lamp[2], &p->aTf[0], &p->aTf[1],
                        &p->aTf[2], &p->aTb[0], &p->aTb[1], &p->aTb[2], &p->aTab64[0],
                        &p->aTab64[1], &p->aTab32[0], &p->aTab32[1], &p->aGf[0], &p->aGf[1],
                        &p->aGf[2], &p->aGb[0], &p->aGb[1], &p->aGb[2], &p->aGtab64[0],
                        &p->aGtab64[1], &p->aGtab32[0], &p->aGtab32[1], &p->tW64, &p->tWT64, &p->tM64,
                        &p->tW32, &p->tWT32, &p->tM32, &p->tR64[0], &p->tR64[1], &p->tR32[0],
                        &p->tR32[1], &p->tgW, &p->tgWT, &p->tnM, &p->dmh, &p->sId, &p->sZero,
                        &p->partial, &p->small, &p->flag};
  for (auto *b : bs) t += b->bytes;
  for (int l = 0; l < 3; ++l) {
    t += p->U64[l].bytes + p->UT64[l].bytes + p->U32[l].bytes + p->UT32[l].bytes +
         p->U16[l].bytes + p->UT16[l].bytes + p->sK[l].bytes + p->sM[l].bytes;
  for (int q = 0; q < 2; ++q)
    t += p->ellC[q].bytes + p->ellM[q].bytes + p->ellK[q].bytes + p->ellR[q].bytes;
    for (int q = 0; q < 3; ++q)
      t += p->hFE[q][l].bytes + p->hFO[q][l].bytes + p->hBE[q][l].bytes + p->hBO[q][l].bytes;
  }
  return t;
}

stig_status stig_quadrature(int n_el, int nq, double length, double *x, double *w) {
  if (n_el < 1 || nq < 1 || !x || !w || !(length > 0)) return fail(STIG_EINVAL, "bad quadrature");
  std::vector<double> xs, ws;
  element_quadrature(n_el, nq, length, xs, ws);
  std::copy(xs.begin(), xs.end(), x);
  std::copy(ws.begin(), ws.end(), w);
  return STIG_OK;
}

stig_status stig_assemble_1d(int n_el, int p, double length, int kind, const double *weight,
                             int nq, double *out) {
  if (n_el < 1 || p < 1 || p > 16 || kind < 0 || kind > 2 || !out || !(length > 0))
    return fail(STIG_EINVAL, "bad 1D assembly arguments");
  assemble_1d(n_el, p, length, kind, weight, nq, out);
  return STIG_OK;
}

stig_status stig_load_1d(int n_el, int p, double length, const double *fvals, int nq,
                         double *out) {
  if (n_el < 1 || p < 1 || nq < 1 || !fvals || !out || !(length > 0))
    return fail(STIG_EINVAL, "bad 1D load arguments");
  load_1d(n_el, p, length, fvals, nq, out);
  return STIG_OK;
}

stig_status stig_sym_eig(int n, const double *K, const double *M, double *U, double *lam) {
  if (n < 1 || !K || !M || !U || !lam) return fail(STIG_EINVAL, "bad eigenproblem arguments");
  if (!sym_eig(n, K, M, U, lam)) return fail(STIG_EBREAKDOWN, "M is not positive definite");
  return STIG_OK;
}

stig_status stig_time_arrowhead(int n, const double *W, const double *M, double *U, double *D,
                                int *nzero) {
  if (n < 2 || !W || !M || !U || !D || !nzero) return fail(STIG_EINVAL, "bad arrowhead arguments");
  if (!time_arrowhead(n, W, M, 1e-10, U, D, nzero))
    return fail(STIG_EBREAKDOWN, "no arrowhead factorization (M not SPD or structure not reached)");
  return STIG_OK;
}

stig_status stig_split_eig(int n, const double *K, const double *M, double *U, double *lam) {
  if (n < 2 || !K || !M || !U || !lam) return fail(STIG_EINVAL, "bad eigenproblem arguments");
  if (!persymmetric(n, K, 1e-13) || !persymmetric(n, M, 1e-13))
    return fail(STIG_EINVAL, "pencil is not persymmetric");
  if (!split_eig(n, K, M, U, lam)) return fail(STIG_EBREAKDOWN, "M is not positive definite");
  return STIG_OK;
}

}  // extern "C"

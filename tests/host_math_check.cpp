// Drives the host-side math of libstig (quadrature, B-spline evaluation, 1D and
// 2D assembly, coefficient separation, the generalized and parity-split
// eigensolvers, the arrowhead factorization of the time pencil) on the CPU, so
// that it can run under AddressSanitizer and UndefinedBehaviorSanitizer, and
// checks the identities each routine must satisfy.  Exit status = number of
// failed checks.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "../paper_1909_07309_amd/csrc/stig_internal.h"

using namespace stig;
typedef std::vector<double> Vec;

static int fails = 0;
static void check(bool ok, const char *what, int a, int b, double v) {
  if (!ok) {
    std::printf("FAIL %s (%d, %d): %.3e\n", what, a, b, v);
    ++fails;
  }
}

// rows/columns [lo, lo + k) of an m x m matrix
static Vec sub(const Vec &A, int m, int lo, int k) {
  Vec B((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) B[(size_t)i * k + j] = A[(size_t)(lo + i) * m + lo + j];
  return B;
}

// max |X^T A Y - R| over the n x n result
static double congruence_err(int n, const Vec &X, const Vec &A, const Vec &Y, const Vec &R) {
  double err = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k)
        for (int l = 0; l < n; ++l) v += X[(size_t)k * n + i] * A[(size_t)k * n + l] * Y[(size_t)l * n + j];
      err = std::max(err, std::fabs(v - R[(size_t)i * n + j]));
    }
  return err;
}

int main() {
  // Gauss-Legendre: weights sum to 2, x^(2nq-2) integrated exactly
  for (int nq = 1; nq <= 12; ++nq) {
    Vec x, w;
    gauss_legendre(nq, x, w);
    double sw = 0.0, sp = 0.0;
    for (int i = 0; i < nq; ++i) {
      sw += w[i];
      sp += w[i] * std::pow(x[i], 2 * nq - 2);
    }
    check(std::fabs(sw - 2.0) < 1e-13, "gauss weights", nq, 0, sw - 2.0);
    check(std::fabs(sp - 2.0 / (2 * nq - 1)) < 1e-13, "gauss exactness", nq, 0, sp);
  }
  for (int p = 1; p <= 5; ++p)
    for (int n_el : {1, 2, 5, 17, 48, 64}) {
      if (n_el > 17 && p != 3) continue;  // the cube workloads' sizes
      const int m = n_el + p;
      // partition of unity and zero derivative sum at interior points
      for (int e = 0; e < n_el; ++e) {
        Vec N(p + 1), D(p + 1);
        const double xe = (e + 0.37) / n_el;
        span_basis(e, n_el, p, 1.0, xe, N.data(), D.data());
        double sn = 0.0, sd = 0.0;
        for (int a = 0; a <= p; ++a) {
          sn += N[a];
          sd += D[a];
        }
        check(std::fabs(sn - 1.0) < 1e-13 && std::fabs(sd) < 1e-10, "partition of unity", p, e, sn);
      }
      Vec M((size_t)m * m), K((size_t)m * m), W((size_t)m * m);
      assemble_1d(n_el, p, 1.0, 0, nullptr, p + 1, M.data());
      assemble_1d(n_el, p, 1.0, 1, nullptr, p + 1, K.data());
      assemble_1d(n_el, p, 1.0, 2, nullptr, p + 1, W.data());
      double tot = 0.0, ksum = 0.0, wid = 0.0, sym = 0.0;
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
          tot += M[(size_t)i * m + j];
          ksum = std::max(ksum, std::fabs(K[(size_t)i * m + j] - K[(size_t)j * m + i]));
          sym = std::max(sym, std::fabs(M[(size_t)i * m + j] - M[(size_t)j * m + i]));
          // W + W^T = b_i b_j evaluated from 0 to 1 = e_m e_m^T - e_1 e_1^T
          const double e = (i == m - 1 && j == m - 1) ? 1.0 : ((i == 0 && j == 0) ? -1.0 : 0.0);
          wid = std::max(wid, std::fabs(W[(size_t)i * m + j] + W[(size_t)j * m + i] - e));
        }
      check(std::fabs(tot - 1.0) < 1e-13, "mass total", p, n_el, tot - 1.0);
      check(sym < 1e-15 && ksum < 1e-12, "symmetry", p, n_el, std::max(sym, ksum));
      check(wid < 1e-12, "W + W^T identity", p, n_el, wid);
      Vec ones((size_t)(n_el * (p + 1)), 1.0), load(m);
      load_1d(n_el, p, 1.0, ones.data(), p + 1, load.data());
      double ls = 0.0;
      for (double v : load) ls += v;
      check(std::fabs(ls - 1.0) < 1e-13, "load of 1", p, n_el, ls - 1.0);
      // spatial pencil on the restricted space, both eigenbases
      const int n = m - 2;
      if (n >= 1) {
        Vec Ks = sub(K, m, 1, n), Ms = sub(M, m, 1, n), U((size_t)n * n), lam(n), I((size_t)n * n, 0.0),
            L((size_t)n * n, 0.0);
        check(sym_eig(n, Ks.data(), Ms.data(), U.data(), lam.data()), "sym_eig", p, n_el, 0.0);
        for (int i = 0; i < n; ++i) {
          I[(size_t)i * n + i] = 1.0;
          L[(size_t)i * n + i] = lam[i];
        }
        const double scale = std::max(1.0, lam[n - 1]);
        check(congruence_err(n, U, Ms, U, I) < 1e-11, "U^T M U = I", p, n_el, congruence_err(n, U, Ms, U, I));
        check(congruence_err(n, U, Ks, U, L) < 1e-11 * scale, "U^T K U = Lambda", p, n_el,
              congruence_err(n, U, Ks, U, L));
        for (int i = 1; i < n; ++i) check(lam[i] >= lam[i - 1], "ascending", p, i, lam[i]);
        check(persymmetric(n, Ks.data(), 1e-13) && persymmetric(n, Ms.data(), 1e-13), "persymmetric", p,
              n_el, 0.0);
        Vec Us((size_t)n * n), ls2(n), L2((size_t)n * n, 0.0);
        check(split_eig(n, Ks.data(), Ms.data(), Us.data(), ls2.data()), "split_eig", p, n_el, 0.0);
        for (int i = 0; i < n; ++i) L2[(size_t)i * n + i] = ls2[i];
        check(congruence_err(n, Us, Ms, Us, I) < 1e-11, "split U^T M U = I", p, n_el,
              congruence_err(n, Us, Ms, Us, I));
        check(congruence_err(n, Us, Ks, Us, L2) < 1e-11 * scale, "split U^T K U = Lambda", p, n_el,
              congruence_err(n, Us, Ks, Us, L2));
        const int ne = n / 2 + n % 2;
        for (int k = 0; k < n; ++k)
          for (int x = 0; x < n; ++x) {
            const double a = Us[(size_t)x * n + k], b = Us[(size_t)(n - 1 - x) * n + k];
            check(k < ne ? a == b : a == -b, "exact parity", k, x, a - (k < ne ? b : -b));
          }
      }
      // time pencil (first function removed) and its arrowhead factorization
      const int nt = m - 1;
      if (nt >= 2) {
        Vec Wt = sub(W, m, 1, nt), Mt = sub(M, m, 1, nt), Ut((size_t)nt * nt), Dt((size_t)nt * nt);
        int nzero = -1;
        const bool ok = time_arrowhead(nt, Wt.data(), Mt.data(), 1e-10, Ut.data(), Dt.data(), &nzero);
        check(ok, "time_arrowhead", p, n_el, 0.0);
        if (ok) {
          Vec I((size_t)nt * nt, 0.0);
          for (int i = 0; i < nt; ++i) I[(size_t)i * nt + i] = 1.0;
          check(congruence_err(nt, Ut, Mt, Ut, I) < 1e-10, "arrow U^T M U = I", p, n_el,
                congruence_err(nt, Ut, Mt, Ut, I));
          check(congruence_err(nt, Ut, Wt, Ut, Dt) < 1e-10, "arrow U^T W U = D", p, n_el,
                congruence_err(nt, Ut, Wt, Ut, Dt));
          check(nzero == (nt - 1) % 2, "zero modes", p, n_el, nzero);
        }
      }
    }
  // 2D assembly with unit coefficients = Kronecker forms of the 1D matrices
  for (int p = 1; p <= 4; ++p) {
    const int n_el = 6, nq = p + 3, m = n_el + p, n = m - 2, nqt = n_el * nq;
    Vec c((size_t)nqt * nqt, 1.0);
    const int64_t nnz = assemble_2d(n_el, p, nq, c.data(), c.data(), c.data(), nullptr, nullptr,
                                    nullptr, nullptr);
    std::vector<int64_t> rp((size_t)n * n + 1);
    std::vector<int32_t> col(nnz);
    Vec vK(nnz), vM(nnz);
    check(assemble_2d(n_el, p, nq, c.data(), c.data(), c.data(), rp.data(), col.data(), vK.data(),
                      vM.data()) == nnz,
          "2d nnz", p, 0, (double)nnz);
    Vec M((size_t)m * m), K((size_t)m * m);
    assemble_1d(n_el, p, 1.0, 0, nullptr, p + 1, M.data());
    assemble_1d(n_el, p, 1.0, 1, nullptr, p + 1, K.data());
    Vec Ms = sub(M, m, 1, n), Ks = sub(K, m, 1, n);
    double err = 0.0;
    for (int64_t s = 0; s < (int64_t)n * n; ++s) {
      check(rp[s + 1] > rp[s], "row pointers", p, (int)s, 0.0);
      const int i1 = (int)(s % n), i2 = (int)(s / n);
      for (int64_t k = rp[s]; k < rp[s + 1]; ++k) {
        check(col[k] >= 0 && col[k] < n * n && (k == rp[s] || col[k] > col[k - 1]), "columns", p,
              (int)k, col[k]);
        const int j1 = col[k] % n, j2 = col[k] / n;
        const double m1 = Ms[(size_t)i1 * n + j1], m2 = Ms[(size_t)i2 * n + j2];
        const double k1 = Ks[(size_t)i1 * n + j1], k2 = Ks[(size_t)i2 * n + j2];
        err = std::max(err, std::fabs(vM[k] - m1 * m2));
        err = std::max(err, std::fabs(vK[k] - (k1 * m2 + m1 * k2)));
      }
    }
    check(err < 1e-12, "2d = Kronecker forms", p, 0, err);
  }
  // separation is exact for products of univariate factors
  {
    const int n1 = 5, n2 = 7;
    Vec C11(n1 * n2), C22(n1 * n2), C33(n1 * n2), f1(n1), f2(n2), F1(n1), F2(n2);
    for (int e2 = 0; e2 < n2; ++e2)
      for (int e1 = 0; e1 < n1; ++e1) {
        const double a = 1.0 + 0.1 * e1, b = 2.0 - 0.05 * e2;
        C33[(size_t)e2 * n1 + e1] = a * b;
        C11[(size_t)e2 * n1 + e1] = (0.5 + e1) * b;
        C22[(size_t)e2 * n1 + e1] = a * (1.5 + 0.2 * e2);
      }
    separate_2d(n1, n2, C11.data(), C22.data(), C33.data(), f1.data(), f2.data(), F1.data(), F2.data());
    double err = 0.0;
    for (int e2 = 0; e2 < n2; ++e2)
      for (int e1 = 0; e1 < n1; ++e1) {
        const size_t g = (size_t)e2 * n1 + e1;
        err = std::max(err, std::fabs(f1[e1] * f2[e2] - C33[g]) / C33[g]);
        err = std::max(err, std::fabs(F1[e1] * f2[e2] - C11[g]) / C11[g]);
        err = std::max(err, std::fabs(f1[e1] * F2[e2] - C22[g]) / C22[g]);
      }
    check(err < 1e-13, "separation", n1, n2, err);
  }
  // padded column-major copy of a sparse pair: dense reconstruction of the matrix and of its
  // transpose, padding with column i and value 0, and rejection of bad input
  {
    const int64_t n = 7;
    // irregular pattern: row i holds columns (i * 3 + j * 5) % n for j < 1 + i % 4 (distinct)
    std::vector<int64_t> rp(n + 1, 0);
    std::vector<int32_t> col;
    Vec vM, vK, DM(n * n, 0.0), DK(n * n, 0.0);
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t j = 0; j < 1 + i % 4; ++j) {
        const int32_t c = (int32_t)((i * 3 + j * 5) % n);
        col.push_back(c);
        vM.push_back(1.0 + i + 0.1 * c);
        vK.push_back(-2.0 + 0.5 * i - 0.3 * c);
        DM[i * n + c] += vM.back();
        DK[i * n + c] += vK.back();
      }
      rp[i + 1] = (int64_t)col.size();
    }
    for (int tr = 0; tr < 2; ++tr) {
      std::vector<int32_t> ce;
      Vec me, ke;
      const int align = tr ? 3 : 1;
      const int w =
          spatial_ell(n, rp.data(), col.data(), vM.data(), vK.data(), tr == 1, align, &ce, &me, &ke);
      check(w == spatial_ell(n, rp.data(), col.data(), vM.data(), vK.data(), tr == 1, align, nullptr,
                             nullptr, nullptr),
            "ell width query", tr, w, 0.0);
      int longest = 0;
      for (int64_t i = 0; i < n; ++i) {
        int len = 0;
        for (int64_t e = 0; e < rp[n]; ++e) len += tr ? (col[e] == i) : (e >= rp[i] && e < rp[i + 1]);
        longest = std::max(longest, len);
      }
      check(w == (longest + align - 1) / align * align && ce.size() == (size_t)(w * n), "ell width", tr,
            w, longest);
      Vec RM(n * n, 0.0), RK(n * n, 0.0);
      for (int64_t k = 0; k < w; ++k)
        for (int64_t i = 0; i < n; ++i) {
          const size_t e = (size_t)(k * n + i);
          check(ce[e] >= 0 && ce[e] < n, "ell column range", tr, (int)e, ce[e]);
          if (me[e] == 0.0 && ke[e] == 0.0) check(ce[e] == i, "ell padding column", tr, (int)e, ce[e]);
          RM[i * n + ce[e]] += me[e];
          RK[i * n + ce[e]] += ke[e];
        }
      double err = 0.0;
      for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
          const size_t src = tr ? (size_t)(j * n + i) : (size_t)(i * n + j);
          err = std::max(err, std::fabs(RM[i * n + j] - DM[src]) + std::fabs(RK[i * n + j] - DK[src]));
        }
      check(err == 0.0, "ell reproduces the matrix", tr, 0, err);
    }
    std::vector<int32_t> bad = col;
    bad[3] = (int32_t)n;
    check(spatial_ell(n, rp.data(), bad.data(), vM.data(), vK.data(), false, 1, nullptr, nullptr, nullptr) ==
              -1,
          "ell rejects a column out of range", 0, 0, 0.0);
    std::vector<int64_t> brp = rp;
    brp[4] = brp[3] - 1;
    check(spatial_ell(n, brp.data(), col.data(), vM.data(), vK.data(), true, 1, nullptr, nullptr, nullptr) ==
              -1,
          "ell rejects decreasing row pointers", 0, 0, 0.0);
  }
  // diagonal layout: dense reconstruction of the matrix and its transpose (with a duplicate
  // entry, summed), clamped padding, and the diagonal-count limit
  {
    const int64_t n = 9;
    std::vector<int64_t> rp(n + 1, 0);
    std::vector<int32_t> col;
    Vec vM, vK, DM(n * n, 0.0), DK(n * n, 0.0);
    const int offsets[4] = {-3, -1, 0, 2};
    for (int64_t i = 0; i < n; ++i) {
      for (int o : offsets) {
        const int64_t j = i + o;
        if (j < 0 || j >= n || (i + o) % 4 == 3) continue;  // a few holes away from the boundary
        col.push_back((int32_t)j);
        vM.push_back(1.0 + 0.5 * i - 0.25 * j);
        vK.push_back(2.0 - 0.125 * i + 0.75 * j);
        DM[i * n + j] += vM.back();
        DK[i * n + j] += vK.back();
      }
      if (i == 4) {  // a duplicate of (4, 4)
        col.push_back(4);
        vM.push_back(0.5);
        vK.push_back(-1.5);
        DM[4 * n + 4] += 0.5;
        DK[4 * n + 4] += -1.5;
      }
      rp[i + 1] = (int64_t)col.size();
    }
    for (int tr = 0; tr < 2; ++tr) {
      std::vector<int32_t> offs;
      Vec me, ke;
      const int nd = spatial_dia(n, rp.data(), col.data(), vM.data(), vK.data(), tr == 1, 3, 64, &offs,
                                 &me, &ke);
      check(nd == 6 && offs.size() == 6 && me.size() == (size_t)(6 * n), "dia count", tr, nd, 0.0);
      for (int k = 1; k < nd; ++k) check(offs[k] >= offs[k - 1], "dia offsets ascending", tr, k, offs[k]);
      Vec RM(n * n, 0.0), RK(n * n, 0.0);
      double pad = 0.0;
      for (int64_t k = 0; k < nd; ++k)
        for (int64_t i = 0; i < n; ++i) {
          const size_t e = (size_t)(k * n + i);
          const int64_t j = i + offs[k];
          if (j < 0 || j >= n) {
            pad = std::max(pad, std::fabs(me[e]) + std::fabs(ke[e]));
            continue;
          }
          if (k > 0 && offs[k] == offs[k - 1]) {  // alignment padding repeats the last offset
            pad = std::max(pad, std::fabs(me[e]) + std::fabs(ke[e]));
            continue;
          }
          RM[i * n + j] += me[e];
          RK[i * n + j] += ke[e];
        }
      check(pad == 0.0, "dia padding is zero", tr, 0, pad);
      double err = 0.0;
      for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
          const size_t src = tr ? (size_t)(j * n + i) : (size_t)(i * n + j);
          err = std::max(err, std::fabs(RM[i * n + j] - DM[src]) + std::fabs(RK[i * n + j] - DK[src]));
        }
      check(err < 1e-15, "dia reproduces the matrix", tr, 0, err);
    }
    check(spatial_dia(n, rp.data(), col.data(), vM.data(), vK.data(), false, 1, 3, nullptr, nullptr,
                      nullptr) == 0,
          "dia gives up beyond the limit", 0, 0, 0.0);
    std::vector<int32_t> bad = col;
    bad[2] = -1;
    check(spatial_dia(n, rp.data(), bad.data(), vM.data(), vK.data(), false, 1, 64, nullptr, nullptr,
                      nullptr) == -1,
          "dia rejects a bad column", 0, 0, 0.0);
  }
  std::printf("%s: %d failed checks\n", fails ? "host math FAILED" : "host math ok", fails);
  return fails;
}

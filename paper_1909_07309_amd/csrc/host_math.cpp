// Host-side numerics of libstig: Gauss-Legendre rules, B-spline evaluation,
// 1D Galerkin matrices and the symmetric-definite eigensolver of the setup step.
//
// B-splines (Section 2.1): open uniform knot vector with p+1 repeated end knots
// and n_el-1 simple interior knots, so m = n_el + p functions of maximal
// continuity.  On a knot span only p+1 functions are nonzero; they are computed
// with the triangular de Boor table (the Cox-de Boor recursion restricted to
// the nonzero functions), and derivatives from the degree p-1 values.
//
// Eigensolver (step 1 of Algorithm 1, eq. space_eig): K U = M U Lambda with
// U^T M U = I.  With M = L L^T (Cholesky), C = L^{-1} K L^{-T} is symmetric;
// cyclic Jacobi rotations diagonalise C = Q Lambda Q^T; U = L^{-T} Q.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <stdexcept>
#include <vector>

#include "stig_internal.h"

namespace stig {

void gauss_legendre(int nq, std::vector<double> &x, std::vector<double> &w) {
  // Nodes on [-1, 1]: Newton iteration on P_nq from the Chebyshev-like guess,
  // P_n evaluated with the three-term recurrence (n+1)P_{n+1} = (2n+1)xP_n - nP_{n-1}.
  x.assign(nq, 0.0);
  w.assign(nq, 0.0);
  for (int i = 0; i < nq; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (nq + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= nq; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (nq == 1) { p1 = z; p0 = 1.0; }
      dp = nq * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= nq; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (nq == 1) { p1 = z; p0 = 1.0; }
      dp = nq * (z * p1 - p0) / (z * z - 1.0);
    }
    x[nq - 1 - i] = z;  // ascending order
    w[nq - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void element_quadrature(int n_el, int nq, double length, std::vector<double> &x,
                        std::vector<double> &w) {
  std::vector<double> g, gw;
  gauss_legendre(nq, g, gw);
  x.resize((size_t)n_el * nq);
  w.resize((size_t)n_el * nq);
  double h = length / n_el;
  for (int e = 0; e < n_el; ++e)
    for (int q = 0; q < nq; ++q) {
      x[(size_t)e * nq + q] = e * h + 0.5 * h * (g[q] + 1.0);
      w[(size_t)e * nq + q] = 0.5 * h * gw[q];
    }
}

// Knot value xi_j (0-based, j = 0 .. m+p) of the open uniform knot vector.
static inline double knot(int j, int n_el, int p, double length) {
  int k = j - p;  // interior index
  if (k <= 0) return 0.0;
  if (k >= n_el) return length;
  return length * (double)k / n_el;
}

// Values N[0..p] and derivatives D[0..p] of the p+1 B-splines that are nonzero on
// element e (functions e .. e+p, 0-based) at the point x inside that element.
void span_basis(int e, int n_el, int p, double length, double x, double *N, double *D) {
  // de Boor triangle: degree-k values of functions e+p-k .. e+p on span [xi_{e+p}, xi_{e+p+1})
  std::vector<double> left(p + 1), right(p + 1), val(p + 1, 0.0), prev(p + 1, 0.0);
  int s = e + p;  // index of the span's left knot
  val[0] = 1.0;
  for (int k = 1; k <= p; ++k) {
    left[k] = x - knot(s + 1 - k, n_el, p, length);
    right[k] = knot(s + k, n_el, p, length) - x;
    if (k == p) std::copy(val.begin(), val.begin() + p, prev.begin());  // degree p-1 values
    double saved = 0.0;
    for (int r = 0; r < k; ++r) {
      double den = right[r + 1] + left[k - r];
      double t = den != 0.0 ? val[r] / den : 0.0;
      val[r] = saved + right[r + 1] * t;
      saved = left[k - r] * t;
    }
    val[k] = saved;
  }
  for (int r = 0; r <= p; ++r) N[r] = val[r];
  if (D) {
    if (p == 0) { D[0] = 0.0; return; }
    // prev[0..p-1]: degree p-1 functions e+1 .. e+p (global indices), nonzero on the span.
    // b'_{i,p} = p/(xi_{i+p}-xi_i) b_{i,p-1} - p/(xi_{i+p+1}-xi_{i+1}) b_{i+1,p-1}
    for (int r = 0; r <= p; ++r) {
      int i = e + r;  // global function index
      double a = 0.0, b = 0.0;
      // b_{i,p-1} nonzero on this span iff e+1 <= i <= e+p  -> prev[i-e-1]
      if (i >= e + 1) {
        double den = knot(i + p, n_el, p, length) - knot(i, n_el, p, length);
        if (den != 0.0) a = p / den * prev[i - e - 1];
      }
      if (i + 1 <= e + p) {
        double den = knot(i + p + 1, n_el, p, length) - knot(i + 1, n_el, p, length);
        if (den != 0.0) b = p / den * prev[i + 1 - e - 1];
      }
      D[r] = a - b;
    }
  }
}

void assemble_1d(int n_el, int p, double length, int kind, const double *weight, int nq,
                 double *out) {
  if (nq <= 0) nq = p + 1;
  int m = n_el + p;
  std::fill(out, out + (size_t)m * m, 0.0);
  std::vector<double> x, w;
  element_quadrature(n_el, nq, length, x, w);
  std::vector<double> N(p + 1), D(p + 1);
  for (int e = 0; e < n_el; ++e)
    for (int q = 0; q < nq; ++q) {
      size_t iq = (size_t)e * nq + q;
      span_basis(e, n_el, p, length, x[iq], N.data(), D.data());
      double c = w[iq] * (weight ? weight[iq] : 1.0);
      for (int a = 0; a <= p; ++a)
        for (int b = 0; b <= p; ++b) {
          double v;
          if (kind == 0) v = N[a] * N[b];
          else if (kind == 1) v = D[a] * D[b];
          else v = D[b] * N[a];  // row i = test function (value), column j = trial (derivative)
          out[(size_t)(e + a) * m + (e + b)] += c * v;
        }
    }
}

void load_1d(int n_el, int p, double length, const double *fvals, int nq, double *out) {
  int m = n_el + p;
  std::fill(out, out + m, 0.0);
  std::vector<double> x, w;
  element_quadrature(n_el, nq, length, x, w);
  std::vector<double> N(p + 1);
  for (int e = 0; e < n_el; ++e)
    for (int q = 0; q < nq; ++q) {
      size_t iq = (size_t)e * nq + q;
      span_basis(e, n_el, p, length, x[iq], N.data(), nullptr);
      for (int a = 0; a <= p; ++a) out[e + a] += w[iq] * fvals[iq] * N[a];
    }
}

int64_t assemble_2d(int n_el, int p, int nq, const double *c11, const double *c22,
                    const double *c33, int64_t *rowptr, int32_t *col, double *valK, double *valM) {
  // Restricted (Dirichlet) tensor-product space on (0,1)^2, n = n_el + p - 2 per
  // direction, unknown s = i1 + n * i2.  Pattern: all j with |i1-j1| <= p and
  // |i2-j2| <= p inside the grid (the overlap pattern of the B-splines).
  const int n = n_el + p - 2;
  const int64_t Ns = (int64_t)n * n;
  if (!rowptr) {  // size query
    int64_t nnz = 0;
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1) {
        int w1 = std::min(n - 1, i1 + p) - std::max(0, i1 - p) + 1;
        int w2 = std::min(n - 1, i2 + p) - std::max(0, i2 - p) + 1;
        nnz += (int64_t)w1 * w2;
      }
    return nnz;
  }
  rowptr[0] = 0;
  for (int64_t s = 0; s < Ns; ++s) {
    int i1 = (int)(s % n), i2 = (int)(s / n);
    int64_t k = rowptr[s];
    for (int j2 = std::max(0, i2 - p); j2 <= std::min(n - 1, i2 + p); ++j2)
      for (int j1 = std::max(0, i1 - p); j1 <= std::min(n - 1, i1 + p); ++j1) {
        col[k] = j1 + n * j2;
        valK[k] = 0.0;
        valM[k] = 0.0;
        ++k;
      }
    rowptr[s + 1] = k;
  }
  // element loop: local functions e + a (unrestricted) -> restricted e + a - 1
  std::vector<double> x, w;
  element_quadrature(n_el, nq, 1.0, x, w);
  std::vector<double> N1((size_t)nq * (p + 1)), D1((size_t)nq * (p + 1));
  std::vector<double> N2((size_t)nq * (p + 1)), D2((size_t)nq * (p + 1));
  const int nqt = n_el * nq;  // points per direction
  for (int e2 = 0; e2 < n_el; ++e2) {
    for (int k2 = 0; k2 < nq; ++k2)
      span_basis(e2, n_el, p, 1.0, x[(size_t)e2 * nq + k2], &N2[(size_t)k2 * (p + 1)],
                 &D2[(size_t)k2 * (p + 1)]);
    for (int e1 = 0; e1 < n_el; ++e1) {
      for (int k1 = 0; k1 < nq; ++k1)
        span_basis(e1, n_el, p, 1.0, x[(size_t)e1 * nq + k1], &N1[(size_t)k1 * (p + 1)],
                   &D1[(size_t)k1 * (p + 1)]);
      for (int a2 = 0; a2 <= p; ++a2)
        for (int a1 = 0; a1 <= p; ++a1) {
          int i1 = e1 + a1 - 1, i2 = e2 + a2 - 1;
          if (i1 < 0 || i1 >= n || i2 < 0 || i2 >= n) continue;
          int64_t row = (int64_t)i1 + (int64_t)n * i2;
          for (int b2 = 0; b2 <= p; ++b2)
            for (int b1 = 0; b1 <= p; ++b1) {
              int j1 = e1 + b1 - 1, j2 = e2 + b2 - 1;
              if (j1 < 0 || j1 >= n || j2 < 0 || j2 >= n) continue;
              double kv = 0.0, mv = 0.0;
              for (int k2 = 0; k2 < nq; ++k2)
                for (int k1 = 0; k1 < nq; ++k1) {
                  size_t g = (size_t)(e2 * nq + k2) * nqt + (size_t)(e1 * nq + k1);
                  double ww = w[(size_t)e2 * nq + k2] * w[(size_t)e1 * nq + k1];
                  double n1a = N1[k1 * (p + 1) + a1], n1b = N1[k1 * (p + 1) + b1];
                  double n2a = N2[k2 * (p + 1) + a2], n2b = N2[k2 * (p + 1) + b2];
                  double d1a = D1[k1 * (p + 1) + a1], d1b = D1[k1 * (p + 1) + b1];
                  double d2a = D2[k2 * (p + 1) + a2], d2b = D2[k2 * (p + 1) + b2];
                  kv += ww * (c11[g] * d1a * d1b * n2a * n2b + c22[g] * n1a * n1b * d2a * d2b);
                  mv += ww * c33[g] * n1a * n1b * n2a * n2b;
                }
              // locate column (j1, j2) in row's pattern
              int lo1 = std::max(0, i1 - p), lo2 = std::max(0, i2 - p);
              int wd1 = std::min(n - 1, i1 + p) - lo1 + 1;
              int64_t k = rowptr[row] + (int64_t)(j2 - lo2) * wd1 + (j1 - lo1);
              valK[k] += kv;
              valM[k] += mv;
            }
        }
    }
  }
  return rowptr[Ns];
}

void separate_2d(int n1, int n2, const double *C11, const double *C22, const double *C33,
                 double *phi1, double *phi2, double *Phi1, double *Phi2) {
  // Rank-one fits in log space of element-midpoint samples [e2][e1]:
  //   log phi1(e1) = mean_e2 log C33,  log phi2(e2) = mean_e1 log C33 - mean log C33,
  //   log Phi1(e1) = mean_e2 log(C11 / phi2),  log Phi2(e2) = mean_e1 log(C22 / phi1).
  // Exact whenever the sampled coefficient is itself a product of univariate factors.
  double tot = 0.0;
  std::vector<double> r1(n1, 0.0), r2(n2, 0.0);
  for (int e2 = 0; e2 < n2; ++e2)
    for (int e1 = 0; e1 < n1; ++e1) {
      double l = std::log(C33[(size_t)e2 * n1 + e1]);
      r1[e1] += l;
      r2[e2] += l;
      tot += l;
    }
  tot /= (double)n1 * n2;
  for (int e1 = 0; e1 < n1; ++e1) phi1[e1] = std::exp(r1[e1] / n2);
  for (int e2 = 0; e2 < n2; ++e2) phi2[e2] = std::exp(r2[e2] / n1 - tot);
  for (int e1 = 0; e1 < n1; ++e1) {
    double acc = 0.0;
    for (int e2 = 0; e2 < n2; ++e2) acc += std::log(C11[(size_t)e2 * n1 + e1] / phi2[e2]);
    Phi1[e1] = std::exp(acc / n2);
  }
  for (int e2 = 0; e2 < n2; ++e2) {
    double acc = 0.0;
    for (int e1 = 0; e1 < n1; ++e1) acc += std::log(C22[(size_t)e2 * n1 + e1] / phi1[e1]);
    Phi2[e2] = std::exp(acc / n1);
  }
}

int64_t assemble_3d(int n_el, int p, int nq, const double *c11, const double *c22,
                    const double *c33, const double *c00, int64_t *rowptr, int32_t *col,
                    double *valK, double *valM) {
  // Restricted tensor-product space on (0,1)^3, n = n_el + p - 2 per direction,
  // unknown s = i1 + n (i2 + n i3); pattern: |i_l - j_l| <= p in every direction.
  const int n = n_el + p - 2;
  const int64_t Ns = (int64_t)n * n * n;
  auto width = [&](int i) { return std::min(n - 1, i + p) - std::max(0, i - p) + 1; };
  if (!rowptr) {  // size query
    int64_t w = 0;
    for (int i = 0; i < n; ++i) w += width(i);
    return w * w * w;
  }
  rowptr[0] = 0;
  for (int64_t s = 0; s < Ns; ++s) {
    const int i1 = (int)(s % n), i2 = (int)((s / n) % n), i3 = (int)(s / ((int64_t)n * n));
    int64_t k = rowptr[s];
    for (int j3 = std::max(0, i3 - p); j3 <= std::min(n - 1, i3 + p); ++j3)
      for (int j2 = std::max(0, i2 - p); j2 <= std::min(n - 1, i2 + p); ++j2)
        for (int j1 = std::max(0, i1 - p); j1 <= std::min(n - 1, i1 + p); ++j1) {
          col[k] = j1 + n * (j2 + n * j3);
          valK[k] = 0.0;
          valM[k] = 0.0;
          ++k;
        }
    rowptr[s + 1] = k;
  }
  std::vector<double> x, w;
  element_quadrature(n_el, nq, 1.0, x, w);
  const int P1 = p + 1, nqt = n_el * nq;
  // basis values / derivatives at the points of every element: [e][k][a]
  std::vector<double> Nv((size_t)n_el * nq * P1), Dv((size_t)n_el * nq * P1);
  for (int e = 0; e < n_el; ++e)
    for (int k = 0; k < nq; ++k)
      span_basis(e, n_el, p, 1.0, x[(size_t)e * nq + k], &Nv[((size_t)e * nq + k) * P1],
                 &Dv[((size_t)e * nq + k) * P1]);
  const size_t L6 = (size_t)P1 * P1 * P1 * P1 * P1 * P1;
  std::vector<double> T1((size_t)nq * nq * P1 * P1), T2((size_t)nq * P1 * P1 * P1 * P1);
  std::vector<double> locK(L6), locM(L6);
  // one term: loc += sum_q c(q) w(q) F3 G3 F2 G2 F1 G1 (F, G = values or derivatives),
  // contracted one direction at a time
  auto term = [&](const double *c, bool d1, bool d2, bool d3, int e1, int e2, int e3,
                  std::vector<double> &loc) {
    const double *B1 = &(d1 ? Dv : Nv)[(size_t)e1 * nq * P1];
    const double *B2 = &(d2 ? Dv : Nv)[(size_t)e2 * nq * P1];
    const double *B3 = &(d3 ? Dv : Nv)[(size_t)e3 * nq * P1];
    const double *w1 = &w[(size_t)e1 * nq], *w2 = &w[(size_t)e2 * nq], *w3 = &w[(size_t)e3 * nq];
    // T1[k3][k2][a1][b1]
    for (int k3 = 0; k3 < nq; ++k3)
      for (int k2 = 0; k2 < nq; ++k2) {
        double *t = &T1[((size_t)k3 * nq + k2) * P1 * P1];
        std::fill(t, t + P1 * P1, 0.0);
        for (int k1 = 0; k1 < nq; ++k1) {
          const size_t g = ((size_t)(e3 * nq + k3) * nqt + (e2 * nq + k2)) * nqt + (e1 * nq + k1);
          const double cw = c[g] * w1[k1];
          for (int a1 = 0; a1 < P1; ++a1)
            for (int b1 = 0; b1 < P1; ++b1) t[a1 * P1 + b1] += cw * B1[k1 * P1 + a1] * B1[k1 * P1 + b1];
        }
      }
    // T2[k3][a2][b2][a1][b1]
    for (int k3 = 0; k3 < nq; ++k3) {
      double *t2 = &T2[(size_t)k3 * P1 * P1 * P1 * P1];
      std::fill(t2, t2 + P1 * P1 * P1 * P1, 0.0);
      for (int k2 = 0; k2 < nq; ++k2) {
        const double *t = &T1[((size_t)k3 * nq + k2) * P1 * P1];
        for (int a2 = 0; a2 < P1; ++a2)
          for (int b2 = 0; b2 < P1; ++b2) {
            const double f = w2[k2] * B2[k2 * P1 + a2] * B2[k2 * P1 + b2];
            double *o = t2 + (a2 * P1 + b2) * P1 * P1;
            for (int ab = 0; ab < P1 * P1; ++ab) o[ab] += f * t[ab];
          }
      }
    }
    // loc[a3][b3][a2][b2][a1][b1]
    for (int k3 = 0; k3 < nq; ++k3) {
      const double *t2 = &T2[(size_t)k3 * P1 * P1 * P1 * P1];
      for (int a3 = 0; a3 < P1; ++a3)
        for (int b3 = 0; b3 < P1; ++b3) {
          const double f = w3[k3] * B3[k3 * P1 + a3] * B3[k3 * P1 + b3];
          double *o = &loc[(size_t)(a3 * P1 + b3) * P1 * P1 * P1 * P1];
          for (int r = 0; r < P1 * P1 * P1 * P1; ++r) o[r] += f * t2[r];
        }
    }
  };
  for (int e3 = 0; e3 < n_el; ++e3)
    for (int e2 = 0; e2 < n_el; ++e2)
      for (int e1 = 0; e1 < n_el; ++e1) {
        std::fill(locK.begin(), locK.end(), 0.0);
        std::fill(locM.begin(), locM.end(), 0.0);
        term(c11, true, false, false, e1, e2, e3, locK);
        term(c22, false, true, false, e1, e2, e3, locK);
        term(c33, false, false, true, e1, e2, e3, locK);
        term(c00, false, false, false, e1, e2, e3, locM);
        for (int a3 = 0; a3 < P1; ++a3)
          for (int a2 = 0; a2 < P1; ++a2)
            for (int a1 = 0; a1 < P1; ++a1) {
              const int i1 = e1 + a1 - 1, i2 = e2 + a2 - 1, i3 = e3 + a3 - 1;
              if (i1 < 0 || i1 >= n || i2 < 0 || i2 >= n || i3 < 0 || i3 >= n) continue;
              const int64_t row = i1 + (int64_t)n * (i2 + (int64_t)n * i3);
              const int lo1 = std::max(0, i1 - p), lo2 = std::max(0, i2 - p), lo3 = std::max(0, i3 - p);
              const int wd1 = width(i1), wd2 = width(i2);
              for (int b3 = 0; b3 < P1; ++b3)
                for (int b2 = 0; b2 < P1; ++b2)
                  for (int b1 = 0; b1 < P1; ++b1) {
                    const int j1 = e1 + b1 - 1, j2 = e2 + b2 - 1, j3 = e3 + b3 - 1;
                    if (j1 < 0 || j1 >= n || j2 < 0 || j2 >= n || j3 < 0 || j3 >= n) continue;
                    const size_t li = ((((size_t)(a3 * P1 + b3) * P1 + a2) * P1 + b2) * P1 + a1) * P1 + b1;
                    const int64_t k =
                        rowptr[row] + ((int64_t)(j3 - lo3) * wd2 + (j2 - lo2)) * wd1 + (j1 - lo1);
                    valK[k] += locK[li];
                    valM[k] += locM[li];
                  }
            }
      }
  return rowptr[Ns];
}

int spatial_ell(int64_t n, const int64_t *rowptr, const int32_t *col, const double *valM,
                const double *valK, bool transpose, int align, std::vector<int32_t> *ce,
                std::vector<double> *me, std::vector<double> *ke) {
  if (rowptr[0] != 0) return -1;
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return -1;
  const int64_t nnz = rowptr[n];
  for (int64_t e = 0; e < nnz; ++e)
    if (col[e] < 0 || col[e] >= n) return -1;
  // row lengths of the stored matrix (of the transpose: column counts)
  std::vector<int64_t> len(n, 0);
  if (transpose) {
    for (int64_t e = 0; e < nnz; ++e) ++len[col[e]];
  } else {
    for (int64_t i = 0; i < n; ++i) len[i] = rowptr[i + 1] - rowptr[i];
  }
  int64_t width = 0;
  for (int64_t i = 0; i < n; ++i) width = std::max(width, len[i]);
  align = std::max(align, 1);
  width = (std::max<int64_t>(width, 1) + align - 1) / align * align;
  if (!ce) return (int)width;
  ce->assign((size_t)(width * n), 0);
  me->assign((size_t)(width * n), 0.0);
  ke->assign((size_t)(width * n), 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = 0; k < width; ++k) (*ce)[(size_t)(k * n + i)] = (int32_t)i;
  std::vector<int64_t> fill(n, 0);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      // stored entry (i, j): (r, col) or, for the transpose, (col, r)
      const int64_t i = transpose ? col[e] : r, j = transpose ? r : col[e];
      const size_t slot = (size_t)(fill[i]++ * n + i);
      (*ce)[slot] = (int32_t)j;
      (*me)[slot] = valM[e];
      (*ke)[slot] = valK[e];
    }
  return (int)width;
}

int spatial_dia(int64_t n, const int64_t *rowptr, const int32_t *col, const double *valM,
                const double *valK, bool transpose, int align, int max_diags,
                std::vector<int32_t> *offs, std::vector<double> *me, std::vector<double> *ke) {
  if (rowptr[0] != 0) return -1;
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return -1;
  const int64_t nnz = rowptr[n];
  for (int64_t e = 0; e < nnz; ++e)
    if (col[e] < 0 || col[e] >= n) return -1;
  // distinct offsets of the stored matrix (transpose: offsets negated)
  // sorted set of the offsets seen so far (at most max_diags + 1 of them)
  std::vector<int64_t> o;
  for (int64_t r = 0; r < n; ++r)
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      const int64_t d = transpose ? r - col[e] : col[e] - r;
      auto it = std::lower_bound(o.begin(), o.end(), d);
      if (it == o.end() || *it != d) {
        o.insert(it, d);
        if ((int64_t)o.size() > max_diags) return 0;
      }
    }
  if (o.empty()) o.push_back(0);
  align = std::max(align, 1);
  const int64_t nd = ((int64_t)o.size() + align - 1) / align * align;
  if (nd > max_diags) return 0;
  if (!offs) return (int)nd;
  offs->assign((size_t)nd, 0);
  for (int64_t k = 0; k < nd; ++k) (*offs)[(size_t)k] = (int32_t)o[std::min<int64_t>(k, o.size() - 1)];
  me->assign((size_t)(nd * n), 0.0);
  ke->assign((size_t)(nd * n), 0.0);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      const int64_t i = transpose ? col[e] : r, j = transpose ? r : col[e];
      const int64_t k = std::lower_bound(o.begin(), o.end(), j - i) - o.begin();
      (*me)[(size_t)(k * n + i)] += valM[e];
      (*ke)[(size_t)(k * n + i)] += valK[e];
    }
  return (int)nd;
}

void separate_3d(int n1, int n2, int n3, const double *C11, const double *C22, const double *C33,
                 const double *C00, double *phi1, double *phi2, double *phi3, double *Phi1,
                 double *Phi2, double *Phi3) {
  // Rank-one fits in log space of element-midpoint samples [e3][e2][e1]: the
  // mass coefficient C00 ~ phi1(e1) phi2(e2) phi3(e3) with
  //   log phi1 = mean over (e2, e3) of log C00,
  //   log phi_l = mean over the other two of log C00 - mean log C00  (l = 2, 3),
  // and C_ll ~ Phi_l(e_l) prod_{m != l} phi_m with log Phi_l the mean over the
  // other two directions of log(C_ll / prod_{m != l} phi_m).  Exact whenever
  // the samples are products of univariate factors.
  const size_t tot_n = (size_t)n1 * n2 * n3;
  std::vector<double> r1(n1, 0.0), r2(n2, 0.0), r3(n3, 0.0);
  double tot = 0.0;
  auto at = [&](int e1, int e2, int e3) { return ((size_t)e3 * n2 + e2) * n1 + e1; };
  for (int e3 = 0; e3 < n3; ++e3)
    for (int e2 = 0; e2 < n2; ++e2)
      for (int e1 = 0; e1 < n1; ++e1) {
        const double l = std::log(C00[at(e1, e2, e3)]);
        r1[e1] += l;
        r2[e2] += l;
        r3[e3] += l;
        tot += l;
      }
  tot /= (double)tot_n;
  for (int e1 = 0; e1 < n1; ++e1) phi1[e1] = std::exp(r1[e1] / ((double)n2 * n3));
  for (int e2 = 0; e2 < n2; ++e2) phi2[e2] = std::exp(r2[e2] / ((double)n1 * n3) - tot);
  for (int e3 = 0; e3 < n3; ++e3) phi3[e3] = std::exp(r3[e3] / ((double)n1 * n2) - tot);
  std::vector<double> s1(n1, 0.0), s2(n2, 0.0), s3(n3, 0.0);
  for (int e3 = 0; e3 < n3; ++e3)
    for (int e2 = 0; e2 < n2; ++e2)
      for (int e1 = 0; e1 < n1; ++e1) {
        const size_t g = at(e1, e2, e3);
        s1[e1] += std::log(C11[g] / (phi2[e2] * phi3[e3]));
        s2[e2] += std::log(C22[g] / (phi1[e1] * phi3[e3]));
        s3[e3] += std::log(C33[g] / (phi1[e1] * phi2[e2]));
      }
  for (int e1 = 0; e1 < n1; ++e1) Phi1[e1] = std::exp(s1[e1] / ((double)n2 * n3));
  for (int e2 = 0; e2 < n2; ++e2) Phi2[e2] = std::exp(s2[e2] / ((double)n1 * n3));
  for (int e3 = 0; e3 < n3; ++e3) Phi3[e3] = std::exp(s3[e3] / ((double)n1 * n2));
}

// Returns false if M is not positive definite.
bool sym_eig(int n, const double *K, const double *M, double *U, double *lam) {
  std::vector<double> L((size_t)n * n, 0.0);
  // Cholesky M = L L^T (lower)
  for (int j = 0; j < n; ++j) {
    double s = M[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0.0)) return false;
    double d = std::sqrt(s);
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = M[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / d;
    }
  }
  // C = L^{-1} K L^{-T}: first Y = L^{-1} K (forward substitution per column),
  // then C = L^{-1} Y^T (Y^T = K L^{-T} since K is symmetric).
  std::vector<double> Y((size_t)n * n), C((size_t)n * n);
  auto lower_solve = [&](const double *B, double *X) {  // X = L^{-1} B, B n x n row-major
    for (int c = 0; c < n; ++c)
      for (int i = 0; i < n; ++i) {
        double s = B[(size_t)i * n + c];
        for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * X[(size_t)k * n + c];
        X[(size_t)i * n + c] = s / L[(size_t)i * n + i];
      }
  };
  lower_solve(K, Y.data());
  std::vector<double> Yt((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Yt[(size_t)i * n + j] = Y[(size_t)j * n + i];
  lower_solve(Yt.data(), C.data());
  for (int i = 0; i < n; ++i)  // symmetrise rounding
    for (int j = i + 1; j < n; ++j) {
      double a = 0.5 * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
      C[(size_t)i * n + j] = C[(size_t)j * n + i] = a;
    }
  // cyclic Jacobi on C, accumulating rotations in Q
  std::vector<double> Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += C[(size_t)i * n + i] * C[(size_t)i * n + i];
      for (int j = i + 1; j < n; ++j) off += C[(size_t)i * n + j] * C[(size_t)i * n + j];
    }
    if (off <= 1e-34 * diag) break;
    for (int pi = 0; pi < n - 1; ++pi)
      for (int qi = pi + 1; qi < n; ++qi) {
        double apq = C[(size_t)pi * n + qi];
        if (apq == 0.0) continue;
        double app = C[(size_t)pi * n + pi], aqq = C[(size_t)qi * n + qi];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns pi, qi
          double ckp = C[(size_t)k * n + pi], ckq = C[(size_t)k * n + qi];
          C[(size_t)k * n + pi] = c * ckp - s * ckq;
          C[(size_t)k * n + qi] = s * ckp + c * ckq;
        }
        for (int k = 0; k < n; ++k) {  // rows pi, qi
          double cpk = C[(size_t)pi * n + k], cqk = C[(size_t)qi * n + k];
          C[(size_t)pi * n + k] = c * cpk - s * cqk;
          C[(size_t)qi * n + k] = s * cpk + c * cqk;
        }
        C[(size_t)pi * n + qi] = C[(size_t)qi * n + pi] = 0.0;
        for (int k = 0; k < n; ++k) {
          double qkp = Q[(size_t)k * n + pi], qkq = Q[(size_t)k * n + qi];
          Q[(size_t)k * n + pi] = c * qkp - s * qkq;
          Q[(size_t)k * n + qi] = s * qkp + c * qkq;
        }
      }
  }
  // sort ascending
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(),
            [&](int a, int b) { return C[(size_t)a * n + a] < C[(size_t)b * n + b]; });
  // U = L^{-T} Q (back substitution with L^T per column), columns reordered
  for (int cc = 0; cc < n; ++cc) {
    int c = ord[cc];
    lam[cc] = C[(size_t)c * n + c];
    for (int i = n - 1; i >= 0; --i) {
      double s = Q[(size_t)i * n + c];
      for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * U[(size_t)k * n + cc];
      U[(size_t)i * n + cc] = s / L[(size_t)i * n + i];
    }
  }
  // deterministic sign: largest-magnitude entry of each eigenvector positive
  for (int c = 0; c < n; ++c) {
    int imax = 0;
    for (int i = 1; i < n; ++i)
      if (std::fabs(U[(size_t)i * n + c]) > std::fabs(U[(size_t)imax * n + c])) imax = i;
    if (U[(size_t)imax * n + c] < 0)
      for (int i = 0; i < n; ++i) U[(size_t)i * n + c] = -U[(size_t)i * n + c];
  }
  return true;
}

bool persymmetric(int n, const double *A, double tol) {
  double amax = 0.0, dmax = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      amax = std::max(amax, std::abs(A[(size_t)i * n + j]));
      dmax = std::max(dmax, std::abs(A[(size_t)i * n + j] - A[(size_t)(n - 1 - i) * n + (n - 1 - j)]));
    }
  return dmax <= tol * amax;
}

// Parity-split eigenbasis of a persymmetric pencil.  With the orthonormal
// even / odd bases q_x = (e_x +- e_{n-1-x}) / sqrt(2) (x < m = n/2) and, for odd
// n, the middle unit vector e_m (even), K and M become block diagonal; each
// block is a symmetric definite pencil of its own.  Their eigenvectors, mapped
// back, are eigenvectors of (K, M) that are exactly even or odd.
bool split_eig(int n, const double *K, const double *M, double *U, double *lam) {
  const int m = n / 2, odd = n & 1, ne = m + odd;
  const double h = 1.0 / std::sqrt(2.0);
  auto block = [&](const double *A, bool even, std::vector<double> &B) {
    const int nb = even ? ne : m;
    B.assign((size_t)nb * nb, 0.0);
    const double sg = even ? 1.0 : -1.0;
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j) {
        const bool mi = odd && even && i == m, mj = odd && even && j == m;
        double v;
        if (mi && mj) v = A[(size_t)m * n + m];
        else if (mi) v = h * (A[(size_t)m * n + j] + A[(size_t)m * n + (n - 1 - j)]);
        else if (mj) v = h * (A[(size_t)i * n + m] + A[(size_t)(n - 1 - i) * n + m]);
        else
          v = 0.5 * (A[(size_t)i * n + j] + sg * A[(size_t)i * n + (n - 1 - j)] +
                     sg * A[(size_t)(n - 1 - i) * n + j] + A[(size_t)(n - 1 - i) * n + (n - 1 - j)]);
        B[(size_t)i * nb + j] = v;
      }
  };
  std::vector<double> Ke, Me, Ko, Mo, Ve((size_t)ne * ne), Vo((size_t)m * m);
  block(K, true, Ke);
  block(M, true, Me);
  block(K, false, Ko);
  block(M, false, Mo);
  if (!sym_eig(ne, Ke.data(), Me.data(), Ve.data(), lam)) return false;
  if (m > 0 && !sym_eig(m, Ko.data(), Mo.data(), Vo.data(), lam + ne)) return false;
  std::fill(U, U + (size_t)n * n, 0.0);
  for (int k = 0; k < ne; ++k) {
    for (int x = 0; x < m; ++x) {
      U[(size_t)x * n + k] = h * Ve[(size_t)x * ne + k];
      U[(size_t)(n - 1 - x) * n + k] = h * Ve[(size_t)x * ne + k];
    }
    if (odd) U[(size_t)m * n + k] = Ve[(size_t)m * ne + k];
  }
  for (int k = 0; k < m; ++k)
    for (int x = 0; x < m; ++x) {
      U[(size_t)x * n + ne + k] = h * Vo[(size_t)x * m + k];
      U[(size_t)(n - 1 - x) * n + ne + k] = -h * Vo[(size_t)x * m + k];
    }
  return true;
}

// Real block form of the arrowhead factorization of a time pencil (W, M)
// (Section 4.2.2, eq. time_eig_2).  The leading (n-1) blocks W0, M0 have
// W0 + W0^T = 0 (eq. integral_W), so with M0 = L L^T the matrix
// S = L^{-1} W0 L^{-T} is real skew-symmetric.  Its real Schur form
// S = Q B Q^T has 2 x 2 blocks [[0, mu], [-mu, 0]] and, for odd n-1, one zero;
// it is found from the symmetric eigenproblem of S^T S = -S^2 (eigenvalues
// mu^2 twice): for each pair, q1 is an eigenvector (orthogonalised against the
// ones already taken) and q2 = S q1 / |S q1|.  U0 = L^{-T} Q, the last column
// of U is (-M0^{-1} m, 1) normalised in the M norm (eq. syst_v), so that
// U^T M U = I and D = U^T W U is block diagonal plus the last row and column.
// Output (all row-major, modes in the order: zero mode first if n-1 is odd,
// then the pairs, then the last mode): U (n x n), D (n x n); returns false if
// M0 is not SPD or the block structure is not reached to tol relative.
bool time_arrowhead(int n, const double *W, const double *M, double tol, double *U, double *D,
                    int *nzero) {
  const int m = n - 1;
  if (m < 1) return false;
  std::vector<double> L((size_t)m * m, 0.0);
  for (int j = 0; j < m; ++j) {  // Cholesky of M0
    double d = M[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * m + k] * L[(size_t)j * m + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    L[(size_t)j * m + j] = d;
    for (int i = j + 1; i < m; ++i) {
      double v = M[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * m + k] * L[(size_t)j * m + k];
      L[(size_t)i * m + j] = v / d;
    }
  }
  auto lsolve = [&](std::vector<double> &x) {  // x <- L^{-1} x
    for (int i = 0; i < m; ++i) {
      double v = x[i];
      for (int k = 0; k < i; ++k) v -= L[(size_t)i * m + k] * x[k];
      x[i] = v / L[(size_t)i * m + i];
    }
  };
  auto ltsolve = [&](std::vector<double> &x) {  // x <- L^{-T} x
    for (int i = m - 1; i >= 0; --i) {
      double v = x[i];
      for (int k = i + 1; k < m; ++k) v -= L[(size_t)k * m + i] * x[k];
      x[i] = v / L[(size_t)i * m + i];
    }
  };
  // S = L^{-1} W0 L^{-T}, column by column, then skew-symmetrised
  std::vector<double> S((size_t)m * m), col(m);
  std::vector<double> T((size_t)m * m);  // T = W0 L^{-T}  (rows of T^T = L^{-1} W0^T)
  for (int i = 0; i < m; ++i) {  // row i of W0 L^{-T} = (L^{-1} W0[i, :]^T)^T
    for (int k = 0; k < m; ++k) col[k] = W[(size_t)i * n + k];
    lsolve(col);
    for (int k = 0; k < m; ++k) T[(size_t)i * m + k] = col[k];
  }
  for (int j = 0; j < m; ++j) {  // column j of L^{-1} T
    for (int k = 0; k < m; ++k) col[k] = T[(size_t)k * m + j];
    lsolve(col);
    for (int k = 0; k < m; ++k) S[(size_t)k * m + j] = col[k];
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < i; ++j) {
      const double a = 0.5 * (S[(size_t)i * m + j] - S[(size_t)j * m + i]);
      S[(size_t)i * m + j] = a;
      S[(size_t)j * m + i] = -a;
    }
  for (int i = 0; i < m; ++i) S[(size_t)i * m + i] = 0.0;
  // eigenvectors of S^T S
  std::vector<double> StS((size_t)m * m, 0.0), I((size_t)m * m, 0.0), V((size_t)m * m), mu2(m);
  for (int i = 0; i < m; ++i) {
    I[(size_t)i * m + i] = 1.0;
    for (int j = 0; j < m; ++j) {
      double v = 0.0;
      for (int k = 0; k < m; ++k) v += S[(size_t)k * m + i] * S[(size_t)k * m + j];
      StS[(size_t)i * m + j] = v;
    }
  }
  if (!sym_eig(m, StS.data(), I.data(), V.data(), mu2.data())) return false;
  const int nz = m % 2;
  std::vector<std::vector<double>> Q;
  auto ortho = [&](std::vector<double> &x) {
    for (auto &q : Q) {
      double d = 0.0;
      for (int k = 0; k < m; ++k) d += q[k] * x[k];
      for (int k = 0; k < m; ++k) x[k] -= d * q[k];
    }
    double nr = 0.0;
    for (int k = 0; k < m; ++k) nr += x[k] * x[k];
    return std::sqrt(nr);
  };
  for (int idx = 0; idx < m && (int)Q.size() < m; ++idx) {  // ascending mu^2
    std::vector<double> q1(m);
    for (int k = 0; k < m; ++k) q1[k] = V[(size_t)k * m + idx];
    const double nr = ortho(q1);
    if (nr < 0.5) continue;  // partner of a pair already taken
    for (auto &x : q1) x /= nr;
    Q.push_back(q1);
    if (nz && Q.size() == 1) continue;  // the zero mode stands alone
    std::vector<double> q2(m, 0.0);
    for (int i = 0; i < m; ++i)
      for (int k = 0; k < m; ++k) q2[i] += S[(size_t)i * m + k] * q1[k];
    const double n2 = ortho(q2);
    if (!(n2 > 0.0)) return false;
    for (auto &x : q2) x /= n2;
    Q.push_back(q2);
  }
  if ((int)Q.size() != m) return false;
  // U = [[L^{-T} Q, v], [0, c]]
  std::fill(U, U + (size_t)n * n, 0.0);
  for (int j = 0; j < m; ++j) {
    col = Q[j];
    ltsolve(col);
    for (int i = 0; i < m; ++i) U[(size_t)i * n + j] = col[i];
  }
  std::vector<double> v(m);
  for (int i = 0; i < m; ++i) v[i] = -M[(size_t)i * n + m];
  lsolve(v);
  ltsolve(v);  // v = -M0^{-1} m
  std::vector<double> c(n);
  for (int i = 0; i < m; ++i) c[i] = v[i];
  c[m] = 1.0;
  double cmc = 0.0;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) cmc += c[i] * M[(size_t)i * n + k] * c[k];
  const double cs = 1.0 / std::sqrt(cmc);
  for (int i = 0; i < n; ++i) U[(size_t)i * n + m] = c[i] * cs;
  // D = U^T W U
  std::vector<double> WU((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double w = W[(size_t)i * n + k];
      if (w == 0.0) continue;
      for (int j = 0; j < n; ++j) WU[(size_t)i * n + j] += w * U[(size_t)k * n + j];
    }
  double dmax = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v2 = 0.0;
      for (int k = 0; k < n; ++k) v2 += U[(size_t)k * n + i] * WU[(size_t)k * n + j];
      D[(size_t)i * n + j] = v2;
      dmax = std::max(dmax, std::abs(v2));
    }
  // structure check: inside the leading block only the 2 x 2 pair blocks
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const bool inpair = i >= nz && j >= nz && (i - nz) / 2 == (j - nz) / 2 && i != j;
      if (!inpair && std::abs(D[(size_t)i * n + j]) > tol * dmax) return false;
    }
  *nzero = nz;
  return true;
}

}  // namespace stig

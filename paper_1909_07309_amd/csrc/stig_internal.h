// Internal declarations shared by the host translation units of libstig.
#pragma once

#include <cstdint>
#include <vector>

namespace stig {

// Gauss-Legendre rule with nq points on [-1, 1], nodes ascending.
void gauss_legendre(int nq, std::vector<double> &x, std::vector<double> &w);

// nq Gauss points per element of [0, length] split into n_el equal elements.
void element_quadrature(int n_el, int nq, double length, std::vector<double> &x,
                        std::vector<double> &w);

// Values (and derivatives if D != nullptr) of the p+1 B-splines nonzero on
// element e at the point x of that element; function indices e .. e+p.
void span_basis(int e, int n_el, int p, double length, double x, double *N, double *D);

// Dense m x m 1D Galerkin matrix (kind 0 mass, 1 stiffness, 2 advection).
void assemble_1d(int n_el, int p, double length, int kind, const double *weight, int nq,
                 double *out);

// Load vector from values of f at the element quadrature points.
void load_1d(int n_el, int p, double length, const double *fvals, int nq, double *out);

// 2D stiffness / mass on the restricted tensor space from coefficient samples at
// the tensor Gauss grid (see stig_assemble_2d); rowptr == nullptr: size query.
int64_t assemble_2d(int n_el, int p, int nq, const double *c11, const double *c22,
                    const double *c33, int64_t *rowptr, int32_t *col, double *valK, double *valM);

// 3D stiffness / mass on the restricted tensor space (unknown s = i1 + n (i2 +
// n i3)) from coefficient samples at the tensor Gauss grid [q3][q2][q1]:
// K = int c11 d1B d1B + c22 d2B d2B + c33 d3B d3B, M = int c00 B B;
// rowptr == nullptr: size query.
int64_t assemble_3d(int n_el, int p, int nq, const double *c11, const double *c22,
                    const double *c33, const double *c00, int64_t *rowptr, int32_t *col,
                    double *valK, double *valM);

// Padded column-major copy of a square CSR pair (M, K) with one shared pattern
// (or of its transpose pair): entry k of row i at k * n + i, the width the
// longest row rounded up to a multiple of align, shorter rows padded with column
// i and value 0.  Returns the width, or -1 if a column is out of range or rowptr
// is not non-decreasing (outputs untouched).  With ce == nullptr only the width
// is computed.
int spatial_ell(int64_t n, const int64_t *rowptr, const int32_t *col, const double *valM,
                const double *valK, bool transpose, int align, std::vector<int32_t> *ce,
                std::vector<double> *me, std::vector<double> *ke);

// Diagonal layout of the same pair (or of its transpose pair) when it has few
// distinct offsets o = col - row: offs[k] (ascending, padded to a multiple of
// align with repeats of the last offset), and the values of diagonal k of row i
// at k * n + i (zero where row i has no entry at offset o_k; duplicates
// summed).  Returns the number of diagonals, 0 if it would exceed max_diags
// (outputs untouched), -1 on a bad rowptr or column as spatial_ell.  With
// offs == nullptr only the count is computed.
int spatial_dia(int64_t n, const int64_t *rowptr, const int32_t *col, const double *valM,
                const double *valK, bool transpose, int align, int max_diags,
                std::vector<int32_t> *offs, std::vector<double> *me, std::vector<double> *ke);

// Separable (rank-one, log-space) approximation of 3D samples [e3][e2][e1]:
// C00 ~ phi1 phi2 phi3 and C_ll ~ Phi_l prod_{m != l} phi_m.
void separate_3d(int n1, int n2, int n3, const double *C11, const double *C22, const double *C33,
                 const double *C00, double *phi1, double *phi2, double *phi3, double *Phi1,
                 double *Phi2, double *Phi3);

// Separable (rank-one, log-space) approximation of sampled coefficients.
void separate_2d(int n1, int n2, const double *C11, const double *C22, const double *C33,
                 double *phi1, double *phi2, double *Phi1, double *Phi2);

// K U = M U Lambda, U^T M U = I, ascending; false if M is not SPD.
bool sym_eig(int n, const double *K, const double *M, double *U, double *lam);

// max |A[i][j] - A[n-1-i][n-1-j]| <= tol * max |A|.
bool persymmetric(int n, const double *A, double tol);

// Eigenbasis of a persymmetric pencil with the even modes first (n/2 + n%2 of
// them, U[n-1-x][k] = U[x][k]) and the odd modes after (U[n-1-x][k] = -U[x][k]);
// ascending within each group; same normalisation as sym_eig.
bool split_eig(int n, const double *K, const double *M, double *U, double *lam);

// Real block form of the arrowhead factorization of a time pencil: U (n x n)
// with U^T M U = I and D = U^T W U block diagonal (a zero mode first when n-1
// is odd, then 2 x 2 skew blocks) plus the last row and column.
bool time_arrowhead(int n, const double *W, const double *M, double tol, double *U, double *D,
                    int *nzero);

}  // namespace stig

/*
 * stig.h -- C ABI of libstig, an MI355X (gfx950) implementation of the hot path
 * of the space-time isogeometric Galerkin heat-equation solver of Loli,
 * Montardini, Sangalli and Tani (arXiv:1909.07309): applying the Kronecker-sum
 * preconditioner A-hat = gamma W_t (x) M_s + nu M_t (x) K_s by fast
 * diagonalization inside (flexible) GMRES.
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - Unknown tensors are contiguous FP64 arrays in device memory with layout
 *    [rhs][t][x_d]...[x_1] (x_1 fastest): the colexicographic vec of Section 2.3.
 *    One tensor has N = n_t * n_1 * ... * n_d entries; a batch holds nrhs of them.
 *  - "host" pointers are ordinary CPU memory, "device" pointers are HIP device
 *    memory on the plan's device.  The caller owns every buffer it passes; the
 *    library never frees caller memory.
 *  - Memory: the setup calls (stig_setup_1d_pencils, stig_set_diag_scaling*,
 *    stig_set_spatial_factors) allocate the plan's own factors (eigenvector
 *    matrices, shifts, band coefficients, sparse spatial factors: a few MB to a
 *    few hundred MB, reported by stig_plan_device_bytes) and a small pinned host
 *    staging area; stig_plan_destroy frees them.  Everything a call needs beyond
 *    that (the intermediate tensors of the apply, matvec, mass and lifting
 *    products and the Krylov bases of GMRES) lives in a caller-owned device
 *    workspace given by stig_set_workspace and sized by stig_workspace_bytes.
 *    stig_apply_Pinv, stig_matvec_A, stig_apply_mass, stig_lift_* and
 *    stig_gmres_solve never allocate or free device memory.
 *  - Every device operation is ordered on the plan's stream.  stig_apply_Pinv,
 *    stig_matvec_A and stig_apply_mass return as soon as their kernels are
 *    queued; stig_gmres_solve synchronises the stream (the Givens rotations run
 *    on the host) and returns when the solution is written.
 *  - Errors are returned as codes, never thrown across the ABI; a description of
 *    the last error on the calling thread is available from stig_last_error().
 *    Negative codes mean nothing usable was written; positive codes are warnings
 *    with a result written.
 *  - A plan is not thread-safe: calls on one plan must not overlap.
 */
#ifndef STIG_H
#define STIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stig_plan stig_plan;

typedef enum {
  STIG_OK = 0,
  STIG_NOT_CONVERGED = 1,   /* gmres: maxit reached; best iterate written */
  STIG_EINVAL = -1,         /* bad size, null pointer, out-of-band matrix entry */
  STIG_ENOMEM = -2,         /* device allocation failed */
  STIG_EHIP = -3,           /* a HIP runtime call failed */
  STIG_EBREAKDOWN = -4,     /* non-positive pivot in a shifted time system, or
                               non-positive-definite spatial mass matrix */
  STIG_ENONFINITE = -5,     /* NaN/Inf met in a residual norm */
  STIG_ESTATE = -6          /* call made before the setup it needs */
} stig_status;

/* Arithmetic of the fast-diagonalization apply (the mode-k GEMMs and the time
 * solves).  Boundary I/O is FP64 in every case.
 *   STIG_FP64: FP64 MFMA GEMMs, FP64 time solves, FP64 intermediates.
 *   STIG_FP32: FP32 MFMA GEMMs (FP32 accumulation), FP32 time solves and
 *              intermediates.
 *   STIG_BF16: BF16 MFMA operands with FP32 accumulation, FP32 time solves,
 *              BF16 intermediates. */
typedef enum { STIG_FP64 = 0, STIG_FP32 = 1, STIG_BF16 = 2 } stig_prec;

typedef struct {
  int iters;            /* total inner (Arnoldi) iterations over all restarts */
  int restarts;         /* number of restart cycles started after the first */
  double relres_true;   /* ||f - A u||_2 / ||f||_2 at exit, from a fresh FP64
                           product A u (see stig_gmres_solve), not from the GMRES
                           estimate */
  double relres_est;    /* GMRES residual estimate at exit (relative) */
  double t_solve_ms;    /* wall time of the call (host clock, stream synchronised) */
} stig_info;

/* ------------------------------------------------------------- plan lifetime */

/* Create a plan for d spatial dimensions (1 <= d <= 3) with n_s[l] unknowns in
 * direction l+1 (host array of d ints), n_t unknowns in time, spline degrees
 * p_s (space) and p_t (time) that bound the bandwidths of the 1D factors
 * (Section 4.5: bandwidth 2p+1), on HIP stream `stream` (hipStream_t; NULL is
 * the null stream) of the current device.  No device memory is touched.
 * Sizes: 1 <= n_s[l] <= 200, 2 <= n_t <= 1024, 1 <= p_s, p_t <= 5. */
stig_status stig_plan_create(stig_plan **out, int d, const int *n_s, int n_t,
                             int p_s, int p_t, void *stream);

void stig_plan_destroy(stig_plan *plan);

/* Change the stream later calls are ordered on. */
stig_status stig_set_stream(stig_plan *plan, void *stream);

/* Bytes of device workspace that calls with up to nrhs right-hand sides need:
 * stig_apply_Pinv in precision prec, stig_matvec_A, stig_apply_mass and
 * stig_lift_*, and, when restart > 0, stig_gmres_solve with that restart length
 * (its first restart cycle runs up to min(nrhs, 64) right-hand sides in
 * lockstep; with a smaller workspace it runs fewer at a time).  Layout, per
 * right-hand side, of the largest parts: the Krylov bases V (restart + 1
 * vectors), Z = A-hat^{-1} V and A Z (restart vectors each) and one more
 * vector, all FP64 of N entries (Section 4.5: restarted GMRES); the two
 * intermediate tensors of the apply in the storage type of prec (Algorithm 1,
 * steps 2-4).  flexible does not change the size (GMRES and FGMRES keep the
 * same vectors).  The result depends on the plan's setup and options (diagonal
 * scaling, sparse spatial factors or CSR, kernel choices): query it after them.
 * Returns 0 for a NULL plan or arguments out of range. */
size_t stig_workspace_bytes(const stig_plan *plan, int restart, int flexible, stig_prec prec,
                            int nrhs);

/* Give the plan its workspace: ws (device, 256-byte aligned, on the plan's
 * device) of `bytes` bytes, owned by the caller, kept alive and not used for
 * anything else while calls on the plan are queued or running.  Calls check
 * that their part fits (else STIG_EINVAL, nothing launched) and fail with
 * STIG_ESTATE when no workspace was given.  Contents need not be initialised
 * and are not preserved between calls.  ws = NULL detaches it. */
stig_status stig_set_workspace(stig_plan *plan, void *ws, size_t bytes);

/* Kernel choices of apply_Pinv (stig_set_option).  Every choice computes the
 * same result up to rounding order.
 *   STIG_OPT_PLANE_FUSION: 1 (default) = the mode-1 and mode-2 products of
 *     steps 2 and 4 (Section 2.3, Algorithm 1) in one fused pass per plane when
 *     n_s[0] == n_s[1] <= 80 and no diagonal scaling is set; 0 = one pass per mode.
 *   STIG_OPT_TIME_KERNEL: how step 3 treats the shifted time systems.
 *     0 (default): for the register-resident shapes (n_t, p_t) = (66, 3),
 *     (50, 3), (9, 2), banded elimination right-looking with window-state
 *     checkpoints, the forward substitution redone segment by segment in the
 *     backward sweep (nothing stored); for n_t = 131 or 33 with fewer than
 *     262,144 systems per call (N_s times the right-hand sides), the arrowhead
 *     form of 4 (its products along t have a compile-time kernel there); otherwise the
 *     generic banded kernel of 2.
 *     3 = as 0, with the forward-substituted values stored and read back;
 *     1 = left-looking, U-row checkpoints (register shapes; generic otherwise);
 *     2 = the generic banded kernel with scratch memory;
 *     4 = the paper's own form (Section 4.2.2, eq. time_eig_2, eq. block_LU):
 *     the time pencil transformed by the real block form of its arrowhead
 *     factorization (dense products along t on MFMA) and the arrowhead middle
 *     factor solved by block LU: one fused kernel for n_t = 34 and 66, three
 *     passes (product, middle factor, product) for any other n_t <= 200.
 *     STIG_EINVAL for other n_t or when the set-up time pencil has no arrowhead
 *     factorization; stig_setup_1d_pencils returns STIG_EBREAKDOWN if it cannot
 *     build it while 4 is selected.
 *   STIG_OPT_PARITY_SPLIT: 1 (default) = where a spatial pencil is
 *     persymmetric (stig_setup_1d_pencils then picks an eigenbasis of even and
 *     odd modes), its mode products run as two half-size products around a
 *     butterfly (sizes n_s = 32, 33, 64, 65); 0 = dense products.
 * Unknown options or values: STIG_EINVAL. */
enum { STIG_OPT_PLANE_FUSION = 0, STIG_OPT_TIME_KERNEL = 1, STIG_OPT_PARITY_SPLIT = 2 };
stig_status stig_set_option(stig_plan *plan, int option, int value);

/* ------------------------------------------------------------------ setup */

/* Step 1 of Algorithm 1 (Section 4.4) for the banded-time form of A-hat^{-1}.
 *   K1d[l], M1d[l] (host, l = 0..d-1): dense row-major n_s[l] x n_s[l] spatial
 *       stiffness and mass factors of direction l+1 (eq. space_univ_par_mat, or the
 *       geometry-weighted K-tilde_l, M-tilde_l of Section 4.3).  Symmetric, M SPD.
 *   Wt, Mt (host): dense row-major n_t x n_t time factors (eq. time_mat).
 *   gamma, nu: coefficients of eq. prec_definition.
 * The library solves K_l U_l = M_l U_l Lambda_l with U_l^T M_l U_l = I
 * (eq. space_eig) by Cholesky + cyclic Jacobi on the host, uploads U_l, U_l^T,
 * Lambda_l (and FP32/BF16 copies), and the band coefficients of W_t, W_t^T, M_t.
 * The same factors define the matrix-free matvec of stig_matvec_A (the time
 * factors always; the spatial ones unless stig_set_spatial_factors or
 * stig_set_A_csr is called).  Entries outside the bandwidth p_s / p_t must be 0
 * (else STIG_EINVAL).  May be called again to replace the factors. */
stig_status stig_setup_1d_pencils(stig_plan *plan, const double *const *K1d,
                                  const double *const *M1d, const double *Wt,
                                  const double *Mt, double gamma, double nu);

/* Optional: geometry-aware scaling of eq. prec_geo.  D (device, N doubles,
 * layout [t][x_d]..[x_1]) holds D_ii = A_ii / A-tilde_ii > 0.  After this call,
 * stig_apply_Pinv applies (D^{1/2} A-tilde D^{1/2})^{-1} = D^{-1/2} A-tilde^{-1} D^{-1/2},
 * with the D^{-1/2} scalings fused into the first and last spatial passes.
 * The library keeps its own copy of D^{-1/2}.  D = NULL removes the scaling. */
stig_status stig_set_diag_scaling(stig_plan *plan, const double *D);

/* Optional: use an explicit CSR matrix for stig_matvec_A instead of the
 * matrix-free Kronecker form (the quarter-annulus workload of Section 4.3.1,
 * whose spatial factors are not Kronecker products).  Device arrays, owned by
 * the caller and kept alive while the plan uses them: rowptr (N+1 int64),
 * col (nnz int32, sorted within a row), val (nnz FP64).  Pass rowptr = NULL to
 * go back to the matrix-free form.  Transposed products are not supported on
 * the CSR form (STIG_EINVAL). */
stig_status stig_set_A_csr(stig_plan *plan, const int64_t *rowptr,
                           const int32_t *col, const double *val, int64_t nnz);

/* Optional: the matvec of Section 4.5 with sparse spatial factors.  Only the
 * factors of A are stored, not A itself:
 *   A = gamma W_t (x) M_s + nu M_t (x) K_s,
 * with the plan's time factors and general sparse N_s x N_s spatial matrices
 * M_s, K_s (the variable-coefficient and geometry case of Section 4.3.1, whose
 * spatial matrices are not Kronecker products).  Host CSR with one pattern for
 * both: rowptr (N_s + 1 int64, rowptr[0] = 0, non-decreasing), col (int32 in
 * [0, N_s), any order within a row), valM, valK (FP64), spatial unknown order
 * [x_d]..[x_1].  The library keeps its own device copies of M_s, K_s and of
 * their transposes: by diagonals (2 x diagonals x N_s x 16 bytes) when the
 * pattern has at most 5/4 as many distinct offsets col - row as entries in its
 * longest row, as every tensor-product spline pattern does, else as padded rows
 * (2 x width x N_s x 20 bytes, width = the longest row or column); duplicate
 * entries add up.  stig_matvec_A then runs one sparse
 * spatial pass per time level and one banded pass along t; transposed products
 * are supported.  Synchronises.  rowptr = NULL removes the factors.  Setting
 * the factors clears a matrix given to stig_set_A_csr, and setting that matrix
 * clears the factors.  STIG_EINVAL if rowptr or col are out of range (nothing
 * changed). */
stig_status stig_set_spatial_factors(stig_plan *plan, const int64_t *rowptr, const int32_t *col,
                                     const double *valM, const double *valK);

/* Optional: the geometry-aware scaling of eq. prec_geo computed by the library
 * when the true system has the same time factors as the plan and spatial
 * factors M_s, K_s (any sparsity, e.g. a non-separable conductivity): with the
 * host diagonals dMs, dKs (N_s doubles each, [x_d]..[x_1]) of M_s and K_s,
 *   D[t][s] = (gamma W_tt dMs_s + nu M_tt dKs_s) / (gamma W_tt dMs~_s + nu M_tt dKs~_s),
 * where dMs~, dKs~ are the diagonals of the plan's Kronecker factors.  Then as
 * stig_set_diag_scaling(D).  STIG_EBREAKDOWN if a diagonal is not positive. */
stig_status stig_set_diag_scaling_kron(stig_plan *plan, const double *dMs, const double *dKs);

/* ---------------------------------------------- 2D spatial assembly, full CSR */

/* Spatial stiffness and mass on the unit square in parametric coordinates
 * (Section 4.3: the geometry and coefficients enter through the coefficient
 * matrix), for the Dirichlet-restricted open uniform B-spline space of degree p
 * with n_el elements per direction (n = n_el + p - 2 unknowns per direction,
 * unknown s = i_1 + n i_2):
 *   K_ij = int c11 d1B_i d1B_j + c22 d2B_i d2B_j,   M_ij = int c33 B_i B_j,
 * from coefficient values at the tensor Gauss grid (host, [q2][q1] with
 * n_el * nq points per direction, as stig_quadrature).  Output CSR (host):
 * rowptr (n^2 + 1), col (int32, sorted), valK, valM over the B-spline overlap
 * pattern.  With rowptr == NULL only *nnz is returned (size query). */
stig_status stig_assemble_2d(int n_el, int p, int nq, const double *c11, const double *c22,
                             const double *c33, int64_t *rowptr, int32_t *col, double *valK,
                             double *valM, int64_t *nnz);

/* The same in 3D on the unit cube in parametric coordinates (n = n_el + p - 2
 * unknowns per direction, unknown s = i_1 + n (i_2 + n i_3), n^3 < 2^31):
 *   K_ij = int c11 d1B_i d1B_j + c22 d2B_i d2B_j + c33 d3B_i d3B_j,
 *   M_ij = int c00 B_i B_j,
 * from coefficient values at the tensor Gauss grid (host, [q3][q2][q1] with
 * n_el * nq points per direction).  Output CSR (host): rowptr (n^3 + 1), col
 * (int32, sorted), valK, valM over the overlap pattern (|i_l - j_l| <= p).
 * With rowptr == NULL only *nnz is returned (size query). */
stig_status stig_assemble_3d(int n_el, int p, int nq, const double *c11, const double *c22,
                             const double *c33, const double *c00, int64_t *rowptr, int32_t *col,
                             double *valK, double *valM, int64_t *nnz);

/* 3D form of eq. separation from element-midpoint samples (host, [e3][e2][e1],
 * all positive): the mass coefficient C00 ~ phi1(e1) phi2(e2) phi3(e3) by a
 * rank-one fit in log space (log phi1 = mean over (e2, e3) of log C00, log
 * phi_l = mean over the other two of log C00 minus the global mean for l = 2, 3),
 * then C_ll ~ Phi_l(e_l) prod_{m != l} phi_m with log Phi_l the mean over the
 * other two directions of log(C_ll / prod_{m != l} phi_m).  Exact for products of
 * univariate factors.  Outputs (host): phi_l, Phi_l of length n_l.  STIG_EINVAL
 * for a non-positive sample. */
stig_status stig_separate_3d(int n1, int n2, int n3, const double *C11, const double *C22,
                             const double *C33, const double *C00, double *phi1, double *phi2,
                             double *phi3, double *Phi1, double *Phi2, double *Phi3);

/* Separable approximation of eq. separation from element-midpoint samples
 * (host, [e2][e1], n1 x n2 elements) of the diagonal coefficients C11, C22 and
 * C33: C33 ~ phi1(e1) phi2(e2), C11 ~ Phi1(e1) phi2(e2), C22 ~ phi1(e1) Phi2(e2),
 * by rank-one fits in log space (exact for separable samples).  Outputs host. */
stig_status stig_separate_2d(int n1, int n2, const double *C11, const double *C22,
                             const double *C33, double *phi1, double *phi2, double *Phi1,
                             double *Phi2);

/* Row pointers (host, n_t * ns + 1) of the space-time CSR of
 * W (x) M_s + M_t (x) K_s for banded time factors of bandwidth p_t and a spatial
 * pattern with host row pointers rowptr2d (ns + 1). */
stig_status stig_kron_csr_rowptr(int n_t, int p_t, int64_t ns, const int64_t *rowptr2d,
                                 int64_t *rowptr);

/* Fill (device) col/val of that CSR: rowptr (device, from stig_kron_csr_rowptr),
 * spatial pattern and values (device: rowptr2d, col2d, valM2d, valK2d) and the
 * dense host time factors Wt, Mt (n_t x n_t, bandwidth p_t of the plan).  The
 * columns are int32 (N < 2^31).  Synchronises. */
stig_status stig_kron_csr_fill(stig_plan *plan, const int64_t *rowptr, int32_t *col, double *val,
                               const int64_t *rowptr2d, const int32_t *col2d,
                               const double *valM2d, const double *valK2d, const double *Wt,
                               const double *Mt);

/* ---------------------------------------------------------------- hot path */

/* s = A-hat^{-1} r (transpose = 0) or s = A-hat^{-T} r (transpose = 1) for nrhs
 * right-hand sides: eq. prec_appl solved by Algorithm 1 with the time pencil
 * kept banded: forward spatial transform with U_l^T (mode-l products,
 * eq. kron_vec_multi), one shifted system (gamma W_t + nu lambda_k M_t) per
 * spatial eigen-index k (transposed W_t for the adjoint), back transform with
 * U_l.  r, s: device, nrhs * N doubles; r and s may not overlap.  prec selects
 * the arithmetic (stig_prec). */
stig_status stig_apply_Pinv(stig_plan *plan, const double *r, double *s,
                            int nrhs, int transpose, stig_prec prec);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same apply as
 * stig_apply_Pinv, same arguments, results and kernels, but its intermediate
 * tensors live in a static device array of the library (128 MiB, one per GPU,
 * held until the process ends) instead of the plan's workspace; it calls no
 * allocation routine and needs no stig_set_workspace.  The plan's device must be
 * current.  Sizes whose intermediates exceed 128 MiB (stig_workspace_bytes with
 * restart = 0 gives an upper bound) are refused with STIG_EINVAL, nothing
 * launched: e.g. FP64 fits up to about 8 million unknowns per call.  Every call
 * on one GPU, from any plan, shares that array: calls that overlap on one GPU
 * (other streams or host threads) race; calls ordered on one stream do not.
 * Nothing in the array needs to start at zero (every intermediate is written
 * before it is read). */
stig_status stig_apply_Pinv_noalloc(stig_plan *plan, const double *r, double *s, int nrhs,
                                    int transpose, stig_prec prec);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1), FP64, eq. syst_mat:
 * A = gamma W_t (x) M_s + nu M_t (x) K_s, computed matrix-free by banded mode
 * products (Section 4.5), with the sparse spatial factors of
 * stig_set_spatial_factors, or with the CSR matrix of stig_set_A_csr.
 * x, y: device, nrhs * N doubles, not overlapping. */
stig_status stig_matvec_A(stig_plan *plan, const double *x, double *y, int nrhs,
                          int transpose);

/* y = (M_t (x) M_d (x) ... (x) M_1) z, FP64: the load vector of the spline
 * function with coefficients z (used to build smooth synthetic sources).
 * Uses the factors given to stig_setup_1d_pencils. */
stig_status stig_apply_mass(stig_plan *plan, const double *z, double *y, int nrhs);

/* Initial-datum lifting (Section 3.1, non-homogeneous initial condition), read
 * discretely: the initial datum is u_0(x) = sum_i c0_i B_i(x) times the removed
 * first time B-spline.  Its contribution to the kept equations is
 *     y = A_{I,0} c0 = gamma (a (x) M_s) c0 + nu (b (x) K_s) c0,
 * with a (host, n_t) the column of the unrestricted W_t that belongs to the
 * removed first time function, restricted to the kept rows, and b (host, n_t)
 * the same column of the unrestricted M_t.  c0: device, nrhs * N_s doubles
 * ([rhs][x_d]..[x_1]); y: device, nrhs * N doubles.  The system solved for the
 * kept unknowns is A u = f - A_{I,0} c0: with f (device, nrhs * N doubles) given,
 * y = f - A_{I,0} c0 is written directly (f may equal y); with f = NULL,
 * y = A_{I,0} c0.  Synchronises (a and b are read from host memory). */
stig_status stig_lift_apply(stig_plan *plan, const double *a_col, const double *b_col,
                            const double *c0, const double *f, double *y, int nrhs);

/* Spatial part of the initial-datum lifting (Section 3.1, non-homogeneous
 * initial condition): with a (host, n_t) = column of the unrestricted W for the
 * removed first time function restricted to the kept rows, and b (host, n_t) the
 * same column of the unrestricted M_t,
 *     g = -( gamma M_s (sum_t a_t lam_t) + nu K_s (sum_t b_t lam_t) ),
 * i.e. g = -A_{I,0}^T lam for lam (device, nrhs * N) and g (device, nrhs * N_s).
 * It is the gradient of a loss with respect to the initial-datum coefficients
 * when lam is the adjoint state. */
stig_status stig_lift_adjoint(stig_plan *plan, const double *a_col,
                              const double *b_col, const double *lam, double *g,
                              int nrhs);

/* Solve A u = f for nrhs right-hand sides by restarted GMRES(restart) with right
 * preconditioning by A-hat^{-1} (or A-hat^{-T} with transpose = 1, which solves
 * A^T u = f).  flexible = 1 selects flexible GMRES, required when prec !=
 * STIG_FP64 because the low-precision apply is not a fixed linear operator.  Both
 * variants keep the m preconditioned basis vectors on the device (m * N doubles)
 * and form the update as u += Z y, which for a fixed preconditioner equals
 * P^{-1} (V y) and saves one apply per cycle.  A zero initial guess skips the
 * first product (r_0 = f).  Arnoldi with classical Gram-Schmidt and one
 * re-orthogonalisation delayed to the next step (one reduction and two passes
 * over the basis per step), all in FP64 on the device; the small least-squares
 * problem by Givens rotations on the host.
 * A cycle ends when the GMRES estimate reaches rtol, on a happy breakdown, when
 * maxit is spent, or after `restart` iterations.  In the first three cases the
 * residual r = f - A u is computed afresh (one FP64 product of A); if it is still
 * above rtol (and iterations remain), the next cycle starts from it.  After a
 * full cycle without convergence the next cycle's residual is
 * r_0 - sum_i y_i (A z_i), from the products A z_i of that cycle kept as computed
 * (one stored vector per iteration, m * N doubles).  A nonzero initial guess
 * gets its r_0 = f - A u from a direct product.
 * u: device, in = initial guess, out = solution.  Returns STIG_OK when the fresh
 * relative residual ||f - A u|| / ||f|| <= rtol (reported in info->relres_true),
 * else STIG_NOT_CONVERGED after maxit inner iterations per right-hand side.
 * Several right-hand sides: the first cycle runs in lockstep for as many as the
 * workspace holds (batched applies and products, one host round trip per step
 * for all of them); the others continue one after another.  info (host, may be
 * NULL) receives the worst case over the batch.  Needs the workspace of
 * stig_workspace_bytes(plan, restart, flexible, prec, 1) at least. */
stig_status stig_gmres_solve(stig_plan *plan, const double *f, double *u, int nrhs,
                             int restart, double rtol, int maxit, int flexible,
                             int transpose, stig_prec prec, stig_info *info);

/* ---------------------------------------------------------------- profiling */

/* Kernel classes timed by the optional event profiler. */
enum {
  STIG_K_MODE_GEMM = 0,   /* mode-k MFMA products of the FD apply */
  STIG_K_TIME_SOLVE = 1,  /* banded shifted time solves */
  STIG_K_BAND_PASS = 2,   /* banded mode products of the matvec / mass apply */
  STIG_K_KRYLOV = 3,      /* Arnoldi dot products and updates */
  STIG_K_CSR = 4,         /* CSR matvec, sparse spatial factor pass */
  STIG_K_PLANE_GEMM = 5,  /* fused mode-1/mode-2 MFMA products of the FD apply */
  STIG_NUM_KERNEL_KINDS = 6
};

/* on != 0: every kernel launch of the plan is bracketed by two HIP events on
 * the plan's stream; stig_profile_get synchronises the stream and returns, per
 * kernel class, the summed event time (ms), the summed algorithmic bytes of
 * those launches (compulsory reads + writes of each launch's inputs and outputs,
 * e.g. 16 bytes per unknown for an FP64 mode product) and the launch count.
 * Host pointers may be NULL.  Events cost a few microseconds per launch. */
stig_status stig_profile_enable(stig_plan *plan, int on);
stig_status stig_profile_reset(stig_plan *plan);
stig_status stig_profile_get(stig_plan *plan, int kind, double *total_ms, double *bytes,
                             long long *launches);

/* Device bytes the plan itself holds (its factors; the caller's workspace is
 * not counted).  Constant after the setup calls. */
size_t stig_plan_device_bytes(const stig_plan *plan);

/* ------------------------------------------------------- 1D spline assembly */

/* Gauss-Legendre points and weights on [0, length] split into n_el equal
 * elements, nq points per element (host arrays of n_el * nq). */
stig_status stig_quadrature(int n_el, int nq, double length, double *x, double *w);

/* Dense row-major m x m matrix (m = n_el + p) of the open uniform
 * maximal-continuity B-spline basis of degree p on [0, length] (Section 2.1):
 *   kind 0: mass       [M]_ij = int c b_i b_j
 *   kind 1: stiffness  [K]_ij = int c b_i' b_j'
 *   kind 2: advection  [W]_ij = int c b_j' b_i      (eq. time_mat)
 * c = 1 if weight is NULL, else the values of the coefficient at the nq points
 * per element of stig_quadrature (host, n_el * nq).  nq <= 0 selects p + 1. */
stig_status stig_assemble_1d(int n_el, int p, double length, int kind,
                             const double *weight, int nq, double *out);

/* Load vector [g]_i = int f b_i (host, m entries) from the values of f at the
 * stig_quadrature points (host, n_el * nq). */
stig_status stig_load_1d(int n_el, int p, double length, const double *fvals,
                         int nq, double *out);

/* Symmetric-definite generalized eigenproblem K U = M U Lambda, U^T M U = I,
 * eigenvalues ascending (host, n x n row-major in/out; lam: n).  The routine the
 * setup uses; exposed for testing. */
stig_status stig_sym_eig(int n, const double *K, const double *M, double *U,
                         double *lam);

/* The same eigenproblem for a persymmetric pencil (K[n-1-i][n-1-j] = K[i][j],
 * likewise M, to 1e-13 relative), solved as two half-size pencils on the even
 * and odd vectors: columns 0 .. n/2 + n%2 - 1 of U are even (U[n-1-x][k] =
 * U[x][k]), the rest odd (U[n-1-x][k] = -U[x][k]), eigenvalues ascending within
 * each group.  The basis stig_setup_1d_pencils uses for persymmetric factors;
 * exposed for testing.  STIG_EINVAL if the pencil is not persymmetric. */
stig_status stig_split_eig(int n, const double *K, const double *M, double *U,
                           double *lam);

/* Real block form of the paper's arrowhead factorization of a time pencil
 * (Section 4.2.2, eq. time_eig_2): W, M (host, n x n row-major, the leading
 * (n-1) block of W skew-symmetric, M SPD) -> U and D = U^T W U (host, n x n
 * row-major) with U^T M U = I; D is block diagonal in its leading n-1 rows and
 * columns (a zero 1 x 1 block first when n-1 is odd, then 2 x 2 blocks
 * [[0, d], [-d, 0]]) plus its last row and column.  *nzero receives 1 or 0.
 * The factorization stig_setup_1d_pencils uses for STIG_OPT_TIME_KERNEL = 4;
 * exposed for testing.  STIG_EBREAKDOWN if M is not SPD or the block structure
 * is not reached to 1e-10 relative. */
stig_status stig_time_arrowhead(int n, const double *W, const double *M, double *U, double *D,
                                int *nzero);

const char *stig_status_string(stig_status status);
const char *stig_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STIG_H */

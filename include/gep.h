/*
 * libgep: dense generalized symmetric-definite eigensolver for one AMD MI355X
 * (gfx950) GPU.
 *
 * Problem (section 1, Eq. 1; section 3.1, Eq. 2): given real symmetric M x M
 * matrices A and B with B positive definite, find all eigenvalues lambda_k and
 * eigenvectors y_k with  A y_k = lambda_k B y_k,  i.e.  A Y = B Y Lambda  with the
 * normalisation  Y^T B Y = I.
 *
 * Method (section 3.1, Eqs. 3-6, written with L = U^T):
 *   reducer     B = L L^T (Eq. 4), C = L^{-1} A L^{-T} (Eq. 5) formed without an
 *               explicit inverse of L;
 *   SEP solver  C -> band -> tridiagonal (two-stage Householder reduction),
 *               tridiagonal divide and conquer, back transformation through both
 *               Householder stages (the TRD/BAND, D&C and BACK phases of Table 3);
 *   back        Y = L^{-T} Z (Eq. 6).
 *
 * Conventions for every entry point:
 *   - matrices are column-major with a leading dimension, FP64;
 *   - every matrix and vector pointer is a DEVICE pointer, except arrays whose
 *     name ends in _host;
 *   - only the LOWER triangle of a symmetric input is read; inputs are never
 *     modified;
 *   - work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and is
 *     asynchronous: outputs are valid once the stream has reached that point;
 *   - the caller owns every buffer, including the workspace (size from the
 *     matching *_workspace_size function); the library keeps no pointer after
 *     return and does not allocate device memory on these paths;
 *   - argument errors are detected on the host before any device work and return
 *     a negative gep_status synchronously (gep_last_bad_arg() names the 1-based
 *     argument); HIP errors return GEP_ERR_HIP;
 *   - numerical failures are reported asynchronously in the device int32 `info`
 *     (LAPACK generalized-driver convention): 0 = success; k in [1, M] = the
 *     tridiagonal eigensolver did not converge for eigenvalue k; M + k = the
 *     leading minor of order k of B is not positive definite.  Two device-side
 *     failures that LAPACK does not have use negative codes (argument errors
 *     never reach info: they return synchronously):
 *       GEP_INFO_WAIT_TIMEOUT (-1): a bounded wait between workgroups gave up
 *         (the full -> band reduction's grid barrier or the bulge chase's hand-off
 *         between sweeps waited longer than 10 s); the remaining panels or sweeps
 *         were skipped and lambda / Y are not valid;
 *       GEP_INFO_REFINE_FAILED (-2): GEP_PREC_MIXED only, a block of Y^T B Y in
 *         the FP64 refinement was not positive definite; lambda / Y not valid.
 *     The first failure recorded wins; later ones do not overwrite it.
 *   - M = 0 is a no-op.
 *
 * Eigenvalues are returned in ascending order; for each eigenvector the entry of
 * largest magnitude is positive (lowest index on ties).
 */
#ifndef GEP_H
#define GEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GEP_OK = 0,
  GEP_ERR_ARG = -1,        /* invalid argument: see gep_last_bad_arg() */
  GEP_ERR_WORKSPACE = -2,  /* workspace smaller than the *_workspace_size value */
  GEP_ERR_HIP = -3,        /* a HIP runtime call failed */
  GEP_ERR_NO_DEVICE = -4,  /* no usable gfx950 device */
  GEP_ERR_INTERNAL = -5
} gep_status;

/* Negative device info codes (see the conventions above). */
#define GEP_INFO_WAIT_TIMEOUT (-1)
#define GEP_INFO_REFINE_FAILED (-2)

typedef enum { GEP_JOB_VALUES = 0, GEP_JOB_VECTORS = 1 } gep_job;
typedef enum { GEP_PREC_FP64 = 0, GEP_PREC_MIXED = 1 } gep_prec;

/* Human-readable name of a gep_status value. */
const char* gep_status_string(int status);
/* 1-based index of the offending argument of the last GEP_ERR_ARG (per thread). */
int gep_last_bad_arg(void);
/* Library version string. */
const char* gep_version(void);

/* Bytes of workspace gep_solve needs for order M. */
size_t gep_workspace_size(int64_t M, int job, int prec);

/*
 * Solve A Y = B Y Lambda (all eigenpairs, or eigenvalues only for
 * job = GEP_JOB_VALUES, the paper's T_evo case of section 4).
 * The call can be captured in a HIP graph and replayed (so can gep_solve_noalloc
 * and gep_solve_lowest): on a capturing stream the workgroup-synchronised kernels
 * are launched without the cooperative attribute, with identical results.
 *   A [lda x M], B [ldb x M]: lower triangles read.
 *   lambda [M]: eigenvalues, ascending.
 *   Y [ldy x M]: B-orthonormal eigenvectors (unused and may be NULL for VALUES).
 *   prec: GEP_PREC_FP64 (every step in FP64), or GEP_PREC_MIXED (job must be
 *     GEP_JOB_VECTORS): the interior GEMM tiles of the Cholesky, the reduced
 *     matrix, the full -> band reduction, the Q1 back-transformation and
 *     Y = L^-T Z run in FP32 arithmetic (FP64 storage; Cholesky diagonal blocks,
 *     bulge chase, Q2 and the tridiagonal solver stay FP64), then one FP64
 *     refinement pass: S = Y^T A Y and T = Y^T B Y in FP64, exact FP64 solves of
 *     gap-aligned blocks of consecutive eigenvalues, and first-order coupling
 *     between blocks (eigenvalues corrected to second order).  This extends the
 *     paper, which uses FP64 throughout.
 *   workspace: >= gep_workspace_size(M, job, prec) bytes, 256-byte aligned.
 *   info: device int32, see above.
 */
int gep_solve(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
              double* lambda, double* Y, int64_t ldy, int job, int prec, void* workspace,
              size_t ws_bytes, int32_t* info, void* stream);

/*
 * gep_solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same solve
 * with the same arguments except the workspace, which is a fixed array built into
 * the library's device image (gep_noalloc_max_bytes() bytes, 272 MiB, held on
 * each device the library runs on until the process ends).  Nothing is allocated
 * by this call, and no phase timing events are recorded.
 *   Limit: gep_workspace_size(M, job, prec) <= gep_noalloc_max_bytes(); every
 *   M <= 2303 for FP64 eigenpairs (so every order of a batch in [64, 2048]),
 *   M <= 1858 mixed, M <= 3889 eigenvalues only.  Larger problems return
 *   GEP_ERR_WORKSPACE before any device work.
 *   Every call on one device uses that device's single array: calls that overlap
 *   in time on one device (other streams, other host threads) race and give wrong
 *   results; calls on different devices do not interfere.  Each call clears the
 *   parts of the array it relies on, so the previous call's contents do no harm.
 *   Argument errors name the argument by its position (1 = M ... 11 = info).
 */
int gep_solve_noalloc(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
                      double* lambda, double* Y, int64_t ldy, int job, int prec, int32_t* info,
                      void* stream);
/* Bytes of the fixed workspace gep_solve_noalloc uses on each device. */
size_t gep_noalloc_max_bytes(void);

/*
 * Partial spectrum: all M eigenvalues and the eigenvectors of the k smallest.
 * Electronic-structure calculations need eigenpairs on the order of the number
 * of electrons (section 2.1), and the eigenvector part of a solve,
 * T_vec = T_full - T_evo, is dominated by the back transformation (section 4.1);
 * here the tridiagonal solver still returns all M eigenvectors (in the
 * workspace), and only the first k go through the Q2, Q1 and L^{-T} back
 * transformations, whose cost falls from 5M^3 to 5M^2 k flops.
 *   k: 0..M (0: eigenvalues only, via the tridiagonal solver; M: as gep_solve).
 *   lambda: device [M], ascending.  Y: device M x k (ldy >= max(1, M)), column j
 *   the B-orthonormal eigenvector of lambda[j], same sign convention as gep_solve.
 *   A, B, lda, ldb, info: as gep_solve (FP64 only).
 *   workspace: >= gep_workspace_size_lowest(M, k) bytes, 256-byte aligned (for
 *   k < M, one M x M buffer more than gep_solve's).
 * Argument errors name the argument by its position (1 = M ... 12 = info).
 */
size_t gep_workspace_size_lowest(int64_t M, int64_t k);
int gep_solve_lowest(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
                     int64_t k, double* lambda, double* Y, int64_t ldy, void* workspace,
                     size_t ws_bytes, int32_t* info, void* stream);

/*
 * Cholesky-free reducer (section 3.1, Eqs. 7-9): instead of B = L L^T, the
 * symmetric eigenproblem of B itself, B W = W D, is solved by the same two-stage
 * SEP path; the reduced matrix is C = (W D^{-1/2})^T A (W D^{-1/2}) and the
 * eigenvectors are Y = W D^{-1/2} Z with C Z = Z Lambda.  Two SEP solves and three
 * M^3 GEMMs: slower than gep_solve on one GPU, but no triangular factor or solve.
 *   A, B, lda, ldb, lambda, Y, ldy: as gep_solve with job = GEP_JOB_VECTORS (FP64).
 *   workspace: >= gep_workspace_size_cholfree(M) bytes, 256-byte aligned (one
 *   M x M buffer and M doubles more than gep_solve's).
 *   info: as gep_solve, except that M + c means that c eigenvalues of B are not
 *   positive (B is not positive definite; Y and lambda are then meaningless).
 * Argument errors name the argument by its position (1 = M ... 11 = info).
 */
size_t gep_workspace_size_cholfree(int64_t M);
int gep_solve_cholfree(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
                       double* lambda, double* Y, int64_t ldy, void* workspace, size_t ws_bytes,
                       int32_t* info, void* stream);

/*
 * Explicit-inverse (ELPA-style) reducer (section 3.1): the Cholesky factorization
 * B = L L^T as in gep_solve, then the inverse R = L^{-1} formed explicitly (the
 * paper's R = U^{-1} with U = L^T; recursive, from the Cholesky's inverted
 * diagonal blocks, M^3/3 flops), the reduced matrix by two successive matrix
 * products, C = (R A) R^T (a triangular multiply and the lower triangle of a
 * GEMM, 2 M^3), and the back transformation as one triangular multiply,
 * Y = R^T Z (M^3).  All of it runs as GEMMs on the matrix cores.
 *   A, B, lda, ldb, lambda, Y, ldy, info: as gep_solve with job = GEP_JOB_VECTORS
 *   (FP64).
 *   workspace: >= gep_workspace_size_explicit_inverse(M) bytes, 256-byte aligned
 *   (one M x M buffer more than gep_solve's).
 * Argument errors name the argument by its position (1 = M ... 11 = info).
 */
size_t gep_workspace_size_explicit_inverse(int64_t M);
int gep_solve_explicit_inverse(int64_t M, const double* A, int64_t lda, const double* B,
                               int64_t ldb, double* lambda, double* Y, int64_t ldy,
                               void* workspace, size_t ws_bytes, int32_t* info, void* stream);

/*
 * Block Jacobi SEP solver behind the reducer: the combination the paper's outlook
 * proposes (section 6: a solver of a different mathematical foundation that only
 * handles standard problems, made usable for generalized ones by the reducer).
 * B = L L^T and C = L^{-1} A L^{-T} as in gep_solve (Eqs. 4-5); the eigenpairs of
 * C by parallel two-sided block Jacobi (32-row blocks, all disjoint block pairs
 * of a round at once: each 64 x 64 pair matrix diagonalised exactly in LDS, the
 * rotations applied to C and to the eigenvector matrix on the matrix cores) until
 * the off-diagonal norm is at rounding level; Y = L^{-T} Z (Eq. 6).  No band or
 * tridiagonal form is formed.  About 12 M^3 flops per sweep, 6-10 sweeps: several
 * times the work of gep_solve, which it does not replace; the stream is
 * synchronised once per sweep (convergence test), so the call cannot be captured
 * in a graph.
 *   A, B, lda, ldb, lambda, Y, ldy: as gep_solve with job = GEP_JOB_VECTORS (FP64).
 *   workspace: >= gep_workspace_size_jacobi(M) bytes, 256-byte aligned.
 *   info: as gep_solve, with k = M when the sweeps have not converged after 30.
 * gep_last_jacobi_sweeps: sweeps of the last gep_solve_jacobi on this process.
 * Argument errors name the argument by its position (1 = M ... 11 = info).
 */
size_t gep_workspace_size_jacobi(int64_t M);
int gep_solve_jacobi(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
                     double* lambda, double* Y, int64_t ldy, void* workspace, size_t ws_bytes,
                     int32_t* info, void* stream);
int gep_last_jacobi_sweeps(void);

/*
 * Many independent problems of different orders in one call (the k-point-like
 * batches of electronic-structure codes; the paper solves one problem per run).
 * Arrays ending in _host are HOST arrays of length `batch` (orders, leading
 * dimensions, and the device pointers of each instance's A, B, lambda, Y);
 * info is a DEVICE int32 array [batch], one LAPACK-style code per instance.
 * The instances are spread over worker streams forked from `stream` with events
 * (largest first, each to the least loaded stream) and joined back into it, so
 * the call can be captured in a HIP graph and replayed.  Outside capture each
 * worker stream's instances are enqueued by a host thread of its own (the
 * launches and their order per stream are the same as from one thread, and so
 * are the results; gep_batched_threads(0) enqueues from the calling thread
 * only).  Workspace: gep_workspace_size_batched bytes for the same M_host list.
 */
size_t gep_workspace_size_batched(int batch, const int64_t* M_host, int job, int prec);
int gep_solve_batched(int batch, const int64_t* M_host, const double* const* A_host,
                      const int64_t* lda_host, const double* const* B_host,
                      const int64_t* ldb_host, double* const* lambda_host, double* const* Y_host,
                      const int64_t* ldy_host, int job, int prec, void* workspace, size_t ws_bytes,
                      int32_t* info, void* stream);
/* Enqueue batched solves from one host thread per worker stream (1, the
 * default) or from the calling thread only (0); process-wide.  Returns GEP_OK. */
int gep_batched_threads(int on);

/*
 * Phase entry points (same conventions).  They expose the steps of gep_solve one
 * at a time so that each can be checked and timed on its own.
 *
 * gep_reduce: reducer of section 3.1 (Eqs. 4-5).  L [ldl x M] receives the
 *   Cholesky factor (strict upper triangle zero), C [ldc x M] the reduced matrix
 *   L^{-1} A L^{-T} (full symmetric).  info as for gep_solve (M + k only).
 */
size_t gep_reduce_workspace_size(int64_t M);
int gep_reduce(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb, double* L,
               int64_t ldl, double* C, int64_t ldc, void* workspace, size_t ws_bytes,
               int32_t* info, void* stream);

/*
 * gep_band_reduce: first stage of the two-stage reduction (TRD/BAND of Table 3):
 *   symmetric C (lower read) -> band matrix with the same eigenvalues, returned in
 *   lower band storage: element (i, j), 0 <= i - j <= band_width, at
 *   band[(i - j) + j * ldband], ldband >= band_width + 1.
 *   band_width: 1..64, or 0 for the value gep_solve uses.
 */
size_t gep_band_reduce_workspace_size(int64_t M, int band_width);
int gep_band_reduce(int64_t M, const double* C, int64_t ldc, int band_width, double* band,
                    int64_t ldband, void* workspace, size_t ws_bytes, void* stream);

/*
 * gep_tridiagonalize: both stages: symmetric C (lower read) -> symmetric
 *   tridiagonal T with the same eigenvalues: d [M] diagonal, e [M-1] subdiagonal.
 */
size_t gep_tridiagonalize_workspace_size(int64_t M, int band_width);
int gep_tridiagonalize(int64_t M, const double* C, int64_t ldc, int band_width, double* d,
                       double* e, void* workspace, size_t ws_bytes, void* stream);

/*
 * gep_tridiag_eig: eigen-decomposition of the symmetric tridiagonal (d, e) (D&C
 *   phase of Table 3): lambda [M] ascending; for job = GEP_JOB_VECTORS, Z [ldz x M]
 *   orthonormal eigenvectors (divide and conquer); for GEP_JOB_VALUES, Sturm
 *   bisection and Z unused.  info: k in [1, M] on non-convergence.
 */
size_t gep_tridiag_eig_workspace_size(int64_t M, int job);
int gep_tridiag_eig(int64_t M, const double* d, const double* e, double* lambda, double* Z,
                    int64_t ldz, int job, void* workspace, size_t ws_bytes, int32_t* info,
                    void* stream);

/*
 * Adjoint of gep_solve for symmetric perturbations (reverse-mode derivative):
 * given the solution (lambda, Y) and cotangents lambda_bar = dL/dlambda [M] and
 * Y_bar = dL/dY [ldyb x M] (either may be NULL = zero), writes the symmetric
 * gradients A_bar = dL/dA [ldab x M] and B_bar = dL/dB [ldbb x M] (full, both
 * triangles).  Derived by differentiating A Y = B Y Lambda and Y^T B Y = I
 * (section 3.1, Eq. 2): d lambda_k = y_k^T (dA - lambda_k dB) y_k, and the
 * eigenvector term couples pairs (i, j) through 1 / (lambda_j - lambda_i).  That
 * coupling is regularised near degeneracies: F_ij = D / (D^2 + eta^2) with
 * D = lambda_j - lambda_i, and F_ij = 0 when |D| <= tau_c; it multiplies only the
 * antisymmetric part of Y^T Y_bar, which is exact for losses invariant under
 * rotations inside degenerate eigenspaces.  eta >= 0, tau_c >= 0.
 */
size_t gep_backward_workspace_size(int64_t M);
int gep_backward(int64_t M, const double* lambda, const double* Y, int64_t ldy,
                 const double* lambda_bar, const double* Y_bar, int64_t ldyb, double eta,
                 double tau_c, double* A_bar, int64_t ldab, double* B_bar, int64_t ldbb,
                 void* workspace, size_t ws_bytes, void* stream);

/*
 * Building block: C = alpha op(A) op(B) + beta C in FP64 on the matrix cores
 * (the contraction every blocked step of the solver is made of).  op(X) = X or
 * X^T (trans = 0 / 1); op(A) is m x k, op(B) k x n, C m x n, all column-major
 * device pointers.  uplo = 1 writes only the lower triangle of C (m == n).
 * arith = 0: FP64 arithmetic throughout.  arith = 1: the 128 x 128 interior tiles
 * round both operands to FP32 and accumulate in FP32 on the matrix cores (the
 * mixed-precision solver's trailing updates); inputs and outputs stay FP64,
 * edge strips stay FP64.  Any other value returns GEP_ERR_ARG (argument 15).
 */
int gep_dgemm(int transA, int transB, int uplo, int64_t m, int64_t n, int64_t k, double alpha,
              const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
              int64_t ldc, int arith, void* stream);

/*
 * Per-phase timing of the last gep_solve on this process: when enabled,
 * gep_solve records HIP events around its phases on `stream`.
 * gep_profile_read synchronises on the last event and writes up to n phase times
 * in milliseconds, in the order R1 (Cholesky), R2-4 (reduced matrix), S1 (full ->
 * band), S2 (band -> tridiagonal), S3 (tridiagonal eigensolver), S4 (Q2), S5 (Q1),
 * R5 (Y = L^{-T} Z), REF (mixed-precision refinement; zero for FP64), F (sign
 * convention).  Returns the number of phases written.
 */
int gep_profile_enable(int on);
int gep_profile_read(double* ms, int n);
/*
 * Flops of the divide-and-conquer merge products of the last profiled gep_solve
 * (job = VECTORS): 2 m n k summed over every merge's two products with their
 * sizes after deflation, i.e. the data-dependent part of that phase's work.
 * Valid once gep_profile_read has returned for that solve; 0 before any.
 */
double gep_profile_dc_flops(void);

/*
 * Launch probes: when enabled, every launch of the probed kernels records a HIP
 * event pair on the stream it is launched on, with the launch's algorithmic
 * flops.  Kernels: 0 = the 128 x 128 interior GEMM tile kernel (flops 2 m n k,
 * or k n (n + 1) for a lower-triangle product), 1 = the Q2 application (2 n^2
 * ncols), 2 = the bulge chase, either kernel (6 b n^2), 3 = the band-reduction panel QR
 * (2 n w^2 - 2 w^3 / 3 for an n x w panel).
 * gep_probe_read synchronises on the recorded events, returns the number of
 * launches, their summed duration in milliseconds and their summed flops since
 * the previous read of that kernel, and forgets them.  Any output pointer may be
 * NULL.  An unknown kernel index returns GEP_ERR_ARG (argument 1).
 * gep_probe_name returns the kernel's name (NULL for an unknown index).
 */
int gep_probe_enable(int on);
int gep_probe_read(int kernel, int64_t* launches, double* ms, double* flops);
const char* gep_probe_name(int kernel);

/*
 * Tuned parameters.  The blocking and launch parameters below have built-in
 * rules; a table of (parameter, orders m_lo..m_hi, value) entries replaces a
 * rule for the orders it covers.  The table is read when the library is first
 * used from the JSON file named by the environment variable GEP_TUNE_FILE, else
 * from tuning.json beside libgep.so (written by the package's autotune.py from
 * timings on the GPU); with no file the built-in rules apply.  Format:
 *   {"parameters": {"band_width": [{"m_lo": 64, "m_hi": 127, "value": 16}, ...]}}
 * (other keys and fields are ignored).  Parameters (admissible values):
 *   band_width          width b of the full -> band reduction (1..64; built in:
 *                       64 from order 2048, 32 from 256, else 16); b = 64 selects
 *                       the register-window Q2 back transformation;
 *   q2_wide_min_cols    Q2 back transformation with 32 columns per wave (one wave
 *                       per SIMD) when at least this many columns are transformed
 *                       (>= 0; built in: 2^40, i.e. always 16 per wave);
 *   dc_leaf             largest leaf of the divide-and-conquer tree (8..64; 64);
 *   symm_split_rows     the band reduction's symmetric products split their sum
 *                       over workgroups from this many rows (>= 1; 2048);
 *   chase_extra_groups  bulge chase workgroups beyond half the first sweep's
 *                       positions (0..512; 8);
 *   q2_mixed_fp32       GEP_PREC_MIXED: the Q2 back transformation in FP32
 *                       arithmetic on the matrix cores (1) or in FP64 (0; built
 *                       in: 0, measured faster at M = 32768);
 *   q2_staged           FP64 Q2 back transformation with 16 columns per wave:
 *                       V / T staged by direct-to-LDS loads and Z read and
 *                       written in 16-byte accesses (1; needs an even leading
 *                       dimension and a 16-byte aligned Z, else the
 *                       register-staged kernel runs) or the register-staged
 *                       kernel (0).  Built in: 1.
 *   chase_stationary    single solves (not batched ones): the data-stationary
 *                       bulge chase, each workgroup keeping its positions' blocks
 *                       in LDS across sweeps (1: one position per workgroup when
 *                       all fit on the device at once, else two; 2: two), or the
 *                       ticketed chase (0).  Same results bitwise.  Built in: 0
                       (two long test runs went silent inside single solves
                       that used the data-stationary chase; cause not found).
 * Results depend on band_width and dc_leaf only through rounding; every
 * parameter value gives a correct solve.  A batched instance and a single solve
 * of the same order use the same values.
 *
 * gep_tune_load: (re)read the table from `path` (NULL: the default location,
 *   where a missing file means no table).  Returns the number of entries read, or
 *   GEP_ERR_ARG when the file is missing (explicit path) or malformed (the
 *   previous table is kept then).
 * gep_tune_set: add a run-time override for orders m_lo..m_hi (it takes
 *   precedence over the table; the latest override covering an order wins).
 *   GEP_ERR_ARG for an unknown parameter, an empty range or a value outside the
 *   admissible ones.
 * gep_tune_reset_overrides: drop every run-time override (the table stays).
 * gep_tune_clear: drop the table and every override: built-in rules only.
 * gep_tune_get: the value in effect for order M, or -1 for an unknown name.
 * The table is process-wide; change it only while no solve is being enqueued.
 */
int gep_tune_load(const char* path);
int gep_tune_set(const char* key, int64_t m_lo, int64_t m_hi, int64_t value);
int gep_tune_reset_overrides(void);
int gep_tune_clear(void);
int64_t gep_tune_get(const char* key, int64_t M);

/*
 * Failure injection for tests: while on (process-wide), every bounded wait of
 * the full -> band reduction's grid barrier and of the bulge chase that is not
 * already satisfied at its first poll gives up at once, exactly as if its 10 s
 * limit had passed.  Every kernel still runs to its normal exit; the solves then
 * report GEP_INFO_WAIT_TIMEOUT in info.  Off by default; affects launches
 * enqueued while it is on.  Returns GEP_OK.
 */
int gep_debug_force_wait_timeout(int on);

/*
 * Failure injection for tests: while on (process-wide), the divide-and-conquer
 * tridiagonal eigensolver's leaf iteration cap is zero, so the first leaf that
 * needs an implicit QL iteration reports non-convergence through info
 * (k in [1, M], the leaf's first eigenvalue index + 1), the path a real
 * non-convergence takes.  Off by default.  Returns GEP_OK.
 */
int gep_debug_force_eig_failure(int on);

#ifdef __cplusplus
}
#endif

#endif /* GEP_H */

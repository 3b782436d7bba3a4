// Internal interfaces between the phases of the solver (not part of the C ABI).
#pragma once
#include "common.h"

namespace gep {

// Diagonal block size of the Cholesky factor and the triangular solves.
constexpr int NB = 128;

// A lower-triangular operand: L (ld) whose row/column 0 is global index `off`
// (a multiple of NB); Linv holds the inverses of all NB x NB diagonal blocks of
// the global factor, block b at Linv + b*NB*NB (ld NB).
struct Tri {
  const double* L;
  int64_t ld;
  const double* Linv;
  int64_t off;
};

size_t potrf_leaf_lds();
void potrf_rec(double* a, int64_t lda, int64_t n, int64_t off, double* linv, int32_t* info,
               int64_t info_add, double* tmp, hipStream_t s);
void trsm_lln(const Tri& t, int64_t n, double* X, int64_t ldx, int64_t ncols, double* tmp,
              hipStream_t s);
void trsm_llt(const Tri& t, int64_t n, double* X, int64_t ldx, int64_t ncols, double* tmp,
              hipStream_t s);
void trsm_rlt(const Tri& t, int64_t n, double* X, int64_t ldx, int64_t nrows, double* tmp,
              hipStream_t s);
void trsm_rlt_lower(const Tri& t, int64_t n, double* X, int64_t ldx, double* tmp, hipStream_t s);

// ---------------------------------------------------------------- full -> band
// Band storage used by the band-to-tridiagonal stage: element (i, j), i >= j,
// |i - j| <= 2*b, at band[(i - j) + j * ldband] with ldband >= 2*b + 1 (room for
// the bulges).
struct BandReduction {
  int64_t n = 0;
  int b = 0;
  double* C = nullptr;   // n x n, lower triangle holds the matrix; on exit the
  int64_t ldc = 0;       // panels below the band hold explicit V (unit diag)
  double* T = nullptr;   // b x b per panel, panel p at T + p*b*b
  double* band = nullptr;
  int64_t ldband = 0;
  bool coop = true;      // cooperative launch of the panel QR
  int32_t* info = nullptr;  // device: INFO_WAIT_TIMEOUT if a panel's grid barrier
                            // gave up (optional)
};
size_t sy2sb_workspace(int64_t n, int b);
void sy2sb(const BandReduction& r, Arena& ws, hipStream_t s);
// Z (n x ncols) <- Q1 Z with the reflectors left by sy2sb.
size_t apply_q1_workspace(int64_t n, int64_t ncols, int b);
void apply_q1(const BandReduction& r, double* Z, int64_t ldz, int64_t ncols, Arena& ws,
              hipStream_t s);

// ---------------------------------------------------------------- band -> tridiagonal
struct BulgeChase {
  int64_t n = 0;
  int b = 0;
  double* band = nullptr;  // in/out (destroyed)
  int64_t ldband = 0;
  double* d = nullptr;     // out: diagonal (n)
  double* e = nullptr;     // out: subdiagonal (n-1)
  double* V = nullptr;     // out: reflectors in Q2 block layout (sb2st_block_storage doubles)
  double* tau = nullptr;   // out: tau at tau[s*kmax + k]
  int64_t kmax = 0;        // reflector positions per sweep = ceil((n-1)/b)
  int32_t* sync = nullptr; // device scratch: progress flags (n + 8 ints)
  int32_t* err = nullptr;  // device: set to nonzero if a wait timed out
  int32_t* info = nullptr; // device: INFO_WAIT_TIMEOUT if so (optional)
  // Cooperative launches allowed (single solves): the data-stationary chase runs
  // when msg holds at least sb2st_message_bytes(n, b) of device scratch, which it
  // uses only while it runs.  Otherwise (batched solves) the ticketed chase.
  bool coop = false;
  double* msg = nullptr;
  size_t msg_bytes = 0;
};
size_t sb2st_message_bytes(int64_t n, int b);
size_t sb2st_reflector_count(int64_t n, int b);
size_t sb2st_block_storage(int64_t n, int b);
void sb2st(const BulgeChase& c, hipStream_t s);
// Z (n x ncols) <- Q2 Z with the bulge-chasing reflectors.
size_t apply_q2_workspace(int64_t n, int b);
void apply_q2(const BulgeChase& c, double* Z, int64_t ldz, int64_t ncols, Arena& ws,
              hipStream_t s);

// ---------------------------------------------------------------- tridiagonal eigensolver
size_t stedc_workspace(int64_t n);
// Eigenvalues (ascending) and eigenvectors of the symmetric tridiagonal (d, e).
// d, e are read only.  info: set to k > 0 if a secular equation failed.
// flops_host (optional, pinned host memory): receives, asynchronously, the merge
// products' flops (2 m n k summed after deflation).
void stedc(int64_t n, const double* d, const double* e, double* lambda, double* Z, int64_t ldz,
           int32_t* info, Arena& ws, hipStream_t s, double* flops_host = nullptr);
// Eigenvalues only, by bisection; bounds2 is 2 doubles of device scratch.
void stebz_ws(int64_t n, const double* d, const double* e, double* lambda, double* bounds2,
              hipStream_t s);

// ---------------------------------------------------------------- block Jacobi SEP
// Eigenvalues (ascending, into lam) and eigenvectors (into Z, ldz) of the
// symmetric n x n matrix C (full storage, destroyed) by parallel two-sided block
// Jacobi.  Synchronises the stream once per sweep (convergence test on the
// host).  info <- n if it has not converged after 30 sweeps.  Returns the number
// of sweeps.
size_t jacobi_workspace(int64_t n);
int jacobi_eig(int64_t n, double* C, int64_t ldc, double* lam, double* Z, int64_t ldz,
               int32_t* info, Arena& ws, hipStream_t s);

// ---------------------------------------------------------------- adjoint
size_t backward_workspace(int64_t M);
void backward(int64_t M, const double* lam, const double* Y, int64_t ldy, const double* lam_bar,
              const double* Y_bar, int64_t ldyb, double eta, double tau_c, double* A_bar,
              int64_t ldab, double* B_bar, int64_t ldbb, Arena& ws, hipStream_t s);

// ---------------------------------------------------------------- finishing
void sign_fix(int64_t n, int64_t ncols, double* Y, int64_t ldy, hipStream_t s);

// FP64 refinement of approximate eigenvectors Y (M x M, ldy) of (A, B), lower
// triangles of A and B read: overwrites Y and lambda with the refined,
// ascending eigenpairs.  W1, W2: M x M scratch (leading dimension M).  Writes the
// largest first-order coupling left between blocks to *coupling_out (device).
size_t refine_workspace(int64_t M);
// info (device, optional): INFO_REFINE_FAILED when a block's Y^T B Y is not
// positive definite.
void refine(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb, double* Y,
            int64_t ldy, double* lambda, double* W1, double* W2, Arena& ws, double* coupling_out,
            int32_t* info, hipStream_t s);

}  // namespace gep

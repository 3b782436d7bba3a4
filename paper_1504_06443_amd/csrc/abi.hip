// C ABI of libgep: argument validation on the host, workspace planning, and the
// phase sequence of the solver (reducer, two-stage reduction, tridiagonal
// eigensolver, back transformations).
#include <algorithm>
#include <cstring>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/gep.h"
#include "common.h"
#include "internal.h"

namespace gep {
namespace {

thread_local int g_bad_arg = 0;

int bad(int idx) {
  g_bad_arg = idx;
  return GEP_ERR_ARG;
}

// Band width of the full -> band reduction (tuning table; by default 64 from
// order 2048, 32 from 256, else 16).
int default_band(int64_t M) { return (int)tune("band_width", M); }

// ---------------------------------------------------------------- finishing
__global__ void sign_fix_kernel(int64_t n, double* __restrict__ Y, int64_t ldy) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  double* y = Y + (int64_t)blockIdx.x * ldy;
  double best = -1.0;
  int64_t idx = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double a = fabs(y[i]);
    if (a > best) { best = a; idx = i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double o = bv[threadIdx.x + s];
      const int64_t oi = bi[threadIdx.x + s];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  // One thread reads the pivot's sign before any entry of the column changes: a
  // wave that read it after another wave had already negated it would skip the
  // flip and leave the column half negated.
  __shared__ int flip;
  if (threadIdx.x == 0) flip = y[bi[0]] < 0.0;
  __syncthreads();
  if (flip)
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) y[i] = -y[i];
}

__global__ void band_copy_out(int64_t n, int b, const double* __restrict__ band, int64_t ldw,
                              double* __restrict__ out, int64_t ldo) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int d = 0; d <= b; ++d) out[d + j * ldo] = (j + d < n) ? band[d + j * ldw] : 0.0;
}

// W(:, j) <- W(:, j) / sqrt(d_j): the columns of W D^{-1/2} (section 3.1, Eqs. 8
// and 9); a column whose d_j is not positive is zeroed.
__global__ void scale_cols_rsqrt(int64_t n, const double* __restrict__ d, double* __restrict__ W,
                                 int64_t ldw) {
  const double dj = d[blockIdx.x];
  const double sc = dj > 0.0 ? 1.0 / sqrt(dj) : 0.0;
  double* w = W + (int64_t)blockIdx.x * ldw;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) w[i] *= sc;
}

// info <- n + (number of d_i that are not positive), unless info is already set.
__global__ void count_nonpositive(int64_t n, const double* __restrict__ d, int32_t* info) {
  __shared__ int cnt[256];
  int c = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) c += (d[i] > 0.0) ? 0 : 1;
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) cnt[threadIdx.x] += cnt[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && cnt[0] > 0) atomicCAS(info, 0, (int32_t)(n + cnt[0]));
}

// ---------------------------------------------------------------- profiling
constexpr int NPHASE = 10;
bool g_prof = false;
hipEvent_t g_ev[NPHASE + 1];
bool g_ev_ok = false;
bool g_ev_recorded = false;
double* g_dc_flops = nullptr;  // pinned host: the last profiled solve's merge flops

double* dc_flops_host() {
  if (!g_dc_flops) {
    GEP_HIP(hipHostMalloc((void**)&g_dc_flops, sizeof(double), hipHostMallocDefault));
    *g_dc_flops = 0.0;
  }
  return g_dc_flops;
}

struct Prof {
  hipStream_t s;
  explicit Prof(hipStream_t st) : s(st) {
    if (g_prof && !g_ev_ok) {
      for (int i = 0; i <= NPHASE; ++i) GEP_HIP(hipEventCreate(&g_ev[i]));
      g_ev_ok = true;
    }
  }
  void mark(int i) {
    if (g_prof) GEP_HIP(hipEventRecord(g_ev[i], s));
    if (g_prof && i == NPHASE) g_ev_recorded = true;
  }
};

// ---------------------------------------------------------------- workspace plan
struct Plan {
  int64_t M;
  int b;
  int64_t ldband, kmax, nblk;
  bool vectors, mixed;
  char* refine_ws;  // mixed precision: refinement workspace
  size_t refine_bytes;
  double* coupling;
  double *L, *Linv, *tmp, *C, *T1, *band, *d, *e, *V2, *tau2, *bounds;
  double* Zd;     // partial spectrum: the tridiagonal solver's M x M eigenvectors
  int32_t *sync, *err;
  int32_t* info;  // the caller's info word (device), set by the solve
  char* scratch;  // phase scratch (reused by S1, S3, S4, S5)
  size_t scratch_bytes;
};

size_t phase_scratch_bytes(int64_t M, int b, bool vectors) {
  size_t s = sy2sb_workspace(M, b);
  if (vectors) {
    s = s > stedc_workspace(M) ? s : stedc_workspace(M);
    const size_t q2 = apply_q2_workspace(M, b);
    s = s > q2 ? s : q2;
    const size_t q1 = apply_q1_workspace(M, M, b);
    s = s > q1 ? s : q1;
  }
  return s;
}

void carve(Plan& p, Arena& a, int64_t M, bool vectors, bool mixed = false, bool partial = false) {
  p.M = M;
  p.b = default_band(M);
  p.vectors = vectors;
  p.mixed = mixed;
  p.ldband = 2 * p.b + 1;
  p.kmax = M > 1 ? cdiv(M - 1, p.b) : 1;
  p.nblk = cdiv(M, NB);
  p.L = a.take<double>((size_t)M * M);
  p.Linv = a.take<double>((size_t)p.nblk * NB * NB);
  p.tmp = a.take<double>((size_t)NB * M);
  p.C = a.take<double>((size_t)M * M);
  p.T1 = a.take<double>((size_t)cdiv(M, p.b) * p.b * p.b);
  p.band = a.take<double>((size_t)p.ldband * M);
  p.d = a.take<double>(M);
  p.e = a.take<double>(M);
  p.bounds = a.take<double>(2);
  p.sync = a.take<int32_t>(M + 8);
  p.err = a.take<int32_t>(1);
  if (vectors) {
    p.V2 = a.take<double>(sb2st_block_storage(M, p.b));
    p.tau2 = a.take<double>(sb2st_reflector_count(M, p.b));
  } else {
    p.V2 = p.tau2 = nullptr;
  }
  p.scratch_bytes = phase_scratch_bytes(M, p.b, vectors);
  p.scratch = a.take<char>(p.scratch_bytes);
  p.Zd = (vectors && partial) ? a.take<double>((size_t)M * M) : nullptr;
  p.refine_ws = nullptr;
  p.refine_bytes = 0;
  p.coupling = nullptr;
  p.info = nullptr;
  if (mixed) {
    p.refine_bytes = refine_workspace(M);
    p.refine_ws = a.take<char>(p.refine_bytes);
    p.coupling = a.take<double>(1);
  }
}

Arena scratch_arena(const Plan& p) {
  Arena a;
  a.base = p.scratch;
  a.cap = p.scratch_bytes;
  return a;
}

void reduce_steps(const Plan& p, const double* A, int64_t lda, const double* B, int64_t ldb,
                  int32_t* info, hipStream_t s, Prof* prof) {
  const int64_t M = p.M;
  // R1: L = chol(B)
  copy_matrix(M, M, B, ldb, p.L, M, s);
  potrf_rec(p.L, M, M, 0, p.Linv, info, M, p.tmp, s);
  if (prof) prof->mark(1);
  // R2-4: C = L^{-1} A L^{-T}
  symmetrize_from_lower(M, A, lda, p.C, M, s);
  Tri t{p.L, M, p.Linv, 0};
  trsm_lln(t, M, p.C, M, M, p.tmp, s);
  trsm_rlt_lower(t, M, p.C, M, p.tmp, s);
  if (prof) prof->mark(2);
}

BandReduction band_of(const Plan& p) {
  BandReduction r;
  r.n = p.M; r.b = p.b; r.C = p.C; r.ldc = p.M; r.T = p.T1; r.band = p.band; r.ldband = p.ldband;
  r.info = p.info;
  return r;
}

BulgeChase chase_of(const Plan& p) {
  BulgeChase c;
  c.n = p.M; c.b = p.b; c.band = p.band; c.ldband = p.ldband; c.d = p.d; c.e = p.e;
  c.V = p.V2; c.tau = p.tau2; c.kmax = p.kmax; c.sync = p.sync; c.err = p.err;
  c.info = p.info;
  // the phase scratch is idle between S1 and S3
  c.msg = (double*)p.scratch;
  c.msg_bytes = p.scratch_bytes;
  return c;
}

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const HipError& e) {
    if (e.err == hipErrorOutOfMemory) return GEP_ERR_WORKSPACE;
    return GEP_ERR_HIP;
  } catch (...) {
    return GEP_ERR_INTERNAL;
  }
}

// True while s is being captured into a graph.  A single solve captured that way
// launches the panel QR and the bulge chase as plain launches, the form batched
// solves use: the same kernels with the same arithmetic, so the same results.  The
// panel QR's grid is no larger than the device holds at once and its barrier wait
// is bounded (a timeout reaches info); the ticketed chase hands out its work in
// order, so no workgroup waits on one that has not started.  No phase events are
// recorded.
bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  GEP_HIP(hipStreamIsCapturing(s, &cs));
  return cs != hipStreamCaptureStatusNone;
}

// One generalized eigenproblem, enqueued on s (arguments already validated).
// coop: launch the panel QR cooperatively (co-residency guaranteed by the runtime);
// prof: record the phase events.  mixed (vectors only): the interior GEMM tiles of
// R1, R2-4, S1, S5 and R5 run in FP32 arithmetic, S2-S4 and the diagonal blocks of
// the Cholesky stay FP64, and the eigenpairs are then refined in FP64 (REF).
// nvec: with vectors, the number of eigenvectors wanted (those of the nvec smallest
// eigenvalues; all when nvec < 0 or nvec >= M).  Fewer than M: the tridiagonal
// solver writes all M eigenvectors to the workspace, and only the first nvec
// columns are copied to Y and taken through the back transformations.
void solve_one(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
               double* lambda, double* Y, int64_t ldy, bool vectors, void* workspace,
               size_t ws_bytes, int32_t* info, hipStream_t s, bool coop, bool prof_on,
               bool mixed = false, int64_t nvec = -1) {
  fill_i32(info, 1, 0, s);
  if (M == 0) return;
  mixed = mixed && vectors;
  const int64_t k = (nvec < 0 || nvec > M) ? M : nvec;
  const bool partial = vectors && k < M;
  Plan p;
  Arena a;
  a.base = (char*)workspace;
  a.cap = ws_bytes;
  carve(p, a, M, vectors, mixed, partial);
  p.info = info;
  Prof prof(s);
  Prof* pp = prof_on ? &prof : nullptr;
  const MathMode trailing = mixed ? MathMode::Fp32 : MathMode::Fp64;
  MathScope scope(trailing);
  if (pp) pp->mark(0);
  reduce_steps(p, A, lda, B, ldb, info, s, pp);
  {
    Arena sa = scratch_arena(p);
    BandReduction r = band_of(p);
    r.coop = coop;
    sy2sb(r, sa, s);
  }
  if (pp) pp->mark(3);
  {
    BulgeChase c = chase_of(p);
    c.coop = coop;
    sb2st(c, s);
  }
  if (pp) pp->mark(4);
  if (!vectors) {
    stebz_ws(M, p.d, p.e, lambda, p.bounds, s);
    if (pp)
      for (int i = 5; i <= NPHASE; ++i) pp->mark(i);
    return;
  }
  {
    MathScope fp64(MathMode::Fp64);
    Arena sa = scratch_arena(p);
    stedc(M, p.d, p.e, lambda, partial ? p.Zd : Y, partial ? M : ldy, info, sa, s,
          (pp && g_prof) ? dc_flops_host() : nullptr);
    if (partial && k > 0) copy_matrix(M, k, p.Zd, M, Y, ldy, s);
  }
  if (pp) pp->mark(5);
  {
    Arena sa = scratch_arena(p);
    apply_q2(chase_of(p), Y, ldy, k, sa, s);
  }
  if (pp) pp->mark(6);
  {
    Arena sa = scratch_arena(p);
    apply_q1(band_of(p), Y, ldy, k, sa, s);
  }
  if (pp) pp->mark(7);
  trsm_llt(Tri{p.L, M, p.Linv, 0}, M, Y, ldy, k, p.tmp, s);
  if (pp) pp->mark(8);
  if (mixed) {
    // L and C are no longer needed: they are the refinement's M x M scratch
    Arena ra;
    ra.base = p.refine_ws;
    ra.cap = p.refine_bytes;
    refine(M, A, lda, B, ldb, Y, ldy, lambda, p.L, p.C, ra, p.coupling, info, s);
  }
  if (pp) pp->mark(9);
  if (k > 0) {
    hipLaunchKernelGGL(sign_fix_kernel, dim3((unsigned)k), dim3(256), 0, s, M, Y, ldy);
    GEP_LAUNCH_CHECK();
  }
  if (pp) pp->mark(10);
}

// Eigenvalues (ascending) and all eigenvectors of the symmetric matrix whose
// lower triangle is in p.C (destroyed): the SEP path S1 .. S5 into lam and Z.
void sep_vectors(const Plan& p, double* lam, double* Z, int64_t ldz, int32_t* info,
                 hipStream_t s) {
  const int64_t M = p.M;
  {
    Arena sa = scratch_arena(p);
    BandReduction r = band_of(p);
    r.coop = true;
    sy2sb(r, sa, s);
  }
  {
    BulgeChase c = chase_of(p);
    c.coop = true;
    sb2st(c, s);
  }
  {
    Arena sa = scratch_arena(p);
    stedc(M, p.d, p.e, lam, Z, ldz, info, sa, s);
  }
  {
    Arena sa = scratch_arena(p);
    apply_q2(chase_of(p), Z, ldz, M, sa, s);
  }
  {
    Arena sa = scratch_arena(p);
    apply_q1(band_of(p), Z, ldz, M, sa, s);
  }
}

// Extra workspace of the Cholesky-free solve beyond the plan: W (M x M) and D (M).
void carve_cholfree(Plan& p, Arena& a, int64_t M, double** W, double** dB) {
  carve(p, a, M, true);
  *W = a.take<double>((size_t)M * M);
  *dB = a.take<double>((size_t)M);
}

// Cholesky-free reducer (section 3.1, Eqs. 7-9): the SEP of B itself, B W = W D,
// replaces the Cholesky factorization; the reduced matrix is
// C = (W D^{-1/2})^T A (W D^{-1/2}) and the eigenvectors are Y = W D^{-1/2} Z, where
// C Z = Z Lambda.  Both SEPs run through the same two-stage path.  Phase events:
// 0 start, 1 after the SEP of B, 2 after C is formed, 3 after the SEP of C, 4 .. 10
// after Y.
void solve_cholfree(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
                    double* lambda, double* Y, int64_t ldy, void* workspace, size_t ws_bytes,
                    int32_t* info, hipStream_t s, bool prof_on) {
  fill_i32(info, 1, 0, s);
  if (M == 0) return;
  Plan p;
  Arena a;
  a.base = (char*)workspace;
  a.cap = ws_bytes;
  double *W = nullptr, *dB = nullptr;
  carve_cholfree(p, a, M, &W, &dB);
  p.info = info;
  Prof prof(s);
  Prof* pp = prof_on ? &prof : nullptr;
  MathScope fp64(MathMode::Fp64);
  if (pp) pp->mark(0);
  // B W = W D
  symmetrize_from_lower(M, B, ldb, p.C, M, s);
  sep_vectors(p, dB, W, M, info, s);
  if (pp) pp->mark(1);
  // W <- W D^{-1/2}; B is positive definite iff every d_j > 0
  hipLaunchKernelGGL(count_nonpositive, dim3(1), dim3(256), 0, s, M, (const double*)dB, info);
  GEP_LAUNCH_CHECK();
  hipLaunchKernelGGL(scale_cols_rsqrt, dim3((unsigned)M), dim3(256), 0, s, M, (const double*)dB, W,
                     M);
  GEP_LAUNCH_CHECK();
  // C = W^T (A W), lower triangle; p.L is the M x M product scratch
  symmetrize_from_lower(M, A, lda, p.C, M, s);
  {
    Gemm g;
    g.m = M; g.n = M; g.k = M;
    g.A = p.C; g.lda = M; g.B = W; g.ldb = M; g.C = p.L; g.ldc = M;
    gemm(g, s);
  }
  {
    Gemm g;
    g.transA = true;
    g.uplo = 1;
    g.m = M; g.n = M; g.k = M;
    g.A = W; g.lda = M; g.B = p.L; g.ldb = M; g.C = p.C; g.ldc = M;
    gemm(g, s);
  }
  if (pp) pp->mark(2);
  // C Z = Z Lambda, Z in p.L
  sep_vectors(p, lambda, p.L, M, info, s);
  if (pp) pp->mark(3);
  // Y = (W D^{-1/2}) Z
  {
    Gemm g;
    g.m = M; g.n = M; g.k = M;
    g.A = W; g.lda = M; g.B = p.L; g.ldb = M; g.C = Y; g.ldc = ldy;
    gemm(g, s);
  }
  hipLaunchKernelGGL(sign_fix_kernel, dim3((unsigned)M), dim3(256), 0, s, M, Y, ldy);
  GEP_LAUNCH_CHECK();
  if (pp)
    for (int i = 4; i <= NPHASE; ++i) pp->mark(i);
}

// X = alpha op(R) A, out of place, for a lower-triangular R (n x n, leading
// dimension ldr, upper triangle zero): op(R) = R, or R^T when trans.  A and X are
// n x ncols.  Recursive halving at a multiple of NB; M^3 flops for n = ncols = M
// instead of a full GEMM's 2 M^3.
void trmm_lower(bool trans, int64_t n, const double* R, int64_t ldr, const double* A,
                int64_t lda, double* X, int64_t ldx, int64_t ncols, hipStream_t s,
                double alpha = 1.0) {
  if (n <= 0 || ncols <= 0) return;
  if (n <= NB) {
    Gemm g;
    g.transA = trans;
    g.alpha = alpha;
    g.m = n; g.n = ncols; g.k = n;
    g.A = R; g.lda = ldr; g.B = A; g.ldb = lda; g.C = X; g.ldc = ldx;
    gemm(g, s);
    return;
  }
  const int64_t n1 = NB * ((cdiv(n, NB) + 1) / 2), n2 = n - n1;
  const double* R21 = R + n1;               // n2 x n1
  const double* R22 = R + n1 + n1 * ldr;    // n2 x n2
  trmm_lower(trans, n1, R, ldr, A, lda, X, ldx, ncols, s, alpha);
  trmm_lower(trans, n2, R22, ldr, A + n1, lda, X + n1, ldx, ncols, s, alpha);
  Gemm g;
  g.alpha = alpha;
  g.beta = 1.0;
  g.n = ncols;
  g.A = R21; g.lda = ldr; g.ldb = lda; g.ldc = ldx;
  if (!trans) {  // X2 += R21 A1
    g.m = n2; g.k = n1;
    g.B = A; g.C = X + n1;
  } else {       // X1 += R21^T A2
    g.transA = true;
    g.m = n1; g.k = n2;
    g.B = A + n1; g.C = X;
  }
  gemm(g, s);
}

// X = A R, out of place, for a lower-triangular R (n x n, upper triangle zero) and
// A, X of m x n: [X1 X2] = [A1 R11 + A2 R21, A2 R22].
void trmm_right_lower(int64_t m, int64_t n, const double* A, int64_t lda, const double* R,
                      int64_t ldr, double* X, int64_t ldx, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  if (n <= NB) {
    Gemm g;
    g.m = m; g.n = n; g.k = n;
    g.A = A; g.lda = lda; g.B = R; g.ldb = ldr; g.C = X; g.ldc = ldx;
    gemm(g, s);
    return;
  }
  const int64_t n1 = NB * ((cdiv(n, NB) + 1) / 2), n2 = n - n1;
  trmm_right_lower(m, n1, A, lda, R, ldr, X, ldx, s);
  trmm_right_lower(m, n2, A + n1 * lda, lda, R + n1 + n1 * ldr, ldr, X + n1 * ldx, ldx, s);
  Gemm g;  // X1 += A2 R21
  g.beta = 1.0;
  g.m = m; g.n = n1; g.k = n2;
  g.A = A + n1 * lda; g.lda = lda; g.B = R + n1; g.ldb = ldr; g.C = X; g.ldc = ldx;
  gemm(g, s);
}

// R = L^{-1} for the Cholesky factor's diagonal block at global offset `off` (a
// multiple of NB) of order n: the NB x NB leaves are the inverses the Cholesky
// already formed (Linv), and above them R21 = -R22 (L21 R11), two triangular
// multiplies; M^3 / 3 flops in all.  R's upper triangle must be zero on entry;
// T is scratch for the n/2 x n/2 product (leading dimension ldt).
void trtri_lower(int64_t n, const double* L, int64_t ldl, const double* Linv, int64_t off,
                 double* R, int64_t ldr, double* T, int64_t ldt, hipStream_t s) {
  if (n <= 0) return;
  if (n <= NB) {
    copy_matrix(n, n, Linv + (off / NB) * (int64_t)NB * NB, NB, R, ldr, s);
    return;
  }
  const int64_t n1 = NB * ((cdiv(n, NB) + 1) / 2), n2 = n - n1;
  trtri_lower(n1, L, ldl, Linv, off, R, ldr, T, ldt, s);
  trtri_lower(n2, L + n1 + n1 * ldl, ldl, Linv, off + n1, R + n1 + n1 * ldr, ldr, T, ldt, s);
  trmm_right_lower(n2, n1, L + n1, ldl, R, ldr, T, ldt, s);                   // T = L21 R11
  trmm_lower(false, n2, R + n1 + n1 * ldr, ldr, T, ldt, R + n1, ldr, n1, s, -1.0);  // R21
}

// Explicit-inverse (ELPA-style) reducer (section 3.1): after B = L L^T the inverse
// R = L^{-1} is formed explicitly (recursive triangular inversion from the
// Cholesky's inverted diagonal blocks; its upper triangle is zero), the reduced
// matrix is formed
// by two successive matrix products, C = (R A) R^T (a triangular multiply, then the
// lower triangle of a GEMM), and the back transformation is one triangular
// multiply, Y = R^T Z.  Phase events: 0 start,
// 1 after the Cholesky factorization, 2 after C is formed, 3 after the SEP of C,
// 4 .. 10 after Y.
void solve_explicit_inverse(int64_t M, const double* A, int64_t lda, const double* B,
                            int64_t ldb, double* lambda, double* Y, int64_t ldy, void* workspace,
                            size_t ws_bytes, int32_t* info, hipStream_t s, bool prof_on) {
  fill_i32(info, 1, 0, s);
  if (M == 0) return;
  Plan p;
  Arena a;
  a.base = (char*)workspace;
  a.cap = ws_bytes;
  carve(p, a, M, true);
  p.info = info;
  double* R = a.take<double>((size_t)M * M);
  Prof prof(s);
  Prof* pp = prof_on ? &prof : nullptr;
  MathScope fp64(MathMode::Fp64);
  if (pp) pp->mark(0);
  // B = L L^T
  copy_matrix(M, M, B, ldb, p.L, M, s);
  potrf_rec(p.L, M, M, 0, p.Linv, info, M, p.tmp, s);
  if (pp) pp->mark(1);
  // R = L^{-1} (p.C is the scratch of the recursion)
  set_matrix(M, M, 0.0, 0.0, R, M, s);
  trtri_lower(M, p.L, M, p.Linv, 0, R, M, p.C, M, s);
  // X = R A (into p.L: L is no longer needed), then C = X R^T, lower triangle
  symmetrize_from_lower(M, A, lda, p.C, M, s);
  trmm_lower(false, M, R, M, p.C, M, p.L, M, M, s);
  {
    Gemm g;
    g.transB = true;
    g.uplo = 1;
    g.m = M; g.n = M; g.k = M;
    g.A = p.L; g.lda = M; g.B = R; g.ldb = M; g.C = p.C; g.ldc = M;
    gemm(g, s);
  }
  if (pp) pp->mark(2);
  // C Z = Z Lambda, Z in p.L
  sep_vectors(p, lambda, p.L, M, info, s);
  if (pp) pp->mark(3);
  // Y = R^T Z
  trmm_lower(true, M, R, M, p.L, M, Y, ldy, M, s);
  hipLaunchKernelGGL(sign_fix_kernel, dim3((unsigned)M), dim3(256), 0, s, M, Y, ldy);
  GEP_LAUNCH_CHECK();
  if (pp)
    for (int i = 4; i <= NPHASE; ++i) pp->mark(i);
}

// Block Jacobi SEP solver behind the reducer (the combination the paper's outlook
// proposes, section 6): B = L L^T and C = L^{-1} A L^{-T} as in gep_solve, then
// the eigenpairs of C by parallel block Jacobi, then Y = L^{-T} Z.  Phase events:
// 0 start, 1 after the Cholesky factorization, 2 after C, 3 after the Jacobi
// sweeps, 4 .. 10 after Y.
int g_last_jacobi_sweeps = 0;

struct JacobiPlan {
  double *L, *Linv, *tmp, *C;
  char* ws;
  size_t ws_bytes;
};

void carve_jacobi(JacobiPlan& p, Arena& a, int64_t M) {
  p.L = a.take<double>((size_t)M * M);
  p.Linv = a.take<double>((size_t)cdiv(M, NB) * NB * NB);
  p.tmp = a.take<double>((size_t)NB * M);
  p.C = a.take<double>((size_t)M * M);
  p.ws_bytes = jacobi_workspace(M);
  p.ws = a.take<char>(p.ws_bytes);
}

void solve_jacobi(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
                  double* lambda, double* Y, int64_t ldy, void* workspace, size_t ws_bytes,
                  int32_t* info, hipStream_t s, bool prof_on) {
  fill_i32(info, 1, 0, s);
  if (M == 0) return;
  JacobiPlan jp;
  Arena a;
  a.base = (char*)workspace;
  a.cap = ws_bytes;
  carve_jacobi(jp, a, M);
  Prof prof(s);
  Prof* pp = prof_on ? &prof : nullptr;
  MathScope fp64(MathMode::Fp64);
  if (pp) pp->mark(0);
  copy_matrix(M, M, B, ldb, jp.L, M, s);
  potrf_rec(jp.L, M, M, 0, jp.Linv, info, M, jp.tmp, s);
  if (pp) pp->mark(1);
  symmetrize_from_lower(M, A, lda, jp.C, M, s);
  Tri t{jp.L, M, jp.Linv, 0};
  trsm_lln(t, M, jp.C, M, M, jp.tmp, s);
  trsm_rlt_lower(t, M, jp.C, M, jp.tmp, s);
  symmetrize_from_lower(M, jp.C, M, jp.C, M, s);
  if (pp) pp->mark(2);
  Arena ja;
  ja.base = jp.ws;
  ja.cap = jp.ws_bytes;
  g_last_jacobi_sweeps = jacobi_eig(M, jp.C, M, lambda, Y, ldy, info, ja, s);
  if (pp) pp->mark(3);
  trsm_llt(t, M, Y, ldy, M, jp.tmp, s);
  hipLaunchKernelGGL(sign_fix_kernel, dim3((unsigned)M), dim3(256), 0, s, M, Y, ldy);
  GEP_LAUNCH_CHECK();
  if (pp)
    for (int i = 4; i <= NPHASE; ++i) pp->mark(i);
}

// ---------------------------------------------------------------- batches
// Instances run on NSTREAM worker streams forked from the caller's stream with
// events (so the whole batch can be captured in one graph).  Longest-processing-
// time order: instances sorted by M^3, each to the least loaded stream; every
// stream owns one workspace slot sized for its largest instance.
constexpr int NSTREAM = 16;

struct BatchPlan {
  std::vector<int> order;          // instance indices, largest first
  std::vector<int> lane;           // instance -> stream
  std::vector<size_t> slot_off;    // stream -> byte offset of its workspace slot
  std::vector<size_t> slot_bytes;
  size_t total = 0;
};

BatchPlan plan_batch(int batch, const int64_t* Mh, bool vectors) {
  BatchPlan bp;
  bp.order.resize(batch);
  for (int i = 0; i < batch; ++i) bp.order[i] = i;
  std::stable_sort(bp.order.begin(), bp.order.end(),
                   [&](int a, int b) { return Mh[a] > Mh[b]; });
  bp.lane.assign(batch, 0);
  // Plain-launched panel grids spin at a barrier until all their workgroups are
  // resident; keep the sum of concurrently possible grids within half the CUs.
  int64_t gmax = 1;
  for (int i = 0; i < batch; ++i) {
    const int64_t g = cdiv(Mh[i] > 0 ? Mh[i] : 1, 256);
    if (g > gmax) gmax = g;
  }
  int nlanes = (int)(128 / gmax);
  if (nlanes < 1) nlanes = 1;
  if (nlanes > NSTREAM) nlanes = NSTREAM;
  std::vector<double> load(NSTREAM, 0.0);
  std::vector<int64_t> maxm(NSTREAM, 0);
  for (int i : bp.order) {
    int best = 0;
    for (int k = 1; k < nlanes; ++k)
      if (load[k] < load[best]) best = k;
    bp.lane[i] = best;
    load[best] += (double)Mh[i] * Mh[i] * Mh[i];
    if (Mh[i] > maxm[best]) maxm[best] = Mh[i];
  }
  bp.slot_off.assign(NSTREAM, 0);
  bp.slot_bytes.assign(NSTREAM, 0);
  size_t off = 0;
  for (int k = 0; k < NSTREAM; ++k) {
    size_t bytes = 0;
    if (maxm[k] > 0) {
      Plan p;
      Arena a;
      a.dry = true;
      carve(p, a, maxm[k], vectors);
      bytes = (a.used + 255) & ~size_t(255);
    }
    bp.slot_off[k] = off;
    bp.slot_bytes[k] = bytes;
    off += bytes;
  }
  bp.total = off + 256;
  return bp;
}

bool g_batched_threads = true;
bool batched_threads() { return g_batched_threads; }

struct Workers {
  hipStream_t st[NSTREAM];
  hipEvent_t fork;
  hipEvent_t join[NSTREAM];
  bool ok = false;
};

Workers& workers() {
  static Workers w;
  if (!w.ok) {
    for (int k = 0; k < NSTREAM; ++k) {
      GEP_HIP(hipStreamCreateWithFlags(&w.st[k], hipStreamNonBlocking));
      GEP_HIP(hipEventCreateWithFlags(&w.join[k], hipEventDisableTiming));
    }
    GEP_HIP(hipEventCreateWithFlags(&w.fork, hipEventDisableTiming));
    w.ok = true;
  }
  return w;
}

// ---------------------------------------------------------------- allocation-free solves
// gep_solve_noalloc's workspace: one array per device, part of the library's
// device image, so using it allocates nothing.  In host code `scratch` is only a
// stand-in for the symbol: its device address comes from hipGetSymbolAddress,
// once per device with that device current, and only that address is ever
// passed to a kernel.  Every call on a device shares the array, so calls that
// overlap on one device race; the solve clears everything it needs cleared.
constexpr size_t NOALLOC_BYTES = (size_t)272 << 20;
static __device__ __align__(256) char scratch[NOALLOC_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`.
void* scratch_on_current_device() {
  int dev = 0;
  GEP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw HipError{hipErrorInvalidDevice, "device index"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    GEP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw HipError{hipErrorInvalidSymbol, "scratch address"};
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace gep

using namespace gep;

extern "C" {

const char* gep_status_string(int status) {
  switch (status) {
    case GEP_OK: return "ok";
    case GEP_ERR_ARG: return "invalid argument";
    case GEP_ERR_WORKSPACE: return "workspace too small";
    case GEP_ERR_HIP: return "HIP runtime error";
    case GEP_ERR_NO_DEVICE: return "no gfx950 device";
    case GEP_ERR_INTERNAL: return "internal error";
    default: return "unknown status";
  }
}

int gep_last_bad_arg(void) { return g_bad_arg; }

const char* gep_version(void) { return "libgep 0.2 (gfx950; FP64 and FP32/FP64 mixed)"; }

size_t gep_workspace_size(int64_t M, int job, int prec) {
  if (M <= 0) return 256;
  Plan p;
  Arena a;
  a.dry = true;
  carve(p, a, M, job == GEP_JOB_VECTORS, prec == GEP_PREC_MIXED && job == GEP_JOB_VECTORS);
  return a.used + 256;
}

int gep_solve(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
              double* lambda, double* Y, int64_t ldy, int job, int prec, void* workspace,
              size_t ws_bytes, int32_t* info, void* stream) {
  g_bad_arg = 0;
  if (M < 0) return bad(1);
  const int64_t m1 = M > 1 ? M : 1;
  if (M > 0 && !A) return bad(2);
  if (lda < m1) return bad(3);
  if (M > 0 && !B) return bad(4);
  if (ldb < m1) return bad(5);
  if (M > 0 && !lambda) return bad(6);
  if (job != GEP_JOB_VALUES && job != GEP_JOB_VECTORS) return bad(9);
  if (job == GEP_JOB_VECTORS) {
    if (M > 0 && !Y) return bad(7);
    if (ldy < m1) return bad(8);
  }
  if (prec != GEP_PREC_FP64 && !(prec == GEP_PREC_MIXED && job == GEP_JOB_VECTORS)) return bad(10);
  if (!info) return bad(13);
  const size_t need = gep_workspace_size(M, job, prec);
  if (M > 0 && (!workspace || ((uintptr_t)workspace & 255))) return bad(11);
  if (ws_bytes < need) return GEP_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    const bool eager = !stream_capturing(s);
    solve_one(M, A, lda, B, ldb, lambda, Y, ldy, job == GEP_JOB_VECTORS, workspace, ws_bytes, info,
              s, eager, eager, prec == GEP_PREC_MIXED);
    return GEP_OK;
  });
}

int gep_solve_noalloc(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
                      double* lambda, double* Y, int64_t ldy, int job, int prec, int32_t* info,
                      void* stream) {
  g_bad_arg = 0;
  if (M < 0) return bad(1);
  const int64_t m1 = M > 1 ? M : 1;
  if (M > 0 && !A) return bad(2);
  if (lda < m1) return bad(3);
  if (M > 0 && !B) return bad(4);
  if (ldb < m1) return bad(5);
  if (M > 0 && !lambda) return bad(6);
  if (job != GEP_JOB_VALUES && job != GEP_JOB_VECTORS) return bad(9);
  if (job == GEP_JOB_VECTORS) {
    if (M > 0 && !Y) return bad(7);
    if (ldy < m1) return bad(8);
  }
  if (prec != GEP_PREC_FP64 && !(prec == GEP_PREC_MIXED && job == GEP_JOB_VECTORS)) return bad(10);
  if (!info) return bad(11);
  const size_t need = gep_workspace_size(M, job, prec);
  if (need > NOALLOC_BYTES) return GEP_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    void* ws = scratch_on_current_device();
    // no phase events: creating them is the one resource a profiled gep_solve adds
    solve_one(M, A, lda, B, ldb, lambda, Y, ldy, job == GEP_JOB_VECTORS, ws, NOALLOC_BYTES, info,
              s, !stream_capturing(s), false, prec == GEP_PREC_MIXED);
    return GEP_OK;
  });
}

size_t gep_noalloc_max_bytes(void) { return NOALLOC_BYTES; }

size_t gep_workspace_size_lowest(int64_t M, int64_t k) {
  if (M <= 0) return 256;
  Plan p;
  Arena a;
  a.dry = true;
  carve(p, a, M, true, false, k >= 0 && k < M);
  return a.used + 256;
}

int gep_solve_lowest(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
                     int64_t k, double* lambda, double* Y, int64_t ldy, void* workspace,
                     size_t ws_bytes, int32_t* info, void* stream) {
  g_bad_arg = 0;
  if (M < 0) return bad(1);
  const int64_t m1 = M > 1 ? M : 1;
  if (M > 0 && !A) return bad(2);
  if (lda < m1) return bad(3);
  if (M > 0 && !B) return bad(4);
  if (ldb < m1) return bad(5);
  if (k < 0 || k > M) return bad(6);
  if (M > 0 && !lambda) return bad(7);
  if (k > 0 && !Y) return bad(8);
  if (ldy < m1) return bad(9);
  if (!info) return bad(12);
  if (M > 0 && (!workspace || ((uintptr_t)workspace & 255))) return bad(10);
  if (ws_bytes < gep_workspace_size_lowest(M, k)) return GEP_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    const bool eager = !stream_capturing(s);
    solve_one(M, A, lda, B, ldb, lambda, Y, ldy, true, workspace, ws_bytes, info, s, eager, eager,
              false, k);
    return GEP_OK;
  });
}

size_t gep_workspace_size_cholfree(int64_t M) {
  if (M <= 0) return 256;
  Plan p;
  Arena a;
  a.dry = true;
  double *W = nullptr, *dB = nullptr;
  carve_cholfree(p, a, M, &W, &dB);
  return a.used + 256;
}

int gep_solve_cholfree(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
                       double* lambda, double* Y, int64_t ldy, void* workspace, size_t ws_bytes,
                       int32_t* info, void* stream) {
  g_bad_arg = 0;
  if (M < 0) return bad(1);
  const int64_t m1 = M > 1 ? M : 1;
  if (M > 0 && !A) return bad(2);
  if (lda < m1) return bad(3);
  if (M > 0 && !B) return bad(4);
  if (ldb < m1) return bad(5);
  if (M > 0 && !lambda) return bad(6);
  if (M > 0 && !Y) return bad(7);
  if (ldy < m1) return bad(8);
  if (!info) return bad(11);
  if (M > 0 && (!workspace || ((uintptr_t)workspace & 255))) return bad(9);
  if (ws_bytes < gep_workspace_size_cholfree(M)) return GEP_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    solve_cholfree(M, A, lda, B, ldb, lambda, Y, ldy, workspace, ws_bytes, info, s, true);
    return GEP_OK;
  });
}

size_t gep_workspace_size_explicit_inverse(int64_t M) {
  if (M <= 0) return 256;
  Plan p;
  Arena a;
  a.dry = true;
  carve(p, a, M, true);
  a.take<double>((size_t)M * M);
  return a.used + 256;
}

int gep_solve_explicit_inverse(int64_t M, const double* A, int64_t lda, const double* B,
                               int64_t ldb, double* lambda, double* Y, int64_t ldy,
                               void* workspace, size_t ws_bytes, int32_t* info, void* stream) {
  g_bad_arg = 0;
  if (M < 0) return bad(1);
  const int64_t m1 = M > 1 ? M : 1;
  if (M > 0 && !A) return bad(2);
  if (lda < m1) return bad(3);
  if (M > 0 && !B) return bad(4);
  if (ldb < m1) return bad(5);
  if (M > 0 && !lambda) return bad(6);
  if (M > 0 && !Y) return bad(7);
  if (ldy < m1) return bad(8);
  if (!info) return bad(11);
  if (M > 0 && (!workspace || ((uintptr_t)workspace & 255))) return bad(9);
  if (ws_bytes < gep_workspace_size_explicit_inverse(M)) return GEP_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    solve_explicit_inverse(M, A, lda, B, ldb, lambda, Y, ldy, workspace, ws_bytes, info, s, true);
    return GEP_OK;
  });
}

size_t gep_workspace_size_jacobi(int64_t M) {
  if (M <= 0) return 256;
  JacobiPlan jp;
  Arena a;
  a.dry = true;
  carve_jacobi(jp, a, M);
  return a.used + 256;
}

int gep_solve_jacobi(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb,
                     double* lambda, double* Y, int64_t ldy, void* workspace, size_t ws_bytes,
                     int32_t* info, void* stream) {
  g_bad_arg = 0;
  if (M < 0) return bad(1);
  const int64_t m1 = M > 1 ? M : 1;
  if (M > 0 && !A) return bad(2);
  if (lda < m1) return bad(3);
  if (M > 0 && !B) return bad(4);
  if (ldb < m1) return bad(5);
  if (M > 0 && !lambda) return bad(6);
  if (M > 0 && !Y) return bad(7);
  if (ldy < m1) return bad(8);
  if (!info) return bad(11);
  if (M > 0 && (!workspace || ((uintptr_t)workspace & 255))) return bad(9);
  if (ws_bytes < gep_workspace_size_jacobi(M)) return GEP_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    solve_jacobi(M, A, lda, B, ldb, lambda, Y, ldy, workspace, ws_bytes, info, s, true);
    return GEP_OK;
  });
}

int gep_last_jacobi_sweeps(void) { return g_last_jacobi_sweeps; }

size_t gep_workspace_size_batched(int batch, const int64_t* M_host, int job, int prec) {
  (void)prec;
  if (batch <= 0 || !M_host) return 256;
  return plan_batch(batch, M_host, job == GEP_JOB_VECTORS).total;
}

int gep_solve_batched(int batch, const int64_t* M_host, const double* const* A_host,
                      const int64_t* lda_host, const double* const* B_host,
                      const int64_t* ldb_host, double* const* lambda_host, double* const* Y_host,
                      const int64_t* ldy_host, int job, int prec, void* workspace, size_t ws_bytes,
                      int32_t* info, void* stream) {
  g_bad_arg = 0;
  if (batch < 0) return bad(1);
  if (batch == 0) return GEP_OK;
  if (!M_host) return bad(2);
  if (!A_host) return bad(3);
  if (!lda_host) return bad(4);
  if (!B_host) return bad(5);
  if (!ldb_host) return bad(6);
  if (!lambda_host) return bad(7);
  if (job != GEP_JOB_VALUES && job != GEP_JOB_VECTORS) return bad(10);
  const bool vectors = job == GEP_JOB_VECTORS;
  if (vectors && (!Y_host || !ldy_host)) return bad(8);
  if (prec != GEP_PREC_FP64) return bad(11);
  for (int i = 0; i < batch; ++i) {
    const int64_t M = M_host[i];
    const int64_t m1 = M > 1 ? M : 1;
    if (M < 0) return bad(2);
    if (M > 0 && (!A_host[i] || !B_host[i] || !lambda_host[i])) return bad(3);
    if (lda_host[i] < m1) return bad(4);
    if (ldb_host[i] < m1) return bad(6);
    if (vectors && ((M > 0 && !Y_host[i]) || ldy_host[i] < m1)) return bad(9);
  }
  if (!info) return bad(14);
  const BatchPlan bp = plan_batch(batch, M_host, vectors);
  if (ws_bytes < bp.total) return GEP_ERR_WORKSPACE;
  if (!workspace || ((uintptr_t)workspace & 255)) return bad(12);
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    Workers& w = workers();
    GEP_HIP(hipEventRecord(w.fork, s));
    for (int k = 0; k < NSTREAM; ++k) GEP_HIP(hipStreamWaitEvent(w.st[k], w.fork, 0));
    auto lane_work = [&](int k) {
      for (int i : bp.order) {
        if (bp.lane[i] != k) continue;
        solve_one(M_host[i], A_host[i], lda_host[i], B_host[i], ldb_host[i], lambda_host[i],
                  vectors ? Y_host[i] : nullptr, vectors ? ldy_host[i] : 1, vectors,
                  (char*)workspace + bp.slot_off[k], bp.slot_bytes[k], info + i, w.st[k], false,
                  false);
      }
    };
    // Each instance is a few hundred small launches, so one host thread cannot
    // keep 16 streams fed: outside graph capture every stream's instances are
    // enqueued by a thread of its own (the launches and their order on each
    // stream are the same as from one thread, so the results are too).  Under
    // capture one thread enqueues everything.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    GEP_HIP(hipStreamIsCapturing(s, &cs));
    int lanes = 0;
    for (int k = 0; k < NSTREAM; ++k)
      if (bp.slot_bytes[k] > 0) ++lanes;
    if (cs == hipStreamCaptureStatusNone && lanes > 1 && batched_threads()) {
      int dev = 0;
      GEP_HIP(hipGetDevice(&dev));
      std::vector<int> rc(NSTREAM, GEP_OK);
      std::vector<std::thread> th;
      for (int k = 0; k < NSTREAM; ++k) {
        if (bp.slot_bytes[k] == 0) continue;
        th.emplace_back([&, k]() {
          rc[k] = guarded([&]() -> int {
            GEP_HIP(hipSetDevice(dev));
            lane_work(k);
            return GEP_OK;
          });
        });
      }
      for (auto& t : th) t.join();
      for (int k = 0; k < NSTREAM; ++k)
        if (rc[k] != GEP_OK) return rc[k];
    } else {
      for (int k = 0; k < NSTREAM; ++k) lane_work(k);
    }
    for (int k = 0; k < NSTREAM; ++k) {
      GEP_HIP(hipEventRecord(w.join[k], w.st[k]));
      GEP_HIP(hipStreamWaitEvent(s, w.join[k], 0));
    }
    return GEP_OK;
  });
}

size_t gep_reduce_workspace_size(int64_t M) {
  if (M <= 0) return 256;
  Arena a;
  a.dry = true;
  a.take<double>((size_t)cdiv(M, NB) * NB * NB);
  a.take<double>((size_t)NB * M);
  return a.used + 256;
}

int gep_reduce(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb, double* L,
               int64_t ldl, double* C, int64_t ldc, void* workspace, size_t ws_bytes,
               int32_t* info, void* stream) {
  g_bad_arg = 0;
  if (M < 0) return bad(1);
  const int64_t m1 = M > 1 ? M : 1;
  if (M > 0 && !A) return bad(2);
  if (lda < m1) return bad(3);
  if (M > 0 && !B) return bad(4);
  if (ldb < m1) return bad(5);
  if (M > 0 && !L) return bad(6);
  if (ldl < m1) return bad(7);
  if (M > 0 && !C) return bad(8);
  if (ldc < m1) return bad(9);
  if (!info) return bad(12);
  if (ws_bytes < gep_reduce_workspace_size(M)) return GEP_ERR_WORKSPACE;
  if (M > 0 && (!workspace || ((uintptr_t)workspace & 255))) return bad(10);
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    fill_i32(info, 1, 0, s);
    if (M == 0) return GEP_OK;
    Arena a;
    a.base = (char*)workspace;
    a.cap = ws_bytes;
    double* linv = a.take<double>((size_t)cdiv(M, NB) * NB * NB);
    double* tmp = a.take<double>((size_t)NB * M);
    copy_matrix(M, M, B, ldb, L, ldl, s);
    potrf_rec(L, ldl, M, 0, linv, info, M, tmp, s);
    symmetrize_from_lower(M, A, lda, C, ldc, s);
    Tri t{L, ldl, linv, 0};
    trsm_lln(t, M, C, ldc, M, tmp, s);
    trsm_rlt_lower(t, M, C, ldc, tmp, s);
    // outputs: L with zero strict upper triangle, C full symmetric
    zero_upper(M, L, ldl, s);
    symmetrize_from_lower(M, C, ldc, C, ldc, s);
    return GEP_OK;
  });
}

size_t gep_band_reduce_workspace_size(int64_t M, int band_width) {
  if (M <= 0) return 256;
  const int b = band_width > 0 ? band_width : default_band(M);
  Arena a;
  a.dry = true;
  a.take<double>((size_t)M * M);
  a.take<double>((size_t)cdiv(M, b) * b * b);
  a.take<double>((size_t)(2 * b + 1) * M);
  a.take<char>(sy2sb_workspace(M, b));
  return a.used + 256;
}

int gep_band_reduce(int64_t M, const double* C, int64_t ldc, int band_width, double* band,
                    int64_t ldband, void* workspace, size_t ws_bytes, void* stream) {
  g_bad_arg = 0;
  if (M < 0) return bad(1);
  const int64_t m1 = M > 1 ? M : 1;
  if (M > 0 && !C) return bad(2);
  if (ldc < m1) return bad(3);
  if (band_width < 0 || band_width > 64) return bad(4);
  const int b = band_width > 0 ? band_width : default_band(M);
  if (M > 0 && !band) return bad(5);
  if (ldband < b + 1) return bad(6);
  if (ws_bytes < gep_band_reduce_workspace_size(M, band_width)) return GEP_ERR_WORKSPACE;
  if (M > 0 && (!workspace || ((uintptr_t)workspace & 255))) return bad(7);
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    if (M == 0) return GEP_OK;
    Arena a;
    a.base = (char*)workspace;
    a.cap = ws_bytes;
    BandReduction r;
    r.n = M; r.b = b;
    r.C = a.take<double>((size_t)M * M);
    r.ldc = M;
    r.T = a.take<double>((size_t)cdiv(M, b) * b * b);
    r.ldband = 2 * b + 1;
    r.band = a.take<double>((size_t)r.ldband * M);
    Arena sa;
    sa.cap = sy2sb_workspace(M, b);
    sa.base = a.take<char>(sa.cap);
    copy_matrix(M, M, C, ldc, r.C, M, s);
    sy2sb(r, sa, s);
    hipLaunchKernelGGL(band_copy_out, dim3((unsigned)cdiv(M, 256)), dim3(256), 0, s, M, b,
                       (const double*)r.band, r.ldband, band, ldband);
    GEP_LAUNCH_CHECK();
    return GEP_OK;
  });
}

size_t gep_tridiagonalize_workspace_size(int64_t M, int band_width) {
  if (M <= 0) return 256;
  const int b = band_width > 0 ? band_width : default_band(M);
  Arena a;
  a.dry = true;
  a.take<double>((size_t)M * M);
  a.take<double>((size_t)cdiv(M, b) * b * b);
  a.take<double>((size_t)(2 * b + 1) * M);
  a.take<int32_t>(M + 8);
  a.take<int32_t>(1);
  a.take<char>(sy2sb_workspace(M, b));
  return a.used + 256;
}

int gep_tridiagonalize(int64_t M, const double* C, int64_t ldc, int band_width, double* d,
                       double* e, void* workspace, size_t ws_bytes, void* stream) {
  g_bad_arg = 0;
  if (M < 0) return bad(1);
  const int64_t m1 = M > 1 ? M : 1;
  if (M > 0 && !C) return bad(2);
  if (ldc < m1) return bad(3);
  if (band_width < 0 || band_width > 64) return bad(4);
  const int b = band_width > 0 ? band_width : default_band(M);
  if (M > 0 && !d) return bad(5);
  if (M > 1 && !e) return bad(6);
  if (ws_bytes < gep_tridiagonalize_workspace_size(M, band_width)) return GEP_ERR_WORKSPACE;
  if (M > 0 && (!workspace || ((uintptr_t)workspace & 255))) return bad(7);
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    if (M == 0) return GEP_OK;
    Arena a;
    a.base = (char*)workspace;
    a.cap = ws_bytes;
    BandReduction r;
    r.n = M; r.b = b;
    r.C = a.take<double>((size_t)M * M);
    r.ldc = M;
    r.T = a.take<double>((size_t)cdiv(M, b) * b * b);
    r.ldband = 2 * b + 1;
    r.band = a.take<double>((size_t)r.ldband * M);
    int32_t* sync = a.take<int32_t>(M + 8);
    int32_t* err = a.take<int32_t>(1);
    Arena sa;
    sa.cap = sy2sb_workspace(M, b);
    sa.base = a.take<char>(sa.cap);
    copy_matrix(M, M, C, ldc, r.C, M, s);
    sy2sb(r, sa, s);
    BulgeChase c;
    c.n = M; c.b = b; c.band = r.band; c.ldband = r.ldband; c.d = d;
    double* e_or_dummy = e ? e : r.T;  // e unused for M = 1
    c.e = e_or_dummy;
    c.V = nullptr; c.tau = nullptr; c.kmax = M > 1 ? cdiv(M - 1, b) : 1;
    c.sync = sync; c.err = err;
    c.coop = true;
    c.msg = (double*)sa.base;  // the band reduction's workspace, idle now
    c.msg_bytes = sa.cap;
    sb2st(c, s);
    return GEP_OK;
  });
}

size_t gep_tridiag_eig_workspace_size(int64_t M, int job) {
  if (M <= 0) return 256;
  if (job == GEP_JOB_VALUES) return 4096;
  return stedc_workspace(M) + 256;
}

int gep_tridiag_eig(int64_t M, const double* d, const double* e, double* lambda, double* Z,
                    int64_t ldz, int job, void* workspace, size_t ws_bytes, int32_t* info,
                    void* stream) {
  g_bad_arg = 0;
  if (M < 0) return bad(1);
  const int64_t m1 = M > 1 ? M : 1;
  if (M > 0 && !d) return bad(2);
  if (M > 1 && !e) return bad(3);
  if (M > 0 && !lambda) return bad(4);
  if (job != GEP_JOB_VALUES && job != GEP_JOB_VECTORS) return bad(7);
  if (job == GEP_JOB_VECTORS) {
    if (M > 0 && !Z) return bad(5);
    if (ldz < m1) return bad(6);
  }
  if (!info) return bad(10);
  if (ws_bytes < gep_tridiag_eig_workspace_size(M, job)) return GEP_ERR_WORKSPACE;
  if (M > 0 && (!workspace || ((uintptr_t)workspace & 255))) return bad(8);
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    fill_i32(info, 1, 0, s);
    if (M == 0) return GEP_OK;
    Arena a;
    a.base = (char*)workspace;
    a.cap = ws_bytes;
    if (job == GEP_JOB_VALUES) {
      double* bounds = a.take<double>(2);
      stebz_ws(M, d, e, lambda, bounds, s);
    } else {
      stedc(M, d, e, lambda, Z, ldz, info, a, s);
    }
    return GEP_OK;
  });
}

size_t gep_backward_workspace_size(int64_t M) {
  if (M <= 0) return 256;
  return backward_workspace(M);
}

int gep_backward(int64_t M, const double* lambda, const double* Y, int64_t ldy,
                 const double* lambda_bar, const double* Y_bar, int64_t ldyb, double eta,
                 double tau_c, double* A_bar, int64_t ldab, double* B_bar, int64_t ldbb,
                 void* workspace, size_t ws_bytes, void* stream) {
  g_bad_arg = 0;
  if (M < 0) return bad(1);
  const int64_t m1 = M > 1 ? M : 1;
  if (M > 0 && !lambda) return bad(2);
  if (M > 0 && !Y) return bad(3);
  if (ldy < m1) return bad(4);
  if (Y_bar && ldyb < m1) return bad(7);
  if (!(eta >= 0.0)) return bad(8);
  if (!(tau_c >= 0.0)) return bad(9);
  if (M > 0 && !A_bar) return bad(10);
  if (ldab < m1) return bad(11);
  if (M > 0 && !B_bar) return bad(12);
  if (ldbb < m1) return bad(13);
  if (ws_bytes < gep_backward_workspace_size(M)) return GEP_ERR_WORKSPACE;
  if (M > 0 && (!workspace || ((uintptr_t)workspace & 255))) return bad(14);
  hipStream_t s = (hipStream_t)stream;
  return guarded([&]() -> int {
    if (M == 0) return GEP_OK;
    Arena a;
    a.base = (char*)workspace;
    a.cap = ws_bytes;
    backward(M, lambda, Y, ldy, lambda_bar, Y_bar, ldyb, eta, tau_c, A_bar, ldab, B_bar, ldbb, a,
             s);
    return GEP_OK;
  });
}

int gep_dgemm(int transA, int transB, int uplo, int64_t m, int64_t n, int64_t k, double alpha,
              const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
              int64_t ldc, int arith, void* stream) {
  g_bad_arg = 0;
  if (transA != 0 && transA != 1) return bad(1);
  if (transB != 0 && transB != 1) return bad(2);
  if (uplo != 0 && (uplo != 1 || m != n)) return bad(3);
  if (m < 0) return bad(4);
  if (n < 0) return bad(5);
  if (k < 0) return bad(6);
  const int64_t arows = transA ? k : m, brows = transB ? n : k;
  if (m > 0 && k > 0 && !A) return bad(8);
  if (lda < (arows > 1 ? arows : 1)) return bad(9);
  if (n > 0 && k > 0 && !B) return bad(10);
  if (ldb < (brows > 1 ? brows : 1)) return bad(11);
  if (m > 0 && n > 0 && !C) return bad(13);
  if (ldc < (m > 1 ? m : 1)) return bad(14);
  if (arith != 0 && arith != 1) return bad(15);
  return guarded([&]() -> int {
    MathScope mode(arith == 1 ? MathMode::Fp32 : MathMode::Fp64);
    Gemm g;
    g.transA = transA; g.transB = transB; g.uplo = uplo;
    g.m = m; g.n = n; g.k = k; g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
    gemm(g, (hipStream_t)stream);
    return GEP_OK;
  });
}

int gep_debug_force_wait_timeout(int on) {
  set_force_wait_timeout(on != 0);
  return GEP_OK;
}

int gep_batched_threads(int on) {
  g_batched_threads = on != 0;
  return GEP_OK;
}

int gep_debug_force_eig_failure(int on) {
  set_force_eig_failure(on != 0);
  return GEP_OK;
}

int gep_profile_enable(int on) {
  g_prof = on != 0;
  return GEP_OK;
}

int gep_probe_enable(int on) {
  probe_enable(on != 0);
  return GEP_OK;
}

int gep_probe_read(int kernel, int64_t* launches, double* ms, double* flops) {
  if (kernel < 0 || kernel >= PROBE_COUNT) return bad(1);
  return guarded([&]() -> int {
    probe_read(kernel, launches, ms, flops);
    return GEP_OK;
  });
}

const char* gep_probe_name(int kernel) {
  switch (kernel) {
    case PROBE_GEMM: return "dgemm_fast_kernel";
    case PROBE_Q2_APPLY: return "q2_apply";
    case PROBE_CHASE: return "chase";
    case PROBE_PANEL_QR: return "panel_qr_coop";
    default: return nullptr;
  }
}

double gep_profile_dc_flops(void) { return g_dc_flops ? *g_dc_flops : 0.0; }

int gep_profile_read(double* ms, int n) {
  if (!g_prof || !g_ev_recorded || !ms) return 0;
  return guarded([&]() -> int {
    GEP_HIP(hipEventSynchronize(g_ev[NPHASE]));
    int k = 0;
    for (int i = 0; i < NPHASE && i < n; ++i, ++k) {
      float t = 0.0f;
      GEP_HIP(hipEventElapsedTime(&t, g_ev[i], g_ev[i + 1]));
      ms[i] = t;
    }
    return k;
  });
}

}  // extern "C"

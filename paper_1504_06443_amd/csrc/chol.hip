// Cholesky factorisation B = L L^T and the triangular solves built on it.
//
// Recursive (blocked) formulations: every level splits the triangle in two halves
// whose sizes are multiples of NB, so almost all flops land in large MFMA GEMMs.
// The NB x NB diagonal blocks are factorised in one workgroup with the block held
// in LDS (128 x 129 doubles = 132 KB of the 160 KB per CU), and their inverses are
// formed there too; a solve against a diagonal block is then a small GEMM with
// that inverse.
#include "common.h"
#include "internal.h"

namespace gep {
namespace {

constexpr int LDS_LD = NB + 1;

// Factor the n x n (n <= NB) diagonal block in place (lower triangle; the upper
// triangle of the block is set to zero) and write its inverse (lower, NB x NB
// slot, zeros above the diagonal) to linv.  A non-positive pivot at local column
// j records info = info_add + row0 + j + 1 (first failure wins) and the pivot is
// replaced by 1 so that later steps stay finite.
//
// Right-looking: step j scales column j of L and updates the trailing lower
// triangle.  The inverse X = L^{-1} is built in the same steps by applying each
// step's elimination to the identity (row j of X divided by L(j,j), then
// X(i, 0:j) -= L(i,j) X(j, 0:j) for i > j), which is as parallel as the trailing
// update; the strictly lower part of X is kept transposed in the unused upper
// triangle of the LDS block (X(i,c) at row c, column i) and its diagonal in xd.
// LEAF_NT threads, TPC of them per column (trailing update) or row (inverse
// update), so a column step is at most two rounds of eight elements per thread.
constexpr int LEAF_NT = 1024;
constexpr int TPC = LEAF_NT / NB;

__global__ void __launch_bounds__(LEAF_NT)
potrf_trtri_leaf(int n, double* __restrict__ a, int64_t lda, double* __restrict__ linv,
                 int32_t* __restrict__ info, int64_t row0, int64_t info_add) {
  extern __shared__ double S[];  // column-major, ld LDS_LD
  double* xd = S + (size_t)NB * LDS_LD;
  const int tid = threadIdx.x;
  for (int j = tid >> 7; j < n; j += LEAF_NT / 128)
    for (int i = tid & 127; i < n; i += 128) S[i + j * LDS_LD] = (i >= j) ? a[i + j * lda] : 0.0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double piv = S[j + j * LDS_LD];
    const bool ok = piv > 0.0;  // false for NaN too
    const double ljj = ok ? sqrt(piv) : 1.0;
    if (!ok && tid == 0 && info) atomicCAS(info, 0, (int32_t)(info_add + row0 + j + 1));
    __syncthreads();
    const double rl = 1.0 / ljj;
    if (tid == 0) {
      S[j + j * LDS_LD] = ljj;
      xd[j] = rl;
    }
    for (int i = j + 1 + tid; i < n; i += LEAF_NT) S[i + j * LDS_LD] *= rl;  // L(j+1:, j)
    for (int c = tid; c < j; c += LEAF_NT) S[c + j * LDS_LD] *= rl;          // X(j, 0:j)
    __syncthreads();
    // trailing update of L's lower triangle: TPC threads per column, eight rows'
    // operands read before any of their updates is written (one LDS round trip
    // per eight elements instead of one per element)
    for (int k = j + 1 + tid / TPC; k < n; k += LEAF_NT / TPC) {
      const double lkj = S[k + j * LDS_LD];
      int i = k + tid % TPC;
      for (; i + 7 * TPC < n; i += 8 * TPC) {
        double lj[8], sk[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          lj[u] = S[i + TPC * u + j * LDS_LD];
          sk[u] = S[i + TPC * u + k * LDS_LD];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) S[i + TPC * u + k * LDS_LD] = sk[u] - lj[u] * lkj;
      }
      for (; i < n; i += TPC) S[i + k * LDS_LD] -= S[i + j * LDS_LD] * lkj;
    }
    // X(i, 0:j+1) -= L(i,j) X(j, 0:j+1) for i > j: TPC threads per row, batched
    // the same way
    for (int i = j + 1 + tid / TPC; i < n; i += LEAF_NT / TPC) {
      const double lij = S[i + j * LDS_LD];
      int c = tid % TPC;
      for (; c + 7 * TPC < j; c += 8 * TPC) {
        double xj[8], xi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          xj[u] = S[c + TPC * u + j * LDS_LD];
          xi[u] = S[c + TPC * u + i * LDS_LD];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) S[c + TPC * u + i * LDS_LD] = xi[u] - lij * xj[u];
      }
      for (; c <= j; c += TPC) {
        const double xjc = (c == j) ? rl : S[c + j * LDS_LD];
        S[c + i * LDS_LD] -= lij * xjc;
      }
    }
    __syncthreads();
  }
  for (int j = tid >> 7; j < n; j += LEAF_NT / 128)
    for (int i = tid & 127; i < n; i += 128) a[i + j * lda] = (i >= j) ? S[i + j * LDS_LD] : 0.0;
  for (int j = tid >> 7; j < NB; j += LEAF_NT / 128)
    for (int i = tid & 127; i < NB; i += 128) {
      double x = 0.0;
      if (i < n && j < n && i >= j) x = (i == j) ? xd[j] : S[j + i * LDS_LD];
      linv[i + j * NB] = x;
    }
}

int64_t split_point(int64_t n) {
  const int64_t nblk = cdiv(n, NB);
  return NB * ((nblk + 1) / 2);
}

const double* leaf_inv(const Tri& t) { return t.Linv + (t.off / NB) * (int64_t)NB * NB; }

Tri sub(const Tri& t, int64_t k) {
  Tri s = t;
  s.L = t.L + k + k * t.ld;
  s.off = t.off + k;
  return s;
}

}  // namespace

size_t potrf_leaf_lds() { return sizeof(double) * ((size_t)NB * LDS_LD + NB); }

void potrf_leaf(int64_t n, double* a, int64_t lda, double* linv_blk, int32_t* info, int64_t row0,
                int64_t info_add, hipStream_t s) {
  // set once per process (thread-safe initialisation; retried if it throws)
  static const bool attr_set = [] {
    GEP_HIP(hipFuncSetAttribute((const void*)potrf_trtri_leaf,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)potrf_leaf_lds()));
    return true;
  }();
  (void)attr_set;
  hipLaunchKernelGGL(potrf_trtri_leaf, dim3(1), dim3(LEAF_NT), potrf_leaf_lds(), s, (int)n, a, lda,
                     linv_blk, info, row0, info_add);
  GEP_LAUNCH_CHECK();
}

// X (n x ncols) <- L^{-1} X
void trsm_lln(const Tri& t, int64_t n, double* X, int64_t ldx, int64_t ncols, double* tmp,
              hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  if (n <= NB) {
    Gemm g;
    g.m = n; g.n = ncols; g.k = n;
    g.A = leaf_inv(t); g.lda = NB; g.B = X; g.ldb = ldx; g.C = tmp; g.ldc = n;
    gemm(g, s);
    copy_matrix(n, ncols, tmp, n, X, ldx, s);
    return;
  }
  const int64_t n1 = split_point(n);
  trsm_lln(t, n1, X, ldx, ncols, tmp, s);
  Gemm g;
  g.m = n - n1; g.n = ncols; g.k = n1; g.alpha = -1.0; g.beta = 1.0;
  g.A = t.L + n1; g.lda = t.ld; g.B = X; g.ldb = ldx; g.C = X + n1; g.ldc = ldx;
  gemm(g, s);
  trsm_lln(sub(t, n1), n - n1, X + n1, ldx, ncols, tmp, s);
}

// X (n x ncols) <- L^{-T} X
void trsm_llt(const Tri& t, int64_t n, double* X, int64_t ldx, int64_t ncols, double* tmp,
              hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  if (n <= NB) {
    Gemm g;
    g.transA = true;
    g.m = n; g.n = ncols; g.k = n;
    g.A = leaf_inv(t); g.lda = NB; g.B = X; g.ldb = ldx; g.C = tmp; g.ldc = n;
    gemm(g, s);
    copy_matrix(n, ncols, tmp, n, X, ldx, s);
    return;
  }
  const int64_t n1 = split_point(n);
  trsm_llt(sub(t, n1), n - n1, X + n1, ldx, ncols, tmp, s);
  Gemm g;
  g.transA = true;
  g.m = n1; g.n = ncols; g.k = n - n1; g.alpha = -1.0; g.beta = 1.0;
  g.A = t.L + n1; g.lda = t.ld; g.B = X + n1; g.ldb = ldx; g.C = X; g.ldc = ldx;
  gemm(g, s);
  trsm_llt(t, n1, X, ldx, ncols, tmp, s);
}

// X (nrows x n) <- X L^{-T}
void trsm_rlt(const Tri& t, int64_t n, double* X, int64_t ldx, int64_t nrows, double* tmp,
              hipStream_t s) {
  if (n <= 0 || nrows <= 0) return;
  if (n <= NB) {
    Gemm g;
    g.transB = true;
    g.m = nrows; g.n = n; g.k = n;
    g.A = X; g.lda = ldx; g.B = leaf_inv(t); g.ldb = NB; g.C = tmp; g.ldc = nrows;
    gemm(g, s);
    copy_matrix(nrows, n, tmp, nrows, X, ldx, s);
    return;
  }
  const int64_t n1 = split_point(n);
  trsm_rlt(t, n1, X, ldx, nrows, tmp, s);
  Gemm g;
  g.transB = true;
  g.m = nrows; g.n = n - n1; g.k = n1; g.alpha = -1.0; g.beta = 1.0;
  g.A = X; g.lda = ldx; g.B = t.L + n1; g.ldb = t.ld; g.C = X + n1 * ldx; g.ldc = ldx;
  gemm(g, s);
  trsm_rlt(sub(t, n1), n - n1, X + n1 * ldx, ldx, nrows, tmp, s);
}

// In place: lower triangle of a (n x n) -> L, Linv blocks written at linv + (off/NB)*NB*NB.
void potrf_rec(double* a, int64_t lda, int64_t n, int64_t off, double* linv, int32_t* info,
               int64_t info_add, double* tmp, hipStream_t s) {
  if (n <= 0) return;
  if (n <= NB) {
    potrf_leaf(n, a, lda, linv + (off / NB) * (int64_t)NB * NB, info, off, info_add, s);
    return;
  }
  const int64_t n1 = split_point(n);
  potrf_rec(a, lda, n1, off, linv, info, info_add, tmp, s);
  Tri t{a, lda, linv, off};
  trsm_rlt(t, n1, a + n1, lda, n - n1, tmp, s);
  Gemm g;
  g.transB = true;
  g.uplo = 1;
  g.m = n - n1; g.n = n - n1; g.k = n1; g.alpha = -1.0; g.beta = 1.0;
  g.A = a + n1; g.lda = lda; g.B = a + n1; g.ldb = lda; g.C = a + n1 + n1 * lda; g.ldc = lda;
  gemm(g, s);
  potrf_rec(a + n1 + n1 * lda, lda, n - n1, off + n1, linv, info, info_add, tmp, s);
}

// Lower triangle of X (n x n) <- lower triangle of X L^{-T}.  Only the lower
// triangle of the result is formed; it reads only the lower triangle of X.
void trsm_rlt_lower(const Tri& t, int64_t n, double* X, int64_t ldx, double* tmp, hipStream_t s) {
  if (n <= 0) return;
  if (n <= NB) {
    trsm_rlt(t, n, X, ldx, n, tmp, s);
    return;
  }
  const int64_t n1 = split_point(n);
  trsm_rlt_lower(t, n1, X, ldx, tmp, s);
  trsm_rlt(t, n1, X + n1, ldx, n - n1, tmp, s);
  Gemm g;
  g.transB = true;
  g.uplo = 1;
  g.m = n - n1; g.n = n - n1; g.k = n1; g.alpha = -1.0; g.beta = 1.0;
  g.A = X + n1; g.lda = ldx; g.B = t.L + n1; g.ldb = t.ld; g.C = X + n1 + n1 * ldx; g.ldc = ldx;
  gemm(g, s);
  trsm_rlt_lower(sub(t, n1), n - n1, X + n1 + n1 * ldx, ldx, tmp, s);
}

}  // namespace gep

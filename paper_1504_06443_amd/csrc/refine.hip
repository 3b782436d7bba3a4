// FP64 eigenpair refinement for the mixed-precision path (one pass).
//
// Input: approximate eigenvectors Yh of the pencil (A, B) (B-orthonormal to about
// FP32 accuracy, ordered by approximate eigenvalue).  In the basis Yh the pencil
// becomes (S, T) = (Yh^T A Yh, Yh^T B Yh), computed in FP64; its exact
// eigenpairs give those of (A, B).  S and T are diagonal up to FP32-sized
// off-diagonal entries, and an off-diagonal entry couples two eigenvectors
// strongly only when their eigenvalues are close.  So:
//  1. the indices are cut into blocks of consecutive eigenvalues, at the largest
//     gap in each window of admissible block ends;
//  2. each block's pencil (S_II, T_II) is solved exactly in FP64 (Cholesky of
//     T_II, cyclic Jacobi on L^-1 S_II L^-T), giving K = blockdiag(W_I) and the
//     rotated pencil (S', T') = (K^T S K, K^T T K);
//  3. couplings between blocks are removed by first-order Rayleigh-Schroedinger
//     perturbation: for i, j in different blocks
//        c_ji = -(s'_ji - d_i t'_ji) / (t'_jj (d_j - d_i)),   d_i = s'_ii / t'_ii,
//     the eigenvalue gets the second-order term
//        lambda_i = d_i - sum_j (s'_ji - d_i t'_ji)^2 / (t'_ii t'_jj (d_j - d_i)),
//     and Y = Yh K (I + E) with E_ji = c_ji across blocks, -t'_ji / 2 inside a
//     block and 1 / sqrt(t'_ii) - 1 on the diagonal (first-order B-normalisation).
// The eigenvalues are then accurate to second order in the cross-block coupling
// and the eigenvectors to first order.  Cost: four FP64 GEMMs of 6 M^3 flops in
// total (A Yh, B Yh and the lower halves of S and T), O(M^2 b) for the block
// transforms, and one 2 M^3 update Yh K E that runs in FP32 arithmetic (E is
// small, so its rounding enters the vectors at FP32 precision times |E|).
#include "common.h"
#include "internal.h"

namespace gep {
namespace {

constexpr int NT = 256;
constexpr int RB_MIN = 32;   // block sizes: [RB_MIN, RB_MAX] except the last block
constexpr int RB_MAX = 64;
constexpr int JLD = RB_MAX + 1;

// d_i = s_ii / t_ii; t_i = t_ii
__global__ void diag_ratio(int64_t M, const double* __restrict__ S, const double* __restrict__ T,
                           int64_t ld, double* __restrict__ d, double* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const double tii = T[i + i * ld];
  d[i] = S[i + i * ld] / tii;
  t[i] = tii;
}

// Block boundaries: from the current start s, the next start is the k in
// [s + RB_MIN, s + RB_MAX] with the largest gap d_k - d_{k-1} (first one on ties),
// until at most RB_MAX indices remain.  One wave walks the blocks in order; then
// every index gets its block number.
__global__ void __launch_bounds__(NT) partition_blocks(int64_t M, const double* __restrict__ d,
                                                       int32_t* __restrict__ starts,
                                                       int32_t* __restrict__ nblk,
                                                       int32_t* __restrict__ blk) {
  __shared__ int32_t nb_sh;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < 64) {
    int64_t s = 0;
    int32_t nb = 0;
    while (M - s > RB_MAX) {
      const int64_t lo = s + RB_MIN;
      const int64_t hi = (s + RB_MAX) < (M - 1) ? (s + RB_MAX) : (M - 1);
      const int64_t k = lo + lane;
      // every lane holds a valid candidate (lanes past hi stand for lo with gap
      // -inf, a NaN gap counts as -inf), so all lanes agree on the maximum and
      // the next start always advances by at least RB_MIN
      double g = -INFINITY;
      if (k <= hi) g = d[k] - d[k - 1];
      if (!(g >= -INFINITY)) g = -INFINITY;
      int64_t best = k <= hi ? k : lo;
      for (int off = 32; off >= 1; off >>= 1) {
        const double g2 = __shfl_xor(g, off, 64);
        const int64_t b2 = __shfl_xor(best, off, 64);
        if (g2 > g || (g2 == g && b2 < best)) {
          g = g2;
          best = b2;
        }
      }
      if (lane == 0) starts[nb] = (int32_t)s;
      ++nb;
      s = best;
    }
    if (lane == 0) {
      starts[nb] = (int32_t)s;
      starts[nb + 1] = (int32_t)M;
      nb_sh = nb + 1;
      *nblk = nb + 1;
    }
  }
  __syncthreads();
  const int32_t nb = nb_sh;
  for (int64_t i = threadIdx.x; i < M; i += NT) {
    int32_t lo = 0, hi = nb - 1;  // last block whose start <= i
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (starts[mid] <= i) lo = mid; else hi = mid - 1;
    }
    blk[i] = lo;
  }
}

// Exact FP64 solution of one block's pencil (S_II, T_II), n <= RB_MAX, in LDS:
// T = L L^T, C = L^-1 S L^-T, cyclic Jacobi (round-robin pairs, all disjoint
// rotations of a round applied together), W = L^-T Z, eigenpairs sorted
// ascending.  Writes W into K (rows s0.., columns 0..n-1, leading dimension ldk).
__global__ void __launch_bounds__(NT) block_eig([[maybe_unused]] int64_t M,
                                                const double* __restrict__ S,
                                                const double* __restrict__ T, int64_t ld,
                                                const int32_t* __restrict__ starts,
                                                const int32_t* __restrict__ nblk,
                                                double* __restrict__ K, int64_t ldk,
                                                int32_t* __restrict__ err) {
  const int b = blockIdx.x;
  if (b >= *nblk) return;
  const int64_t s0 = starts[b];
  const int n = (int)(starts[b + 1] - s0);
  __shared__ double C[RB_MAX * JLD];
  __shared__ double L[RB_MAX * JLD];
  __shared__ double Z[RB_MAX * JLD];
  __shared__ double rc[RB_MAX / 2], rs[RB_MAX / 2];
  __shared__ int rp[RB_MAX / 2], rq[RB_MAX / 2];
  __shared__ int rotated;
  __shared__ double fro;
  const int tid = threadIdx.x;
  // [r * JLD + c] holds row r, column c
  for (int idx = tid; idx < n * n; idx += NT) {
    const int r = idx % n, c = idx / n;
    C[r * JLD + c] = S[(s0 + r) + (s0 + c) * ld];
    L[r * JLD + c] = T[(s0 + r) + (s0 + c) * ld];
  }
  __syncthreads();
  // Cholesky (lower) of T, right-looking
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      const double p = L[k * JLD + k];
      if (!(p > 0.0)) atomicExch(err, 1);
      L[k * JLD + k] = sqrt(p > 0.0 ? p : 1.0);
    }
    __syncthreads();
    const double lkk = L[k * JLD + k];
    for (int i = k + 1 + tid; i < n; i += NT) L[i * JLD + k] /= lkk;
    __syncthreads();
    const int m = n - k - 1;
    for (int idx = tid; idx < m * m; idx += NT) {
      const int i = k + 1 + idx % m, j = k + 1 + idx / m;
      if (i >= j) L[i * JLD + j] -= L[i * JLD + k] * L[j * JLD + k];
    }
    __syncthreads();
  }
  // Z = L^-1 S (column c solved by thread c), then C = L^-1 Z^T
  for (int c = tid; c < n; c += NT)
    for (int r = 0; r < n; ++r) {
      double v = C[r * JLD + c];
      for (int q = 0; q < r; ++q) v -= L[r * JLD + q] * Z[q * JLD + c];
      Z[r * JLD + c] = v / L[r * JLD + r];
    }
  __syncthreads();
  for (int c = tid; c < n; c += NT)
    for (int r = 0; r < n; ++r) {
      double v = Z[c * JLD + r];  // (Z^T)[r][c]
      for (int q = 0; q < r; ++q) v -= L[r * JLD + q] * C[q * JLD + c];
      C[r * JLD + c] = v / L[r * JLD + r];
    }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += NT) {
    const int r = idx % n, c = idx / n;
    if (r > c) {
      const double v = 0.5 * (C[r * JLD + c] + C[c * JLD + r]);
      C[r * JLD + c] = v;
      C[c * JLD + r] = v;
    }
    Z[r * JLD + c] = (r == c) ? 1.0 : 0.0;
  }
  if (tid == 0) fro = 0.0;
  __syncthreads();
  if (tid < 64) {
    double f = 0.0;
    for (int idx = tid; idx < n * n; idx += 64) {
      const double v = C[(idx % n) * JLD + idx / n];
      f += v * v;
    }
    for (int off = 32; off >= 1; off >>= 1) f += __shfl_xor(f, off, 64);
    if (tid == 0) fro = sqrt(f);
  }
  __syncthreads();
  const double tol = 1e-16 * fro;
  // round-robin over np (even) slots; slot n (odd n) is a dummy
  const int np = n + (n & 1);
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      // pair t: slots (a, b) of the circle method with slot np - 1 fixed
      if (tid < np / 2) {
        int a, bb;
        if (tid == 0) {
          a = np - 1;
          bb = round;
        } else {
          a = (round + tid) % (np - 1);
          bb = (round - tid + (np - 1)) % (np - 1);
        }
        const int p = a < bb ? a : bb, q = a < bb ? bb : a;
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = C[p * JLD + q];
          if (fabs(apq) > tol) {
            const double app = C[p * JLD + p], aqq = C[q * JLD + q];
            const double theta = (aqq - app) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            rotated = 1;
          }
        }
        rp[tid] = p;
        rq[tid] = q < n ? q : p;
        rc[tid] = c;
        rs[tid] = (q < n) ? s : 0.0;
      }
      __syncthreads();
      // rows p, q of C (all pairs at once, disjoint rows)
      const int half = np / 2;
      for (int idx = tid; idx < half * n; idx += NT) {
        const int t = idx % half, k = idx / half;
        const double s = rs[t];
        if (s == 0.0) continue;
        const int p = rp[t], q = rq[t];
        const double c = rc[t];
        const double xp = C[p * JLD + k], xq = C[q * JLD + k];
        C[p * JLD + k] = c * xp - s * xq;
        C[q * JLD + k] = s * xp + c * xq;
      }
      __syncthreads();
      // columns p, q of C and of Z
      for (int idx = tid; idx < half * n; idx += NT) {
        const int t = idx % half, k = idx / half;
        const double s = rs[t];
        if (s == 0.0) continue;
        const int p = rp[t], q = rq[t];
        const double c = rc[t];
        const double xp = C[k * JLD + p], xq = C[k * JLD + q];
        C[k * JLD + p] = c * xp - s * xq;
        C[k * JLD + q] = s * xp + c * xq;
        const double zp = Z[k * JLD + p], zq = Z[k * JLD + q];
        Z[k * JLD + p] = c * zp - s * zq;
        Z[k * JLD + q] = s * zp + c * zq;
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // W = L^-T Z (column c by thread c), kept in Z
  for (int c = tid; c < n; c += NT)
    for (int r = n - 1; r >= 0; --r) {
      double v = Z[r * JLD + c];
      for (int q = r + 1; q < n; ++q) v -= L[q * JLD + r] * Z[q * JLD + c];
      Z[r * JLD + c] = v / L[r * JLD + r];
    }
  __syncthreads();
  // ascending order of the eigenvalues diag(C): rank by counting
  for (int c = tid; c < n; c += NT) {
    const double lc = C[c * JLD + c];
    int rank = 0;
    for (int q = 0; q < n; ++q) {
      const double lq = C[q * JLD + q];
      rank += (lq < lc) || (lq == lc && q < c);
    }
    for (int r = 0; r < n; ++r) K[(s0 + r) + (int64_t)rank * ldk] = Z[r * JLD + c];
  }
}

// Grouped-GEMM problems for the block-diagonal products.
//  mode 0: X[:, I] = S[:, I] W_I        (M x n, k = n)
//  mode 1: S'[I, :] = W_I^T X[I, :]     (n x M, k = n)
//  mode 2: Y'[:, I] = Yh[:, I] W_I      (M x n, k = n)
__global__ void block_descs(int64_t M, int mode, const int32_t* __restrict__ starts,
                            const int32_t* __restrict__ nblk, int maxblk, const double* K,
                            int64_t ldk, const double* X, int64_t ldx, double* Out, int64_t ldo,
                            GemmDesc* __restrict__ desc) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= maxblk) return;
  GemmDesc g;
  g.alpha = 1.0; g.beta = 0.0; g.transA = 0; g.transB = 0;
  if (b >= *nblk) {
    g.m = g.n = g.k = 0;
    g.A = g.B = nullptr; g.C = nullptr; g.lda = g.ldb = g.ldc = 1;
    desc[b] = g;
    return;
  }
  const int64_t s0 = starts[b], n = starts[b + 1] - s0;
  const double* W = K + s0;  // n x n at rows s0.., columns 0..n-1
  if (mode == 1) {
    g.m = n; g.n = M; g.k = n;
    g.A = W; g.lda = ldk; g.transA = 1;
    g.B = X + s0; g.ldb = ldx;
    g.C = Out + s0; g.ldc = ldo;
  } else {
    g.m = M; g.n = n; g.k = n;
    g.A = X + s0 * ldx; g.lda = ldx;
    g.B = W; g.ldb = ldk;
    g.C = Out + s0 * ldo; g.ldc = ldo;
  }
  desc[b] = g;
}

// Column i of E and the refined eigenvalue lambda_i (one workgroup per column).
__global__ void __launch_bounds__(NT) cross_correct(int64_t M, const double* __restrict__ Sp,
                                                    const double* __restrict__ Tp, int64_t ld,
                                                    const double* __restrict__ d,
                                                    const double* __restrict__ t,
                                                    const int32_t* __restrict__ blk,
                                                    double* __restrict__ E, int64_t lde,
                                                    double* __restrict__ lam,
                                                    double* __restrict__ coupling) {
  const int64_t i = blockIdx.x;
  const double di = d[i], ti = t[i];
  const int32_t bi = blk[i];
  double corr = 0.0, cmax = 0.0;
  for (int64_t j = threadIdx.x; j < M; j += NT) {
    const double sji = Sp[j + i * ld], tji = Tp[j + i * ld];
    double e;
    if (j == i) {
      e = 1.0 / sqrt(ti) - 1.0;
    } else if (blk[j] == bi) {
      e = -0.5 * tji;
    } else {
      const double gap = d[j] - di;
      const double r = sji - di * tji;
      // exactly (or to rounding) degenerate pair: any rotation inside the
      // eigenspace is exact, keep only the B-normalisation
      if (fabs(gap) <= 64.0 * 2.220446049250313e-16 * (fabs(di) + fabs(d[j]))) {
        e = -0.5 * tji;
      } else {
        const double den = t[j] * gap;
        e = -r / den;
        corr += r * r / (ti * den);
        cmax = fmax(cmax, fabs(e));
      }
    }
    E[j + i * lde] = e;
  }
  __shared__ double red[NT / 64], redm[NT / 64];
  for (int off = 32; off >= 1; off >>= 1) {
    corr += __shfl_xor(corr, off, 64);
    cmax = fmax(cmax, __shfl_xor(cmax, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = corr;
    redm[threadIdx.x >> 6] = cmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double c = 0.0, m = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      c += red[w];
      m = fmax(m, redm[w]);
    }
    lam[i] = di - c;
    // coupling >= 0, so the bit pattern orders like the value
    atomicMax(reinterpret_cast<unsigned long long*>(coupling),
              (unsigned long long)__double_as_longlong(m));
  }
}

// rank_i = #{j : lam_j < lam_i or (lam_j == lam_i and j < i)}
__global__ void __launch_bounds__(NT) rank_values(int64_t M, const double* __restrict__ lam,
                                                  int32_t* __restrict__ rank) {
  __shared__ double tile[NT];
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  const double li = i < M ? lam[i] : 0.0;
  int64_t r = 0;
  for (int64_t j0 = 0; j0 < M; j0 += NT) {
    __syncthreads();
    if (j0 + threadIdx.x < M) tile[threadIdx.x] = lam[j0 + threadIdx.x];
    __syncthreads();
    const int cnt = (M - j0) < NT ? (int)(M - j0) : NT;
    for (int q = 0; q < cnt; ++q) {
      const double lq = tile[q];
      r += (lq < li) || (lq == li && j0 + q < i);
    }
  }
  if (i < M) rank[i] = (int32_t)r;
}

// Y[:, rank_i] = X[:, i], lambda[rank_i] = lam_i
__global__ void scatter_columns(int64_t M, const int32_t* __restrict__ rank,
                                const double* __restrict__ lam, const double* __restrict__ X,
                                int64_t ldx, double* __restrict__ lambda, double* __restrict__ Y,
                                int64_t ldy) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = blockIdx.y; i < M; i += gridDim.y) {
    const int64_t dst = rank[i];
    if (r < M) Y[r + dst * ldy] = X[r + i * ldx];
    if (r == 0) lambda[dst] = lam[i];
  }
}

struct RefineBufs {
  double *W3, *W4, *K, *d, *t, *lam, *coupling;
  int32_t *starts, *nblk, *blk, *rank, *err;
  GemmDesc* desc;
  int maxblk;
};

RefineBufs carve_refine(int64_t M, Arena& a) {
  RefineBufs r;
  r.maxblk = (int)cdiv(M, RB_MIN) + 1;
  r.W3 = a.take<double>((size_t)M * M);
  r.W4 = a.take<double>((size_t)M * M);
  r.K = a.take<double>((size_t)M * RB_MAX);
  r.d = a.take<double>(M);
  r.t = a.take<double>(M);
  r.lam = a.take<double>(M);
  r.coupling = a.take<double>(1);
  r.starts = a.take<int32_t>(r.maxblk + 2);
  r.nblk = a.take<int32_t>(1);
  r.blk = a.take<int32_t>(M);
  r.rank = a.take<int32_t>(M);
  r.err = a.take<int32_t>(1);
  r.desc = a.take<GemmDesc>(r.maxblk);
  return r;
}

void block_product(int64_t M, int mode, const RefineBufs& r, const double* X, int64_t ldx,
                   double* Out, int64_t ldo, hipStream_t s) {
  hipLaunchKernelGGL(block_descs, dim3((unsigned)cdiv(r.maxblk, 256)), dim3(256), 0, s, M, mode,
                     (const int32_t*)r.starts, (const int32_t*)r.nblk, r.maxblk,
                     (const double*)r.K, M, X, ldx, Out, ldo, r.desc);
  GEP_LAUNCH_CHECK();
  if (mode == 1)
    gemm_grouped(r.desc, r.maxblk, RB_MAX, M, s);
  else
    gemm_grouped(r.desc, r.maxblk, M, RB_MAX, s);
}

}  // namespace

size_t refine_workspace(int64_t M) {
  Arena a;
  a.dry = true;
  carve_refine(M, a);
  return a.used + 256;
}

void refine(int64_t M, const double* A, int64_t lda, const double* B, int64_t ldb, double* Y,
            int64_t ldy, double* lambda, double* W1, double* W2, Arena& ws, double* coupling_out,
            int32_t* info, hipStream_t s) {
  if (M <= 0) return;
  MathScope fp64(MathMode::Fp64);
  RefineBufs r = carve_refine(M, ws);
  double* S = r.W3;
  double* T = r.W4;
  fill_i32(r.err, 1, 0, s);
  fill_f64(r.coupling, 1, 0.0, s);
  {  // S = Yh^T (A Yh), T = Yh^T (B Yh): lower triangles, then mirrored.  A and B
     // are expanded to full storage in W2 first, so the products run as plain
     // GEMMs on the interior tile kernel.
    Gemm g;
    g.m = M; g.n = M; g.k = M;
    g.A = W2; g.lda = M; g.B = Y; g.ldb = ldy; g.C = W1; g.ldc = M;
    Gemm h;
    h.transA = true;
    h.uplo = 1;
    h.m = M; h.n = M; h.k = M;
    h.A = Y; h.lda = ldy; h.B = W1; h.ldb = M; h.C = S; h.ldc = M;
    symmetrize_from_lower(M, A, lda, W2, M, s);
    gemm(g, s);
    gemm(h, s);
    symmetrize_from_lower(M, B, ldb, W2, M, s);
    gemm(g, s);
    h.C = T;
    gemm(h, s);
  }
  symmetrize_from_lower(M, S, M, S, M, s);
  symmetrize_from_lower(M, T, M, T, M, s);
  hipLaunchKernelGGL(diag_ratio, dim3((unsigned)cdiv(M, 256)), dim3(256), 0, s, M,
                     (const double*)S, (const double*)T, M, r.d, r.t);
  GEP_LAUNCH_CHECK();
  hipLaunchKernelGGL(partition_blocks, dim3(1), dim3(NT), 0, s, M, (const double*)r.d, r.starts,
                     r.nblk, r.blk);
  GEP_LAUNCH_CHECK();
  hipLaunchKernelGGL(block_eig, dim3((unsigned)r.maxblk), dim3(NT), 0, s, M, (const double*)S,
                     (const double*)T, M, (const int32_t*)r.starts, (const int32_t*)r.nblk, r.K,
                     M, r.err);
  GEP_LAUNCH_CHECK();
  raise_info_if(r.err, info, INFO_REFINE_FAILED, s);
  // S' = K^T (S K) into W2, T' = K^T (T K) into S's buffer
  block_product(M, 0, r, S, M, W1, M, s);
  block_product(M, 1, r, W1, M, W2, M, s);
  block_product(M, 0, r, T, M, W1, M, s);
  block_product(M, 1, r, W1, M, S, M, s);
  double* Sp = W2;
  double* Tp = S;
  hipLaunchKernelGGL(diag_ratio, dim3((unsigned)cdiv(M, 256)), dim3(256), 0, s, M,
                     (const double*)Sp, (const double*)Tp, M, r.d, r.t);
  GEP_LAUNCH_CHECK();
  // E into T's buffer, refined eigenvalues into r.lam
  hipLaunchKernelGGL(cross_correct, dim3((unsigned)M), dim3(NT), 0, s, M, (const double*)Sp,
                     (const double*)Tp, M, (const double*)r.d, (const double*)r.t,
                     (const int32_t*)r.blk, T, M, r.lam, r.coupling);
  GEP_LAUNCH_CHECK();
  double* E = T;
  // Y' = Yh K into W1; X = Y' + Y' E into W2 (the update product in FP32 arithmetic)
  block_product(M, 2, r, Y, ldy, W1, M, s);
  copy_matrix(M, M, W1, M, W2, M, s);
  {
    MathScope fp32(MathMode::Fp32);
    Gemm g;
    g.m = M; g.n = M; g.k = M;
    g.A = W1; g.lda = M; g.B = E; g.ldb = M; g.beta = 1.0; g.C = W2; g.ldc = M;
    gemm(g, s);
  }
  hipLaunchKernelGGL(rank_values, dim3((unsigned)cdiv(M, NT)), dim3(NT), 0, s, M,
                     (const double*)r.lam, r.rank);
  GEP_LAUNCH_CHECK();
  hipLaunchKernelGGL(scatter_columns, dim3((unsigned)cdiv(M, 256), (unsigned)(M < 65535 ? M : 65535)),
                     dim3(256), 0, s,
                     M, (const int32_t*)r.rank, (const double*)r.lam, (const double*)W2, M, lambda,
                     Y, ldy);
  GEP_LAUNCH_CHECK();
  if (coupling_out) GEP_HIP(hipMemcpyAsync(coupling_out, r.coupling, sizeof(double),
                                           hipMemcpyDeviceToDevice, s));
}

}  // namespace gep

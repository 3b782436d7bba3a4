// Parallel two-sided block Jacobi eigensolver for a dense symmetric matrix: the
// SEP solver of a different mathematical foundation that the paper's outlook
// (section 6) proposes to combine with its reducer, which makes it usable for the
// generalized problem.  It diagonalises C directly, with no band or tridiagonal
// form in between.
//
// C (n x n, full symmetric storage) is cut into nblk blocks of nb rows (the last
// one ragged; an odd count gets an empty block so the count is even).  A sweep
// visits every pair of blocks once, in 2K - 1 rounds of K = nblk / 2 disjoint
// pairs (the round-robin "circle" ordering).  For a pair (p, q) the symmetric
// matrix [C_pp C_pq; C_qp C_qq] (order <= 2 nb <= 64) is diagonalised exactly by
// cyclic Jacobi in LDS, J^T C_PP J = diag; then all pairs of the round are
// applied at once (they touch disjoint rows and columns):
//   C(P, :) <- J^T C(P, :),   C(:, P) <- C(:, P) J,   V(:, P) <- V(:, P) J.
// The off-diagonal norm is measured after every sweep (one reduction and a read
// back to the host) and the sweeps stop once it is at rounding level; the
// diagonal of C then holds the eigenvalues and V the eigenvectors.  Cost: about
// 12 n^3 flops per sweep in the updates (on the matrix cores) plus the pair
// solves; Jacobi converges quadratically, typically in 6-10 sweeps.
#include <cmath>
#include <vector>

#include "common.h"
#include "internal.h"

namespace gep {
namespace {

constexpr int NT = 256;
constexpr int JB = 32;          // block rows
constexpr int PN = 2 * JB;      // order of a pair matrix
constexpr int PLD = PN + 1;     // LDS row stride of a pair matrix
constexpr int MAX_SWEEPS = 30;

struct Layout {
  int64_t n;
  int nb;        // rows per block
  int nblk;      // blocks, even (the last may be empty)
};

__host__ __device__ inline int64_t blk_lo(const Layout& L, int b) {
  const int64_t lo = (int64_t)b * L.nb;
  return lo < L.n ? lo : L.n;
}
__host__ __device__ inline int blk_len(const Layout& L, int b) {
  const int64_t hi = (int64_t)(b + 1) * L.nb;
  return (int)((hi < L.n ? hi : L.n) - blk_lo(L, b));
}

// Pair t of round r in the circle ordering of nblk (even) blocks: block nblk - 1
// stays fixed, the others rotate.
__device__ inline void pair_of(int nblk, int r, int t, int& p, int& q) {
  const int m = nblk - 1;
  int a, b;
  if (t == 0) {
    a = m;
    b = r;
  } else {
    a = (r + t) % m;
    b = (r - t + m) % m;
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// Local row k (0 .. np + nq - 1) of pair (p, q) -> global row.
__device__ inline int64_t pair_row(const Layout& L, int p, int q, int k) {
  const int np = blk_len(L, p);
  return k < np ? blk_lo(L, p) + k : blk_lo(L, q) + (k - np);
}

// One workgroup per pair of the round: J (PN x PN, column-major with leading
// dimension PN, zero beyond the pair's order) with J^T C_PP J diagonal.  Cyclic
// Jacobi with the circle ordering inside the pair; a rotation is skipped when
// its off-diagonal entry is at most `tol` (absolute, from the whole matrix's
// norm), so nearly diagonal pair matrices cost one pass.
__global__ void __launch_bounds__(NT) pair_eig(Layout L, const double* __restrict__ C,
                                               int64_t ldc, int round, double tol,
                                               double* __restrict__ J) {
  __shared__ double A[PN * PLD];
  __shared__ double Z[PN * PLD];
  __shared__ double rc[PN / 2], rs[PN / 2];
  __shared__ int rp[PN / 2], rq[PN / 2];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  int p, q;
  pair_of(L.nblk, round, blockIdx.x, p, q);
  const int n = blk_len(L, p) + blk_len(L, q);
  double* Jout = J + (int64_t)blockIdx.x * PN * PN;
  for (int idx = tid; idx < PN * PN; idx += NT) {
    const int r = idx % PN, c = idx / PN;
    double v = 0.0;
    if (r < n && c < n) v = C[pair_row(L, p, q, r) + pair_row(L, p, q, c) * ldc];
    A[r * PLD + c] = v;
    Z[r * PLD + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int np2 = n + (n & 1);  // slots of the inner circle ordering
  for (int sweep = 0; sweep < 16 && np2 >= 2; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < np2 - 1; ++r) {
      if (tid < np2 / 2) {
        int a, b;
        const int m = np2 - 1;
        if (tid == 0) {
          a = m;
          b = r;
        } else {
          a = (r + tid) % m;
          b = (r - tid + m) % m;
        }
        const int i = a < b ? a : b, j = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (j < n) {
          const double aij = A[i * PLD + j];
          if (fabs(aij) > tol) {
            const double aii = A[i * PLD + i], ajj = A[j * PLD + j];
            const double theta = (ajj - aii) / (2.0 * aij);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            rotated = 1;
          }
        }
        rp[tid] = i;
        rq[tid] = j < n ? j : i;
        rc[tid] = c;
        rs[tid] = j < n ? s : 0.0;
      }
      __syncthreads();
      const int half = np2 / 2;
      // rows i, j of A for every rotation of the round (disjoint rows)
      for (int idx = tid; idx < half * n; idx += NT) {
        const int t = idx % half, k = idx / half;
        const double s = rs[t];
        if (s == 0.0) continue;
        const int i = rp[t], j = rq[t];
        const double c = rc[t];
        const double xi = A[i * PLD + k], xj = A[j * PLD + k];
        A[i * PLD + k] = c * xi - s * xj;
        A[j * PLD + k] = s * xi + c * xj;
      }
      __syncthreads();
      // columns i, j of A and of Z
      for (int idx = tid; idx < half * n; idx += NT) {
        const int t = idx % half, k = idx / half;
        const double s = rs[t];
        if (s == 0.0) continue;
        const int i = rp[t], j = rq[t];
        const double c = rc[t];
        const double xi = A[k * PLD + i], xj = A[k * PLD + j];
        A[k * PLD + i] = c * xi - s * xj;
        A[k * PLD + j] = s * xi + c * xj;
        const double zi = Z[k * PLD + i], zj = Z[k * PLD + j];
        Z[k * PLD + i] = c * zi - s * zj;
        Z[k * PLD + j] = s * zi + c * zj;
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // Z is a product of up to a thousand plane rotations, orthogonal only to a
  // few tens of ulps; the sweeps apply it to every column of C and V once per
  // round, so that departure accumulates in the eigenvectors.  One
  // Newton-Schulz step towards Z's orthogonal polar factor,
  // J = Z (3 I - Z^T Z) / 2, squares it (rounding of two 64-term products
  // aside).  A is free by now and holds 3 I - Z^T Z.
  __syncthreads();
  for (int idx = tid; idx < PN * PN; idx += NT) {
    const int r = idx % PN, c = idx / PN;
    double g = 0.0;
    for (int k = 0; k < PN; ++k) g = fma(Z[k * PLD + r], Z[k * PLD + c], g);
    A[c * PLD + r] = (r == c ? 3.0 : 0.0) - g;
  }
  __syncthreads();
  for (int idx = tid; idx < PN * PN; idx += NT) {
    const int r = idx % PN, c = idx / PN;
    double v = 0.0;
    for (int k = 0; k < PN; ++k) v = fma(Z[r * PLD + k], A[c * PLD + k], v);
    Jout[r + c * PN] = 0.5 * v;
  }
}

// The update of one 64 x 64 tile on the matrix cores: rows = false:
// X(P, cols) <- J^T X(P, cols) for the 64 columns starting at blockIdx.x * 64;
// rows = true is the column update X(rows, P) <- X(rows, P) J for 64 rows.  One
// workgroup per (tile, pair of the round); each wave computes 16 output rows.
template <bool COLS>
__global__ void __launch_bounds__(NT) pair_apply(Layout L, double* __restrict__ X, int64_t ldx,
                                                 int64_t nother, int round,
                                                 const double* __restrict__ J) {
  __shared__ double T[PN * PLD];   // the tile: [local k][64 other] (rows) or [64 other][local k]
  __shared__ double Js[PN * PLD];  // J[k][j]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l15 = lane & 15, l4 = lane >> 4;
  int p, q;
  pair_of(L.nblk, round, blockIdx.y, p, q);
  const int n = blk_len(L, p) + blk_len(L, q);
  const int64_t o0 = (int64_t)blockIdx.x * 64;  // first row (COLS) or column (rows pass)
  const double* Jg = J + (int64_t)blockIdx.y * PN * PN;
  for (int idx = tid; idx < PN * PN; idx += NT) {
    const int k = idx % PN, j = idx / PN;
    Js[k * PLD + j] = Jg[k + j * PN];
  }
  if (!COLS) {
    // T[k][c] = X(P_k, o0 + c); column-major X: consecutive threads walk c? rows of
    // P are scattered, so threads walk k (contiguous within a block) for coalescing
    for (int idx = tid; idx < PN * 64; idx += NT) {
      const int k = idx % PN, c = idx / PN;
      const int64_t col = o0 + c;
      T[k * PLD + c] = (k < n && col < nother) ? X[pair_row(L, p, q, k) + col * ldx] : 0.0;
    }
  } else {
    // T[r][k] = X(o0 + r, P_k): threads walk r (contiguous rows of a column)
    for (int idx = tid; idx < PN * 64; idx += NT) {
      const int r = idx % 64, k = idx / 64;
      const int64_t row = o0 + r;
      T[r * PLD + k] = (k < n && row < nother) ? X[row + pair_row(L, p, q, k) * ldx] : 0.0;
    }
  }
  __syncthreads();
  v4d acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
  // output D[m][cc] (m: this wave's 16 rows), 4 tiles of 16 columns
#pragma unroll 4
  for (int s = 0; s < PN / 4; ++s) {
    const int k = 4 * s + l4;
    double a;
    if (!COLS)
      a = Js[k * PLD + 16 * wave + l15];          // (J^T)[m][k] = J[k][m]
    else
      a = T[(16 * wave + l15) * PLD + k];         // T[m][k]
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      double b;
      if (!COLS)
        b = T[k * PLD + 16 * t + l15];            // T[k][cc]
      else
        b = Js[k * PLD + 16 * t + l15];           // J[k][cc]
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
  // element r of acc[t]: D[16 wave + l4 + 4 r][16 t + l15]
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * wave + l4 + 4 * r, cc = 16 * t + l15;
      if (!COLS) {
        const int64_t col = o0 + cc;
        if (m < n && col < nother) X[pair_row(L, p, q, m) + col * ldx] = acc[t][r];
      } else {
        const int64_t row = o0 + m;
        if (cc < n && row < nother) X[row + pair_row(L, p, q, cc) * ldx] = acc[t][r];
      }
    }
}

// sums[0] += squares of the off-diagonal entries, sums[1] += squares of the
// diagonal (summed apart: their difference from |C|_F^2 would cancel)
__global__ void __launch_bounds__(NT) frob_parts(int64_t n, const double* __restrict__ C,
                                                 int64_t ldc, double* sums) {
  __shared__ double red[2][NT / 64];
  const int64_t j = blockIdx.x;
  double a = 0.0, d = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    const double v = C[i + j * ldc];
    if (i == j)
      d += v * v;
    else
      a += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    d += __shfl_xor(d, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = d;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sd = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      sa += red[0][w];
      sd += red[1][w];
    }
    atomicAdd(&sums[0], sa);
    atomicAdd(&sums[1], sd);
  }
}

// Eigenvalues from the diagonal in ascending order (rank by counting, ties by
// index) and the matching columns of V gathered into Z.
__global__ void __launch_bounds__(NT) rank_diag(int64_t n, const double* __restrict__ C,
                                                int64_t ldc, int32_t* __restrict__ rank) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const double v = C[i + i * ldc];
  int64_t r = 0;
  for (int64_t j = 0; j < n; ++j) {
    const double w = C[j + j * ldc];
    r += (w < v) || (w == v && j < i);
  }
  rank[i] = (int32_t)r;
}

__global__ void __launch_bounds__(NT) gather_sorted(int64_t n, const double* __restrict__ C,
                                                    int64_t ldc, const int32_t* __restrict__ rank,
                                                    const double* __restrict__ V, int64_t ldv,
                                                    double* __restrict__ lam, double* __restrict__ Z,
                                                    int64_t ldz) {
  const int64_t j = blockIdx.y;  // source column
  const int64_t dst = rank[j];
  if (blockIdx.x == 0 && threadIdx.x == 0) lam[dst] = C[j + j * ldc];
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    Z[i + dst * ldz] = V[i + j * ldv];
}

// Z(:, j) <- Z(:, j) / |Z(:, j)|: the accumulated rotations keep the columns
// orthogonal to rounding level but let their norms drift by about eps times the
// number of rounds; one rescaling restores them.
__global__ void __launch_bounds__(NT) normalize_columns(int64_t n, double* __restrict__ Z,
                                                        int64_t ldz) {
  __shared__ double red[NT / 64];
  double* z = Z + (int64_t)blockIdx.x * ldz;
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) a += z[i] * z[i];
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < NT / 64; ++w) t += red[w];
  const double sc = t > 0.0 ? 1.0 / sqrt(t) : 1.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) z[i] *= sc;
}

Layout layout_of(int64_t n) {
  Layout L;
  L.n = n;
  L.nb = JB;
  int64_t nblk = cdiv(n, JB);
  if (nblk & 1) ++nblk;
  if (nblk < 2) nblk = 2;
  L.nblk = (int)nblk;
  return L;
}

}  // namespace

size_t jacobi_workspace(int64_t n) {
  const Layout L = layout_of(n);
  Arena a;
  a.dry = true;
  a.take<double>((size_t)n * n);                 // V
  a.take<double>((size_t)(L.nblk / 2) * PN * PN);  // J of a round
  a.take<double>(2);                             // norm sums
  a.take<int32_t>(n);                            // rank
  return a.used + 256;
}

int jacobi_eig(int64_t n, double* C, int64_t ldc, double* lam, double* Z, int64_t ldz,
               int32_t* info, Arena& ws, hipStream_t s) {
  if (n <= 0) return 0;
  const Layout L = layout_of(n);
  const int K = L.nblk / 2;
  double* V = ws.take<double>((size_t)n * n);
  double* J = ws.take<double>((size_t)K * PN * PN);
  double* sums = ws.take<double>(2);
  int32_t* rank = ws.take<int32_t>(n);
  set_matrix(n, n, 0.0, 1.0, V, n, s);
  double h[2] = {0.0, 0.0};
  auto norms = [&]() {
    fill_f64(sums, 2, 0.0, s);
    hipLaunchKernelGGL(frob_parts, dim3((unsigned)n), dim3(NT), 0, s, n, (const double*)C, ldc,
                       sums);
    GEP_LAUNCH_CHECK();
    GEP_HIP(hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s));
    GEP_HIP(hipStreamSynchronize(s));
  };
  norms();
  const double fro2 = h[0] + h[1];
  const double eps = 2.220446049250313e-16;
  // rotations below this size change no eigenvalue at working precision
  const double tol = eps * sqrt(fro2) / (double)(n > 1 ? n : 1);
  // Converged when off(C) <= sqrt(n) eps |C|_F (about n eps |C|_2, the rounding
  // level the updates leave: of the order of eps |C| per entry), or when a sweep
  // no longer divides off(C) by four while it is below 1e-10 |C|_F (the
  // quadratic phase is over and that floor reached).
  const double stop = (double)n * eps * eps * fro2, floor2 = 1e-20 * fro2;
  double off2 = h[0];
  int sweeps = 0;
  bool converged = !(off2 > stop);
  const unsigned tiles = (unsigned)cdiv(n, 64);
  while (!converged && sweeps < MAX_SWEEPS) {
    for (int r = 0; r < L.nblk - 1; ++r) {
      hipLaunchKernelGGL(pair_eig, dim3((unsigned)K), dim3(NT), 0, s, L, (const double*)C, ldc, r,
                         tol, J);
      GEP_LAUNCH_CHECK();
      hipLaunchKernelGGL(pair_apply<false>, dim3(tiles, (unsigned)K), dim3(NT), 0, s, L, C, ldc, n,
                         r, (const double*)J);
      GEP_LAUNCH_CHECK();
      hipLaunchKernelGGL(pair_apply<true>, dim3(tiles, (unsigned)K), dim3(NT), 0, s, L, C, ldc, n, r,
                         (const double*)J);
      GEP_LAUNCH_CHECK();
      hipLaunchKernelGGL(pair_apply<true>, dim3(tiles, (unsigned)K), dim3(NT), 0, s, L, V, n, n, r,
                         (const double*)J);
      GEP_LAUNCH_CHECK();
    }
    ++sweeps;
    norms();
    const double prev = off2;
    off2 = h[0];
    converged = off2 <= stop || (off2 <= floor2 && off2 > prev / 16.0);
  }
  hipLaunchKernelGGL(rank_diag, dim3((unsigned)cdiv(n, NT)), dim3(NT), 0, s, n, (const double*)C,
                     ldc, rank);
  GEP_LAUNCH_CHECK();
  hipLaunchKernelGGL(gather_sorted, dim3((unsigned)cdiv(n, NT), (unsigned)n), dim3(NT), 0, s, n,
                     (const double*)C, ldc, (const int32_t*)rank, (const double*)V, n, lam, Z, ldz);
  GEP_LAUNCH_CHECK();
  hipLaunchKernelGGL(normalize_columns, dim3((unsigned)n), dim3(NT), 0, s, n, Z, ldz);
  GEP_LAUNCH_CHECK();
  if (!converged) raise_info(info, (int32_t)n, s);
  return sweeps;
}

}  // namespace gep

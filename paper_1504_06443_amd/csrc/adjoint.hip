// Adjoint of the generalized eigen-decomposition (A, B) -> (lambda, Y) for
// symmetric perturbations.  Differentiating A Y = B Y Lambda and Y^T B Y = I
// (section 3.1, Eq. 2) with P = Y^T dA Y and Q = Y^T dB Y gives
//   d lambda_i = P_ii - lambda_i Q_ii,
//   dY = Y Omega,  Omega_ij = (P_ij - lambda_j Q_ij) / (lambda_j - lambda_i)  (i != j),
//                  Omega_ii = -Q_ii / 2.
// Transposing this map for the cotangents (lambda_bar, Y_bar):
//   Wb = Y^T Y_bar,  Wa = (Wb - Wb^T)/2,  Ws = (Wb + Wb^T)/2,
//   F_ij = D / (D^2 + eta^2), D = lambda_j - lambda_i, F_ij = 0 when |D| <= tau_c,
//   Pb = F o Wa + diag(lambda_bar)                         (symmetric),
//   Qb = -1/2 (Lambda Pb + Pb Lambda + Ws)                 (symmetric),
//   A_bar = Y Pb Y^T,  B_bar = Y Qb Y^T.
// Cost: Wb (2 M^3), Y [Pb Qb] (4 M^3), the two lower triangles (2 x M^3) on the MFMA.
#include "common.h"
#include "internal.h"

namespace gep {
namespace {

// PQ = [Pb | Qb] (M x 2M, ld M) from Wb (or zero when absent) and lambda.
__global__ void adjoint_core(int64_t M, const double* __restrict__ lam,
                             const double* __restrict__ lam_bar, const double* __restrict__ Wb,
                             int64_t ldw, double eta, double tau_c, double* __restrict__ PQ) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M) return;
  const double li = lam[i], lj = lam[j];
  double wij = 0.0, wji = 0.0;
  if (Wb) {
    wij = Wb[i + j * ldw];
    wji = Wb[j + i * ldw];
  }
  const double wa = 0.5 * (wij - wji), ws = 0.5 * (wij + wji);
  double p = 0.0;
  if (i != j) {
    const double d = lj - li;
    if (fabs(d) > tau_c) p = d / (d * d + eta * eta) * wa;
  } else if (lam_bar) {
    p = lam_bar[i];
  }
  PQ[i + j * M] = p;
  PQ[i + (j + M) * M] = -0.5 * (li * p + p * lj + ws);
}

__global__ void mirror_lower(int64_t M, double* __restrict__ X, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M || i >= j) return;  // strict upper triangle: i < j
  X[i + j * ld] = X[j + i * ld];
}

}  // namespace

size_t backward_workspace(int64_t M) {
  Arena a;
  a.dry = true;
  a.take<double>((size_t)M * M);      // Wb
  a.take<double>((size_t)M * 2 * M);  // [Pb Qb]
  a.take<double>((size_t)M * 2 * M);  // Y [Pb Qb]
  return a.used + 256;
}

void backward(int64_t M, const double* lam, const double* Y, int64_t ldy, const double* lam_bar,
              const double* Y_bar, int64_t ldyb, double eta, double tau_c, double* A_bar,
              int64_t ldab, double* B_bar, int64_t ldbb, Arena& ws, hipStream_t s) {
  double* Wb = ws.take<double>((size_t)M * M);
  double* PQ = ws.take<double>((size_t)M * 2 * M);
  double* T = ws.take<double>((size_t)M * 2 * M);
  if (Y_bar) {
    Gemm g;
    g.transA = true;
    g.m = M; g.n = M; g.k = M;
    g.A = Y; g.lda = ldy; g.B = Y_bar; g.ldb = ldyb; g.C = Wb; g.ldc = M;
    gemm(g, s);
  }
  hipLaunchKernelGGL(adjoint_core, dim3((unsigned)cdiv(M, 256), (unsigned)M), dim3(256), 0, s, M,
                     lam, lam_bar, (const double*)(Y_bar ? Wb : nullptr), M, eta, tau_c, PQ);
  GEP_LAUNCH_CHECK();
  {  // T = Y [Pb Qb]
    Gemm g;
    g.m = M; g.n = 2 * M; g.k = M;
    g.A = Y; g.lda = ldy; g.B = PQ; g.ldb = M; g.C = T; g.ldc = M;
    gemm(g, s);
  }
  {  // A_bar = (Y Pb) Y^T, lower triangle, then mirrored
    Gemm g;
    g.transB = true;
    g.uplo = 1;
    g.m = M; g.n = M; g.k = M;
    g.A = T; g.lda = M; g.B = Y; g.ldb = ldy; g.C = A_bar; g.ldc = ldab;
    gemm(g, s);
  }
  {  // B_bar = (Y Qb) Y^T
    Gemm g;
    g.transB = true;
    g.uplo = 1;
    g.m = M; g.n = M; g.k = M;
    g.A = T + M * M; g.lda = M; g.B = Y; g.ldb = ldy; g.C = B_bar; g.ldc = ldbb;
    gemm(g, s);
  }
  hipLaunchKernelGGL(mirror_lower, dim3((unsigned)cdiv(M, 256), (unsigned)M), dim3(256), 0, s, M,
                     A_bar, ldab);
  GEP_LAUNCH_CHECK();
  hipLaunchKernelGGL(mirror_lower, dim3((unsigned)cdiv(M, 256), (unsigned)M), dim3(256), 0, s, M,
                     B_bar, ldbb);
  GEP_LAUNCH_CHECK();
}

}  // namespace gep

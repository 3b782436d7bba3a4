// First stage of the two-stage reduction: full symmetric -> band of width b
// (the "narrow-band reduction" route of the two-stage solvers compared in
// section 3.1, whose TRD/BAND / BACK phases are timed in Table 3), and the
// matching back transformation Z <- Q1 Z.
//
// Panel p covers columns [p*b, p*b + b).  Its block below the band, P (n x b,
// n = N - p*b - b), is QR-factored with Householder reflectors,
// P = (I - V T V^T) R, and the trailing matrix A22 is updated two-sidedly:
//   X = A22 V T,  W = X - 1/2 V (T^T V^T X),  A22 <- A22 - V W^T - W V^T.
// R goes to the band; V (explicit: unit diagonal, zeros above) stays in the panel's
// place for the back transformation, T is kept per panel.
//
// The panel QR is latency-bound: one launch per column.  Each launch owns row
// slices of the panel in G workgroups: it applies the previous reflector to the
// remaining columns and accumulates, for the next column x, |x|^2 and x^T P_j.
// The last workgroup to finish (counter + device-scope fences) reduces the
// partial sums and forms the next reflector, so no grid-wide barrier is needed.
// All the O(n^2 b) work is in MFMA GEMMs.
#include "common.h"
#include "internal.h"

namespace gep {
namespace {

constexpr int NT = 256;
constexpr int MAXB = 64;  // largest supported band width

struct PanelState {
  double beta[MAXB];   // R(c, c)
  double tau[MAXB];
  double scal[MAXB];   // 1 / (x0 - beta): scales x(c+1:) into v
  double wv[MAXB];     // tau * v^T P_j for the current reflector
  unsigned int counter;
};

// Partial sums: part[g * (MAXB + 1) + q]; q = 0 -> sum_{i>c} x_i^2, q = 1 + j -> sum_{i>=c} x_i P(i, j).
__global__ void __launch_bounds__(NT)
panel_step(int64_t n, int w, int kmax, int c, double* __restrict__ P, int64_t ld,
           PanelState* __restrict__ st, double* __restrict__ part, int64_t rows_per) {
  __shared__ double red[NT / 64][MAXB + 1];
  __shared__ bool last;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  int64_t r1 = r0 + rows_per;
  if (r1 > n) r1 = n;

  // 1) apply reflector c-1 to columns c..w-1 (rows >= c-1) and store v_{c-1}
  if (c > 0) {
    const int p = c - 1;
    const double scal = st->scal[p];
    for (int64_t i = r0 + tid; i < r1; i += NT) {
      if (i < p) continue;
      double v;
      if (i == p) {
        v = 1.0;
      } else {
        v = P[i + (int64_t)p * ld] * scal;
        P[i + (int64_t)p * ld] = v;
      }
      for (int j = c; j < w; ++j) P[i + (int64_t)j * ld] -= v * st->wv[j];
    }
  }
  if (c >= kmax) return;

  // 2) partial sums for column c
  double acc[MAXB + 1];
#pragma unroll
  for (int q = 0; q <= MAXB; ++q) acc[q] = 0.0;
  for (int64_t i = r0 + tid; i < r1; i += NT) {
    if (i < c) continue;
    const double x = P[i + (int64_t)c * ld];
    if (i > c) acc[0] += x * x;
#pragma unroll
    for (int j = 0; j < MAXB; ++j)
      if (j > c && j < w) acc[1 + j] += x * P[i + (int64_t)j * ld];
  }
  // wave reduction then workgroup reduction
#pragma unroll
  for (int q = 0; q <= MAXB; ++q) {
    double v = acc[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  if (tid <= MAXB) {
    double v = 0.0;
    for (int wv = 0; wv < NT / 64; ++wv) v += red[wv][tid];
    part[(int64_t)blockIdx.x * (MAXB + 1) + tid] = v;
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const unsigned int prev = atomicAdd(&st->counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();

  // 3) last workgroup: reduce and form reflector c
  __shared__ double tot[MAXB + 1];
  if (tid <= MAXB) {
    double v = 0.0;
    for (unsigned int g = 0; g < gridDim.x; ++g) v += part[(int64_t)g * (MAXB + 1) + tid];
    tot[tid] = v;
  }
  __syncthreads();
  if (tid == 0) {
    const double x0 = P[c + (int64_t)c * ld];
    const double sigma = tot[0];
    double beta, tau, scal;
    if (sigma == 0.0) {
      beta = x0;
      tau = 0.0;
      scal = 0.0;
    } else {
      const double mu = sqrt(x0 * x0 + sigma);
      beta = (x0 >= 0.0) ? -mu : mu;
      tau = (beta - x0) / beta;
      scal = 1.0 / (x0 - beta);
    }
    st->beta[c] = beta;
    st->tau[c] = tau;
    st->scal[c] = scal;
    st->counter = 0u;
  }
  __syncthreads();
  if (tid < MAXB) {
    const int j = tid;
    double wvj = 0.0;
    if (j > c && j < w) {
      const double x0 = P[c + (int64_t)c * ld];
      const double pcj = P[c + (int64_t)j * ld];
      const double vtp = pcj + st->scal[c] * (tot[1 + j] - x0 * pcj);
      wvj = st->tau[c] * vtp;
    }
    st->wv[j] = wvj;
  }
  __threadfence();
}

// After the panel QR: move R (upper trapezoid of the first kmax rows) to the band,
// replace it by the explicit V (unit diagonal, zeros above), zero the V columns
// without a reflector, and publish tau.
__global__ void panel_finish(int64_t n, int w, int kmax, double* __restrict__ P, int64_t ld,
                             const PanelState* __restrict__ st, double* __restrict__ band,
                             int64_t ldband, int64_t col0, int b, double* __restrict__ tau_out) {
  const int c = blockIdx.x;  // one block per panel column
  const int tid = threadIdx.x;
  // R entries: rows i <= c, i < n
  for (int i = tid; i <= c && i < n; i += blockDim.x) {
    double r;
    if (i == c && c < kmax) r = st->beta[c];
    else r = P[i + (int64_t)c * ld];
    band[(b + i - c) + (col0 + c) * ldband] = r;
  }
  __syncthreads();
  for (int64_t i = tid; i < n; i += blockDim.x) {
    double v;
    if (c >= kmax) v = 0.0;
    else if (i < c) v = 0.0;
    else if (i == c) v = 1.0;
    else continue;  // already holds v
    P[i + (int64_t)c * ld] = v;
  }
  if (tid == 0) tau_out[c] = (c < kmax) ? st->tau[c] : 0.0;
}

// Copy the lower triangle of the diagonal block [col0, col0 + w) into the band.
__global__ void diag_to_band(const double* __restrict__ C, int64_t ldc, int64_t col0, int w,
                             double* __restrict__ band, int64_t ldband) {
  const int c = blockIdx.x;
  for (int i = c + threadIdx.x; i < w; i += blockDim.x)
    band[(i - c) + (col0 + c) * ldband] = C[(col0 + i) + (col0 + c) * ldc];
}

// T factor of the compact WY form: T(c,c) = tau_c,
// T(0:c, c) = -tau_c T(0:c, 0:c) G(0:c, c) with G = V^T V.  One workgroup.
__global__ void form_t(int w, const double* __restrict__ G, const double* __restrict__ tau,
                       double* __restrict__ T) {
  __shared__ double Ts[MAXB][MAXB + 1];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < w * w; idx += blockDim.x) Ts[idx % w][idx / w] = 0.0;
  __syncthreads();
  for (int c = 0; c < w; ++c) {
    const double tc = tau[c];
    if (tid < c) {
      double s = 0.0;
      for (int k = tid; k < c; ++k) s += Ts[tid][k] * G[k + c * w];
      Ts[tid][c] = -tc * s;
    }
    if (tid == 0) Ts[c][c] = tc;
    __syncthreads();
  }
  for (int idx = tid; idx < w * w; idx += blockDim.x) T[idx] = Ts[idx % w][idx / w];
}

// VW = [V | W], WV = [W | V]  (n x 2w, ld n)
__global__ void pack_vw(int64_t n, int w, const double* __restrict__ V, int64_t ldv,
                        const double* __restrict__ W, double* __restrict__ VW,
                        double* __restrict__ WV) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = blockIdx.y;
  const double v = V[i + (int64_t)c * ldv];
  const double x = W[i + (int64_t)c * n];
  VW[i + (int64_t)c * n] = v;
  VW[i + (int64_t)(w + c) * n] = x;
  WV[i + (int64_t)c * n] = x;
  WV[i + (int64_t)(w + c) * n] = v;
}

int panel_blocks(int64_t n) {
  // aim for ~256-row slices, at most 512 workgroups
  int64_t g = cdiv(n, 256);
  if (g > 512) g = 512;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

size_t sy2sb_workspace(int64_t n, int b) {
  const size_t nb = (size_t)n * b;
  size_t e = 0;
  e += 2 * nb;               // X, X2
  e += 4 * nb;               // VW, WV
  e += 4 * (size_t)b * b;    // G, Y, Ws, tau
  e += splitk_work_elems(b, b, n) + 64;
  e += 512 * (MAXB + 1);     // partials
  return e * sizeof(double) + sizeof(PanelState) + 16 * 256;
}

void sy2sb(const BandReduction& r, Arena& ws, hipStream_t s) {
  const int64_t N = r.n;
  const int b = r.b;
  if (b > MAXB || b < 1) throw HipError{hipErrorInvalidValue, "band width"};
  double* X = ws.take<double>((size_t)N * b);
  double* X2 = ws.take<double>((size_t)N * b);
  double* VW = ws.take<double>((size_t)N * 2 * b);
  double* WV = ws.take<double>((size_t)N * 2 * b);
  double* G = ws.take<double>((size_t)b * b);
  double* Y = ws.take<double>((size_t)b * b);
  double* Ws = ws.take<double>((size_t)b * b);
  double* tau = ws.take<double>((size_t)b);
  const size_t skw = splitk_work_elems(b, b, N) + 64;
  double* skbuf = ws.take<double>(skw);
  double* part = ws.take<double>(512 * (MAXB + 1));
  PanelState* st = ws.take<PanelState>(1);
  GEP_HIP(hipMemsetAsync(st, 0, sizeof(PanelState), s));
  fill_f64(r.band, r.ldband * N, 0.0, s);

  for (int64_t col0 = 0; col0 < N; col0 += b) {
    const int w = (int)((N - col0) < b ? (N - col0) : b);
    hipLaunchKernelGGL(diag_to_band, dim3(w), dim3(64), 0, s, (const double*)r.C, r.ldc, col0, w,
                       r.band, r.ldband);
    GEP_LAUNCH_CHECK();
    const int64_t p0 = col0 + b;
    const int64_t n = N - p0;
    if (n <= 0) break;
    double* P = r.C + p0 + col0 * r.ldc;
    const int kmax = (int)(n < w ? n : w);
    const int gb = panel_blocks(n);
    const int64_t rows_per = cdiv(n, gb);
    for (int c = 0; c <= kmax; ++c) {
      hipLaunchKernelGGL(panel_step, dim3(gb), dim3(NT), 0, s, n, w, kmax, c, P, r.ldc, st, part,
                         rows_per);
      GEP_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(panel_finish, dim3(w), dim3(256), 0, s, n, w, kmax, P, r.ldc,
                       (const PanelState*)st, r.band, r.ldband, col0, b, tau);
    GEP_LAUNCH_CHECK();
    double* T = r.T + (col0 / b) * (int64_t)b * b;
    {  // G = V^T V
      Gemm g;
      g.transA = true;
      g.m = w; g.n = w; g.k = n;
      g.A = P; g.lda = r.ldc; g.B = P; g.ldb = r.ldc; g.C = G; g.ldc = w;
      g.work = skbuf; g.work_elems = skw;
      gemm(g, s);
    }
    hipLaunchKernelGGL(form_t, dim3(1), dim3(256), 0, s, w, (const double*)G, (const double*)tau, T);
    GEP_LAUNCH_CHECK();
    double* A22 = r.C + p0 + p0 * r.ldc;
    {  // X = A22 V   (A22 symmetric, lower stored)
      Gemm g;
      g.symA = true;
      g.m = n; g.n = w; g.k = n;
      g.A = A22; g.lda = r.ldc; g.B = P; g.ldb = r.ldc; g.C = X; g.ldc = n;
      gemm(g, s);
    }
    {  // X2 = X T
      Gemm g;
      g.m = n; g.n = w; g.k = w;
      g.A = X; g.lda = n; g.B = T; g.ldb = w; g.C = X2; g.ldc = n;
      gemm(g, s);
    }
    {  // Y = V^T X2
      Gemm g;
      g.transA = true;
      g.m = w; g.n = w; g.k = n;
      g.A = P; g.lda = r.ldc; g.B = X2; g.ldb = n; g.C = Y; g.ldc = w;
      g.work = skbuf; g.work_elems = skw;
      gemm(g, s);
    }
    {  // Ws = T^T Y
      Gemm g;
      g.transA = true;
      g.m = w; g.n = w; g.k = w;
      g.A = T; g.lda = w; g.B = Y; g.ldb = w; g.C = Ws; g.ldc = w;
      gemm(g, s);
    }
    {  // W = X2 - 1/2 V Ws   (in X2)
      Gemm g;
      g.m = n; g.n = w; g.k = w; g.alpha = -0.5; g.beta = 1.0;
      g.A = P; g.lda = r.ldc; g.B = Ws; g.ldb = w; g.C = X2; g.ldc = n;
      gemm(g, s);
    }
    hipLaunchKernelGGL(pack_vw, dim3((unsigned)cdiv(n, 256), (unsigned)w), dim3(256), 0, s, n, w,
                       (const double*)P, r.ldc, (const double*)X2, VW, WV);
    GEP_LAUNCH_CHECK();
    {  // A22 -= V W^T + W V^T   (lower triangle)
      Gemm g;
      g.transB = true;
      g.uplo = 1;
      g.m = n; g.n = n; g.k = 2 * w; g.alpha = -1.0; g.beta = 1.0;
      g.A = VW; g.lda = n; g.B = WV; g.ldb = n; g.C = A22; g.ldc = r.ldc;
      gemm(g, s);
    }
  }
}

// Z <- Q1 Z, Q1 = Q_0 Q_1 ... Q_last with Q_p = I - V_p T_p V_p^T:
// apply the panels in reverse order.
void apply_q1(const BandReduction& r, double* Z, int64_t ldz, int64_t ncols, Arena& ws,
              hipStream_t s) {
  const int64_t N = r.n;
  const int b = r.b;
  double* W1 = ws.take<double>((size_t)b * ncols);
  double* W2 = ws.take<double>((size_t)b * ncols);
  int64_t last = 0;
  for (int64_t col0 = 0; col0 + b < N; col0 += b) last = col0;
  if (N <= b) return;
  for (int64_t col0 = last; col0 >= 0; col0 -= b) {
    const int64_t p0 = col0 + b;
    const int64_t n = N - p0;
    const int w = (int)((N - col0) < b ? (N - col0) : b);
    const double* V = r.C + p0 + col0 * r.ldc;
    const double* T = r.T + (col0 / b) * (int64_t)b * b;
    {
      Gemm g;
      g.transA = true;
      g.m = w; g.n = ncols; g.k = n;
      g.A = V; g.lda = r.ldc; g.B = Z + p0; g.ldb = ldz; g.C = W1; g.ldc = w;
      gemm(g, s);
    }
    {
      Gemm g;
      g.m = w; g.n = ncols; g.k = w;
      g.A = T; g.lda = w; g.B = W1; g.ldb = w; g.C = W2; g.ldc = w;
      gemm(g, s);
    }
    {
      Gemm g;
      g.m = n; g.n = ncols; g.k = w; g.alpha = -1.0; g.beta = 1.0;
      g.A = V; g.lda = r.ldc; g.B = W2; g.ldb = w; g.C = Z + p0; g.ldc = ldz;
      gemm(g, s);
    }
  }
}

}  // namespace gep

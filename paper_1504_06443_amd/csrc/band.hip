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
// The panel QR is latency-bound (one reduction per column); it runs as one
// cooperative launch per panel with the panel held in LDS across the grid.  All
// the O(n^2 b) work is in MFMA GEMMs.
#include "common.h"
#include "internal.h"

namespace gep {
namespace {

constexpr int NT = 256;
constexpr int MAXB = 64;  // largest supported band width

// Band data shared between workgroups of one launch: agent-scope relaxed atomics
// (coherent across XCDs, written through).
__device__ inline double cld(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void cst(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whole-panel QR in one cooperative launch.  Workgroup g keeps rows
// [g*rows_per, (g+1)*rows_per) of the panel in LDS for the whole factorisation.
// Column c: every workgroup forms partial sums (|x|^2 below row c, x^T P_j), the
// grid meets at a barrier, every workgroup reduces all partials in the same order
// (so all derive the identical reflector) and updates its slice.  Partials and the
// top row are double buffered by column parity, so one barrier per column is
// enough.  On exit: V explicit (unit diagonal, zeros above) in P, R in the band,
// tau[0..w).
struct PanelArgs {
  int64_t n;
  int w, kmax;
  double* P;
  int64_t ld;
  double* part;     // [2][G][MAXB]
  double* top;      // [2][MAXB]
  unsigned* bar;    // barrier counter (zero on entry)
  double* tau;
  double* band;
  int64_t ldband, col0;
  int b;
  int rows_per;
  int32_t* err;     // sticky across the panels of one reduction
  uint64_t timeout_ticks;
  int force_fail;   // debug: a barrier not passed at its first poll gives up
};

__device__ bool grid_barrier(const PanelArgs& a, unsigned target) {
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(a.bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t0 = wall_clock64();
    ok = 1;
    while (__hip_atomic_load(a.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (a.force_fail || wall_clock64() - t0 > a.timeout_ticks) {
        __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return ok != 0;
}

// Sum of the partials gg = qt, qt + 4, qt + 8, ... < G of column q, added in
// that order; K loads are issued before the first is used.
template <int K>
__device__ inline double gather_partials(const double* part, int G, int qt, int q) {
  double s = 0.0;
  for (int gg0 = qt; gg0 < G; gg0 += 4 * K) {
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int gg = gg0 + 4 * k;
      v[k] = cld(&part[(size_t)(gg < G ? gg : G - 1) * MAXB + q]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) s += (gg0 + 4 * k < G) ? v[k] : 0.0;
  }
  return s;
}

__global__ void __launch_bounds__(NT) panel_qr_coop(PanelArgs a) {
  extern __shared__ double Ps[];  // rows_per x (MAXB + 1), row-major
  __shared__ double wv[MAXB];
  __shared__ double red[NT / MAXB][MAXB];  // quarter sums of the partials
  __shared__ double tops[MAXB];             // the panel's current top row
  constexpr int LDP = MAXB + 1;
  const int tid = threadIdx.x;
  const int G = gridDim.x, g = blockIdx.x;
  const int w = a.w;
  const int64_t r0 = (int64_t)g * a.rows_per;
  int nr = (int)((a.n - r0) < a.rows_per ? (a.n - r0) : a.rows_per);
  if (nr < 0) nr = 0;
  // After a failed barrier (this panel or an earlier one) the reduction is
  // abandoned: the remaining panels leave at once with every reflector the
  // identity (tau = 0), so the later steps run on finite data, and the caller
  // learns of the failure through info.
  __shared__ int failed_sh;
  if (tid == 0)
    failed_sh = __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  __syncthreads();
  if (failed_sh) {
    if (g == 0)
      for (int c = tid; c < w; c += NT) a.tau[c] = 0.0;
    return;
  }
  // load the slice
  for (int j = 0; j < w; ++j)
    for (int i = tid; i < nr; i += NT) Ps[i * LDP + j] = a.P[(r0 + i) + (int64_t)j * a.ld];
  __syncthreads();
  for (int c = 0; c < a.kmax; ++c) {
    const int buf = c & 1;
    double* part = a.part + (size_t)buf * G * MAXB;
    double* top = a.top + buf * MAXB;
    // partial sums: thread (q, sub) sums rows sub, sub + 4, ... of the slice that
    // lie at or below the panel's top row c (strictly below it for column c's own
    // norm), in eight independent sums so that eight row pairs are in flight
    {
      const int q = tid >> 2, sub = tid & 3;
      double acc = 0.0;
      if (q >= c && q < w) {
        const int64_t lo = (q == c) ? (int64_t)c + 1 : (int64_t)c;
        int i = sub;
        if (r0 + i < lo) i += (int)((lo - r0 - i + 3) / 4) * 4;
        double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (; i < nr; i += 32) {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int iu = i + 4 * u;
            const int ii = iu < nr ? iu : nr - 1;  // clamped row, in the slice
            const double x = Ps[ii * LDP + c] * Ps[ii * LDP + q];
            s8[u] += iu < nr ? x : 0.0;
          }
        }
        acc = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      if (sub == 0 && q >= c && q < w) cst(&part[(size_t)g * MAXB + q], acc);
    }
    if (c >= r0 && c < r0 + nr) {
      const int li = (int)(c - r0);
      for (int q = c + tid; q < w; q += NT) cst(&top[q], Ps[li * LDP + q]);
    }
    if (!grid_barrier(a, (unsigned)(G * (c + 1)))) {
      if (g == 0)
        for (int cc = tid; cc < w; cc += NT) a.tau[cc] = 0.0;
      return;
    }
    // Every workgroup reduces the partials in the same fixed order, so all derive
    // the identical reflector.  Thread (quarter, q) sums partials quarter,
    // quarter + 4, ... of column q, with all of its remote loads in flight at once
    // for G <= 128 (each round of remote loads costs a full memory latency), and
    // the quarter sums are added in LDS in a fixed order.  The top row is fetched
    // in the same round.
    {
      const int q = tid & (MAXB - 1), qt = tid >> 6;
      double s = 0.0;
      if (q >= c && q < w) {
        const double tq = qt == 0 ? cld(&top[q]) : 0.0;
        s = G <= 32 ? gather_partials<8>(part, G, qt, q) : gather_partials<32>(part, G, qt, q);
        if (qt == 0) tops[q] = tq;
      }
      red[qt][q] = s;
    }
    __syncthreads();
    // reflector scalars, computed redundantly by every thread from the same values
    double beta, tau, scal;
    {
      const double x0 = tops[c];
      const double sigma = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
      if (sigma == 0.0) {
        beta = x0; tau = 0.0; scal = 0.0;
      } else {
        const double mu = sqrt(x0 * x0 + sigma);
        beta = (x0 >= 0.0) ? -mu : mu;
        tau = (beta - x0) / beta;
        scal = 1.0 / (x0 - beta);
      }
      if (tid < MAXB) {
        double wvq = 0.0;
        if (tid > c && tid < w) {
          const double pcj = tops[tid];
          const double tot = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
          wvq = tau * (pcj + scal * (tot - x0 * pcj));
        }
        wv[tid] = wvq;
      }
    }
    __syncthreads();
    // apply H_c to the slice, store v_c
    for (int i = tid; i < nr; i += NT) {
      const int64_t gi = r0 + i;
      if (gi < c) continue;
      double v;
      if (gi == c) {
        v = 1.0;
        Ps[i * LDP + c] = beta;
      } else {
        v = Ps[i * LDP + c] * scal;
        Ps[i * LDP + c] = v;
      }
      // eight columns' operands read before their updates are written (one LDS
      // round trip per eight elements)
      int j = c + 1;
      for (; j + 7 < w; j += 8) {
        double x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          x[u] = Ps[i * LDP + j + u];
          y[u] = wv[j + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) Ps[i * LDP + j + u] = x[u] - v * y[u];
      }
      for (; j < w; ++j) Ps[i * LDP + j] -= v * wv[j];
    }
    if (g == 0 && tid == 0) a.tau[c] = tau;
    __syncthreads();
  }
  if (g == 0)
    for (int c = a.kmax + tid; c < w; c += NT) a.tau[c] = 0.0;
  // write back: R to the band, explicit V to the panel
  for (int j = 0; j < w; ++j) {
    for (int i = tid; i < nr; i += NT) {
      const int64_t gi = r0 + i;
      const double x = Ps[i * LDP + j];
      double v;
      if (gi <= j || j >= a.kmax) {
        if (gi <= j) a.band[(a.b + gi - j) + (a.col0 + j) * a.ldband] = x;  // R(gi, j)
        v = (gi == j && j < a.kmax) ? 1.0 : 0.0;
      } else {
        v = x;
      }
      a.P[gi + (int64_t)j * a.ld] = v;
    }
  }
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
  __shared__ double Gs[MAXB][MAXB + 1];
  const int tid = threadIdx.x;
  for (int j = tid >> 6; j < w; j += 4)
    for (int i = tid & 63; i < w; i += 64) {
      Gs[i][j] = G[i + j * w];
      Ts[i][j] = 0.0;
    }
  __syncthreads();
  for (int c = 0; c < w; ++c) {
    const double tc = tau[c];
    // 4 threads per row of T(0:c, c)
    const int row = tid >> 2, q = tid & 3;
    double acc = 0.0;
    if (row < c)
      for (int k = row + q; k < c; k += 4) acc += Ts[row][k] * Gs[k][c];
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (row < c && q == 0) Ts[row][c] = -tc * acc;
    if (tid == 0) Ts[c][c] = tc;
    __syncthreads();
  }
  for (int j = tid >> 6; j < w; j += 4)
    for (int i = tid & 63; i < w; i += 64) T[i + j * w] = Ts[i][j];
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

// Combined update of a panel pair (p, p+1) on the trailing matrix of p+1:
//   VW4 = [V_p | W_p | V_q | W_q],  WV4 = [W_p | V_p | W_q | V_q]   (n1 x 2w + 2w1, ld n1)
// with V_p, W_p taken from rows off.. of the packed VW of panel p (ld n).
__global__ void pack_vw2(int64_t n1, int w, int w1, int64_t off, const double* __restrict__ VWp,
                         int64_t n, const double* __restrict__ Vq, int64_t ldv,
                         const double* __restrict__ Wq, double* __restrict__ VW4,
                         double* __restrict__ WV4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n1) return;
  const int c = blockIdx.y;  // 0 .. 2w + 2w1 - 1
  double vw, wv;
  if (c < w) {
    vw = VWp[off + i + (int64_t)c * n];            // V_p
    wv = VWp[off + i + (int64_t)(w + c) * n];      // W_p
  } else if (c < 2 * w) {
    vw = VWp[off + i + (int64_t)c * n];            // W_p
    wv = VWp[off + i + (int64_t)(c - w) * n];      // V_p
  } else if (c < 2 * w + w1) {
    const int cc = c - 2 * w;
    vw = Vq[i + (int64_t)cc * ldv];
    wv = Wq[i + (int64_t)cc * n1];
  } else {
    const int cc = c - 2 * w - w1;
    vw = Wq[i + (int64_t)cc * n1];
    wv = Vq[i + (int64_t)cc * ldv];
  }
  VW4[i + (int64_t)c * n1] = vw;
  WV4[i + (int64_t)c * n1] = wv;
}

size_t panel_lds() { return sizeof(double) * 256 * (MAXB + 1); }

// Largest grid of panel_qr_coop whose workgroups are all resident at once.
int coop_blocks() {
  // computed once per process (thread-safe initialisation; retried if it throws)
  static const int cached = [] {
    int dev = 0, cus = 0, per = 0;
    GEP_HIP(hipGetDevice(&dev));
    GEP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    GEP_HIP(hipFuncSetAttribute((const void*)panel_qr_coop,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)panel_lds()));
    GEP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)panel_qr_coop, NT,
                                                         panel_lds()));
    const int c = cus * (per > 0 ? per : 1);
    return c > 512 ? 512 : c;
  }();
  return cached;
}

}  // namespace

size_t sy2sb_workspace(int64_t n, int b) {
  const size_t nb = (size_t)n * b;
  size_t e = 0;
  e += 2 * nb;               // X, X2
  e += 4 * nb;               // VW, WV
  e += 8 * nb;               // VW4, WV4 (panel pairs)
  e += 6 * (size_t)b * b;    // G, Y, Ws, tau, U (2b x b)
  e += splitk_work_elems(2 * b, b, n) + 64;
  e += 2 * 512 * MAXB + 2 * MAXB;  // partials, top row
  return e * sizeof(double) + (cdiv(n, b) + 1) * sizeof(unsigned) + 16 * 256;
}

void sy2sb(const BandReduction& r, Arena& ws, hipStream_t s) {
  const int64_t N = r.n;
  const int b = r.b;
  if (b > MAXB || b < 1) throw HipError{hipErrorInvalidValue, "band width"};
  double* X = ws.take<double>((size_t)N * b);
  double* X2 = ws.take<double>((size_t)N * b);
  double* VW = ws.take<double>((size_t)N * 2 * b);
  double* WV = ws.take<double>((size_t)N * 2 * b);
  double* VW4 = ws.take<double>((size_t)N * 4 * b);
  double* WV4 = ws.take<double>((size_t)N * 4 * b);
  double* G = ws.take<double>((size_t)b * b);
  double* Y = ws.take<double>((size_t)b * b);
  double* Ws = ws.take<double>((size_t)b * b);
  double* U = ws.take<double>((size_t)2 * b * b);
  double* tau = ws.take<double>((size_t)b);
  const size_t skw = splitk_work_elems(2 * b, b, N) + 64;
  double* skbuf = ws.take<double>(skw);
  double* part = ws.take<double>(2 * 512 * MAXB);
  double* top = ws.take<double>(2 * MAXB);
  const int64_t npanels = cdiv(N, b);
  unsigned* bar = ws.take<unsigned>(npanels + 1);
  int32_t* err = ws.take<int32_t>(1);
  fill_i32((int32_t*)bar, npanels + 1, 0, s);
  fill_i32(err, 1, 0, s);
  fill_f64(tau, b, 0.0, s);
  fill_f64(r.band, r.ldband * N, 0.0, s);
  const int coop_max = coop_blocks();
  const uint64_t timeout_ticks = wait_limit_ticks();
  const int force_fail = force_wait_timeout() ? 1 : 0;

  // Diagonal block of the panel at col0 into the band, then the QR of the n x w
  // panel below it (reflectors stay in place, R goes to the band) and its T.
  auto factor = [&](int64_t col0, int w, int64_t n) {
    hipLaunchKernelGGL(diag_to_band, dim3(w), dim3(64), 0, s, (const double*)r.C, r.ldc, col0, w,
                       r.band, r.ldband);
    GEP_LAUNCH_CHECK();
    double* P = r.C + (col0 + b) + col0 * r.ldc;
    const int kmax = (int)(n < w ? n : w);
    {
      const int Gn = (int)cdiv(n, 256) < coop_max ? (int)cdiv(n, 256) : coop_max;
      PanelArgs pa;
      pa.n = n; pa.w = w; pa.kmax = kmax; pa.P = P; pa.ld = r.ldc; pa.part = part; pa.top = top;
      pa.bar = bar + (col0 / b); pa.tau = tau; pa.band = r.band; pa.ldband = r.ldband;
      pa.col0 = col0; pa.b = b; pa.rows_per = (int)cdiv(n, Gn); pa.err = err;
      pa.timeout_ticks = timeout_ticks;
      pa.force_fail = force_fail;
      if (pa.rows_per > 256) throw HipError{hipErrorInvalidValue, "panel too tall"};
      // Householder QR of an n x kmax panel: 2 n kmax^2 - 2 kmax^3 / 3 flops
      ProbeScope probe(PROBE_PANEL_QR, s,
                       2.0 * (double)n * kmax * kmax - 2.0 * (double)kmax * kmax * kmax / 3.0);
      if (r.coop) {
        void* args[] = {&pa};
        GEP_HIP(hipLaunchCooperativeKernel((const void*)panel_qr_coop, dim3(Gn), dim3(NT), args,
                                           panel_lds(), s));
      } else {
        // Batched solves: plain launch (graph-capturable).  Few workgroups (G <= 8
        // for n <= 2048) per panel and at most 16 panels in flight, so the grid's
        // workgroups always find free CUs; the barrier wait is bounded in time.
        hipLaunchKernelGGL(panel_qr_coop, dim3(Gn), dim3(NT), panel_lds(), s, pa);
        GEP_LAUNCH_CHECK();
      }
    }
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
  };
  // X (n x w) holds A22 V on entry; leaves W = X T - 1/2 V (T^T V^T X T) in X2.
  auto form_w = [&](int64_t col0, int w, int64_t n) {
    const double* P = r.C + (col0 + b) + col0 * r.ldc;
    const double* T = r.T + (col0 / b) * (int64_t)b * b;
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
  };
  // X = A22 V (A22 symmetric, lower stored).  Products of at least split_rows
  // rows (tuning table, by default 2048) split K over the pair buffer VW4, which
  // is idle between a trailing update and the next pair's packing.  Smaller ones
  // (all of a batch of orders <= 2048, whose instances already share the GPU) stay
  // unsplit; the rule depends on the order alone, so a batched instance and a
  // single solve of the same problem take the same path and give the same bits.
  const int64_t split_rows = tune("symm_split_rows", N);
  auto symm_v = [&](int64_t col0, int w, int64_t n) {
    const int64_t p0 = col0 + b;
    Gemm g;
    g.symA = true;
    g.m = n; g.n = w; g.k = n;
    g.A = r.C + p0 + p0 * r.ldc; g.lda = r.ldc;
    g.B = r.C + p0 + col0 * r.ldc; g.ldb = r.ldc;
    g.C = X; g.ldc = n;
    if (n >= split_rows) {
      g.work = VW4;
      g.work_elems = (size_t)N * 4 * b;
    }
    gemm(g, s);
  };

  // Panels are taken in pairs (p, q = p + 1).  After p only q's block column is
  // updated; q is factored against the stale trailing matrix, with its product
  // corrected by the pending rank-2w term:
  //   A22' = A22 - V_p W_p^T - W_p V_p^T   on rows / columns past q's block,
  //   A22' V_q = A22 V_q - [V_p W_p] ([W_p V_p]^T V_q),
  // and the trailing matrix gets one update of rank 2w + 2w_q instead of two.
  for (int64_t col0 = 0; col0 < N;) {
    const int w = (int)((N - col0) < b ? (N - col0) : b);
    const int64_t p0 = col0 + b;
    const int64_t n = N - p0;
    if (n <= 0) {  // last diagonal block
      hipLaunchKernelGGL(diag_to_band, dim3(w), dim3(64), 0, s, (const double*)r.C, r.ldc, col0,
                         w, r.band, r.ldband);
      GEP_LAUNCH_CHECK();
      break;
    }
    factor(col0, w, n);
    symm_v(col0, w, n);
    form_w(col0, w, n);
    const double* P = r.C + p0 + col0 * r.ldc;
    hipLaunchKernelGGL(pack_vw, dim3((unsigned)cdiv(n, 256), (unsigned)w), dim3(256), 0, s, n, w,
                       P, r.ldc, (const double*)X2, VW, WV);
    GEP_LAUNCH_CHECK();
    double* A22 = r.C + p0 + p0 * r.ldc;
    const int64_t n1 = n - b;  // trailing order after the next panel
    if (n1 <= 0) {
      // no second panel with rows below its block: plain rank-2w update
      Gemm g;
      g.transB = true;
      g.uplo = 1;
      g.m = n; g.n = n; g.k = 2 * w; g.alpha = -1.0; g.beta = 1.0;
      g.A = VW; g.lda = n; g.B = WV; g.ldb = n; g.C = A22; g.ldc = r.ldc;
      gemm(g, s);
      col0 += b;
      continue;
    }
    {  // block column of q: A22[:, 0:b] -= [V W] [W V](0:b, :)^T
      Gemm g;
      g.transB = true;
      g.m = n; g.n = b; g.k = 2 * w; g.alpha = -1.0; g.beta = 1.0;
      g.A = VW; g.lda = n; g.B = WV; g.ldb = n; g.C = A22; g.ldc = r.ldc;
      gemm(g, s);
    }
    const int64_t col1 = p0;
    const int w1 = b;  // n1 > 0, so q has a full block
    factor(col1, w1, n1);
    symm_v(col1, w1, n1);
    {  // U = [W_p V_p](b:, :)^T V_q   (2w x w1, k = n1)
      Gemm g;
      g.transA = true;
      g.m = 2 * w; g.n = w1; g.k = n1;
      g.A = WV + b; g.lda = n; g.B = r.C + (col1 + b) + col1 * r.ldc; g.ldb = r.ldc;
      g.C = U; g.ldc = 2 * w;
      g.work = skbuf; g.work_elems = skw;
      gemm(g, s);
    }
    {  // X -= [V_p W_p](b:, :) U
      Gemm g;
      g.m = n1; g.n = w1; g.k = 2 * w; g.alpha = -1.0; g.beta = 1.0;
      g.A = VW + b; g.lda = n; g.B = U; g.ldb = 2 * w; g.C = X; g.ldc = n1;
      gemm(g, s);
    }
    form_w(col1, w1, n1);
    hipLaunchKernelGGL(pack_vw2, dim3((unsigned)cdiv(n1, 256), (unsigned)(2 * w + 2 * w1)), dim3(256),
                       0, s, n1, w, w1, (int64_t)b, (const double*)VW, n,
                       (const double*)(r.C + (col1 + b) + col1 * r.ldc), r.ldc, (const double*)X2,
                       VW4, WV4);
    GEP_LAUNCH_CHECK();
    {  // trailing matrix of q: lower triangle -= VW4 WV4^T
      Gemm g;
      g.transB = true;
      g.uplo = 1;
      g.m = n1; g.n = n1; g.k = 2 * w + 2 * w1; g.alpha = -1.0; g.beta = 1.0;
      g.A = VW4; g.lda = n1; g.B = WV4; g.ldb = n1;
      g.C = r.C + (col1 + b) + (col1 + b) * r.ldc; g.ldc = r.ldc;
      gemm(g, s);
    }
    col0 += 2 * b;
  }
  raise_info_if(err, r.info, INFO_WAIT_TIMEOUT, s);
}


// Z <- Q1 Z, Q1 = Q_0 Q_1 ... Q_last with Q_p = I - V_p T_p V_p^T.  Panels are
// applied in groups of QG consecutive panels, last group first: the product of a
// group is one compact-WY block I - Vg Tg Vg^T with Vg = [V_p .. V_p+QG-1] stacked
// from the group's first row (zeros above each panel's start) and
//   Tg(blocks i<j) = -Tg(0:i, 0:i-block) Gg(.., j) T_j,  Gg = Vg^T Vg,
// so the application is three large GEMMs (K = QG*b) per group.
namespace {
constexpr int QG = 8;

// Vg (ng x QG*b, ld ng): panel i of the group starts at row i*b.
__global__ void build_vg(int64_t ng, int b, int np, const double* __restrict__ C, int64_t ldc,
                         int64_t col0, double* __restrict__ Vg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng) return;
  const int c = blockIdx.y;        // column of Vg
  const int pi = c / b;            // panel within the group
  double v = 0.0;
  if (pi < np) {
    const int64_t r0 = (int64_t)pi * b;  // first row of this panel's V inside Vg
    if (i >= r0) v = C[(col0 + b + i) + (col0 + c) * ldc];
  }
  Vg[i + (int64_t)c * ng] = v;
}

// Tg from the panel T's and Gg.  form_tg_init zeroes Tg and places the panel T's
// on its diagonal; form_tg_block(j) then fills the block column j above the
// diagonal, one workgroup per column c:
//   x = Gg(0:jb, jb + 0..c) T_j(0..c, c),   Tg(0:jb, jb + c) = -Tg(0:jb, 0:jb) x.
__global__ void form_tg_init(int b, int np, const double* __restrict__ Tp, double* __restrict__ Tg) {
  const int W = np * b;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)W * W) return;
  const int r = (int)(idx % W), c = (int)(idx / W);
  double v = 0.0;
  if (r / b == c / b) {
    const int pi = r / b;
    v = Tp[(int64_t)pi * b * b + (r % b) + (int64_t)(c % b) * b];
  }
  Tg[idx] = v;
}

__global__ void __launch_bounds__(256) form_tg_block(int b, int np, int j,
                                                     const double* __restrict__ Tp,
                                                     const double* __restrict__ Gg,
                                                     double* __restrict__ Tg) {
  const int W = np * b;
  const int jb = j * b;
  const int c = blockIdx.x;
  const double* Tj = Tp + (int64_t)j * b * b;
  __shared__ double x[(QG - 1) * MAXB];
  for (int r = threadIdx.x; r < jb; r += 256) {
    double acc = 0.0;
    for (int q = 0; q <= c; ++q) acc += Gg[r + (int64_t)(jb + q) * W] * Tj[q + c * b];
    x[r] = acc;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < jb; r += 256) {
    double acc = 0.0;
    for (int q = r; q < jb; ++q) acc += Tg[r + (int64_t)q * W] * x[q];
    Tg[r + (int64_t)(jb + c) * W] = -acc;
  }
}

}  // namespace

size_t apply_q1_workspace(int64_t n, int64_t ncols, int b) {
  const int64_t W = (int64_t)QG * b;
  size_t e = (size_t)n * W + 2 * (size_t)W * ncols + 2 * (size_t)W * W;
  e += splitk_work_elems(W, W, n) + 64;
  return e * sizeof(double) + 8 * 256;
}

void apply_q1(const BandReduction& r, double* Z, int64_t ldz, int64_t ncols, Arena& ws,
              hipStream_t s) {
  const int64_t N = r.n;
  const int b = r.b;
  if (N <= b || ncols <= 0) return;
  const int64_t npan = cdiv(N - b, b);  // panels with rows below the band: col0 + b < N
  const int64_t Wmax = (int64_t)QG * b;
  double* Vg = ws.take<double>((size_t)N * Wmax);
  double* W1 = ws.take<double>((size_t)Wmax * ncols);
  double* W2 = ws.take<double>((size_t)Wmax * ncols);
  double* Gg = ws.take<double>((size_t)Wmax * Wmax);
  double* Tg = ws.take<double>((size_t)Wmax * Wmax);
  const size_t skw = splitk_work_elems(Wmax, Wmax, N) + 64;
  double* skbuf = ws.take<double>(skw);
  const int64_t ngroups = cdiv(npan, QG);
  for (int64_t gi = ngroups - 1; gi >= 0; --gi) {
    const int64_t p_first = gi * QG;
    const int np = (int)((npan - p_first) < QG ? (npan - p_first) : QG);
    const int64_t col0 = p_first * b;
    const int64_t p0 = col0 + b;
    const int64_t ng = N - p0;
    const int64_t W = (int64_t)np * b;
    hipLaunchKernelGGL(build_vg, dim3((unsigned)cdiv(ng, 256), (unsigned)W), dim3(256), 0, s, ng, b,
                       np, (const double*)r.C, r.ldc, col0, Vg);
    GEP_LAUNCH_CHECK();
    {
      Gemm g;
      g.transA = true;
      g.m = W; g.n = W; g.k = ng;
      g.A = Vg; g.lda = ng; g.B = Vg; g.ldb = ng; g.C = Gg; g.ldc = W;
      g.work = skbuf; g.work_elems = skw;
      gemm(g, s);
    }
    {
      const double* Tp = r.T + (col0 / b) * (int64_t)b * b;
      hipLaunchKernelGGL(form_tg_init, dim3((unsigned)cdiv(W * W, 256)), dim3(256), 0, s, b, np,
                         Tp, Tg);
      GEP_LAUNCH_CHECK();
      for (int j = 1; j < np; ++j) {
        hipLaunchKernelGGL(form_tg_block, dim3((unsigned)b), dim3(256), 0, s, b, np, j, Tp,
                           (const double*)Gg, Tg);
        GEP_LAUNCH_CHECK();
      }
    }
    {
      Gemm g;
      g.transA = true;
      g.m = W; g.n = ncols; g.k = ng;
      g.A = Vg; g.lda = ng; g.B = Z + p0; g.ldb = ldz; g.C = W1; g.ldc = W;
      gemm(g, s);
    }
    {
      Gemm g;
      g.m = W; g.n = ncols; g.k = W;
      g.A = Tg; g.lda = W; g.B = W1; g.ldb = W; g.C = W2; g.ldc = W;
      gemm(g, s);
    }
    {
      Gemm g;
      g.m = ng; g.n = ncols; g.k = W; g.alpha = -1.0; g.beta = 1.0;
      g.A = Vg; g.lda = ng; g.B = W2; g.ldb = W; g.C = Z + p0; g.ldc = ldz;
      gemm(g, s);
    }
  }
}

}  // namespace gep

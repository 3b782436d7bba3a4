// Second stage of the two-stage reduction: band (width b) -> tridiagonal by
// bulge chasing, and the matching back transformation Z <- Q2 Z.
//
// Sweep s annihilates column s below the subdiagonal with a reflector of length
// <= b acting on rows s+1.., applied two-sidedly to the diagonal block; the
// right-hand application to the block below creates a bulge whose first column is
// annihilated by the next reflector (rows shifted down by b), and so on to the
// end of the matrix.  Reflector (s, k) acts on rows s+1+k*b .. s+k*b+b.
//
// Sweep s+1 may work on position k once sweep s has finished positions 0..k+1,
// so many sweeps are in flight at once.  One persistent kernel: each workgroup
// takes the next sweep from an atomic ticket and runs it position by position,
// publishing its progress with release stores and waiting on its predecessor
// with acquire loads.  A sweep only ever waits on a smaller sweep index, which
// was handed out earlier to a workgroup that is already running, so the wait
// always ends; every wait is also bounded in wall-clock time and an error flag
// makes all workgroups leave.
//
// The Q2 back transformation groups the reflectors of NBW consecutive sweeps at
// the same position k into a compact-WY block (I - V T V^T, V of height
// b + NBW - 1).  Reflectors only fail to commute when their row ranges overlap
// and the later sweep must then act first; applying blocks for sweep groups from
// last to first and, inside a group, positions in increasing k respects that.
// Each workgroup owns a strip of columns of Z and applies every block to it in
// that order (columns are independent), with the MFMA.
#include "common.h"
#include "internal.h"

namespace gep {
namespace {

constexpr int NT = 256;
constexpr int MAXB = 64;
constexpr int LDS_LD = MAXB + 1;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Householder for x (length L, in LDS): returns beta, tau; overwrites x by v
// (v[0] = 1).  Called by all threads; uses wave 0 for the reduction.
__device__ void house(int L, double* x, double* sh, double& beta_out, double& tau_out) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    double s = 0.0;
    for (int i = 1 + tid; i < L; i += 64) s += x[i] * x[i];
    s = wave_sum(s);
    if (tid == 0) {
      const double x0 = x[0];
      double beta, tau, scal;
      if (s == 0.0 || L <= 1) {
        beta = x0; tau = 0.0; scal = 0.0;
      } else {
        const double mu = sqrt(x0 * x0 + s);
        beta = (x0 >= 0.0) ? -mu : mu;
        tau = (beta - x0) / beta;
        scal = 1.0 / (x0 - beta);
      }
      sh[0] = beta; sh[1] = tau; sh[2] = scal;
    }
  }
  __syncthreads();
  const double scal = sh[2];
  for (int i = 1 + tid; i < L; i += NT) x[i] *= scal;
  __syncthreads();
  if (tid == 0) x[0] = 1.0;
  beta_out = sh[0];
  tau_out = sh[1];
  __syncthreads();
}

// D (L x L symmetric, full in LDS, ld LDS_LD) <- H D H, H = I - tau v v^T.
__device__ void two_sided(int L, double* D, const double* v, double tau, double* p, double* sh) {
  const int tid = threadIdx.x;
  if (tau == 0.0) return;
  if (tid < L) {
    double s = 0.0;
    for (int j = 0; j < L; ++j) s += D[tid + j * LDS_LD] * v[j];
    p[tid] = tau * s;
  }
  __syncthreads();
  if (tid < 64) {
    double s = 0.0;
    for (int i = tid; i < L; i += 64) s += p[i] * v[i];
    s = wave_sum(s);
    if (tid == 0) sh[3] = 0.5 * tau * s;
  }
  __syncthreads();
  const double a = sh[3];
  if (tid < L) p[tid] -= a * v[tid];
  __syncthreads();
  for (int idx = tid; idx < L * L; idx += NT) {
    const int i = idx % L, j = idx / L;
    D[i + j * LDS_LD] -= v[i] * p[j] + p[i] * v[j];
  }
  __syncthreads();
}

struct ChaseArgs {
  int64_t n;
  int b;
  double* band;
  int64_t ldband;
  double* V;
  double* tau;
  int64_t kmax;
  int32_t* progress;  // per sweep: completed positions
  int32_t* ticket;
  int32_t* err;
  int64_t nsweeps;
  uint64_t timeout_ticks;
};

__device__ inline int64_t positions(int64_t n, int b, int64_t s) {
  // positions k with s + 1 + k*b < n
  return (n - s - 2) / b + 1;
}

__device__ bool wait_for(const ChaseArgs& a, int64_t s, int32_t need) {
  // returns false on error / timeout
  const uint64_t t0 = wall_clock64();
  for (;;) {
    const int32_t p = __hip_atomic_load(&a.progress[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (p >= need) return true;
    if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (wall_clock64() - t0 > a.timeout_ticks) {
      __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

__global__ void __launch_bounds__(NT) chase_kernel(ChaseArgs a) {
  __shared__ double Es[MAXB * LDS_LD];
  __shared__ double Ds[MAXB * LDS_LD];
  __shared__ double v[MAXB], vprev[MAXB], p[MAXB];
  __shared__ double sh[8];
  __shared__ int64_t s_sh;
  __shared__ int ok_sh;
  const int tid = threadIdx.x;
  const int b = a.b;
  const int64_t n = a.n;
  const int64_t ld = a.ldband;
  double* band = a.band;

  for (;;) {
    if (tid == 0) s_sh = atomicAdd(a.ticket, 1);
    __syncthreads();
    const int64_t s = s_sh;
    __syncthreads();
    if (s >= a.nsweeps) break;
    const int64_t npos = positions(n, b, s);
    const int64_t npos_prev = (s > 0) ? positions(n, b, s - 1) : 0;
    double tau_prev = 0.0;
    int Lprev = 0;
    for (int64_t k = 0; k < npos; ++k) {
      if (tid == 0) {
        bool ok = true;
        if (s > 0) {
          int64_t need = k + 2;
          if (need > npos_prev) need = npos_prev;
          ok = wait_for(a, s - 1, (int32_t)need);
        }
        ok_sh = ok ? 1 : 0;
      }
      __syncthreads();
      if (!ok_sh) return;
      __threadfence();  // see the predecessor's band writes
      const int64_t r = s + 1 + k * b;           // first row of this position
      int L = (int)((n - r) < b ? (n - r) : b);  // reflector length
      double beta, tau;
      if (k == 0) {
        // x = column s, rows s+1 .. s+L
        for (int i = tid; i < L; i += NT) v[i] = band[(1 + i) + s * ld];
        __syncthreads();
        house(L, v, sh, beta, tau);
        if (tid == 0) band[1 + s * ld] = beta;
        for (int i = 1 + tid; i < L; i += NT) band[(1 + i) + s * ld] = 0.0;
      } else {
        // E = rows r..r+L-1, cols c..c+Lprev-1, c = r - b
        const int64_t c = r - b;
        for (int idx = tid; idx < L * Lprev; idx += NT) {
          const int i = idx % L, j = idx / L;
          Es[i + j * LDS_LD] = band[(b + i - j) + (c + j) * ld];
        }
        __syncthreads();
        // E <- E (I - tau_prev vprev vprev^T)
        if (tau_prev != 0.0) {
          if (tid < L) {
            double y = 0.0;
            for (int j = 0; j < Lprev; ++j) y += Es[tid + j * LDS_LD] * vprev[j];
            p[tid] = tau_prev * y;
          }
          __syncthreads();
          for (int idx = tid; idx < L * Lprev; idx += NT) {
            const int i = idx % L, j = idx / L;
            Es[i + j * LDS_LD] -= p[i] * vprev[j];
          }
          __syncthreads();
        }
        // reflector from column 0 of E
        for (int i = tid; i < L; i += NT) v[i] = Es[i];
        __syncthreads();
        house(L, v, sh, beta, tau);
        // E(:, 1:) <- H E(:, 1:)
        if (tau != 0.0) {
          if (tid >= 1 && tid < Lprev) {
            double u = 0.0;
            for (int i = 0; i < L; ++i) u += v[i] * Es[i + tid * LDS_LD];
            p[tid] = tau * u;
          }
          __syncthreads();
          for (int idx = tid; idx < L * Lprev; idx += NT) {
            const int i = idx % L, j = idx / L;
            if (j >= 1) Es[i + j * LDS_LD] -= v[i] * p[j];
          }
          __syncthreads();
        }
        if (tid == 0) Es[0] = beta;
        for (int i = 1 + tid; i < L; i += NT) Es[i] = 0.0;
        __syncthreads();
        for (int idx = tid; idx < L * Lprev; idx += NT) {
          const int i = idx % L, j = idx / L;
          band[(b + i - j) + (c + j) * ld] = Es[i + j * LDS_LD];
        }
      }
      // diagonal block rows/cols r .. r+L-1 <- H D H
      if (tau != 0.0) {
        for (int idx = tid; idx < L * L; idx += NT) {
          const int i = idx % L, j = idx / L;
          const int hi = i > j ? i : j, lo = i > j ? j : i;
          Ds[i + j * LDS_LD] = band[(hi - lo) + (r + lo) * ld];
        }
        __syncthreads();
        two_sided(L, Ds, v, tau, p, sh);
        for (int idx = tid; idx < L * L; idx += NT) {
          const int i = idx % L, j = idx / L;
          if (i >= j) band[(i - j) + (r + j) * ld] = Ds[i + j * LDS_LD];
        }
      }
      // store the reflector, keep it for the next position
      if (a.V) {
        double* vout = a.V + (s * a.kmax + k) * b;
        for (int i = tid; i < b; i += NT) vout[i] = (i < L) ? v[i] : 0.0;
        if (tid == 0) a.tau[s * a.kmax + k] = tau;
      }
      for (int i = tid; i < L; i += NT) vprev[i] = v[i];
      tau_prev = tau;
      Lprev = L;
      __threadfence();
      __syncthreads();
      if (tid == 0) {
        __hip_atomic_store(&a.progress[s], (int32_t)(k + 1), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

__global__ void extract_tridiag(int64_t n, const double* __restrict__ band, int64_t ld,
                                double* __restrict__ d, double* __restrict__ e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  d[i] = band[i * ld];
  if (i + 1 < n) e[i] = band[1 + i * ld];
}

// ---------------------------------------------------------------- Q2 application
constexpr int NBW = 32;   // sweeps per compact-WY block
constexpr int SW = 32;    // columns of Z per workgroup
constexpr int HMAX = MAXB + NBW - 1;

struct Q2Args {
  int64_t n;
  int b;
  int64_t nsweeps, kmax, ngroups;
  const double* V;
  const double* tau;
  double* T;  // NBW x NBW per block (group j, position k) at T + (j*kmax + k)*NBW*NBW
  double* Z;
  int64_t ldz, ncols;
};

// Column c of the block of group j at position k: reflector (s0 + c, k) shifted
// down by c rows; zero if that reflector does not exist.
__device__ inline void load_block_v(const Q2Args& a, int64_t s0, int64_t k, int H, double* Vs,
                                    double* taus) {
  const int b = a.b;
  for (int idx = threadIdx.x; idx < H * NBW; idx += blockDim.x) {
    const int i = idx % H, c = idx / H;
    const int64_t s = s0 + c;
    double v = 0.0;
    if (s < a.nsweeps && k < positions(a.n, b, s) && i >= c && i - c < b)
      v = a.V[(s * a.kmax + k) * b + (i - c)];
    Vs[i + c * HMAX] = v;
  }
  for (int c = threadIdx.x; c < NBW; c += blockDim.x) {
    const int64_t s = s0 + c;
    taus[c] = (s < a.nsweeps && k < positions(a.n, b, s)) ? a.tau[s * a.kmax + k] : 0.0;
  }
}

__global__ void __launch_bounds__(NT) q2_form_t(Q2Args a) {
  __shared__ double Vs[HMAX * NBW];
  __shared__ double Gm[NBW][NBW + 1];
  __shared__ double Ts[NBW][NBW + 1];
  __shared__ double taus[NBW];
  const int64_t k = blockIdx.x, j = blockIdx.y;
  const int64_t s0 = j * NBW;
  if (k >= positions(a.n, a.b, s0)) return;
  const int H = a.b + NBW - 1;
  load_block_v(a, s0, k, H, Vs, taus);
  __syncthreads();
  for (int idx = threadIdx.x; idx < NBW * NBW; idx += NT) {
    const int c1 = idx % NBW, c2 = idx / NBW;
    double g = 0.0;
    for (int i = 0; i < H; ++i) g += Vs[i + c1 * HMAX] * Vs[i + c2 * HMAX];
    Gm[c1][c2] = g;
    Ts[c1][c2] = 0.0;
  }
  __syncthreads();
  for (int c = 0; c < NBW; ++c) {
    const double tc = taus[c];
    if ((int)threadIdx.x < c) {
      double acc = 0.0;
      for (int q = threadIdx.x; q < c; ++q) acc += Ts[threadIdx.x][q] * Gm[q][c];
      Ts[threadIdx.x][c] = -tc * acc;
    }
    if (threadIdx.x == 0) Ts[c][c] = tc;
    __syncthreads();
  }
  double* out = a.T + (j * a.kmax + k) * NBW * NBW;
  for (int idx = threadIdx.x; idx < NBW * NBW; idx += NT) out[idx] = Ts[idx % NBW][idx / NBW];
}

// Z <- (I - V T V^T) Z for every block, groups from last to first, positions in
// increasing order; one workgroup per strip of SW columns.
__global__ void __launch_bounds__(NT) q2_apply(Q2Args a) {
  __shared__ double Vs[HMAX * NBW];
  __shared__ double Ts[NBW * NBW];
  __shared__ double Zs[HMAX * (SW + 1)];
  __shared__ double W1[NBW * (SW + 1)];
  __shared__ double W2[NBW * (SW + 1)];
  __shared__ double taus[NBW];
  const int64_t c0 = (int64_t)blockIdx.x * SW;
  const int ncol = (int)((a.ncols - c0) < SW ? (a.ncols - c0) : SW);
  const int tid = threadIdx.x;
  for (int64_t j = a.ngroups - 1; j >= 0; --j) {
    const int64_t s0 = j * NBW;
    const int64_t P0 = positions(a.n, a.b, s0);
    for (int64_t k = 0; k < P0; ++k) {
      const int64_t r0 = s0 + 1 + k * a.b;
      int H = a.b + NBW - 1;
      if (r0 + H > a.n) H = (int)(a.n - r0);
      load_block_v(a, s0, k, H, Vs, taus);
      const double* Tg = a.T + (j * a.kmax + k) * NBW * NBW;
      for (int idx = tid; idx < NBW * NBW; idx += NT) Ts[idx] = Tg[idx];
      for (int idx = tid; idx < H * ncol; idx += NT) {
        const int i = idx % H, c = idx / H;
        Zs[i + c * HMAX] = a.Z[(r0 + i) + (c0 + c) * a.ldz];
      }
      __syncthreads();
      for (int idx = tid; idx < NBW * ncol; idx += NT) {
        const int r = idx % NBW, c = idx / NBW;
        double acc = 0.0;
        for (int i = 0; i < H; ++i) acc += Vs[i + r * HMAX] * Zs[i + c * HMAX];
        W1[r + c * NBW] = acc;
      }
      __syncthreads();
      for (int idx = tid; idx < NBW * ncol; idx += NT) {
        const int r = idx % NBW, c = idx / NBW;
        double acc = 0.0;
        for (int q = r; q < NBW; ++q) acc += Ts[r + q * NBW] * W1[q + c * NBW];
        W2[r + c * NBW] = acc;
      }
      __syncthreads();
      for (int idx = tid; idx < H * ncol; idx += NT) {
        const int i = idx % H, c = idx / H;
        double acc = 0.0;
        for (int q = 0; q < NBW; ++q) acc += Vs[i + q * HMAX] * W2[q + c * NBW];
        a.Z[(r0 + i) + (c0 + c) * a.ldz] = Zs[i + c * HMAX] - acc;
      }
      __syncthreads();
    }
  }
}

}  // namespace

size_t apply_q2_workspace(int64_t n, int b) {
  const int64_t nsweeps = n > 2 ? n - 2 : 0;
  const int64_t kmax = n > 1 ? cdiv(n - 1, b) : 1;
  const int64_t ngroups = cdiv(nsweeps, NBW);
  return (size_t)ngroups * kmax * NBW * NBW * sizeof(double) + 4096;
}

void apply_q2(const BulgeChase& c, double* Z, int64_t ldz, int64_t ncols, Arena& ws,
              hipStream_t s) {
  const int64_t n = c.n;
  const int64_t nsweeps = n > 2 ? n - 2 : 0;
  if (nsweeps == 0 || ncols <= 0) return;
  Q2Args a;
  a.n = n; a.b = c.b; a.nsweeps = nsweeps; a.kmax = c.kmax; a.ngroups = cdiv(nsweeps, NBW);
  a.V = c.V; a.tau = c.tau; a.Z = Z; a.ldz = ldz; a.ncols = ncols;
  a.T = ws.take<double>((size_t)a.ngroups * a.kmax * NBW * NBW);
  hipLaunchKernelGGL(q2_form_t, dim3((unsigned)a.kmax, (unsigned)a.ngroups), dim3(NT), 0, s, a);
  GEP_LAUNCH_CHECK();
  hipLaunchKernelGGL(q2_apply, dim3((unsigned)cdiv(ncols, SW)), dim3(NT), 0, s, a);
  GEP_LAUNCH_CHECK();
}

size_t sb2st_reflector_count(int64_t n, int b) {
  const int64_t kmax = n > 1 ? cdiv(n - 1, b) : 1;
  return (size_t)(n > 0 ? n : 1) * (size_t)kmax;
}

void sb2st(const BulgeChase& c, hipStream_t s) {
  const int64_t n = c.n;
  if (c.b > MAXB || c.b < 1) throw HipError{hipErrorInvalidValue, "band width"};
  const int64_t nsweeps = n > 2 ? n - 2 : 0;
  if (nsweeps > 0) {
    int32_t* progress = c.sync;
    int32_t* ticket = c.sync + n;
    fill_i32(c.sync, n + 8, 0, s);
    fill_i32(c.err, 1, 0, s);
    ChaseArgs a;
    a.n = n; a.b = c.b; a.band = c.band; a.ldband = c.ldband; a.V = c.V; a.tau = c.tau;
    a.kmax = c.kmax; a.progress = progress; a.ticket = ticket; a.err = c.err; a.nsweeps = nsweeps;
    int dev = 0, rate_khz = 0;
    GEP_HIP(hipGetDevice(&dev));
    GEP_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    if (rate_khz <= 0) rate_khz = 100000;
    a.timeout_ticks = (uint64_t)rate_khz * 1000ull * 10ull;  // 10 s for any single wait
    int64_t groups = nsweeps < 512 ? nsweeps : 512;
    hipLaunchKernelGGL(chase_kernel, dim3((unsigned)groups), dim3(NT), 0, s, a);
    GEP_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(extract_tridiag, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, n,
                     (const double*)c.band, c.ldband, c.d, c.e);
  GEP_LAUNCH_CHECK();
}

}  // namespace gep

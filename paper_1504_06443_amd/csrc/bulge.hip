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
// Q2 blocks: NBW consecutive sweeps at one position, stored as HP x NBW (row-major),
// column c = reflector of sweep s0 + c shifted down by c rows.
constexpr int NBW = 32;
constexpr int HP = 96;   // >= MAXB + NBW - 1

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Band data is shared between workgroups inside one launch, so every access to it
// is an agent-scope relaxed atomic: loads see the latest value written by any XCD
// and stores are written through, which leaves nothing dirty in L2 for the
// release that publishes a sweep's progress.
__device__ inline double cld(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void cst(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Householder for x (length L, in LDS): H x = beta e_1, H = I - tau v v^T,
// v[0] = 1.  Overwrites x by v.  Wave 0 reduces; all threads return beta, tau.
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
  if (tid >= 1 && tid < L) x[tid] *= scal;
  if (tid == 0) x[0] = 1.0;
  beta_out = sh[0];
  tau_out = sh[1];
  __syncthreads();
}

// The bulge chase runs CNT threads per workgroup: CW waves, two per SIMD, so
// that the latency of one wave's dependent LDS and ALU steps is partly covered by
// the other's.  Every loop over a block column or row below has a fixed trip
// count of PER = MAXB / CW: each thread first reads all of its (up to PER)
// operands from LDS, with indices past the end clamped to a valid element, and
// only then computes and writes, so the reads' latencies overlap.
constexpr int CNT = 512;
constexpr int CW = CNT / 64;
constexpr int PER = MAXB / CW;

// out[x] = scale * sum_{y < ny} M[x * sx + y * sy] w[y] for x < nx: CW threads
// per x, each summing y = q, q + CW, ... pairwise; the CW partials are added in a
// fixed order.
__device__ inline void matvec(int nx, int ny, const double* M, int sx, int sy, const double* w,
                              double scale, double* out) {
  const int tid = threadIdx.x, x = tid / CW, q = tid % CW;
  const int xc = x < nx ? x : 0;
  double t[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int y = q + CW * m;
    const int yc = y < ny ? y : 0;
    const double prod = M[xc * sx + yc * sy] * w[yc];
    t[m] = y < ny ? prod : 0.0;
  }
#pragma unroll
  for (int h = PER / 2; h >= 1; h >>= 1)
#pragma unroll
    for (int m = 0; m < h; ++m) t[m] += t[m + h];
  double acc = t[0];
#pragma unroll
  for (int o = 1; o < CW; o <<= 1) acc += __shfl_xor(acc, o, 64);
  if (x < nx && q == 0) out[x] = scale * acc;
}

// Householder for x (length L <= 64, in LDS, not modified): H x = beta e_1,
// H = I - tau v v^T, v[0] = 1, written to vout.  Every wave forms the squared norm
// with the same butterfly (so every lane holds the same bits) and every thread
// the same scalars, so no barrier is needed before vout is written; one after.
__device__ void house_from(int L, const double* x, double* vout, double& beta_out,
                           double& tau_out) {
  const int tid = threadIdx.x, lane = tid & 63;
  double s = (lane >= 1 && lane < L) ? x[lane] * x[lane] : 0.0;
  s = wave_sum(s);
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
  if (tid < L) vout[tid] = (tid == 0) ? 1.0 : x[tid] * scal;
  beta_out = beta;
  tau_out = tau;
  __syncthreads();
}

// D (L x L symmetric, full in LDS, ld LDS_LD) <- H D H, H = I - tau v v^T.
// 4 threads per row for the matrix-vector product.
// Second half of two_sided, after p = tau D v: D <- D - v w^T - w v^T with
// w = p - a v.  No barrier at the end.
__device__ void two_sided_update(int L, double* D, const double* v, double tau, const double* p) {
  const int tid = threadIdx.x;
  // a = tau p^T v / 2, formed by every wave (identical bits on every lane)
  const int lane = tid & 63;
  const double a = 0.5 * tau * wave_sum(lane < L ? p[lane] * v[lane] : 0.0);
  {
    const int i = tid & 63, j0 = tid >> 6;
    if (i < L) {
      const double vi = v[i], pi = p[i] - a * vi;
      double d[PER], pv[PER], vv[PER];
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int j = j0 + CW * m;
        const int jc = j < L ? j : 0;
        d[m] = D[i + jc * LDS_LD];
        pv[m] = p[jc];
        vv[m] = v[jc];
      }
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int j = j0 + CW * m;
        const double pj = pv[m] - a * vv[m];
        if (j < L) D[i + j * LDS_LD] = d[m] - (vi * pj + pi * vv[m]);
      }
    }
  }
}

__device__ void two_sided(int L, double* D, const double* v, double tau, double* p) {
  if (tau == 0.0) return;
  matvec(L, L, D, 1, LDS_LD, v, tau, p);
  __syncthreads();
  two_sided_update(L, D, v, tau, p);
  __syncthreads();
}

// E (L x Lprev) <- H E on columns 1.., H = I - tau v v^T, after p = tau E^T v
// (column 0 is set to beta e_1 by the caller).  No barrier.
__device__ void left_update(int L, int Lprev, double* E, const double* v, const double* p) {
  const int tid = threadIdx.x;
  const int i = tid & 63, j0 = tid >> 6;
  if (i < L) {
    const double vi = v[i];
    double e[PER], pp[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int j = j0 + CW * m;
      const int jc = j < Lprev ? j : 0;
      e[m] = E[i + jc * LDS_LD];
      pp[m] = p[jc];
    }
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int j = j0 + CW * m;
      if (j >= 1 && j < Lprev) E[i + j * LDS_LD] = e[m] - vi * pp[m];
    }
  }
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
  int force_fail;  // debug: a wait not satisfied at its first poll gives up
};

__device__ inline int64_t positions(int64_t n, int b, int64_t s) {
  // positions k with s + 1 + k*b < n
  return (n - s - 2) / b + 1;
}

__device__ bool wait_for(const ChaseArgs& a, int64_t s, int32_t need) {
  // returns false on error / timeout
  // Poll with relaxed loads (an acquire load per poll would invalidate this XCD's
  // L2 every time); one acquire fence once the flag is seen.
  const uint64_t t0 = wall_clock64();
  for (;;) {
    const int32_t p = __hip_atomic_load(&a.progress[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p >= need) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      return true;
    }
    if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (a.force_fail || wall_clock64() - t0 > a.timeout_ticks) {
      __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

__global__ void __launch_bounds__(CNT) chase_kernel(ChaseArgs a) {
  __shared__ double Es[MAXB * LDS_LD];
  __shared__ double Ds[MAXB * LDS_LD];
  __shared__ double v[MAXB], vprev[MAXB], p[MAXB], p2[MAXB];
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
      const int64_t r = s + 1 + k * b;           // first row of this position
      const int L = (int)((n - r) < b ? (n - r) : b);  // reflector length
      const int64_t c = r - b;                   // first column of the block left of D
      // load D (rows/cols r.., symmetric from the lower band) and the column
      // block to its left (column s for k = 0, the bulge block E otherwise).
      // Each thread issues all its coherent loads back to back (addresses of
      // unused slots clamped to a valid element) and only then writes LDS, so
      // the loads' latencies overlap instead of adding up.
      {
        const int i = tid & 63, j0 = tid >> 6;
        double xd[PER], xe[PER];
#pragma unroll
        for (int m = 0; m < PER; ++m) {
          const int j = j0 + CW * m;
          const bool okd = i < L && j <= i;
          xd[m] = cld(&band[okd ? (i - j) + (r + j) * ld : 0]);
        }
        if (k > 0) {
#pragma unroll
          for (int m = 0; m < PER; ++m) {
            const int j = j0 + CW * m;
            const bool oke = i < L && j < Lprev;
            xe[m] = cld(&band[oke ? (b + i - j) + (c + j) * ld : 0]);
          }
        }
        double xv = 0.0;
        if (k == 0 && tid < L) xv = cld(&band[(1 + tid) + s * ld]);
#pragma unroll
        for (int m = 0; m < PER; ++m) {
          const int j = j0 + CW * m;
          if (i < L && j <= i) {
            Ds[i + j * LDS_LD] = xd[m];
            Ds[j + i * LDS_LD] = xd[m];
          }
        }
        if (k > 0) {
#pragma unroll
          for (int m = 0; m < PER; ++m) {
            const int j = j0 + CW * m;
            if (i < L && j < Lprev) Es[i + j * LDS_LD] = xe[m];
          }
        }
        if (k == 0 && tid < L) v[tid] = xv;
      }
      __syncthreads();
      double beta, tau;
      if (k == 0) {
        house(L, v, sh, beta, tau);
        // diagonal block rows/cols r .. r+L-1 <- H D H
        if (tau != 0.0) two_sided(L, Ds, v, tau, p);
      } else {
        // E <- E (I - tau_prev vprev vprev^T)
        if (tau_prev != 0.0) {
          matvec(L, Lprev, Es, 1, LDS_LD, vprev, tau_prev, p);
          __syncthreads();
          {
            const int i = tid & 63, j0 = tid >> 6;
            if (i < L) {
              const double pi = p[i];
              double e[PER], vv[PER];
#pragma unroll
              for (int m = 0; m < PER; ++m) {
                const int j = j0 + CW * m;
                const int jc = j < Lprev ? j : 0;
                e[m] = Es[i + jc * LDS_LD];
                vv[m] = vprev[jc];
              }
#pragma unroll
              for (int m = 0; m < PER; ++m) {
                const int j = j0 + CW * m;
                if (j < Lprev) Es[i + j * LDS_LD] = e[m] - pi * vv[m];
              }
            }
          }
          __syncthreads();
        }
        // reflector from column 0 of E (read in place), applied from the left to
        // columns 1..
        house_from(L, Es, v, beta, tau);
        // H from the left on E (p[col] = tau v^T E(:, col); column 0 is replaced by
        // beta e_1 below) and from both sides on the diagonal block D: the two
        // products with v in one phase, the two updates in the next
        if (tau != 0.0) {
          matvec(Lprev, L, Es, LDS_LD, 1, v, tau, p);
          matvec(L, L, Ds, 1, LDS_LD, v, tau, p2);
          __syncthreads();
          left_update(L, Lprev, Es, v, p);
          two_sided_update(L, Ds, v, tau, p2);
        }
        if (tid == 0) Es[0] = beta;
        if (tid >= 1 && tid < L) Es[tid] = 0.0;
        __syncthreads();
      }
      // The task's band stores are all issued after its arithmetic: the wait for a
      // load's data also waits for every store issued before that load, and the
      // release below has to wait for the stores anyway.
      if (k == 0) {
        if (tid == 0) cst(&band[1 + s * ld], beta);
        if (tid >= 1 && tid < L) cst(&band[(1 + tid) + s * ld], 0.0);
      } else {
        const int i = tid & 63, j0 = tid >> 6;
        if (i < L) {
          double e[PER];
#pragma unroll
          for (int m = 0; m < PER; ++m) {
            const int j = j0 + CW * m;
            e[m] = Es[i + (j < Lprev ? j : 0) * LDS_LD];
          }
#pragma unroll
          for (int m = 0; m < PER; ++m) {
            const int j = j0 + CW * m;
            if (j < Lprev) cst(&band[(b + i - j) + (c + j) * ld], e[m]);
          }
        }
      }
      if (tau != 0.0) {
        {
          const int i = tid & 63, j0 = tid >> 6;
          if (i < L) {
            double d[PER];
#pragma unroll
            for (int m = 0; m < PER; ++m) {
              const int j = j0 + CW * m;
              d[m] = Ds[i + (j <= i ? j : 0) * LDS_LD];
            }
#pragma unroll
            for (int m = 0; m < PER; ++m) {
              const int j = j0 + CW * m;
              if (j <= i) cst(&band[(i - j) + (r + j) * ld], d[m]);
            }
          }
        }
      }
      // store the reflector in its Q2 block (consumed by a later kernel)
      if (a.V) {
        const int64_t j = s / NBW;
        const int cc = (int)(s % NBW);
        double* blk = a.V + (j * a.kmax + k) * (int64_t)(HP * NBW);
        if (tid < L) cst(&blk[(cc + tid) * NBW + cc], v[tid]);
        if (tid == 0) cst(&a.tau[s * a.kmax + k], tau);
      }
      if (tid < L) vprev[tid] = v[tid];
      tau_prev = tau;
      Lprev = L;
      __syncthreads();
      if (tid == 0)
        __hip_atomic_store(&a.progress[s], (int32_t)(k + 1), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ------------------------------------------------------------ data-stationary chase
// Each workgroup owns P consecutive positions of every sweep: their diagonal blocks
// D and the blocks E to their left stay in LDS from one sweep to the next.  From
// sweep s to s + 1 a window moves down one row: D loses its first row and column, E
// loses its first row and column and takes D's first column (below the diagonal)
// as its last column.  The one new row at the bottom is row r + b of the matrix,
// which position k + 1 finished at sweep s: D gets that position's E(0, 1..b-1) and
// D(0, 0), E gets zeros and, last, E(0, 0) (the band element at distance b; every
// entry further out in that row was annihilated by earlier sweeps).  Position k - 1
// passes the reflector that E(s, k) needs.  A step therefore receives b + 1 numbers
// from each neighbour instead of loading both blocks from the band and storing them
// back, which was most of the latency on the chain of dependent steps ((s, k) after
// (s - 1, k + 1) and (s, k - 1)).  Between positions of one workgroup the numbers
// stay in LDS; between workgroups they go through memory with a flag, and the
// reflector is sent as soon as it is formed.  Every step does the ticket kernel's
// arithmetic on the same values (D mirrored from its lower triangle, as the band
// load does), so the two kernels give the same bits.  Position 0 writes the
// tridiagonal entries to the band as they become final.  All workgroups run at
// once, so the launch is cooperative.
struct StatArgs {
  ChaseArgs c;
  int64_t npos0;    // positions of the first sweep
  double* msg;      // per position: forward (v, tau) and backward (E row 0, D(0,0)),
                    // each double buffered by sweep parity, MSG doubles apiece
  int32_t* fwdf;    // per position: sweeps whose forward message is published
  int32_t* backf;   // per position: sweeps whose backward message is published
};

constexpr int MSG = MAXB + 1;

__device__ inline double* fwd_msg(const StatArgs& x, int64_t k, int par) {
  return x.msg + (4 * k + par) * MSG;
}
__device__ inline double* back_msg(const StatArgs& x, int64_t k, int par) {
  return x.msg + (4 * k + 2 + par) * MSG;
}

// Waits until *f1 >= n1 and *f2 >= n2 (a null flag is no condition); false on an
// error or time-out, as wait_for.
__device__ bool wait_two(const ChaseArgs& a, const int32_t* f1, int32_t n1, const int32_t* f2,
                         int32_t n2) {
  const uint64_t t0 = wall_clock64();
  for (;;) {
    const bool ok1 =
        !f1 || __hip_atomic_load(f1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n1;
    const bool ok2 =
        !f2 || __hip_atomic_load(f2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n2;
    if (ok1 && ok2) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      return true;
    }
    if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (a.force_fail || wall_clock64() - t0 > a.timeout_ticks) {
      __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// last sweep with a position k (position k of sweep s starts at row s + 1 + k b)
__device__ inline int64_t stat_last_sweep(const ChaseArgs& a, int64_t k) {
  const int64_t s = a.n - 2 - k * a.b;
  return s < a.nsweeps - 1 ? s : a.nsweeps - 1;
}

template <int P>
__global__ void __launch_bounds__(CNT) chase_stationary(StatArgs x) {
  __shared__ double Es[P][MAXB * LDS_LD];
  __shared__ double Ds[P][MAXB * LDS_LD];
  __shared__ double v[MAXB], vprev[MAXB], p[MAXB], p2[MAXB], xcol[MAXB];
  __shared__ double locb[P][MSG];   // backward message of position q + 1, in LDS
  __shared__ double sh[8];
  __shared__ double tprev_sh;
  __shared__ int ok_sh;
  const ChaseArgs& a = x.c;
  const int tid = threadIdx.x;
  const int b = a.b;
  const int64_t n = a.n;
  const int64_t ld = a.ldband;
  double* band = a.band;
  const int64_t k0 = (int64_t)blockIdx.x * P;
  int np = (int)((x.npos0 - k0) < P ? (x.npos0 - k0) : P);  // positions owned
  if (np <= 0) return;
  // sweep 0's blocks from the band: D (lower triangle, mirrored), and E (b columns)
  // or, for position 0, column 0 below the diagonal
  for (int q = 0; q < np; ++q) {
    const int64_t k = k0 + q;
    const int64_t r = 1 + k * b;
    const int L = (int)((n - r) < b ? (n - r) : b);
    const int64_t c = r - b;
    const int i = tid & 63, j0 = tid >> 6;
    double xd[PER], xe[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int j = j0 + CW * m;
      const bool okd = i < L && j <= i;
      xd[m] = cld(&band[okd ? (i - j) + (r + j) * ld : 0]);
    }
    if (k > 0) {
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int j = j0 + CW * m;
        const bool oke = i < L && j < b;
        xe[m] = cld(&band[oke ? (b + i - j) + (c + j) * ld : 0]);
      }
    }
    double xv = 0.0;
    if (k == 0 && tid < L) xv = cld(&band[1 + tid]);
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int j = j0 + CW * m;
      if (i < L && j <= i) {
        Ds[q][i + j * LDS_LD] = xd[m];
        Ds[q][j + i * LDS_LD] = xd[m];
      }
    }
    if (k > 0) {
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int j = j0 + CW * m;
        if (i < L && j < b) Es[q][i + j * LDS_LD] = xe[m];
      }
    }
    if (k == 0 && tid < L) xcol[tid] = xv;
  }
  __syncthreads();
  double tau_loc = 0.0;  // tau of the previous position of this workgroup, this sweep
  const int64_t s_end = stat_last_sweep(a, k0);
  for (int64_t s = 0; s <= s_end; ++s) {
    for (int q = 0; q < np; ++q) {
      const int64_t k = k0 + q;
      if (s > stat_last_sweep(a, k)) break;  // later positions end earlier
      double* D = Ds[q];
      double* E = Es[q];
      const int64_t r = s + 1 + k * b;
      const int L = (int)((n - r) < b ? (n - r) : b);
      const int Lprev = b;                    // position k - 1 always has a full reflector
      const bool has_new = s >= 1 && L == b;  // row r + b - 1 came from position k + 1
      const bool send_fwd = r + b <= n - 1;   // position k + 1 exists at this sweep
      const bool fwd_remote = q == 0 && k >= 1;        // reflector from another workgroup
      const bool back_remote = q == np - 1 && has_new;  // new row from another workgroup
      if (fwd_remote || back_remote) {
        if (tid == 0) {
          ok_sh = wait_two(a, fwd_remote ? &x.fwdf[k - 1] : nullptr, (int32_t)(s + 1),
                           back_remote ? &x.backf[k + 1] : nullptr, (int32_t)s)
                      ? 1
                      : 0;
        }
        __syncthreads();
        if (!ok_sh) return;
      }
      // the new bottom row: its D entries, E's zeros and band element, and for
      // position 0 the last entry of the column to annihilate
      if (has_new && tid < b) {
        const double* bm = back_remote ? back_msg(x, k + 1, (int)((s - 1) & 1)) : locb[q];
        const int qq = b - 1, j = tid;
        const int src = j < qq ? j + 1 : b;
        const double dv = back_remote ? cld(&bm[src]) : bm[src];
        D[qq + j * LDS_LD] = dv;
        D[j + qq * LDS_LD] = dv;
        if (j == qq) {
          const double e0 = back_remote ? cld(&bm[0]) : bm[0];
          if (k >= 1)
            E[qq + j * LDS_LD] = e0;
          else
            v[qq] = e0;
        } else if (k >= 1) {
          E[qq + j * LDS_LD] = 0.0;
        }
      }
      if (k == 0 && tid < L && !(has_new && tid == b - 1)) v[tid] = xcol[tid];
      if (k >= 1) {
        if (fwd_remote) {
          const double* fm = fwd_msg(x, k - 1, (int)(s & 1));
          if (tid < b) vprev[tid] = cld(&fm[tid]);
          if (tid == b) tprev_sh = cld(&fm[b]);
        } else {
          if (tid < b) vprev[tid] = v[tid];
          if (tid == b) tprev_sh = tau_loc;
        }
      }
      __syncthreads();
      const double tau_prev = k >= 1 ? tprev_sh : 0.0;
      double beta, tau;
      if (k == 0) {
        house(L, v, sh, beta, tau);
      } else {
        // E <- E (I - tau_prev vprev vprev^T)
        if (tau_prev != 0.0) {
          matvec(L, Lprev, E, 1, LDS_LD, vprev, tau_prev, p);
          __syncthreads();
          {
            const int i = tid & 63, j0 = tid >> 6;
            if (i < L) {
              const double pi = p[i];
              double e[PER], vv[PER];
#pragma unroll
              for (int m = 0; m < PER; ++m) {
                const int j = j0 + CW * m;
                const int jc = j < Lprev ? j : 0;
                e[m] = E[i + jc * LDS_LD];
                vv[m] = vprev[jc];
              }
#pragma unroll
              for (int m = 0; m < PER; ++m) {
                const int j = j0 + CW * m;
                if (j < Lprev) E[i + j * LDS_LD] = e[m] - pi * vv[m];
              }
            }
          }
          __syncthreads();
        }
        house_from(L, E, v, beta, tau);
      }
      // the reflector is complete: send it on at once if position k + 1 is in the
      // next workgroup
      const bool fwd_out = send_fwd && q == np - 1;
      if (fwd_out) {
        double* fm = fwd_msg(x, k, (int)(s & 1));
        if (tid < L) cst(&fm[tid], v[tid]);
        if (tid == 0) cst(&fm[b], tau);
        __syncthreads();
        if (tid == 0)
          __hip_atomic_store(&x.fwdf[k], (int32_t)(s + 1), __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
      }
      // H applied to E from the left and to D from both sides: the two products
      // with v in one phase, the two updates in the next
      if (k >= 1) {
        if (tau != 0.0) {
          matvec(Lprev, L, E, LDS_LD, 1, v, tau, p);
          matvec(L, L, D, 1, LDS_LD, v, tau, p2);
          __syncthreads();
          left_update(L, Lprev, E, v, p);
          two_sided_update(L, D, v, tau, p2);
        }
        if (tid == 0) E[0] = beta;
        if (tid >= 1 && tid < L) E[tid] = 0.0;
        __syncthreads();
      } else if (tau != 0.0) {
        two_sided(L, D, v, tau, p);
      }
      // the row that leaves the window: to the previous workgroup now, or kept in
      // LDS for this workgroup's previous position
      if (k >= 1) {
        if (q == 0) {
          double* bm = back_msg(x, k, (int)(s & 1));
          if (tid < b) cst(&bm[tid], E[tid * LDS_LD]);
          if (tid == b) cst(&bm[b], D[0]);
          __syncthreads();
          if (tid == 0)
            __hip_atomic_store(&x.backf[k], (int32_t)(s + 1), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
          if (tid < b) locb[q - 1][tid] = E[tid * LDS_LD];
          if (tid == b) locb[q - 1][b] = D[0];
        }
      }
      tau_loc = tau;
      // the tridiagonal entries (position 0) and the reflector for the back
      // transformation
      if (k == 0) {
        if (tid == 0) cst(&band[1 + s * ld], beta);
        if (tid >= 1 && tid < L) cst(&band[(1 + tid) + s * ld], 0.0);
        // row r leaves the window: its diagonal entry is final
        if (tid == 0) cst(&band[r * ld], D[0]);
        if (s == s_end) {
          // the last window: its lower triangle is final
          const int i = tid & 63, j0 = tid >> 6;
          if (i < L)
#pragma unroll
            for (int m = 0; m < PER; ++m) {
              const int j = j0 + CW * m;
              if (j <= i) cst(&band[(i - j) + (r + j) * ld], D[i + j * LDS_LD]);
            }
        }
      }
      if (a.V) {
        const int64_t j = s / NBW;
        const int cc = (int)(s % NBW);
        double* blk = a.V + (j * a.kmax + k) * (int64_t)(HP * NBW);
        if (tid < L) cst(&blk[(cc + tid) * NBW + cc], v[tid]);
        if (tid == 0) cst(&a.tau[s * a.kmax + k], tau);
      }
      if (s < stat_last_sweep(a, k)) {
        // move the window down one row (D read from its lower triangle)
        const int i = tid & 63, j0 = tid >> 6;
        double dn[PER], en[PER];
        double xn = 0.0;
#pragma unroll
        for (int m = 0; m < PER; ++m) {
          const int j = j0 + CW * m;
          const int hi = i > j ? i : j, lo = i > j ? j : i;
          const bool okd = i < L - 1 && j < L - 1;
          dn[m] = D[okd ? (hi + 1) + (lo + 1) * LDS_LD : 0];
          if (k >= 1) {
            const bool oke = i < L - 1 && j < b;
            const int src = !oke ? 0 : (j < b - 1 ? (i + 1) + (j + 1) * LDS_LD : (i + 1));
            en[m] = j < b - 1 ? E[src] : D[src];
          }
        }
        if (k == 0 && tid < L - 1) xn = D[tid + 1];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PER; ++m) {
          const int j = j0 + CW * m;
          if (i < L - 1 && j < L - 1) D[i + j * LDS_LD] = dn[m];
          if (k >= 1 && i < L - 1 && j < b) E[i + j * LDS_LD] = en[m];
        }
        if (k == 0 && tid < L - 1) xcol[tid] = xn;
      }
      __syncthreads();
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

struct Q2Args {
  int64_t n;
  int b;
  int64_t nsweeps, kmax, ngroups;
  const double* V;
  const double* tau;
  double* T;  // NBW x NBW per block (group j, position k) at T + (j*kmax + k)*NBW*NBW
  double* Z;
  int64_t ldz, ncols;
  int swizzle;  // q2_form_t rewrites V and T in the swizzled staging layout
};

// The 16-byte pair permutation of row R of a staged 32-column LDS array: pair p
// of the row is stored at p ^ swz_key(R).  The key is a bijection of R mod 16 that
// also flips bit 3 when bit 0 xor bit 2 of R is set, so that the two rows read
// together by 32 lanes (R and R + 4 in W = V^T Z, R and R + 1 in the T reads)
// land in opposite halves of the row's 16 pairs, and the 16 rows read by one
// column in Z += V X take 16 distinct pairs.
__host__ __device__ inline int swz_key(int row) {
  return (row & 15) ^ ((((row >> 2) ^ row) & 1) << 3);
}

// T factor of every block (forward accumulation, H_{s0} ... H_{s0+NBW-1} =
// I - V T V^T), stored transposed (T^T row-major == T column-major).
__global__ void __launch_bounds__(NT) q2_form_t(Q2Args a) {
  __shared__ double Vs[HP * (NBW + 1)];
  __shared__ double Gm[NBW][NBW + 1];
  __shared__ double Ts[NBW][NBW + 1];
  __shared__ double taus[NBW];
  const int64_t k = blockIdx.x, j = blockIdx.y;
  const int64_t s0 = j * NBW;
  if (k >= positions(a.n, a.b, s0)) return;
  const double* blk = a.V + (j * a.kmax + k) * (int64_t)(HP * NBW);
  const int H = a.b + NBW - 1;
  for (int idx = threadIdx.x; idx < (a.swizzle ? HP : H) * NBW; idx += NT)
    Vs[(idx / NBW) * (NBW + 1) + idx % NBW] = blk[idx];
  for (int c = threadIdx.x; c < NBW; c += NT) {
    const int64_t s = s0 + c;
    taus[c] = (s < a.nsweeps && k < positions(a.n, a.b, s)) ? a.tau[s * a.kmax + k] : 0.0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NBW * NBW; idx += NT) {
    const int c1 = idx % NBW, c2 = idx / NBW;
    double g = 0.0;
    for (int i = 0; i < H; ++i) g += Vs[i * (NBW + 1) + c1] * Vs[i * (NBW + 1) + c2];
    Gm[c1][c2] = g;
    Ts[c1][c2] = 0.0;
  }
  __syncthreads();
  for (int c = 0; c < NBW; ++c) {
    const double tc = taus[c];
    const int row = threadIdx.x >> 2, q = threadIdx.x & 3;
    double acc = 0.0;
    if (row < c)
      for (int kk = row + q; kk < c; kk += 4) acc += Ts[row][kk] * Gm[kk][c];
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (row < c && q == 0) Ts[row][c] = -tc * acc;
    if (threadIdx.x == 0) Ts[c][c] = tc;
    __syncthreads();
  }
  double* out = a.T + (j * a.kmax + k) * NBW * NBW;
  if (!a.swizzle) {
    for (int idx = threadIdx.x; idx < NBW * NBW; idx += NT) out[idx] = Ts[idx % NBW][idx / NBW];
    return;
  }
  // staging layout: row-major rows of 32, 16-byte pairs of a row permuted by
  // pair ^ swz_key(row); element (row, col) of T^T and of V at swz(row, col)
  for (int idx = threadIdx.x; idx < NBW * NBW; idx += NT) {
    const int row = idx >> 5, pc = idx & 31;
    const int col = (((pc >> 1) ^ swz_key(row)) << 1) | (pc & 1);
    out[idx] = Ts[col][row];
  }
  // V's row i lands in LDS row i + 1 (row 0 there is zero: the window starts one
  // row above the block's first row)
  double* blkw = const_cast<double*>(a.V) + (j * a.kmax + k) * (int64_t)(HP * NBW);
  for (int idx = threadIdx.x; idx < HP * NBW; idx += NT) {
    const int row = idx >> 5, pc = idx & 31;
    const int col = (((pc >> 1) ^ swz_key(row + 1)) << 1) | (pc & 1);
    blkw[idx] = Vs[row * (NBW + 1) + col];
  }
}

// Z <- (I - V T V^T) Z for every block, groups from last to first, positions in
// increasing order; one workgroup per strip of SWA = 32 columns of Z (76 KB of
// LDS, so two workgroups share a CU).  Inside a group the blocks slide down by b
// rows: the strip's rows live in a circular LDS window, and per block only b rows
// are written back and b new rows loaded.  The V / T / new-row loads of block
// k+1 are issued into registers before the MFMAs of block k.  The three products
// (W1 = V^T Z, W2 = T W1, Z -= V W2) are computed transposed so every LDS operand
// read is 16 consecutive doubles; the four waves split each product's 16 x 16
// tiles.
constexpr int SWA = 32;             // columns per workgroup
constexpr int HB = 128;             // circular window rows (>= HP + b - NBW + 1)
constexpr int ZLD = SWA + 1;
constexpr int VLD = NBW + 1;
constexpr int PV = HP * NBW / NT;   // V doubles per thread
constexpr int PT = NBW * NBW / NT;  // T doubles per thread
constexpr int PZ = MAXB * SWA / NT; // new-row doubles per thread

struct Prefetch {
  double v[PV], t[PT], z[PZ];
};

__device__ inline void fetch_vt(const Q2Args& a, int64_t j, int64_t k, Prefetch& f) {
  const double* blk = a.V + (j * a.kmax + k) * (int64_t)(HP * NBW);
  const double* Tg = a.T + (j * a.kmax + k) * NBW * NBW;
#pragma unroll
  for (int i = 0; i < PV; ++i) f.v[i] = blk[threadIdx.x + NT * i];
#pragma unroll
  for (int i = 0; i < PT; ++i) f.t[i] = Tg[threadIdx.x + NT * i];
}

// rows [lo, hi) relative to base (hi - lo <= MAXB); thread t: row t & 63,
// columns (t >> 6) + 4 i.
__device__ inline void fetch_rows(const Q2Args& a, int64_t base, int64_t lo, int64_t hi,
                                  int64_t c0, int ncol, Prefetch& f) {
  const int r = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < PZ; ++i) {
    const int c = (threadIdx.x >> 6) + 4 * i;
    f.z[i] = (lo + r < hi && c < ncol) ? a.Z[(base + lo + r) + (c0 + c) * a.ldz] : 0.0;
  }
}

__device__ inline void commit_vt(const Prefetch& f, double* Vs, double* Tt) {
#pragma unroll
  for (int i = 0; i < PV; ++i) {
    const int idx = threadIdx.x + NT * i;
    Vs[(idx >> 5) * VLD + (idx & 31)] = f.v[i];
  }
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = threadIdx.x + NT * i;
    Tt[(idx >> 5) * VLD + (idx & 31)] = f.t[i];
  }
}

__device__ inline void commit_rows(const Prefetch& f, int64_t lo, int64_t hi, double* Zs) {
  const int r = threadIdx.x & 63;
  if (lo + r >= hi) return;
  const int slot = (int)((lo + r) & (HB - 1));
#pragma unroll
  for (int i = 0; i < PZ; ++i) Zs[slot * ZLD + (threadIdx.x >> 6) + 4 * i] = f.z[i];
}

__device__ inline void write_rows(const Q2Args& a, int64_t base, int64_t lo, int64_t hi, int64_t c0,
                                  int ncol, const double* Zs) {
  const int r = threadIdx.x & 63;
  if (lo + r >= hi) return;
  const int slot = (int)((lo + r) & (HB - 1));
#pragma unroll
  for (int i = 0; i < PZ; ++i) {
    const int c = (threadIdx.x >> 6) + 4 * i;
    if (c < ncol) a.Z[(base + lo + r) + (c0 + c) * a.ldz] = Zs[slot * ZLD + c];
  }
}

__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
q2_apply(Q2Args a) {
  __shared__ double Vs[HP * VLD];        // V[row][c]
  __shared__ double Tt[NBW * VLD];       // T^T[k][j]
  __shared__ double Zs[HB * ZLD];        // Z[slot][col]
  __shared__ double Ws[SWA * VLD];       // W1^T, then W2^T  [col][c]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: scalar loop control
  const int ti = wave >> 1, tj = wave & 1;  // this wave's 16 x 16 tile of W (cols, c)
  const int b = a.b;
  const int64_t c0 = (int64_t)blockIdx.x * SWA;
  const int ncol = (int)((a.ncols - c0) < SWA ? (a.ncols - c0) : SWA);
  const int Hfull = b + NBW - 1;
  const int KS1 = (Hfull + 3) / 4;       // k-steps of W1 (rows beyond Hfull are zero in V)
  for (int idx = tid; idx < HB * ZLD; idx += NT) Zs[idx] = 0.0;
  Prefetch f;
  if (a.ngroups > 0) fetch_vt(a, a.ngroups - 1, 0, f);
  // Passes over Z take two sweep groups at once, jh = jl + 1 (group 0 alone when
  // the count is odd).  Window rows are relative to the lower group's base; the
  // blocks run in the order (jh, 0), (jl, 0), (jh, 1), (jl, 1), ...: block (jl, t)
  // meets only (jh, t-1) and (jh, t) among the upper group's blocks and shares no
  // row with (jh, t+1), so this order gives the same product as the upper group
  // followed by the lower one, while Z is streamed once per two groups.  After
  // (jl, t), rows [t b, t b + b) are final; the live rows never exceed b + 63.
  for (int64_t jh = a.ngroups - 1; jh >= 0; jh -= 2) {
    const bool two = jh >= 1;
    const int64_t jl = two ? jh - 1 : jh;
    const int64_t base = jl * NBW + 1;
    const int64_t nrel = a.n - base;
    const int64_t Pl = positions(a.n, b, jl * NBW);
    const int64_t Ph = two ? positions(a.n, b, jh * NBW) : 0;
    const int64_t nblk = Pl + Ph;
    // block q of the pass: group, position, row offset in the window
    auto decode = [&](int64_t q, int64_t& g, int64_t& t, int64_t& rb) {
      if (q < 2 * Ph) {
        t = q >> 1;
        g = (q & 1) ? jl : jh;
        rb = t * b + ((q & 1) ? 0 : NBW);
      } else {
        t = q - Ph;
        g = jl;
        rb = t * b;
      }
    };
    // first window (not prefetched: the previous pass has just been written back)
    int64_t loaded;
    __syncthreads();
    {
      int64_t g0, t0, rb0;
      decode(0, g0, t0, rb0);
      const int64_t hi = (rb0 + Hfull) < nrel ? (rb0 + Hfull) : nrel;
      for (int64_t lo = 0; lo < hi; lo += MAXB) {
        Prefetch g;
        const int64_t h2 = (lo + MAXB) < hi ? (lo + MAXB) : hi;
        fetch_rows(a, base, lo, h2, c0, ncol, g);
        commit_rows(g, lo, h2, Zs);
      }
      loaded = hi;
    }
    int64_t pend_lo = 0, pend_hi = 0;  // prefetched rows not yet in the window
    for (int64_t q = 0; q < nblk; ++q) {
      int64_t gq, tq, kb;
      decode(q, gq, tq, kb);
      __syncthreads();  // the previous block's write-back frees the slots refilled here
      commit_vt(f, Vs, Tt);
      if (pend_hi > pend_lo) {
        commit_rows(f, pend_lo, pend_hi, Zs);
        loaded = pend_hi;
        pend_lo = pend_hi = 0;
      }
      __syncthreads();
      // prefetch the next block (or the next pass's first block)
      if (q + 1 < nblk) {
        int64_t gn, tn, rbn;
        decode(q + 1, gn, tn, rbn);
        fetch_vt(a, gn, tn, f);
        int64_t hi = rbn + Hfull;
        if (hi > nrel) hi = nrel;
        if (hi > loaded) {
          fetch_rows(a, base, loaded, hi, c0, ncol, f);
          pend_lo = loaded;
          pend_hi = hi;
        }
      } else if (jl > 0) {
        fetch_vt(a, jl - 1, 0, f);
      }
      // W1^T (SWA x NBW) = Z_w^T V, tile (ti, tj).  Reflector c of the block is
      // supported on rows [c, c + b) of the window, so tile tj only needs rows
      // [16 tj, 16 tj + 15 + b); two accumulator chains (even / odd k steps).  The
      // loop is software pipelined: the LDS operands of the next two k steps are
      // read while the MFMAs of the current two run (reads past the last step stay
      // inside the window and V's rows, and are not used).
      {
        const int ks_lo = 4 * tj;
        int ks_hi = (16 * tj + 15 + b + 3) / 4;
        if (ks_hi > KS1) ks_hi = KS1;
        const double* zcol = Zs + ti * 16 + (lane & 15);
        const double* vcol = Vs + tj * 16 + (lane & 15);
        auto zat = [&](int ks) { return zcol[(int)((kb + ks * 4 + (lane >> 4)) & (HB - 1)) * ZLD]; };
        auto vat = [&](int ks) {
          const int row = ks * 4 + (lane >> 4);
          return vcol[(row < HP ? row : HP - 1) * VLD];
        };
        v4d w0 = {0.0, 0.0, 0.0, 0.0}, w1 = {0.0, 0.0, 0.0, 0.0};
        double a0 = zat(ks_lo), b0 = vat(ks_lo), a1 = zat(ks_lo + 1), b1 = vat(ks_lo + 1);
        int ks = ks_lo;
        for (; ks + 1 < ks_hi; ks += 2) {
          const double na0 = zat(ks + 2), nb0 = vat(ks + 2);
          const double na1 = zat(ks + 3), nb1 = vat(ks + 3);
          w0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, w0, 0, 0, 0);
          w1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, w1, 0, 0, 0);
          a0 = na0; b0 = nb0; a1 = na1; b1 = nb1;
        }
        if (ks < ks_hi) w0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, w0, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          Ws[(ti * 16 + (lane >> 4) + 4 * r) * VLD + tj * 16 + (lane & 15)] = w0[r] + w1[r];
      }
      __syncthreads();
      // W2^T = W1^T T^T, tile (ti, tj), two chains
      v4d u0 = {0.0, 0.0, 0.0, 0.0}, u1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < NBW / 4; ks += 2) {
        const int k0 = ks * 4 + (lane >> 4), k1 = k0 + 4;
        const double a0 = Ws[(ti * 16 + (lane & 15)) * VLD + k0];
        const double b0 = Tt[k0 * VLD + tj * 16 + (lane & 15)];
        const double a1 = Ws[(ti * 16 + (lane & 15)) * VLD + k1];
        const double b1 = Tt[k1 * VLD + tj * 16 + (lane & 15)];
        u0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, u0, 0, 0, 0);
        u1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, u1, 0, 0, 0);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Ws[(ti * 16 + (lane >> 4) + 4 * r) * VLD + tj * 16 + (lane & 15)] = u0[r] + u1[r];
      __syncthreads();
      // Z_w^T -= W2^T V^T : (SWA x HP) = 2 x 6 tiles, 3 per wave (column block ti)
      {
        v4d acc[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < NBW / 4; ++ks) {
          const int cc = ks * 4 + (lane >> 4);
          const double av = Ws[(ti * 16 + (lane & 15)) * VLD + cc];
#pragma unroll
          for (int t = 0; t < 3; ++t) {
            const int rt = tj * 3 + t;
            const double bv = Vs[(rt * 16 + (lane & 15)) * VLD + cc];
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
          }
        }
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const int rt = tj * 3 + t;
          const int slot = (int)((kb + rt * 16 + (lane & 15)) & (HB - 1));
#pragma unroll
          for (int r = 0; r < 4; ++r) Zs[slot * ZLD + ti * 16 + (lane >> 4) + 4 * r] -= acc[t][r];
        }
      }
      __syncthreads();
      // after a lower-group block, rows [kb, kb + b) are final for this pass; the
      // last block writes back everything still in the window
      if (gq == jl) {
        int64_t hi = kb + b;
        if (q + 1 == nblk) hi = loaded;
        if (hi > nrel) hi = nrel;
        for (int64_t lo = kb; lo < hi; lo += MAXB) {
          const int64_t h2 = (lo + MAXB) < hi ? (lo + MAXB) : hi;
          write_rows(a, base, lo, h2, c0, ncol, Zs);
        }
      }
    }
  }
}

// ---------------------------------------------------------------- b = 64: window in registers
//
// Each wave owns 16 columns of Z and keeps its 128-row window (8 tiles of 16 rows)
// in registers as MFMA accumulator tiles: slot s holds window rows
// 16 T + (lane >> 4) + 4 r (r = 0..3), column lane & 15, of the tile T with
// T mod 8 == s.  That is the output layout of the update Z += V X, and also the
// B-operand layout of W1 = V^T Z (k step 4u + r of a block is element r of its
// tile u); the output of W1 is in turn the B operand of X = -T W1.  A block is
// therefore three chained MFMA products with no data movement, and only V and T
// go through LDS (double buffered: one barrier per block).  With b = 64 and
// NBW = 32, block (jh, t) covers window tiles 4t + 2 .. 4t + 7 and block (jl, t)
// tiles 4t .. 4t + 5, so the slots repeat every two positions and the position
// loop is unrolled by two with every slot number fixed at compile time.  Zeros
// known from the shapes are skipped: reflector c of a block is supported on rows
// [c, c + 64), and T is upper triangular.
constexpr int RCOLS = 64;  // columns per workgroup, 16 per wave

struct Q2Pass {
  int64_t jh, jl, base, nrel, Ph, Pl;
  bool two;
};

__device__ inline Q2Pass q2_pass(const Q2Args& a, int64_t jh) {
  Q2Pass p;
  p.jh = jh;
  p.two = jh >= 1;
  p.jl = p.two ? jh - 1 : jh;
  p.base = p.jl * NBW + 1;
  p.nrel = a.n - p.base;
  p.Pl = positions(a.n, a.b, p.jl * NBW);
  p.Ph = p.two ? positions(a.n, a.b, jh * NBW) : 0;
  return p;
}

// The block applied after (upper ? jh : jl, t): its group g and position tn;
// false after the last block of the last pass.
__device__ inline bool q2_next(const Q2Args& a, const Q2Pass& p, bool upper, int64_t t,
                               int64_t& g, int64_t& tn) {
  if (upper) {
    g = p.jl;
    tn = t;
    return true;
  }
  if (t + 1 < p.Pl) {
    g = (p.two && t + 1 < p.Ph) ? p.jh : p.jl;
    tn = t + 1;
    return true;
  }
  if (p.jh - 2 < 0) return false;
  const Q2Pass q = q2_pass(a, p.jh - 2);
  g = q.Ph > 0 ? q.jh : q.jl;
  tn = 0;
  return true;
}

struct VTStage {
  double v[PV], t[PT];
};

__device__ inline void vt_fetch(const Q2Args& a, int64_t g, int64_t t, VTStage& f) {
  const double* blk = a.V + (g * a.kmax + t) * (int64_t)(HP * NBW);
  const double* Tg = a.T + (g * a.kmax + t) * NBW * NBW;
#pragma unroll
  for (int i = 0; i < PV; ++i) f.v[i] = blk[threadIdx.x + NT * i];
#pragma unroll
  for (int i = 0; i < PT; ++i) f.t[i] = Tg[threadIdx.x + NT * i];
}

__device__ inline void vt_commit(const VTStage& f, double* Vs, double* Tt) {
#pragma unroll
  for (int i = 0; i < PV; ++i) {
    const int idx = threadIdx.x + NT * i;
    Vs[(idx >> 5) * VLD + (idx & 31)] = f.v[i];
  }
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = threadIdx.x + NT * i;
    Tt[(idx >> 5) * VLD + (idx & 31)] = f.t[i];
  }
}

// The window of G column groups of 16: group g is lane & 15 of columns
// col0 + 16 g (G = 2 shares every V / T operand read from LDS between the two
// groups, and the groups' independent product chains fill each other's pipe
// drains).  Z is read and written through a buffer descriptor over the wave's
// 16 G columns: an element outside the matrix (a row past its end, a column past
// the last one) gets an offset beyond the descriptor's range, so the hardware's
// bounds check returns zero for the load and drops the store, with no branch and
// only 32-bit offsets kept per lane.
constexpr uint32_t OOB = 0x80000000u;

template <int G>
struct ZCol {
  // G = 1: this lane's column of Z (row 0) and whether it lies inside Z
  double* z;
  bool ok;
  // G = 2: the wave's columns through a buffer descriptor
  __amdgpu_buffer_rsrc_t rsrc;  // the wave's columns
  uint32_t coff[G];             // byte offset of this lane's column in group g, or OOB
  int64_t base;                 // matrix row of window row 0
  int64_t nrel;                 // window rows inside the matrix
};

template <int G>
__device__ inline uint32_t z_off(const ZCol<G>& zc, int g, int64_t tile, int r) {
  const int64_t row = 16 * tile + ((threadIdx.x & 63) >> 4) + 4 * r;
  return (zc.coff[g] != OOB && row < zc.nrel) ? zc.coff[g] + (uint32_t)((zc.base + row) * 8) : OOB;
}

template <int G>
__device__ inline v4d z_load(const ZCol<G>& zc, int g, int64_t tile) {
  v4d v;
  if constexpr (G == 1) {
    const int l4 = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = 16 * tile + l4 + 4 * r;
      v[r] = (zc.ok && row < zc.nrel) ? zc.z[zc.base + row] : 0.0;
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      v[r] = __builtin_bit_cast(
          double, __builtin_amdgcn_raw_buffer_load_b64(zc.rsrc, z_off(zc, g, tile, r), 0, 0));
  }
  return v;
}

template <int G>
__device__ inline void z_store(const ZCol<G>& zc, int g, int64_t tile, const v4d& v) {
  if constexpr (G == 1) {
    const int l4 = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = 16 * tile + l4 + 4 * r;
      if (zc.ok && row < zc.nrel) zc.z[zc.base + row] = v[r];
    }
  } else {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // the element goes through a scalar: this compiler's bit cast of a vector
      // element taken by reference reads element 0 whatever the index
      const double x = v[r];
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), zc.rsrc,
                                            z_off(zc, g, tile, r), 0, 0);
    }
  }
}

// One block on window slots S0 .. S0 + 5 (mod 8), V / T from LDS buffer cur; the
// next block's V / T are fetched meanwhile and committed to the other buffer.
template <int S0, int G>
__device__ __forceinline__ void q2_block(const Q2Args& a, const Q2Pass& p, bool upper, int64_t t,
                                         v4d (&Z)[G][8], double (*Vs)[HP * VLD],
                                         double (*Tt)[NBW * VLD], int& cur) {
  const int lane = threadIdx.x & 63, l15 = lane & 15, l4 = lane >> 4;
  int64_t gn = 0, tn = 0;
  const bool more = q2_next(a, p, upper, t, gn, tn);
  VTStage st;
  if (more) vt_fetch(a, gn, tn, st);
  const double* V = Vs[cur];
  const double* Tb = Tt[cur];
  // W (32 x 16) = V^T Z: c tile 0 meets window tiles 0..4, c tile 1 tiles 1..5
  v4d W0[G], W1[G];
#pragma unroll
  for (int g = 0; g < G; ++g) W0[g] = W1[g] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < 6; ++u) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double* vr = V + (16 * u + 4 * r + l4) * VLD + l15;
      if (u <= 4) {
        const double v0 = vr[0];
#pragma unroll
        for (int g = 0; g < G; ++g)
          W0[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(v0, Z[g][(S0 + u) & 7][r], W0[g], 0, 0, 0);
      }
      if (u >= 1) {
        const double v1 = vr[16];
#pragma unroll
        for (int g = 0; g < G; ++g)
          W1[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(v1, Z[g][(S0 + u) & 7][r], W1[g], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    W0[g] = -W0[g];
    W1[g] = -W1[g];
  }
  // X = T (-W): T(c', c) = Tt[c][c'], zero for c' > c
  v4d X0[G], X1[G];
#pragma unroll
  for (int g = 0; g < G; ++g) X0[g] = X1[g] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double* t0 = Tb + (4 * r + l4) * VLD + l15;
    const double* t1 = Tb + (16 + 4 * r + l4) * VLD + l15;
    const double t00 = t0[0], t11 = t1[16], t10 = t1[0];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      X0[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(t00, W0[g][r], X0[g], 0, 0, 0);
      X1[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(t11, W1[g][r], X1[g], 0, 0, 0);
      X0[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(t10, W1[g][r], X0[g], 0, 0, 0);
    }
  }

  // Z += V X: window tile u meets c tile 0 for u <= 4 and c tile 1 for u >= 1.
  // Consecutive products go to different window tiles (k step outermost).
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int u = 0; u <= 4; ++u) {
      const double v0 = V[(16 * u + l15) * VLD + 4 * r + l4];
#pragma unroll
      for (int g = 0; g < G; ++g)
        Z[g][(S0 + u) & 7] =
            __builtin_amdgcn_mfma_f64_16x16x4f64(v0, X0[g][r], Z[g][(S0 + u) & 7], 0, 0, 0);
    }
#pragma unroll
    for (int u = 1; u < 6; ++u) {
      const double v1 = V[(16 * u + l15) * VLD + 16 + 4 * r + l4];
#pragma unroll
      for (int g = 0; g < G; ++g)
        Z[g][(S0 + u) & 7] =
            __builtin_amdgcn_mfma_f64_16x16x4f64(v1, X1[g][r], Z[g][(S0 + u) & 7], 0, 0, 0);
    }
  }
  if (more) vt_commit(st, Vs[cur ^ 1], Tt[cur ^ 1]);
  __syncthreads();
  cur ^= 1;
}

// Positions t of one pass with t mod 2 == P: tiles 4t .. 4t + 7 sit in slots
// 4P .. 4P + 7 (mod 8).  Before the upper block, the four tiles it adds
// (4t + 4 .. 4t + 7, prefetched into S) replace the tiles the previous lower
// block finished; after the lower block, tiles 4t .. 4t + 3 are final.
template <int P, int G>
__device__ __forceinline__ void q2_position(const Q2Args& a, const Q2Pass& p, const ZCol<G>& zc,
                                            int64_t t, v4d (&Z)[G][8], v4d (&S)[G][4],
                                            double (*Vs)[HP * VLD], double (*Tt)[NBW * VLD],
                                            int& cur) {
  constexpr int SL = (4 * P) & 7, SU = (4 * P + 2) & 7, SN = (4 * P + 4) & 7;
  if (t >= 1) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int i = 0; i < 4; ++i) Z[g][(SN + i) & 7] = S[g][i];
#pragma unroll
      for (int i = 0; i < 4; ++i) S[g][i] = z_load(zc, g, 4 * t + 8 + i);
    }
  }
  if (p.two && t < p.Ph) q2_block<SU, G>(a, p, true, t, Z, Vs, Tt, cur);
  q2_block<SL, G>(a, p, false, t, Z, Vs, Tt, cur);
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int i = 0; i < 4; ++i) z_store(zc, g, 4 * t + i, Z[g][(SL + i) & 7]);
}

// ---------------------------------------------------------------- b = 64: staged window
//
// The same register window with its memory traffic reshaped.  Timing copies of
// the register-staged kernel that skipped one memory stream each ran 15-19%
// faster per stream (Z stores, Z prefetch loads, V / T staging): the phase is
// bound by its vector-memory traffic, not by the matrix cores.  Here
//  - V and T reach LDS through direct-to-LDS loads (1 KB per instruction, eight
//    per wave per block): no registers hold them and no LDS stores are issued.
//    q2_form_t writes both in the LDS layout (rows of 32, the 16-byte pairs of
//    row R permuted by pair ^ swz_key(R), so that the row-wise reads of W = V^T Z
//    and the column-wise reads of Z += V X stay spread over the banks);
//  - inside each 16-row tile the rows are relabelled so that accumulator element
//    r of lane (l15, l4) is tile row 4 l4 + r (V's rows are relabelled alike; the
//    products are unchanged): a lane holds four consecutive rows of its column,
//    read and written as two 16-byte accesses instead of four 8-byte ones;
//  - the window starts one row above the pass's first row (at jl NBW, an even
//    row), so those accesses are 16-byte aligned given an even leading dimension;
//    that row meets a zero row of V (LDS row 0) and is written back unchanged.
// Window rows past the matrix use the 8-byte accesses with out-of-range offsets.

// Element (row, col) of a staged 32-column LDS array.
__device__ __forceinline__ int swz(int row, int col) {
  return row * 32 + ((((col >> 1) ^ swz_key(row)) << 1) | (col & 1));
}

typedef __attribute__((address_space(3))) void* lds_ptr;

// Wait until this wave's direct-to-LDS loads have written LDS: first the loads
// (vector memory count), then, in an instruction of its own, the LDS writes they
// queued (LDS count).  One combined wait may find the LDS count at zero before
// the last load has queued its write.
__device__ __forceinline__ void dma_landed() {
  asm volatile("s_waitcnt vmcnt(0)\n\ts_waitcnt lgkmcnt(0)" ::: "memory");
}

// Block (g, t)'s V (24 KB) and T (8 KB) into LDS in 1 KB direct-to-LDS loads,
// eight per wave; no registers hold them and no LDS stores are issued.
__device__ __forceinline__ void vt_dma(const Q2Args& a, int64_t g, int64_t t, double* Vd,
                                       double* Td) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const char* vsrc = (const char*)(a.V + (g * a.kmax + t) * (int64_t)(HP * NBW));
  const char* tsrc = (const char*)(a.T + (g * a.kmax + t) * NBW * NBW);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int q = wave * 8 + i;
    if (q < 24)
      __builtin_amdgcn_global_load_lds((const void*)(vsrc + q * 1024 + lane * 16),
                                       (lds_ptr)((char*)Vd + q * 1024), 16, 0, 0);
    else
      __builtin_amdgcn_global_load_lds((const void*)(tsrc + (q - 24) * 1024 + lane * 16),
                                       (lds_ptr)((char*)Td + (q - 24) * 1024), 16, 0, 0);
  }
}

// The wave's columns of Z for the staged kernel: window row w is matrix row
// base + w, with base = jl NBW (one above the pass's first row, even).
struct ZColS {
  __amdgpu_buffer_rsrc_t rsrc;  // the wave's 16 columns
  uint32_t coff;                // byte offset of the lane's column + 32 l4, or OOB
  int64_t base;                 // matrix row of window row 0 (even)
  int64_t nrel;                 // window rows inside the matrix
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2v __attribute__((ext_vector_type(2)));

__device__ inline v4d zs_load(const ZColS& zc, int64_t tile) {
  v4d v;
  const int l4 = (threadIdx.x & 63) >> 4;
  const int64_t row0 = 16 * tile;
  if (row0 + 16 <= zc.nrel) {
    const uint32_t off = zc.coff == OOB ? OOB : zc.coff + (uint32_t)((zc.base + row0) * 8);
    const u32x4 lo = __builtin_amdgcn_raw_buffer_load_b128(zc.rsrc, off, 0, 0);
    const u32x4 hi = __builtin_amdgcn_raw_buffer_load_b128(zc.rsrc, off == OOB ? OOB : off + 16, 0, 0);
    v[0] = __builtin_bit_cast(double, u32x2v{lo.x, lo.y});
    v[1] = __builtin_bit_cast(double, u32x2v{lo.z, lo.w});
    v[2] = __builtin_bit_cast(double, u32x2v{hi.x, hi.y});
    v[3] = __builtin_bit_cast(double, u32x2v{hi.z, hi.w});
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + 4 * l4 + r;
      const uint32_t off = (zc.coff != OOB && row < zc.nrel)
                               ? zc.coff - 32 * l4 + (uint32_t)((zc.base + row) * 8)
                               : OOB;
      v[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(zc.rsrc, off, 0, 0));
    }
  }
  return v;
}

__device__ inline void zs_store(const ZColS& zc, int64_t tile, const v4d& v) {
  const int l4 = (threadIdx.x & 63) >> 4;
  const int64_t row0 = 16 * tile;
  const double x0 = v[0], x1 = v[1], x2 = v[2], x3 = v[3];
  const u32x2v a0 = __builtin_bit_cast(u32x2v, x0), a1 = __builtin_bit_cast(u32x2v, x1),
               a2 = __builtin_bit_cast(u32x2v, x2), a3 = __builtin_bit_cast(u32x2v, x3);
  if (row0 + 16 <= zc.nrel) {
    const uint32_t off = zc.coff == OOB ? OOB : zc.coff + (uint32_t)((zc.base + row0) * 8);
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{a0.x, a0.y, a1.x, a1.y}, zc.rsrc, off, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{a2.x, a2.y, a3.x, a3.y}, zc.rsrc,
                                           off == OOB ? OOB : off + 16, 0, 0);
  } else {
    const u32x2v e[4] = {a0, a1, a2, a3};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + 4 * l4 + r;
      const uint32_t off = (zc.coff != OOB && row < zc.nrel)
                               ? zc.coff - 32 * l4 + (uint32_t)((zc.base + row) * 8)
                               : OOB;
      __builtin_amdgcn_raw_buffer_store_b64(e[r], zc.rsrc, off, 0, 0);
    }
  }
}

constexpr int VROWS = HP + 1;  // LDS rows of a V buffer (row 0 zero)

template <int S0>
__device__ __forceinline__ void q2_block_staged(const Q2Args& a, const Q2Pass& p, bool upper,
                                            int64_t t, v4d (&Z)[8], double (*Vs)[VROWS * 32],
                                            double (*Tt)[NBW * 32], int& cur) {
  const int lane = threadIdx.x & 63, l15 = lane & 15, l4 = lane >> 4;
  const int pl = 4 * (l15 & 3) + (l15 >> 2);  // tile row of lane l15 as an output row
  int64_t gn = 0, tn = 0;
  const bool more = q2_next(a, p, upper, t, gn, tn);
  if (more) vt_dma(a, gn, tn, Vs[cur ^ 1] + 32, Tt[cur ^ 1]);
  const double* V = Vs[cur];
  const double* Tb = Tt[cur];
  v4d W0 = {0.0, 0.0, 0.0, 0.0}, W1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < 6; ++u) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * u + 4 * l4 + r;
      if (u <= 4) W0 = __builtin_amdgcn_mfma_f64_16x16x4f64(V[swz(row, l15)], Z[(S0 + u) & 7][r], W0, 0, 0, 0);
      if (u >= 1) W1 = __builtin_amdgcn_mfma_f64_16x16x4f64(V[swz(row, 16 + l15)], Z[(S0 + u) & 7][r], W1, 0, 0, 0);
    }
  }
  W0 = -W0;
  W1 = -W1;
  v4d X0 = {0.0, 0.0, 0.0, 0.0}, X1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double t00 = Tb[swz(4 * r + l4, l15)], t11 = Tb[swz(16 + 4 * r + l4, 16 + l15)],
                 t10 = Tb[swz(16 + 4 * r + l4, l15)];
    X0 = __builtin_amdgcn_mfma_f64_16x16x4f64(t00, W0[r], X0, 0, 0, 0);
    X1 = __builtin_amdgcn_mfma_f64_16x16x4f64(t11, W1[r], X1, 0, 0, 0);
    X0 = __builtin_amdgcn_mfma_f64_16x16x4f64(t10, W1[r], X0, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int u = 0; u <= 4; ++u)
      Z[(S0 + u) & 7] = __builtin_amdgcn_mfma_f64_16x16x4f64(V[swz(16 * u + pl, 4 * r + l4)], X0[r], Z[(S0 + u) & 7], 0, 0, 0);
#pragma unroll
    for (int u = 1; u < 6; ++u)
      Z[(S0 + u) & 7] = __builtin_amdgcn_mfma_f64_16x16x4f64(V[swz(16 * u + pl, 16 + 4 * r + l4)], X1[r], Z[(S0 + u) & 7], 0, 0, 0);
  }
  dma_landed();
  __syncthreads();
  cur ^= 1;
}

template <int P>
__device__ __forceinline__ void q2_position_staged(const Q2Args& a, const Q2Pass& p, const ZColS& zc,
                                               int64_t t, v4d (&Z)[8], v4d (&S)[4],
                                               double (*Vs)[VROWS * 32], double (*Tt)[NBW * 32],
                                               int& cur) {
  constexpr int SL = (4 * P) & 7, SU = (4 * P + 2) & 7, SN = (4 * P + 4) & 7;
  if (t >= 1) {
#pragma unroll
    for (int i = 0; i < 4; ++i) Z[(SN + i) & 7] = S[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) S[i] = zs_load(zc, 4 * t + 8 + i);
  }
  if (p.two && t < p.Ph) q2_block_staged<SU>(a, p, true, t, Z, Vs, Tt, cur);
  q2_block_staged<SL>(a, p, false, t, Z, Vs, Tt, cur);
#pragma unroll
  for (int i = 0; i < 4; ++i) zs_store(zc, 4 * t + i, Z[(SL + i) & 7]);
}

__device__ __forceinline__ void q2_apply_staged_body(const Q2Args& a) {
  __shared__ double Vs[2][VROWS * 32];
  __shared__ double Tt[2][NBW * 32];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  ZColS zc;
  {
    const int64_t wcol = (int64_t)blockIdx.x * RCOLS + wave * 16;
    int64_t nw = a.ncols - wcol;
    if (nw > 16) nw = 16;
    if (nw < 0) nw = 0;
    const int64_t bytes = nw > 0 ? ((nw - 1) * a.ldz + a.n) * 8 : 0;
    zc.rsrc = __builtin_amdgcn_make_buffer_rsrc(a.Z + (nw > 0 ? wcol : 0) * a.ldz, (short)0,
                                                (int)bytes, 0x00020000);
    const int c = lane & 15;
    zc.coff = c < nw ? (uint32_t)(c * a.ldz * 8 + 32 * (lane >> 4)) : OOB;
  }
  if (a.ngroups <= 0) return;
  if (tid < 32) {
    Vs[0][tid] = 0.0;
    Vs[1][tid] = 0.0;
  }
  int cur = 0;
  {
    const Q2Pass p = q2_pass(a, a.ngroups - 1);
    vt_dma(a, p.Ph > 0 ? p.jh : p.jl, 0, Vs[0] + 32, Tt[0]);
    dma_landed();
  }
  __syncthreads();
  v4d Z[8], S[4];
  for (int64_t jh = a.ngroups - 1; jh >= 0; jh -= 2) {
    const Q2Pass p = q2_pass(a, jh);
    zc.base = p.base - 1;
    zc.nrel = p.nrel + 1;
#pragma unroll
    for (int s = 0; s < 8; ++s) Z[s] = zs_load(zc, s);
#pragma unroll
    for (int i = 0; i < 4; ++i) S[i] = zs_load(zc, 8 + i);
    for (int64_t t = 0; t < p.Pl; t += 2) {
      q2_position_staged<0>(a, p, zc, t, Z, S, Vs, Tt, cur);
      if (t + 1 < p.Pl) q2_position_staged<1>(a, p, zc, t + 1, Z, S, Vs, Tt, cur);
    }
    if ((p.Pl & 1) == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) zs_store(zc, 4 * p.Pl + i, Z[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) zs_store(zc, 4 * p.Pl + i, Z[4 + i]);
    }
  }
}

// The whole Q2 application for the G column groups of each wave: 64 G columns
// per workgroup of four waves.
template <int G>
__device__ __forceinline__ void q2_apply_reg_body(const Q2Args& a) {
  __shared__ double Vs[2][HP * VLD];
  __shared__ double Tt[2][NBW * VLD];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  ZCol<G> zc;
  {
    const int64_t col = (int64_t)blockIdx.x * RCOLS + wave * 16 + (lane & 15);
    zc.ok = col < a.ncols;
    zc.z = a.Z + (zc.ok ? col : 0) * a.ldz;
  }
  if constexpr (G > 1) {
    const int64_t wcol = (int64_t)blockIdx.x * (RCOLS * G) + wave * (16 * G);
    int64_t nw = a.ncols - wcol;  // columns of this wave inside Z
    if (nw > 16 * G) nw = 16 * G;
    if (nw < 0) nw = 0;
    const int64_t bytes = nw > 0 ? ((nw - 1) * a.ldz + a.n) * 8 : 0;
    zc.rsrc = __builtin_amdgcn_make_buffer_rsrc(a.Z + (nw > 0 ? wcol : 0) * a.ldz, (short)0,
                                                (int)bytes, 0x00020000);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int c = 16 * g + (lane & 15);
      zc.coff[g] = c < nw ? (uint32_t)(c * a.ldz * 8) : OOB;
    }
  }
  if (a.ngroups <= 0) return;
  int cur = 0;
  {
    const Q2Pass p = q2_pass(a, a.ngroups - 1);
    VTStage st;
    vt_fetch(a, p.Ph > 0 ? p.jh : p.jl, 0, st);
    vt_commit(st, Vs[0], Tt[0]);
  }
  __syncthreads();
  v4d Z[G][8], S[G][4];
  for (int64_t jh = a.ngroups - 1; jh >= 0; jh -= 2) {
    const Q2Pass p = q2_pass(a, jh);
    zc.base = p.base;
    zc.nrel = p.nrel;
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int s = 0; s < 8; ++s) Z[g][s] = z_load(zc, g, s);
#pragma unroll
      for (int i = 0; i < 4; ++i) S[g][i] = z_load(zc, g, 8 + i);
    }
    for (int64_t t = 0; t < p.Pl; t += 2) {
      q2_position<0, G>(a, p, zc, t, Z, S, Vs, Tt, cur);
      if (t + 1 < p.Pl) q2_position<1, G>(a, p, zc, t + 1, Z, S, Vs, Tt, cur);
    }
    // the four tiles loaded last, 4 Pl .. 4 Pl + 3
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if ((p.Pl & 1) == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) z_store(zc, g, 4 * p.Pl + i, Z[g][i]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) z_store(zc, g, 4 * p.Pl + i, Z[g][4 + i]);
      }
    }
  }
}

// ---------------------------------------------------------------- FP32 arithmetic
//
// The same register-window application in FP32 arithmetic (the mixed-precision
// path: Z, V and T rounded to FP32, products accumulated in FP32 on the matrix
// cores, Z stored back in FP64).  v_mfma_f32_16x16x4f32 takes its operands in the
// FP64 instruction's layout, but element r of lane l of its accumulator is row
// 4 (l >> 4) + r of the 16 x 16 tile (FP64: (l >> 4) + 4 r).  Since the window
// tiles are also the B operand of W = V^T Z, a k step of a tile now covers rows
// {4 l4 + r} instead of {l4 + 4 r}; only the row and column indices of the V, T
// and Z accesses change, the zero structure (tiles 0..4 / 1..5, T upper
// triangular) is the same.
struct ZColF {
  double* z;      // this lane's column of Z (row 0 of the matrix)
  bool ok;        // column inside Z
  int64_t base;   // matrix row of window row 0
  int64_t nrel;   // window rows inside the matrix
};

__device__ inline v4f zf_load(const ZColF& zc, int64_t tile) {
  const int l4 = (threadIdx.x & 63) >> 4;
  v4f v;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = 16 * tile + 4 * l4 + r;
    v[r] = (zc.ok && row < zc.nrel) ? (float)zc.z[zc.base + row] : 0.0f;
  }
  return v;
}

__device__ inline void zf_store(const ZColF& zc, int64_t tile, const v4f& v) {
  const int l4 = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = 16 * tile + 4 * l4 + r;
    if (zc.ok && row < zc.nrel) zc.z[zc.base + row] = (double)v[r];
  }
}

__device__ inline void vt_commit_f32(const VTStage& f, float* Vs, float* Tt) {
#pragma unroll
  for (int i = 0; i < PV; ++i) {
    const int idx = threadIdx.x + NT * i;
    Vs[(idx >> 5) * VLD + (idx & 31)] = (float)f.v[i];
  }
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int idx = threadIdx.x + NT * i;
    Tt[(idx >> 5) * VLD + (idx & 31)] = (float)f.t[i];
  }
}

__device__ inline v4f mfma_f32(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int S0>
__device__ __forceinline__ void q2_block_f32(const Q2Args& a, const Q2Pass& p, bool upper,
                                             int64_t t, v4f (&Z)[8], float (*Vs)[HP * VLD],
                                             float (*Tt)[NBW * VLD], int& cur) {
  const int lane = threadIdx.x & 63, l15 = lane & 15, l4 = lane >> 4;
  int64_t gn = 0, tn = 0;
  const bool more = q2_next(a, p, upper, t, gn, tn);
  VTStage st;
  if (more) vt_fetch(a, gn, tn, st);
  const float* V = Vs[cur];
  const float* Tb = Tt[cur];
  // W (32 x 16) = V^T Z; k step r of window tile u: rows 16 u + 4 l4 + r
  v4f W0 = {0.0f, 0.0f, 0.0f, 0.0f}, W1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int u = 0; u < 6; ++u) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float* vr = V + (16 * u + 4 * l4 + r) * VLD + l15;
      if (u <= 4) W0 = mfma_f32(vr[0], Z[(S0 + u) & 7][r], W0);
      if (u >= 1) W1 = mfma_f32(vr[16], Z[(S0 + u) & 7][r], W1);
    }
  }
  W0 = -W0;
  W1 = -W1;
  // X = T (-W); k step r: c = 4 l4 + r
  v4f X0 = {0.0f, 0.0f, 0.0f, 0.0f}, X1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float* t0 = Tb + (4 * l4 + r) * VLD + l15;
    const float* t1 = Tb + (16 + 4 * l4 + r) * VLD + l15;
    X0 = mfma_f32(t0[0], W0[r], X0);
    X1 = mfma_f32(t1[16], W1[r], X1);
    X0 = mfma_f32(t1[0], W1[r], X0);
  }
  // Z += V X; k step r: c = 4 l4 + r
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int u = 0; u <= 4; ++u)
      Z[(S0 + u) & 7] = mfma_f32(V[(16 * u + l15) * VLD + 4 * l4 + r], X0[r], Z[(S0 + u) & 7]);
#pragma unroll
    for (int u = 1; u < 6; ++u)
      Z[(S0 + u) & 7] =
          mfma_f32(V[(16 * u + l15) * VLD + 16 + 4 * l4 + r], X1[r], Z[(S0 + u) & 7]);
  }
  if (more) vt_commit_f32(st, Vs[cur ^ 1], Tt[cur ^ 1]);
  __syncthreads();
  cur ^= 1;
}

template <int P>
__device__ __forceinline__ void q2_position_f32(const Q2Args& a, const Q2Pass& p,
                                                const ZColF& zc, int64_t t, v4f (&Z)[8],
                                                v4f (&S)[4], float (*Vs)[HP * VLD],
                                                float (*Tt)[NBW * VLD], int& cur) {
  constexpr int SL = (4 * P) & 7, SU = (4 * P + 2) & 7, SN = (4 * P + 4) & 7;
  if (t >= 1) {
#pragma unroll
    for (int i = 0; i < 4; ++i) Z[(SN + i) & 7] = S[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) S[i] = zf_load(zc, 4 * t + 8 + i);
  }
  if (p.two && t < p.Ph) q2_block_f32<SU>(a, p, true, t, Z, Vs, Tt, cur);
  q2_block_f32<SL>(a, p, false, t, Z, Vs, Tt, cur);
#pragma unroll
  for (int i = 0; i < 4; ++i) zf_store(zc, 4 * t + i, Z[(SL + i) & 7]);
}

// 16 columns per wave, FP32 window (half the registers and LDS of the FP64 one).
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
q2_apply_reg_f32(Q2Args a) {
  __shared__ float Vs[2][HP * VLD];
  __shared__ float Tt[2][NBW * VLD];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  ZColF zc;
  const int64_t col = (int64_t)blockIdx.x * RCOLS + wave * 16 + (lane & 15);
  zc.ok = col < a.ncols;
  zc.z = a.Z + (zc.ok ? col : 0) * a.ldz;
  if (a.ngroups <= 0) return;
  int cur = 0;
  {
    const Q2Pass p = q2_pass(a, a.ngroups - 1);
    VTStage st;
    vt_fetch(a, p.Ph > 0 ? p.jh : p.jl, 0, st);
    vt_commit_f32(st, Vs[0], Tt[0]);
  }
  __syncthreads();
  v4f Z[8], S[4];
  for (int64_t jh = a.ngroups - 1; jh >= 0; jh -= 2) {
    const Q2Pass p = q2_pass(a, jh);
    zc.base = p.base;
    zc.nrel = p.nrel;
#pragma unroll
    for (int s = 0; s < 8; ++s) Z[s] = zf_load(zc, s);
#pragma unroll
    for (int i = 0; i < 4; ++i) S[i] = zf_load(zc, 8 + i);
    for (int64_t t = 0; t < p.Pl; t += 2) {
      q2_position_f32<0>(a, p, zc, t, Z, S, Vs, Tt, cur);
      if (t + 1 < p.Pl) q2_position_f32<1>(a, p, zc, t + 1, Z, S, Vs, Tt, cur);
    }
    if ((p.Pl & 1) == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) zf_store(zc, 4 * p.Pl + i, Z[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) zf_store(zc, 4 * p.Pl + i, Z[4 + i]);
    }
  }
}

// One column group per wave, two waves per SIMD (two workgroups per CU): for
// column counts that would leave CUs idle with 128 columns per workgroup.
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
q2_apply_reg(Q2Args a) {
  q2_apply_reg_body<1>(a);
}

// The staged window (16 columns per wave, two waves per SIMD): the default for
// FP64 with b = 64.
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
q2_apply_staged(Q2Args a) {
  q2_apply_staged_body(a);
}

// Two column groups per wave, one wave per SIMD: the full register file (no
// spills) and twice the independent MFMA chains per wave.
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1)))
q2_apply_reg2(Q2Args a) {
  q2_apply_reg_body<2>(a);
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
  enum class Kernel { Lds, Reg, Reg2, RegF32, Staged } kern = Kernel::Lds;
  if (c.b == 64) {
    if (math_mode() == MathMode::Fp32 && tune("q2_mixed_fp32", n) == 1)
      kern = Kernel::RegF32;
    else if (ncols >= tune("q2_wide_min_cols", n))
      kern = Kernel::Reg2;
    else if (tune("q2_staged", n) == 1 && ldz % 2 == 0 && ((uintptr_t)Z & 15) == 0)
      kern = Kernel::Staged;
    else
      kern = Kernel::Reg;
  }
  // the staged kernel reads V and T in its swizzled layout, which q2_form_t then
  // writes (V in place: the chase's reflectors are consumed by this one call)
  a.swizzle = kern == Kernel::Staged ? 1 : 0;
  a.T = ws.take<double>((size_t)a.ngroups * a.kmax * NBW * NBW);
  hipLaunchKernelGGL(q2_form_t, dim3((unsigned)a.kmax, (unsigned)a.ngroups), dim3(NT), 0, s, a);
  GEP_LAUNCH_CHECK();
  {
    // algorithmic flops: ~n^2 / (2b) reflectors of length b, 4b flops per column each
    ProbeScope probe(PROBE_Q2_APPLY, s, 2.0 * (double)n * (double)n * (double)ncols);
    // the register-window kernels address a wave's 16 or 32 columns of Z with
    // 32-bit byte offsets
    if (c.b == 64 && (32 * ldz + n) * 8 >= (int64_t)OOB)
      throw HipError{hipErrorInvalidValue, "leading dimension of Z too large"};
    switch (kern) {
      case Kernel::RegF32:
        hipLaunchKernelGGL(q2_apply_reg_f32, dim3((unsigned)cdiv(ncols, RCOLS)), dim3(NT), 0, s, a);
        break;
      case Kernel::Reg2:
        hipLaunchKernelGGL(q2_apply_reg2, dim3((unsigned)cdiv(ncols, 2 * RCOLS)), dim3(NT), 0, s, a);
        break;
      case Kernel::Staged:
        hipLaunchKernelGGL(q2_apply_staged, dim3((unsigned)cdiv(ncols, RCOLS)), dim3(NT), 0, s, a);
        break;
      case Kernel::Reg:
        hipLaunchKernelGGL(q2_apply_reg, dim3((unsigned)cdiv(ncols, RCOLS)), dim3(NT), 0, s, a);
        break;
      case Kernel::Lds:
        hipLaunchKernelGGL(q2_apply, dim3((unsigned)cdiv(ncols, SWA)), dim3(NT), 0, s, a);
        break;
    }
    GEP_LAUNCH_CHECK();
  }
}

size_t sb2st_reflector_count(int64_t n, int b) {
  const int64_t kmax = n > 1 ? cdiv(n - 1, b) : 1;
  return (size_t)(n > 0 ? n : 1) * (size_t)kmax;
}

size_t sb2st_block_storage(int64_t n, int b) {
  const int64_t kmax = n > 1 ? cdiv(n - 1, b) : 1;
  const int64_t nsweeps = n > 2 ? n - 2 : 0;
  const int64_t ngroups = nsweeps > 0 ? cdiv(nsweeps, NBW) : 1;
  return (size_t)ngroups * kmax * HP * NBW;
}

size_t sb2st_message_bytes(int64_t n, int b) {
  const int64_t npos0 = n > 2 && b > 0 ? (n - 2) / b + 1 : 0;
  return (size_t)(4 * npos0 * MSG) * sizeof(double);
}

namespace {
// Workgroups of the data-stationary chase (P positions each) that can be resident
// at once.
template <int P>
int64_t stationary_capacity() {
  static const int64_t cached = [] {
    int dev = 0, cus = 0, per = 0;
    GEP_HIP(hipGetDevice(&dev));
    GEP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    GEP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)chase_stationary<P>,
                                                         CNT, 0));
    return (int64_t)cus * per;
  }();
  return cached;
}
}  // namespace

void sb2st(const BulgeChase& c, hipStream_t s) {
  const int64_t n = c.n;
  if (c.b > MAXB || c.b < 1) throw HipError{hipErrorInvalidValue, "band width"};
  const int64_t nsweeps = n > 2 ? n - 2 : 0;
  // Reflectors a failed chase never reaches stay the identity (V = 0, tau = 0).
  if (c.V) fill_f64(c.V, (int64_t)sb2st_block_storage(n, c.b), 0.0, s);
  if (c.tau) fill_f64(c.tau, (int64_t)sb2st_reflector_count(n, c.b), 0.0, s);
  if (nsweeps > 0) {
    int32_t* progress = c.sync;
    int32_t* ticket = c.sync + n;
    fill_i32(c.sync, n + 8, 0, s);
    fill_i32(c.err, 1, 0, s);
    ChaseArgs a;
    a.n = n; a.b = c.b; a.band = c.band; a.ldband = c.ldband; a.V = c.V; a.tau = c.tau;
    a.kmax = c.kmax; a.progress = progress; a.ticket = ticket; a.err = c.err; a.nsweeps = nsweeps;
    a.timeout_ticks = wait_limit_ticks();  // 10 s for any single wait
    a.force_fail = force_wait_timeout() ? 1 : 0;
    // Sweep s + 1 trails sweep s by about two positions, so at most about half of
    // a sweep's positions are ever worked on at once: more workgroups would only
    // spin (and, in batched solves, keep other instances' chases off the CUs).
    const int64_t npos0 = (n - 2) / c.b + 1;
    // Data-stationary chase: one position per workgroup if all fit at once, else two
    // (tuning value 2: two in any case)
    int per_group = 0;
    const int64_t mode = tune("chase_stationary", n);
    if (c.coop && c.b >= 8 && c.msg && c.msg_bytes >= sb2st_message_bytes(n, c.b) &&
        2 * npos0 <= n + 8 && mode >= 1) {
      if (mode == 1 && npos0 <= stationary_capacity<1>())
        per_group = 1;
      else if (cdiv(npos0, 2) <= stationary_capacity<2>())
        per_group = 2;
    }
    ProbeScope probe(PROBE_CHASE, s, 6.0 * c.b * (double)n * (double)n);
    if (per_group > 0) {
      StatArgs x;
      x.c = a;
      x.npos0 = npos0;
      x.msg = c.msg;
      x.fwdf = c.sync;
      x.backf = c.sync + npos0;
      void* args[] = {&x};
      const void* fn = per_group == 1 ? (const void*)chase_stationary<1>
                                      : (const void*)chase_stationary<2>;
      GEP_HIP(hipLaunchCooperativeKernel(fn, dim3((unsigned)cdiv(npos0, per_group)), dim3(CNT),
                                         args, 0, s));
    } else {
      int64_t groups = npos0 / 2 + tune("chase_extra_groups", n);
      if (groups > nsweeps) groups = nsweeps;
      if (groups > 512) groups = 512;
      hipLaunchKernelGGL(chase_kernel, dim3((unsigned)groups), dim3(CNT), 0, s, a);
      GEP_LAUNCH_CHECK();
    }
    raise_info_if(c.err, c.info, INFO_WAIT_TIMEOUT, s);
  }
  hipLaunchKernelGGL(extract_tridiag, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, n,
                     (const double*)c.band, c.ldband, c.d, c.e);
  GEP_LAUNCH_CHECK();
}

}  // namespace gep

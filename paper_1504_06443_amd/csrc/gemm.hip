// FP64 (and FP32) matrix contraction on CDNA4 matrix cores.
//
// Every blocked step of the solver (Cholesky trailing update, reduced-matrix
// solves, the two-sided band-reduction update, the divide-and-conquer merges and
// the back transformations) ends up here.
//
// Design:
//  * a workgroup of 4 waves (2 x 2) owns a BM x BN tile of C; each wave owns a
//    (BM/2) x (BN/2) sub-tile made of 16 x 16 MFMA blocks (v_mfma_f64_16x16x4f64);
//  * A and B tiles of depth BK are staged in LDS (double buffered: the global
//    loads of step k+1 are in flight while step k is multiplied);
//  * the MFMA is issued with the operands swapped (C^T = op(B)^T op(A)^T), which
//    puts 16 consecutive rows of one column of C in 16 consecutive lanes, so the
//    column-major store of C is coalesced;
//  * workgroup ids are remapped so that the workgroups that land on one XCD (ids
//    equal mod 8) take a contiguous range of tiles, and that range is walked in
//    groups of 8 tile rows, which keeps the shared A rows / B columns in that
//    XCD's L2.
#include <type_traits>

#include "common.h"

namespace gep {
namespace {

constexpr int NT = 256;  // threads per workgroup (4 waves)

struct Params {
  int64_t m, n, k;
  double alpha, beta;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  int64_t sA, sB, sC;
  int transA, transB, symA, uplo;
  int tiles_m, tiles_n;
  int lower_grid = 0;  // 1: the grid holds only the tiles on or below the diagonal
  int64_t kchunk;  // > 0: batch index z sums k in [z*kchunk, (z+1)*kchunk) into C + z*sC
  int vecA, vecB;  // operand base 16-byte aligned and leading dimension even
};

__device__ inline void tile_coords(int tiles_m, int tiles_n, int& tm, int& tn) {
  const int nb = gridDim.x;
  const int bid = blockIdx.x;
  const int nfull = (nb / 8) * 8;
  int logical = bid;
  if (bid < nfull) logical = (bid % 8) * (nfull / 8) + bid / 8;
  constexpr int G = 8;
  const int per_group = G * tiles_n;
  const int group = logical / per_group;
  const int first_m = group * G;
  int gsz = tiles_m - first_m;
  if (gsz > G) gsz = G;
  const int in_group = logical % per_group;
  tm = first_m + in_group % gsz;
  tn = in_group / gsz;
}

// Lower-triangle launches: the grid holds the T (T + 1) / 2 tiles on or below the
// diagonal, numbered row by row; the workgroups of one XCD again take a
// contiguous range, which now holds an equal share of the work (a full-grid
// launch would hand the XCDs of the first tile rows almost nothing to do).
__device__ inline void lower_tile_coords(int& tm, int& tn) {
  const int nb = gridDim.x;
  const int bid = blockIdx.x;
  const int nfull = (nb / 8) * 8;
  int logical = bid;
  if (bid < nfull) logical = (bid % 8) * (nfull / 8) + bid / 8;
  int r = (int)((sqrt(8.0 * (double)logical + 1.0) - 1.0) * 0.5);
  while ((int64_t)r * (r + 1) / 2 > logical) --r;
  while ((int64_t)(r + 1) * (r + 2) / 2 <= logical) ++r;
  tm = r;
  tn = logical - r * (r + 1) / 2;
}

template <int BM, int BK>
__device__ inline void load_a(const Params& p, const double* __restrict__ A, int64_t m0, int64_t k0,
                              int64_t kend, double* ra) {
  constexpr int PER = BM * BK / NT;
  const int tid = threadIdx.x;
  int mode = p.transA ? 1 : 0;
  if (p.symA) {
    if (m0 >= k0 + BK - 1) mode = 0;          // tile entirely on/below the diagonal
    else if (m0 + BM - 1 < k0) mode = 3;      // entirely above: read the mirror
    else mode = 2;                             // straddles the diagonal
  }
  if (mode == 0 || mode == 2) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + NT * i;
      const int64_t r = m0 + idx % BM, c = k0 + idx / BM;
      double v = 0.0;
      if (r < p.m && c < kend) {
        if (mode == 2 && r < c) v = A[c + r * p.lda];
        else v = A[r + c * p.lda];
      }
      ra[i] = v;
    }
  } else {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + NT * i;
      const int64_t c = k0 + idx % BK, r = m0 + idx / BK;
      ra[i] = (r < p.m && c < kend) ? A[c + r * p.lda] : 0.0;
    }
  }
}

template <int BM, int BK, int LDA_S>
__device__ inline void store_a(const Params& p, int64_t m0, int64_t k0, const double* ra,
                               double* As) {
  constexpr int PER = BM * BK / NT;
  const int tid = threadIdx.x;
  bool rfast = !p.transA;
  if (p.symA) rfast = !(m0 + BM - 1 < k0);
  if (rfast) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + NT * i;
      As[(idx / BM) * LDA_S + idx % BM] = ra[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + NT * i;
      As[(idx % BK) * LDA_S + idx / BK] = ra[i];
    }
  }
}

template <int BN, int BK>
__device__ inline void load_b(const Params& p, const double* __restrict__ B, int64_t k0, int64_t n0,
                              double* rb) {
  constexpr int PER = BN * BK / NT;
  const int tid = threadIdx.x;
  if (!p.transB) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + NT * i;
      const int64_t kk = k0 + idx % BK, j = n0 + idx / BK;
      rb[i] = (kk < p.k && j < p.n) ? B[kk + j * p.ldb] : 0.0;
    }
  } else {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + NT * i;
      const int64_t j = n0 + idx % BN, kk = k0 + idx / BN;
      rb[i] = (kk < p.k && j < p.n) ? B[j + kk * p.ldb] : 0.0;
    }
  }
}

template <int BN, int BK, int LDB_S>
__device__ inline void store_b(const Params& p, const double* rb, double* Bs) {
  constexpr int PER = BN * BK / NT;
  const int tid = threadIdx.x;
  if (!p.transB) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + NT * i;
      Bs[(idx % BK) * LDB_S + idx / BK] = rb[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + NT * i;
      Bs[(idx / BN) * LDB_S + idx % BN] = rb[i];
    }
  }
}

template <int BM, int BN, int BK, bool FAST>
__device__ inline void dgemm_tile(Params& p, int tm, int tn, int64_t z);

// FAST: every tile is interior, k is a multiple of BK and both operands are
// 16-byte aligned with even leading dimensions (no bounds checks at all).
template <int BM, int BN, int BK, bool FAST>
__global__ void __launch_bounds__(NT) dgemm_kernel(Params p) {
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, tm, tn);
  dgemm_tile<BM, BN, BK, FAST>(p, tm, tn, blockIdx.y);
}

// 64 x 64 tiles fit two workgroups' registers per SIMD: ask for that occupancy.
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
dgemm_kernel_64(Params p) {
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, tm, tn);
  dgemm_tile<64, 64, 16, false>(p, tm, tn, blockIdx.y);
}

// Problems whose sizes live in device memory (written by an earlier kernel).
template <int BM, int BN, int BK>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
dgemm_grouped_kernel(const GemmDesc* __restrict__ desc) {
  const GemmDesc d = desc[blockIdx.y];
  if (d.m <= 0 || d.n <= 0) return;
  const int tiles_m = (int)((d.m + BM - 1) / BM), tiles_n = (int)((d.n + BN - 1) / BN);
  if ((int)blockIdx.x >= tiles_m * tiles_n) return;
  Params p;
  p.m = d.m; p.n = d.n; p.k = d.k; p.alpha = d.alpha; p.beta = d.beta;
  p.A = d.A; p.lda = d.lda; p.B = d.B; p.ldb = d.ldb; p.C = d.C; p.ldc = d.ldc;
  p.sA = p.sB = p.sC = 0;
  p.transA = d.transA; p.transB = d.transB; p.symA = 0; p.uplo = 0;
  p.tiles_m = tiles_m; p.tiles_n = tiles_n; p.kchunk = 0;
  p.vecA = ((uintptr_t)d.A % 16 == 0) && (d.lda % 2 == 0);
  p.vecB = ((uintptr_t)d.B % 16 == 0) && (d.ldb % 2 == 0);
  dgemm_tile<BM, BN, BK, false>(p, (int)blockIdx.x % tiles_m, (int)blockIdx.x / tiles_m, 0);
}

// Interior tiles with a full k step and 16-byte aligned operands: unchecked
// double2 loads.  ta selects op(A) read transposed (element (r, c) at A[c + r*lda]).
template <int BM, int BN, int BK, int LDA_S, int LDB_S>
struct FastIO {
  static constexpr int PA2 = BM * BK / 2 / NT, PB2 = BN * BK / 2 / NT;
  __device__ static inline void load(const Params& p, bool ta, const double* At, const double* Bt,
                                     double* ra, double* rb) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < PA2; ++i) {
      const int idx = tid + NT * i;
      double2 v;
      if (!ta) {
        const int rp = idx % (BM / 2), c = idx / (BM / 2);
        v = *reinterpret_cast<const double2*>(At + 2 * rp + (int64_t)c * p.lda);
      } else {
        const int cp = idx % (BK / 2), r = idx / (BK / 2);
        v = *reinterpret_cast<const double2*>(At + 2 * cp + (int64_t)r * p.lda);
      }
      ra[2 * i] = v.x;
      ra[2 * i + 1] = v.y;
    }
#pragma unroll
    for (int i = 0; i < PB2; ++i) {
      const int idx = tid + NT * i;
      double2 v;
      if (!p.transB) {
        const int kp = idx % (BK / 2), j = idx / (BK / 2);
        v = *reinterpret_cast<const double2*>(Bt + 2 * kp + (int64_t)j * p.ldb);
      } else {
        const int jp = idx % (BN / 2), kk = idx / (BN / 2);
        v = *reinterpret_cast<const double2*>(Bt + 2 * jp + (int64_t)kk * p.ldb);
      }
      rb[2 * i] = v.x;
      rb[2 * i + 1] = v.y;
    }
  }
  __device__ static inline void store(const Params& p, bool ta, const double* ra, const double* rb,
                                      double* As, double* Bs) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < PA2; ++i) {
      const int idx = tid + NT * i;
      if (!ta) {
        const int rp = idx % (BM / 2), c = idx / (BM / 2);
        *reinterpret_cast<double2*>(As + c * LDA_S + 2 * rp) = double2{ra[2 * i], ra[2 * i + 1]};
      } else {
        const int cp = idx % (BK / 2), r = idx / (BK / 2);
        As[(2 * cp) * LDA_S + r] = ra[2 * i];
        As[(2 * cp + 1) * LDA_S + r] = ra[2 * i + 1];
      }
    }
#pragma unroll
    for (int i = 0; i < PB2; ++i) {
      const int idx = tid + NT * i;
      if (!p.transB) {
        const int kp = idx % (BK / 2), j = idx / (BK / 2);
        Bs[(2 * kp) * LDB_S + j] = rb[2 * i];
        Bs[(2 * kp + 1) * LDB_S + j] = rb[2 * i + 1];
      } else {
        const int jp = idx % (BN / 2), kk = idx / (BN / 2);
        *reinterpret_cast<double2*>(Bs + kk * LDB_S + 2 * jp) = double2{rb[2 * i], rb[2 * i + 1]};
      }
    }
  }
};

// Symmetric operand, k step straddling the diagonal, interior tile: element-wise
// mirror select straight into LDS (no bounds checks).
template <int BM, int BK, int LDA_S>
__device__ inline void sym_diag_to_lds(const Params& p, const double* A, int64_t m0, int64_t k0,
                                       double* As) {
  for (int idx = threadIdx.x; idx < BM * BK; idx += NT) {
    const int r = idx % BM, c = idx / BM;
    const int64_t gr = m0 + r, gc = k0 + c;
    As[c * LDA_S + r] = (gr >= gc) ? A[gr + gc * p.lda] : A[gc + gr * p.lda];
  }
}

template <int BM, int BN, int BK, bool FAST>
__device__ inline void dgemm_tile(Params& p, int tm, int tn, int64_t z) {
  constexpr int PAD = 4;
  constexpr int LDA_S = BM + PAD, LDB_S = BN + PAD;
  constexpr int WM = BM / 2, WN = BN / 2;  // per-wave sub-tile
  constexpr int FR = WM / 16, FC = WN / 16;
  constexpr int PA = BM * BK / NT, PB = BN * BK / NT;
  using IO = FastIO<BM, BN, BK, LDA_S, LDB_S>;
  __shared__ double As[2][BK * LDA_S];
  __shared__ double Bs[2][BK * LDB_S];

  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  if (p.uplo == 1 && m0 + BM - 1 < n0) return;  // strictly upper tile

  const double* __restrict__ A = p.A + z * p.sA;
  const double* __restrict__ B = p.B + z * p.sB;
  double* __restrict__ C = p.C + z * p.sC;
  // ka: absolute k of this tile's first k step.  A symmetric A is addressed with
  // absolute k (its diagonal decides between the stored and the mirrored read), so
  // under split-K it stays unshifted and ka carries the chunk start instead.
  int64_t ka = 0;
  if (p.kchunk > 0) {
    const int64_t kb = z * p.kchunk;
    if (p.symA) ka = kb;
    else A = p.A + (p.transA ? kb : kb * p.lda);
    B = p.B + (p.transB ? kb * p.ldb : kb);
    int64_t kl = p.k - kb;
    p.k = kl < p.kchunk ? kl : p.kchunk;
  }

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  v4d acc[FR][FC];
#pragma unroll
  for (int i = 0; i < FR; ++i)
#pragma unroll
    for (int j = 0; j < FC; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  const int64_t nk = (p.k + BK - 1) / BK;
  const int64_t nk_full = p.k / BK;
  const bool fast = FAST || (p.vecA && p.vecB && m0 + BM <= p.m && n0 + BN <= p.n);
  // Per k step: 0 = fast, op(A) as stored; 1 = fast, op(A) read transposed;
  // 2 = checked element-wise path.  A symmetric A (lower stored) is read as is on
  // and below the diagonal and through its mirror above it.
  auto mode_of = [&](int64_t kt) -> int {
    if (!fast || kt >= nk_full) return 2;
    if (!p.symA) return p.transA ? 1 : 0;
    const int64_t k0 = ka + kt * BK;
    if (m0 >= k0 + BK - 1) return 0;
    if (m0 + BM - 1 < k0) return 1;
    return FAST ? 3 : 2;
  };
  auto a_ptr = [&](int mode, int64_t kt) -> const double* {
    const int64_t k0 = ka + kt * BK;
    return mode == 1 ? A + k0 + m0 * p.lda : A + m0 + k0 * p.lda;
  };
  auto b_ptr = [&](int64_t kt) -> const double* {
    const int64_t k0 = kt * BK;
    return p.transB ? B + n0 + k0 * p.ldb : B + k0 + n0 * p.ldb;
  };

  double ra[PA], rb[PB];
  if (nk > 0) {
    const int mode = mode_of(0);
    if (FAST && mode == 3) {
      IO::load(p, false, a_ptr(0, 0), b_ptr(0), ra, rb);  // B part; A part replaced below
      IO::store(p, false, ra, rb, As[0], Bs[0]);
      __syncthreads();
      sym_diag_to_lds<BM, BK, LDA_S>(p, A, m0, ka, As[0]);
    } else if (FAST || mode != 2) {
      IO::load(p, mode == 1, a_ptr(mode, 0), b_ptr(0), ra, rb);
      IO::store(p, mode == 1, ra, rb, As[0], Bs[0]);
    } else {
      load_a<BM, BK>(p, A, m0, ka, ka + p.k, ra);
      load_b<BN, BK>(p, B, 0, n0, rb);
      store_a<BM, BK, LDA_S>(p, m0, ka, ra, As[0]);
      store_b<BN, BK, LDB_S>(p, rb, Bs[0]);
    }
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const bool more = kt + 1 < nk;
    const int nmode = more ? mode_of(kt + 1) : 2;
    // fast path: next k step prefetched into registers across the MFMAs
    if (more && (FAST || nmode != 2))
      IO::load(p, nmode == 1, a_ptr(nmode == 3 ? 0 : nmode, kt + 1), b_ptr(kt + 1), ra, rb);
    const double* as = As[buf];
    const double* bs = Bs[buf];
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int krow = ks * 4 + (lane >> 4);
      double af[FR], bf[FC];
#pragma unroll
      for (int i = 0; i < FR; ++i) af[i] = as[krow * LDA_S + wr * WM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < FC; ++j) bf[j] = bs[krow * LDB_S + wc * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < FR; ++i)
#pragma unroll
        for (int j = 0; j < FC; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[j], af[i], acc[i][j], 0, 0, 0);
    }
    if (more) {
      if (FAST && nmode == 3) {
        IO::store(p, false, ra, rb, As[buf ^ 1], Bs[buf ^ 1]);
        __syncthreads();
        sym_diag_to_lds<BM, BK, LDA_S>(p, A, m0, ka + (kt + 1) * BK, As[buf ^ 1]);
      } else if (FAST || nmode != 2) {
        IO::store(p, nmode == 1, ra, rb, As[buf ^ 1], Bs[buf ^ 1]);
      } else {
        // edge / unaligned / diagonal-straddling tile: checked loads, not prefetched
        load_a<BM, BK>(p, A, m0, ka + (kt + 1) * BK, ka + p.k, ra);
        load_b<BN, BK>(p, B, (kt + 1) * BK, n0, rb);
        store_a<BM, BK, LDA_S>(p, m0, ka + (kt + 1) * BK, ra, As[buf ^ 1]);
        store_b<BN, BK, LDB_S>(p, rb, Bs[buf ^ 1]);
      }
    }
    __syncthreads();
  }

  // Epilogue: element r of acc[i][j] is C(row, col) with
  //   row = m0 + wr*WM + i*16 + lane%16,  col = n0 + wc*WN + j*16 + lane/16 + 4r.
  // The old C values of one row group are all loaded before any of them is
  // stored: interleaved load / store pairs would each wait a full memory latency
  // (the compiler cannot prove that a store does not alias the next load).
#pragma unroll
  for (int i = 0; i < FR; ++i) {
    const int64_t row = m0 + wr * WM + i * 16 + (lane & 15);
    if (row >= p.m) continue;
    double cold[FC][4];
    if (p.beta != 0.0) {
#pragma unroll
      for (int j = 0; j < FC; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t col = n0 + wc * WN + j * 16 + (lane >> 4) + 4 * r;
          const bool ok = col < p.n && !(p.uplo == 1 && row < col);
          cold[j][r] = ok ? C[row + col * p.ldc] : 0.0;
        }
    }
#pragma unroll
    for (int j = 0; j < FC; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t col = n0 + wc * WN + j * 16 + (lane >> 4) + 4 * r;
        if (col >= p.n) continue;
        if (p.uplo == 1 && row < col) continue;
        double v = p.alpha * acc[i][j][r];
        if (p.beta != 0.0) v += p.beta * cold[j][r];
        C[row + col * p.ldc] = v;
      }
    }
  }
}

constexpr int FAST_BK = 16;

// two consecutive staged elements in one LDS write (even offsets)
__device__ inline void store_pair(double* dst, double2 v) { *reinterpret_cast<double2*>(dst) = v; }
__device__ inline void store_pair(float* dst, double2 v) {
  *reinterpret_cast<float2*>(dst) = make_float2((float)v.x, (float)v.y);
}

__device__ inline v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Interior region: 128 x 128 tiles, BK = FAST_BK, k a multiple of BK, operands 16-byte
// aligned with even leading dimensions, transposes fixed at compile time.  The
// steady-state loop has no control flow besides the loop itself, which keeps the
// accumulators resident in the matrix-core registers.
//
// F32: the staged operands are rounded to FP32 and multiplied with
// v_mfma_f32_16x16x4f32 (FP32 accumulation, twice the FP64 rate).  Its output
// layout differs from the FP64 instruction's: register r of lane l holds row
// 4 (l / 16) + r of the 16 x 16 block instead of l / 16 + 4 r.
template <bool TA, bool TB, bool F32>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
dgemm_fast_kernel(Params p) {
  using S = typename std::conditional<F32, float, double>::type;
  using Acc = typename std::conditional<F32, v4f, v4d>::type;
  constexpr int BM = 128, BN = 128, BK = FAST_BK;
  // LDS row strides.  An operand staged with 16-byte stores (A plain, B
  // transposed) needs an even stride; one staged element by element lands 8
  // lanes on rows 2p (p = 0..7) of one column, which an odd stride (129) spreads
  // over all banks (an even one, 132, folds them onto two).
  constexpr int LDA_S = TA ? BM + 1 : BM + 4;
  constexpr int LDB_S = TB ? BN + 4 : BN + 1;
  constexpr int WM = 64, WN = 64, FR = 4, FC = 4;
  constexpr int PA2 = BM * BK / 2 / NT, PB2 = BN * BK / 2 / NT;
  __shared__ S As[2][BK * LDA_S];
  __shared__ S Bs[2][BK * LDB_S];
  int tm, tn;
  if (p.lower_grid)
    lower_tile_coords(tm, tn);
  else
    tile_coords(p.tiles_m, p.tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  if (p.uplo == 1 && m0 + BM - 1 < n0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  // per-thread global and LDS offsets of the staged double2 pieces
  const double* Ap[PA2];
  const double* Bp[PB2];
  int as_off[PA2], bs_off[PB2];
#pragma unroll
  for (int i = 0; i < PA2; ++i) {
    const int idx = tid + NT * i;
    if (!TA) {
      const int rp = idx % (BM / 2), c = idx / (BM / 2);
      Ap[i] = p.A + m0 + 2 * rp + (int64_t)c * p.lda;
      as_off[i] = c * LDA_S + 2 * rp;
    } else {
      const int cp = idx % (BK / 2), r = idx / (BK / 2);
      Ap[i] = p.A + (m0 + r) * p.lda + 2 * cp;
      as_off[i] = (2 * cp) * LDA_S + r;
    }
  }
#pragma unroll
  for (int i = 0; i < PB2; ++i) {
    const int idx = tid + NT * i;
    if (!TB) {
      const int kp = idx % (BK / 2), j = idx / (BK / 2);
      Bp[i] = p.B + (n0 + j) * p.ldb + 2 * kp;
      bs_off[i] = (2 * kp) * LDB_S + j;
    } else {
      const int jp = idx % (BN / 2), kk = idx / (BN / 2);
      Bp[i] = p.B + n0 + 2 * jp + (int64_t)kk * p.ldb;
      bs_off[i] = kk * LDB_S + 2 * jp;
    }
  }
  const int64_t dA = TA ? BK : BK * p.lda;
  const int64_t dB = TB ? BK * p.ldb : BK;

  double2 ra[PA2], rb[PB2];
#define GEP_FAST_GLOAD(kt_)                                                               \
  {                                                                                       \
    _Pragma("unroll") for (int i = 0; i < PA2; ++i) ra[i] =                               \
        *reinterpret_cast<const double2*>(Ap[i] + (kt_) * dA);                            \
    _Pragma("unroll") for (int i = 0; i < PB2; ++i) rb[i] =                               \
        *reinterpret_cast<const double2*>(Bp[i] + (kt_) * dB);                            \
  }
#define GEP_FAST_LSTORE(buf_)                                                             \
  {                                                                                       \
    _Pragma("unroll") for (int i = 0; i < PA2; ++i) {                                     \
      if (!TA) {                                                                          \
        store_pair(&As[buf_][as_off[i]], ra[i]);                                          \
      } else {                                                                            \
        As[buf_][as_off[i]] = (S)ra[i].x;                                                 \
        As[buf_][as_off[i] + LDA_S] = (S)ra[i].y;                                         \
      }                                                                                   \
    }                                                                                     \
    _Pragma("unroll") for (int i = 0; i < PB2; ++i) {                                     \
      if (!TB) {                                                                          \
        Bs[buf_][bs_off[i]] = (S)rb[i].x;                                                 \
        Bs[buf_][bs_off[i] + LDB_S] = (S)rb[i].y;                                         \
      } else {                                                                            \
        store_pair(&Bs[buf_][bs_off[i]], rb[i]);                                          \
      }                                                                                   \
    }                                                                                     \
  }
#define GEP_FAST_COMPUTE(buf_)                                                            \
  {                                                                                       \
    const S* as = As[buf_];                                                               \
    const S* bs = Bs[buf_];                                                               \
    _Pragma("unroll") for (int ks = 0; ks < BK / 4; ++ks) {                               \
      const int krow = ks * 4 + (lane >> 4);                                              \
      S af[FR], bf[FC];                                                                   \
      _Pragma("unroll") for (int i = 0; i < FR; ++i) af[i] =                              \
          as[krow * LDA_S + wr * WM + i * 16 + (lane & 15)];                              \
      _Pragma("unroll") for (int j = 0; j < FC; ++j) bf[j] =                              \
          bs[krow * LDB_S + wc * WN + j * 16 + (lane & 15)];                              \
      _Pragma("unroll") for (int i = 0; i < FR; ++i)                                      \
          _Pragma("unroll") for (int j = 0; j < FC; ++j) acc[i][j] =                      \
              mfma16(bf[j], af[i], acc[i][j]);                                            \
    }                                                                                     \
  }

  Acc acc[FR][FC];
#pragma unroll
  for (int i = 0; i < FR; ++i)
#pragma unroll
    for (int j = 0; j < FC; ++j) acc[i][j] = Acc{0, 0, 0, 0};

  const int64_t nk = p.k / BK;
  GEP_FAST_GLOAD(0)
  GEP_FAST_LSTORE(0)
  __syncthreads();
  for (int64_t kt = 0; kt + 1 < nk; ++kt) {
    GEP_FAST_GLOAD(kt + 1)
    GEP_FAST_COMPUTE(kt & 1)
    GEP_FAST_LSTORE((kt + 1) & 1)
    __syncthreads();
  }
  GEP_FAST_COMPUTE((nk - 1) & 1)
#undef GEP_FAST_GLOAD
#undef GEP_FAST_LSTORE
#undef GEP_FAST_COMPUTE

  // old C values of a row group loaded together before the stores (see dgemm_tile)
  const double beta_epi = p.beta;
#pragma unroll
  for (int i = 0; i < FR; ++i) {
    const int64_t row = m0 + wr * WM + i * 16 + (lane & 15);
    double cold[FC][4];
    if (beta_epi != 0.0) {
#pragma unroll
      for (int j = 0; j < FC; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t col =
              n0 + wc * WN + j * 16 + (F32 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r);
          cold[j][r] = (p.uplo == 1 && row < col) ? 0.0 : p.C[row + col * p.ldc];
        }
    }
#pragma unroll
    for (int j = 0; j < FC; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t col =
            n0 + wc * WN + j * 16 + (F32 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r);
        if (p.uplo == 1 && row < col) continue;
        double v = p.alpha * (double)acc[i][j][r];
        if (beta_epi != 0.0) v += beta_epi * cold[j][r];
        p.C[row + col * p.ldc] = v;
      }
    }
  }
}

template <int BM, int BN, int BK, bool FAST = false>
void launch(const Gemm& g, hipStream_t s, int64_t kchunk = 0, int nsplit = 1) {
  Params p;
  p.kchunk = kchunk;
  p.m = g.m; p.n = g.n; p.k = g.k;
  p.alpha = g.alpha; p.beta = g.beta;
  p.A = g.A; p.lda = g.lda; p.B = g.B; p.ldb = g.ldb; p.C = g.C; p.ldc = g.ldc;
  p.sA = g.strideA; p.sB = g.strideB; p.sC = g.strideC;
  p.transA = g.transA; p.transB = g.transB; p.symA = g.symA; p.uplo = g.uplo;
  p.tiles_m = (int)cdiv(g.m, BM);
  p.tiles_n = (int)cdiv(g.n, BN);
  const bool kshift_ok = kchunk == 0 || (kchunk % 2 == 0);
  p.vecA = kshift_ok && ((uintptr_t)g.A % 16 == 0) && (g.lda % 2 == 0) &&
           (g.batch == 1 || g.strideA % 2 == 0);
  p.vecB = kshift_ok && ((uintptr_t)g.B % 16 == 0) && (g.ldb % 2 == 0) &&
           (g.batch == 1 || g.strideB % 2 == 0);
  dim3 grid((unsigned)((int64_t)p.tiles_m * p.tiles_n), (unsigned)(kchunk > 0 ? nsplit : g.batch));
  if (BM == 64 && BN == 64 && BK == 16 && !FAST)
    hipLaunchKernelGGL(dgemm_kernel_64, grid, dim3(NT), 0, s, p);
  else
    hipLaunchKernelGGL((dgemm_kernel<BM, BN, BK, FAST>), grid, dim3(NT), 0, s, p);
  GEP_LAUNCH_CHECK();
}

__global__ void splitk_reduce(int64_t m, int64_t n, int nsplit, const double* __restrict__ work,
                              double alpha, double beta, double* __restrict__ C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t i = idx % m, j = idx / m;
  double acc = 0.0;
  for (int z = 0; z < nsplit; ++z) acc += work[(size_t)z * m * n + idx];
  double v = alpha * acc;
  if (beta != 0.0) v += beta * C[i + j * ldc];
  C[i + j * ldc] = v;
}

template <bool F32>
void launch_fast_kernel(const Gemm& g, const Params& p, dim3 grid, hipStream_t s) {
  if (!g.transA && !g.transB)
    hipLaunchKernelGGL((dgemm_fast_kernel<false, false, F32>), grid, dim3(NT), 0, s, p);
  else if (g.transA && !g.transB)
    hipLaunchKernelGGL((dgemm_fast_kernel<true, false, F32>), grid, dim3(NT), 0, s, p);
  else if (!g.transA && g.transB)
    hipLaunchKernelGGL((dgemm_fast_kernel<false, true, F32>), grid, dim3(NT), 0, s, p);
  else
    hipLaunchKernelGGL((dgemm_fast_kernel<true, true, F32>), grid, dim3(NT), 0, s, p);
}

void launch_fast(const Gemm& g, hipStream_t s) {
  Params p;
  p.m = g.m; p.n = g.n; p.k = g.k;
  p.alpha = g.alpha; p.beta = g.beta;
  p.A = g.A; p.lda = g.lda; p.B = g.B; p.ldb = g.ldb; p.C = g.C; p.ldc = g.ldc;
  p.sA = p.sB = p.sC = 0;
  p.transA = g.transA; p.transB = g.transB; p.symA = 0; p.uplo = g.uplo;
  p.tiles_m = (int)(g.m / 128);
  p.tiles_n = (int)(g.n / 128);
  p.kchunk = 0;
  p.vecA = p.vecB = 1;
  p.lower_grid = (g.uplo == 1 && g.m == g.n) ? 1 : 0;
  dim3 grid((unsigned)(p.lower_grid ? (int64_t)p.tiles_m * (p.tiles_m + 1) / 2
                                    : (int64_t)p.tiles_m * p.tiles_n));
  // algorithmic flops: every element of C that is asked for (lower triangle with
  // the diagonal when uplo = 1) costs 2k
  const double elems = g.uplo == 1 ? 0.5 * (double)g.n * (double)(g.n + 1) : (double)g.m * g.n;
  ProbeScope probe(PROBE_GEMM, s, 2.0 * (double)g.k * elems);
  if (math_mode() == MathMode::Fp32)
    launch_fast_kernel<true>(g, p, grid, s);
  else
    launch_fast_kernel<false>(g, p, grid, s);
  GEP_LAUNCH_CHECK();
}

constexpr int64_t KCHUNK_MIN = 512;
constexpr int MAX_SPLIT = 64;

int choose_split(int64_t m, int64_t n, int64_t k) {
  const int64_t tiles = cdiv(m, 64) * cdiv(n, 64);
  if (tiles >= 128 || k < 2 * KCHUNK_MIN) return 1;
  int64_t want = cdiv(256, tiles);
  int64_t by_k = k / KCHUNK_MIN;
  int64_t sp = want < by_k ? want : by_k;
  if (sp > MAX_SPLIT) sp = MAX_SPLIT;
  return sp < 2 ? 1 : (int)sp;
}

// Symmetric-operand products here are tall and skinny (C = A22 V, n = band width,
// k = m): m / 64 tiles of K = m each leave the CUs unevenly loaded.  Split K so the
// launch has about 1024 workgroups, limited by the scratch the caller passes.
int choose_split_sym(int64_t m, int64_t n, int64_t k, size_t work_elems) {
  const int64_t tiles = cdiv(m, 64) * cdiv(n, 64);
  int64_t sp = cdiv(2048, tiles);
  const int64_t by_k = k / KCHUNK_MIN;
  if (sp > by_k) sp = by_k;
  const int64_t by_work = (int64_t)(work_elems / ((size_t)m * (size_t)n));
  if (sp > by_work) sp = by_work;
  if (sp > MAX_SPLIT) sp = MAX_SPLIT;
  return sp < 2 ? 1 : (int)sp;
}

}  // namespace

void gemm_grouped(const GemmDesc* desc, int count, int64_t max_m, int64_t max_n, hipStream_t s) {
  if (count <= 0 || max_m <= 0 || max_n <= 0) return;
  dim3 grid((unsigned)(cdiv(max_m, 64) * cdiv(max_n, 64)), (unsigned)count);
  hipLaunchKernelGGL((dgemm_grouped_kernel<64, 64, 16>), grid, dim3(NT), 0, s, desc);
  GEP_LAUNCH_CHECK();
}

size_t splitk_work_elems(int64_t m, int64_t n, int64_t k) {
  return (size_t)choose_split(m, n, k) * (size_t)m * (size_t)n;
}

void gemm(const Gemm& g, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return;
  if (g.k <= 0 && g.beta == 1.0) return;
  if (g.work && g.batch == 1 && g.uplo == 0) {
    const int sp = g.symA ? choose_split_sym(g.m, g.n, g.k, g.work_elems)
                          : choose_split(g.m, g.n, g.k);
    if (sp > 1 && g.work_elems >= (size_t)sp * g.m * g.n) {
      const int64_t kc = round_up(cdiv(g.k, sp), 16);
      const int nsplit = (int)cdiv(g.k, kc);
      Gemm h = g;
      h.alpha = 1.0; h.beta = 0.0; h.C = g.work; h.ldc = g.m; h.strideC = g.m * g.n;
      launch<64, 64, 16>(h, s, kc, nsplit);
      const int64_t tot = g.m * g.n;
      hipLaunchKernelGGL(splitk_reduce, dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, s, g.m, g.n,
                         nsplit, (const double*)g.work, g.alpha, g.beta, g.C, g.ldc);
      GEP_LAUNCH_CHECK();
      return;
    }
  }
  const int64_t t128 = cdiv(g.m, 128) * cdiv(g.n, 128) * g.batch;
  if (t128 >= 256 || (g.m > 64 && g.n > 64 && t128 >= 128)) {
    // interior tiles on the unchecked kernel, edge strips / k tail on the checked one
    constexpr int BM = 128, BN = 128, BK = FAST_BK;
    const int64_t mm = (g.m / BM) * BM, nm = (g.n / BN) * BN, km = (g.k / BK) * BK;
    const bool aligned = ((uintptr_t)g.A % 16 == 0) && (g.lda % 2 == 0) &&
                         ((uintptr_t)g.B % 16 == 0) && (g.ldb % 2 == 0);
    bool ok = aligned && g.batch == 1 && mm > 0 && nm > 0 && km > 0;
    ok = ok && !g.symA;
    if (g.uplo == 1) ok = ok && g.m == g.n;
    if (!ok) {
      launch<BM, BN, 16>(g, s);
      return;
    }
    Gemm in = g;
    in.m = mm; in.n = nm; in.k = km;
    launch_fast(in, s);
    if (g.k > km) {  // C_interior += alpha op(A)(:, km:) op(B)(km:, :)
      Gemm t = in;
      t.k = g.k - km;
      t.beta = 1.0;
      t.A = g.transA ? g.A + km : g.A + km * g.lda;
      t.B = g.transB ? g.B + km * g.ldb : g.B + km;
      launch<64, 64, 16>(t, s);
    }
    if (g.n > nm) {  // right strip: columns nm.., rows 0.. (lower-only: rows nm.. only)
      Gemm r = g;
      const int64_t r0 = g.uplo == 1 ? nm : 0;
      r.m = g.m - r0;
      r.n = g.n - nm;
      r.B = g.transB ? g.B + nm : g.B + nm * g.ldb;
      if (!g.symA) r.A = g.transA ? g.A + r0 * g.lda : g.A + r0;
      r.C = g.C + r0 + nm * g.ldc;
      if (g.symA) {
        r.m = g.m;  // symmetric operand: rows must start at 0 (mm == m, so r0 == 0 here)
      }
      launch<64, 64, 16>(r, s);
    }
    if (g.m > mm) {  // bottom strip: rows mm.., columns 0..nm (not reached for symmetric A)
      Gemm bt = g;
      bt.m = g.m - mm;
      bt.n = nm;
      bt.uplo = 0;
      bt.A = g.transA ? g.A + mm * g.lda : g.A + mm;
      bt.C = g.C + mm;
      launch<64, 64, 16>(bt, s);
    }
    return;
  } else {
    launch<64, 64, 16>(g, s);
  }
}

}  // namespace gep

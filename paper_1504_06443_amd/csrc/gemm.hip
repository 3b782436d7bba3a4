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
  int64_t kchunk;  // > 0: batch index z sums k in [z*kchunk, (z+1)*kchunk) into C + z*sC
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

template <int BM, int BK>
__device__ inline void load_a(const Params& p, const double* __restrict__ A, int64_t m0, int64_t k0,
                              double* ra) {
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
      if (r < p.m && c < p.k) {
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
      ra[i] = (r < p.m && c < p.k) ? A[c + r * p.lda] : 0.0;
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

template <int BM, int BN, int BK>
__device__ inline void dgemm_tile(Params& p, int tm, int tn, int64_t z);

template <int BM, int BN, int BK>
__global__ void __launch_bounds__(NT) dgemm_kernel(Params p) {
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, tm, tn);
  dgemm_tile<BM, BN, BK>(p, tm, tn, blockIdx.y);
}

// Problems whose sizes live in device memory (written by an earlier kernel).
template <int BM, int BN, int BK>
__global__ void __launch_bounds__(NT) dgemm_grouped_kernel(const GemmDesc* __restrict__ desc) {
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
  dgemm_tile<BM, BN, BK>(p, (int)blockIdx.x % tiles_m, (int)blockIdx.x / tiles_m, 0);
}

template <int BM, int BN, int BK>
__device__ inline void dgemm_tile(Params& p, int tm, int tn, int64_t z) {
  constexpr int PAD = 4;
  constexpr int LDA_S = BM + PAD, LDB_S = BN + PAD;
  constexpr int WM = BM / 2, WN = BN / 2;  // per-wave sub-tile
  constexpr int FR = WM / 16, FC = WN / 16;
  constexpr int PA = BM * BK / NT, PB = BN * BK / NT;
  __shared__ double As[2][BK * LDA_S];
  __shared__ double Bs[2][BK * LDB_S];

  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  if (p.uplo == 1 && m0 + BM - 1 < n0) return;  // strictly upper tile

  const double* __restrict__ A = p.A + z * p.sA;
  const double* __restrict__ B = p.B + z * p.sB;
  double* __restrict__ C = p.C + z * p.sC;
  if (p.kchunk > 0) {
    const int64_t kb = z * p.kchunk;
    A = p.A + (p.transA ? kb : kb * p.lda);
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
  double ra[PA], rb[PB];
  if (nk > 0) {
    load_a<BM, BK>(p, A, m0, 0, ra);
    load_b<BN, BK>(p, B, 0, n0, rb);
    store_a<BM, BK, LDA_S>(p, m0, 0, ra, As[0]);
    store_b<BN, BK, LDB_S>(p, rb, Bs[0]);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) {
      load_a<BM, BK>(p, A, m0, (kt + 1) * BK, ra);
      load_b<BN, BK>(p, B, (kt + 1) * BK, n0, rb);
    }
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
      store_a<BM, BK, LDA_S>(p, m0, (kt + 1) * BK, ra, As[buf ^ 1]);
      store_b<BN, BK, LDB_S>(p, rb, Bs[buf ^ 1]);
    }
    __syncthreads();
  }

  // Epilogue: element r of acc[i][j] is C(row, col) with
  //   row = m0 + wr*WM + i*16 + lane%16,  col = n0 + wc*WN + j*16 + lane/16 + 4r.
#pragma unroll
  for (int i = 0; i < FR; ++i) {
    const int64_t row = m0 + wr * WM + i * 16 + (lane & 15);
    if (row >= p.m) continue;
#pragma unroll
    for (int j = 0; j < FC; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t col = n0 + wc * WN + j * 16 + (lane >> 4) + 4 * r;
        if (col >= p.n) continue;
        if (p.uplo == 1 && row < col) continue;
        double* c = C + row + col * p.ldc;
        double v = p.alpha * acc[i][j][r];
        if (p.beta != 0.0) v += p.beta * *c;
        *c = v;
      }
    }
  }
}

template <int BM, int BN, int BK>
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
  dim3 grid((unsigned)((int64_t)p.tiles_m * p.tiles_n), (unsigned)(kchunk > 0 ? nsplit : g.batch));
  hipLaunchKernelGGL((dgemm_kernel<BM, BN, BK>), grid, dim3(NT), 0, s, p);
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
  if (g.work && g.batch == 1 && !g.symA && g.uplo == 0) {
    const int sp = choose_split(g.m, g.n, g.k);
    if (sp > 1 && g.work_elems >= (size_t)sp * g.m * g.n) {
      const int64_t kc = cdiv(g.k, sp);
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
    launch<128, 128, 16>(g, s);
  } else if (cdiv(g.m, 128) * cdiv(g.n, 64) * g.batch >= 128 && g.m > 64) {
    launch<128, 64, 16>(g, s);
  } else {
    launch<64, 64, 16>(g, s);
  }
}

}  // namespace gep

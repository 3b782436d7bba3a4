// Symmetric tridiagonal eigensolver: divide and conquer (Cuppen's rank-one
// tearing, Dongarra-Sorensen deflation, secular equations solved per root with a
// two-pole rational model, Gu-Eisenstat recomputation of z, merge by MFMA GEMM),
// and Sturm bisection for the eigenvalue-only job.  This is the "D&C" phase of
// the SEP solvers timed in Table 3.
//
// Tree: node (t, i) of depth t covers rows [floor(i n / 2^t), floor((i+1) n / 2^t));
// leaves are at the smallest depth D whose nodes have <= LEAF rows.  All merges of
// one depth run together, each step one launch over (merge, item).
//
// Storage: Z (n x n) holds the eigenvectors of node [lo, hi) in its diagonal block
// Z[lo:hi, lo:hi] (zeros elsewhere), lam[lo:hi] the eigenvalues ascending.  Per
// merge the same [lo, hi) range of the work arrays is used.
#include "common.h"
#include "internal.h"

namespace gep {
namespace {

constexpr int LEAF = 64;
constexpr double EPS = 2.220446049250313e-16;

enum : int { TOP = 0, MIXED = 1, BOTTOM = 2 };

struct Node {
  int64_t lo, mid, hi;
};

__host__ __device__ inline int64_t bound(int64_t i, int64_t n, int t) {
  return (int64_t)(((__int128)i * n) >> t);
}

__host__ __device__ inline Node merge_node(int64_t n, int t, int64_t i) {
  Node nd;
  nd.lo = bound(i, n, t);
  nd.hi = bound(i + 1, n, t);
  nd.mid = bound(2 * i + 1, n, t + 1);
  return nd;
}

// Per-merge scalars.
struct MergeInfo {
  double rho;   // 2 |e(mid-1)| (z normalised to unit length)
  double sigma; // sign of e(mid-1)
  int32_t K;    // non-deflated count
  int32_t K1, Km, K2;
  int32_t nrot;
  int32_t ndefl;
};

struct Work {
  double* dd;     // sorted D (n)
  double* zz;     // sorted z (n)
  int32_t* col;   // sorted position -> local column (n)
  double* sd;     // non-deflated D (n)
  double* sz;     // non-deflated z (n)
  int32_t* scol;  // non-deflated -> local column (n)
  int32_t* sclass;
  int32_t* urow;  // non-deflated index -> row of U / column of G
  int32_t* gcol;  // G column -> local column of Z (non-deflated then deflated)
  double* dlam;   // deflated eigenvalues (n)
  int32_t* rot_i; // rotations (n)
  int32_t* rot_j;
  double* rot_c;
  double* rot_s;
  int32_t* orig;  // secular root -> origin index (n)
  double* tau;    // secular root -> offset from origin (n)
  double* zhat;   // (n)
  double* lamw;   // eigenvalues being merged (n)
  MergeInfo* info;  // per merge
  GemmDesc* desc;   // 2 per merge
  double* flops;    // merge products' flops, summed over the levels (1)
  double* G;      // n x n
  double* U;      // n x n
  double* Out;    // n x n
};

// ---------------------------------------------------------------- leaves
// One wave per leaf: tear the boundaries, implicit QL with Wilkinson shifts,
// rotations applied by all lanes (lane = row of the leaf's eigenvector matrix),
// then sort.
__global__ void __launch_bounds__(64)
leaf_kernel(int64_t n, int D, const double* __restrict__ d, const double* __restrict__ e,
            double* __restrict__ lam, double* __restrict__ Z, int64_t ldz, int32_t* info,
            int maxit) {
  __shared__ double zs[LEAF][LEAF + 1];
  __shared__ double dl[LEAF], el[LEAF], cs[LEAF], sn[LEAF];
  __shared__ int nrot_sh, fail_sh, top_sh;
  const int lane = threadIdx.x;
  const int64_t lo = bound(blockIdx.x, n, D), hi = bound(blockIdx.x + 1, n, D);
  const int m = (int)(hi - lo);
  for (int i = lane; i < m; i += 64) {
    double di = d[lo + i];
    if (i == 0 && lo > 0) di -= fabs(e[lo - 1]);
    if (i == m - 1 && hi < n) di -= fabs(e[hi - 1]);
    dl[i] = di;
    el[i] = (i + 1 < m) ? e[lo + i] : 0.0;
  }
  for (int j = 0; j < m; ++j)
    if (lane < m) zs[lane][j] = (lane == j) ? 1.0 : 0.0;
  if (lane == 0) fail_sh = 0;
  __syncthreads();
  for (int l = 0; l < m; ++l) {
    int iter = 0;
    for (;;) {
      // lane 0 runs the scalar recurrence, all lanes then rotate their row
      if (lane == 0) {
        int mm = l;
        for (; mm + 1 < m; ++mm) {
          const double dd = fabs(dl[mm]) + fabs(dl[mm + 1]);
          if (fabs(el[mm]) <= EPS * dd || fabs(el[mm]) < 1e-300) break;
        }
        int nrot = 0;
        if (mm != l) {
          if (++iter > maxit) {
            fail_sh = 1;
          } else {
            double g = (dl[l + 1] - dl[l]) / (2.0 * el[l]);
            double r = hypot(g, 1.0);
            g = dl[mm] - dl[l] + el[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool early = false;
            for (int i = mm - 1; i >= l; --i) {
              const double f = s * el[i], bb = c * el[i];
              r = hypot(f, g);
              el[i + 1] = r;
              if (r == 0.0) {
                dl[i + 1] -= p;
                el[mm] = 0.0;
                early = true;
                break;
              }
              s = f / r;
              c = g / r;
              g = dl[i + 1] - p;
              r = (dl[i] - g) * s + 2.0 * c * bb;
              p = s * r;
              dl[i + 1] = g + p;
              g = c * r - bb;
              cs[nrot] = c;
              sn[nrot] = s;
              ++nrot;
            }
            if (!early) {
              dl[l] -= p;
              el[l] = g;
              el[mm] = 0.0;
            }
            top_sh = mm - 1;  // rotation t acts on columns (mm-1-t, mm-t)
          }
        } else {
          nrot = -1;  // converged for this l
        }
        nrot_sh = nrot;
      }
      __syncthreads();
      const int nrot = nrot_sh;
      if (nrot < 0 || fail_sh) break;
      if (nrot > 0) {
        const int top = top_sh;
        if (lane < m) {
          for (int t = 0; t < nrot; ++t) {
            const int ii = top - t;
            const double f = zs[lane][ii + 1];
            const double zi = zs[lane][ii];
            zs[lane][ii + 1] = sn[t] * zi + cs[t] * f;
            zs[lane][ii] = cs[t] * zi - sn[t] * f;
          }
        }
      }
      __syncthreads();
    }
    if (fail_sh) break;
  }
  if (fail_sh && lane == 0 && info) atomicCAS(info, 0, (int32_t)(lo + 1));
  __syncthreads();
  // sort ascending (rank by value, ties by index) and write out
  if (lane < m) {
    const double v = dl[lane];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double w = dl[j];
      rank += (w < v) || (w == v && j < lane);
    }
    lam[lo + rank] = v;
    for (int i = 0; i < m; ++i) Z[(lo + i) + (lo + rank) * ldz] = zs[i][lane];
  }
}

// ---------------------------------------------------------------- merge steps
// (a) z, D and their merged ascending order; one workgroup per merge.
__global__ void merge_prepare(int64_t n, int t, const double* __restrict__ e,
                              const double* __restrict__ lam, const double* __restrict__ Z,
                              int64_t ldz, Work w) {
  const Node nd = merge_node(n, t, blockIdx.x);
  const int64_t N = nd.hi - nd.lo, n1 = nd.mid - nd.lo;
  const double beta = e[nd.mid - 1];
  const double sgn = beta >= 0.0 ? 1.0 : -1.0;
  const double* L = lam + nd.lo;
  if (threadIdx.x == 0) {
    w.info[blockIdx.x].rho = 2.0 * fabs(beta);
    w.info[blockIdx.x].sigma = sgn;
  }
  const double r2 = 0.7071067811865476;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    const double D = L[i];
    double z;
    int64_t pos;
    if (i < n1) {
      z = Z[(nd.mid - 1) + (nd.lo + i) * ldz];
      // rank among the right half: count of right values < D
      int64_t a = n1, b = N;
      while (a < b) {
        const int64_t m = (a + b) / 2;
        if (L[m] < D) a = m + 1; else b = m;
      }
      pos = i + (a - n1);
    } else {
      z = sgn * Z[nd.mid + (nd.lo + i) * ldz];
      int64_t a = 0, b = n1;  // count of left values <= D
      while (a < b) {
        const int64_t m = (a + b) / 2;
        if (L[m] <= D) a = m + 1; else b = m;
      }
      pos = (i - n1) + a;
    }
    w.dd[nd.lo + pos] = D;
    w.zz[nd.lo + pos] = z * r2;
    w.col[nd.lo + pos] = (int32_t)i;
  }
}

// (b) deflation scan (sequential per merge, staged through LDS in chunks).
constexpr int CHUNK = 1024;
__global__ void __launch_bounds__(256) merge_deflate(int64_t n, int t, Work w) {
  __shared__ double cd[CHUNK], cz[CHUNK];
  __shared__ int32_t cc[CHUNK];
  __shared__ double red[2][4];
  __shared__ double tol_sh;
  const Node nd = merge_node(n, t, blockIdx.x);
  const int64_t lo = nd.lo, N = nd.hi - nd.lo, n1 = nd.mid - nd.lo;
  MergeInfo* mi = &w.info[blockIdx.x];
  const double rho = mi->rho;
  const int tid = threadIdx.x;
  // tolerance: 8 eps max(max|D|, rho)
  double md = 0.0;
  for (int64_t i = tid; i < N; i += 256) md = fmax(md, fabs(w.dd[lo + i]));
  for (int off = 32; off > 0; off >>= 1) md = fmax(md, __shfl_xor(md, off, 64));
  if ((tid & 63) == 0) red[0][tid >> 6] = md;
  __syncthreads();
  if (tid == 0) {
    double m = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
    tol_sh = 8.0 * EPS * fmax(m, rho);
  }
  __syncthreads();
  const double tol = tol_sh;
  // sequential scan by thread 0 over chunks staged in LDS
  int K = 0, nrot = 0, ndefl = 0;
  int pj = -1;            // pending candidate (sorted position)
  double pd = 0, pz = 0;  // its (possibly rotated) D and z
  int pcol = 0, pcls = 0;
  int32_t* cls_of = w.sclass + lo;  // temp: class per local column (reused below)
  for (int64_t i = tid; i < N; i += 256) cls_of[i] = (i < n1) ? TOP : BOTTOM;
  __syncthreads();
  for (int64_t c0 = 0; c0 < N; c0 += CHUNK) {
    const int len = (int)((N - c0) < CHUNK ? (N - c0) : CHUNK);
    for (int i = tid; i < len; i += 256) {
      cd[i] = w.dd[lo + c0 + i];
      cz[i] = w.zz[lo + c0 + i];
      cc[i] = w.col[lo + c0 + i];
    }
    __syncthreads();
    if (tid == 0) {
      for (int i = 0; i < len; ++i) {
        const double dj = cd[i], zj = cz[i];
        const int colj = cc[i];
        if (rho * fabs(zj) <= tol) {  // negligible coupling: deflate
          w.dlam[lo + ndefl] = dj;
          w.gcol[lo + (N - 1 - ndefl)] = colj;  // deflated columns fill G from the back
          ++ndefl;
          continue;
        }
        if (pj < 0) {
          pj = 1; pd = dj; pz = zj; pcol = colj; pcls = cls_of[colj];
          continue;
        }
        const double tau = hypot(pz, zj);
        const double c = zj / tau, s = pz / tau;
        if (fabs((dj - pd) * c * s) <= tol) {
          // rotate (pending, j): new pending column deflates, j carries tau
          const int cj = cls_of[colj];
          const int nc = (cj == pcls) ? cj : MIXED;
          w.rot_i[lo + nrot] = pcol;
          w.rot_j[lo + nrot] = colj;
          w.rot_c[lo + nrot] = c;
          w.rot_s[lo + nrot] = s;
          ++nrot;
          const double dp = pd * c * c + dj * s * s;
          const double dn = pd * s * s + dj * c * c;
          w.dlam[lo + ndefl] = dp;
          w.gcol[lo + (N - 1 - ndefl)] = pcol;
          ++ndefl;
          cls_of[pcol] = nc;
          cls_of[colj] = nc;
          pd = dn; pz = tau; pcol = colj; pcls = nc;
        } else {
          w.sd[lo + K] = pd;
          w.sz[lo + K] = pz;
          w.scol[lo + K] = pcol;
          ++K;
          pd = dj; pz = zj; pcol = colj; pcls = cls_of[colj];
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (pj >= 0) {
      w.sd[lo + K] = pd;
      w.sz[lo + K] = pz;
      w.scol[lo + K] = pcol;
      ++K;
    }
    mi->K = K;
    mi->nrot = nrot;
    mi->ndefl = ndefl;
  }
  __syncthreads();
  // order the non-deflated columns [TOP | MIXED | BOTTOM] for the merge GEMMs
  if (tid == 0) {
    int k1 = 0, km = 0, k2 = 0;
    for (int q = 0; q < K; ++q) {
      const int c = cls_of[w.scol[lo + q]];
      k1 += c == TOP;
      km += c == MIXED;
      k2 += c == BOTTOM;
    }
    int o1 = 0, om = k1, o2 = k1 + km;
    for (int q = 0; q < K; ++q) {
      const int col = w.scol[lo + q];
      const int c = cls_of[col];
      const int g = (c == TOP) ? o1++ : (c == MIXED) ? om++ : o2++;
      w.urow[lo + q] = g;
      w.gcol[lo + g] = col;
    }
    mi->K1 = k1;
    mi->Km = km;
    mi->K2 = k2;
    // deflated columns were stored from the back in reverse order; flip them so
    // G column K + q holds deflated eigenvalue q
    for (int q = 0; q < ndefl / 2; ++q) {
      const int a = (int)(N - 1 - q), b = (int)(N - ndefl + q);
      const int32_t tmp = w.gcol[lo + a];
      w.gcol[lo + a] = w.gcol[lo + b];
      w.gcol[lo + b] = tmp;
    }
  }
}

// (c) apply the deflation rotations to the columns of the node's block of Z.
__global__ void merge_rotate(int64_t n, int t, Work w, double* __restrict__ Z, int64_t ldz) {
  const Node nd = merge_node(n, t, blockIdx.y);
  const int64_t N = nd.hi - nd.lo;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= N) return;
  const int nrot = w.info[blockIdx.y].nrot;
  double* zr = Z + nd.lo + row + nd.lo * ldz;
  for (int r = 0; r < nrot; ++r) {
    const int64_t i = w.rot_i[nd.lo + r], j = w.rot_j[nd.lo + r];
    const double c = w.rot_c[nd.lo + r], s = w.rot_s[nd.lo + r];
    const double a = zr[i * ldz], b = zr[j * ldz];
    // new pending (deflated) = c*q_i - s*q_j ; new j = s*q_i + c*q_j
    zr[i * ldz] = c * a - s * b;
    zr[j * ldz] = s * a + c * b;
  }
}

// w(x) = 1/rho + sum_l z_l^2 / (D_l - x) in coordinates relative to the origin pole.
// (d) secular equation, one thread per root.
// Sum over the aligned group of SEC_LANES lanes that share one root.
constexpr int SEC_LANES = 8;
__device__ inline double group_sum(double v) {
#pragma unroll
  for (int off = 1; off < SEC_LANES; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One root per group of SEC_LANES lanes: the lanes split the pole sums (terms
// l = sub, sub + SEC_LANES, ...) and every lane gets the group's totals, so all
// lanes of a group take the same steps and the same convergence decision.
__global__ void merge_secular(int64_t n, int t, Work w, int32_t* info) {
  const Node nd = merge_node(n, t, blockIdx.y);
  const MergeInfo mi = w.info[blockIdx.y];
  const int K = mi.K;
  const int sub = threadIdx.x & (SEC_LANES - 1);
  const int q = blockIdx.x * (blockDim.x / SEC_LANES) + threadIdx.x / SEC_LANES;
  if (q >= K) return;  // whole groups leave together
  const double* d = w.sd + nd.lo;
  const double* z = w.sz + nd.lo;
  const double rho = mi.rho;
  const double rrho = 1.0 / rho;
  int o;
  double lo, hi;
  if (q == K - 1) {
    double zs = 0.0;
    for (int l = sub; l < K; l += SEC_LANES) zs += z[l] * z[l];
    zs = group_sum(zs);
    o = q;
    lo = 0.0;
    hi = rho * zs;
  } else {
    const double gap = d[q + 1] - d[q];
    const double mid = 0.5 * gap;
    double wp = 0.0;
    for (int l = sub; l < K; l += SEC_LANES) wp += z[l] * z[l] / ((d[l] - d[q]) - mid);
    const double wv = rrho + group_sum(wp);
    if (wv >= 0.0) {
      o = q; lo = 0.0; hi = mid;
    } else {
      o = q + 1; lo = -mid; hi = 0.0;
    }
  }
  const double dorg = d[o];
  double tau = 0.5 * (lo + hi);
  bool conv = false;
  for (int it = 0; it < 200; ++it) {
    double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
    for (int l = sub; l < K; l += SEC_LANES) {
      const double del = (d[l] - dorg) - tau;
      const double r = z[l] / del;
      if (l <= q) { psi += z[l] * r; dpsi += r * r; }
      else { phi += z[l] * r; dphi += r * r; }
    }
    psi = group_sum(psi);
    dpsi = group_sum(dpsi);
    phi = group_sum(phi);
    dphi = group_sum(dphi);
    const double wv = rrho + psi + phi;
    const double err = 8.0 * (rrho + fabs(psi) + fabs(phi)) + fabs(tau) * (dpsi + dphi);
    if (fabs(wv) <= EPS * err) { conv = true; break; }
    if (wv < 0.0) lo = tau; else hi = tau;
    if (hi - lo <= 2.0 * EPS * fmax(fabs(lo), fabs(hi))) { conv = true; break; }
    // two-pole rational model c + s/(dq - eta) + S/(dq1 - eta) around tau
    const double dq = (d[q] - dorg) - tau;
    double step;
    bool have = false;
    if (q == K - 1) {
      const double s = dpsi * dq * dq;
      const double c = wv - s / dq;  // psi part matched, no right pole
      if (c > 0.0) { step = dq + s / c; have = true; }
    } else {
      const double dq1 = (d[q + 1] - dorg) - tau;
      const double s = dpsi * dq * dq, S = dphi * dq1 * dq1;
      const double c = wv - s / dq - S / dq1;
      const double B = c * (dq + dq1) + s + S;
      const double C = dq * dq1 * wv;
      if (c == 0.0) {
        if (B != 0.0) { step = C / B; have = true; }
      } else {
        const double disc = B * B - 4.0 * c * C;
        if (disc >= 0.0) {
          const double sq = sqrt(disc);
          const double r1 = (B >= 0.0) ? (B + sq) / (2.0 * c) : (B - sq) / (2.0 * c);
          const double r2 = (r1 != 0.0) ? C / (c * r1) : 0.0;
          const double t1 = tau + r1, t2 = tau + r2;
          if (t2 > lo && t2 < hi) { step = r2; have = true; }
          else if (t1 > lo && t1 < hi) { step = r1; have = true; }
        }
      }
    }
    double nt = have ? tau + step : 0.5 * (lo + hi);
    if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
    tau = nt;
  }
  if (sub != 0) return;
  if (!conv && info) atomicCAS(info, 0, (int32_t)(nd.lo + q + 1));
  w.orig[nd.lo + q] = o;
  w.tau[nd.lo + q] = tau;
  w.lamw[nd.lo + q] = dorg + tau;
}

// (e) Gu-Eisenstat: zhat_l^2 = (lam_l - d_l)/rho * prod_{i != l} (lam_i - d_l)/(d_i - d_l)
__global__ void merge_zhat(int64_t n, int t, Work w) {
  const Node nd = merge_node(n, t, blockIdx.y);
  const MergeInfo mi = w.info[blockIdx.y];
  const int K = mi.K;
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= K) return;
  const double* d = w.sd + nd.lo;
  const int32_t* org = w.orig + nd.lo;
  const double* tau = w.tau + nd.lo;
  const double dl = d[l];
  double prod = ((d[org[l]] - dl) + tau[l]) / mi.rho;
  for (int i = 0; i < K; ++i) {
    if (i == l) continue;
    prod *= ((d[org[i]] - dl) + tau[i]) / (d[i] - dl);
  }
  const double zh = sqrt(fabs(prod));
  w.zhat[nd.lo + l] = copysign(zh, w.sz[nd.lo + l]);
}

// (f) U(:, i) = (zhat_l / (d_l - lam_i))_l normalised; row order given by urow.
__global__ void __launch_bounds__(256) merge_vectors(int64_t n, int t, Work w) {
  const Node nd = merge_node(n, t, blockIdx.y);
  const int K = w.info[blockIdx.y].K;
  const int i = blockIdx.x;
  if (i >= K) return;
  const double* d = w.sd + nd.lo;
  const int o = w.orig[nd.lo + i];
  const double ti = w.tau[nd.lo + i];
  const double dorg = d[o];
  __shared__ double red[4];
  double ss = 0.0;
  for (int l = threadIdx.x; l < K; l += 256) {
    const double u = w.zhat[nd.lo + l] / ((d[l] - dorg) - ti);
    ss += u * u;
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
  __syncthreads();
  const double inv = 1.0 / sqrt(red[0] + red[1] + red[2] + red[3]);
  double* Ucol = w.U + nd.lo + (nd.lo + i) * n;
  for (int l = threadIdx.x; l < K; l += 256) {
    const double u = w.zhat[nd.lo + l] / ((d[l] - dorg) - ti);
    Ucol[w.urow[nd.lo + l]] = u * inv;
  }
}

// (g) gather: G column g <- Z column gcol[g] (node block), and write the GEMM descriptors.
__global__ void merge_gather(int64_t n, int t, Work w, const double* __restrict__ Z, int64_t ldz) {
  const Node nd = merge_node(n, t, blockIdx.y);
  const int64_t N = nd.hi - nd.lo;
  const int64_t g = blockIdx.x;
  if (g >= N) return;
  const int64_t c = w.gcol[nd.lo + g];
  const double* src = Z + nd.lo + (nd.lo + c) * ldz;
  double* dst = w.G + nd.lo + (nd.lo + g) * n;
  for (int64_t r = threadIdx.x; r < N; r += blockDim.x) dst[r] = src[r];
  if (g == 0 && threadIdx.x == 0) {
    const MergeInfo mi = w.info[blockIdx.y];
    const int64_t n1 = nd.mid - nd.lo, n2 = nd.hi - nd.mid;
    GemmDesc top, bot;
    top.m = n1; top.n = mi.K; top.k = mi.K1 + mi.Km;
    top.alpha = 1.0; top.beta = 0.0; top.transA = 0; top.transB = 0;
    top.A = w.G + nd.lo + nd.lo * n; top.lda = n;
    top.B = w.U + nd.lo + nd.lo * n; top.ldb = n;
    top.C = w.Out + nd.lo + nd.lo * n; top.ldc = n;
    bot = top;
    bot.m = n2; bot.k = mi.Km + mi.K2;
    bot.A = w.G + nd.mid + (nd.lo + mi.K1) * n;
    bot.B = w.U + (nd.lo + mi.K1) + nd.lo * n;
    bot.C = w.Out + nd.mid + nd.lo * n;
    w.desc[2 * blockIdx.y] = top;
    w.desc[2 * blockIdx.y + 1] = bot;
  }
}

// (h) final order: rank of every eigenvalue of the merge, write lam and Z columns.
__global__ void __launch_bounds__(256) merge_scatter(int64_t n, int t, Work w, double* __restrict__ lam,
                                                     double* __restrict__ Z, int64_t ldz) {
  const Node nd = merge_node(n, t, blockIdx.y);
  const int64_t N = nd.hi - nd.lo;
  const int64_t j = blockIdx.x;  // entry of the combined list: [0, K) roots, [K, N) deflated
  if (j >= N) return;
  const int K = w.info[blockIdx.y].K;
  const double* roots = w.lamw + nd.lo;
  const double* defl = w.dlam + nd.lo;
  const double v = (j < K) ? roots[j] : defl[j - K];
  __shared__ int64_t part[4];
  int64_t cnt = 0;
  for (int64_t q = threadIdx.x; q < N; q += 256) {
    const double u = (q < K) ? roots[q] : defl[q - K];
    cnt += (u < v) || (u == v && q < j);
  }
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
  __syncthreads();
  const int64_t rank = part[0] + part[1] + part[2] + part[3];
  if (threadIdx.x == 0) lam[nd.lo + rank] = v;
  const double* src = (j < K) ? (w.Out + nd.lo + (nd.lo + j) * n) : (w.G + nd.lo + (nd.lo + j) * n);
  double* dst = Z + nd.lo + (nd.lo + rank) * ldz;
  for (int64_t r = threadIdx.x; r < N; r += 256) dst[r] = src[r];
}

// ---------------------------------------------------------------- bisection
__global__ void gersh_kernel(int64_t n, const double* __restrict__ d, const double* __restrict__ e,
                             double* __restrict__ out) {
  __shared__ double slo[256], shi[256];
  double lo = 1e308, hi = -1e308;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    double r = 0.0;
    if (i > 0) r += fabs(e[i - 1]);
    if (i + 1 < n) r += fabs(e[i]);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + s]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double pad = 4.0 * EPS * fmax(fabs(slo[0]), fabs(shi[0])) + 1e-300;
    out[0] = slo[0] - pad;
    out[1] = shi[0] + pad;
  }
}

// One thread per eigenvalue: bisection on Sturm counts inside the Gershgorin
// interval g[0..1] (computed on the device by gersh_kernel).
__global__ void bisect_dev(int64_t n, const double* __restrict__ d, const double* __restrict__ e,
                           const double* __restrict__ g, double* __restrict__ lam) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double tiny = 2.2250738585072014e-308 / EPS;
  double a = g[0], b = g[1];
  for (int it = 0; it < 128; ++it) {
    const double mid = 0.5 * (a + b);
    if (b - a <= 2.0 * EPS * fmax(fabs(a), fabs(b)) || mid <= a || mid >= b) break;
    int64_t cnt = 0;
    double q = d[0] - mid;
    if (q == 0.0) q = -tiny;
    cnt += q < 0.0;
    for (int64_t i = 1; i < n; ++i) {
      q = (d[i] - mid) - e[i - 1] * e[i - 1] / q;
      if (q == 0.0) q = -tiny;
      cnt += q < 0.0;
    }
    if (cnt > k) b = mid; else a = mid;
  }
  lam[k] = 0.5 * (a + b);
}

// Leaves hold at most `dc_leaf` (tuning table, 8 .. LEAF) rows.
int tree_depth(int64_t n) {
  int64_t leaf = tune("dc_leaf", n);
  if (leaf < 8) leaf = 8;
  if (leaf > LEAF) leaf = LEAF;
  int D = 0;
  while (cdiv(n, (int64_t)1 << D) > leaf) ++D;
  return D;
}

Work carve(Arena& ws, int64_t n) {
  Work w;
  const int D = tree_depth(n);
  const int64_t maxm = D > 0 ? ((int64_t)1 << (D - 1)) : 1;
  w.dd = ws.take<double>(n);
  w.zz = ws.take<double>(n);
  w.col = ws.take<int32_t>(n);
  w.sd = ws.take<double>(n);
  w.sz = ws.take<double>(n);
  w.scol = ws.take<int32_t>(n);
  w.sclass = ws.take<int32_t>(n);
  w.urow = ws.take<int32_t>(n);
  w.gcol = ws.take<int32_t>(n);
  w.dlam = ws.take<double>(n);
  w.rot_i = ws.take<int32_t>(n);
  w.rot_j = ws.take<int32_t>(n);
  w.rot_c = ws.take<double>(n);
  w.rot_s = ws.take<double>(n);
  w.orig = ws.take<int32_t>(n);
  w.tau = ws.take<double>(n);
  w.zhat = ws.take<double>(n);
  w.lamw = ws.take<double>(n);
  w.info = ws.take<MergeInfo>(maxm);
  w.desc = ws.take<GemmDesc>(2 * maxm);
  w.flops = ws.take<double>(1);
  if (D > 0) {
    w.G = ws.take<double>((size_t)n * n);
    w.U = ws.take<double>((size_t)n * n);
    w.Out = ws.take<double>((size_t)n * n);
  } else {
    w.G = w.U = w.Out = nullptr;
  }
  return w;
}

}  // namespace

namespace {

constexpr int64_t HOST_SIZED_MIN = 8192;
constexpr unsigned HOST_SIZED_MAX_P = 4;  // merges per level (top three levels)

// flops += 2 m n k over a level's merge products (their sizes after deflation
// live on the device).  One workgroup; levels are added in order.
__global__ void __launch_bounds__(64) sum_merge_flops(const GemmDesc* __restrict__ desc, int count,
                                                      double* flops) {
  double f = 0.0;
  for (int i = threadIdx.x; i < count; i += 64) {
    const GemmDesc d = desc[i];
    if (d.m > 0 && d.n > 0 && d.k > 0) f += 2.0 * (double)d.m * (double)d.n * (double)d.k;
  }
  for (int off = 32; off > 0; off >>= 1) f += __shfl_xor(f, off, 64);
  if (threadIdx.x == 0) *flops += f;
}

bool fast_aligned(const GemmDesc& d) {
  return (uintptr_t)d.A % 16 == 0 && (uintptr_t)d.B % 16 == 0 && d.lda % 2 == 0 && d.ldb % 2 == 0;
}

// Run a level's merge GEMMs (descriptor pairs top, bottom per merge, written by
// merge_gather) with sizes read back to the host.  The bottom product starts at
// column K1 of G (K1: the top half's undeflated count, the row offset of its B
// operand in U relative to the top product's); an odd K1 leaves that operand off
// the 16-byte alignment of the fast path.  G's column K1 - 1 is then a top-half
// eigenvector, exactly zero in the bottom half's rows, so starting one column
// earlier adds an exact zero term.  A product still misaligned (an odd node start
// in a ragged order) runs as a grouped launch of its own descriptor.
void merge_gemms_host(const GemmDesc* desc, int count, hipStream_t s) {
  GemmDesc hd[2 * HOST_SIZED_MAX_P];
  GEP_HIP(hipMemcpyAsync(hd, desc, (size_t)count * sizeof(GemmDesc), hipMemcpyDeviceToHost, s));
  GEP_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i) {
    GemmDesc d = hd[i];
    if (d.m <= 0 || d.n <= 0) continue;
    if ((i & 1) && (uintptr_t)d.B % 16 != 0) {
      const int64_t K1 = d.B - hd[i - 1].B;
      if (K1 >= 1) {
        d.A -= d.lda;
        d.B -= 1;
        d.k += 1;
      }
    }
    if (!fast_aligned(d)) {
      gemm_grouped(desc + i, 1, d.m, d.n, s);
      continue;
    }
    Gemm g;
    g.transA = d.transA != 0;
    g.transB = d.transB != 0;
    g.m = d.m; g.n = d.n; g.k = d.k;
    g.alpha = d.alpha; g.beta = d.beta;
    g.A = d.A; g.lda = d.lda; g.B = d.B; g.ldb = d.ldb; g.C = d.C; g.ldc = d.ldc;
    gemm(g, s);
  }
}

}  // namespace

size_t stedc_workspace(int64_t n) {
  Arena a;
  a.dry = true;
  carve(a, n);
  return a.used + 4096;
}

void stedc(int64_t n, const double* d, const double* e, double* lam, double* Z, int64_t ldz,
           int32_t* info, Arena& ws, hipStream_t s, double* flops_host) {
  if (n <= 0) return;
  Work w = carve(ws, n);
  if (flops_host) fill_f64(w.flops, 1, 0.0, s);
  const int D = tree_depth(n);
  // The top merges' GEMMs dominate large orders.  Their sizes depend on deflation
  // and live on the device; for an order >= HOST_SIZED_MIN on a stream that is not
  // being captured, the few descriptors of each of the top levels are read back
  // (one small copy and stream sync per level) and run on the tiled GEMM path with
  // host-side sizes, whose 128 x 128 interior kernel is faster than the grouped
  // one.  Graph capture allows no sync, and small orders (batched solves) keep the
  // launching thread free, so both use the grouped launch.
  bool host_sized = false;
  if (n >= HOST_SIZED_MIN) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    GEP_HIP(hipStreamIsCapturing(s, &cs));
    host_sized = cs == hipStreamCaptureStatusNone;
  }
  set_matrix(n, n, 0.0, 0.0, Z, ldz, s);
  // implicit QL converges in a few iterations per eigenvalue; 60 is the cap
  const int maxit = force_eig_failure() ? 0 : 60;
  hipLaunchKernelGGL(leaf_kernel, dim3((unsigned)((int64_t)1 << D)), dim3(64), 0, s, n, D, d, e, lam,
                     Z, ldz, info, maxit);
  GEP_LAUNCH_CHECK();
  for (int t = D - 1; t >= 0; --t) {
    const unsigned P = 1u << t;
    const int64_t Nmax = cdiv(n, (int64_t)P);
    hipLaunchKernelGGL(merge_prepare, dim3(P), dim3(256), 0, s, n, t, e, (const double*)lam,
                       (const double*)Z, ldz, w);
    GEP_LAUNCH_CHECK();
    hipLaunchKernelGGL(merge_deflate, dim3(P), dim3(256), 0, s, n, t, w);
    GEP_LAUNCH_CHECK();
    hipLaunchKernelGGL(merge_rotate, dim3((unsigned)cdiv(Nmax, 256), P), dim3(256), 0, s, n, t, w, Z,
                       ldz);
    GEP_LAUNCH_CHECK();
    hipLaunchKernelGGL(merge_secular, dim3((unsigned)cdiv(Nmax, 64 / SEC_LANES), P), dim3(64), 0, s,
                       n, t, w, info);
    GEP_LAUNCH_CHECK();
    hipLaunchKernelGGL(merge_zhat, dim3((unsigned)cdiv(Nmax, 64), P), dim3(64), 0, s, n, t, w);
    GEP_LAUNCH_CHECK();
    hipLaunchKernelGGL(merge_vectors, dim3((unsigned)Nmax, P), dim3(256), 0, s, n, t, w);
    GEP_LAUNCH_CHECK();
    hipLaunchKernelGGL(merge_gather, dim3((unsigned)Nmax, P), dim3(256), 0, s, n, t, w,
                       (const double*)Z, ldz);
    GEP_LAUNCH_CHECK();
    if (flops_host) {
      hipLaunchKernelGGL(sum_merge_flops, dim3(1), dim3(64), 0, s, (const GemmDesc*)w.desc,
                         (int)(2 * P), w.flops);
      GEP_LAUNCH_CHECK();
    }
    if (host_sized && P <= HOST_SIZED_MAX_P)
      merge_gemms_host(w.desc, (int)(2 * P), s);
    else
      gemm_grouped(w.desc, (int)(2 * P), Nmax, Nmax, s);
    hipLaunchKernelGGL(merge_scatter, dim3((unsigned)Nmax, P), dim3(256), 0, s, n, t, w, lam, Z, ldz);
    GEP_LAUNCH_CHECK();
  }
  if (flops_host)
    GEP_HIP(hipMemcpyAsync(flops_host, w.flops, sizeof(double), hipMemcpyDeviceToHost, s));
}

void stebz_ws(int64_t n, const double* d, const double* e, double* lam, double* bounds2,
              hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gersh_kernel, dim3(1), dim3(256), 0, s, n, d, e, bounds2);
  GEP_LAUNCH_CHECK();
  hipLaunchKernelGGL(bisect_dev, dim3((unsigned)cdiv(n, 64)), dim3(64), 0, s, n, d, e,
                     (const double*)bounds2, lam);
  GEP_LAUNCH_CHECK();
}

}  // namespace gep

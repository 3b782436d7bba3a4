// Internal helpers shared by the HIP sources of libgep (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <cstdio>

namespace gep {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Column-major element access.
#define GEP_AT(p, i, j, ld) ((p)[(size_t)(j) * (size_t)(ld) + (size_t)(i)])

struct HipError {
  hipError_t err;
  const char* what;
};

// Every HIP call on the host side goes through this; a failure is turned into a
// C++ exception that the C ABI layer converts into GEP_ERR_HIP.
#define GEP_HIP(call)                                         \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) throw ::gep::HipError{e_, #call};   \
  } while (0)

#define GEP_LAUNCH_CHECK() GEP_HIP(hipGetLastError())

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// Bump allocator over the caller's workspace.  Every region is 256-byte aligned.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  bool dry = false;  // size planning only: no pointer is dereferenced
  template <class T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    size_t off = used;
    used += bytes;
    if (dry) return reinterpret_cast<T*>(off + 256);  // never dereferenced
    if (used > cap) throw HipError{hipErrorOutOfMemory, "workspace too small"};
    return reinterpret_cast<T*>(base + off);
  }
};

// ---------------------------------------------------------------- GEMM
// C = alpha * op(A) * op(B) + beta * C, FP64, column-major, on MFMA.
//  uplo = 0: full C; uplo = 1: only the lower triangle (row >= col) of C is
//  written and tiles strictly above the diagonal are skipped.
//  symA: op(A) is a symmetric matrix of which only the lower triangle of A is
//  stored (transA is ignored).
struct Gemm {
  bool transA = false, transB = false, symA = false;
  int uplo = 0;
  int64_t m = 0, n = 0, k = 0;
  double alpha = 1.0, beta = 0.0;
  const double* A = nullptr;
  int64_t lda = 0;
  const double* B = nullptr;
  int64_t ldb = 0;
  double* C = nullptr;
  int64_t ldc = 0;
  // Strided batch: problem z uses A + z*strideA etc.
  int batch = 1;
  int64_t strideA = 0, strideB = 0, strideC = 0;
  // Optional scratch for splitting a long k loop over several workgroups (used
  // when C has few tiles).  Needs splitk_work_elems(m, n, k) doubles.
  double* work = nullptr;
  size_t work_elems = 0;
};
void gemm(const Gemm& g, hipStream_t s);

// A problem of a grouped launch, written to device memory by an earlier kernel.
struct GemmDesc {
  int64_t m, n, k;
  double alpha, beta;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  int transA, transB;
};
// One launch for `count` problems; max_m / max_n bound every problem's size.
void gemm_grouped(const GemmDesc* desc, int count, int64_t max_m, int64_t max_n, hipStream_t s);
size_t splitk_work_elems(int64_t m, int64_t n, int64_t k);

// Arithmetic of the 128 x 128 interior GEMM tiles.  FP64 by default; under
// MathMode::Fp32 both operands are rounded to FP32 as they are staged in LDS and
// the products accumulate in FP32 on the matrix cores, while inputs and outputs
// stay FP64 in memory.  Edge strips and small problems always run in FP64.  The
// mode belongs to the calling host thread and is set by a MathScope.
enum class MathMode { Fp64 = 0, Fp32 = 1 };
MathMode math_mode();
struct MathScope {
  MathMode saved;
  explicit MathScope(MathMode m);
  ~MathScope();
  MathScope(const MathScope&) = delete;
  MathScope& operator=(const MathScope&) = delete;
};

// Launch timing: when enabled, a ProbeScope records a HIP event pair on the
// launch stream around one kernel launch and remembers the launch's algorithmic
// flops.  Off by default (no events are recorded then).
enum ProbeKernel { PROBE_GEMM = 0, PROBE_Q2_APPLY = 1, PROBE_CHASE = 2, PROBE_PANEL_QR = 3,
                   PROBE_COUNT = 4 };
void probe_enable(bool on);
bool probe_read(int id, int64_t* launches, double* ms, double* flops);
struct ProbeScope {
  int id;
  hipStream_t s;
  double flops;
  bool on;
  hipEvent_t start, stop;  // this launch's pair (the record is kept when the scope ends)
  ProbeScope(int id_, hipStream_t s_, double flops_);
  ~ProbeScope();
  ProbeScope(const ProbeScope&) = delete;
  ProbeScope& operator=(const ProbeScope&) = delete;
};

// Small elementwise helpers (in misc.hip).
void copy_matrix(int64_t m, int64_t n, const double* src, int64_t lds, double* dst, int64_t ldd,
                 hipStream_t s);
void symmetrize_from_lower(int64_t n, const double* src, int64_t lds, double* dst, int64_t ldd,
                           hipStream_t s);
void set_matrix(int64_t m, int64_t n, double offdiag, double diag, double* dst, int64_t ldd,
                hipStream_t s);
void zero_upper(int64_t n, double* dst, int64_t ldd, hipStream_t s);
void fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
void fill_f64(double* p, int64_t n, double v, hipStream_t s);
// Enqueue: if *flag != 0, set *info = code unless info already holds a failure.
// A one-thread kernel, so it needs no host synchronisation and can be captured.
void raise_info_if(const int32_t* flag, int32_t* info, int32_t code, hipStream_t s);
// Enqueue: *info = code unless info already holds a failure.
void raise_info(int32_t* info, int32_t code, hipStream_t s);

// Device-side failure codes written to info besides the LAPACK ones (mirrored in
// gep.h): a bounded wait between workgroups gave up, or the mixed-precision
// refinement met a block of Y^T B Y that is not positive definite.
constexpr int32_t INFO_WAIT_TIMEOUT = -1;
constexpr int32_t INFO_REFINE_FAILED = -2;

// Debug switch for the bounded waits of the band reduction's grid barrier and the
// bulge chase: when set, every such wait that is not already satisfied at its
// first poll gives up as if its time limit had passed (so the failure path can be
// exercised while every kernel still exits normally).  Off by default.
void set_force_wait_timeout(bool on);
bool force_wait_timeout();
// Debug switch for the tridiagonal eigensolver: when set, the leaf solver's
// iteration cap is zero, so the first leaf that needs a QL iteration reports
// non-convergence (info = its first index + 1), as a real failure would.
void set_force_eig_failure(bool on);
bool force_eig_failure();
// Tuned parameter `key` for order M: a run-time override, else the tuning
// table's entry, else the built-in rule (tune.hip lists the keys).
int64_t tune(const char* key, int64_t M);
// Wall-clock ticks a bounded wait may last before it gives up (10 s).
uint64_t wait_limit_ticks();

}  // namespace gep

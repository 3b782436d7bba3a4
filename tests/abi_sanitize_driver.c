/* Host-only exercise of libgep's C ABI, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the library's host code: workspace sizing for
 * every entry point over a range of orders, the batched plan (LPT lanes and
 * workspace slots) for a 256-order batch, argument validation of the solve
 * entry points (every call here fails validation before any device work), status
 * and probe names, and the tuning table: the committed file, run-time overrides,
 * and malformed files (every prefix of the committed file, deep nesting,
 * unterminated strings and escapes, out-of-range numbers).
 * Usage: abi_sanitize_driver <tuning.json> <scratch directory>
 * Prints "sanitized abi run ok" and exits 0 when every check held. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/gep.h"

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      printf("FAIL line %d: %s\n", __LINE__, #c);                  \
      ++fails;                                                     \
    }                                                              \
  } while (0)

#define FAKE ((void*)0x100000)        /* never dereferenced: validation fails first */
#define FAKE_WS ((void*)0x200000)     /* 256-byte aligned */

static const char* KEYS[] = {"band_width", "q2_wide_min_cols", "dc_leaf", "symm_split_rows",
                             "chase_extra_groups", "q2_mixed_fp32", "q2_staged",
                             "chase_stationary"};
#define NKEYS (int)(sizeof(KEYS) / sizeof(KEYS[0]))

static void sizes(void) {
  static const int64_t Ms[] = {0, 1, 2, 3, 8, 17, 63, 64, 65, 255, 256, 257, 1000, 2047, 2048,
                               2049, 4096, 8192, 8195, 32768};
  for (size_t i = 0; i < sizeof(Ms) / sizeof(Ms[0]); ++i) {
    const int64_t M = Ms[i];
    for (int job = 0; job <= 1; ++job)
      for (int prec = 0; prec <= 1; ++prec) CHECK(gep_workspace_size(M, job, prec) >= 256);
    CHECK(gep_workspace_size(M, 1, 0) >= gep_workspace_size(M, 0, 0));
    const int64_t ks[] = {0, 1, M / 2, M};
    for (int k = 0; k < 4; ++k) CHECK(gep_workspace_size_lowest(M, ks[k]) >= 256);
    CHECK(gep_workspace_size_cholfree(M) >= 256);
    CHECK(gep_workspace_size_explicit_inverse(M) >= 256);
    CHECK(gep_workspace_size_jacobi(M) >= 256);
    CHECK(gep_reduce_workspace_size(M) >= 1);
    for (int b = 0; b <= 64; b += 8) {
      (void)gep_band_reduce_workspace_size(M, b == 0 ? 1 : b);
      (void)gep_tridiagonalize_workspace_size(M, b == 0 ? 1 : b);
    }
    (void)gep_tridiag_eig_workspace_size(M, 0);
    (void)gep_tridiag_eig_workspace_size(M, 1);
    (void)gep_backward_workspace_size(M);
  }
  CHECK(gep_noalloc_max_bytes() > 0);
}

/* Orders log-uniform in [64, 2048] from a fixed linear congruential sequence. */
static void batch_orders(int64_t* M, int n) {
  uint64_t x = 12345;
  for (int i = 0; i < n; ++i) {
    x = x * 6364136223846793005ULL + 1442695040888963407ULL;
    const double u = (double)(x >> 11) / 9007199254740992.0;
    const int64_t m = (int64_t)(64.0 * exp(u * log(32.0)) + 0.5);
    M[i] = m < 64 ? 64 : (m > 2048 ? 2048 : m);
  }
}

static void batched(void) {
  enum { N = 256 };
  int64_t M[N], ld[N];
  const double* A[N];
  double* lam[N];
  double* Y[N];
  batch_orders(M, N);
  for (int i = 0; i < N; ++i) {
    ld[i] = M[i];
    A[i] = (const double*)FAKE;
    lam[i] = (double*)FAKE;
    Y[i] = (double*)FAKE;
  }
  const size_t need = gep_workspace_size_batched(N, M, 1, 0);
  CHECK(need > gep_workspace_size(2048, 1, 0));
  CHECK(gep_workspace_size_batched(N, M, 0, 0) <= need);
  CHECK(gep_workspace_size_batched(0, M, 1, 0) == 256);
  CHECK(gep_workspace_size_batched(3, NULL, 1, 0) == 256);
  /* the plan is built, then the workspace check fails: no device work */
  CHECK(gep_solve_batched(N, M, A, ld, A, ld, lam, Y, ld, 1, 0, FAKE_WS, need - 1, (int32_t*)FAKE,
                          NULL) == GEP_ERR_WORKSPACE);
  CHECK(gep_solve_batched(-1, M, A, ld, A, ld, lam, Y, ld, 1, 0, FAKE_WS, need, (int32_t*)FAKE,
                          NULL) == GEP_ERR_ARG && gep_last_bad_arg() == 1);
  CHECK(gep_solve_batched(0, M, A, ld, A, ld, lam, Y, ld, 1, 0, FAKE_WS, need, (int32_t*)FAKE,
                          NULL) == GEP_OK);
  CHECK(gep_solve_batched(N, NULL, A, ld, A, ld, lam, Y, ld, 1, 0, FAKE_WS, need, (int32_t*)FAKE,
                          NULL) == GEP_ERR_ARG && gep_last_bad_arg() == 2);
  CHECK(gep_solve_batched(N, M, A, ld, A, ld, lam, Y, ld, 1, 1, FAKE_WS, need, (int32_t*)FAKE,
                          NULL) == GEP_ERR_ARG && gep_last_bad_arg() == 11);
  CHECK(gep_solve_batched(N, M, A, ld, A, ld, lam, Y, ld, 1, 0, FAKE_WS, need, NULL, NULL) ==
            GEP_ERR_ARG && gep_last_bad_arg() == 14);
  ld[N - 1] = M[N - 1] - 1;
  CHECK(gep_solve_batched(N, M, A, ld, A, ld, lam, Y, ld, 1, 0, FAKE_WS, need, (int32_t*)FAKE,
                          NULL) == GEP_ERR_ARG && gep_last_bad_arg() == 4);
  ld[N - 1] = M[N - 1];
  M[7] = -3;
  CHECK(gep_solve_batched(N, M, A, ld, A, ld, lam, Y, ld, 1, 0, FAKE_WS, need, (int32_t*)FAKE,
                          NULL) == GEP_ERR_ARG && gep_last_bad_arg() == 2);
  (void)gep_workspace_size_batched(N, M, 1, 0); /* a negative order in the plan */
}

static void solve_args(void) {
  const int64_t M = 10;
  const size_t ws = gep_workspace_size(M, 1, 0);
  CHECK(gep_solve(-1, FAKE, 1, FAKE, 1, FAKE, FAKE, 1, 1, 0, FAKE_WS, ws, FAKE, NULL) ==
            GEP_ERR_ARG && gep_last_bad_arg() == 1);
  CHECK(gep_solve(M, NULL, M, FAKE, M, FAKE, FAKE, M, 1, 0, FAKE_WS, ws, FAKE, NULL) ==
            GEP_ERR_ARG && gep_last_bad_arg() == 2);
  CHECK(gep_solve(M, FAKE, M - 1, FAKE, M, FAKE, FAKE, M, 1, 0, FAKE_WS, ws, FAKE, NULL) ==
            GEP_ERR_ARG && gep_last_bad_arg() == 3);
  CHECK(gep_solve(M, FAKE, M, FAKE, M, FAKE, FAKE, M, 7, 0, FAKE_WS, ws, FAKE, NULL) ==
            GEP_ERR_ARG && gep_last_bad_arg() == 9);
  CHECK(gep_solve(M, FAKE, M, FAKE, M, FAKE, FAKE, M, 1, 0, (void*)0x200010, ws, FAKE, NULL) ==
            GEP_ERR_ARG && gep_last_bad_arg() == 11);
  CHECK(gep_solve(M, FAKE, M, FAKE, M, FAKE, FAKE, M, 1, 0, FAKE_WS, ws - 1, FAKE, NULL) ==
        GEP_ERR_WORKSPACE);
  CHECK(gep_solve_noalloc(M, FAKE, M, FAKE, M, FAKE, FAKE, M, 1, 0, NULL, NULL) == GEP_ERR_ARG &&
        gep_last_bad_arg() == 11);
  CHECK(gep_solve_noalloc(100000, FAKE, 100000, FAKE, 100000, FAKE, FAKE, 100000, 1, 0, FAKE,
                          NULL) == GEP_ERR_WORKSPACE);
  CHECK(gep_solve_lowest(M, FAKE, M, FAKE, M, M + 1, FAKE, FAKE, M, FAKE_WS, 1 << 30, FAKE,
                         NULL) == GEP_ERR_ARG && gep_last_bad_arg() == 6);
  CHECK(gep_dgemm(2, 0, 0, 4, 4, 4, 1.0, FAKE, 4, FAKE, 4, 0.0, FAKE, 4, 0, NULL) == GEP_ERR_ARG &&
        gep_last_bad_arg() == 1);
}

static void names(void) {
  for (int s = -8; s <= 2; ++s) {
    const char* t = gep_status_string(s);
    CHECK(t != NULL && strlen(t) > 0);
  }
  CHECK(gep_version() != NULL && strlen(gep_version()) > 0);
  for (int k = -2; k <= 6; ++k) {
    const char* t = gep_probe_name(k);
    if (t) CHECK(strlen(t) > 0);
  }
  CHECK(gep_probe_read(99, NULL, NULL, NULL) == GEP_ERR_ARG);
}

static int write_file(const char* path, const char* data, size_t n) {
  FILE* f = fopen(path, "wb");
  if (!f) return 0;
  fwrite(data, 1, n, f);
  fclose(f);
  return 1;
}

static void tuning(const char* table, const char* dir) {
  FILE* f = fopen(table, "rb");
  CHECK(f != NULL);
  if (!f) return;
  fseek(f, 0, SEEK_END);
  const long n = ftell(f);
  fseek(f, 0, SEEK_SET);
  char* text = (char*)malloc((size_t)n + 1);
  CHECK(fread(text, 1, (size_t)n, f) == (size_t)n);
  fclose(f);
  text[n] = 0;

  const int entries = gep_tune_load(table);
  CHECK(entries >= 0);
  int64_t before[NKEYS][4];
  static const int64_t probeM[4] = {64, 700, 8192, 32768};
  for (int k = 0; k < NKEYS; ++k)
    for (int j = 0; j < 4; ++j) {
      before[k][j] = gep_tune_get(KEYS[k], probeM[j]);
      CHECK(before[k][j] >= 0);
    }
  CHECK(gep_tune_get("no_such_parameter", 100) == -1);
  CHECK(gep_tune_get(NULL, 100) == -1);
  CHECK(gep_tune_set("band_width", 100, 200, 8) == GEP_OK);
  CHECK(gep_tune_get("band_width", 150) == 8);
  CHECK(gep_tune_set("band_width", 100, 200, 65) == GEP_ERR_ARG);
  CHECK(gep_tune_set("band_width", 200, 100, 8) == GEP_ERR_ARG);
  CHECK(gep_tune_set(NULL, 0, 1, 1) == GEP_ERR_ARG);
  CHECK(gep_tune_reset_overrides() == GEP_OK);

  char path[4096];
  snprintf(path, sizeof(path), "%s/malformed.json", dir);
  /* every prefix of the committed file: each load either parses or is refused,
   * and a refused load keeps the previous table */
  for (long cut = 0; cut < n; ++cut) {
    CHECK(write_file(path, text, (size_t)cut));
    const int r = gep_tune_load(path);
    CHECK(r == GEP_ERR_ARG || r >= 0);
  }
  static const char* bad[] = {
      "",
      "{",
      "{\"parameters\": ",
      "{\"parameters\": {\"band_width\": [{\"m_lo\": 1, \"m_hi\": 2, \"value\": 1e999}]}}",
      "{\"parameters\": {\"band_width\": [{\"m_lo\": -1, \"m_hi\": 2, \"value\": 8}]}}",
      "{\"parameters\": {\"band_width\": [{\"m_lo\": 1, \"m_hi\": 2, \"value\": nan}]}}",
      "{\"parameters\": {\"band_width\": [{\"m_lo\": 1, \"m_hi\": 2, \"value\": 8.5}]}}",
      "{\"parameters\": {\"band_width\": [{\"m_lo\": 9.3e18, \"m_hi\": 2, \"value\": 8}]}}",
      "{\"parameters\": {\"band_width\": [{\"m_lo\": 1, \"m_hi\": 2}]}}",
      "{\"parameters\": {\"band_width\": 5}}",
      "{\"parameters\": [1, 2]}",
      "{\"a\": \"unterminated",
      "{\"a\": \"escape at end\\",
      "{\"a\": \"short unicode \\u12",
      "{\"a\": \"\\u0041\\n\\t\\\"\"} trailing",
      "[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]",
      "{\"x\": tru}",
      "{\"x\": [1, 2,]}",
      "{\"x\": {\"y\": 1,}}",
      "{\"x\" 1}",
      "   \n\t ",
  };
  for (size_t i = 0; i < sizeof(bad) / sizeof(bad[0]); ++i) {
    CHECK(write_file(path, bad[i], strlen(bad[i])));
    CHECK(gep_tune_load(path) == GEP_ERR_ARG);
  }
  static const char* good[] = {
      "{}",
      "{\"parameters\": {}}",
      "{\"parameters\": {\"not_a_parameter\": [1, \"x\"]}, \"other\": [true, false, null]}",
      "{\"parameters\": {\"dc_leaf\": [{\"m_lo\": 0, \"m_hi\": 100, \"value\": 32, \"ms\": 1.5}]}}",
  };
  for (size_t i = 0; i < sizeof(good) / sizeof(good[0]); ++i) {
    CHECK(write_file(path, good[i], strlen(good[i])));
    CHECK(gep_tune_load(path) >= 0);
  }
  CHECK(gep_tune_get("dc_leaf", 50) == 32);
  snprintf(path, sizeof(path), "%s/does_not_exist.json", dir);
  CHECK(gep_tune_load(path) == GEP_ERR_ARG);
  CHECK(gep_tune_clear() == GEP_OK);
  CHECK(gep_tune_load(table) == entries);
  for (int k = 0; k < NKEYS; ++k)
    for (int j = 0; j < 4; ++j) CHECK(gep_tune_get(KEYS[k], probeM[j]) == before[k][j]);
  free(text);
}

int main(int argc, char** argv) {
  if (argc < 3) {
    printf("usage: %s <tuning.json> <scratch directory>\n", argv[0]);
    return 2;
  }
  names();
  sizes();
  batched();
  solve_args();
  tuning(argv[1], argv[2]);
  if (fails) {
    printf("%d checks failed\n", fails);
    return 1;
  }
  printf("sanitized abi run ok\n");
  return 0;
}

/*
 * Host-side checks of the C ABI, built against a copy of the library whose
 * host code is compiled with AddressSanitizer and UndefinedBehaviorSanitizer
 * (and no device code): every workspace query on valid and invalid shapes
 * and options, every compute entry point on arguments it must reject before
 * any device work, the status strings, the last-error text and the phase
 * profiler.  No call here reaches the GPU.  Exit status 0 when every result
 * is as expected; the sanitizers abort on the first memory or UB error.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "skls.h"

static int failures = 0;

static void expect(int cond, const char* what) {
  if (!cond) {
    ++failures;
    fprintf(stderr, "FAILED: %s (last error: %s)\n", what, skls_last_error());
  }
}

static skls_matrix dense(int64_t n, int64_t d, int32_t dtype) {
  skls_matrix m;
  memset(&m, 0, sizeof m);
  m.layout = SKLS_DENSE;
  m.dtype = dtype;
  m.n = n;
  m.d = d;
  m.ld = d;
  m.val = (const void*)0x1000; /* never dereferenced on these paths */
  return m;
}

static skls_matrix csr(int64_t n, int64_t d, int64_t nnz) {
  skls_matrix m = dense(n, d, SKLS_F32);
  m.layout = SKLS_CSR;
  m.nnz = nnz;
  m.row_ptr = (const void*)0x1000;
  m.col_idx = (const int32_t*)0x1000;
  return m;
}

int main(void) {
  size_t bytes = 0;
  /* status strings and version */
  for (int32_t st = -2; st < 12; ++st) expect(skls_status_str(st) != NULL && skls_status_str(st)[0] != 0, "status_str");
  expect(strcmp(skls_status_str(0), "SKLS_OK") == 0, "status_str(0)");
  expect(skls_version() != NULL && strlen(skls_version()) > 0, "version");

  /* sketch workspaces: valid dense and CSR, every variant */
  skls_matrix A = dense(100000, 64, SKLS_F32);
  skls_matrix C = csr(100000, 256, 1600000);
  for (int32_t v = 0; v <= 3; ++v) {
    expect(skls_sketch_workspace(&A, 4096, v, &bytes) == SKLS_OK, "sketch_workspace dense");
    int32_t st = skls_sketch_workspace(&C, 4096, v, &bytes);
    expect(st == SKLS_OK || st == SKLS_ERR_SHAPE, "sketch_workspace csr");
    st = skls_sketch_plan_workspace(&C, 4096, v, SKLS_F32, &bytes);
    expect(st == SKLS_OK || st == SKLS_ERR_SHAPE || st == SKLS_ERR_ARG, "sketch_plan_workspace");
  }
  /* invalid inputs */
  expect(skls_sketch_workspace(NULL, 4096, 0, &bytes) != SKLS_OK, "sketch_workspace NULL A");
  expect(skls_sketch_workspace(&A, 0, 0, &bytes) != SKLS_OK, "sketch_workspace t = 0");
  expect(skls_sketch_workspace(&A, 4096, 9, &bytes) != SKLS_OK, "sketch_workspace bad variant");
  expect(strlen(skls_last_error()) > 0, "last_error set");
  skls_matrix bad = dense(10, 4, 77);
  expect(skls_sketch_workspace(&bad, 16, 0, &bytes) != SKLS_OK, "bad dtype");
  bad = dense(10, 4, SKLS_F32);
  bad.ld = 2;
  expect(skls_sketch_workspace(&bad, 16, 0, &bytes) != SKLS_OK, "ld < d");
  bad = csr(10, 4, 5);
  bad.row_ptr = NULL;
  expect(skls_sketch_workspace(&bad, 16, 0, &bytes) != SKLS_OK, "CSR without row_ptr");
  expect(skls_sketch(NULL, NULL, SKLS_F64, 16, 1, NULL, 0, NULL, NULL, SKLS_F64, NULL, 0, NULL) != SKLS_OK,
         "sketch NULL");
  expect(skls_sketch(&A, NULL, SKLS_F64, 16, 1, NULL, 0, NULL, NULL, SKLS_F64, NULL, 0, NULL) != SKLS_OK,
         "sketch NULL SA");
  expect(skls_sketch_rows(&A, -1, NULL, SKLS_F64, 16, 1, NULL, 0, NULL, NULL, SKLS_F64, NULL, 0, NULL) != SKLS_OK,
         "sketch_rows negative start");
  expect(skls_hash(10, 0, 1, 0, NULL, NULL, NULL) != SKLS_OK, "hash t = 0");
  expect(skls_hash(-1, 16, 1, 0, NULL, NULL, NULL) != SKLS_OK, "hash n < 0");

  /* generalized embedding */
  expect(skls_sketch_general_workspace(&A, 64, 16, 0, &bytes) == SKLS_OK, "general_workspace");
  expect(skls_sketch_general_workspace(&A, 0, 16, 0, &bytes) != SKLS_OK, "general_workspace q = 0");

  /* QR, least squares, second stage */
  expect(skls_qr_r_workspace(5000, 64, &bytes) == SKLS_OK && bytes > 0, "qr_r_workspace");
  expect(skls_qr_r_workspace(10, 64, &bytes) != SKLS_OK, "qr_r_workspace m < d");
  expect(skls_qr_r(NULL, SKLS_F64, 100, 4, NULL, NULL, NULL, 0, NULL) != SKLS_OK, "qr_r NULL");
  skls_lstsq_opts o;
  memset(&o, 0, sizeof o);
  o.t = 4096;
  o.seed = 7;
  for (int32_t prec = 0; prec <= 1; ++prec) {
    o.precision = prec;
    expect(skls_lstsq_workspace(&A, &o, &bytes) == SKLS_OK && bytes > 0, "lstsq_workspace");
    expect(skls_lstsq_workspace(&C, &o, &bytes) == SKLS_OK && bytes > 0, "lstsq_workspace csr");
  }
  o.second_stage = 256;
  expect(skls_lstsq_workspace(&A, &o, &bytes) == SKLS_OK, "lstsq_workspace second stage");
  o.second_stage = 8;
  expect(skls_lstsq_workspace(&A, &o, &bytes) != SKLS_OK, "second stage below d");
  o.second_stage = 0;
  o.precision = 3;
  expect(skls_lstsq_workspace(&A, &o, &bytes) != SKLS_OK, "bad precision");
  o.precision = 0;
  o.max_retries = 100;
  expect(skls_lstsq_workspace(&A, &o, &bytes) != SKLS_OK, "too many retries");
  o.max_retries = 0;
  o.t = 10;
  expect(skls_lstsq_workspace(&A, &o, &bytes) != SKLS_OK, "t < d");
  o.t = 4096;
  expect(skls_lstsq(&A, NULL, &o, NULL, NULL, NULL, 0, NULL) != SKLS_OK, "lstsq NULL b");
  expect(skls_second_stage_workspace(65536, 512, 2048, &bytes) == SKLS_OK && bytes > 0, "second_stage_workspace");
  expect(skls_second_stage_workspace(65536, 512, 0, &bytes) != SKLS_OK, "second_stage m = 0");
  expect(skls_second_stage(NULL, NULL, SKLS_F32, 100, 4, 8, 1, NULL, NULL, NULL, 0, NULL) != SKLS_OK,
         "second_stage NULL");

  /* leverage, Gram, learned values */
  expect(skls_leverage_workspace(&A, 4096, 32, &bytes) == SKLS_OK, "leverage_workspace");
  expect(skls_leverage_workspace(&A, 4096, 0, &bytes) != SKLS_OK, "leverage k = 0");
  expect(skls_leverage_from_r_workspace(&A, 32, &bytes) == SKLS_OK, "leverage_from_r_workspace");
  expect(skls_leverage_scores(&A, 4096, 1, 0, NULL, NULL, NULL, 0, NULL) != SKLS_OK, "leverage_scores k = 0");
  expect(skls_gram_workspace(&A, &bytes) == SKLS_OK, "gram_workspace");
  expect(skls_gram(NULL, NULL, NULL, 0, NULL) != SKLS_OK, "gram NULL");
  expect(skls_learned_workspace(&A, 1024, &bytes) == SKLS_OK, "learned_workspace");
  expect(skls_learned_workspace(&A, 0, &bytes) != SKLS_OK, "learned_workspace t = 0");
  expect(skls_learned_batch_workspace(&A, 1024, &bytes) == SKLS_OK && bytes > 0, "learned_batch_workspace");
  expect(skls_learned_batch_workspace(&A, 0, &bytes) != SKLS_OK, "learned_batch_workspace t = 0");
  expect(skls_learned_grad_batch(0, &A, NULL, NULL, NULL, NULL, 0, NULL, 0, NULL, NULL, NULL, 0, NULL) != SKLS_OK,
         "learned_grad_batch count = 0");

  /* multiple responses, l_p, low rank */
  skls_multi_opts mo;
  memset(&mo, 0, sizeof mo);
  mo.t = 4096;
  mo.t_s = 2048;
  expect(skls_multi_lstsq_workspace(&A, 16, &mo, &bytes) == SKLS_OK, "multi_workspace");
  mo.t = 8;
  expect(skls_multi_lstsq_workspace(&A, 16, &mo, &bytes) != SKLS_OK, "multi t < d");
  skls_lp_opts lo;
  memset(&lo, 0, sizeof lo);
  lo.p = 1.0;
  expect(skls_lp_regression_workspace(&C, &lo, &bytes) == SKLS_OK, "lp_workspace");
  lo.p = 0.5;
  expect(skls_lp_regression_workspace(&C, &lo, &bytes) != SKLS_OK, "lp p < 1");
  skls_low_rank_opts ro;
  memset(&ro, 0, sizeof ro);
  ro.k = 8;
  ro.t_r = 64;
  expect(skls_low_rank_workspace(&C, &ro, &bytes) == SKLS_OK, "low_rank_workspace");
  ro.k = 0;
  expect(skls_low_rank_workspace(&C, &ro, &bytes) != SKLS_OK, "low_rank k = 0");
  expect(skls_low_rank(&C, &ro, NULL, NULL, NULL, NULL, NULL, 0, NULL) != SKLS_OK, "low_rank k = 0 call");

  /* phase profiler (host bookkeeping only) */
  expect(skls_profile_enable(1) == SKLS_OK, "profile_enable");
  expect(skls_profile_count() >= 0, "profile_count");
  const char* name = NULL;
  int64_t launches = 0;
  double ms = 0.0;
  expect(skls_profile_get(1 << 20, &name, &launches, &ms) != SKLS_OK, "profile_get out of range");
  expect(skls_profile_enable(0) == SKLS_OK, "profile_disable");

  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("abi host checks passed\n");
  return 0;
}

/* Host-code paths of libads that run without a GPU, for a build whose host
 * code carries AddressSanitizer and UndefinedBehaviorSanitizer: argument
 * validation of every entry point, the clean-up of a setup that fails at
 * its first device allocation, the tuning-cache file parser, the weights
 * file parser and the network shape arithmetic.  Exit status 0 when every
 * call returned the expected status; a sanitizer report aborts the run.
 * Usage: host_sanitize_driver <scratch directory> */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ads.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
  if (got != want) {
    fprintf(stderr, "FAIL %s: status %d (%s), expected %d\n", what, got, ads_status_string(got), want);
    ++failures;
  }
}

static void expect_error(int got, const char* what) {  /* any error, with a message */
  if (got >= 0 || !ads_last_error() || !ads_last_error()[0]) {
    fprintf(stderr, "FAIL %s: status %d, expected an error with a message\n", what, got);
    ++failures;
  }
}

static void write_file(const char* path, const void* data, size_t n) {
  FILE* f = fopen(path, "wb");
  if (!f) { perror(path); exit(2); }
  if (n) fwrite(data, 1, n, f);
  fclose(f);
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  const char* dir = argv[1];
  char path[4096];
  for (int s = -8; s <= 3; ++s) {
    const char* m = ads_status_string(s);
    if (!m || !m[0]) { fprintf(stderr, "FAIL status string %d\n", s); ++failures; }
  }
  (void)ads_last_error();

  /* a 1D Laplacian of 8 rows in 2 parts */
  int64_t rp[9];
  int32_t col[22];
  double val[22];
  int64_t k = 0;
  for (int i = 0; i < 8; ++i) {
    rp[i] = k;
    if (i > 0) { col[k] = i - 1; val[k++] = -1.0; }
    col[k] = i; val[k++] = 2.0;
    if (i < 7) { col[k] = i + 1; val[k++] = -1.0; }
  }
  rp[8] = k;
  ads_csr A = {8, k, rp, col, val, 0};
  int32_t part[8] = {0, 0, 0, 0, 1, 1, 1, 1};
  ads_options o;
  memset(&o, 0, sizeof o);
  o.abi_version = ADS_ABI_VERSION;
  o.overlap = 1;
  o.nev = 2;
  ads_ctx* ctx = NULL;

  expect(ads_setup(NULL, part, 2, &o, NULL, &ctx), ADS_ERR_ARG, "setup null A");
  expect(ads_setup(&A, NULL, 2, &o, NULL, &ctx), ADS_ERR_ARG, "setup null part");
  expect(ads_setup(&A, part, 2, NULL, NULL, &ctx), ADS_ERR_ARG, "setup null options");
  expect(ads_setup(&A, part, 2, &o, NULL, NULL), ADS_ERR_ARG, "setup null out");
  expect(ads_setup(&A, part, 0, &o, NULL, &ctx), ADS_ERR_ARG, "setup nparts 0");
  ads_options bad = o;
  bad.abi_version = ADS_ABI_VERSION + 1;
  expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "setup abi");
  bad = o; bad.overlap = -1;
  expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "setup overlap");
  bad = o; bad.nev = 1000;
  expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "setup nev");
  bad = o; bad.variant = 99;
  expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "setup variant");
  bad = o; bad.precision = -3;
  expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "setup precision");
  bad = o; bad.eig_solver = 7;
  expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "setup eig_solver");
  bad = o; bad.warm_start = 1;
  expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "setup warm start without file");
  ads_csr An = A;
  An.n = -5;
  expect(ads_setup(&An, part, 2, &o, NULL, &ctx), ADS_ERR_ARG, "setup n < 0");
  An = A; An.col = NULL;
  expect(ads_setup(&An, part, 2, &o, NULL, &ctx), ADS_ERR_ARG, "setup null col");
  expect(ads_setup_batched(0, &A, NULL, NULL, &o, NULL, &ctx), ADS_ERR_ARG, "batched nsys 0");

  /* complex systems: (re, im) pairs; nev counts complex vectors (<= 15) and
   * the learned start is for real A only */
  double zval[44];
  for (int64_t q = 0; q < k; ++q) {
    zval[2 * q] = val[q];
    zval[2 * q + 1] = (col[q] == 0 && q == 0) ? 0.5 : 0.25 * (double)(q % 3);
  }
  ads_csr Z = {8, k, rp, col, zval, 0};
  const int32_t* zparts[1] = {part};
  int32_t znp = 2;
  expect(ads_setup_complex(0, &Z, zparts, &znp, &o, NULL, &ctx), ADS_ERR_ARG, "complex nsys 0");
  expect(ads_setup_complex(1, NULL, zparts, &znp, &o, NULL, &ctx), ADS_ERR_ARG, "complex null A");
  bad = o; bad.nev = 16;
  expect(ads_setup_complex(1, &Z, zparts, &znp, &bad, NULL, &ctx), ADS_ERR_ARG, "complex nev 16");
  bad = o; bad.nev = 31; bad.tau = 0.3;
  expect(ads_setup_complex(1, &Z, zparts, &znp, &bad, NULL, &ctx), ADS_ERR_ARG, "complex tau cap");
  bad = o; bad.warm_start = 1; bad.gnn_weights_path = "unused";
  expect(ads_setup_complex(1, &Z, zparts, &znp, &bad, NULL, &ctx), ADS_ERR_UNSUPPORTED,
         "complex warm start");
  {
    int zs = ads_setup_complex(1, &Z, zparts, &znp, &o, NULL, &ctx);
    if (zs == ADS_OK) {
      ads_info zi;
      memset(&zi, 0, sizeof zi);
      expect(ads_get_info(ctx, &zi), ADS_OK, "complex get_info");
      if (zi.is_complex != 1 || zi.n != 16) { fprintf(stderr, "FAIL complex info\n"); ++failures; }
      expect(ads_destroy(ctx), ADS_OK, "complex destroy");
    } else {
      expect_error(zs, "complex setup without a device");
    }
  }

  /* weights files: missing, empty, wrong magic, bad shape, truncated body */
  bad = o; bad.warm_start = 1;
  snprintf(path, sizeof path, "%s/none.adsgnn", dir);
  bad.gnn_weights_path = path;
  expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "weights missing");
  write_file(path, "", 0);
  expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "weights empty");
  write_file(path, "NOTAGNN1xxxxxxxxxxxxxxxxxxxxxxxx", 32);
  expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "weights magic");
  {
    unsigned char h[32];
    memcpy(h, "ADSGNN01", 8);
    int32_t sh[4] = {ADS_GNN_FEATURES, 1000, 2, 4};
    int64_t np = 12;
    memcpy(h + 8, sh, 16);
    memcpy(h + 24, &np, 8);
    write_file(path, h, 32);
    expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "weights shape");
    ads_gnn_shape gs = {ADS_GNN_FEATURES, 8, 2, 4};
    const int64_t npar = ads_gnn_nparams(&gs);
    sh[1] = 8;
    memcpy(h + 8, sh, 16);
    memcpy(h + 24, &npar, 8);
    unsigned char* body = (unsigned char*)calloc(32 + 4 * (size_t)npar, 1);
    memcpy(body, h, 32);
    write_file(path, body, 32 + 4 * (size_t)(npar - 1));  /* one parameter short */
    expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "weights truncated");
    np = npar + 1;
    memcpy(body + 24, &np, 8);
    write_file(path, body, 32 + 4 * (size_t)npar);
    expect(ads_setup(&A, part, 2, &bad, NULL, &ctx), ADS_ERR_ARG, "weights count");
    free(body);
  }

  /* a valid setup: without a GPU it fails at its first device call and must
   * release what it built; with one it succeeds */
  int st = ads_setup(&A, part, 2, &o, NULL, &ctx);
  if (st == ADS_OK) {
    ads_info info;
    expect(ads_get_info(ctx, &info), ADS_OK, "get_info");
    expect(ads_destroy(ctx), ADS_OK, "destroy");
  } else {
    expect_error(st, "setup without a device");
  }

  /* null contexts everywhere */
  ads_info info;
  expect(ads_get_info(NULL, &info), ADS_ERR_ARG, "get_info null");
  expect(ads_apply(NULL, NULL, NULL, 1, NULL), ADS_ERR_ARG, "apply null");
  expect(ads_apply_noalloc(NULL, NULL, NULL, 1, NULL), ADS_ERR_ARG, "apply_noalloc null");
  ads_ksp_options ko;
  memset(&ko, 0, sizeof ko);
  ads_ksp_result kr;
  expect(ads_solve(NULL, NULL, NULL, 1, &ko, &kr, NULL), ADS_ERR_ARG, "solve null");
  expect(ads_set_graphs(NULL, 1), ADS_ERR_ARG, "set_graphs null");
  expect(ads_export_splitting(NULL, NULL), ADS_ERR_ARG, "export_splitting null");
  expect(ads_partition_bfs(NULL, 2, NULL, NULL, NULL), ADS_ERR_ARG, "partition null");
  (void)ads_destroy(NULL);

  /* network shapes */
  ads_gnn_shape gs = {ADS_GNN_FEATURES, 32, 3, 8};
  if (ads_gnn_nparams(&gs) <= 0) { fprintf(stderr, "FAIL nparams\n"); ++failures; }
  gs.width = 0;
  if (ads_gnn_nparams(&gs) >= 0) { fprintf(stderr, "FAIL nparams of a bad shape\n"); ++failures; }
  if (ads_gnn_nparams(NULL) >= 0) { fprintf(stderr, "FAIL nparams null\n"); ++failures; }

  /* tuning cache: save, load back, malformed files */
  expect(ads_tune_cache_clear(), ADS_OK, "cache clear");
  snprintf(path, sizeof path, "%s/tune.txt", dir);
  expect(ads_tune_cache_save(path), ADS_OK, "cache save");
  expect(ads_tune_cache_load(path), ADS_OK, "cache load");
  const char* good = "ads-tune 1\nshape-a 1.5\nshape-b 2\n";
  write_file(path, good, strlen(good));
  expect(ads_tune_cache_load(path), ADS_OK, "cache load entries");
  expect(ads_tune_cache_save(path), ADS_OK, "cache save entries");
  const char* range = "ads-tune 1\nshape-a 99\n";
  write_file(path, range, strlen(range));
  expect(ads_tune_cache_load(path), ADS_ERR_ARG, "cache out of range");
  const char* head = "something-else 3\n";
  write_file(path, head, strlen(head));
  expect(ads_tune_cache_load(path), ADS_ERR_ARG, "cache header");
  write_file(path, "", 0);
  expect(ads_tune_cache_load(path), ADS_ERR_ARG, "cache empty");
  {
    char longkey[2048];
    memset(longkey, 'k', sizeof longkey);
    memcpy(longkey, "ads-tune 1\n", 11);
    longkey[sizeof longkey - 6] = ' ';
    memcpy(longkey + sizeof longkey - 5, "2.0\n", 4);
    longkey[sizeof longkey - 1] = 0;
    write_file(path, longkey, strlen(longkey));
    (void)ads_tune_cache_load(path);  /* any status; no overflow */
  }
  snprintf(path, sizeof path, "%s/missing/tune.txt", dir);
  expect(ads_tune_cache_load(path), ADS_ERR_ARG, "cache missing file");
  expect(ads_tune_cache_load(NULL), ADS_ERR_ARG, "cache null path");
  expect(ads_tune_cache_save(NULL), ADS_ERR_ARG, "cache save null path");
  expect(ads_tune_cache_clear(), ADS_OK, "cache clear again");

  if (failures) fprintf(stderr, "%d failures\n", failures);
  else printf("host paths: all expected statuses\n");
  return failures ? 1 : 0;
}

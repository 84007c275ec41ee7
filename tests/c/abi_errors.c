/* Error paths of the C ABI (test driver, plain C99), meant to run under the
 * host address and undefined-behaviour sanitizers: every entry point with
 * NULL handles and bad arguments; with a GPU also a small context whose saved
 * state is restored from corrupted buffers (wrong length, magic, sizes,
 * sample count) before the intact one, and the SHC and virial objects'
 * argument checks.  Exit status 0 when every call returns what the header
 * promises; the first mismatch is printed and gives 1.  Without a GPU the
 * device part is skipped (exit 0, "no device" printed). */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "mhc.h"

static int fails = 0;

#define EXPECT(call, want)                                                                       \
  do {                                                                                           \
    mhc_status st_ = (call);                                                                     \
    if (st_ != (want)) {                                                                         \
      fprintf(stderr, "line %d: %s returned %s, expected %s\n", __LINE__, #call,               \
              mhc_status_string(st_), mhc_status_string(want));                                  \
      ++fails;                                                                                   \
    }                                                                                            \
  } while (0)

static void host_only(void) {
  for (int s = -1; s <= 8; ++s)
    if (!mhc_status_string((mhc_status)s)) ++fails;
  if (mhc_abi_version() != MHC_ABI_VERSION) ++fails;
  double f[257];
  int32_t b[257];
  for (int i = 0; i < 257; ++i) f[i] = 0.125 * i - 3.0;
  EXPECT(mhc_bins_uniform(257, f, 17, 0.0, 20.0, b), MHC_OK);
  for (int i = 0; i < 257; ++i)
    if (b[i] < -1 || b[i] >= 17) ++fails;
  EXPECT(mhc_bins_uniform(0, f, 17, 0.0, 20.0, b), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_bins_uniform(257, NULL, 17, 0.0, 20.0, b), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_bins_uniform(257, f, 0, 0.0, 20.0, b), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_bins_uniform(257, f, 17, 1.0, 1.0, b), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_bins_uniform(257, f, 17, 0.0, 20.0, NULL), MHC_ERR_INVALID_ARG);
  /* NULL handles */
  EXPECT(mhc_create(0, NULL, NULL), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_destroy(NULL), MHC_OK);
  EXPECT(mhc_load_system(NULL, 1, f, 1, f), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_set_bins(NULL, 1, b), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_set_bins_uniform(NULL, 1, 0.0, 1.0), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_configure(NULL, NULL), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_load_eigvec_rows(NULL, 0, 1, f, 0), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_finalize(NULL), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_push(NULL, 1, NULL, NULL, 0), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_push_noalloc(NULL, 1, NULL, NULL), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_read_hnema(NULL, NULL, NULL, NULL), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_read_gkma(NULL, NULL, NULL, NULL, NULL), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_save_state(NULL, NULL, NULL), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_load_state(NULL, NULL, 0), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_group_create(NULL, 0, 0, NULL), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_group_push(NULL, 1, NULL, NULL, 0), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_group_destroy(NULL), MHC_OK);
  EXPECT(mhc_shc_create(0, NULL, 0, 10, 64, NULL), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_shc_push(NULL, 1, NULL, NULL, 0), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_shc_load_state(NULL, NULL, 0), MHC_ERR_INVALID_ARG);
  {
    mhc_shc_group* gr = NULL;
    mhc_shc* none[2] = {NULL, NULL};
    EXPECT(mhc_shc_group_create(none, 2, NULL), MHC_ERR_INVALID_ARG);
    EXPECT(mhc_shc_group_create(NULL, 1, &gr), MHC_ERR_INVALID_ARG);
    EXPECT(mhc_shc_group_create(none, 0, &gr), MHC_ERR_INVALID_ARG);
    EXPECT(mhc_shc_group_create(none, 2, &gr), MHC_ERR_INVALID_ARG);
    EXPECT(mhc_shc_group_push(NULL, 1, NULL, NULL, 0), MHC_ERR_INVALID_ARG);
    EXPECT(mhc_shc_group_destroy(NULL), MHC_OK);
    if (!mhc_shc_group_last_error(NULL)) ++fails;
  }
  EXPECT(mhc_virial_compute(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_virial_destroy(NULL), MHC_OK);
  if (!mhc_last_error(NULL) || !mhc_shc_last_error(NULL) || !mhc_virial_last_error(NULL)) ++fails;
  /* virial argument checks (before any HIP call) */
  mhc_tersoff_params p = {1830.8, 471.18, 2.4799, 1.7322, 0.0, 3, 0, 1.1e-6, 0.78734, 1.0039e5, 16.217, -0.59825,
                          1.0, 2.85, 0.15};
  double m[8] = {28, 28, 28, 28, 28, 28, 28, 28}, box[3] = {5.0, 10.0, 10.0};
  mhc_virial* v = NULL;
  EXPECT(mhc_virial_create(0, NULL, 8, m, box, &p, 16, 0.0, &v), MHC_ERR_INVALID_ARG);
  box[0] = 10.0;
  p.m = 2;
  EXPECT(mhc_virial_create(0, NULL, 8, m, box, &p, 16, 0.0, &v), MHC_ERR_INVALID_ARG);
  p.m = 3;
  EXPECT(mhc_virial_create(0, NULL, 8, m, box, &p, 0, 0.0, &v), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_virial_create(0, NULL, 8, m, box, &p, 16, -1.0, &v), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_virial_create(0, NULL, 0, m, box, &p, 16, 0.0, &v), MHC_ERR_INVALID_ARG);
}

static void device_part(mhc_ctx* ctx) {
  const int64_t N = 4, M = 12, S = 70;
  double mass[4] = {28.0, 29.0, 30.0, 28.5}, freq[12], rows[12 * 12];
  for (int i = 0; i < 12; ++i) freq[i] = 1.5 * i;
  memset(rows, 0, sizeof rows);
  for (int i = 0; i < 12; ++i) rows[i * 12 + i] = 1.0;     /* identity basis: orthonormal */
  float* vv = malloc(sizeof(float) * S * N * 3);
  float* WW = malloc(sizeof(float) * S * N * 9);
  if (!vv || !WW) exit(3);
  unsigned s = 12345u;
  for (int64_t i = 0; i < S * N * 3; ++i) vv[i] = (float)((s = s * 1103515245u + 12345u) % 2001) * 1e-3f - 1.0f;
  for (int64_t i = 0; i < S * N * 9; ++i) WW[i] = (float)((s = s * 1103515245u + 12345u) % 2001) * 1e-3f - 1.0f;
  mhc_run_config cfg = {MHC_HNEMA | MHC_GKMA, MHC_PREC_FP32, 32, 8, 1.0, 1, MHC_SCHED_AUTO, {0, 0}};
  EXPECT(mhc_finalize(ctx), MHC_ERR_STATE);
  EXPECT(mhc_load_system(ctx, 0, mass, 1, freq), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_load_system(ctx, N, mass, 3 * N + 1, freq), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_load_system(ctx, N, mass, M, freq), MHC_OK);
  EXPECT(mhc_set_bins_uniform(ctx, 5, 0.0, 20.0), MHC_OK);
  cfg.reserved[0] = 1;
  EXPECT(mhc_configure(ctx, &cfg), MHC_ERR_INVALID_ARG);
  cfg.reserved[0] = 0;
  cfg.t_block = 48;
  EXPECT(mhc_configure(ctx, &cfg), MHC_ERR_INVALID_ARG);
  cfg.t_block = 32;
  EXPECT(mhc_configure(ctx, &cfg), MHC_OK);
  EXPECT(mhc_load_eigvec_rows(ctx, 5, 8, rows, 0), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_load_eigvec_rows(ctx, 0, M, NULL, 0), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_load_eigvec_rows(ctx, 0, M, rows, 2), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_load_eigvec_rows(ctx, 0, 5, rows, 0), MHC_OK);
  EXPECT(mhc_finalize(ctx), MHC_ERR_STATE);                   /* rows 5.. missing */
  EXPECT(mhc_load_eigvec_rows(ctx, 5, M - 5, rows + 5 * 12, 0), MHC_OK);
  size_t len = 0;
  EXPECT(mhc_save_state(ctx, NULL, &len), MHC_ERR_STATE);
  EXPECT(mhc_finalize(ctx), MHC_OK);
  EXPECT(mhc_push(ctx, -1, vv, WW, 0), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_push(ctx, 3, NULL, WW, 0), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_push(ctx, (int32_t)S, vv, WW, 0), MHC_OK);
  WW[17] = 1.0f / 0.0f;                                        /* check_finite = 1 */
  EXPECT(mhc_push(ctx, 3, vv, WW, 0), MHC_ERR_NONFINITE);
  WW[17] = 0.5f;
  EXPECT(mhc_save_state(ctx, NULL, NULL), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_save_state(ctx, NULL, &len), MHC_OK);
  char* buf = malloc(len + 16);
  char* bad = malloc(len + 16);
  if (!buf || !bad) exit(3);
  size_t small = len - 1;
  EXPECT(mhc_save_state(ctx, buf, &small), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_save_state(ctx, buf, &len), MHC_OK);
  double avg0[15], avg1[15];
  int64_t n0 = 0, n1 = 0;
  EXPECT(mhc_read_hnema(ctx, avg0, NULL, &n0), MHC_OK);
  EXPECT(mhc_reset(ctx), MHC_OK);
  EXPECT(mhc_load_state(ctx, buf, len - 1), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_load_state(ctx, buf, len + 1), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_load_state(ctx, NULL, len), MHC_ERR_INVALID_ARG);
  /* corrupted header fields: magic, N, M, nb, L, methods, a negative sample count */
  const size_t offs[] = {0, 8, 16, 24, 32, 64};
  for (size_t k = 0; k < sizeof offs / sizeof offs[0]; ++k) {
    memcpy(bad, buf, len);
    bad[offs[k]] ^= 0x5A;
    EXPECT(mhc_load_state(ctx, bad, len), MHC_ERR_INVALID_ARG);
  }
  memcpy(bad, buf, len);
  int64_t neg = -5;
  memcpy(bad + 56, &neg, 8);
  EXPECT(mhc_load_state(ctx, bad, len), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_read_hnema(ctx, avg1, NULL, &n1), MHC_OK);
  if (n1 != 0) ++fails;                                        /* still the reset state */
  EXPECT(mhc_load_state(ctx, buf, len), MHC_OK);
  EXPECT(mhc_read_hnema(ctx, avg1, NULL, &n1), MHC_OK);
  if (n1 != n0 || memcmp(avg0, avg1, sizeof avg0) != 0) {
    fprintf(stderr, "restored state differs\n");
    ++fails;
  }
  EXPECT(mhc_read_gkma(ctx, NULL, NULL, NULL, NULL), MHC_OK);
  EXPECT(mhc_read_block_currents(ctx, 1000, avg1), MHC_ERR_INVALID_ARG);
  /* groups: duplicates and wrong counts */
  mhc_ctx* two[2] = {ctx, ctx};
  mhc_group* g = NULL;
  EXPECT(mhc_group_create(two, 2, 0, &g), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_group_create(two, 0, 0, &g), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_group_create(two, 1, 0, &g), MHC_OK);
  EXPECT(mhc_group_push(g, -1, NULL, NULL, 0), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_group_destroy(g), MHC_OK);
  /* SHC: arguments and a corrupted state */
  mhc_shc* sh = NULL;
  EXPECT(mhc_shc_create(0, NULL, N, 0, 64, &sh), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_shc_create(0, NULL, N, 10, 63, &sh), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_shc_create(0, NULL, N, 10, 64, &sh), MHC_OK);
  EXPECT(mhc_shc_push(sh, (int32_t)S, vv, WW, 0), MHC_OK);
  size_t sl = 0;
  EXPECT(mhc_shc_save_state(sh, NULL, &sl), MHC_OK);
  char* sb = malloc(sl);
  if (!sb) exit(3);
  EXPECT(mhc_shc_save_state(sh, sb, &sl), MHC_OK);
  EXPECT(mhc_shc_load_state(sh, sb, sl - 8), MHC_ERR_INVALID_ARG);
  sb[0] ^= 0x21;
  EXPECT(mhc_shc_load_state(sh, sb, sl), MHC_ERR_INVALID_ARG);
  double Kw[3], om = 0.1;
  EXPECT(mhc_shc_spectrum(sh, 0, &om, 1.0, 0, Kw), MHC_ERR_INVALID_ARG);
  EXPECT(mhc_shc_spectrum(sh, 1, &om, 1.0, 0, Kw), MHC_OK);
  /* SHC groups: duplicates, arguments, one host push */
  {
    mhc_shc* dup[2] = {sh, sh};
    mhc_shc_group* sg = NULL;
    const float* gv[1] = {vv};
    const float* gW[1] = {WW};
    const float* gnull[1] = {NULL};
    EXPECT(mhc_shc_group_create(dup, 2, &sg), MHC_ERR_INVALID_ARG);
    EXPECT(mhc_shc_group_create(dup, 1, &sg), MHC_OK);
    EXPECT(mhc_shc_group_push(sg, -1, gv, gW, 0), MHC_ERR_INVALID_ARG);
    EXPECT(mhc_shc_group_push(sg, 1, gnull, gW, 0), MHC_ERR_INVALID_ARG);
    EXPECT(mhc_shc_group_push(sg, 1, gv, gW, 2), MHC_ERR_INVALID_ARG);
    EXPECT(mhc_shc_group_push(sg, (int32_t)S, gv, gW, 0), MHC_OK);
    EXPECT(mhc_shc_group_destroy(sg), MHC_OK);
  }
  EXPECT(mhc_shc_destroy(sh), MHC_OK);
  free(sb);
  free(buf);
  free(bad);
  free(vv);
  free(WW);
}

int main(void) {
  host_only();
  mhc_ctx* ctx = NULL;
  const mhc_status st = mhc_create(0, NULL, &ctx);
  if (st == MHC_OK) {
    device_part(ctx);
    EXPECT(mhc_destroy(ctx), MHC_OK);
  } else {
    printf("no device (%s): host-only paths checked\n", mhc_last_error(NULL));
  }
  /* Leave without the HIP runtime's own global teardown: under the host
   * sanitizer runtime that teardown trips the sanitizer's device-allocator
   * check after main returns.  Everything of ours was released above. */
  if (fails) {
    fprintf(stderr, "%d unexpected result(s)\n", fails);
    fflush(NULL);
    _Exit(1);
  }
  printf("abi_errors: ok\n");
  fflush(NULL);
  _Exit(0);
}

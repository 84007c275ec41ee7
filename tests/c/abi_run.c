/* End-to-end use of the C ABI from plain C99 (test driver): reads a case
 * written by the Python test, runs HNEMA + GKMA on the GPU through
 * include/mhc.h, writes the results.
 *
 * Input file (native endianness):
 *   int64 N, M, S; int32 nb, L, T, prec
 *   double mass[N], freq[M]; int32 bins[M]; double rows[M][3N] (E^T)
 *   float v[S][N][3], W[S][N][3][3]
 * Output file: double avg[nb][3], total[3], corr[L][nb][3][3], hcacf[L][3][3]; int64 n_samples */
#include <stdio.h>
#include <stdlib.h>
#include "mhc.h"

#define CHECK(call)                                                                  \
  do {                                                                               \
    mhc_status st_ = (call);                                                         \
    if (st_ != MHC_OK) {                                                             \
      fprintf(stderr, "%s failed: %s: %s\n", #call, mhc_status_string(st_),          \
              mhc_last_error(ctx));                                                  \
      return 2;                                                                      \
    }                                                                                \
  } while (0)

static void* read_all(FILE* f, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (p && bytes && fread(p, 1, bytes, f) != bytes) {
    free(p);
    return NULL;
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 3) return 1;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 1;
  int64_t N, M, S;
  int32_t nb, L, T, prec;
  if (fread(&N, 8, 1, f) != 1 || fread(&M, 8, 1, f) != 1 || fread(&S, 8, 1, f) != 1 || fread(&nb, 4, 1, f) != 1 ||
      fread(&L, 4, 1, f) != 1 || fread(&T, 4, 1, f) != 1 || fread(&prec, 4, 1, f) != 1)
    return 1;
  double* mass = read_all(f, (size_t)N * 8);
  double* freq = read_all(f, (size_t)M * 8);
  int32_t* bins = read_all(f, (size_t)M * 4);
  double* rows = read_all(f, (size_t)M * 3 * N * 8);
  float* v = read_all(f, (size_t)S * N * 3 * 4);
  float* W = read_all(f, (size_t)S * N * 9 * 4);
  fclose(f);
  if (!mass || !freq || !bins || !rows || !v || !W) return 1;

  mhc_ctx* ctx = NULL;
  if (mhc_create(0, NULL, &ctx) != MHC_OK) {
    fprintf(stderr, "create: %s\n", mhc_last_error(NULL));
    return 2;
  }
  mhc_run_config cfg = {MHC_HNEMA | MHC_GKMA, prec, T, L, 1.0, 0, MHC_SCHED_AUTO, {0, 0}};
  CHECK(mhc_load_system(ctx, N, mass, M, freq));
  CHECK(mhc_set_bins(ctx, nb, bins));
  CHECK(mhc_configure(ctx, &cfg));
  for (int64_t r0 = 0; r0 < M; r0 += 100) {
    const int64_t n = M - r0 < 100 ? M - r0 : 100;
    CHECK(mhc_load_eigvec_rows(ctx, r0, n, rows + r0 * 3 * N, 0));
  }
  CHECK(mhc_finalize(ctx));
  /* uneven pushes from host memory */
  CHECK(mhc_push(ctx, 1, v, W, 0));
  CHECK(mhc_push(ctx, (int32_t)(S - 1), v + N * 3, W + N * 9, 0));

  double* avg = malloc((size_t)nb * 3 * 8);
  double total[3];
  double* corr = malloc((size_t)L * nb * 9 * 8);
  double* hcacf = malloc((size_t)L * 9 * 8);
  int64_t n_samples = 0, n2 = 0;
  CHECK(mhc_read_hnema(ctx, avg, total, &n_samples));
  CHECK(mhc_read_gkma(ctx, corr, NULL, hcacf, &n2));
  CHECK(mhc_destroy(ctx));
  if (n2 != n_samples) return 3;

  FILE* o = fopen(argv[2], "wb");
  if (!o) return 1;
  fwrite(avg, 8, (size_t)nb * 3, o);
  fwrite(total, 8, 3, o);
  fwrite(corr, 8, (size_t)L * nb * 9, o);
  fwrite(hcacf, 8, (size_t)L * 9, o);
  fwrite(&n_samples, 8, 1, o);
  fclose(o);
  free(mass); free(freq); free(bins); free(rows); free(v); free(W); free(avg); free(corr); free(hcacf);
  /* without the HIP runtime's global teardown (see abi_errors.c) */
  fflush(NULL);
  _Exit(0);
}

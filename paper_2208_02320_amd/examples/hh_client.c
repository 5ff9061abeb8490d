/*
 * A plain C client of the library: no Python, no torch, host buffers only.
 *
 *   hh_client host   the host-only entry points (size table, Voigt moduli,
 *                    n^-1 fit) and context creation, which fails with
 *                    HH_EDEVICE where there is no gfx950 device
 *   hh_client solve  one solve on device 0: a two-phase laminate with
 *                    layers of `t` voxels normal to z in an n^3 box, then
 *                    the two-level scheme (n/2 blocks) on the same image;
 *                    prints both C
 *
 * Output lines are `key value...` so that a caller can parse them.
 * Exit status: 0 on success, 1 on a failing call (its message is printed).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hh.h"

static void print_matrix(const char *key, const double C[36]) {
  printf("%s", key);
  for (int i = 0; i < 36; ++i) printf(" %.17g", C[i]);
  printf("\n");
}

static int host_checks(void) {
  printf("supported_f32 256 %d 7 %d\n", hh_size_supported(256, 0), hh_size_supported(7, 0));
  /* isotropic stiffness with lambda = 2, mu = 3 (Voigt, engineering shear) */
  double C[36] = {0};
  const double lam = 2.0, mu = 3.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i * 6 + j] = lam + (i == j ? 2.0 * mu : 0.0);
  for (int i = 3; i < 6; ++i) C[i * 6 + i] = mu;
  double K = 0.0, G = 0.0;
  if (hh_moduli(C, &K, &G) != HH_OK) return 1;
  printf("moduli %.17g %.17g\n", K, G);
  /* exact data M(n) = 5 + 40 / n for every entry */
  const int n[3] = {16, 32, 64};
  double Cm[3 * 36], Cinf[36], slope[36];
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 36; ++i) Cm[k * 36 + i] = 5.0 + 40.0 / n[k];
  if (hh_richardson(n, Cm, 3, Cinf, slope) != HH_OK) return 1;
  printf("richardson %.17g %.17g\n", Cinf[0], slope[0]);
  hh_ctx *ctx = NULL;
  const int rc = hh_create(&ctx, 0, NULL);
  printf("create %d\n", rc);
  if (rc != HH_OK) fprintf(stderr, "hh_create: %s\n", hh_last_error(NULL));
  hh_destroy(ctx);
  return 0;
}

static int solve(int n, int t) {
  hh_ctx *ctx = NULL;
  if (hh_create(&ctx, 0, NULL) != HH_OK) {
    fprintf(stderr, "hh_create failed: %s\n", hh_last_error(NULL));
    hh_destroy(ctx);
    return 1;
  }
  const size_t nv = (size_t)n * n * n;
  uint8_t *lab = (uint8_t *)malloc(nv);
  if (!lab) {
    hh_destroy(ctx);
    return 1;
  }
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) lab[((size_t)z * n + y) * n + x] = (uint8_t)((z / t) % 2);
  const hh_phase ph[2] = {{37.0, 44.0}, {2.25, 1.0}};
  hh_opts o;
  hh_default_opts(&o);
  o.tol = 1e-6;
  double C[36], Craw[36];
  hh_report rep;
  int rc = hh_homogenize(ctx, lab, n, n, n, 0, ph, 2, NULL, NULL, &o, C, Craw, &rep);
  if (rc != HH_OK) {
    fprintf(stderr, "hh_homogenize: %s\n", hh_last_error(ctx));
  } else {
    print_matrix("C", C);
    printf("iters %d %d %d %d %d %d\n", rep.iters[0], rep.iters[1], rep.iters[2], rep.iters[3], rep.iters[4],
           rep.iters[5]);
    double Ch[36];
    rc = hh_hierarchical(ctx, lab, n, n, n, 0, ph, 2, n / 2, 0, 0, &o, Ch, NULL, &rep);
    if (rc != HH_OK)
      fprintf(stderr, "hh_hierarchical: %s\n", hh_last_error(ctx));
    else
      print_matrix("C_two_level", Ch);
  }
  free(lab);
  hh_destroy(ctx);
  return rc == HH_OK ? 0 : 1;
}

int main(int argc, char **argv) {
  if (argc >= 2 && strcmp(argv[1], "host") == 0) return host_checks();
  if (argc >= 2 && strcmp(argv[1], "solve") == 0) {
    const int n = argc >= 3 ? atoi(argv[2]) : 16;
    const int t = argc >= 4 ? atoi(argv[3]) : 4;
    if (n <= 0 || t <= 0) return 1;
    return solve(n, t);
  }
  fprintf(stderr, "usage: %s host | solve [n [t]]\n", argv[0]);
  return 2;
}

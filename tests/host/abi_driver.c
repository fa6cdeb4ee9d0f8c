/* Host-side exercise of the C ABI for the sanitizer build
 * (tests/test_host_sanitizers.py): every validation path, the axis tables
 * and plans over many lengths with exactly sized output buffers, the kernel
 * shape table, and the calls that must refuse NULL arguments.  Needs no GPU:
 * plan creation may report MPOIS_ERR_DEVICE.  Prints "ok" and returns 0 when
 * every result is one the header allows. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "mpois.h"

static int fails = 0;

static void expect(int cond, const char* what) {
  if (!cond) {
    fprintf(stderr, "FAILED: %s\n", what);
    ++fails;
  }
}

static mpois_grid_desc desc(int ndim, const int64_t* n, const double* h, const int (*bc)[2], const int* grid,
                            double shift) {
  mpois_grid_desc d;
  d.ndim = ndim;
  for (int i = 0; i < 3; ++i) {
    d.n[i] = i < ndim ? n[i] : 1;
    d.h[i] = i < ndim ? h[i] : 1.0;
    d.bc[i][0] = i < ndim ? bc[i][0] : 0;
    d.bc[i][1] = i < ndim ? bc[i][1] : 0;
    d.grid[i] = i < ndim ? grid[i] : 0;
  }
  d.shift = shift;
  return d;
}

int main(void) {
  for (int s = -1; s <= 8; ++s) expect(mpois_status_string((mpois_status)s) != NULL, "status string");

  /* validation over face pairs, grids, sizes, spacings, shifts */
  const int64_t sizes[] = {0, 1, 2, 3, 17, 1024, -5};
  const double spacings[] = {1.0, 0.0, -1.0, NAN, INFINITY, 1e-300};
  const double shifts[] = {0.0, 2.5, -1.0, NAN};
  for (int ndim = 0; ndim <= 4; ++ndim)
    for (int lo = -1; lo <= 3; ++lo)
      for (int hi = 0; hi <= 2; ++hi)
        for (int g = -1; g <= 2; ++g)
          for (int si = 0; si < 7; ++si)
            for (int hi2 = 0; hi2 < 6; ++hi2) {
              int64_t n[3] = {sizes[si], 5, 7};
              double h[3] = {spacings[hi2], 0.1, 0.2};
              int bc[3][2] = {{lo, hi}, {0, 0}, {2, 2}};
              int grid[3] = {g, 1, 0};
              mpois_grid_desc d = desc(ndim < 3 ? ndim : 3, n, h, (const int(*)[2])bc, grid, shifts[(si + hi2) % 4]);
              d.ndim = ndim;
              for (int approx = -1; approx <= 2; ++approx)
                for (int prec = -1; prec <= 3; ++prec) {
                  mpois_status st = mpois_validate(&d, approx, prec, 2);
                  expect(st == MPOIS_OK || st == MPOIS_ERR_INVALID || st == MPOIS_ERR_UNSUPPORTED, "validate status");
                }
            }
  expect(mpois_validate(NULL, 1, 0, 1) == MPOIS_ERR_INVALID, "validate NULL");

  /* eigenvalues and plans: output buffers sized exactly */
  for (int code = 0; code <= 4; ++code)
    for (int g = 0; g <= 1; ++g)
      for (int approx = 0; approx <= 1; ++approx)
        for (int64_t n = 1; n <= 700; n += (n < 64 ? 1 : 37)) {
          double* out = (double*)malloc((size_t)n * sizeof(double));
          mpois_status st = mpois_axis_eigenvalues(code, g, approx, n, 0.01, out);
          expect(st == MPOIS_OK || st == MPOIS_ERR_INVALID || st == MPOIS_ERR_UNSUPPORTED, "eigenvalue status");
          if (st == MPOIS_OK)
            for (int64_t k = 0; k < n; ++k) expect(isfinite(out[k]) && out[k] <= 0.0, "eigenvalue sign");
          free(out);
        }
  for (int code = 0; code <= 4; ++code)
    for (int g = 0; g <= 1; ++g)
      for (int64_t n = 1; n <= 2100; ++n) {
        int kf, kb, M, P, nr;
        int* rad = (int*)malloc(16 * sizeof(int));
        mpois_status st = mpois_axis_plan(code, g, n, &kf, &kb, &M, &P, rad, 16, &nr);
        expect(st == MPOIS_OK || st == MPOIS_ERR_INVALID || st == MPOIS_ERR_UNSUPPORTED, "axis plan status");
        if (st == MPOIS_OK) {
          long prod = 1;
          for (int i = 0; i < nr && i < 16; ++i) prod *= rad[i];
          expect(nr <= 16 && prod == P && P >= M, "radices multiply to P");
        }
        free(rad);
      }
  for (int cfg = -2; cfg < 400; ++cfg) {
    int eb, np, nt, ml;
    mpois_status st = mpois_kernel_shape(cfg, &eb, &np, &nt, &ml);
    expect(st == MPOIS_OK || st == MPOIS_ERR_INVALID, "kernel shape status");
  }

  /* NULL handles and arguments */
  expect(mpois_destroy(NULL) == MPOIS_OK, "destroy NULL");
  expect(mpois_workspace_bytes(NULL) == 0, "workspace NULL");
  expect(mpois_execute(NULL, NULL, NULL, NULL) == MPOIS_ERR_INVALID, "execute NULL");
  expect(mpois_execute_view(NULL, NULL, NULL, NULL, NULL, NULL) == MPOIS_ERR_INVALID, "execute_view NULL");
  expect(mpois_execute_noalloc(NULL, NULL, NULL, NULL) == MPOIS_ERR_INVALID, "noalloc NULL");
  expect(mpois_execute_batch(NULL, NULL, NULL, NULL) == MPOIS_ERR_INVALID, "batch NULL");
  expect(mpois_project(NULL, NULL, NULL, 0.5, NULL, NULL) == MPOIS_ERR_INVALID, "project NULL");
  mpois_info info;
  expect(mpois_get_info(NULL, NULL, &info) == MPOIS_ERR_INVALID, "info NULL");

  /* plan creation: without a GPU the library reports DEVICE; with one, a plan */
  {
    int64_t n[3] = {8, 9, 10};
    double h[3] = {0.1, 0.2, 0.3};
    int bc[3][2] = {{0, 0}, {1, 2}, {2, 2}};
    int grid[3] = {0, 1, 0};
    mpois_grid_desc d = desc(3, n, h, (const int(*)[2])bc, grid, 0.0);
    for (int prec = 0; prec <= 2; ++prec) {
      mpois_plan p = NULL;
      mpois_status st = mpois_plan_create(&d, 1, prec, 0.0, 2, 0, &p);
      expect(st == MPOIS_OK || st == MPOIS_ERR_DEVICE, "plan create");
      expect((st == MPOIS_OK) == (p != NULL), "plan handle only on success");
      if (p) expect(mpois_destroy(p) == MPOIS_OK, "destroy");
    }
    mpois_plan p = NULL;
    expect(mpois_plan_create_batch(&d, 0, 1, 0, 0.0, 2, 0, &p) == MPOIS_ERR_INVALID && !p, "empty batch");
  }
  /* plans whose tables take every construction path (Rader-73, Bluestein,
   * odd radices, mixed faces, Helmholtz), single and batched, with the tuner */
  {
    const int64_t lens[] = {512, 1021, 147, 200, 33, 2, 1000};
    mpois_grid_desc ds[28];
    int nd = 0;
    for (int i = 0; i < 7; ++i)
      for (int code = 0; code < 4; ++code) {
        int64_t n[3] = {lens[i], 6, 5};
        double h[3] = {1.0 / (double)lens[i], 0.2, 0.1};
        int lo = code == 3 ? 1 : code, hi = code == 3 ? 2 : code;
        int bc[3][2] = {{lo, hi}, {2, 2}, {0, 0}};
        int grid[3] = {i % 2, 1, 0};
        ds[nd++] = desc(1 + i % 3, n, h, (const int(*)[2])bc, grid, code == 2 ? 0.5 : 0.0);
      }
    for (int i = 0; i < nd; ++i)
      for (int prec = 0; prec <= 2; ++prec) {
        mpois_plan p = NULL;
        mpois_status st = mpois_plan_create(&ds[i], 1, prec, 0.0, 2, i % 5 == 0 ? MPOIS_FLAG_TUNE : 0u, &p);
        expect(st == MPOIS_OK || st == MPOIS_ERR_DEVICE || st == MPOIS_ERR_INVALID, "plan create (tables)");
        if (p) mpois_destroy(p);
      }
    /* a batch needs one ndim: the 2D descriptors */
    mpois_grid_desc b2[28];
    int nb = 0;
    for (int i = 0; i < nd; ++i)
      if (ds[i].ndim == 2 && mpois_validate(&ds[i], 1, 2, 2) == MPOIS_OK) b2[nb++] = ds[i];
    mpois_plan p = NULL;
    mpois_status st = mpois_plan_create_batch(b2, nb, 1, 2, 0.0, 2, MPOIS_FLAG_TUNE, &p);
    expect(st == MPOIS_OK || st == MPOIS_ERR_DEVICE, "batch plan create");
    if (p) mpois_destroy(p);
  }
  if (fails) return 1;
  printf("ok\n");
  return 0;
}

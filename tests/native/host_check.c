/* Host-code check of the C-ABI under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (test infrastructure). Linked against a host-only build of the
 * library (no device code: on a machine without a GPU every call that needs
 * a device must fail cleanly), it exercises argument validation, error
 * reporting and the CMA-ES search (Sec. 4), which run entirely on the host.
 * Exit status 0 when every check holds; sanitizer reports abort the run. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "sos.h"

static int failures = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

static int setup_code(sos_mesh* m, sos_partition* p, sos_robin* r, sos_opts* o) {
  sos_ctx* ctx = (sos_ctx*)0x1;
  const int rc = sos_setup(m, p, r, o, &ctx);
  CHECK(ctx == NULL);
  if (rc != SOS_OK) CHECK(strlen(sos_last_error()) > 0);
  return rc;
}

int main(void) {
  sos_opts o;
  CHECK(sos_opts_default(&o, SOS_FP64) == SOS_OK);
  CHECK(o.mode == SOS_STEPWISE && o.inner_abs == 1e-10 && o.G == 6.672e-11);
  CHECK(sos_opts_default(&o, SOS_FP32_INNER) == SOS_OK && o.mode == SOS_BATCHED && o.inner_tol == 1e-2);
  CHECK(sos_opts_default(NULL, SOS_FP64) == SOS_EINVAL);

  sos_mesh m = {{4, 4, 4}, {1.0, 1.0, 1.0}, {0, 0, 0, 0, 0, 0}};
  sos_partition p = {{2, 1, 1}, {NULL, NULL, NULL}};
  sos_robin r = {0, 8.0, 0.0, NULL, NULL};
  sos_opts_default(&o, SOS_FP64);

  /* invalid arguments: SOS_EINVAL before any device access */
  int bad_cuts[2] = {2, 2};
  sos_partition pc = {{3, 1, 1}, {bad_cuts, NULL, NULL}};
  CHECK(setup_code(&m, &pc, &r, &o) == SOS_EINVAL);
  sos_partition pe = {{3, 1, 1}, {NULL, NULL, NULL}};
  CHECK(setup_code(&m, &pe, &r, &o) == SOS_EINVAL);           /* 3 does not divide 4 */
  sos_robin rneg = {0, -1.0, 0.0, NULL, NULL};
  CHECK(setup_code(&m, &p, &rneg, &o) == SOS_EINVAL);         /* p <= 0 */
  sos_robin rnan = {0, NAN, 0.0, NULL, NULL};
  CHECK(setup_code(&m, &p, &rnan, &o) == SOS_EINVAL);
  sos_robin rq = {2, 8.0, -0.5, NULL, NULL};
  CHECK(setup_code(&m, &p, &rq, &o) == SOS_EINVAL);           /* q < 0 */
  sos_mesh mn = {{4, 4, 4}, {1.0, 1.0, 1.0}, {1, 1, 1, 1, 1, 1}};
  CHECK(setup_code(&mn, &p, &r, &o) == SOS_EINVAL);           /* all Neumann */
  sos_mesh m0 = {{0, 4, 4}, {1.0, 1.0, 1.0}, {0, 0, 0, 0, 0, 0}};
  CHECK(setup_code(&m0, &p, &r, &o) == SOS_EINVAL);
  sos_opts ob = o;
  ob.max_outer = 0;
  CHECK(setup_code(&m, &p, &r, &ob) == SOS_EINVAL);
  ob = o;
  ob.block = 100;
  CHECK(setup_code(&m, &p, &r, &ob) == SOS_EINVAL);
  ob = o;
  ob.team = 9;
  CHECK(setup_code(&m, &p, &r, &ob) == SOS_EINVAL);
  ob = o;
  ob.schedule = 2;
  CHECK(setup_code(&m, &p, &r, &ob) == SOS_EINVAL);
  double pf[2] = {1.0, 0.0};
  sos_robin rpf = {0, 0.0, 0.0, pf, NULL};
  CHECK(setup_code(&m, &p, &rpf, &o) == SOS_EINVAL);          /* per-face p <= 0 */
  CHECK(sos_setup(NULL, &p, &r, &o, NULL) == SOS_EINVAL);
  sos_ctx* ctx = NULL;
  CHECK(sos_setup_batch(&m, &p, 0, &r, &o, &ctx) == SOS_EINVAL && ctx == NULL);

  /* a valid problem needs a device: without one it fails cleanly */
  const int rc = setup_code(&m, &p, &r, &o);
  CHECK(rc == SOS_OK || rc == SOS_ESTATE);
  if (rc == SOS_OK) fprintf(stderr, "note: a device is present\n");

  /* calls on a NULL context */
  CHECK(sos_solve(NULL, NULL, 1e-8, NULL, NULL) == SOS_EINVAL);
  CHECK(sos_iterate(NULL, 1, NULL) == SOS_EINVAL);
  int32_t n = -1;
  CHECK(sos_faces(NULL, &n, NULL) == SOS_EINVAL);
  CHECK(sos_history(NULL, 0, &n, NULL, NULL) == SOS_EINVAL);
  CHECK(sos_inner_iters(NULL, 0, &n, NULL) == SOS_EINVAL);
  sos_destroy(NULL);

  /* CMA-ES on the two-subdomain Fourier factor, every kind */
  double pq[4], rho = 0.0, rho0 = 0.0;
  int32_t it = 0;
  for (int kind = 0; kind < 4; ++kind) {
    CHECK(sos_optimize_robin(kind, 0.0174, 1.0, 401, 25, 2000, 5e-11, 3, pq, &rho, &it) == SOS_OK);
    CHECK(rho > 0.0 && rho < 1.0 && it > 0);
    CHECK(pq[0] > 0.0 && pq[2] > 0.0 && pq[1] >= 0.0 && pq[3] >= 0.0);
    if (kind == 0) rho0 = rho;
    else CHECK(rho <= rho0 * (1 + 1e-9)); /* every richer family does at least as well */
  }
  CHECK(sos_optimize_robin(4, 0.0174, 1.0, 401, 25, 100, 5e-11, 3, pq, &rho, NULL) == SOS_EINVAL);
  CHECK(sos_optimize_robin(0, 1.0, 0.5, 401, 25, 100, 5e-11, 3, pq, &rho, NULL) == SOS_EINVAL);
  CHECK(sos_optimize_robin(0, 0.0174, 1.0, 401, 2, 100, 5e-11, 3, pq, &rho, NULL) == SOS_EINVAL);
  CHECK(sos_optimize_robin(0, 0.0174, 1.0, 401, 25, 100, 5e-11, 3, NULL, &rho, NULL) == SOS_EINVAL);

  if (failures) fprintf(stderr, "%d checks failed\n", failures);
  else printf("host checks passed\n");
  return failures ? 1 : 0;
}

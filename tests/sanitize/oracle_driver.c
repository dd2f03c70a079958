/* Drives the FP64 oracle through every code path a test run takes (2D and
 * 3D, periodic and walled axes, each force kind, both schemes, the
 * constitutive models, read-back and state transfer) so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer can check it.  Exit
 * status 0 when the runs completed and stayed finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void *or_create(int d, int nx, int ny, int nz);
void or_destroy(void *p);
void or_set_params(void *p, double tau_f, double tau_h, double lambda, double eta_p);
void or_set_walls(void *p, const int *walls);
void or_set_force(void *p, int kind, const double *amp, double omega);
void or_set_scheme(void *p, int scheme);
void or_set_model(void *p, int model, double param);
void or_init(void *p, const double *u, const double *tau, const double *pr);
void or_step(void *p, long n);
void or_moments(void *p, double *u, double *pr, double *A, double *tau);
void or_get_state(void *p, double *f, double *h, double *chi, double *up);
void or_set_state(void *p, const double *f, const double *h, const double *chi,
                  const double *up);

static int run(int d, int nx, int ny, int nz, const int *walls, int force, int scheme,
               int model) {
  const int q = d == 2 ? 9 : 19, nc = d == 2 ? 3 : 6;
  const long N = (long)nx * ny * nz;
  void *s = or_create(d, nx, ny, nz);
  if (!s) return 1;
  or_set_params(s, 0.8, 0.501, 50.0, 0.1);
  or_set_walls(s, walls);
  const double amp[3] = {2e-6, -1e-6, 1e-6};
  or_set_force(s, force, amp, 0.1);
  or_set_scheme(s, scheme);
  or_set_model(s, model, 0.2);
  double *u = calloc((size_t)N * d, sizeof(double));
  double *tau = calloc((size_t)N * nc, sizeof(double));
  double *pr = calloc((size_t)N, sizeof(double));
  double *A = calloc((size_t)N * nc, sizeof(double));
  double *f = calloc((size_t)N * q, sizeof(double));
  double *h = calloc((size_t)N * q * nc, sizeof(double));
  double *chi = calloc((size_t)N * nc, sizeof(double));
  double *up = calloc((size_t)N * d, sizeof(double));
  for (long n = 0; n < N; ++n) {
    for (int b = 0; b < d; ++b) u[n * d + b] = 1e-3 * sin(0.3 * n + b);
    for (int c = 0; c < nc; ++c) tau[n * nc + c] = 1e-5 * cos(0.2 * n + c);
    pr[n] = 1e-5 * sin(0.1 * n);
  }
  or_init(s, u, tau, pr);
  or_step(s, 7);
  or_get_state(s, f, h, chi, up);
  or_set_state(s, f, h, chi, up);
  or_step(s, 3);
  or_moments(s, u, pr, A, tau);
  int bad = 0;
  for (long n = 0; n < N * d; ++n) bad |= !isfinite(u[n]);
  for (long n = 0; n < N * nc; ++n) bad |= !isfinite(A[n]);
  or_destroy(s);
  free(u); free(tau); free(pr); free(A); free(f); free(h); free(chi); free(up);
  return bad;
}

int main(void) {
  const int none[3] = {0, 0, 0}, wy[3] = {0, 1, 0}, wall_all[3] = {1, 1, 1};
  int bad = 0;
  for (int force = 0; force < 4; ++force) {
    bad |= run(2, 7, 5, 1, force == 2 ? none : wy, force, 0, 0);
    bad |= run(3, 5, 4, 6, force == 2 ? none : wall_all, force, 0, 0);
  }
  for (int scheme = 0; scheme < 2; ++scheme)
    for (int model = 0; model < 4; ++model) {
      bad |= run(2, 6, 3, 1, wy, 1, scheme, model);
      bad |= run(3, 4, 3, 5, wall_all, 1, scheme, model);
    }
  bad |= run(2, 1, 9, 1, none, 1, 0, 0);   /* one node thin */
  bad |= run(3, 2, 2, 2, wall_all, 1, 1, 0); /* two nodes between walls */
  printf("oracle driver: %s\n", bad ? "non-finite values" : "ok");
  return bad;
}

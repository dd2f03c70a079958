/*
 * vflb_oracle.c -- plain, slow, FP64, single-threaded CPU oracle of the
 * fluctuating lattice Boltzmann method for Oldroyd-B flows
 * (Wang, Liu, Wang, Yu, Ji; "A fluctuating lattice Boltzmann method for
 * viscoelastic fluid flows", arXiv 2506.13072).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP path of the package.
 *
 * Every function follows one passage of the paper, cited in its comment:
 *   Sec. 2.1  governing equations (polymer stress from the conformation
 *             tensor, Oldroyd-B constitutive equation)
 *   Sec. 2.2  fluctuating evolution equation for f_i, Guo forcing term,
 *             incompressible equilibrium, velocity moment, pressure,
 *             D2Q9 velocities/weights, tau_f from the solvent viscosity,
 *             the constraints on f^B from the Chapman-Enskog analysis and
 *             the pseudo-inverse closed form for f^B
 *   Sec. 2.3  advection-diffusion LB for the conformation tensor h_abi
 *   Sec. 3    dimensionless groups, tau_h = 0.501, boundary conditions
 *   App. A    pseudo-inverse matrices (D2Q9 and D3Q19)
 *   App. B    pressure recovery
 * Readings where the paper is silent (gradient stencil, time derivative of
 * the source, wall treatment, D3Q19 weights) are stated at each use.
 *
 * Storage is node-major and unshifted: f[n*Q+i], h[(n*NC+c)*Q+i].  The
 * conformation tensor is symmetric; its independent components are kept in
 * the order (xx, xy, yy) in 2D and (xx, yy, zz, xy, xz, yz) in 3D.
 * State held between steps: the pre-collision populations f, h at time t,
 * and chi(t-1), u(t-1) for the backward difference of the source term.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Velocity sets.  D2Q9 order and weights as printed in Sec. 2.2.      */
/* D3Q19 order as printed in App. A; the weights are not printed, the  */
/* standard isotropic set 1/3, 1/18, 1/36 is used.                     */
/* ------------------------------------------------------------------ */
static const int C2[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W2[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int C3[19][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W3[19] = {
    1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

static const double CS2 = 1.0 / 3.0; /* c_s^2 = c^2/3, c = 1 */

/* symmetric component c -> tensor indices (alpha, beta) */
static const int COMP2[3][2] = {{0, 0}, {0, 1}, {1, 1}};
static const int COMP3[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};

typedef struct {
  int d, q, nc;
  const int (*c)[3];
  const double *w;
  const int (*comp)[2];
  int opp[19];
} lattice;

/* opposite direction: c_j = -c_i */
static int find_opposite(const int (*c)[3], int q, int i) {
  for (int j = 0; j < q; ++j)
    if (c[j][0] == -c[i][0] && c[j][1] == -c[i][1] && c[j][2] == -c[i][2])
      return j;
  return -1;
}

static lattice lat_of(int d) {
  lattice L;
  L.d = d;
  if (d == 2) {
    L.q = 9; L.nc = 3; L.c = C2; L.w = W2; L.comp = COMP2;
  } else {
    L.q = 19; L.nc = 6; L.c = C3; L.w = W3; L.comp = COMP3;
  }
  for (int i = 0; i < L.q; ++i) L.opp[i] = find_opposite(L.c, L.q, i);
  return L;
}

static double cdot(const lattice *L, int i, const double *v) {
  double s = 0.0;
  for (int a = 0; a < L->d; ++a) s += L->c[i][a] * v[a];
  return s;
}

/* ------------------------------------------------------------------ */
/* Pseudo-inverse matrices of App. A, entered as printed.               */
/* ------------------------------------------------------------------ */

/* D2Q9: f^B = -1/(72 tau_f) * M * (tau_yx, tau_xx, tau_xy, tau_yy)^T */
static const double PINV2[9][4] = {
    {0, -24, 0, -24}, {0, 12, 0, -24}, {0, -24, 0, 12},
    {0, 12, 0, -24},  {0, -24, 0, 12}, {9, 12, 9, 12},
    {-9, 12, -9, 12}, {9, 12, 9, 12},  {-9, 12, -9, 12}};

/* D3Q19: f^B = P * b with b = (-t_xx, -t_yy, -t_zz, -t_xy, -t_xz, -t_yx,
 * -t_yz, -t_zx, -t_zy, 0, 0, 0, 0)/tau_f.  Columns 9..12 multiply zeros. */
#define F(a, b) ((double)(a) / (double)(b))
static const double PINV3[19][13] = {
    {F(-5, 21), F(-5, 21), F(-5, 21), 0, 0, 0, 0, 0, 0, 0, 0, 0, F(3, 7)},
    {F(1, 42), F(-1, 7), F(-1, 7), 0, 0, 0, 0, 0, 0, F(1, 10), 0, 0, F(4, 21)},
    {F(1, 42), F(-1, 7), F(-1, 7), 0, 0, 0, 0, 0, 0, F(-1, 10), 0, 0, F(4, 21)},
    {F(-1, 7), F(1, 42), F(-1, 7), 0, 0, 0, 0, 0, 0, 0, F(1, 10), 0, F(4, 21)},
    {F(-1, 7), F(1, 42), F(-1, 7), 0, 0, 0, 0, 0, 0, 0, F(-1, 10), 0, F(4, 21)},
    {F(-1, 7), F(-1, 7), F(1, 42), 0, 0, 0, 0, 0, 0, 0, 0, F(1, 10), F(4, 21)},
    {F(-1, 7), F(-1, 7), F(1, 42), 0, 0, 0, 0, 0, 0, 0, 0, F(-1, 10), F(4, 21)},
    {F(5, 42), F(5, 42), F(-1, 21), F(1, 8), 0, F(1, 8), 0, 0, 0, F(1, 10), F(1, 10), 0, F(-1, 21)},
    {F(5, 42), F(5, 42), F(-1, 21), F(1, 8), 0, F(1, 8), 0, 0, 0, F(-1, 10), F(-1, 10), 0, F(-1, 21)},
    {F(5, 42), F(5, 42), F(-1, 21), F(-1, 8), 0, F(-1, 8), 0, 0, 0, F(1, 10), F(-1, 10), 0, F(-1, 21)},
    {F(5, 42), F(5, 42), F(-1, 21), F(-1, 8), 0, F(-1, 8), 0, 0, 0, F(-1, 10), F(1, 10), 0, F(-1, 21)},
    {F(5, 42), F(-1, 21), F(5, 42), 0, F(1, 8), 0, 0, F(1, 8), 0, F(1, 10), 0, F(1, 10), F(-1, 21)},
    {F(5, 42), F(-1, 21), F(5, 42), 0, F(1, 8), 0, 0, F(1, 8), 0, F(-1, 10), 0, F(-1, 10), F(-1, 21)},
    {F(5, 42), F(-1, 21), F(5, 42), 0, F(-1, 8), 0, 0, F(-1, 8), 0, F(1, 10), 0, F(-1, 10), F(-1, 21)},
    {F(5, 42), F(-1, 21), F(5, 42), 0, F(-1, 8), 0, 0, F(-1, 8), 0, F(-1, 10), 0, F(1, 10), F(-1, 21)},
    {F(-1, 21), F(5, 42), F(5, 42), 0, 0, 0, F(1, 8), 0, F(1, 8), 0, F(1, 10), F(1, 10), F(-1, 21)},
    {F(-1, 21), F(5, 42), F(5, 42), 0, 0, 0, F(1, 8), 0, F(1, 8), 0, F(-1, 10), F(-1, 10), F(-1, 21)},
    {F(-1, 21), F(5, 42), F(5, 42), 0, 0, 0, F(-1, 8), 0, F(-1, 8), 0, F(1, 10), F(-1, 10), F(-1, 21)},
    {F(-1, 21), F(5, 42), F(5, 42), 0, 0, 0, F(-1, 8), 0, F(-1, 8), 0, F(-1, 10), F(1, 10), F(-1, 21)}};
#undef F

/* Copies of the printed matrices, so tests can compare them with a
 * Moore-Penrose pseudo-inverse computed by a library routine. */
void or_pinv_matrix(int d, double *out) {
  if (d == 2) {
    for (int i = 0; i < 9; ++i)
      for (int k = 0; k < 4; ++k) out[i * 4 + k] = PINV2[i][k];
  } else {
    for (int i = 0; i < 19; ++i)
      for (int k = 0; k < 13; ++k) out[i * 13 + k] = PINV3[i][k];
  }
}

/* ------------------------------------------------------------------ */
/* Per-node building blocks.  Vectors have d entries, symmetric tensors */
/* nc entries in the component order above.                             */
/* ------------------------------------------------------------------ */

static void sym_to_full(const lattice *L, const double *s, double T[3][3]) {
  memset(T, 0, 9 * sizeof(double));
  for (int c = 0; c < L->nc; ++c) {
    T[L->comp[c][0]][L->comp[c][1]] = s[c];
    T[L->comp[c][1]][L->comp[c][0]] = s[c];
  }
}

/* Polymer stress from the conformation tensor (Sec. 2.1):
 * tau_p = (mu_p / lambda) (A - I), with mu_p = rho0 nu_p and rho0 = 1. */
void or_polymer_stress(int d, double eta_p, double lambda, const double *A,
                       double *tau) {
  lattice L = lat_of(d);
  for (int c = 0; c < L.nc; ++c) {
    double delta = (L.comp[c][0] == L.comp[c][1]) ? 1.0 : 0.0;
    tau[c] = eta_p / lambda * (A[c] - delta);
  }
}

/* Fluctuation term f^B (Sec. 2.2, App. A): the pseudo-inverse matrix
 * applied to the right-hand side b built from -tau_p/tau_f. */
void or_fB(int d, double tau_f, const double *tau, double *fB) {
  lattice L = lat_of(d);
  double T[3][3];
  sym_to_full(&L, tau, T);
  if (d == 2) {
    double v[4] = {T[1][0], T[0][0], T[0][1], T[1][1]};
    for (int i = 0; i < 9; ++i) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += PINV2[i][k] * v[k];
      fB[i] = -1.0 / (72.0 * tau_f) * s;
    }
  } else {
    double b[13] = {-T[0][0] / tau_f, -T[1][1] / tau_f, -T[2][2] / tau_f,
                    -T[0][1] / tau_f, -T[0][2] / tau_f, -T[1][0] / tau_f,
                    -T[1][2] / tau_f, -T[2][0] / tau_f, -T[2][1] / tau_f,
                    0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
      double s = 0.0;
      for (int k = 0; k < 13; ++k) s += PINV3[i][k] * b[k];
      fB[i] = s;
    }
  }
}

/* Incompressible equilibrium (Sec. 2.2):
 * f_i^eq = lambda_i p + w_i [c_i.u/cs2 + uu:(c_i c_i - cs2 I)/(2 cs2^2)],
 * lambda_i = w_i/cs2 (i != 0), lambda_0 = (w_0 - 1)/cs2. */
void or_feq(int d, double p, const double *u, double *feq) {
  lattice L = lat_of(d);
  for (int i = 0; i < L.q; ++i) {
    double lam = (i == 0) ? (L.w[0] - 1.0) / CS2 : L.w[i] / CS2;
    double cu = cdot(&L, i, u);
    double uu_Q = 0.0; /* uu : (c c - cs2 I) */
    for (int a = 0; a < L.d; ++a)
      for (int b = 0; b < L.d; ++b)
        uu_Q += u[a] * u[b] * (L.c[i][a] * L.c[i][b] - (a == b ? CS2 : 0.0));
    feq[i] = lam * p + L.w[i] * (cu / CS2 + uu_Q / (2.0 * CS2 * CS2));
  }
}

/* Guo forcing term (Sec. 2.2):
 * F_i = w_i (1 - 1/(2 tau_f)) [c_i.F/cs2 + (Fu + uF):(c_i c_i - cs2 I)/(2 cs2^2)]. */
void or_guo(int d, double tau_f, const double *F, const double *u, double *Fi) {
  lattice L = lat_of(d);
  for (int i = 0; i < L.q; ++i) {
    double cF = cdot(&L, i, F);
    double S = 0.0;
    for (int a = 0; a < L.d; ++a)
      for (int b = 0; b < L.d; ++b)
        S += (F[a] * u[b] + u[a] * F[b]) *
             (L.c[i][a] * L.c[i][b] - (a == b ? CS2 : 0.0));
    Fi[i] = L.w[i] * (1.0 - 1.0 / (2.0 * tau_f)) *
            (cF / CS2 + S / (2.0 * CS2 * CS2));
  }
}

/* Velocity moment (Sec. 2.2): u = sum_{i != 0} c_i f_i + (dt/2) F. */
void or_velocity(int d, const double *f, const double *F, double *u) {
  lattice L = lat_of(d);
  for (int a = 0; a < L.d; ++a) {
    double s = 0.0;
    for (int i = 1; i < L.q; ++i) s += L.c[i][a] * f[i];
    u[a] = s + 0.5 * F[a];
  }
}

/* Pressure (Sec. 2.2, derived in App. B):
 * p = cs2/(1 - w_0) [sum_{i != 0} f_i + s_0(u) + tau_f F_0 + tau_f f_0^B],
 * s_0(u) = w_0 [3 e_0.u + 4.5 (e_0.u)^2 - 1.5 |u|^2] = -1.5 w_0 |u|^2. */
double or_pressure(int d, double tau_f, const double *f, const double *u,
                   double F0, double fB0) {
  lattice L = lat_of(d);
  double s = 0.0;
  for (int i = 1; i < L.q; ++i) s += f[i];
  double uu = 0.0;
  for (int a = 0; a < L.d; ++a) uu += u[a] * u[a];
  double s0 = L.w[0] * (-1.5 * uu);
  return CS2 / (1.0 - L.w[0]) * (s + s0 + tau_f * F0 + tau_f * fB0);
}

/* Equilibrium of the conformation populations (Sec. 2.3):
 * h^eq_abi = w_i A_ab [1 + c_i.u/cs2]. */
void or_heq(int d, double A, const double *u, double *heq) {
  lattice L = lat_of(d);
  for (int i = 0; i < L.q; ++i)
    heq[i] = L.w[i] * A * (1.0 + cdot(&L, i, u) / CS2);
}

/* Source distribution (Sec. 2.3):
 * chi_abi = w_i chi_ab [1 + (1 - 1/(2 tau_h)) c_i.u/cs2]. */
void or_chi_i(int d, double tau_h, double chi, const double *u, double *chii) {
  lattice L = lat_of(d);
  for (int i = 0; i < L.q; ++i)
    chii[i] = L.w[i] * chi *
              (1.0 + (1.0 - 1.0 / (2.0 * tau_h)) * cdot(&L, i, u) / CS2);
}

/* Source tensor of the conformation equation (Sec. 2.3):
 * chi = -R(E)/lambda + A . grad(u) + grad(u)^T . A,  E = A - I,
 * with (grad u)_ab = d_a u_b, the convention under which the constitutive
 * equation of Sec. 2.1 is the upper-convected derivative.  R(E) = E is the
 * Oldroyd-B model of the paper.  The paper names the Giesekus and
 * Phan-Thien-Tanner models as the next constitutive models for the method
 * (Introduction, Conclusion); in conformation form their relaxation terms
 * are (standard forms; the polymer stress stays tau_p = (eta_p/lambda) E):
 *   Giesekus, mobility alpha:        R(E) = E + alpha E.E
 *   linear PTT, parameter eps:        R(E) = (1 + eps tr E) E
 *   exponential PTT, parameter eps:   R(E) = exp(eps tr E) E
 * G is the full d x d gradient, G[a*d+b] = d_a u_b. */
enum { OR_MODEL_OLDROYD_B = 0, OR_MODEL_GIESEKUS = 1, OR_MODEL_LPTT = 2, OR_MODEL_EPTT = 3 };

void or_chi_tensor_model(int d, double lambda, int model, double param, const double *A,
                         const double *G, double *chi) {
  lattice L = lat_of(d);
  double At[3][3], Gt[3][3], E[3][3];
  sym_to_full(&L, A, At);
  memset(Gt, 0, sizeof Gt);
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) Gt[a][b] = G[a * d + b];
  double trE = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) E[a][b] = At[a][b] - (a == b && a < d ? 1.0 : 0.0);
  for (int a = 0; a < d; ++a) trE += E[a][a];
  double scale = 1.0;
  if (model == OR_MODEL_LPTT) scale = 1.0 + param * trE;
  if (model == OR_MODEL_EPTT) scale = exp(param * trE);
  for (int c = 0; c < L.nc; ++c) {
    int a = L.comp[c][0], b = L.comp[c][1];
    double relax = scale * E[a][b];
    if (model == OR_MODEL_GIESEKUS) {
      double ee = 0.0;
      for (int g = 0; g < d; ++g) ee += E[a][g] * E[g][b];
      relax += param * ee;
    }
    double s = -relax / lambda;
    for (int g = 0; g < d; ++g) s += At[a][g] * Gt[g][b] + Gt[g][a] * At[g][b];
    chi[c] = s;
  }
}

void or_chi_tensor(int d, double lambda, const double *A, const double *G, double *chi) {
  or_chi_tensor_model(d, lambda, OR_MODEL_OLDROYD_B, 0.0, A, G, chi);
}

/* Map the dimensionless groups of Sec. 3 to lattice units (dx = dt = 1):
 * nu = U0 L / Re, nu_s = beta nu, nu_p = (1 - beta) nu,
 * tau_f = nu_s / cs2 + 1/2 (Sec. 2.2), lambda = Wi L / U0 unless given,
 * eta_p = rho0 nu_p with rho0 = 1.
 * out = {nu_s, nu_p, tau_f, lambda, eta_p}. */
void or_lattice_params(double Re, double Wi, double beta, double U0, double L,
                       double lambda_override, double *out) {
  double nu = U0 * L / Re;
  double nu_s = beta * nu, nu_p = (1.0 - beta) * nu;
  out[0] = nu_s;
  out[1] = nu_p;
  out[2] = nu_s / CS2 + 0.5;
  out[3] = lambda_override > 0.0 ? lambda_override : Wi * L / U0;
  out[4] = nu_p;
}

/* ------------------------------------------------------------------ */
/* Whole-lattice simulation.                                             */
/* ------------------------------------------------------------------ */

enum { OR_FORCE_NONE = 0, OR_FORCE_CONST = 1, OR_FORCE_FOUR_ROLL = 2,
       OR_FORCE_COS_T = 3 };

typedef struct {
  lattice L;
  int n[3];
  long N;
  int wall[3];
  double tau_f, tau_h, lambda, eta_p;
  int force_kind;
  double famp[3], omega;
  long t;
  double *f, *h;        /* pre-collision populations at time t */
  double *fp, *hp;      /* post-collision scratch                */
  double *chi_prev;     /* chi(t-1) [N][nc]                      */
  double *u_prev;       /* u(t-1)   [N][d]                       */
  double *u, *A;        /* per-step scratch: u(t), A(t)          */
  int scheme;           /* OR_SCHEME_* below                     */
  int model;            /* OR_MODEL_*: constitutive model        */
  double mparam;        /* its parameter (alpha or eps)          */
  double *tp;           /* scratch of the stress-divergence scheme: tau_p(t) [N][nc] */
} osim;

void *or_create(int d, int nx, int ny, int nz) {
  if ((d != 2 && d != 3) || nx < 1 || ny < 1 || nz < 1) return NULL;
  if (d == 2) nz = 1;
  osim *s = (osim *)calloc(1, sizeof(osim));
  s->L = lat_of(d);
  s->n[0] = nx; s->n[1] = ny; s->n[2] = nz;
  s->N = (long)nx * ny * nz;
  s->tau_f = 1.0; s->tau_h = 0.501; s->lambda = 1.0; s->eta_p = 0.0;
  int q = s->L.q, nc = s->L.nc;
  s->f = (double *)calloc(s->N * q, sizeof(double));
  s->fp = (double *)calloc(s->N * q, sizeof(double));
  s->h = (double *)calloc(s->N * nc * q, sizeof(double));
  s->hp = (double *)calloc(s->N * nc * q, sizeof(double));
  s->chi_prev = (double *)calloc(s->N * nc, sizeof(double));
  s->u_prev = (double *)calloc(s->N * d, sizeof(double));
  s->u = (double *)calloc(s->N * d, sizeof(double));
  s->A = (double *)calloc(s->N * nc, sizeof(double));
  s->tp = (double *)calloc(s->N * nc, sizeof(double));
  return s;
}

void or_destroy(void *p) {
  osim *s = (osim *)p;
  if (!s) return;
  free(s->f); free(s->fp); free(s->h); free(s->hp);
  free(s->chi_prev); free(s->u_prev); free(s->u); free(s->A); free(s->tp);
  free(s);
}

void or_set_params(void *p, double tau_f, double tau_h, double lambda,
                   double eta_p) {
  osim *s = (osim *)p;
  s->tau_f = tau_f; s->tau_h = tau_h; s->lambda = lambda; s->eta_p = eta_p;
}

void or_set_walls(void *p, const int *wall) {
  osim *s = (osim *)p;
  for (int a = 0; a < 3; ++a) s->wall[a] = wall[a];
}

void or_set_force(void *p, int kind, const double *amp, double omega) {
  osim *s = (osim *)p;
  s->force_kind = kind;
  for (int a = 0; a < 3; ++a) s->famp[a] = amp[a];
  s->omega = omega;
}

/* The two schemes compared in Sec. 3 (Tables of the Poiseuille and
 * Taylor-Green performance tests):
 *   OR_SCHEME_FLUCTUATING: the paper's method, the polymer stress enters
 *     the f equation through the fluctuation term f^B (Sec. 2.2);
 *   OR_SCHEME_STRESS_DIVERGENCE: the "original" scheme the paper describes
 *     in prose (Introduction), the divergence of the polymer stress is a
 *     body force, F_tot = F + div tau_p, in the Guo forcing, the velocity
 *     and the pressure, with f^B = 0.  The conformation equation is the
 *     same in both.  The paper gives no stencil for the divergence: it is
 *     taken here with second-order central differences of tau_p(t) at the
 *     same time level, and one-sided second-order differences
 *     (-3 t_0 + 4 t_1 - t_2)/2 normal to a wall (no wall value of tau_p is
 *     known). */
enum { OR_SCHEME_FLUCTUATING = 0, OR_SCHEME_STRESS_DIVERGENCE = 1 };

void or_set_scheme(void *p, int scheme) { ((osim *)p)->scheme = scheme; }

void or_set_model(void *p, int model, double param) {
  osim *s = (osim *)p;
  s->model = model;
  s->mparam = param;
}

long or_time(void *p) { return ((osim *)p)->t; }
void or_set_time(void *p, long t) { ((osim *)p)->t = t; }

static void node_xyz(const osim *s, long n, int x[3]) {
  x[0] = (int)(n % s->n[0]);
  x[1] = (int)((n / s->n[0]) % s->n[1]);
  x[2] = (int)(n / ((long)s->n[0] * s->n[1]));
}

static long node_index(const osim *s, const int x[3]) {
  return ((long)x[2] * s->n[1] + x[1]) * s->n[0] + x[0];
}

/* Body force at a node and time level t.  Four-roll mill (Sec. 3.1):
 * g = (A_x sin(kx x) cos(ky y), A_y cos(kx x) sin(ky y)) at node
 * coordinates x = 2 pi i / N; the caller supplies the amplitudes in
 * lattice units.  Womersley (Sec. 3.3): g = A cos(omega t), evaluated at
 * the time level of the step. */
static void body_force(const osim *s, const int x[3], long t, double *F) {
  F[0] = F[1] = F[2] = 0.0;
  switch (s->force_kind) {
    case OR_FORCE_CONST:
      for (int a = 0; a < s->L.d; ++a) F[a] = s->famp[a];
      break;
    case OR_FORCE_FOUR_ROLL: {
      double X = 2.0 * OR_PI * x[0] / s->n[0];
      double Y = 2.0 * OR_PI * x[1] / s->n[1];
      F[0] = s->famp[0] * sin(X) * cos(Y);
      F[1] = s->famp[1] * cos(X) * sin(Y);
      break;
    }
    case OR_FORCE_COS_T:
      for (int a = 0; a < s->L.d; ++a) F[a] = s->famp[a] * cos(s->omega * t);
      break;
    default:
      break;
  }
}

/* Equilibrium-only initial state: f = f^eq(p0, u0), h = h^eq(A0, u0) with
 * A0 = I + lambda tau0 / eta_p (the inverse of the polymer-stress relation).
 * NULL arrays mean zero fields.  u is [N][d], tau [N][nc], p [N]. */
void or_init(void *p, const double *u, const double *tau, const double *pr) {
  osim *s = (osim *)p;
  const lattice *L = &s->L;
  int d = L->d, q = L->q, nc = L->nc;
  for (long n = 0; n < s->N; ++n) {
    double un[3] = {0, 0, 0}, A[6];
    if (u)
      for (int a = 0; a < d; ++a) un[a] = u[n * d + a];
    for (int c = 0; c < nc; ++c) {
      double delta = (L->comp[c][0] == L->comp[c][1]) ? 1.0 : 0.0;
      double tc = tau ? tau[n * nc + c] : 0.0;
      A[c] = delta + (s->eta_p > 0.0 ? s->lambda * tc / s->eta_p : 0.0);
    }
    or_feq(d, pr ? pr[n] : 0.0, un, &s->f[n * q]);
    for (int c = 0; c < nc; ++c) or_heq(d, A[c], un, &s->h[(n * nc + c) * q]);
    for (int c = 0; c < nc; ++c) s->chi_prev[n * nc + c] = 0.0;
    for (int a = 0; a < d; ++a) s->u_prev[n * d + a] = un[a];
  }
  s->t = 0;
}

/* Neighbour along axis a at offset +-1: periodic wrap, or -1 when the
 * neighbour lies beyond a wall. */
static long neighbour(const osim *s, const int x[3], int a, int off) {
  int y[3] = {x[0], x[1], x[2]};
  y[a] += off;
  if (y[a] < 0 || y[a] >= s->n[a]) {
    if (s->wall[a]) return -1;
    y[a] = (y[a] + s->n[a]) % s->n[a];
  }
  return node_index(s, y);
}

/* Velocity gradient G[a*d+b] = d_a u_b at node n.  The paper does not give
 * the stencil; second-order central differences of u at the same time
 * level over the face neighbours are used.  Next to a halfway bounce-back
 * wall (wall half a spacing outside the first node, u = 0 there) the
 * derivative normal to the wall is that of the parabola through the wall
 * value and the first two nodes: d u(0) = u_0 + u_1/3 (mirrored at the far
 * wall). */
static void velocity_gradient(const osim *s, long n, double *G) {
  int d = s->L.d, x[3];
  node_xyz(s, n, x);
  for (int a = 0; a < d; ++a) {
    long np = neighbour(s, x, a, +1), nm = neighbour(s, x, a, -1);
    for (int b = 0; b < d; ++b) {
      double g;
      if (np >= 0 && nm >= 0)
        g = 0.5 * (s->u[np * d + b] - s->u[nm * d + b]);
      else if (nm < 0 && np >= 0)
        g = s->u[n * d + b] + s->u[np * d + b] / 3.0;
      else if (np < 0 && nm >= 0)
        g = -(s->u[n * d + b] + s->u[nm * d + b] / 3.0);
      else
        g = 0.0; /* single node between two walls */
      G[a * d + b] = g;
    }
  }
}

/* tau_p(t) of every node from the current (pre-collision) h. */
static void stress_field(osim *s) {
  const lattice *L = &s->L;
  int q = L->q, nc = L->nc;
  for (long n = 0; n < s->N; ++n) {
    double A[6];
    for (int c = 0; c < nc; ++c) {
      double sum = 0.0;
      for (int i = 0; i < q; ++i) sum += s->h[(n * nc + c) * q + i];
      A[c] = sum;
    }
    or_polymer_stress(L->d, s->eta_p, s->lambda, A, &s->tp[n * nc]);
  }
}

/* Derivative along axis a of component c of the field s->tp at node n:
 * central, or one-sided second order next to a wall. */
static double stress_derivative(const osim *s, long n, int a, int c) {
  int x[3], nc = s->L.nc;
  node_xyz(s, n, x);
  long np = neighbour(s, x, a, +1), nm = neighbour(s, x, a, -1);
  if (np >= 0 && nm >= 0) return 0.5 * (s->tp[np * nc + c] - s->tp[nm * nc + c]);
  if (nm < 0 && np >= 0) {
    int y[3] = {x[0], x[1], x[2]};
    y[a] += 1;
    long np2 = neighbour(s, y, a, +1);
    if (np2 < 0) return s->tp[np * nc + c] - s->tp[n * nc + c];
    return 0.5 * (-3.0 * s->tp[n * nc + c] + 4.0 * s->tp[np * nc + c] - s->tp[np2 * nc + c]);
  }
  if (np < 0 && nm >= 0) {
    int y[3] = {x[0], x[1], x[2]};
    y[a] -= 1;
    long nm2 = neighbour(s, y, a, -1);
    if (nm2 < 0) return s->tp[n * nc + c] - s->tp[nm * nc + c];
    return 0.5 * (3.0 * s->tp[n * nc + c] - 4.0 * s->tp[nm * nc + c] + s->tp[nm2 * nc + c]);
  }
  return 0.0;
}

/* (div tau_p)_b = sum_a d_a tau_ab at node n, added to F. */
static void add_stress_divergence(const osim *s, long n, double *F) {
  const lattice *L = &s->L;
  int d = L->d;
  for (int c = 0; c < L->nc; ++c) {
    int a = L->comp[c][0], b = L->comp[c][1];
    F[b] += stress_derivative(s, n, a, c);
    if (a != b) F[a] += stress_derivative(s, n, b, c);
  }
  for (int b = d; b < 3; ++b) F[b] = 0.0;
}

/* One time step of the method:
 *  (1) per node: A = sum_i h_i (Sec. 2.3), tau_p (Sec. 2.1), f^B (App. A),
 *      F(x, t), u (Sec. 2.2), F_i, p (App. B), f^eq, then the collision of
 *      the fluctuating evolution equation (Sec. 2.2)
 *      f* = f - (f - f^eq)/tau_f + f^B + dt F_i;
 *  (2) per node, after every node has u(t): grad u, chi, chi_i, and the
 *      collision of the conformation populations (Sec. 2.3)
 *      h* = h - (h - h^eq)/tau_h + dt chi_i + dt^2/2 d(chi_i)/dt,
 *      where d(chi_i)/dt is read as the first-order backward difference
 *      chi_i(t) - chi_i(t-1) rebuilt from chi(t-1), u(t-1) (zero at the
 *      first step; the paper does not state the discretisation);
 *  (3) streaming of f* and h* to x + c_i: periodic wrap, or halfway
 *      bounce-back at walls (the populations leaving through a wall return
 *      to their node in the opposite direction), for f and for h. */
static void one_step(osim *s) {
  const lattice *L = &s->L;
  int d = L->d, q = L->q, nc = L->nc;
  double tf = s->tau_f, th = s->tau_h;
  const int divergence = s->scheme == OR_SCHEME_STRESS_DIVERGENCE;
  if (divergence) stress_field(s);

  for (long n = 0; n < s->N; ++n) {
    int x[3];
    node_xyz(s, n, x);
    double *f = &s->f[n * q];
    double A[6], tau[6], fB[19], F[3], u[3], Fi[19], feq[19];
    for (int c = 0; c < nc; ++c) {
      double sum = 0.0;
      for (int i = 0; i < q; ++i) sum += s->h[(n * nc + c) * q + i];
      A[c] = sum;
    }
    or_polymer_stress(d, s->eta_p, s->lambda, A, tau);
    body_force(s, x, s->t, F);
    if (divergence) {
      for (int i = 0; i < q; ++i) fB[i] = 0.0;
      add_stress_divergence(s, n, F);
    } else {
      or_fB(d, tf, tau, fB);
    }
    or_velocity(d, f, F, u);
    or_guo(d, tf, F, u, Fi);
    double pr = or_pressure(d, tf, f, u, Fi[0], fB[0]);
    or_feq(d, pr, u, feq);
    for (int i = 0; i < q; ++i)
      s->fp[n * q + i] = f[i] - (f[i] - feq[i]) / tf + fB[i] + Fi[i];
    for (int a = 0; a < d; ++a) s->u[n * d + a] = u[a];
    for (int c = 0; c < nc; ++c) s->A[n * nc + c] = A[c];
  }

  for (long n = 0; n < s->N; ++n) {
    double G[9], chi[6], un[3] = {0, 0, 0}, up[3] = {0, 0, 0};
    velocity_gradient(s, n, G);
    or_chi_tensor_model(d, s->lambda, s->model, s->mparam, &s->A[n * nc], G, chi);
    for (int a = 0; a < d; ++a) {
      un[a] = s->u[n * d + a];
      up[a] = s->u_prev[n * d + a];
    }
    for (int c = 0; c < nc; ++c) {
      double chii[19], chip[19], heq[19];
      or_chi_i(d, th, chi[c], un, chii);
      or_chi_i(d, th, s->chi_prev[n * nc + c], up, chip);
      or_heq(d, s->A[n * nc + c], un, heq);
      for (int i = 0; i < q; ++i) {
        double hv = s->h[(n * nc + c) * q + i];
        double dchi = (s->t == 0) ? 0.0 : chii[i] - chip[i];
        s->hp[(n * nc + c) * q + i] =
            hv - (hv - heq[i]) / th + chii[i] + 0.5 * dchi;
      }
    }
    for (int c = 0; c < nc; ++c) s->chi_prev[n * nc + c] = chi[c];
    for (int a = 0; a < d; ++a) s->u_prev[n * d + a] = un[a];
  }

  for (long n = 0; n < s->N; ++n) {
    int x[3];
    node_xyz(s, n, x);
    for (int i = 0; i < q; ++i) {
      int y[3] = {x[0] + L->c[i][0], x[1] + L->c[i][1], x[2] + L->c[i][2]};
      int bounce = 0;
      for (int a = 0; a < 3; ++a) {
        if (y[a] < 0 || y[a] >= s->n[a]) {
          if (s->wall[a]) bounce = 1;
          else y[a] = (y[a] + s->n[a]) % s->n[a];
        }
      }
      long m;
      int j;
      if (bounce) { m = n; j = L->opp[i]; }
      else { m = node_index(s, y); j = i; }
      s->f[m * q + j] = s->fp[n * q + i];
      for (int c = 0; c < nc; ++c)
        s->h[(m * nc + c) * q + j] = s->hp[(n * nc + c) * q + i];
    }
  }
  s->t += 1;
}

void or_step(void *p, long nsteps) {
  osim *s = (osim *)p;
  for (long k = 0; k < nsteps; ++k) one_step(s);
}

/* Macroscopic fields of the pre-collision state at time t, with F(t):
 * u [N][d], p [N], A [N][nc], tau [N][nc].  Any pointer may be NULL. */
void or_moments(void *p, double *u, double *pr, double *A, double *tau) {
  osim *s = (osim *)p;
  const lattice *L = &s->L;
  int d = L->d, q = L->q, nc = L->nc;
  const int divergence = s->scheme == OR_SCHEME_STRESS_DIVERGENCE;
  if (divergence) stress_field(s);
  for (long n = 0; n < s->N; ++n) {
    int x[3];
    node_xyz(s, n, x);
    double An[6], tn[6], fB[19], F[3], un[3], Fi[19];
    for (int c = 0; c < nc; ++c) {
      double sum = 0.0;
      for (int i = 0; i < q; ++i) sum += s->h[(n * nc + c) * q + i];
      An[c] = sum;
    }
    or_polymer_stress(d, s->eta_p, s->lambda, An, tn);
    body_force(s, x, s->t, F);
    if (divergence) {
      for (int i = 0; i < q; ++i) fB[i] = 0.0;
      add_stress_divergence(s, n, F);
    } else {
      or_fB(d, s->tau_f, tn, fB);
    }
    or_velocity(d, &s->f[n * q], F, un);
    or_guo(d, s->tau_f, F, un, Fi);
    if (u) for (int a = 0; a < d; ++a) u[n * d + a] = un[a];
    if (pr) pr[n] = or_pressure(d, s->tau_f, &s->f[n * q], un, Fi[0], fB[0]);
    if (A) for (int c = 0; c < nc; ++c) A[n * nc + c] = An[c];
    if (tau) for (int c = 0; c < nc; ++c) tau[n * nc + c] = tn[c];
  }
}

/* Raw state access for tests: f [N][q], h [N][nc][q], chi_prev [N][nc],
 * u_prev [N][d]. */
void or_get_state(void *p, double *f, double *h, double *chi_prev,
                  double *u_prev) {
  osim *s = (osim *)p;
  int d = s->L.d, q = s->L.q, nc = s->L.nc;
  if (f) memcpy(f, s->f, s->N * q * sizeof(double));
  if (h) memcpy(h, s->h, s->N * nc * q * sizeof(double));
  if (chi_prev) memcpy(chi_prev, s->chi_prev, s->N * nc * sizeof(double));
  if (u_prev) memcpy(u_prev, s->u_prev, s->N * d * sizeof(double));
}

void or_set_state(void *p, const double *f, const double *h,
                  const double *chi_prev, const double *u_prev) {
  osim *s = (osim *)p;
  int d = s->L.d, q = s->L.q, nc = s->L.nc;
  if (f) memcpy(s->f, f, s->N * q * sizeof(double));
  if (h) memcpy(s->h, h, s->N * nc * q * sizeof(double));
  if (chi_prev) memcpy(s->chi_prev, chi_prev, s->N * nc * sizeof(double));
  if (u_prev) memcpy(s->u_prev, u_prev, s->N * d * sizeof(double));
}

/* The body force the oracle applies at every node at time t, [N][d]. */
void or_force_field(void *p, long t, double *F) {
  osim *s = (osim *)p;
  int d = s->L.d;
  for (long n = 0; n < s->N; ++n) {
    int x[3];
    double Fn[3];
    node_xyz(s, n, x);
    body_force(s, x, t, Fn);
    for (int a = 0; a < d; ++a) F[n * d + a] = Fn[a];
  }
}

/* div tau_p of the current state at every node, [N][d], with the stencil
 * of the stress-divergence scheme. */
void or_stress_divergence(void *p, double *div) {
  osim *s = (osim *)p;
  int d = s->L.d;
  stress_field(s);
  for (long n = 0; n < s->N; ++n) {
    double F[3] = {0, 0, 0};
    add_stress_divergence(s, n, F);
    for (int a = 0; a < d; ++a) div[n * d + a] = F[a];
  }
}

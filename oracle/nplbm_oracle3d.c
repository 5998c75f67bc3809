/*
 * nplbm_oracle3d.c -- FP64 CPU oracle of the N-phase phase-field lattice
 * Boltzmann model (Yuan, Liang, Chai & Shi, arXiv:1904.12553) on the
 * three-dimensional D3Q15 lattice the paper lists in Sec. 3.1.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU baseline
 * of the benchmark call it; the GPU library never does.
 *
 * The model is the same as in nplbm_oracle.c (which is 2-D), written again
 * for three velocity components and the D3Q15 velocity set:
 *   - setup and closure (eq:N1, eq:N12, eq:N14-N18, eq:N30, eq:N36) are
 *     lattice-independent and are taken from the 2-D oracle's exported
 *     functions (orc_create on a 4 x 4 lattice, orc_lambda, orc_closure,
 *     orc_hbulk), which its own tests pin;
 *   - stencils: eq:N31a / eq:N31b written as sums over the D3Q15 velocities;
 *   - NS LBE: eq:24 with g^eq of eq:25 and G_k of eq:N20_1 (3 x 3 tensor
 *     contraction as printed), u from eq:N22_1, p from eq:N23 with the
 *     D3Q15 rest weight, tau_g from eq:N21_1 with mu = sum_k mu~_k c_k;
 *   - CH LBEs: eq:N24 with eq:N25, the source of eq:N26 and the backward
 *     Euler derivative of eq:N27; phi_i by eq:N28;
 *   - streaming: periodic in x and y; periodic or halfway bounce-back in z,
 *     with mirror ghosts zeta(z = -1) = zeta(0), zeta(nz) = zeta(nz - 1)
 *     for the stencils next to a wall (the 2-D oracle's wall rule, moved to
 *     the z direction).
 * The readings of the 2-D oracle carry over unchanged (h_i as eq:N17 prints
 * it, phi_i for the index of eq:N18's last line, equilibrium initial state
 * with p = 0, (phi u) at t = -1 equal to (phi u) at t = 0, u of the same
 * step in h^eq, G_k and R_k, no clipping).
 *
 * Layout: a scalar field is f[(z * ny + y) * nx + x].
 * Build: compiled into liboracle.so next to nplbm_oracle.c (build_oracle.py).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q3 15
#define NMAX3 8

/* D3Q15, Sec. 3.1: velocities in the paper's order, weights, c_s^2 */
static const int EX[Q3] = {0, 1, 0, 0, -1, 0, 0, 1, 1, 1, -1, -1, -1, -1, 1};
static const int EY[Q3] = {0, 0, 1, 0, 0, -1, 0, 1, 1, -1, 1, -1, -1, 1, -1};
static const int EZ[Q3] = {0, 0, 0, 1, 0, 0, -1, 1, -1, 1, 1, -1, 1, -1, -1};
static const double W3[Q3] = {2.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                              1.0 / 9.0,  1.0 / 9.0,  1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0,
                              1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0};
static const double CS2_3 = 1.0 / 3.0;

enum { O3_OK = 0, O3_EINVAL = -1, O3_ENOTSPD = -2, O3_ENOMEM = -3 };

/* the 2-D oracle's exported setup and closure (nplbm_oracle.c) */
typedef struct orc_sim orc_sim;
int orc_create(int N, int nx, int ny, int wall_y, int grad_scheme, int force_form,
               const double *sigma, const double *rho, const double *mu, const double *mob,
               const double *tau_phi, double W, double gx, double gy, double rho0,
               orc_sim **out);
void orc_free(orc_sim *s);
int orc_lambda(const orc_sim *s, double *lam, double *beta2, double *K, double *eta);
int orc_closure(const orc_sim *s, const double *phi, double *c, double *rho);
int orc_hbulk(const orc_sim *s, const double *phi, double *h);

typedef struct orc3_sim {
  int N, nx, ny, nz, wall_z;
  orc_sim *setup; /* closure constants, lambda, beta */
  double rho_t[NMAX3], mu_t[NMAX3], mob[NMAX3], tau[NMAX3], eta_i[NMAX3];
  double gam[NMAX3], Gam;
  double lam[NMAX3][NMAX3], Kc, G[3], rho0;
  long t;
  double *h;    /* [(N-1)][15][n] */
  double *g;    /* [15][n]        */
  double *pphi; /* [(N-1)][n]     */
  double *pu;   /* [3][n]         */
  double *phi, *c, *rho, *Cp, *hb, *gphi, *gC, *grho, *F, *J, *u, *p, *taug;
  double *hs, *gs;
} orc3_sim;

static int wrap3(int a, int n) {
  while (a < 0) a += n;
  while (a >= n) a -= n;
  return a;
}

static size_t nnodes(const orc3_sim *s) { return (size_t)s->nx * s->ny * s->nz; }

/* value of a scalar field at (x, y, z): periodic in x and y; in z periodic
   or a mirror ghost next to a wall */
static double fld3(const orc3_sim *s, const double *f, int x, int y, int z) {
  x = wrap3(x, s->nx);
  y = wrap3(y, s->ny);
  if (s->wall_z) {
    if (z < 0) z = -1 - z;
    if (z >= s->nz) z = 2 * s->nz - 1 - z;
  } else {
    z = wrap3(z, s->nz);
  }
  return f[((size_t)z * s->ny + y) * s->nx + x];
}

/* eq:N31a on D3Q15 */
static void grad3(const orc3_sim *s, const double *f, int x, int y, int z, double *g) {
  double a[3] = {0.0, 0.0, 0.0};
  for (int k = 1; k < Q3; ++k) {
    double d = fld3(s, f, x + EX[k], y + EY[k], z + EZ[k]) -
               fld3(s, f, x - EX[k], y - EY[k], z - EZ[k]);
    a[0] += W3[k] * EX[k] * d;
    a[1] += W3[k] * EY[k] * d;
    a[2] += W3[k] * EZ[k] * d;
  }
  for (int d = 0; d < 3; ++d) g[d] = a[d] / (2.0 * CS2_3);
}

/* eq:N31b on D3Q15 */
static double lap3(const orc3_sim *s, const double *f, int x, int y, int z) {
  double a = 0.0, f0 = fld3(s, f, x, y, z);
  for (int k = 1; k < Q3; ++k)
    a += W3[k] * (fld3(s, f, x + EX[k], y + EY[k], z + EZ[k]) - 2.0 * f0 +
                  fld3(s, f, x - EX[k], y - EY[k], z - EZ[k]));
  return a / CS2_3;
}

/* eq:25 */
static double s3(int k, const double *u) {
  double cu = EX[k] * u[0] + EY[k] * u[1] + EZ[k] * u[2];
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return W3[k] * (cu / CS2_3 + cu * cu / (2.0 * CS2_3 * CS2_3) - uu / (2.0 * CS2_3));
}

static double geq3(const orc3_sim *s, int k, double rho, double p, const double *u) {
  if (k == 0) return s->rho0 + p / CS2_3 * (W3[0] - 1.0) + rho * s3(0, u);
  return p / CS2_3 * W3[k] + rho * s3(k, u);
}

/* eq:N20_1: (c c - cs^2 I) : T / (2 cs^4), T = uF + Fu + cs^2 (u grad rho +
   grad rho u) + J u / (tau_g - 1/2) */
static double G3(int k, const double *u, const double *F, const double *r, const double *J,
                 double taug) {
  double c[3] = {(double)EX[k], (double)EY[k], (double)EZ[k]};
  double contr = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double T = u[a] * F[b] + F[a] * u[b] + CS2_3 * u[a] * r[b] + CS2_3 * r[a] * u[b] +
                 J[a] * u[b] / (taug - 0.5);
      contr += (c[a] * c[b] - CS2_3 * (a == b ? 1.0 : 0.0)) * T;
    }
  double udr = u[0] * r[0] + u[1] * r[1] + u[2] * r[2];
  double cF = c[0] * F[0] + c[1] * F[1] + c[2] * F[2];
  return W3[k] * (udr + cF / CS2_3 + contr / (2.0 * CS2_3 * CS2_3));
}

/* eq:N25 (0-based i) */
static double heq3(const orc3_sim *s, int i, int k, double phi, double Ci, const double *u) {
  double et = s->eta_i[i];
  if (k == 0) return phi + (W3[0] - 1.0) * et * Ci;
  return W3[k] * et * Ci +
         W3[k] * phi * (EX[k] * u[0] + EY[k] * u[1] + EZ[k] * u[2]) / CS2_3;
}

void orc3_free(orc3_sim *s) {
  if (!s) return;
  if (s->setup) orc_free(s->setup);
  free(s->h); free(s->g); free(s->pphi); free(s->pu);
  free(s->phi); free(s->c); free(s->rho); free(s->Cp); free(s->hb); free(s->gphi);
  free(s->gC); free(s->grho); free(s->F); free(s->J); free(s->u); free(s->p);
  free(s->taug); free(s->hs); free(s->gs);
  free(s);
}

int orc3_create(int N, int nx, int ny, int nz, int wall_z, const double *sigma,
                const double *rho, const double *mu, const double *mob,
                const double *tau_phi, double W, double gx, double gy, double gz,
                double rho0, orc3_sim **out) {
  *out = NULL;
  if (N < 2 || N > NMAX3 || nx < 4 || ny < 4 || nz < 4) return O3_EINVAL;
  orc3_sim *s = (orc3_sim *)calloc(1, sizeof(orc3_sim));
  if (!s) return O3_ENOMEM;
  s->N = N; s->nx = nx; s->ny = ny; s->nz = nz; s->wall_z = wall_z ? 1 : 0;
  int rc = orc_create(N, 4, 4, 0, 0, 0, sigma, rho, mu, mob, tau_phi, W, 0.0, 0.0, rho0,
                      &s->setup);
  if (rc) { free(s); return rc; }
  double lam[NMAX3 * NMAX3], b2, eta;
  orc_lambda(s->setup, lam, &b2, &s->Kc, &eta);
  int n1 = N - 1;
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) s->lam[i][j] = lam[i * n1 + j];
  s->Gam = 0.0;
  for (int k = 0; k < N; ++k) {
    s->rho_t[k] = rho[k];
    s->mu_t[k] = mu[k];
    s->gam[k] = 1.0 / rho[k]; /* eq:N1 */
    s->Gam += s->gam[k];
  }
  for (int i = 0; i < n1; ++i) {
    s->mob[i] = mob[i];
    s->tau[i] = tau_phi[i];
    s->eta_i[i] = mob[i] / (CS2_3 * (tau_phi[i] - 0.5)); /* eq:N30 */
  }
  s->G[0] = gx; s->G[1] = gy; s->G[2] = gz; s->rho0 = rho0;
  size_t n = nnodes(s);
  s->h = calloc((size_t)n1 * Q3 * n, sizeof(double));
  s->g = calloc((size_t)Q3 * n, sizeof(double));
  s->pphi = calloc((size_t)n1 * n, sizeof(double));
  s->pu = calloc(3 * n, sizeof(double));
  s->phi = calloc((size_t)n1 * n, sizeof(double));
  s->c = calloc((size_t)N * n, sizeof(double));
  s->rho = calloc(n, sizeof(double));
  s->Cp = calloc((size_t)n1 * n, sizeof(double));
  s->hb = calloc((size_t)n1 * n, sizeof(double));
  s->gphi = calloc((size_t)3 * n1 * n, sizeof(double));
  s->gC = calloc((size_t)3 * n1 * n, sizeof(double));
  s->grho = calloc(3 * n, sizeof(double));
  s->F = calloc(3 * n, sizeof(double));
  s->J = calloc(3 * n, sizeof(double));
  s->u = calloc(3 * n, sizeof(double));
  s->p = calloc(n, sizeof(double));
  s->taug = calloc(n, sizeof(double));
  s->hs = calloc((size_t)n1 * Q3 * n, sizeof(double));
  s->gs = calloc((size_t)Q3 * n, sizeof(double));
  if (!s->h || !s->g || !s->pphi || !s->pu || !s->phi || !s->c || !s->rho || !s->Cp ||
      !s->hb || !s->gphi || !s->gC || !s->grho || !s->F || !s->J || !s->u || !s->p ||
      !s->taug || !s->hs || !s->gs) {
    orc3_free(s);
    return O3_ENOMEM;
  }
  *out = s;
  return O3_OK;
}

/* closure (eq:N18) of every node from s->phi: c, rho, tau_g; then the
   bulk derivative h_i (eq:N17) */
static void closure_all(orc3_sim *s) {
  int N = s->N, n1 = N - 1;
  size_t n = nnodes(s);
  #pragma omp parallel for schedule(static) if (n >= 8192)
  for (size_t x = 0; x < n; ++x) {
    double ph[NMAX3], cc[NMAX3], hh[NMAX3], r;
    for (int i = 0; i < n1; ++i) ph[i] = s->phi[(size_t)i * n + x];
    orc_closure(s->setup, ph, cc, &r);
    orc_hbulk(s->setup, ph, hh);
    double mu = 0.0;
    for (int k = 0; k < N; ++k) {
      s->c[(size_t)k * n + x] = cc[k];
      mu += s->mu_t[k] * cc[k];
    }
    for (int i = 0; i < n1; ++i) s->hb[(size_t)i * n + x] = hh[i];
    s->rho[x] = r;
    s->taug[x] = 0.5 + mu / (r * CS2_3); /* eq:N21_1 with nu = mu / rho */
  }
}

/* C_i = -sum_j lambda_ij lap phi_j + (beta^2 / eta^2) h_i (eq:N18) */
static void chem_all(orc3_sim *s) {
  int n1 = s->N - 1, nx = s->nx, ny = s->ny, nz = s->nz;
  size_t n = nnodes(s);
  #pragma omp parallel for schedule(static) if (n >= 8192)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t id = ((size_t)z * ny + y) * nx + x;
        double lp[NMAX3];
        for (int j = 0; j < n1; ++j) lp[j] = lap3(s, s->phi + (size_t)j * n, x, y, z);
        for (int i = 0; i < n1; ++i) {
          double a = 0.0;
          for (int j = 0; j < n1; ++j) a -= s->lam[i][j] * lp[j];
          s->Cp[(size_t)i * n + id] = a + s->Kc * s->hb[(size_t)i * n + id];
        }
      }
}

/* every macroscopic field of the current state: phi (eq:N28), closure,
   C, gradients (eq:N31a), F = sum_i C_i grad phi_i + rho g, J~ (eq:N18),
   u (eq:N22_1), p (eq:N23) */
static void macroscopic3(orc3_sim *s) {
  int N = s->N, n1 = N - 1, nx = s->nx, ny = s->ny, nz = s->nz;
  size_t n = nnodes(s);
  for (int i = 0; i < n1; ++i)
    #pragma omp parallel for schedule(static) if (n >= 8192)
    for (size_t x = 0; x < n; ++x) {
      double a = 0.0;
      for (int k = 0; k < Q3; ++k) a += s->h[((size_t)i * Q3 + k) * n + x];
      s->phi[(size_t)i * n + x] = a;
    }
  closure_all(s);
  chem_all(s);
  #pragma omp parallel for schedule(static) if (n >= 8192)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t id = ((size_t)z * ny + y) * nx + x;
        double gv[3];
        for (int i = 0; i < n1; ++i) {
          grad3(s, s->phi + (size_t)i * n, x, y, z, gv);
          for (int d = 0; d < 3; ++d) s->gphi[(3 * (size_t)i + d) * n + id] = gv[d];
          grad3(s, s->Cp + (size_t)i * n, x, y, z, gv);
          for (int d = 0; d < 3; ++d) s->gC[(3 * (size_t)i + d) * n + id] = gv[d];
        }
        grad3(s, s->rho, x, y, z, gv);
        for (int d = 0; d < 3; ++d) s->grho[(size_t)d * n + id] = gv[d];
      }
  #pragma omp parallel for schedule(static) if (n >= 8192)
  for (size_t x = 0; x < n; ++x) {
    double F[3] = {0.0, 0.0, 0.0}, J[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < n1; ++i) {
      double Ci = s->Cp[(size_t)i * n + x];
      double coef = (1.0 - (double)N / s->Gam * s->gam[i]) *
                    (s->rho_t[i] + s->rho_t[N - 1]) / 2.0 * s->mob[i];
      for (int d = 0; d < 3; ++d) {
        F[d] += Ci * s->gphi[(3 * (size_t)i + d) * n + x];
        J[d] -= coef * s->gC[(3 * (size_t)i + d) * n + x];
      }
    }
    double r = s->rho[x];
    double mom[3] = {0.0, 0.0, 0.0}, sum = 0.0;
    for (int k = 0; k < Q3; ++k) {
      double gk = s->g[(size_t)k * n + x];
      mom[0] += EX[k] * gk;
      mom[1] += EY[k] * gk;
      mom[2] += EZ[k] * gk;
      if (k > 0) sum += gk;
    }
    double u[3], udr = 0.0;
    for (int d = 0; d < 3; ++d) {
      F[d] += r * s->G[d];
      s->F[(size_t)d * n + x] = F[d];
      s->J[(size_t)d * n + x] = J[d];
      u[d] = (mom[d] + 0.5 * F[d]) / r;
      s->u[(size_t)d * n + x] = u[d];
      udr += u[d] * s->grho[(size_t)d * n + x];
    }
    s->p[x] = CS2_3 / (1.0 - W3[0]) * (sum + 0.5 * udr + r * s3(0, u));
  }
}

/* push streaming, periodic in x and y, periodic or halfway bounce-back in z */
static void stream3(orc3_sim *s, const double *src, double *dst, int nfields) {
  int OPP3[Q3]; /* opposite velocity: c_opp = -c_k */
  for (int k = 0; k < Q3; ++k)
    for (int l = 0; l < Q3; ++l)
      if (EX[l] == -EX[k] && EY[l] == -EY[k] && EZ[l] == -EZ[k]) OPP3[k] = l;
  int nx = s->nx, ny = s->ny, nz = s->nz;
  size_t n = nnodes(s);
  for (int f = 0; f < nfields; ++f)
    for (int k = 0; k < Q3; ++k)
      #pragma omp parallel for schedule(static) if (n >= 8192)
      for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
          for (int x = 0; x < nx; ++x) {
            size_t id = ((size_t)z * ny + y) * nx + x;
            double v = src[((size_t)f * Q3 + k) * n + id];
            int xd = wrap3(x + EX[k], nx), yd = wrap3(y + EY[k], ny), zd = z + EZ[k];
            if (zd < 0 || zd >= nz) {
              if (s->wall_z) {
                dst[((size_t)f * Q3 + OPP3[k]) * n + id] = v;
                continue;
              }
              zd = wrap3(zd, nz);
            }
            dst[((size_t)f * Q3 + k) * n + ((size_t)zd * ny + yd) * nx + xd] = v;
          }
}

/* Initial state from c (N x n) and u (3 x n or NULL): phi_i from eq:N12
   inverted with rho_k = rho~_k c_k, p = 0, g = g^eq, h = h^eq with C_i of
   the initial phi, previous (phi, u) = current */
int orc3_init(orc3_sim *s, const double *c, const double *u) {
  int N = s->N, n1 = N - 1;
  size_t n = nnodes(s);
  for (int i = 0; i < n1; ++i)
    for (size_t x = 0; x < n; ++x) {
      double a = 0.5 * (s->rho_t[i] + s->rho_t[N - 1]);
      double b = 0.5 * (s->rho_t[i] - s->rho_t[N - 1]);
      s->phi[(size_t)i * n + x] =
          (s->rho_t[i] * c[(size_t)i * n + x] - s->rho_t[N - 1] * c[(size_t)(N - 1) * n + x] -
           b) / a;
    }
  closure_all(s);
  chem_all(s);
  for (size_t x = 0; x < n; ++x) {
    double uu[3];
    for (int d = 0; d < 3; ++d) uu[d] = u ? u[(size_t)d * n + x] : 0.0;
    for (int i = 0; i < n1; ++i) {
      double ph = s->phi[(size_t)i * n + x], Ci = s->Cp[(size_t)i * n + x];
      for (int k = 0; k < Q3; ++k) s->h[((size_t)i * Q3 + k) * n + x] = heq3(s, i, k, ph, Ci, uu);
      s->pphi[(size_t)i * n + x] = ph;
    }
    for (int k = 0; k < Q3; ++k) s->g[(size_t)k * n + x] = geq3(s, k, s->rho[x], 0.0, uu);
    for (int d = 0; d < 3; ++d) s->pu[(size_t)d * n + x] = uu[d];
  }
  s->t = 0;
  return O3_OK;
}

/* time steps: macroscopic fields, NS collision (eq:24), CH collisions
   (eq:N24), streaming */
int orc3_step(orc3_sim *s, long nsteps) {
  int n1 = s->N - 1;
  size_t n = nnodes(s);
  for (long it = 0; it < nsteps; ++it) {
    macroscopic3(s);
    #pragma omp parallel for schedule(static) if (n >= 8192)
    for (size_t x = 0; x < n; ++x) {
      double u[3], F[3], r3[3], J[3], pu[3];
      for (int d = 0; d < 3; ++d) {
        u[d] = s->u[(size_t)d * n + x];
        F[d] = s->F[(size_t)d * n + x];
        r3[d] = s->grho[(size_t)d * n + x];
        J[d] = s->J[(size_t)d * n + x];
        pu[d] = s->pu[(size_t)d * n + x];
      }
      double r = s->rho[x], p = s->p[x], tg = s->taug[x];
      for (int k = 0; k < Q3; ++k) {
        double gk = s->g[(size_t)k * n + x];
        s->gs[(size_t)k * n + x] =
            gk - (gk - geq3(s, k, r, p, u)) / tg + (1.0 - 1.0 / (2.0 * tg)) * G3(k, u, F, r3, J, tg);
      }
      for (int i = 0; i < n1; ++i) {
        double ph = s->phi[(size_t)i * n + x], Ci = s->Cp[(size_t)i * n + x];
        double pp = s->pphi[(size_t)i * n + x];
        double dt[3]; /* eq:N27 */
        for (int d = 0; d < 3; ++d) dt[d] = ph * u[d] - pp * pu[d];
        double ti = s->tau[i];
        for (int k = 0; k < Q3; ++k) {
          double R = (1.0 - 1.0 / (2.0 * ti)) * W3[k] *
                     (EX[k] * dt[0] + EY[k] * dt[1] + EZ[k] * dt[2]) / CS2_3; /* eq:N26 */
          double hk = s->h[((size_t)i * Q3 + k) * n + x];
          s->hs[((size_t)i * Q3 + k) * n + x] = hk - (hk - heq3(s, i, k, ph, Ci, u)) / ti + R;
        }
      }
    }
    memcpy(s->pphi, s->phi, (size_t)n1 * n * sizeof(double));
    memcpy(s->pu, s->u, 3 * n * sizeof(double));
    stream3(s, s->hs, s->h, n1);
    stream3(s, s->gs, s->g, 1);
    s->t += 1;
  }
  return O3_OK;
}

/* c (N x n), u (3 x n), p (n) of the current state; any pointer may be NULL */
int orc3_macro(orc3_sim *s, double *c, double *u, double *p) {
  size_t n = nnodes(s);
  macroscopic3(s);
  if (c) memcpy(c, s->c, (size_t)s->N * n * sizeof(double));
  if (u) memcpy(u, s->u, 3 * n * sizeof(double));
  if (p) memcpy(p, s->p, n * sizeof(double));
  return O3_OK;
}

/* phi, rho, C, F (3 x n), J (3 x n), grad rho (3 x n) of the current state */
int orc3_fields(orc3_sim *s, double *phi, double *rho, double *C, double *F, double *J,
                double *grho) {
  int n1 = s->N - 1;
  size_t n = nnodes(s);
  macroscopic3(s);
  if (phi) memcpy(phi, s->phi, (size_t)n1 * n * sizeof(double));
  if (rho) memcpy(rho, s->rho, n * sizeof(double));
  if (C) memcpy(C, s->Cp, (size_t)n1 * n * sizeof(double));
  if (F) memcpy(F, s->F, 3 * n * sizeof(double));
  if (J) memcpy(J, s->J, 3 * n * sizeof(double));
  if (grho) memcpy(grho, s->grho, 3 * n * sizeof(double));
  return O3_OK;
}

int orc3_mass(orc3_sim *s, double *out) {
  size_t n = nnodes(s);
  macroscopic3(s);
  for (int k = 0; k < s->N; ++k) {
    double a = 0.0;
    for (size_t x = 0; x < n; ++x) a += s->c[(size_t)k * n + x];
    out[k] = a;
  }
  return O3_OK;
}

long orc3_time(const orc3_sim *s) { return s->t; }

/* raw state: h [(N-1)][15][n], g [15][n], previous phi [(N-1)][n], u [3][n] */
int orc3_get_state(const orc3_sim *s, double *h, double *g, double *pphi, double *pu) {
  size_t n = nnodes(s);
  int n1 = s->N - 1;
  if (h) memcpy(h, s->h, (size_t)n1 * Q3 * n * sizeof(double));
  if (g) memcpy(g, s->g, (size_t)Q3 * n * sizeof(double));
  if (pphi) memcpy(pphi, s->pphi, (size_t)n1 * n * sizeof(double));
  if (pu) memcpy(pu, s->pu, 3 * n * sizeof(double));
  return O3_OK;
}

/* node pieces for the moment identities: g^eq_k and G_k for all k */
int orc3_node_dists(const orc3_sim *s, double rho, double p, const double *u, const double *F,
                    const double *grho, const double *J, double taug, double *geq, double *G) {
  for (int k = 0; k < Q3; ++k) {
    geq[k] = geq3(s, k, rho, p, u);
    G[k] = G3(k, u, F, grho, J, taug);
  }
  return O3_OK;
}

int orc3_node_heq(const orc3_sim *s, int i, double phi, double C, const double *u,
                  double *heq) {
  for (int k = 0; k < Q3; ++k) heq[k] = heq3(s, i, k, phi, C, u);
  return O3_OK;
}

/* stencils of eq:N31 applied to a field f (n) with the domain's boundary
   handling: lap (n), grad (3 x n) */
int orc3_stencils(const orc3_sim *s, const double *f, double *lap, double *g) {
  size_t n = nnodes(s);
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y)
      for (int x = 0; x < s->nx; ++x) {
        size_t id = ((size_t)z * s->ny + y) * s->nx + x;
        if (lap) lap[id] = lap3(s, f, x, y, z);
        if (g) {
          double gv[3];
          grad3(s, f, x, y, z, gv);
          for (int d = 0; d < 3; ++d) g[(size_t)d * n + id] = gv[d];
        }
      }
  return O3_OK;
}

/*
 * nplbm_oracle.c -- plain, slow FP64 CPU implementation of the N-phase
 * phase-field lattice Boltzmann model of Yuan, Liang, Chai & Shi,
 * "Phase-field-based lattice Boltzmann model for immiscible incompressible
 * N-phase flows" (arXiv:1904.12553).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU path is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant generator with the GPU library; nothing in the product path may
 * call it.
 *
 * Every quantity is computed the way the paper writes it, in the paper's
 * order, with no blocking, fusion or algebraic folding:
 *   - setup   : eq:N1 (gamma, Gamma), eq:N36 (beta), eq:N14-N16 (lambda_ij),
 *               eq:N30 (eta_i from the mobility)
 *   - closure : eq:N18 (rho_i, c_i, C_i, J~, rho), eq:N17 (h_i)
 *   - stencils: eq:N31a / eq:N31b (isotropic central first derivative and
 *               Laplacian, written as the sum over the D2Q9 velocities)
 *   - NS LBE  : eq:24 with g^eq of eq:25 and the total-force distribution
 *               G_k of eq:N20_1 (force_form 0) or of Remark 1 in Sec. 3.1
 *               (force_form 1: F carries -div(J~ u) and the tensor part has
 *               no J~ u term); u from eq:N22_1, p from eq:N23,
 *               tau_g from eq:N21_1 with mu = sum_k mu~_k c_k (Sec. 2)
 *   - CH LBEs : eq:N24 with h^eq of eq:N25, source R_k of eq:N26 and the
 *               backward-Euler time derivative of eq:N27; phi_i by eq:N28
 *   - stream  : periodic in x; periodic or halfway bounce-back in y (Sec. 4.2)
 *
 * Readings taken where the paper is silent or garbled (all listed in the
 * design notes of the repository):
 *   - h_i is used exactly as eq:N17 prints it (it equals d/dphi_i of one
 *     half of the printed H of eq:N11);
 *   - the index phi_j inside the sum over i of eq:N18 (last line) and
 *     eq:N29 is read as phi_i;
 *   - initial distributions are the equilibria with p = 0 and the given u;
 *     (phi u) at t = -1 equals (phi u) at t = 0, so R_k = 0 at the first step;
 *   - stencil values next to a wall use mirror ghosts zeta(x,-1)=zeta(x,0),
 *     zeta(x,ny)=zeta(x,ny-1);
 *   - tau_g varies per node as 1/2 + mu/(rho c_s^2), mu = sum mu~_k c_k;
 *   - the body force is G = rho (gx, gy);
 *   - grad(rho) is the eq:N31a stencil applied to the rho field;
 *   - no clipping of c or phi;
 *   - Remark 1's div(J~ u) is component a = sum_b d_b (J~_b u_a), with J~
 *     of the current step and u of the previous step (the stored u of the
 *     source term eq:N27): u of the current step would need the force at the
 *     neighbours, which itself contains the term.  The derivative is the
 *     same first-derivative stencil as every other gradient.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (see build_oracle.py).
 * The OpenMP loops only split independent per-node work across threads;
 * every value is computed by the same expression in the same order for any
 * thread count, so results do not depend on the number of threads.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q 9
#define NMAX 8

/* D2Q9 lattice, Sec. 3.1: velocities in the paper's order, weights, c_s^2. */
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WK[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOTSPD = -2, ORC_ENOMEM = -3 };

typedef struct orc_sim {
  int N, nx, ny, wall_y, grad_scheme, force_form;
  double rho_t[NMAX], mu_t[NMAX];
  double sigma[NMAX][NMAX];
  double mob[NMAX], tau[NMAX]; /* CH mobility m_i and relaxation tau_i */
  double W, eta, beta2, Kc, gx, gy, rho0;
  double gam[NMAX], Gam;
  double lam[NMAX][NMAX];
  double eta_i[NMAX];
  long t;
  /* state */
  double *h;     /* [(N-1)][9][ny*nx] */
  double *g;     /* [9][ny*nx]        */
  double *pphi;  /* previous phi_i    [(N-1)][ny*nx] */
  double *pu;    /* previous u        [2][ny*nx]     */
  /* scratch (macroscopic fields of the current step) */
  double *phi, *c, *rho, *Cp, *lap, *gphi, *gC, *grho, *F, *J, *u, *p, *taug;
  double *q; /* Remark 1: the four products J~_b u_a of the previous u */
  double *hs, *gs; /* post-collision */
} orc_sim;

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */
static int wrap(int a, int n) {
  while (a < 0) a += n;
  while (a >= n) a -= n;
  return a;
}

/* value of a scalar field at (x,y): periodic in x; in y periodic, or a
   mirror ghost next to a wall (the wall sits half a cell outside). */
static double fld(const orc_sim *s, const double *f, int x, int y) {
  x = wrap(x, s->nx);
  if (s->wall_y) {
    if (y < 0) y = -1 - y;
    if (y >= s->ny) y = 2 * s->ny - 1 - y;
  } else {
    y = wrap(y, s->ny);
  }
  return f[(size_t)y * s->nx + x];
}

/* eq:N31a: isotropic central first derivative, summed over i != 0. */
static void grad_central(const orc_sim *s, const double *f, int x, int y,
                         double *gx, double *gy) {
  double ax = 0.0, ay = 0.0;
  for (int k = 1; k < Q; ++k) {
    double d = fld(s, f, x + CX[k], y + CY[k]) - fld(s, f, x - CX[k], y - CY[k]);
    ax += WK[k] * CX[k] * d;
    ay += WK[k] * CY[k] * d;
  }
  *gx = ax / (2.0 * CS2);
  *gy = ay / (2.0 * CS2);
}

/* eq:N40 with the sign of the x+2c term read as negative (as printed the
   stencil is twice the gradient at leading order). */
static void grad_mixed(const orc_sim *s, const double *f, int x, int y,
                       double *gx, double *gy) {
  double ax = 0.0, ay = 0.0;
  for (int k = 1; k < Q; ++k) {
    double d = -fld(s, f, x + 2 * CX[k], y + 2 * CY[k]) +
               5.0 * fld(s, f, x + CX[k], y + CY[k]) - 3.0 * fld(s, f, x, y) -
               fld(s, f, x - CX[k], y - CY[k]);
    ax += WK[k] * CX[k] * d;
    ay += WK[k] * CY[k] * d;
  }
  *gx = ax / (4.0 * CS2);
  *gy = ay / (4.0 * CS2);
}

static void grad(const orc_sim *s, const double *f, int x, int y, double *gx,
                 double *gy) {
  if (s->grad_scheme == 1)
    grad_mixed(s, f, x, y, gx, gy);
  else
    grad_central(s, f, x, y, gx, gy);
}

/* eq:N31b: isotropic Laplacian, summed over i != 0. */
static double laplacian(const orc_sim *s, const double *f, int x, int y) {
  double a = 0.0;
  double f0 = fld(s, f, x, y);
  for (int k = 1; k < Q; ++k)
    a += WK[k] * (fld(s, f, x + CX[k], y + CY[k]) - 2.0 * f0 +
                  fld(s, f, x - CX[k], y - CY[k]));
  return a / CS2;
}

/* ------------------------------------------------------------------ */
/* closure, eq:N12, eq:N17, eq:N18                                      */
/* ------------------------------------------------------------------ */
/* rho_i - rho_N as a function of phi_i, eq:N12 (1-based i < N). */
static double varphi(const orc_sim *s, int i, double phi_i) {
  int N = s->N;
  return 0.5 * (s->rho_t[i - 1] - s->rho_t[N - 1]) +
         0.5 * (s->rho_t[i - 1] + s->rho_t[N - 1]) * phi_i;
}

/* eq:N18 first and second lines: rho_i and c_i, i = 1..N; fifth line: rho. */
static void closure(const orc_sim *s, const double *phi, double *c,
                    double *rho) {
  int N = s->N;
  double rsum = 0.0;
  for (int i = 1; i <= N; ++i) {
    double ri = 1.0 / s->Gam;
    for (int j = 1; j <= N - 1; ++j)
      ri += ((i == j ? 1.0 : 0.0) - s->gam[j - 1] / s->Gam) *
            varphi(s, j, phi[j - 1]);
    c[i - 1] = s->gam[i - 1] * ri;
  }
  /* eq:N18 fifth line (= eq:N29), index read as phi_i */
  rsum = (double)N / s->Gam;
  for (int i = 1; i <= N - 1; ++i)
    rsum += (1.0 - (double)N * s->gam[i - 1] / s->Gam) *
            varphi(s, i, phi[i - 1]);
  *rho = rsum;
}

/* eq:N17: h_i(phi), i = 1..N-1, from the volume fractions c_k. */
static void hbulk(const orc_sim *s, const double *c, double *hi) {
  int N = s->N;
  for (int i = 1; i <= N - 1; ++i) {
    double a = 0.0;
    for (int k = 1; k <= N; ++k) {
      double ck = c[k - 1];
      a += (s->gam[k - 1] * (k == i ? 1.0 : 0.0) -
            s->gam[k - 1] * s->gam[i - 1] / s->Gam) *
           ck * (1.0 - ck) * (1.0 - 2.0 * ck);
    }
    hi[i - 1] = 0.5 * (s->rho_t[i - 1] + s->rho_t[N - 1]) * a;
  }
}

/* ------------------------------------------------------------------ */
/* NS equilibrium (eq:25) and total-force distribution (eq:N20_1)       */
/* ------------------------------------------------------------------ */
static double s_k(int k, double ux, double uy) {
  double cu = CX[k] * ux + CY[k] * uy;
  return WK[k] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) -
                  (ux * ux + uy * uy) / (2.0 * CS2));
}

static double g_eq(const orc_sim *s, int k, double rho, double p, double ux,
                   double uy) {
  if (k == 0) return s->rho0 + p / CS2 * (WK[0] - 1.0) + rho * s_k(0, ux, uy);
  return p / CS2 * WK[k] + rho * s_k(k, ux, uy);
}

/* eq:N20_1, contracted as written: (c c - cs^2 I) : T / (2 cs^4) with
   T = uF + Fu + cs^2 (u grad rho + grad rho u) + J u / (tau_g - 1/2).
   form 1: the distribution of Remark 1 (Sec. 3.1), the same without the
   J u / (tau_g - 1/2) term (F then carries -div(J u)). */
static double G_force(int form, int k, double ux, double uy, double Fx, double Fy,
                      double rx, double ry, double Jx, double Jy,
                      double taug) {
  double u[2] = {ux, uy}, F[2] = {Fx, Fy}, r[2] = {rx, ry}, J[2] = {Jx, Jy};
  double c[2] = {(double)CX[k], (double)CY[k]};
  double T[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      T[a][b] = u[a] * F[b] + F[a] * u[b] + CS2 * u[a] * r[b] +
                CS2 * r[a] * u[b] +
                (form == 1 ? 0.0 : J[a] * u[b] / (1.0 * (taug - 0.5)));
  double contr = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      contr += (c[a] * c[b] - CS2 * (a == b ? 1.0 : 0.0)) * T[a][b];
  double udr = ux * rx + uy * ry;
  double cF = c[0] * Fx + c[1] * Fy;
  return WK[k] * (udr + cF / CS2 + contr / (2.0 * CS2 * CS2));
}

/* CH equilibrium, eq:N25 (1-based i), u is the velocity of the same step. */
static double h_eq(const orc_sim *s, int i, int k, double phi_i, double Ci,
                   double ux, double uy) {
  double et = s->eta_i[i - 1];
  if (k == 0) return phi_i + (WK[0] - 1.0) * et * Ci;
  return WK[k] * et * Ci + WK[k] * (CX[k] * phi_i * ux + CY[k] * phi_i * uy) / CS2;
}

/* ------------------------------------------------------------------ */
/* setup: eq:N1, eq:N36, eq:N14-N16, eq:N30                             */
/* ------------------------------------------------------------------ */
/* L^{kl}_i of eq:N15 (l = N) and eq:N16 (l < N); 1-based k < l, i. */
static double Lvec(const orc_sim *s, int k, int l, int i) {
  int N = s->N;
  const double *r = s->rho_t;
  if (l == N) {
    if (i == k) return 1.0;
    return r[N - 1] / (r[i - 1] + r[N - 1]);
  }
  if (i == k) return r[k - 1] / (r[k - 1] + r[N - 1]);
  if (i == l) return -r[l - 1] / (r[l - 1] + r[N - 1]);
  return 0.0;
}

/* Solve eq:N14 for the symmetric lambda by Gaussian elimination with
   partial pivoting; reject a singular system or a lambda that is not SPD. */
static int solve_lambda(orc_sim *s) {
  int N = s->N, n1 = N - 1;
  int M = N * (N - 1) / 2;
  double A[NMAX * NMAX][NMAX * NMAX + 1];
  int ui[NMAX * NMAX], uj[NMAX * NMAX];
  int m = 0;
  for (int i = 1; i <= n1; ++i)
    for (int j = i; j <= n1; ++j) {
      ui[m] = i;
      uj[m] = j;
      ++m;
    }
  int e = 0;
  double scale = 0.0;
  for (int k = 1; k <= N; ++k)
    for (int l = k + 1; l <= N; ++l) {
      for (int q = 0; q < M; ++q) {
        int i = ui[q], j = uj[q];
        if (i == j)
          A[e][q] = Lvec(s, k, l, i) * Lvec(s, k, l, i);
        else
          A[e][q] = 2.0 * Lvec(s, k, l, i) * Lvec(s, k, l, j);
      }
      A[e][M] = 4.5 * s->eta * s->eta / s->beta2 * s->sigma[k - 1][l - 1] *
                s->sigma[k - 1][l - 1];
      if (fabs(A[e][M]) > scale) scale = fabs(A[e][M]);
      ++e;
    }
  for (int col = 0; col < M; ++col) {
    int piv = col;
    for (int r = col + 1; r < M; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (fabs(A[piv][col]) < 1e-13) return ORC_ENOTSPD;
    if (piv != col)
      for (int q = 0; q <= M; ++q) {
        double t = A[col][q];
        A[col][q] = A[piv][q];
        A[piv][q] = t;
      }
    for (int r = col + 1; r < M; ++r) {
      double f = A[r][col] / A[col][col];
      for (int q = col; q <= M; ++q) A[r][q] -= f * A[col][q];
    }
  }
  double x[NMAX * NMAX];
  for (int r = M - 1; r >= 0; --r) {
    double a = A[r][M];
    for (int q = r + 1; q < M; ++q) a -= A[r][q] * x[q];
    x[r] = a / A[r][r];
  }
  for (int q = 0; q < M; ++q) {
    s->lam[ui[q] - 1][uj[q] - 1] = x[q];
    s->lam[uj[q] - 1][ui[q] - 1] = x[q];
  }
  /* SPD check by Cholesky */
  double Lc[NMAX][NMAX];
  memset(Lc, 0, sizeof Lc);
  for (int i = 0; i < n1; ++i) {
    for (int j = 0; j <= i; ++j) {
      double a = s->lam[i][j];
      for (int q = 0; q < j; ++q) a -= Lc[i][q] * Lc[j][q];
      if (i == j) {
        if (!(a > 1e-14 * scale * s->eta * s->eta / s->beta2)) return ORC_ENOTSPD;
        Lc[i][i] = sqrt(a);
      } else {
        Lc[i][j] = a / Lc[j][j];
      }
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* creation / destruction                                               */
/* ------------------------------------------------------------------ */
void orc_free(orc_sim *s) {
  if (!s) return;
  free(s->h); free(s->g); free(s->pphi); free(s->pu);
  free(s->phi); free(s->c); free(s->rho); free(s->Cp); free(s->lap);
  free(s->gphi); free(s->gC); free(s->grho); free(s->F); free(s->J);
  free(s->u); free(s->p); free(s->taug); free(s->hs); free(s->gs); free(s->q);
  free(s);
}

int orc_create(int N, int nx, int ny, int wall_y, int grad_scheme,
               int force_form, const double *sigma, const double *rho, const double *mu,
               const double *mob, const double *tau_phi, double W, double gx,
               double gy, double rho0, orc_sim **out) {
  *out = NULL;
  if (N < 2 || N > NMAX || nx < 4 || ny < 4 || !(W > 0.0)) return ORC_EINVAL;
  if (grad_scheme != 0 && grad_scheme != 1) return ORC_EINVAL;
  if (force_form != 0 && force_form != 1) return ORC_EINVAL;
  orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
  if (!s) return ORC_ENOMEM;
  s->N = N; s->nx = nx; s->ny = ny; s->wall_y = wall_y ? 1 : 0;
  s->grad_scheme = grad_scheme;
  s->force_form = force_form;
  for (int k = 0; k < N; ++k) {
    if (!(rho[k] > 0.0) || !(mu[k] > 0.0)) { orc_free(s); return ORC_EINVAL; }
    s->rho_t[k] = rho[k];
    s->mu_t[k] = mu[k];
    for (int l = 0; l < N; ++l) s->sigma[k][l] = sigma[k * N + l];
  }
  double smin = 1e300;
  for (int k = 0; k < N; ++k)
    for (int l = k + 1; l < N; ++l) {
      if (!(sigma[k * N + l] > 0.0) || sigma[k * N + l] != sigma[l * N + k]) {
        orc_free(s);
        return ORC_EINVAL;
      }
      if (sigma[k * N + l] < smin) smin = sigma[k * N + l];
    }
  for (int i = 0; i < N - 1; ++i) {
    if (!(mob[i] > 0.0) || !(tau_phi[i] > 0.5)) { orc_free(s); return ORC_EINVAL; }
    s->mob[i] = mob[i];
    s->tau[i] = tau_phi[i];
  }
  s->W = W; s->gx = gx; s->gy = gy; s->rho0 = rho0;
  /* interface scale: the tanh profile tanh(x / (sqrt(2) eta)) has width
     W = 2 sqrt(2) eta */
  s->eta = W / (2.0 * sqrt(2.0));
  /* eq:N1 */
  s->Gam = 0.0;
  for (int k = 0; k < N; ++k) {
    s->gam[k] = 1.0 / s->rho_t[k];
    s->Gam += s->gam[k];
  }
  /* eq:N36 */
  s->beta2 = 3.0 * sqrt(2.0) * smin * s->eta;
  s->Kc = s->beta2 / (s->eta * s->eta);
  int rc = solve_lambda(s);
  if (rc) { orc_free(s); return rc; }
  /* eq:N30 with dt = 1 */
  for (int i = 0; i < N - 1; ++i) s->eta_i[i] = s->mob[i] / (CS2 * (s->tau[i] - 0.5));

  size_t n = (size_t)nx * ny;
  int n1 = N - 1;
  s->h = calloc((size_t)n1 * Q * n, sizeof(double));
  s->g = calloc((size_t)Q * n, sizeof(double));
  s->pphi = calloc((size_t)n1 * n, sizeof(double));
  s->pu = calloc(2 * n, sizeof(double));
  s->phi = calloc((size_t)n1 * n, sizeof(double));
  s->c = calloc((size_t)N * n, sizeof(double));
  s->rho = calloc(n, sizeof(double));
  s->Cp = calloc((size_t)n1 * n, sizeof(double));
  s->lap = calloc((size_t)n1 * n, sizeof(double));
  s->gphi = calloc((size_t)2 * n1 * n, sizeof(double));
  s->gC = calloc((size_t)2 * n1 * n, sizeof(double));
  s->grho = calloc(2 * n, sizeof(double));
  s->F = calloc(2 * n, sizeof(double));
  s->J = calloc(2 * n, sizeof(double));
  s->u = calloc(2 * n, sizeof(double));
  s->p = calloc(n, sizeof(double));
  s->taug = calloc(n, sizeof(double));
  s->hs = calloc((size_t)n1 * Q * n, sizeof(double));
  s->gs = calloc((size_t)Q * n, sizeof(double));
  s->q = calloc(4 * n, sizeof(double));
  if (!s->h || !s->g || !s->pphi || !s->pu || !s->phi || !s->c || !s->rho ||
      !s->Cp || !s->lap || !s->gphi || !s->gC || !s->grho || !s->F || !s->J ||
      !s->u || !s->p || !s->taug || !s->hs || !s->gs || !s->q) {
    orc_free(s);
    return ORC_ENOMEM;
  }
  *out = s;
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* macroscopic fields of the current state                              */
/* ------------------------------------------------------------------ */
/* phi_i (eq:N28), c_k and rho (eq:N18), tau_g (eq:N21_1 with the local
   viscosity), C_i (eq:N18 third line), grad phi_i, grad C_i, grad rho
   (eq:N31a), F = F_s + G (Sec. 3.1), J~ (eq:N18 fourth line), u (eq:N22_1)
   and p (eq:N23). */
static void macroscopic(orc_sim *s) {
  int N = s->N, n1 = N - 1, nx = s->nx, ny = s->ny;
  size_t n = (size_t)nx * ny;
  /* eq:N28 */
  for (int i = 0; i < n1; ++i)
    #pragma omp parallel for schedule(static) if (s->nx * s->ny >= 8192)
    for (size_t x = 0; x < n; ++x) {
      double a = 0.0;
      for (int k = 0; k < Q; ++k) a += s->h[((size_t)i * Q + k) * n + x];
      s->phi[(size_t)i * n + x] = a;
    }
  /* closure and tau_g */
  #pragma omp parallel for schedule(static) if (s->nx * s->ny >= 8192)
  for (size_t x = 0; x < n; ++x) {
    double ph[NMAX], cc[NMAX], r;
    for (int i = 0; i < n1; ++i) ph[i] = s->phi[(size_t)i * n + x];
    closure(s, ph, cc, &r);
    for (int k = 0; k < N; ++k) s->c[(size_t)k * n + x] = cc[k];
    s->rho[x] = r;
    double mu = 0.0;
    for (int k = 0; k < N; ++k) mu += s->mu_t[k] * cc[k];
    s->taug[x] = 0.5 + mu / (r * CS2);
  }
  /* Laplacians and chemical potentials */
  for (int i = 0; i < n1; ++i)
    #pragma omp parallel for schedule(static) if (s->nx * s->ny >= 8192)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        s->lap[(size_t)i * n + (size_t)y * nx + x] =
            laplacian(s, s->phi + (size_t)i * n, x, y);
  #pragma omp parallel for schedule(static) if (s->nx * s->ny >= 8192)
  for (size_t x = 0; x < n; ++x) {
    double cc[NMAX], hi[NMAX];
    for (int k = 0; k < N; ++k) cc[k] = s->c[(size_t)k * n + x];
    hbulk(s, cc, hi);
    for (int i = 0; i < n1; ++i) {
      double a = 0.0;
      for (int j = 0; j < n1; ++j) a -= s->lam[i][j] * s->lap[(size_t)j * n + x];
      s->Cp[(size_t)i * n + x] = a + s->Kc * hi[i];
    }
  }
  /* gradients */
  #pragma omp parallel for schedule(static) if (s->nx * s->ny >= 8192)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t id = (size_t)y * nx + x;
      for (int i = 0; i < n1; ++i) {
        grad(s, s->phi + (size_t)i * n, x, y, &s->gphi[(2 * (size_t)i) * n + id],
             &s->gphi[(2 * (size_t)i + 1) * n + id]);
        grad(s, s->Cp + (size_t)i * n, x, y, &s->gC[(2 * (size_t)i) * n + id],
             &s->gC[(2 * (size_t)i + 1) * n + id]);
      }
      grad(s, s->rho, x, y, &s->grho[id], &s->grho[n + id]);
    }
  /* forces and flux */
  #pragma omp parallel for schedule(static) if (s->nx * s->ny >= 8192)
  for (size_t x = 0; x < n; ++x) {
    double Fx = 0.0, Fy = 0.0, Jx = 0.0, Jy = 0.0;
    for (int i = 0; i < n1; ++i) {
      double Ci = s->Cp[(size_t)i * n + x];
      Fx += Ci * s->gphi[(2 * (size_t)i) * n + x];
      Fy += Ci * s->gphi[(2 * (size_t)i + 1) * n + x];
      double coef = (1.0 - (double)N / s->Gam * s->gam[i]) *
                    (s->rho_t[i] + s->rho_t[N - 1]) / 2.0 * s->mob[i];
      Jx -= coef * s->gC[(2 * (size_t)i) * n + x];
      Jy -= coef * s->gC[(2 * (size_t)i + 1) * n + x];
    }
    double r = s->rho[x];
    Fx += r * s->gx;
    Fy += r * s->gy;
    s->F[x] = Fx; s->F[n + x] = Fy;
    s->J[x] = Jx; s->J[n + x] = Jy;
  }
  /* Remark 1 (Sec. 3.1): F = -div(J~ u) + F_s + G, component a of the
     divergence being sum_b d_b (J~_b u_a), with the previous step's u */
  if (s->force_form == 1) {
    for (size_t x = 0; x < n; ++x) {
      s->q[x] = s->J[x] * s->pu[x];                  /* J_x u_x */
      s->q[n + x] = s->J[n + x] * s->pu[x];          /* J_y u_x */
      s->q[2 * n + x] = s->J[x] * s->pu[n + x];      /* J_x u_y */
      s->q[3 * n + x] = s->J[n + x] * s->pu[n + x];  /* J_y u_y */
    }
    #pragma omp parallel for schedule(static) if (s->nx * s->ny >= 8192)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t id = (size_t)y * nx + x;
        double axx, axy, ayx, ayy, bxx, bxy, byx, byy;
        grad(s, s->q, x, y, &axx, &axy);          /* d/dx, d/dy of J_x u_x */
        grad(s, s->q + n, x, y, &ayx, &ayy);      /* of J_y u_x */
        grad(s, s->q + 2 * n, x, y, &bxx, &bxy);  /* of J_x u_y */
        grad(s, s->q + 3 * n, x, y, &byx, &byy);  /* of J_y u_y */
        s->F[id] -= axx + ayy;
        s->F[n + id] -= bxx + byy;
      }
  }
  /* velocity and pressure */
  #pragma omp parallel for schedule(static) if (s->nx * s->ny >= 8192)
  for (size_t x = 0; x < n; ++x) {
    double Fx = s->F[x], Fy = s->F[n + x], r = s->rho[x];
    double mx = 0.0, my = 0.0;
    for (int k = 0; k < Q; ++k) {
      mx += CX[k] * s->g[(size_t)k * n + x];
      my += CY[k] * s->g[(size_t)k * n + x];
    }
    double ux = (mx + 0.5 * Fx) / r, uy = (my + 0.5 * Fy) / r;
    s->u[x] = ux; s->u[n + x] = uy;
    double sum = 0.0;
    for (int k = 1; k < Q; ++k) sum += s->g[(size_t)k * n + x];
    s->p[x] = CS2 / (1.0 - WK[0]) *
              (sum + 0.5 * (ux * s->grho[x] + uy * s->grho[n + x]) + r * s_k(0, ux, uy));
  }
}

/* push streaming of post-collision values, periodic in x, periodic or
   halfway bounce-back in y */
static void stream(orc_sim *s, const double *src, double *dst, int nfields) {
  int nx = s->nx, ny = s->ny;
  size_t n = (size_t)nx * ny;
  static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  for (int f = 0; f < nfields; ++f)
    for (int k = 0; k < Q; ++k)
      #pragma omp parallel for schedule(static) if (s->nx * s->ny >= 8192)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          double v = src[((size_t)f * Q + k) * n + (size_t)y * nx + x];
          int xd = wrap(x + CX[k], nx), yd = y + CY[k];
          if (yd < 0 || yd >= ny) {
            if (s->wall_y) {
              dst[((size_t)f * Q + OPP[k]) * n + (size_t)y * nx + x] = v;
              continue;
            }
            yd = wrap(yd, ny);
          }
          dst[((size_t)f * Q + k) * n + (size_t)yd * nx + xd] = v;
        }
}

/* ------------------------------------------------------------------ */
/* public API                                                           */
/* ------------------------------------------------------------------ */
/* Initial state from volume fractions c (N x ny x nx) and velocity u
   (2 x ny x nx, or NULL for rest): phi_i from eq:N12 inverted with
   rho_k = rho~_k c_k, p = 0, g = g^eq, h = h^eq, previous (phi,u) = current. */
int orc_init(orc_sim *s, const double *c, const double *u) {
  int N = s->N, n1 = N - 1;
  size_t n = (size_t)s->nx * s->ny;
  for (int i = 1; i <= n1; ++i)
    for (size_t x = 0; x < n; ++x) {
      double a = 0.5 * (s->rho_t[i - 1] + s->rho_t[N - 1]);
      double b = 0.5 * (s->rho_t[i - 1] - s->rho_t[N - 1]);
      s->phi[(size_t)(i - 1) * n + x] =
          (s->rho_t[i - 1] * c[(size_t)(i - 1) * n + x] -
           s->rho_t[N - 1] * c[(size_t)(N - 1) * n + x] - b) / a;
    }
  /* closure, Laplacians and C_i for the initial phi */
  for (size_t x = 0; x < n; ++x) {
    double ph[NMAX], cc[NMAX], r;
    for (int i = 0; i < n1; ++i) ph[i] = s->phi[(size_t)i * n + x];
    closure(s, ph, cc, &r);
    for (int k = 0; k < N; ++k) s->c[(size_t)k * n + x] = cc[k];
    s->rho[x] = r;
  }
  for (int i = 0; i < n1; ++i)
    for (int y = 0; y < s->ny; ++y)
      for (int x = 0; x < s->nx; ++x)
        s->lap[(size_t)i * n + (size_t)y * s->nx + x] =
            laplacian(s, s->phi + (size_t)i * n, x, y);
  for (size_t x = 0; x < n; ++x) {
    double cc[NMAX], hi[NMAX];
    for (int k = 0; k < N; ++k) cc[k] = s->c[(size_t)k * n + x];
    hbulk(s, cc, hi);
    double ux = u ? u[x] : 0.0, uy = u ? u[n + x] : 0.0;
    for (int i = 0; i < n1; ++i) {
      double a = 0.0;
      for (int j = 0; j < n1; ++j) a -= s->lam[i][j] * s->lap[(size_t)j * n + x];
      double Ci = a + s->Kc * hi[i];
      double ph = s->phi[(size_t)i * n + x];
      for (int k = 0; k < Q; ++k)
        s->h[((size_t)i * Q + k) * n + x] = h_eq(s, i + 1, k, ph, Ci, ux, uy);
      s->pphi[(size_t)i * n + x] = ph;
    }
    for (int k = 0; k < Q; ++k) s->g[(size_t)k * n + x] = g_eq(s, k, s->rho[x], 0.0, ux, uy);
    s->pu[x] = ux;
    s->pu[n + x] = uy;
  }
  s->t = 0;
  return ORC_OK;
}

/* One or more time steps: macroscopic fields, NS collision (eq:24),
   CH collisions (eq:N24), streaming. */
int orc_step(orc_sim *s, long nsteps) {
  int N = s->N, n1 = N - 1;
  size_t n = (size_t)s->nx * s->ny;
  for (long it = 0; it < nsteps; ++it) {
    macroscopic(s);
    #pragma omp parallel for schedule(static) if (s->nx * s->ny >= 8192)
    for (size_t x = 0; x < n; ++x) {
      double ux = s->u[x], uy = s->u[n + x], r = s->rho[x], p = s->p[x];
      double tg = s->taug[x];
      for (int k = 0; k < Q; ++k) {
        double geq = g_eq(s, k, r, p, ux, uy);
        double G = G_force(s->force_form, k, ux, uy, s->F[x], s->F[n + x], s->grho[x],
                           s->grho[n + x], s->J[x], s->J[n + x], tg);
        double gk = s->g[(size_t)k * n + x];
        s->gs[(size_t)k * n + x] = gk - (gk - geq) / tg + (1.0 - 1.0 / (2.0 * tg)) * G;
      }
      for (int i = 0; i < n1; ++i) {
        double ph = s->phi[(size_t)i * n + x], Ci = s->Cp[(size_t)i * n + x];
        /* eq:N27: backward Euler derivative of phi u */
        double dtx = ph * ux - s->pphi[(size_t)i * n + x] * s->pu[x];
        double dty = ph * uy - s->pphi[(size_t)i * n + x] * s->pu[n + x];
        double ti = s->tau[i];
        for (int k = 0; k < Q; ++k) {
          double heq = h_eq(s, i + 1, k, ph, Ci, ux, uy);
          double R = (1.0 - 1.0 / (2.0 * ti)) * WK[k] * (CX[k] * dtx + CY[k] * dty) / CS2;
          double hk = s->h[((size_t)i * Q + k) * n + x];
          s->hs[((size_t)i * Q + k) * n + x] = hk - (hk - heq) / ti + R;
        }
      }
    }
    for (int i = 0; i < n1; ++i)
      memcpy(s->pphi + (size_t)i * n, s->phi + (size_t)i * n, n * sizeof(double));
    memcpy(s->pu, s->u, 2 * n * sizeof(double));
    stream(s, s->hs, s->h, n1);
    stream(s, s->gs, s->g, 1);
    s->t += 1;
  }
  return ORC_OK;
}

/* c (N x n), u (2 x n), p (n) of the current state; any pointer may be NULL. */
int orc_macro(orc_sim *s, double *c, double *u, double *p) {
  size_t n = (size_t)s->nx * s->ny;
  macroscopic(s);
  if (c) memcpy(c, s->c, (size_t)s->N * n * sizeof(double));
  if (u) memcpy(u, s->u, 2 * n * sizeof(double));
  if (p) memcpy(p, s->p, n * sizeof(double));
  return ORC_OK;
}

/* every macroscopic field of the current state, for tests */
int orc_fields(orc_sim *s, double *phi, double *rho, double *C, double *F,
               double *J, double *grho, double *taug) {
  int n1 = s->N - 1;
  size_t n = (size_t)s->nx * s->ny;
  macroscopic(s);
  if (phi) memcpy(phi, s->phi, (size_t)n1 * n * sizeof(double));
  if (rho) memcpy(rho, s->rho, n * sizeof(double));
  if (C) memcpy(C, s->Cp, (size_t)n1 * n * sizeof(double));
  if (F) memcpy(F, s->F, 2 * n * sizeof(double));
  if (J) memcpy(J, s->J, 2 * n * sizeof(double));
  if (grho) memcpy(grho, s->grho, 2 * n * sizeof(double));
  if (taug) memcpy(taug, s->taug, n * sizeof(double));
  return ORC_OK;
}

/* per-phase mass M_k = sum_x c_k */
int orc_mass(orc_sim *s, double *out) {
  size_t n = (size_t)s->nx * s->ny;
  macroscopic(s);
  for (int k = 0; k < s->N; ++k) {
    double a = 0.0;
    for (size_t x = 0; x < n; ++x) a += s->c[(size_t)k * n + x];
    out[k] = a;
  }
  return ORC_OK;
}

long orc_time(const orc_sim *s) { return s->t; }

/* raw distributions: h [(N-1)][9][n], g [9][n], previous phi and u */
int orc_get_state(const orc_sim *s, double *h, double *g, double *pphi, double *pu) {
  size_t n = (size_t)s->nx * s->ny;
  int n1 = s->N - 1;
  if (h) memcpy(h, s->h, (size_t)n1 * Q * n * sizeof(double));
  if (g) memcpy(g, s->g, (size_t)Q * n * sizeof(double));
  if (pphi) memcpy(pphi, s->pphi, (size_t)n1 * n * sizeof(double));
  if (pu) memcpy(pu, s->pu, 2 * n * sizeof(double));
  return ORC_OK;
}

int orc_set_state(orc_sim *s, const double *h, const double *g, const double *pphi,
                  const double *pu) {
  size_t n = (size_t)s->nx * s->ny;
  int n1 = s->N - 1;
  if (h) memcpy(s->h, h, (size_t)n1 * Q * n * sizeof(double));
  if (g) memcpy(s->g, g, (size_t)Q * n * sizeof(double));
  if (pphi) memcpy(s->pphi, pphi, (size_t)n1 * n * sizeof(double));
  if (pu) memcpy(s->pu, pu, 2 * n * sizeof(double));
  return ORC_OK;
}

/* ---- node-level pieces exposed for unit pins ---- */
int orc_lambda(const orc_sim *s, double *lam, double *beta2, double *K, double *eta) {
  int n1 = s->N - 1;
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) lam[i * n1 + j] = s->lam[i][j];
  if (beta2) *beta2 = s->beta2;
  if (K) *K = s->Kc;
  if (eta) *eta = s->eta;
  return ORC_OK;
}

double orc_Lvec(const orc_sim *s, int k, int l, int i) { return Lvec(s, k, l, i); }

int orc_closure(const orc_sim *s, const double *phi, double *c, double *rho) {
  closure(s, phi, c, rho);
  return ORC_OK;
}

int orc_hbulk(const orc_sim *s, const double *phi, double *h) {
  double c[NMAX], r;
  closure(s, phi, c, &r);
  hbulk(s, c, h);
  return ORC_OK;
}

/* g^eq_k and G_k for all k at one node (for the moment identities) */
int orc_node_dists(const orc_sim *s, double rho, double p, double ux, double uy,
                   double Fx, double Fy, double rx, double ry, double Jx,
                   double Jy, double taug, double *geq, double *G) {
  for (int k = 0; k < Q; ++k) {
    geq[k] = g_eq(s, k, rho, p, ux, uy);
    G[k] = G_force(s->force_form, k, ux, uy, Fx, Fy, rx, ry, Jx, Jy, taug);
  }
  return ORC_OK;
}

int orc_node_heq(const orc_sim *s, int i, double phi, double C, double ux, double uy,
                 double *heq) {
  for (int k = 0; k < Q; ++k) heq[k] = h_eq(s, i, k, phi, C, ux, uy);
  return ORC_OK;
}

/* stencils applied to an arbitrary field f (ny x nx) with the domain's
   boundary handling; out_lap (n), out_g (2 x n) */
int orc_stencils(const orc_sim *s, const double *f, double *out_lap, double *out_g) {
  size_t n = (size_t)s->nx * s->ny;
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x) {
      size_t id = (size_t)y * s->nx + x;
      if (out_lap) out_lap[id] = laplacian(s, f, x, y);
      if (out_g) grad(s, f, x, y, &out_g[id], &out_g[n + id]);
    }
  return ORC_OK;
}

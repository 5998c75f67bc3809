// nplbm_host.cpp -- host side of the C ABI declared in include/nplbm.h:
// parameter validation, the eq:N14 mixing-coefficient solve, folding of the
// closure constants, device memory layout, launch orchestration (with HIP
// graphs for long step runs), read-back, diagnostics and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "nplbm.h"
#include "nplbm_internal.h"
#include "host_internal.h"

namespace nplbm {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
void clear_error() { g_err.clear(); }
const char *last_error() { return g_err.c_str(); }

int hip_fail(hipError_t e, const char *what) {
  return fail(NPLBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------- validation
// Mixing coefficients lambda_ij from the pairwise tensions (eq:N14).
// L^{kl} is half the jump of the order parameters between pure phase k and
// pure phase l, with phi_i(pure j) from eq:N12 (this reproduces eq:N15 and
// eq:N16).  The M = N(N-1)/2 equations in the M unknowns lambda_ij, i <= j,
// are solved by Gaussian elimination with complete pivoting; lambda must be
// symmetric positive definite (checked by Jacobi eigenvalues).
static void pure_phi(int N, const double *rho, int j, double *phi) {
  // phi_i = (rho~_i c_i - rho~_N c_N - (rho~_i - rho~_N)/2) / ((rho~_i + rho~_N)/2)
  for (int i = 0; i < N - 1; ++i) {
    const double ci = (i == j) ? 1.0 : 0.0, cN = (j == N - 1) ? 1.0 : 0.0;
    phi[i] = (rho[i] * ci - rho[N - 1] * cN - 0.5 * (rho[i] - rho[N - 1])) /
             (0.5 * (rho[i] + rho[N - 1]));
  }
}

static bool jacobi_min_eig(std::vector<double> A, int n, double &emin, double &emax) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double th = 0.5 * (A[q * n + q] - A[p * n + p]) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  emin = 1e300;
  emax = -1e300;
  for (int i = 0; i < n; ++i) {
    emin = std::min(emin, A[i * n + i]);
    emax = std::max(emax, A[i * n + i]);
  }
  return true;
}

int derive(const nplbm_params *p, Derived &d) {
  if (!p) return fail(NPLBM_EINVAL, "params is NULL");
  const int N = p->N;
  if (N < 2 || N > NPLBM_MAX_PHASES)
    return fail(NPLBM_EINVAL, "N=%d outside [2, %d]", N, NPLBM_MAX_PHASES);
  if (p->nx < 4 || p->ny < 4) return fail(NPLBM_EINVAL, "nx, ny must be >= 4");
  if (p->nz < 0 || p->nz == 2 || p->nz == 3) return fail(NPLBM_EINVAL, "nz must be 0, 1 or >= 4");
  if ((int64_t)p->nx * p->ny * dom_nz(p) > (int64_t)1 << 30)
    return fail(NPLBM_EINVAL, "domain larger than 2^30 nodes");
  if (is3d(p)) {
    if (N > 5) return fail(NPLBM_EINVAL, "3-D domains are built for N <= 5");
    if (p->grad_scheme != kGradCentral || p->force_form != 0)
      return fail(NPLBM_EINVAL, "3-D domains use grad_scheme 0 and force_form 0");
    if (p->wall_y != 0) return fail(NPLBM_EINVAL, "3-D domains are periodic in y (wall_y 0)");
    if (p->wall_z != 0 && p->wall_z != 1) return fail(NPLBM_EINVAL, "wall_z must be 0 or 1");
    if (!std::isfinite(p->gz)) return fail(NPLBM_EINVAL, "gz must be finite");
    // the 3-D kernel addresses one plane of a state group (ny row blocks)
    // with 32-bit byte offsets below 2^31
    if ((int64_t)p->ny * 15 * (N - 1) * state_pitch(p) * (p->precision / 8) >= (int64_t)1 << 31)
      return fail(NPLBM_EINVAL, "nx * ny too large for a 3-D domain: a plane would exceed 2^31 bytes");
  } else if (p->wall_z != 0 || p->gz != 0.0) {
    return fail(NPLBM_EINVAL, "wall_z and gz apply to 3-D domains (nz >= 4) only");
  }
  if (p->precision != 32 && p->precision != 64)
    return fail(NPLBM_EINVAL, "precision must be 32 or 64");
  // the step kernel addresses one row block of a state group (all its
  // planes of one lattice row) with 32-bit byte offsets below 2^31
  if ((int64_t)(is3d(p) ? 15 : 9) * (N - 1) * state_pitch(p) * (p->precision / 8) >=
      (int64_t)1 << 31)
    return fail(NPLBM_EINVAL, "nx=%d too large: a row block would exceed 2^31 bytes", p->nx);
  if (p->grad_scheme != kGradCentral && p->grad_scheme != kGradMixed)
    return fail(NPLBM_EINVAL, "grad_scheme must be 0 (eq:N31a) or 1 (eq:N40)");
  if (p->force_form != 0 && p->force_form != 1)
    return fail(NPLBM_EINVAL, "force_form must be 0 (eq:N20_1) or 1 (Remark 1)");
  if (p->force_form == 1 && p->grad_scheme != kGradCentral)
    return fail(NPLBM_EINVAL, "force_form 1 is built with grad_scheme 0 only");
  if (p->wall_y != 0 && p->wall_y != 1) return fail(NPLBM_EINVAL, "wall_y must be 0 or 1");
  if (!p->sigma || !p->rho || !p->mu || !p->mobility || !p->tau_phi)
    return fail(NPLBM_EINVAL, "a parameter array is NULL");
  if (!(p->interface_width > 0.0) || !std::isfinite(p->interface_width))
    return fail(NPLBM_EINVAL, "interface_width must be > 0");
  if (!std::isfinite(p->gx) || !std::isfinite(p->gy))
    return fail(NPLBM_EINVAL, "gx, gy must be finite");
  double smin = 1e300;
  for (int k = 0; k < N; ++k) {
    if (!(p->rho[k] > 0.0) || !std::isfinite(p->rho[k]))
      return fail(NPLBM_EINVAL, "rho[%d] must be > 0", k);
    if (!(p->mu[k] > 0.0) || !std::isfinite(p->mu[k]))
      return fail(NPLBM_EINVAL, "mu[%d] must be > 0", k);
    for (int l = k + 1; l < N; ++l) {
      const double s = p->sigma[k * N + l];
      if (!(s > 0.0) || !std::isfinite(s)) return fail(NPLBM_EINVAL, "sigma[%d][%d] must be > 0", k, l);
      if (s != p->sigma[l * N + k]) return fail(NPLBM_EINVAL, "sigma is not symmetric");
      smin = std::min(smin, s);
    }
  }
  for (int i = 0; i < N - 1; ++i) {
    if (!(p->mobility[i] > 0.0) || !std::isfinite(p->mobility[i]))
      return fail(NPLBM_EINVAL, "mobility[%d] must be > 0", i);
    if (!(p->tau_phi[i] > 0.5) || !std::isfinite(p->tau_phi[i]))
      return fail(NPLBM_EINVAL, "tau_phi[%d] must be > 1/2", i);
  }
  const int M = N - 1;
  d.N = N;
  d.eta = p->interface_width / (2.0 * std::sqrt(2.0));
  d.beta2 = 3.0 * std::sqrt(2.0) * smin * d.eta;  // eq:N36
  d.K = d.beta2 / (d.eta * d.eta);

  // eq:N14 system
  const int Mu = N * (N - 1) / 2;
  std::vector<int> ui, uj;
  for (int i = 0; i < M; ++i)
    for (int j = i; j < M; ++j) {
      ui.push_back(i);
      uj.push_back(j);
    }
  std::vector<double> A((size_t)Mu * Mu), b(Mu);
  int e = 0;
  double bscale = 0.0;
  std::vector<double> pk(M), pl(M), L(M);
  for (int k = 0; k < N; ++k)
    for (int l = k + 1; l < N; ++l) {
      pure_phi(N, p->rho, k, pk.data());
      pure_phi(N, p->rho, l, pl.data());
      for (int i = 0; i < M; ++i) L[i] = 0.5 * (pk[i] - pl[i]);
      for (int q = 0; q < Mu; ++q)
        A[(size_t)e * Mu + q] = (ui[q] == uj[q] ? 1.0 : 2.0) * L[ui[q]] * L[uj[q]];
      const double s = p->sigma[k * N + l];
      b[e] = 4.5 * d.eta * d.eta / d.beta2 * s * s;
      bscale = std::max(bscale, std::fabs(b[e]));
      ++e;
    }
  // complete pivoting
  std::vector<int> colp(Mu);
  for (int q = 0; q < Mu; ++q) colp[q] = q;
  double amax = 0.0;
  for (double v : A) amax = std::max(amax, std::fabs(v));
  for (int c = 0; c < Mu; ++c) {
    int pr = c, pc = c;
    double best = -1.0;
    for (int r = c; r < Mu; ++r)
      for (int q = c; q < Mu; ++q)
        if (std::fabs(A[(size_t)r * Mu + q]) > best) {
          best = std::fabs(A[(size_t)r * Mu + q]);
          pr = r;
          pc = q;
        }
    if (!(best > 1e-12 * amax))
      return fail(NPLBM_ENOTSPD, "eq:N14 system is singular for these sigma and rho");
    if (pr != c) {
      for (int q = 0; q < Mu; ++q) std::swap(A[(size_t)pr * Mu + q], A[(size_t)c * Mu + q]);
      std::swap(b[pr], b[c]);
    }
    if (pc != c) {
      for (int r = 0; r < Mu; ++r) std::swap(A[(size_t)r * Mu + pc], A[(size_t)r * Mu + c]);
      std::swap(colp[pc], colp[c]);
    }
    for (int r = c + 1; r < Mu; ++r) {
      const double f = A[(size_t)r * Mu + c] / A[(size_t)c * Mu + c];
      if (f == 0.0) continue;
      for (int q = c; q < Mu; ++q) A[(size_t)r * Mu + q] -= f * A[(size_t)c * Mu + q];
      b[r] -= f * b[c];
    }
  }
  std::vector<double> y(Mu);
  for (int r = Mu - 1; r >= 0; --r) {
    double a = b[r];
    for (int q = r + 1; q < Mu; ++q) a -= A[(size_t)r * Mu + q] * y[q];
    y[r] = a / A[(size_t)r * Mu + r];
  }
  std::vector<double> x(Mu);
  for (int q = 0; q < Mu; ++q) x[colp[q]] = y[q];
  d.lam.assign((size_t)M * M, 0.0);
  for (int q = 0; q < Mu; ++q) {
    d.lam[(size_t)ui[q] * M + uj[q]] = x[q];
    d.lam[(size_t)uj[q] * M + ui[q]] = x[q];
  }
  double emin, emax;
  jacobi_min_eig(d.lam, M, emin, emax);
  if (!(emin > 1e-12 * std::fabs(emax)))
    return fail(NPLBM_ENOTSPD,
                "mixing matrix lambda (eq:N14) is not positive definite (min eig %.3e)", emin);

  // folded closure constants, in double
  Consts<double> &K = d.cd;
  std::memset(&K, 0, sizeof K);
  std::vector<double> gam(N);
  double Gam = 0.0;
  for (int k = 0; k < N; ++k) {
    gam[k] = 1.0 / p->rho[k];
    Gam += gam[k];
  }
  std::vector<double> a(M), bb(M), kap(M);
  for (int i = 0; i < M; ++i) {
    a[i] = 0.5 * (p->rho[i] + p->rho[N - 1]);
    bb[i] = 0.5 * (p->rho[i] - p->rho[N - 1]);
    kap[i] = 1.0 - N * gam[i] / Gam;
    d.P1[i] = p->rho[i] / a[i];
    d.PN[i] = -p->rho[N - 1] / a[i];
    d.P0[i] = -bb[i] / a[i];
  }
  auto P = [&](int k, int j) { return gam[k] * ((k == j ? 1.0 : 0.0) - gam[j] / Gam); };
  for (int k = 0; k < N; ++k) {
    double ca = gam[k] / Gam;
    for (int j = 0; j < M; ++j) {
      ca += P(k, j) * bb[j];
      K.cA[k][j] = P(k, j) * a[j];
      K.KH[k][j] = d.K * a[j] * P(k, j);
    }
    K.ca[k] = ca;
  }
  K.ra = (double)N / Gam;
  K.ma = 0.0;
  for (int k = 0; k < N; ++k) K.ma += p->mu[k] * K.ca[k];
  for (int j = 0; j < M; ++j) {
    K.ra += kap[j] * bb[j];
    K.rA[j] = kap[j] * a[j];
    double m = 0.0;
    for (int k = 0; k < N; ++k) m += p->mu[k] * K.cA[k][j];
    K.mA[j] = m;
    K.Jc[j] = -kap[j] * a[j] * p->mobility[j];
    K.eta_i[j] = p->mobility[j] / ((p->tau_phi[j] - 0.5) / 3.0);  // eq:N30
    K.itau_i[j] = 1.0 / p->tau_phi[j];
    K.src_i[j] = 1.0 - 0.5 / p->tau_phi[j];
    for (int i = 0; i < M; ++i) K.lam[j][i] = d.lam[(size_t)j * M + i];
  }
  K.gx = p->gx;
  K.gy = p->gy;
  K.gz = is3d(p) ? p->gz : 0.0;
  // constant tau_g when mu~_k / rho~_k is the same for every phase
  const double nu0 = p->mu[0] / p->rho[0];
  bool cst = true;
  for (int k = 1; k < N; ++k)
    if (std::fabs(p->mu[k] / p->rho[k] - nu0) > 1e-14 * nu0) cst = false;
  K.const_tau = cst ? 1 : 0;
  const double tg = 0.5 + 3.0 * nu0;
  K.itau_g = 1.0 / tg;
  K.src_g = 1.0 - 0.5 / tg;
  K.theta_g = 1.0 / (3.0 * nu0);
  // float copy
  Consts<float> &F = d.cf;
  std::memset(&F, 0, sizeof F);
  for (int k = 0; k < kMaxN; ++k) {
    F.ca[k] = (float)K.ca[k];
    for (int j = 0; j < kMaxM; ++j) {
      F.cA[k][j] = (float)K.cA[k][j];
      F.KH[k][j] = (float)K.KH[k][j];
    }
  }
  F.ra = (float)K.ra;
  F.ma = (float)K.ma;
  for (int j = 0; j < kMaxM; ++j) {
    F.rA[j] = (float)K.rA[j];
    F.mA[j] = (float)K.mA[j];
    F.Jc[j] = (float)K.Jc[j];
    F.eta_i[j] = (float)K.eta_i[j];
    F.itau_i[j] = (float)K.itau_i[j];
    F.src_i[j] = (float)K.src_i[j];
    for (int i = 0; i < kMaxM; ++i) F.lam[j][i] = (float)K.lam[j][i];
  }
  F.gx = (float)K.gx;
  F.gy = (float)K.gy;
  F.gz = (float)K.gz;
  F.itau_g = (float)K.itau_g;
  F.src_g = (float)K.src_g;
  F.theta_g = (float)K.theta_g;
  F.const_tau = K.const_tau;
  return NPLBM_OK;
}

// ------------------------------------------------------------ memory plan
static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Padding (in elements) appended to every population plane.  Without it the
// ~10N planes a node touches are a power of two apart for power-of-two
// lattices and fall onto the same HBM channels.
int64_t plane_pad(size_t elem) {
  if (const char *e = std::getenv("NPLBM_PLANE_PAD")) return std::atoll(e);
  return (int64_t)(kPlanePadBytes / elem);
}

// Padding (in elements) appended to every row block of the row-interleaved
// layout.
int64_t row_pad(size_t elem) {
  if (const char *e = std::getenv("NPLBM_ROW_PAD")) return std::atoll(e);
  return (int64_t)(kRowPadBytes / elem);
}

// Workgroups the step kernel keeps resident on the device at once: as many
// as the registers allow, up to 8 waves per compute unit.  A 16-wave
// configuration (two 8-wave FP32 workgroups at N = 3) measured 4 points of
// the HBM roofline slower than one: twice as many concurrent row streams and
// half-height strips, for no gain in bytes in flight.
int step_scheme(const nplbm_params *p) {
  if (p->grad_scheme == kGradMixed) return kSchemeMixed;
  return p->force_form == 1 ? kSchemeRemark1 : kSchemeCentral;
}

int resident_step_blocks(int N, int precision, int scheme) {
  static int cus = -1;
  if (cus < 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    else
      cus = 0;
  }
  const int bw = step_geom(N, precision, scheme).bw;
  const int per = step_blocks_per_cu(N, precision, scheme, bw);
  const int cap = std::max(1, 8 / std::max(1, bw * kRows / 64));
  return cus > 0 && per > 0 ? cus * std::min(per, cap) : 0;
}

// Strip count for a single-domain launch: one full round of resident
// workgroups (no tail), unless overridden.
int single_domain_target(const nplbm_params *p) {
  if (const char *env = std::getenv("NPLBM_TARGET_BLOCKS")) {
    const int t = std::atoi(env);
    if (t > 0) return t;
  }
  const int r = resident_step_blocks(p->N, p->precision, step_scheme(p));
  return r > 0 ? r : 2048;
}

// Elements between the planes of one lattice row: nx rounded up to whole
// 128-byte lines of FP32 (rows start on lines); in 3-D one extra line when
// that is a multiple of 256 elements (256^3 N = 3 FP32: 40.5% against 38.8%
// of the HBM roofline; 2-D measured no difference).  The validation bounds
// the 32-bit offsets with this same pitch.
int64_t state_pitch(const nplbm_params *p) {
  int64_t pitch = ((int64_t)p->nx + 31) & ~(int64_t)31;
  if (is3d(p) && pitch % 256 == 0) pitch += 32;
  if (const char *e = std::getenv("NPLBM_PITCH_PAD")) pitch += std::max(0, std::atoi(e)) & ~31;
  return pitch;
}

Layout plan_layout(const nplbm_params *p) {
  Layout L;
  const int N = p->N, M = N - 1;
  const size_t s = p->precision == 64 ? 8 : 4;
  L.pitch = (int)state_pitch(p);
  const bool d3 = is3d(p);
  const int nrows = p->ny * dom_nz(p);  // (z, y) lines of nodes
  const size_t n = (size_t)p->nx * nrows;
  // planes per group: CH populations, NS populations k >= 1, previous phi and u
  const int np[3] = {M * (d3 ? 15 : 9), d3 ? 14 : 8, M + (d3 ? 3 : 2)};
  const char *lay = std::getenv("NPLBM_LAYOUT");
  const bool soa = lay && std::strcmp(lay, "soa") == 0;
  for (int G = 0; G < 3; ++G) {
    if (soa) {
      L.ps[G] = (int64_t)L.pitch * nrows + plane_pad(s);
      L.rs[G] = L.pitch;
      L.gbytes[G] = (size_t)np[G] * L.ps[G] * s;
    } else {
      L.ps[G] = L.pitch;
      L.rs[G] = (int64_t)np[G] * L.pitch + row_pad(s);
      L.gbytes[G] = (size_t)nrows * L.rs[G] * s;
    }
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += al256(bytes);
    return o;
  };
  for (int b = 0; b < 2; ++b) L.h[b] = take(L.gbytes[0]);
  for (int b = 0; b < 2; ++b) L.g[b] = take(L.gbytes[1]);
  for (int b = 0; b < 2; ++b) L.prev[b] = take(L.gbytes[2]);
  L.state_end = off;
  L.desc = take(sizeof(DomDesc));
  // room for any strip decomposition (strip height >= 2, XCD padding), or
  // for the 3-D tiles (at least 4 x 4 nodes and 2 planes each)
  L.nstrips = d3 ? ((p->nx + 3) / 4) * ((p->ny + 3) / 4) * ((dom_nz(p) + 1) / 2) + 8
                 : ((p->nx + 7) / 8) * ((p->ny + 1) / 2) + 8;
  L.strips = take(sizeof(StripDesc) * (size_t)L.nstrips);
  L.phi = take((size_t)M * n * 8);
  L.rho = take(n * 8);
  L.C = take((size_t)M * n * 8);
  L.c = take((size_t)N * n * 8);
  L.u = take((d3 ? 3 : 2) * n * 8);
  L.p = take(n * 8);
  // 3-D: the phi array written by the phi pass of each step
  L.phi3 = d3 ? take((size_t)nrows * M * L.pitch * s) : 0;
  // the products J~_b u_a of the Remark 1 force, for the read-back
  L.q = p->force_form == 1 ? take(4 * n * 8) : 0;
  L.nblk = diag_blocks((int64_t)n);
  L.partials = take((size_t)L.nblk * (kMaxN + 2) * 8);
  L.out = take((kMaxN + 2) * 8);
  L.total = off;
  return L;
}

// Strip geometry of the step kernel for a precision and scheme.
// Interior widths are multiples of one 128-byte cache line of state values
// (32 floats or 16 doubles), so no line is written by two workgroups.  Rows
// of 256 threads measured fastest on gfx950 in FP32, and in FP64 with the
// central gradients for N <= 3 (4096^2: N = 2 64.7% of the HBM roofline
// against 60.6% with 64-thread rows, N = 3 65.8% against 59.5%, and 74.4%
// once the rows became interior lanes with 256-column strips); FP64 with
// N >= 4 or the two-hop schemes runs one wave per SIMD, where 64-thread rows
// measured fastest (N = 4: 66.3% against 58.0%).  The two-hop schemes in
// FP32 run two 128-thread-row workgroups per compute unit instead of one
// with 256-thread rows (mixed, rows of interior lanes, 2048^2: N = 3 62.4%
// against 57.4%, N = 4 60.4% against 54.9%, N = 5 61.2% against 56.3%;
// Remark 1 at N >= 4 has LDS rings for no more than 128).  The halo is 2
// columns for the central gradients and 3 for the two-hop ones (eq:N40, or
// the divergence of Remark 1 taken of a product of gradients).
StepGeom step_geom(int N, int precision, int scheme) {
  StepGeom g;
  g.halo = scheme == kSchemeCentral ? 2 : 3;
  const int unit = precision == 64 ? 16 : 32;
  g.bw = precision == 64 ? (scheme == kSchemeCentral && N <= 3 ? 256 : 64)
                         : (scheme == kSchemeCentral ? 256 : 128);
  if (const char *e = std::getenv("NPLBM_BW")) {
    const int b = std::atoi(e);
    g.bw = (b == 128 || b == 256) ? b : 64;
  }
  g.bw = std::min(g.bw, step_max_bw(N, precision, scheme));
  // rows of interior lanes hold no halo columns (their halo phi is pulled
  // by lanes per direction); the other rows hold theirs
  const int cols = interior_lanes(N, precision / 8, scheme) ? g.bw : g.bw - 2 * g.halo;
  g.tx = (cols / unit) * unit;
  if (const char *e = std::getenv("NPLBM_TX")) g.tx = std::atoi(e);
  if (g.tx < 8) g.tx = 8;
  if (g.tx > cols) g.tx = cols;
  g.unit = unit;
  return g;
}

// Strip decomposition of one domain for the marching step kernel.  Strips
// are geom.tx interior columns wide and H rows tall, H chosen so that the whole
// launch has about `target` workgroups; neighbouring strip rows march in
// opposite directions, so the halo rows they share are read at the same
// time (both at their start or both at their end).
void build_strips(int nx, int ny, int dom, const StepGeom &geom, std::vector<StripDesc> &out,
                  int target) {
  const int kTX = geom.tx;
  const int unit = std::max(1, std::min(geom.unit, kTX));
  if (target <= 0) {
    const char *env = std::getenv("NPLBM_TARGET_BLOCKS");
    target = env ? std::atoi(env) : 2048;
    if (target <= 0) target = 2048;
  }
  // strips in x: widths in whole cache-line units, as equal as possible
  const int units = (nx + unit - 1) / unit;
  const int per_max = std::max(1, kTX / unit);
  const int nsx = (units + per_max - 1) / per_max;
  std::vector<int> xs(nsx + 1, 0);
  for (int sx = 0; sx < nsx; ++sx) {
    const int u = units / nsx + (sx < units % nsx ? 1 : 0);
    xs[sx + 1] = std::min(nx, xs[sx] + u * unit);
  }
  int nsy = std::max(1, target / nsx);
  int H = (ny + nsy - 1) / std::max(nsy, 1);
  int hmin = 16;
  if (const char *e = std::getenv("NPLBM_MIN_STRIP_H")) hmin = std::max(2, std::atoi(e));
  H = std::max(H, std::min(hmin, ny));
  H = (H + 1) & ~1;
  nsy = (ny + H - 1) / H;
  for (int sy = 0; sy < nsy; ++sy)
    for (int sx = 0; sx < nsx; ++sx) {
      StripDesc s;
      std::memset(&s, 0, sizeof s);
      s.dom = dom;
      s.x0 = xs[sx];
      s.x1 = xs[sx + 1];
      s.y0 = sy * H;
      s.y1 = std::min(ny, (sy + 1) * H);
      s.dir = (sy & 1) ? -1 : 1;
      out.push_back(s);
    }
}

// Reorder a strip list for the 8 XCDs of the chip: workgroup b is
// dispatched to XCD b % 8, so XCD x receives table entries x, x+8, x+16...
// Give each XCD a contiguous run of the (row-major) strip list, so that the
// halo columns and rows two strips share stay in one XCD's L2.
void xcd_order(std::vector<StripDesc> &s) {
  const int n = (int)s.size();
  if (n < 16) return;
  const int per = (n + 7) / 8;
  std::vector<StripDesc> out((size_t)per * 8);
  for (auto &e : out) {
    std::memset(&e, 0, sizeof e);
    e.dom = -1;
  }
  for (int i = 0; i < n; ++i) {
    const int g = i / per, j = i % per;
    out[(size_t)j * 8 + g] = s[i];
  }
  s.swap(out);
}

// Tile decomposition of a 3-D domain for the marching 3-D step kernel:
// tiles of 64 columns starting on multiples of 64 (the last one ragged) and
// at most ty rows, rows split as equally as possible, each marching
// through nz / nsz planes, nsz chosen so that the launch has about `target`
// workgroups; neighbouring z segments march in opposite directions.
void build_tiles3(int nx, int ny, int nz, int dom, int ty, int target,
                  std::vector<StripDesc> &out) {
  auto split = [](int n, int maxw, std::vector<int> &edges) {
    const int parts = (n + maxw - 1) / maxw;
    edges.assign(parts + 1, 0);
    for (int i = 0; i < parts; ++i) edges[i + 1] = edges[i] + n / parts + (i < n % parts ? 1 : 0);
  };
  std::vector<int> xs, ys;
  for (int x = 0; x < nx; x += 64) xs.push_back(x);
  xs.push_back(nx);
  split(ny, ty, ys);
  const int nxy = (int)((xs.size() - 1) * (ys.size() - 1));
  if (target <= 0) target = 1024;
  // z segments: the count that minimises the rounds of resident workgroups
  // times the planes one workgroup marches (its 4-plane ramp included),
  // with segments of at least 8 planes (or the whole depth).  Rounding the
  // count down instead (nxy tiles per segment against `target`) could leave
  // CUs idle: 192^3 N = 4 FP64 ran 144 workgroups on 256 CUs, at 29% of the
  // HBM roofline against 39% with 7 segments.
  const int hmin = std::min(nz, 8);
  int nsz = 1;
  double best = -1.0;
  for (int k = 1; k <= nz; ++k) {
    const int h = (nz + k - 1) / k;
    if (h < hmin) break;
    if ((nz + h - 1) / h != k) continue;  // the same segments as a smaller count
    const int64_t rounds = ((int64_t)nxy * k + target - 1) / target;
    const double t = (double)rounds * (h + 4);
    if (best < 0.0 || t < best) {
      best = t;
      nsz = k;
    }
  }
  const int H = (nz + nsz - 1) / nsz;
  nsz = (nz + H - 1) / H;
  for (int sz = 0; sz < nsz; ++sz)
    for (size_t iy = 0; iy + 1 < ys.size(); ++iy)
      for (size_t ix = 0; ix + 1 < xs.size(); ++ix) {
        TileDesc3 t;
        t.dom = dom;
        t.x0 = xs[ix];
        t.x1 = xs[ix + 1];
        t.y0 = ys[iy];
        t.y1 = ys[iy + 1];
        t.z0 = sz * H;
        t.z1 = std::min(nz, (sz + 1) * H);
        t.dir = (sz & 1) ? -1 : 1;
        StripDesc s;
        static_assert(sizeof s == sizeof t, "record sizes");
        std::memcpy(&s, &t, sizeof s);
        out.push_back(s);
      }
}

}  // namespace nplbm

// aux_kernels.hip -- initialisation, FP64 read-back of the macroscopic
// fields, FP64 conservation / Laplace reductions and a plain copy kernel.
// None of these run inside the time loop except the diagnostics, which the
// caller invokes every K steps.
#include <algorithm>
#include <mutex>

#include "lattice.h"
#include "nplbm_internal.h"

namespace nplbm {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int wrapi(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

// Neighbour (x + dx, y + dy) of a stencil: periodic in x; in y periodic or a
// mirror ghost beyond a wall.
__device__ __forceinline__ int64_t nb(int x, int y, int dx, int dy, int nx, int ny, bool wall) {
  int xx = wrapi(x + dx, nx);
  int yy = y + dy;
  if (wall) {
    if (yy < 0) yy = -1 - yy;
    if (yy >= ny) yy = 2 * ny - 1 - yy;
  } else {
    yy = wrapi(yy, ny);
  }
  return (int64_t)yy * nx + xx;
}

// Element offset of (plane p, row y, column x) in state group G.
__device__ __forceinline__ int64_t at(const DomDesc *dd, int G, int p, int y, int x) {
  return (int64_t)p * dd->ps[G] + (int64_t)y * dd->rs[G] + x;
}

// eq:N31b on a dense (ny x nx) double plane
__device__ __forceinline__ double lap9(const double *f, int x, int y, int nx, int ny, bool wall) {
  const double c = f[(int64_t)y * nx + x];
  const double ax = f[nb(x, y, 1, 0, nx, ny, wall)] + f[nb(x, y, -1, 0, nx, ny, wall)] +
                    f[nb(x, y, 0, 1, nx, ny, wall)] + f[nb(x, y, 0, -1, nx, ny, wall)];
  const double dg = f[nb(x, y, 1, 1, nx, ny, wall)] + f[nb(x, y, -1, 1, nx, ny, wall)] +
                    f[nb(x, y, 1, -1, nx, ny, wall)] + f[nb(x, y, -1, -1, nx, ny, wall)];
  return (4.0 * ax + dg - 20.0 * c) / 6.0;
}

// eq:N31a on a dense (ny x nx) double plane
__device__ __forceinline__ void grad9(const double *f, int x, int y, int nx, int ny, bool wall,
                                      double &gx, double &gy) {
  const double e = f[nb(x, y, 1, 0, nx, ny, wall)], w = f[nb(x, y, -1, 0, nx, ny, wall)];
  const double n = f[nb(x, y, 0, 1, nx, ny, wall)], s = f[nb(x, y, 0, -1, nx, ny, wall)];
  const double ne = f[nb(x, y, 1, 1, nx, ny, wall)], nw = f[nb(x, y, -1, 1, nx, ny, wall)];
  const double se = f[nb(x, y, 1, -1, nx, ny, wall)], sw = f[nb(x, y, -1, -1, nx, ny, wall)];
  gx = (4.0 * (e - w) + (ne - nw + se - sw)) / 12.0;
  gy = (4.0 * (n - s) + (ne + nw - se - sw)) / 12.0;
}

// eq:N40 (two-hop term read as negative) summed over the D2Q9 directions:
// d/dx = [24 (E - W) - 4 (E2 - W2) + 6 (NE - NW + SE - SW)
//         - (NE2 - NW2 + SE2 - SW2)] / 48, likewise d/dy.
__device__ __forceinline__ void grad_mixed(const double *f, int x, int y, int nx, int ny,
                                           bool wall, double &gx, double &gy) {
  auto v = [&](int dx, int dy) { return f[nb(x, y, dx, dy, nx, ny, wall)]; };
  gx = (24.0 * (v(1, 0) - v(-1, 0)) - 4.0 * (v(2, 0) - v(-2, 0)) +
        6.0 * ((v(1, 1) - v(-1, 1)) + (v(1, -1) - v(-1, -1))) -
        ((v(2, 2) - v(-2, 2)) + (v(2, -2) - v(-2, -2)))) /
       48.0;
  gy = (24.0 * (v(0, 1) - v(0, -1)) - 4.0 * (v(0, 2) - v(0, -2)) +
        6.0 * ((v(1, 1) + v(-1, 1)) - (v(1, -1) + v(-1, -1))) -
        ((v(2, 2) + v(-2, 2)) - (v(2, -2) + v(-2, -2)))) /
       48.0;
}

// ---------------------------------------------------------------- init ----
// phi_i from the volume fractions: eq:N12 inverted with rho_k = rho~_k c_k,
// phi_i = (rho~_i c_i - rho~_N c_N - b_i) / a_i, which the host passes as
// phi_i = P1[i] c_i + PN[i] c_N + P0[i].
struct PhiMap {
  double P1[kMaxM], PN[kMaxM], P0[kMaxM];
};

__global__ void k_init_phi(PhiMap pm, int M, const double *c, double *phi, int64_t n) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const double cN = c[(int64_t)M * n + id];
  for (int i = 0; i < M; ++i)
    phi[(int64_t)i * n + id] = pm.P1[i] * c[(int64_t)i * n + id] + pm.PN[i] * cN + pm.P0[i];
}

// C_i from phi (eq:N18 line 3 with eq:N17), dense planes
__global__ void k_chem(const DomDesc *dd, int M, const double *phi, double *C) {
  const int nx = dd->nx, ny = dd->ny;
  const int64_t n = (int64_t)nx * ny;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int x = (int)(id % nx), y = (int)(id / nx);
  const bool wall = dd->wall != 0;
  const Consts<double> &K = dd->cd;
  const int N = M + 1;
  double ph[kMaxM], lp[kMaxM], wv[kMaxN];
  for (int i = 0; i < M; ++i) {
    ph[i] = phi[(int64_t)i * n + id];
    lp[i] = lap9(phi + (int64_t)i * n, x, y, nx, ny, wall);
  }
  for (int k = 0; k < N; ++k) {
    double ck = K.ca[k];
    for (int i = 0; i < M; ++i) ck += K.cA[k][i] * ph[i];
    wv[k] = ck * (1.0 - ck) * (1.0 - 2.0 * ck);
  }
  for (int i = 0; i < M; ++i) {
    double Ci = 0.0;
    for (int j = 0; j < M; ++j) Ci -= K.lam[i][j] * lp[j];
    for (int k = 0; k < N; ++k) Ci += K.KH[k][i] * wv[k];
    C[(int64_t)i * n + id] = Ci;
  }
}

// Equilibria (eq:25 with p = 0, eq:N25) written in pull layout: the value
// that node x must pull in direction k is stored where the step kernel
// reads it, i.e. at x - c_k, or in the opposite direction at x itself when
// x - c_k lies beyond a wall.  The k = 0 slot holds the deviation of h_0
// from the stored phi (prev), as the step kernel expects.
template <typename Real>
__global__ void k_init_dist(const DomDesc *dd, int M, const double *phi, const double *C,
                            const double *u) {
  const int nx = dd->nx, ny = dd->ny, pitch = dd->pitch;
  const int64_t n = (int64_t)nx * ny;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int x = (int)(id % nx), y = (int)(id / nx);
  const bool wall = dd->wall != 0;
  const Consts<double> &K = dd->cd;
  Real *h = static_cast<Real *>(dd->h[dd->parity0]);
  Real *g = static_cast<Real *>(dd->g[dd->parity0]);
  Real *pv = static_cast<Real *>(dd->prev[dd->parity0]);
  const double ux = u ? u[id] : 0.0, uy = u ? u[n + id] : 0.0;
  double rho = K.ra;
  for (int i = 0; i < M; ++i) rho += K.rA[i] * phi[(int64_t)i * n + id];
  const double usq = ux * ux + uy * uy;
  for (int k = 0; k < 9; ++k) {
    const int cx = cxk(k), cy = cyk(k);
    int ys = y - cy, xs = wrapi(x - cx, nx);
    int kk = k;
    if (wall && (ys < 0 || ys >= ny)) {
      kk = oppk(k);
      ys = y;
      xs = x;
    } else {
      ys = wrapi(ys, ny);
    }
    const double w = wk<double>(k);
    const double cu = cx * ux + cy * uy;
    for (int i = 0; i < M; ++i) {
      const double ph = phi[(int64_t)i * n + id], Ci = C[(int64_t)i * n + id];
      const double ec = K.eta_i[i] * Ci;
      // k = 0: h_0^eq - phi_stored with phi_stored = (Real)phi
      const double v = (k == 0) ? (ph - (double)(Real)ph) + (w - 1.0) * ec
                                : w * ec + w * 3.0 * (cx * ph * ux + cy * ph * uy);
      h[at(dd, 0, i * 9 + kk, ys, xs)] = (Real)v;
    }
    if (k > 0) {
      const double v = rho * w * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq);  // p = 0
      g[at(dd, 1, kk - 1, ys, xs)] = (Real)v;
    }
  }
  for (int i = 0; i < M; ++i) pv[at(dd, 2, i, y, x)] = (Real)phi[(int64_t)i * n + id];
  pv[at(dd, 2, M, y, x)] = (Real)ux;
  pv[at(dd, 2, M + 1, y, x)] = (Real)uy;
}

// --------------------------------------------------------------- macro ----
// phi (pull + eq:N28), c_k, rho in FP64 from the stored populations
template <typename Real>
__global__ void k_macro_phi(const DomDesc *dd, int M, int parity, double *phi, double *rho,
                            double *cout) {
  const int nx = dd->nx, ny = dd->ny, pitch = dd->pitch;
  const int64_t n = (int64_t)nx * ny;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int x = (int)(id % nx), y = (int)(id / nx);
  const bool wall = dd->wall != 0;
  const Real *h = static_cast<const Real *>(dd->h[parity]);
  const Real *pv = static_cast<const Real *>(dd->prev[parity]);
  const Consts<double> &K = dd->cd;
  const int N = M + 1;
  double ph[kMaxM];
  // phi_i = phi_prev + (h_0 - phi_prev) + sum_{k>=1} h_k (eq:N28)
  for (int i = 0; i < M; ++i) ph[i] = (double)pv[at(dd, 2, i, y, x)];
  for (int k = 0; k < 9; ++k) {
    const int cx = cxk(k), cy = cyk(k);
    int ys = y - cy, xs = wrapi(x - cx, nx);
    int kk = k;
    if (wall && (ys < 0 || ys >= ny)) {
      kk = oppk(k);
      ys = y;
      xs = x;
    } else {
      ys = wrapi(ys, ny);
    }
    for (int i = 0; i < M; ++i) ph[i] += (double)h[at(dd, 0, i * 9 + kk, ys, xs)];
  }
  double r = K.ra;
  for (int i = 0; i < M; ++i) {
    phi[(int64_t)i * n + id] = ph[i];
    r += K.rA[i] * ph[i];
  }
  rho[id] = r;
  if (cout)
    for (int k = 0; k < N; ++k) {
      double ck = K.ca[k];
      for (int i = 0; i < M; ++i) ck += K.cA[k][i] * ph[i];
      cout[(int64_t)k * n + id] = ck;
    }
}

// Remark 1 (Sec. 3.1): the products J~_b u_a, J~ from the eq:N31a
// gradients of C (eq:N18 line 4) and u the stored velocity of the previous
// step; planes q[0..3] = J~_x u_x, J~_y u_x, J~_x u_y, J~_y u_y.
template <typename Real>
__global__ void k_macro_q(const DomDesc *dd, int M, int parity, const double *C, double *q) {
  const int nx = dd->nx, ny = dd->ny;
  const int64_t n = (int64_t)nx * ny;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int x = (int)(id % nx), y = (int)(id / nx);
  const bool wall = dd->wall != 0;
  const Real *pv = static_cast<const Real *>(dd->prev[parity]);
  const Consts<double> &K = dd->cd;
  double Jx = 0.0, Jy = 0.0;
  for (int i = 0; i < M; ++i) {
    double gx, gy;
    grad9(C + (int64_t)i * n, x, y, nx, ny, wall, gx, gy);
    Jx += K.Jc[i] * gx;
    Jy += K.Jc[i] * gy;
  }
  const double ux = (double)pv[at(dd, 2, M, y, x)], uy = (double)pv[at(dd, 2, M + 1, y, x)];
  q[id] = Jx * ux;
  q[n + id] = Jy * ux;
  q[2 * n + id] = Jx * uy;
  q[3 * n + id] = Jy * uy;
}

// u (eq:N22_1) and p (eq:N23) in FP64; with q non-null the force also
// carries -div(J~ u) of Remark 1, component a = sum_b d_b q(b, a)
template <typename Real>
__global__ void k_macro_up(const DomDesc *dd, int M, int parity, const double *phi,
                           const double *rho, const double *C, const double *q, double *uout,
                           double *pout) {
  const int nx = dd->nx, ny = dd->ny, pitch = dd->pitch;
  const int64_t n = (int64_t)nx * ny;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int x = (int)(id % nx), y = (int)(id / nx);
  const bool wall = dd->wall != 0;
  const Real *g = static_cast<const Real *>(dd->g[parity]);
  const Consts<double> &K = dd->cd;
  double Fx = 0.0, Fy = 0.0, grx = 0.0, gry = 0.0;
  for (int i = 0; i < M; ++i) {
    double gx, gy;
    if (dd->scheme == kSchemeMixed)
      grad_mixed(phi + (int64_t)i * n, x, y, nx, ny, wall, gx, gy);
    else
      grad9(phi + (int64_t)i * n, x, y, nx, ny, wall, gx, gy);
    const double Ci = C[(int64_t)i * n + id];
    Fx += Ci * gx;
    Fy += Ci * gy;
    grx += K.rA[i] * gx;
    gry += K.rA[i] * gy;
  }
  const double r = rho[id];
  Fx += r * K.gx;
  Fy += r * K.gy;
  if (q) {
    double axx, axy, ayx, ayy, bxx, bxy, byx, byy;
    grad9(q, x, y, nx, ny, wall, axx, axy);
    grad9(q + n, x, y, nx, ny, wall, ayx, ayy);
    grad9(q + 2 * n, x, y, nx, ny, wall, bxx, bxy);
    grad9(q + 3 * n, x, y, nx, ny, wall, byx, byy);
    Fx -= axx + ayy;
    Fy -= bxx + byy;
  }
  double gk[9];
  gk[0] = 0.0;
  for (int k = 1; k < 9; ++k) {
    const int cx = cxk(k), cy = cyk(k);
    int ys = y - cy, xs = wrapi(x - cx, nx);
    int kk = k;
    if (wall && (ys < 0 || ys >= ny)) {
      kk = oppk(k);
      ys = y;
      xs = x;
    } else {
      ys = wrapi(ys, ny);
    }
    gk[k] = (double)g[at(dd, 1, kk - 1, ys, xs)];
  }
  double mx = 0.0, my = 0.0, sg = 0.0;
  for (int k = 1; k < 9; ++k) {
    mx += cxk(k) * gk[k];
    my += cyk(k) * gk[k];
    sg += gk[k];
  }
  const double ux = (mx + 0.5 * Fx) / r, uy = (my + 0.5 * Fy) / r;
  if (uout) {
    uout[id] = ux;
    uout[n + id] = uy;
  }
  if (pout) pout[id] = 0.6 * (sg + 0.5 * (ux * grx + uy * gry) - (2.0 / 3.0) * r * (ux * ux + uy * uy));
}

// ---------------------------------------------------------- reductions ----
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Per-block partial sums of each c_k, max |sum_k c_k - 1| and non-finite
// count; a block strides over the field so the result does not depend on
// scheduling.  partials[b * (N + 2) + q].
__global__ void k_diag_partial(const double *c, int N, int64_t n, double *partials) {
  __shared__ double red[kThreads / 64][kMaxN + 2];
  double acc[kMaxN + 2];
  for (int q = 0; q < N + 2; ++q) acc[q] = 0.0;
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n;
       id += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    bool bad = false;
    for (int k = 0; k < N; ++k) {
      const double v = c[(int64_t)k * n + id];
      bad |= !isfinite(v);
      acc[k] += v;
      s += v;
    }
    acc[N] = fmax(acc[N], fabs(s - 1.0));
    acc[N + 1] += bad ? 1.0 : 0.0;
  }
  const int wv = threadIdx.x / 64, ln = threadIdx.x & 63;
  for (int q = 0; q < N + 2; ++q) {
    const double r = (q == N) ? wave_max(acc[q]) : wave_sum(acc[q]);
    if (ln == 0) red[wv][q] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < N + 2; ++q) {
      double r = red[0][q];
      for (int w = 1; w < kThreads / 64; ++w) r = (q == N) ? fmax(r, red[w][q]) : r + red[w][q];
      partials[(int64_t)blockIdx.x * (N + 2) + q] = r;
    }
  }
}

// entry qmax of each partial record is a maximum, the others are sums
__global__ void k_diag_final(const double *partials, int nq, int nblk, int qmax, double *out) {
  const int q = threadIdx.x;
  if (q >= nq) return;
  double r = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double v = partials[(int64_t)b * nq + q];
    r = q == qmax ? fmax(r, v) : r + v;
  }
  out[q] = r;
}

// Laplace: sums and counts of p inside r <= r_in and outside r >= r_out
__global__ void k_laplace_partial(const double *p, int nx, int ny, int nz, double xc, double yc,
                                  double zc, double r_in, double r_out, double *partials) {
  __shared__ double red[kThreads / 64][4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t n = (int64_t)nx * ny * nz;
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n;
       id += (int64_t)gridDim.x * blockDim.x) {
    const double x = (double)(id % nx), y = (double)((id / nx) % ny),
                 z = (double)(id / ((int64_t)nx * ny));
    const double r = sqrt((x - xc) * (x - xc) + (y - yc) * (y - yc) + (z - zc) * (z - zc));
    if (r <= r_in) {
      acc[0] += p[id];
      acc[1] += 1.0;
    } else if (r >= r_out) {
      acc[2] += p[id];
      acc[3] += 1.0;
    }
  }
  const int wv = threadIdx.x / 64, ln = threadIdx.x & 63;
  for (int q = 0; q < 4; ++q) {
    const double r = wave_sum(acc[q]);
    if (ln == 0) red[wv][q] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) {
      double r = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) r += red[w][q];
      partials[(int64_t)blockIdx.x * 4 + q] = r;
    }
}

__global__ void k_laplace_final(const double *partials, int nblk, double *out) {
  if (threadIdx.x != 0) return;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < nblk; ++b)
    for (int q = 0; q < 4; ++q) a[q] += partials[(int64_t)b * 4 + q];
  out[0] = (a[1] > 0.0 && a[3] > 0.0) ? a[0] / a[1] - a[2] / a[3] : 0.0;
}

// one 16-byte element per thread and a grid covering the buffer: the
// fastest plain copy pattern measured on gfx950 (~6.2 TB/s read + write)
__global__ void k_copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src, int64_t n16) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

__global__ void k_copy1(unsigned char *dst, const unsigned char *src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

static int blocks_for(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

hipError_t launch_init(const DomDesc *dd_dev, const DomDesc &dd, int precision,
                       const double *P1, const double *PN, const double *P0,
                       const double *c_dev, const double *u_dev, double *phi_tmp,
                       double *C_tmp, hipStream_t st) {
  const int M = dd.N - 1;
  const int64_t n = (int64_t)dd.nx * dd.ny;
  PhiMap pm;
  for (int i = 0; i < kMaxM; ++i) {
    pm.P1[i] = i < M ? P1[i] : 0.0;
    pm.PN[i] = i < M ? PN[i] : 0.0;
    pm.P0[i] = i < M ? P0[i] : 0.0;
  }
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_init_phi, dim3(nb), dim3(kThreads), 0, st, pm, M, c_dev, phi_tmp, n);
  hipLaunchKernelGGL(k_chem, dim3(nb), dim3(kThreads), 0, st, dd_dev, M, phi_tmp, C_tmp);
  if (precision == 64)
    hipLaunchKernelGGL(k_init_dist<double>, dim3(nb), dim3(kThreads), 0, st, dd_dev, M,
                       phi_tmp, C_tmp, u_dev);
  else
    hipLaunchKernelGGL(k_init_dist<float>, dim3(nb), dim3(kThreads), 0, st, dd_dev, M,
                       phi_tmp, C_tmp, u_dev);
  return hipGetLastError();
}

hipError_t launch_macro(const DomDesc *dd_dev, const DomDesc &dd, int precision, int parity,
                        double *phi, double *rho, double *C, double *c_out, double *u_out,
                        double *p_out, double *q, hipStream_t st) {
  const int M = dd.N - 1;
  const int64_t n = (int64_t)dd.nx * dd.ny;
  const int nb = blocks_for(n);
  if (precision == 64)
    hipLaunchKernelGGL(k_macro_phi<double>, dim3(nb), dim3(kThreads), 0, st, dd_dev, M, parity,
                       phi, rho, c_out);
  else
    hipLaunchKernelGGL(k_macro_phi<float>, dim3(nb), dim3(kThreads), 0, st, dd_dev, M, parity,
                       phi, rho, c_out);
  if (!u_out && !p_out) return hipGetLastError();
  hipLaunchKernelGGL(k_chem, dim3(nb), dim3(kThreads), 0, st, dd_dev, M, phi, C);
  const double *qq = dd.scheme == kSchemeRemark1 ? q : nullptr;
  if (dd.scheme == kSchemeRemark1) {
    if (!q) return hipErrorInvalidValue;
    if (precision == 64)
      hipLaunchKernelGGL(k_macro_q<double>, dim3(nb), dim3(kThreads), 0, st, dd_dev, M, parity,
                         C, q);
    else
      hipLaunchKernelGGL(k_macro_q<float>, dim3(nb), dim3(kThreads), 0, st, dd_dev, M, parity,
                         C, q);
  }
  if (precision == 64)
    hipLaunchKernelGGL(k_macro_up<double>, dim3(nb), dim3(kThreads), 0, st, dd_dev, M, parity,
                       phi, rho, C, qq, u_out, p_out);
  else
    hipLaunchKernelGGL(k_macro_up<float>, dim3(nb), dim3(kThreads), 0, st, dd_dev, M, parity,
                       phi, rho, C, qq, u_out, p_out);
  return hipGetLastError();
}

// ---- the static scratch of nplbm_diagnostics_noalloc ----
// Partial records of the diagnostics reduction (at most diag_blocks() = 1024
// blocks of N + 2 doubles) followed by room for the final record, in a
// file-scope device array so that the entry point allocates nothing.  Each
// GPU holds its own copy until the process ends.  In host code `scratch`
// names a host-side stand-in, not device memory: kernels and copies get the
// per-device address hipGetSymbolAddress returns (static_diag_scratch).
static __device__ __align__(256) double scratch[kStaticDiagDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {nullptr};
}  // namespace

hipError_t static_diag_scratch(double **out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    // once per device, with that device current
    double *ptr = nullptr;
    e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

int diag_blocks(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_diag(const double *c, int N, int64_t n, double *partials, int nblk,
                       double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_partial, dim3(nblk), dim3(kThreads), 0, st, c, N, n, partials);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, st, partials, N + 2, nblk, N, out);
  return hipGetLastError();
}

hipError_t launch_laplace(const double *p, int nx, int ny, int nz, double xc, double yc,
                          double zc, double r_in, double r_out, double *partials, int nblk,
                          double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_laplace_partial, dim3(nblk), dim3(kThreads), 0, st, p, nx, ny, nz, xc, yc,
                     zc, r_in, r_out, partials);
  hipLaunchKernelGGL(k_laplace_final, dim3(1), dim3(64), 0, st, partials, nblk, out);
  return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t nbytes, hipStream_t st) {
  const bool aligned = (((uintptr_t)dst | (uintptr_t)src) & 15) == 0;
  const int64_t n16 = aligned ? (int64_t)(nbytes / 16) : 0;
  for (int64_t done = 0; done < n16;) {  // chunks of at most 2^30 elements
    const int64_t cnt = std::min<int64_t>(n16 - done, (int64_t)1 << 30);
    const int64_t nb = (cnt + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)nb), dim3(kThreads), 0, st,
                       static_cast<uint4 *>(dst) + done, static_cast<const uint4 *>(src) + done,
                       cnt);
    done += cnt;
  }
  const int64_t rest = (int64_t)nbytes - n16 * 16;
  if (rest > 0)
    hipLaunchKernelGGL(k_copy1, dim3((unsigned)((rest + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, st, static_cast<unsigned char *>(dst) + n16 * 16,
                       static_cast<const unsigned char *>(src) + n16 * 16, rest);
  return hipGetLastError();
}

}  // namespace nplbm

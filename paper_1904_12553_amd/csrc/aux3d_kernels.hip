// aux3d_kernels.hip -- initialisation and FP64 read-back of 3-D (D3Q15)
// domains: the counterparts of the 2-D kernels in aux_kernels.hip, one thread
// per node on dense (nz x ny x nx) FP64 planes.  Not in the time loop.
#include "lattice3.h"
#include "nplbm_internal.h"

namespace nplbm {

namespace {

constexpr int kT3 = 256;

__device__ __forceinline__ int wrap3i(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

struct Geo3 {
  int nx, ny, nz;
  bool wall;
};

// dense index of (x + dx, y + dy, z + dz): periodic in x and y; in z
// periodic or a mirror ghost beyond a wall
__device__ __forceinline__ int64_t nb3(const Geo3 &g, int x, int y, int z, int dx, int dy,
                                       int dz) {
  const int xx = wrap3i(x + dx, g.nx), yy = wrap3i(y + dy, g.ny);
  int zz = z + dz;
  if (g.wall) {
    if (zz < 0) zz = -1 - zz;
    if (zz >= g.nz) zz = 2 * g.nz - 1 - zz;
  } else {
    zz = wrap3i(zz, g.nz);
  }
  return ((int64_t)zz * g.ny + yy) * g.nx + xx;
}

// eq:N31b and eq:N31a on D3Q15, summed over the velocities
__device__ __forceinline__ double lap3d(const double *f, const Geo3 &g, int x, int y, int z) {
  const double c = f[((int64_t)z * g.ny + y) * g.nx + x];
  double a = 0.0;
  for (int k = 1; k < 15; ++k)
    a += w3<double>(k) * (f[nb3(g, x, y, z, ex3(k), ey3(k), ez3(k))] - c);
  return 2.0 * a * 3.0;
}
__device__ __forceinline__ void grad3d(const double *f, const Geo3 &g, int x, int y, int z,
                                       double *out) {
  double a[3] = {0.0, 0.0, 0.0};
  for (int k = 1; k < 15; ++k) {
    const double v = f[nb3(g, x, y, z, ex3(k), ey3(k), ez3(k))];
    a[0] += w3<double>(k) * ex3(k) * v;
    a[1] += w3<double>(k) * ey3(k) * v;
    a[2] += w3<double>(k) * ez3(k) * v;
  }
  for (int d = 0; d < 3; ++d) out[d] = 3.0 * a[d];
}

__device__ __forceinline__ int64_t at3(const DomDesc *dd, int G, int p, int z, int y, int x) {
  return (int64_t)p * dd->ps[G] + ((int64_t)z * dd->ny + y) * dd->rs[G] + x;
}

struct PhiMap3 {
  double P1[kMaxM], PN[kMaxM], P0[kMaxM];
};

__global__ void k3_init_phi(PhiMap3 pm, int M, const double *c, double *phi, int64_t n) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const double cN = c[(int64_t)M * n + id];
  for (int i = 0; i < M; ++i)
    phi[(int64_t)i * n + id] = pm.P1[i] * c[(int64_t)i * n + id] + pm.PN[i] * cN + pm.P0[i];
}

// C_i from phi (eq:N18 line 3 with eq:N17)
__global__ void k3_chem(const DomDesc *dd, int M, const double *phi, double *C) {
  const Geo3 g{dd->nx, dd->ny, dd->nz, dd->wall != 0};
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int x = (int)(id % g.nx), y = (int)((id / g.nx) % g.ny), z = (int)(id / ((int64_t)g.nx * g.ny));
  const Consts<double> &K = dd->cd;
  const int N = M + 1;
  double ph[kMaxM], lp[kMaxM], wv[kMaxN];
  for (int i = 0; i < M; ++i) {
    ph[i] = phi[(int64_t)i * n + id];
    lp[i] = lap3d(phi + (int64_t)i * n, g, x, y, z);
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

// equilibria with p = 0 (eq:25, eq:N25) in pull layout: stored where the
// step kernel reads the population arriving at this node (at x - c_k, or
// in the opposite direction at the node itself across a wall); the k = 0
// slot holds h_0 - phi_stored
template <typename Real>
__global__ void k3_init_dist(const DomDesc *dd, int M, const double *phi, const double *C,
                             const double *u) {
  const Geo3 gg{dd->nx, dd->ny, dd->nz, dd->wall != 0};
  const int64_t n = (int64_t)gg.nx * gg.ny * gg.nz;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int x = (int)(id % gg.nx), y = (int)((id / gg.nx) % gg.ny),
            z = (int)(id / ((int64_t)gg.nx * gg.ny));
  const Consts<double> &K = dd->cd;
  Real *h = static_cast<Real *>(dd->h[dd->parity0]);
  Real *g = static_cast<Real *>(dd->g[dd->parity0]);
  Real *pv = static_cast<Real *>(dd->prev[dd->parity0]);
  double uu[3];
  for (int d = 0; d < 3; ++d) uu[d] = u ? u[(int64_t)d * n + id] : 0.0;
  double rho = K.ra;
  for (int i = 0; i < M; ++i) rho += K.rA[i] * phi[(int64_t)i * n + id];
  const double usq = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
  for (int k = 0; k < 15; ++k) {
    const int cx = ex3(k), cy = ey3(k), cz = ez3(k);
    int zs = z - cz, ys = wrap3i(y - cy, gg.ny), xs = wrap3i(x - cx, gg.nx);
    int kk = k;
    if (gg.wall && (zs < 0 || zs >= gg.nz)) {
      kk = opp3(k);
      zs = z;
      ys = y;
      xs = x;
    } else {
      zs = wrap3i(zs, gg.nz);
    }
    const double w = w3<double>(k);
    const double cu = cx * uu[0] + cy * uu[1] + cz * uu[2];
    for (int i = 0; i < M; ++i) {
      const double ph = phi[(int64_t)i * n + id], ec = K.eta_i[i] * C[(int64_t)i * n + id];
      const double v = (k == 0) ? (ph - (double)(Real)ph) + (w - 1.0) * ec
                                : w * ec + w * 3.0 * ph * cu;
      h[at3(dd, 0, i * 15 + kk, zs, ys, xs)] = (Real)v;
    }
    if (k > 0) g[at3(dd, 1, kk - 1, zs, ys, xs)] = (Real)(rho * w * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
  }
  for (int i = 0; i < M; ++i) pv[at3(dd, 2, i, z, y, x)] = (Real)phi[(int64_t)i * n + id];
  for (int d = 0; d < 3; ++d) pv[at3(dd, 2, M + d, z, y, x)] = (Real)uu[d];
}

// population k arriving at (x, y, z) in the pull layout: its stored location
struct Pull3 {
  int kk, zs, ys, xs;
};
__device__ __forceinline__ Pull3 pull3(const Geo3 &g, int k, int x, int y, int z) {
  Pull3 p{k, z - ez3(k), wrap3i(y - ey3(k), g.ny), wrap3i(x - ex3(k), g.nx)};
  if (g.wall && (p.zs < 0 || p.zs >= g.nz)) {
    p.kk = opp3(k);
    p.zs = z;
    p.ys = y;
    p.xs = x;
  } else {
    p.zs = wrap3i(p.zs, g.nz);
  }
  return p;
}

// phi (eq:N28 on the stored state), rho and c_k in FP64
template <typename Real>
__global__ void k3_macro_phi(const DomDesc *dd, int M, int parity, double *phi, double *rho,
                             double *cout) {
  const Geo3 g{dd->nx, dd->ny, dd->nz, dd->wall != 0};
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int x = (int)(id % g.nx), y = (int)((id / g.nx) % g.ny), z = (int)(id / ((int64_t)g.nx * g.ny));
  const Real *h = static_cast<const Real *>(dd->h[parity]);
  const Real *pv = static_cast<const Real *>(dd->prev[parity]);
  const Consts<double> &K = dd->cd;
  double ph[kMaxM];
  for (int i = 0; i < M; ++i) ph[i] = (double)pv[at3(dd, 2, i, z, y, x)];
  for (int k = 0; k < 15; ++k) {
    const Pull3 p = pull3(g, k, x, y, z);
    for (int i = 0; i < M; ++i) ph[i] += (double)h[at3(dd, 0, i * 15 + p.kk, p.zs, p.ys, p.xs)];
  }
  double r = K.ra;
  for (int i = 0; i < M; ++i) {
    phi[(int64_t)i * n + id] = ph[i];
    r += K.rA[i] * ph[i];
  }
  rho[id] = r;
  if (cout)
    for (int k = 0; k < M + 1; ++k) {
      double ck = K.ca[k];
      for (int i = 0; i < M; ++i) ck += K.cA[k][i] * ph[i];
      cout[(int64_t)k * n + id] = ck;
    }
}

// u (eq:N22_1) and p (eq:N23 with the D3Q15 rest weight) in FP64
template <typename Real>
__global__ void k3_macro_up(const DomDesc *dd, int M, int parity, const double *phi,
                            const double *rho, const double *C, double *uout, double *pout) {
  const Geo3 g{dd->nx, dd->ny, dd->nz, dd->wall != 0};
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int x = (int)(id % g.nx), y = (int)((id / g.nx) % g.ny), z = (int)(id / ((int64_t)g.nx * g.ny));
  const Real *gp = static_cast<const Real *>(dd->g[parity]);
  const Consts<double> &K = dd->cd;
  double F[3] = {0.0, 0.0, 0.0}, gr[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < M; ++i) {
    double gv[3];
    grad3d(phi + (int64_t)i * n, g, x, y, z, gv);
    const double Ci = C[(int64_t)i * n + id];
    for (int d = 0; d < 3; ++d) {
      F[d] += Ci * gv[d];
      gr[d] += K.rA[i] * gv[d];
    }
  }
  const double r = rho[id];
  F[0] += r * K.gx;
  F[1] += r * K.gy;
  F[2] += r * K.gz;
  double m[3] = {0.0, 0.0, 0.0}, sg = 0.0;
  for (int k = 1; k < 15; ++k) {
    const Pull3 p = pull3(g, k, x, y, z);
    const double v = (double)gp[at3(dd, 1, p.kk - 1, p.zs, p.ys, p.xs)];
    m[0] += ex3(k) * v;
    m[1] += ey3(k) * v;
    m[2] += ez3(k) * v;
    sg += v;
  }
  double u[3], usq = 0.0, udr = 0.0;
  for (int d = 0; d < 3; ++d) {
    u[d] = (m[d] + 0.5 * F[d]) / r;
    usq += u[d] * u[d];
    udr += u[d] * gr[d];
  }
  if (uout)
    for (int d = 0; d < 3; ++d) uout[(int64_t)d * n + id] = u[d];
  if (pout) pout[id] = 3.0 / 7.0 * (sg + 0.5 * udr - r * usq / 3.0);
}

int nb3blocks(int64_t n) { return (int)((n + kT3 - 1) / kT3); }

}  // namespace

hipError_t launch_init3(const DomDesc *dd_dev, const DomDesc &dd, int precision,
                        const double *P1, const double *PN, const double *P0,
                        const double *c_dev, const double *u_dev, double *phi_tmp,
                        double *C_tmp, hipStream_t st) {
  const int M = dd.N - 1;
  const int64_t n = (int64_t)dd.nx * dd.ny * dd.nz;
  PhiMap3 pm;
  for (int i = 0; i < kMaxM; ++i) {
    pm.P1[i] = i < M ? P1[i] : 0.0;
    pm.PN[i] = i < M ? PN[i] : 0.0;
    pm.P0[i] = i < M ? P0[i] : 0.0;
  }
  const int nb = nb3blocks(n);
  hipLaunchKernelGGL(k3_init_phi, dim3(nb), dim3(kT3), 0, st, pm, M, c_dev, phi_tmp, n);
  hipLaunchKernelGGL(k3_chem, dim3(nb), dim3(kT3), 0, st, dd_dev, M, phi_tmp, C_tmp);
  if (precision == 64)
    hipLaunchKernelGGL(k3_init_dist<double>, dim3(nb), dim3(kT3), 0, st, dd_dev, M, phi_tmp,
                       C_tmp, u_dev);
  else
    hipLaunchKernelGGL(k3_init_dist<float>, dim3(nb), dim3(kT3), 0, st, dd_dev, M, phi_tmp,
                       C_tmp, u_dev);
  return hipGetLastError();
}

hipError_t launch_macro3(const DomDesc *dd_dev, const DomDesc &dd, int precision, int parity,
                         double *phi, double *rho, double *C, double *c_out, double *u_out,
                         double *p_out, hipStream_t st) {
  const int M = dd.N - 1;
  const int64_t n = (int64_t)dd.nx * dd.ny * dd.nz;
  const int nb = nb3blocks(n);
  if (precision == 64)
    hipLaunchKernelGGL(k3_macro_phi<double>, dim3(nb), dim3(kT3), 0, st, dd_dev, M, parity, phi,
                       rho, c_out);
  else
    hipLaunchKernelGGL(k3_macro_phi<float>, dim3(nb), dim3(kT3), 0, st, dd_dev, M, parity, phi,
                       rho, c_out);
  if (!u_out && !p_out) return hipGetLastError();
  hipLaunchKernelGGL(k3_chem, dim3(nb), dim3(kT3), 0, st, dd_dev, M, phi, C);
  if (precision == 64)
    hipLaunchKernelGGL(k3_macro_up<double>, dim3(nb), dim3(kT3), 0, st, dd_dev, M, parity, phi,
                       rho, C, u_out, p_out);
  else
    hipLaunchKernelGGL(k3_macro_up<float>, dim3(nb), dim3(kT3), 0, st, dd_dev, M, parity, phi,
                       rho, C, u_out, p_out);
  return hipGetLastError();
}

}  // namespace nplbm

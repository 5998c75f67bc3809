// step_kernel.hip -- the fused time step of the N-phase phase-field LB model
// (arXiv:1904.12553, Sec. 3) for gfx950.
//
// One launch advances every node of every listed domain by one time step.
// Work decomposition: a workgroup owns a strip of kTX interior columns and
// [y0, y1) rows and marches along y, two rows per iteration (one wave per
// row, 64 lanes = kTX interior columns + a 2-column halo on each side).
// Per iteration, with march index m counted from the strip start:
//
//   stage A (rows m, m+1 ahead by 2): pull the 9(N-1) CH populations from
//            the neighbours (streaming fused into the load), phi_i = sum_k h
//            (eq:N28) -> LDS ring of 8 rows;
//   stage B (1 row behind A): Laplacian of eq:N31b on the LDS ring, closure
//            eq:N18 and eq:N17 -> chemical potentials C_i -> LDS ring of 4;
//   stage C (2 rows behind A): gradients of phi_i and C_i (eq:N31a) from the
//            rings, forces F (Sec. 3.1) and J~, pull the 8 moving NS
//            populations, u (eq:N22_1), p (eq:N23), NS collision (eq:24 with
//            eq:25 and eq:N20_1) and CH collisions (eq:N24 with eq:N25-N27)
//            using the CH populations this thread pulled one iteration
//            earlier (kept in registers), then store.
//
// So every population is read from HBM once and written once per step; the
// only re-reads are the 2-column x-halo and a 4-row ramp at the strip start,
// both L2/MALL-resident.  Rest populations are dropped or stored as
// deviations from their rest-state value:
//   - g_0 never feeds u, p or phi (c_0 = 0 and eq:N23 sums k != 0), so only
//     g_1..g_8 are stored; at rest (p = 0, u = 0) their equilibria are 0, so
//     they are already deviations;
//   - the rest population h_0 carries the O(1) order parameter.  The
//     collision conserves sum_k h_k = phi_i, so the stored k = 0 value is the
//     deviation d_i = h_0 - phi_i(prev) of h_0 from the rest value phi_i,
//     with phi_i(prev) the rounded phi_i the same node stores for the source
//     term (eq:N27).  phi_i is then carried as an unevaluated sum
//     hi + lo = phi_prev + (d + sum_{k>=1} h_k) and never rounded to one
//     storage word, so in FP32 the state keeps ~1e-11 absolute resolution on
//     phi instead of ~6e-8.
//
// Boundaries: x periodic; y periodic or halfway bounce-back walls (a
// population that would be pulled from outside is the node's own opposite
// post-collision population), with mirror ghost rows for the phi and C
// stencils next to a wall.
#include "lattice.h"
#include "nplbm_internal.h"

namespace nplbm {

template <typename Real>
__device__ __forceinline__ const Consts<Real> &consts_of(const DomDesc *d);
template <>
__device__ __forceinline__ const Consts<double> &consts_of<double>(const DomDesc *d) {
  return d->cd;
}
template <>
__device__ __forceinline__ const Consts<float> &consts_of<float>(const DomDesc *d) {
  return d->cf;
}

template <int N, typename Real>
__global__ void __launch_bounds__(kStepThreads) k_step(StepArgs a) {
  constexpr int M = N - 1;
  const StripDesc sd = a.strips[blockIdx.x];
  if (sd.dom < 0) return;
  const DomDesc *D = a.doms + sd.dom;
  if (a.substep >= D->steps_left) return;
  const int par = (a.substep + D->parity0) & 1;
  const Real *__restrict__ hs = static_cast<const Real *>(D->h[par]);
  Real *__restrict__ hd = static_cast<Real *>(D->h[par ^ 1]);
  const Real *__restrict__ gs = static_cast<const Real *>(D->g[par]);
  Real *__restrict__ gd = static_cast<Real *>(D->g[par ^ 1]);
  const Real *__restrict__ pvs = static_cast<const Real *>(D->prev[par]);
  Real *__restrict__ pvd = static_cast<Real *>(D->prev[par ^ 1]);
  const Consts<Real> &K = consts_of<Real>(D);
  const int nx = D->nx, ny = D->ny, pitch = D->pitch;
  const bool wall = D->wall != 0;
  const int64_t plane = D->plane;

  __shared__ Real sphi[8][M][kBW];
  __shared__ Real sC[4][M][kBW];

  const int lane = threadIdx.x & (kBW - 1);
  const int ry = threadIdx.x / kBW;
  const int xl = sd.x0 - 2 + lane;
  int xc = xl % nx;
  if (xc < 0) xc += nx;
  const int xw = xc == 0 ? nx - 1 : xc - 1;  // x - 1
  const int xe = xc == nx - 1 ? 0 : xc + 1;  // x + 1
  const int xend = min(sd.x0 + kTX, nx);
  const bool interior = lane >= 2 && lane < kBW - 2 && xl < xend;
  const int H = sd.y1 - sd.y0;
  const int dir = sd.dir;

  auto row_of = [&](int m) { return dir > 0 ? sd.y0 + m : sd.y1 - 1 - m; };
  auto phys_row = [&](int r) {
    if (wall) {
      if (r < 0) r = -1 - r;
      if (r >= ny) r = 2 * ny - 1 - r;
      r = r < 0 ? 0 : (r >= ny ? ny - 1 : r);
    } else {
      r %= ny;
      if (r < 0) r += ny;
    }
    return r;
  };

  // Offset of the population k arriving at (xc, yp) in a set of 9-plane
  // groups (CH) -- the source node x - c_k, or the node itself with the
  // opposite direction when x - c_k lies beyond a wall.
  struct Src {
    int64_t o0, oS, oN;  // row offsets of yp, yp - 1, yp + 1 (wrapped)
    bool bS, bN;         // bounce for c_y = +1 / c_y = -1
  };
  auto make_src = [&](int yp) {
    Src s;
    const int yS = yp - 1, yN = yp + 1;
    s.bS = wall && yS < 0;
    s.bN = wall && yN >= ny;
    s.o0 = (int64_t)yp * pitch;
    s.oS = (int64_t)(yS < 0 ? yS + ny : yS) * pitch;
    s.oN = (int64_t)(yN >= ny ? yN - ny : yN) * pitch;
    return s;
  };
  // offset within one plane group for direction k (plane index returned
  // separately so bounce-back can switch to the opposite direction)
  auto src_off = [&](const Src &s, int k, int &kk) -> int64_t {
    const int cx = cxk(k), cy = cyk(k);
    const bool b = (cy == 1 && s.bS) || (cy == -1 && s.bN);
    kk = b ? oppk(k) : k;
    const int64_t ro = b ? s.o0 : (cy == 1 ? s.oS : (cy == -1 ? s.oN : s.o0));
    const int co = b ? xc : (cx == 1 ? xw : (cx == -1 ? xe : xc));
    return ro + co;
  };

  // lo part of phi_i: the stored deviation of h_0 plus the moving populations
  auto lo_sum = [&](const Real (&h)[9]) {
    Real lo = h[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) lo += h[k];
    return lo;
  };

  // ---- stage A: pull CH populations for march index mA, phi -> LDS ----
  auto stageA = [&](int mA, Real (&cur)[M][9], Real (&hi)[M]) {
    const int yp = phys_row(row_of(mA));
    const Src s = make_src(yp);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      int kk;
      const int64_t off = src_off(s, k, kk);
#pragma unroll
      for (int i = 0; i < M; ++i) cur[i][k] = hs[(int64_t)(i * 9 + kk) * plane + off];
    }
#pragma unroll
    for (int i = 0; i < M; ++i) hi[i] = pvs[(int64_t)i * plane + s.o0 + xc];
    const int slot = (mA + 8) & 7;
#pragma unroll
    for (int i = 0; i < M; ++i) sphi[slot][i][lane] = hi[i] + lo_sum(cur[i]);  // eq:N28
  };

  // ---- stage B: chemical potentials for march index mB -> LDS ----
  auto stageB = [&](int mB) {
    if (lane < 1 || lane > kBW - 2) return;
    int me = mB;
    if (wall) {
      const int r = row_of(mB);
      if (r < 0) me = mB + dir;          // ghost below row 0: C(-1) = C(0)
      else if (r >= ny) me = mB - dir;   // ghost above row ny-1
    }
    const int s0 = (me + 8) & 7, s1 = (me + 9) & 7, s2 = (me + 7) & 7;
    Real phi[M], lap[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const Real c = sphi[s0][i][lane];
      const Real e = sphi[s0][i][lane + 1], w = sphi[s0][i][lane - 1];
      const Real n = sphi[s1][i][lane], s = sphi[s2][i][lane];
      const Real ne = sphi[s1][i][lane + 1], nw = sphi[s1][i][lane - 1];
      const Real se = sphi[s2][i][lane + 1], sw = sphi[s2][i][lane - 1];
      // eq:N31b on D2Q9: (4 sum_axis + sum_diag - 20 zeta) / 6
      lap[i] = (Real(4) * ((e + w) + (n + s)) + ((ne + nw) + (se + sw)) - Real(20) * c) *
               (Real(1) / Real(6));
      phi[i] = c;
    }
    Real wv[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      Real ck = K.ca[k];
#pragma unroll
      for (int i = 0; i < M; ++i) ck += K.cA[k][i] * phi[i];
      wv[k] = ck * (Real(1) - ck) * (Real(1) - Real(2) * ck);
    }
    const int sc = (mB + 4) & 3;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      Real Ci = Real(0);
#pragma unroll
      for (int j = 0; j < M; ++j) Ci -= K.lam[i][j] * lap[j];
#pragma unroll
      for (int k = 0; k < N; ++k) Ci += K.KH[k][i] * wv[k];
      sC[sc][i][lane] = Ci;
    }
  };

  // ---- stage C: collide march index mC with the populations in hh ----
  auto stageC = [&](int mC, Real (&hh)[M][9], const Real (&hhi)[M]) {
    if (!interior || mC < 0 || mC >= H) return;
    const int yp = row_of(mC);
    const int p0 = (mC + 8) & 7, pN = (mC + dir + 8) & 7, pS = (mC - dir + 8) & 7;
    const int q0 = (mC + 4) & 3, qN = (mC + dir + 4) & 3, qS = (mC - dir + 4) & 3;
    Real phi[M], Cv[M], gpx[M], gpy[M], gCx[M], gCy[M];
    // eq:N31a on D2Q9: d/dx = [4 (E - W) + (NE - NW + SE - SW)] / 12
#pragma unroll
    for (int i = 0; i < M; ++i) {
      phi[i] = sphi[p0][i][lane];
      {
        const Real e = sphi[p0][i][lane + 1], w = sphi[p0][i][lane - 1];
        const Real n = sphi[pN][i][lane], s = sphi[pS][i][lane];
        const Real ne = sphi[pN][i][lane + 1], nw = sphi[pN][i][lane - 1];
        const Real se = sphi[pS][i][lane + 1], sw = sphi[pS][i][lane - 1];
        gpx[i] = (Real(4) * (e - w) + ((ne - nw) + (se - sw))) * (Real(1) / Real(12));
        gpy[i] = (Real(4) * (n - s) + ((ne + nw) - (se + sw))) * (Real(1) / Real(12));
      }
      Cv[i] = sC[q0][i][lane];
      {
        const Real e = sC[q0][i][lane + 1], w = sC[q0][i][lane - 1];
        const Real n = sC[qN][i][lane], s = sC[qS][i][lane];
        const Real ne = sC[qN][i][lane + 1], nw = sC[qN][i][lane - 1];
        const Real se = sC[qS][i][lane + 1], sw = sC[qS][i][lane - 1];
        gCx[i] = (Real(4) * (e - w) + ((ne - nw) + (se - sw))) * (Real(1) / Real(12));
        gCy[i] = (Real(4) * (n - s) + ((ne + nw) - (se + sw))) * (Real(1) / Real(12));
      }
    }
    // density, relaxation, forces
    Real rho = K.ra, grx = Real(0), gry = Real(0);
    Real Fx = Real(0), Fy = Real(0), Jx = Real(0), Jy = Real(0);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      rho += K.rA[i] * phi[i];
      grx += K.rA[i] * gpx[i];
      gry += K.rA[i] * gpy[i];
      Fx += Cv[i] * gpx[i];
      Fy += Cv[i] * gpy[i];
      Jx += K.Jc[i] * gCx[i];
      Jy += K.Jc[i] * gCy[i];
    }
    Fx += rho * K.gx;
    Fy += rho * K.gy;
    Real itau, srcg, theta;
    if (K.const_tau) {
      itau = K.itau_g;
      srcg = K.src_g;
      theta = K.theta_g;
    } else {
      Real mu = K.ma;
#pragma unroll
      for (int i = 0; i < M; ++i) mu += K.mA[i] * phi[i];
      // tau_g = 1/2 + mu / (rho c_s^2)  (eq:N21_1 with nu = mu / rho)
      const Real tm = Real(3) * mu / rho;  // tau_g - 1/2
      itau = Real(1) / (Real(0.5) + tm);
      srcg = Real(1) - Real(0.5) * itau;
      theta = Real(1) / tm;
    }
    // pull the moving NS populations
    const Src s = make_src(yp);
    Real g[9];
#pragma unroll
    for (int k = 1; k < 9; ++k) {
      int kk;
      const int64_t off = src_off(s, k, kk);
      g[k] = gs[(int64_t)(kk - 1) * plane + off];
    }
    const Real irho = Real(1) / rho;
    const Real mx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const Real my = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const Real ux = (mx + Real(0.5) * Fx) * irho;  // eq:N22_1
    const Real uy = (my + Real(0.5) * Fy) * irho;
    Real sumg = g[1];
#pragma unroll
    for (int k = 2; k < 9; ++k) sumg += g[k];
    const Real usq = ux * ux + uy * uy;
    const Real udr = ux * grx + uy * gry;
    // eq:N23: p = c_s^2 / (1 - w_0) [sum_{k!=0} g_k + u.grad(rho)/2 + rho s_0(u)]
    const Real p = Real(0.6) * (sumg + Real(0.5) * udr - Real(2) / Real(3) * rho * usq);
    const Real uF = ux * Fx + uy * Fy;
    const Real Ju = Jx * ux + Jy * uy;
    // isotropic part of eq:N20_1: u.grad(rho) - tr(T) / (2 c_s^2)
    const Real gbase =
        udr - Real(1.5) * (Real(2) * uF + Real(2) / Real(3) * udr + theta * Ju);
    const int64_t orow = (int64_t)yp * pitch + xc;
#pragma unroll
    for (int k = 1; k < 9; ++k) {
      const Real cx = Real(cxk(k)), cy = Real(cyk(k));
      const Real w = wk<Real>(k);
      const Real cu = cx * ux + cy * uy;
      const Real cF = cx * Fx + cy * Fy;
      const Real cr = cx * grx + cy * gry;
      const Real cJ = cx * Jx + cy * Jy;
      const Real geq =
          w * (Real(3) * p + rho * (Real(3) * cu + Real(4.5) * cu * cu - Real(1.5) * usq));
      const Real G =
          w * (gbase + Real(3) * cF +
               Real(4.5) * cu * (Real(2) * cF + Real(2) / Real(3) * cr + theta * cJ));
      gd[(int64_t)(k - 1) * plane + orow] = g[k] - itau * (g[k] - geq) + srcg * G;
    }
    // CH collisions
    const Real pux = pvs[(int64_t)M * plane + orow];
    const Real puy = pvs[(int64_t)(M + 1) * plane + orow];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const Real pp = hhi[i];  // phi_i of the previous step (stored)
      const Real psx = phi[i] * ux, psy = phi[i] * uy;
      const Real dx = psx - pp * pux, dy = psy - pp * puy;  // eq:N27
      const Real ec = K.eta_i[i] * Cv[i];
      const Real it = K.itau_i[i], sr = K.src_i[i];
      Real hsum = Real(0);
#pragma unroll
      for (int k = 1; k < 9; ++k) {
        const Real cx = Real(cxk(k)), cy = Real(cyk(k));
        const Real w = wk<Real>(k);
        const Real heq = w * (ec + Real(3) * (cx * psx + cy * psy));   // eq:N25
        const Real R = sr * w * Real(3) * (cx * dx + cy * dy);         // eq:N26
        const Real hn = hh[i][k] - it * (hh[i][k] - heq) + R;
        hsum += hn;
        hd[(int64_t)(i * 9 + k) * plane + orow] = hn;
      }
      // phi_i = hi + lo exactly; phi[i] = fl(hi + lo) is stored as the new
      // previous phi and the k = 0 slot keeps (hi + lo - phi[i]) - sum h_k
      // (error-free two-sum for the rounding part).
      const Real lo = lo_sum(hh[i]);
      const Real bb = phi[i] - pp;
      const Real err = (pp - (phi[i] - bb)) + (lo - bb);
      hd[(int64_t)(i * 9) * plane + orow] = err - hsum;
      pvd[(int64_t)i * plane + orow] = phi[i];
    }
    pvd[(int64_t)M * plane + orow] = ux;
    pvd[(int64_t)(M + 1) * plane + orow] = uy;
  };

  Real bufA[M][9], bufB[M][9], hiA[M], hiB[M];
  const int J = (H + 5) / 2;
  for (int j = 0; j < J; j += 2) {
    {
      const int mA = 2 * j - 2 + ry;
      stageA(mA, bufA, hiA);
      __syncthreads();
      stageB(mA - 1);
      __syncthreads();
      stageC(mA - 2, bufB, hiB);
    }
    {
      const int mA = 2 * (j + 1) - 2 + ry;
      stageA(mA, bufB, hiB);
      __syncthreads();
      stageB(mA - 1);
      __syncthreads();
      stageC(mA - 2, bufA, hiA);
    }
  }
}

template <int N>
static hipError_t launch_n(int precision, const StepArgs &a, int nblocks, hipStream_t st) {
  if (precision == 64)
    hipLaunchKernelGGL((k_step<N, double>), dim3(nblocks), dim3(kStepThreads), 0, st, a);
  else
    hipLaunchKernelGGL((k_step<N, float>), dim3(nblocks), dim3(kStepThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_step(int N, int precision, const StepArgs &a, int nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  switch (N) {
    case 2: return launch_n<2>(precision, a, nblocks, st);
    case 3: return launch_n<3>(precision, a, nblocks, st);
    case 4: return launch_n<4>(precision, a, nblocks, st);
    case 5: return launch_n<5>(precision, a, nblocks, st);
    case 6: return launch_n<6>(precision, a, nblocks, st);
    case 7: return launch_n<7>(precision, a, nblocks, st);
    case 8: return launch_n<8>(precision, a, nblocks, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nplbm

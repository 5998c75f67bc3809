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

// Address spaces: the descriptors and constants are read-only for the whole
// launch and uniform per workgroup, so they are read through constant
// (scalar-load) pointers; the state arrays are global-memory pointers so the
// loads are global (not flat) loads with a per-plane scalar base and one
// shared 32-bit lane offset.
#define NPL_GLOBAL __attribute__((address_space(1)))
#define NPL_CONST __attribute__((address_space(4)))

// Element access by 32-bit byte offset from a (scalar) plane base, so that
// every access is one global load/store with an SGPR base and a VGPR offset
// shared by all planes (the host guarantees planes are below 4 GiB).
template <typename Real>
__device__ __forceinline__ Real ld(const NPL_GLOBAL Real *base, uint32_t boff) {
  return *(const NPL_GLOBAL Real *)((const NPL_GLOBAL char *)base + boff);
}
// Stores of the new state are never read again within the step; FP64 runs
// measured faster with them marked nontemporal (streaming), FP32 slower.
template <typename Real>
__device__ __forceinline__ void st(NPL_GLOBAL Real *base, uint32_t boff, Real v) {
  NPL_GLOBAL Real *p = (NPL_GLOBAL Real *)((NPL_GLOBAL char *)base + boff);
  if constexpr (sizeof(Real) == 8)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

#ifndef NPL_WAVES_PER_EU
#define NPL_KERNEL_ATTR
#else
#define NPL_KERNEL_ATTR __attribute__((amdgpu_waves_per_eu(NPL_WAVES_PER_EU)))
#endif

template <typename Real>
__device__ __forceinline__ const NPL_CONST Consts<Real> *consts_of(const NPL_CONST DomDesc *d);
template <>
__device__ __forceinline__ const NPL_CONST Consts<double> *consts_of<double>(
    const NPL_CONST DomDesc *d) {
  return &d->cd;
}
template <>
__device__ __forceinline__ const NPL_CONST Consts<float> *consts_of<float>(
    const NPL_CONST DomDesc *d) {
  return &d->cf;
}

// What one thread pulls for one node ahead of stage A and keeps until it
// collides that node in stage C one iteration later.
template <int M, typename Real>
struct Pulled {
  Real h[M][9];  // h[i][0] is the stored deviation of h_0, h[i][k>=1] streamed in
  Real hi[M];    // stored phi_i of the previous step
};
// NS populations and previous velocity of the row being collided, loaded
// one stage before use.
template <typename Real>
struct PulledNS {
  Real g[9];   // g[1..8] streamed in (g[0] unused)
  Real pu[2];  // stored u of the previous step
};

template <int N, typename Real, int kBW>
__global__ void __launch_bounds__(kBW * kRows) NPL_KERNEL_ATTR k_step(StepArgs a) {
  constexpr int M = N - 1;
  typedef const NPL_GLOBAL Real *GIn;
  typedef NPL_GLOBAL Real *GOut;
  const NPL_CONST StripDesc *sp = (const NPL_CONST StripDesc *)a.strips + blockIdx.x;
  StripDesc sd;
  sd.dom = sp->dom;
  sd.x0 = sp->x0;
  sd.y0 = sp->y0;
  sd.y1 = sp->y1;
  sd.dir = sp->dir;
  sd.x1 = sp->x1;
  if (sd.dom < 0) return;
  const NPL_CONST DomDesc *D = (const NPL_CONST DomDesc *)a.doms + sd.dom;
  if (a.substep >= D->steps_left) return;
  const int par = (a.substep + D->parity0) & 1;
  const GIn hs = (GIn)D->h[par];
  const GOut hd = (GOut)D->h[par ^ 1];
  const GIn gs = (GIn)D->g[par];
  const GOut gd = (GOut)D->g[par ^ 1];
  const GIn pvs = (GIn)D->prev[par];
  const GOut pvd = (GOut)D->prev[par ^ 1];
  const NPL_CONST Consts<Real> &K = *consts_of<Real>(D);
  const int nx = D->nx, ny = D->ny;
  const bool wall = D->wall != 0;
  // element strides between planes and between rows of each state group
  const size_t psh = (size_t)D->ps[0], psg = (size_t)D->ps[1], psp = (size_t)D->ps[2];
  const size_t rsh = (size_t)D->rs[0], rsg = (size_t)D->rs[1], rsp = (size_t)D->rs[2];

  __shared__ Real sphi[8][M][kBW];
  __shared__ Real sC[4][M][kBW];

  const int lane = threadIdx.x & (kBW - 1);
  // the row handled by this wave (uniform; said explicitly so every row,
  // bounce-back and plane decision stays in scalar registers)
  const int ry = __builtin_amdgcn_readfirstlane(threadIdx.x / kBW);
  const int xl = sd.x0 - 2 + lane;
  int xc = xl % nx;
  if (xc < 0) xc += nx;
  constexpr uint32_t SZ = sizeof(Real);
  const uint32_t xcu = (uint32_t)xc * SZ;                              // byte offsets
  const uint32_t xw = (xc == 0 ? (uint32_t)(nx - 1) : (uint32_t)xc - 1) * SZ;  // x - 1
  const uint32_t xe = (xc == nx - 1 ? 0u : (uint32_t)xc + 1) * SZ;             // x + 1
  const int ncol = sd.x1 - sd.x0;  // interior columns of this strip
  const bool interior = lane >= 2 && lane < ncol + 2;
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

  // Sources of the populations arriving at (xc, yp): the node x - c_k, or
  // the node itself with the opposite direction when x - c_k lies beyond a
  // wall.  Rows and directions are uniform over the wave (scalar); only the
  // column byte offset is per lane.
  struct Src {
    int y0, yS, yN;  // rows yp, yp - 1, yp + 1 (wrapped)
    bool bS, bN;     // bounce for c_y = +1 / c_y = -1
  };
  auto make_src = [&](int yp) {
    Src s;
    const int yS = yp - 1, yN = yp + 1;
    s.bS = wall && yS < 0;
    s.bN = wall && yN >= ny;
    s.y0 = yp;
    s.yS = yS < 0 ? yS + ny : yS;
    s.yN = yN >= ny ? yN - ny : yN;
    return s;
  };
  // source row (returned), direction kk and column byte offset co of k
  auto src_of = [&](const Src &s, int k, int &kk, uint32_t &co) -> int {
    const int cx = cxk(k), cy = cyk(k);
    const bool b = (cy == 1 && s.bS) || (cy == -1 && s.bN);
    kk = b ? oppk(k) : k;
    co = b ? xcu : (cx == 1 ? xw : (cx == -1 ? xe : xcu));
    return b ? s.y0 : (cy == 1 ? s.yS : (cy == -1 ? s.yN : s.y0));
  };

  // lo part of phi_i: the stored deviation of h_0 plus the moving populations
  auto lo_sum = [&](const Real (&h)[9]) {
    Real lo = h[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) lo += h[k];
    return lo;
  };

  // ---- pull the CH populations and stored phi of march index m ----
  auto pull_ch = [&](int m, Pulled<M, Real> &P) {
    const int yp = phys_row(row_of(m));
    const Src s = make_src(yp);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      int kk;
      uint32_t co;
      const int ys = src_of(s, k, kk, co);
#pragma unroll
      for (int i = 0; i < M; ++i)
        P.h[i][k] = ld(hs + (size_t)(i * 9 + kk) * psh + (size_t)ys * rsh, co);
    }
#pragma unroll
    for (int i = 0; i < M; ++i) P.hi[i] = ld(pvs + (size_t)i * psp + (size_t)yp * rsp, xcu);
  };
  // ---- pull the NS populations and stored u of march index m ----
  auto pull_ns = [&](int m, PulledNS<Real> &Q) {
    const int yp = phys_row(row_of(m));
    const Src s = make_src(yp);
#pragma unroll
    for (int k = 1; k < 9; ++k) {
      int kk;
      uint32_t co;
      const int ys = src_of(s, k, kk, co);
      Q.g[k] = ld(gs + (size_t)(kk - 1) * psg + (size_t)ys * rsg, co);
    }
    Q.pu[0] = ld(pvs + (size_t)M * psp + (size_t)yp * rsp, xcu);
    Q.pu[1] = ld(pvs + (size_t)(M + 1) * psp + (size_t)yp * rsp, xcu);
  };

  // ---- stage A: phi of march index mA -> LDS ----
  auto stageA = [&](int mA, const Pulled<M, Real> &cur) {
    const int slot = (mA + 8) & 7;
#pragma unroll
    for (int i = 0; i < M; ++i) sphi[slot][i][lane] = cur.hi[i] + lo_sum(cur.h[i]);  // eq:N28
  };

  // ---- stage B: chemical potentials for march index mB -> LDS ----
  auto stageB = [&](int mB) {
    if (lane < 1 || lane > ncol + 2) return;
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

  // ---- stage C: collide march index mC with what was pulled for it ----
  auto stageC = [&](int mC, const Pulled<M, Real> &P, const PulledNS<Real> &Q) {
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
    const Real(&g)[9] = Q.g;
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
    const GOut hrow = hd + (size_t)yp * rsh;
    const GOut grow = gd + (size_t)yp * rsg;
    const GOut prow = pvd + (size_t)yp * rsp;
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
      st(grow + (size_t)(k - 1) * psg, xcu, g[k] - itau * (g[k] - geq) + srcg * G);
    }
    // CH collisions
    const Real pux = Q.pu[0], puy = Q.pu[1];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const Real pp = P.hi[i];  // phi_i of the previous step (stored)
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
        const Real hn = P.h[i][k] - it * (P.h[i][k] - heq) + R;
        hsum += hn;
        st(hrow + (size_t)(i * 9 + k) * psh, xcu, hn);
      }
      // phi_i = hi + lo exactly; phi[i] = fl(hi + lo) is stored as the new
      // previous phi and the k = 0 slot keeps (hi + lo - phi[i]) - sum h_k
      // (error-free two-sum for the rounding part).
      const Real lo = lo_sum(P.h[i]);
      const Real bb = phi[i] - pp;
      const Real err = (pp - (phi[i] - bb)) + (lo - bb);
      st(hrow + (size_t)(i * 9) * psh, xcu, err - hsum);
      st(prow + (size_t)i * psp, xcu, phi[i]);
    }
    st(prow + (size_t)M * psp, xcu, ux);
    st(prow + (size_t)(M + 1) * psp, xcu, uy);
  };

  // March over iterations j (march index mA = 2j - 2 + row).  Each does
  //   phi(mA) -> LDS | barrier | NS pulls of mA - 2 | C(mA - 1) | barrier |
  //   collide mA - 2
  // with the CH pulls of row mA held in registers until their collision two
  // iterations later.  FP32 up to N = 5 has the registers to pipeline one
  // more set: the CH pulls of mA + 2 are issued right after the first
  // barrier, so they are in flight during stages B and C (three sets rotate:
  // cur = mA, next = mA + 2, held = mA - 2).  FP64 and larger N keep two
  // sets and their occupancy; three would halve it or spill.
  const int J = (H + 5) / 2;
  PulledNS<Real> ns;
  constexpr bool kPipeline = sizeof(Real) == 4 && N <= 5;
  if constexpr (kPipeline) {
    Pulled<M, Real> bufA, bufB, bufC;
    auto iteration = [&](int j, const Pulled<M, Real> &cur, Pulled<M, Real> &next,
                         const Pulled<M, Real> &held) {
      const int mA = 2 * j - 2 + ry;
      stageA(mA, cur);
      __syncthreads();
      pull_ns(mA - 2, ns);
      pull_ch(mA + 2, next);
      stageB(mA - 1);
      __syncthreads();
      stageC(mA - 2, held, ns);
    };
    pull_ch(ry - 2, bufA);
    for (int j = 0; j < J; j += 3) {  // j is uniform over the block
      iteration(j, bufA, bufB, bufC);
      if (j + 1 < J) iteration(j + 1, bufB, bufC, bufA);
      if (j + 2 < J) iteration(j + 2, bufC, bufA, bufB);
    }
  } else {
    Pulled<M, Real> bufA, bufB;  // pulled for mA (cur) and for mA - 2 (held)
    auto iteration = [&](int j, Pulled<M, Real> &cur, const Pulled<M, Real> &held) {
      const int mA = 2 * j - 2 + ry;
      pull_ch(mA, cur);
      stageA(mA, cur);
      __syncthreads();
      pull_ns(mA - 2, ns);
      stageB(mA - 1);
      __syncthreads();
      stageC(mA - 2, held, ns);
    };
    for (int j = 0; j < J; j += 2) {  // j is uniform over the block
      iteration(j, bufA, bufB);
      if (j + 1 < J) iteration(j + 1, bufB, bufA);
    }
  }
}

// LDS of one workgroup: rings of 8 phi rows and 4 C rows of (N-1) x BW values
constexpr int lds_bytes(int N, int bytes, int bw) { return 12 * (N - 1) * bw * bytes; }
// the widest row a (N, precision) pair is built for: at most 64 KiB of LDS
constexpr int max_bw(int N, int bytes) {
  return lds_bytes(N, bytes, 256) <= 65536 ? 256 : (lds_bytes(N, bytes, 128) <= 65536 ? 128 : 64);
}

int step_max_bw(int N, int precision) {
  return max_bw(N, precision == 64 ? 8 : 4);
}

template <int N, int BW>
static hipError_t launch_nb(int precision, const StepArgs &a, int nblocks, hipStream_t st) {
  if (precision == 64) {
    if constexpr (BW <= max_bw(N, 8))
      hipLaunchKernelGGL((k_step<N, double, BW>), dim3(nblocks), dim3(BW * kRows), 0, st, a);
    else
      return hipErrorInvalidValue;
  } else {
    if constexpr (BW <= max_bw(N, 4))
      hipLaunchKernelGGL((k_step<N, float, BW>), dim3(nblocks), dim3(BW * kRows), 0, st, a);
    else
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N>
static hipError_t launch_n(int precision, int bw, const StepArgs &a, int nblocks,
                           hipStream_t st) {
  return bw == 256   ? launch_nb<N, 256>(precision, a, nblocks, st)
         : bw == 128 ? launch_nb<N, 128>(precision, a, nblocks, st)
                     : launch_nb<N, 64>(precision, a, nblocks, st);
}

template <int N, int BW>
static int occ_nb(int precision) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  if (precision == 64) {
    if constexpr (BW <= max_bw(N, 8))
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step<N, double, BW>, BW * kRows, 0);
  } else {
    if constexpr (BW <= max_bw(N, 4))
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step<N, float, BW>, BW * kRows, 0);
  }
  return e == hipSuccess ? nb : 0;
}

template <int N>
static int occ_n(int precision, int bw) {
  return bw == 256 ? occ_nb<N, 256>(precision)
                   : (bw == 128 ? occ_nb<N, 128>(precision) : occ_nb<N, 64>(precision));
}

int step_blocks_per_cu(int N, int precision, int bw) {
  switch (N) {
    case 2: return occ_n<2>(precision, bw);
    case 3: return occ_n<3>(precision, bw);
    case 4: return occ_n<4>(precision, bw);
    case 5: return occ_n<5>(precision, bw);
    case 6: return occ_n<6>(precision, bw);
    case 7: return occ_n<7>(precision, bw);
    case 8: return occ_n<8>(precision, bw);
    default: return 0;
  }
}

hipError_t launch_step(int N, int precision, int bw, const StepArgs &a, int nblocks,
                       hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  switch (N) {
    case 2: return launch_n<2>(precision, bw, a, nblocks, st);
    case 3: return launch_n<3>(precision, bw, a, nblocks, st);
    case 4: return launch_n<4>(precision, bw, a, nblocks, st);
    case 5: return launch_n<5>(precision, bw, a, nblocks, st);
    case 6: return launch_n<6>(precision, bw, a, nblocks, st);
    case 7: return launch_n<7>(precision, bw, a, nblocks, st);
    case 8: return launch_n<8>(precision, bw, a, nblocks, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nplbm

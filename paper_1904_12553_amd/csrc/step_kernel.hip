// step_kernel.hip -- the fused time step of the N-phase phase-field LB model
// (arXiv:1904.12553, Sec. 3) for gfx950.
//
// One launch advances every node of every listed domain by one time step.
// Work decomposition: a workgroup owns a strip of interior columns and
// [y0, y1) rows and marches along y, two rows per iteration (one row of
// kBW lanes per march row: one lane per interior column, the phi of the
// halo columns pulled one lane per population; or, for FP64 with N >= 4
// or the two-hop schemes and for N >= 6, the interior columns plus halo
// lanes on each side).  Per iteration, with march index m counted from the
// strip start:
//
//   stage A (rows m, m+1): pull the 9(N-1) CH populations from the
//            neighbours (streaming fused into the load), phi_i = sum_k h
//            (eq:N28) -> LDS ring;
//   stage B (1 row behind A): Laplacian of eq:N31b on the LDS ring, closure
//            eq:N18 and eq:N17 -> chemical potentials C_i -> LDS ring;
//   stage C (kLag rows behind A): gradients of phi_i and C_i from the rings,
//            forces F (Sec. 3.1) and J~, pull the 8 moving NS populations,
//            u (eq:N22_1), p (eq:N23), NS collision (eq:24 with eq:25 and
//            eq:N20_1) and CH collisions (eq:N24 with eq:N25-N27) using the
//            CH populations this thread pulled kLag rows earlier (kept in
//            registers), then store.
//
// Three schemes are built (template parameter kGS):
//   - 0, central (eq:N31a): one-hop stencils; 2-column halo, C needed one
//     row ahead of the collision, so kLag = 2;
//   - 1, mixed (eq:N40 with its two-hop term read as negative): two-hop
//     stencils; 3-column halo, C needed two rows ahead, phi three, and the
//     lag must be even (a row is pulled and collided by the same wave), so
//     kLag = 4 and a third register set holds the pulls in between;
//   - 2, central stencils with the force distribution of Remark 1 (Sec.
//     3.1): G_k loses its J~ u / (tau_g - 1/2) term and F gains
//     -div(J~ u), component a = sum_b d_b (J~_b u_a) with u of the previous
//     step (the stored u of eq:N27).  J~ is needed one row and one column
//     around the collision node, so C two rows ahead and phi three, as for
//     the mixed scheme; a stage J between stages B and C forms the products
//     J~_b u_a into a fourth LDS ring, behind a third barrier.
//
// So every population is read from HBM once and written once per step; the
// only re-reads are the x-halo and a short row ramp at the strip start,
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
#include "buffer_io.h"
#include "lattice.h"
#include "nplbm_internal.h"

namespace nplbm {

// Address spaces: the descriptors and constants are read-only for the whole
// launch and uniform per workgroup, so they are read through constant
// (scalar-load) pointers.
#define NPL_CONST __attribute__((address_space(4)))

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
  Real pu[2];    // stored u of the previous step (Remark 1 scheme only)
};
// NS populations and previous velocity of the row being collided, loaded
// one stage before use.
template <typename Real>
struct PulledNS {
  Real g[9];   // g[1..8] streamed in (g[0] unused)
  Real pu[2];  // stored u of the previous step
};

// Ring sizes and march offsets of each gradient scheme: phi ring, C ring,
// halo columns, rows pulled before the strip start (ramp), and rows between
// the pull and the collision of a node (lag).
template <int kGS>
struct Scheme;
template <>
struct Scheme<0> {
  static constexpr int kPR = 8, kCR = 4, kHalo = 2, kRamp = 2, kLag = 2;
};
template <>
struct Scheme<1> {
  static constexpr int kPR = 10, kCR = 8, kHalo = 3, kRamp = 4, kLag = 4;
};
template <>
struct Scheme<2> {
  static constexpr int kPR = 10, kCR = 8, kHalo = 3, kRamp = 4, kLag = 4;
};
// rings of the Remark 1 scheme: the products J~_b u_a and the previous u
constexpr int kQR = 8, kUR = 4;
// slot of march index m (m >= -16 R) in a ring of R rows
template <int R>
__device__ __forceinline__ int ring(int m) {
  return (m + 16 * R) % R;
}

template <int N, typename Real, int kBW, int kGS>
__global__ void __launch_bounds__(kBW * kRows) NPL_KERNEL_ATTR k_step(StepArgs a) {
  constexpr int M = N - 1;
  using S = Scheme<kGS>;
  constexpr int kPR = S::kPR, kCR = S::kCR, kHalo = S::kHalo;
  constexpr bool kTwoHop = kGS == 1;  // eq:N40 first derivatives
  constexpr bool kR1 = kGS == 2;      // Remark 1 force distribution
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
  const void *hs = D->h[par], *hd = D->h[par ^ 1];
  const void *gs = D->g[par], *gd = D->g[par ^ 1];
  const void *pvs = D->prev[par], *pvd = D->prev[par ^ 1];
  const NPL_CONST Consts<Real> &K = *consts_of<Real>(D);
  // The NS part of the collision (density, u, p, g^eq, G and the g update)
  // is evaluated in FP64 arithmetic in both modes; the FP32 mode still
  // stores FP32 populations.  Evaluated in FP32, the rounding of g^eq
  // and of the update leaves each node's momentum off by a fraction of an
  // ulp, in the same direction wherever the flow state repeats (inside a
  // moving droplet), so droplets gain momentum steadily and interfaces drift
  // as t^2: FP32 vs FP64 on the 512^2 N = 4 droplet collision went from
  // 2.6e-5 to 7e-8 in c after 2000 steps (2e-3 to 7e-7 after 50000), for
  // 2.7% more kernel time, most of which the evaluation per pair of
  // opposite directions below won back.
  using Acc = double;
  const NPL_CONST Consts<double> &KD = *consts_of<double>(D);
  const int nx = D->nx, ny = D->ny;
  const bool wall = D->wall != 0;
  // bytes between planes (the row pitch, the same in every group) and
  // bytes of one row block of each state group
  constexpr uint32_t SZ = sizeof(Real);
  const uint32_t pb = (uint32_t)D->ps[0] * SZ;
  const uint32_t rbh = (uint32_t)D->rs[0] * SZ, rbg = (uint32_t)D->rs[1] * SZ,
                 rbp = (uint32_t)D->rs[2] * SZ;

  // Lane layout.  Interior lanes (interior_lanes: the central scheme at
  // N <= 5 in FP32, N <= 3 in FP64, the two-hop schemes at N <= 5 in
  // FP32): lane l owns interior column x0 + l,
  // ring column l + kHalo, so a strip has up to kBW interior columns and
  // every row of loads and stores starts on the strip's first cache line;
  // phi of the 2 kHalo halo columns is pulled one lane per (halo node,
  // direction) (halo_pull, halo_phi).  Otherwise lane l owns column
  // x0 - kHalo + l, and the halo lanes pull their nodes like the interior
  // ones and do not collide.
  constexpr bool kIL = interior_lanes(N, sizeof(Real), kGS);
  // nontemporal stores of the new state (see bst)
  constexpr bool kNTS = sizeof(Real) == 8 || kIL;
  constexpr int kRW = kIL ? kBW + 2 * kHalo : kBW;  // ring row width
  __shared__ Real sphi[kPR][M][kRW];
  __shared__ Real sC[kCR][M][kRW];
  __shared__ Real sQ[kR1 ? kQR : 1][4][kRW];  // J~_x u_x, J~_y u_x, J~_x u_y, J~_y u_y
  __shared__ Real sU[kR1 ? kUR : 1][2][kRW];  // previous u

  const int lane = threadIdx.x & (kBW - 1);
  const int pos = kIL ? lane + kHalo : lane;  // ring column
  // the row handled by this wave (uniform; said explicitly so every row,
  // bounce-back and plane decision stays in scalar registers)
  const int ry = __builtin_amdgcn_readfirstlane(threadIdx.x / kBW);
  const int xl = kIL ? sd.x0 + lane : sd.x0 - kHalo + lane;
  int xc = xl % nx;
  if (xc < 0) xc += nx;
  const uint32_t xcu = (uint32_t)xc * SZ;                              // byte offsets
  const uint32_t xw = (xc == 0 ? (uint32_t)(nx - 1) : (uint32_t)xc - 1) * SZ;  // x - 1
  const uint32_t xe = (xc == nx - 1 ? 0u : (uint32_t)xc + 1) * SZ;             // x + 1
  const int ncol = sd.x1 - sd.x0;  // interior columns of this strip
  const bool interior = kIL ? lane < ncol : (lane >= kHalo && lane < ncol + kHalo);
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
  // source row block (returned: 0 own row, 1 row below, 2 row above),
  // direction kk and column byte offset co of k
  auto src_of = [&](const Src &s, int k, int &kk, uint32_t &co) -> int {
    const int cx = cxk(k), cy = cyk(k);
    const bool b = (cy == 1 && s.bS) || (cy == -1 && s.bN);
    kk = b ? oppk(k) : k;
    co = b ? xcu : (cx == 1 ? xw : (cx == -1 ? xe : xcu));
    return b ? 0 : (cy == 1 ? 1 : (cy == -1 ? 2 : 0));
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
    const Rsrc r0 = row_rsrc(hs, rbh, s.y0), rS = row_rsrc(hs, rbh, s.yS),
               rN = row_rsrc(hs, rbh, s.yN);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      int kk;
      uint32_t co;
      const int w = src_of(s, k, kk, co);
      const Rsrc r = w == 1 ? rS : (w == 2 ? rN : r0);
#pragma unroll
      for (int i = 0; i < M; ++i) P.h[i][k] = bld<Real>(r, co, (uint32_t)(i * 9 + kk) * pb);
    }
    const Rsrc rp = row_rsrc(pvs, rbp, yp);
#pragma unroll
    for (int i = 0; i < M; ++i) P.hi[i] = bld<Real>(rp, xcu, (uint32_t)i * pb);
    if constexpr (kR1) {
      P.pu[0] = bld<Real>(rp, xcu, (uint32_t)M * pb);
      P.pu[1] = bld<Real>(rp, xcu, (uint32_t)(M + 1) * pb);
    }
  };
  // ---- pull the NS populations and stored u of march index m ----
  auto pull_ns = [&](int m, PulledNS<Real> &Q) {
    const int yp = phys_row(row_of(m));
    const Src s = make_src(yp);
    const Rsrc r0 = row_rsrc(gs, rbg, s.y0), rS = row_rsrc(gs, rbg, s.yS),
               rN = row_rsrc(gs, rbg, s.yN);
#pragma unroll
    for (int k = 1; k < 9; ++k) {
      int kk;
      uint32_t co;
      const int w = src_of(s, k, kk, co);
      const Rsrc r = w == 1 ? rS : (w == 2 ? rN : r0);
      Q.g[k] = bld<Real>(r, co, (uint32_t)(kk - 1) * pb);
    }
    const Rsrc rp = row_rsrc(pvs, rbp, yp);
    Q.pu[0] = bld<Real>(rp, xcu, (uint32_t)M * pb);
    Q.pu[1] = bld<Real>(rp, xcu, (uint32_t)(M + 1) * pb);
  };

  // ---- stage A: phi of march index mA -> LDS ----
  auto stageA = [&](int mA, const Pulled<M, Real> &cur) {
    const int slot = ring<kPR>(mA);
    // (lanes past a ragged strip end would overwrite the right halo)
    if (!kIL || lane < ncol)
#pragma unroll
      for (int i = 0; i < M; ++i) sphi[slot][i][pos] = cur.hi[i] + lo_sum(cur.h[i]);  // eq:N28
    if constexpr (kR1) {
      if (!kIL || lane < ncol) {
        sU[ring<kUR>(mA)][0][pos] = cur.pu[0];
        sU[ring<kUR>(mA)][1][pos] = cur.pu[1];
      }
    }
  };

  // ---- x-halo phi of rows of interior lanes ----
  // Phase i of the kNH halo nodes of a row (columns x0 - kHalo .. x0 - 1
  // and x1 .. x1 + kHalo - 1) is pulled by one wave of the row: lane
  // t < 9 kNH pulls
  // direction t % 9 of halo node t / 9 and lane 9 kNH + n the stored phi of
  // node n, so a phase costs one load instruction instead of the 9 of a
  // lane per node.  The row's waves share the phases (the wave wv of the
  // row takes i = wv, wv + kNW, ...).  halo_phi then sums each node's
  // values in the order of stage A, so a halo phi equals, bit for bit, the
  // phi the neighbouring strip computes for that node.
  constexpr int kNH = 2 * kHalo;                      // halo nodes per row
  constexpr int kNW = kBW / 64;                       // waves per row
  constexpr int kHP = kIL ? (M + kNW - 1) / kNW : 1;  // phases per wave
  __shared__ Real shalo[kIL ? kRows * kNW : 1][10 * kNH];
  const int wv = __builtin_amdgcn_readfirstlane((threadIdx.x % kBW) / 64);  // wave in the row
  // Per-lane halo descriptor, decoded at each pull (kept in one register
  // through the march): the halo node's column (bits 0..26) and what the
  // lane loads (bits 27..30): 0 the stored phi, 1..9 direction 0..8, 10 and
  // 11 the stored u_x and u_y (Remark 1: J~ u is needed one column beyond
  // the interior, so lanes 10 kNH .. 10 kNH + 3 load the previous u of
  // the halo nodes x0 - 1 and x1, once per row), 15 nothing.
  static_assert(!kIL || 10 * kNH + (kR1 ? 4 : 0) <= 64, "halo lanes");
  uint32_t hdesc = 15u << 27;
  if constexpr (kIL) {
    const int wl = threadIdx.x & 63;  // lane in the wave
    int hn = -1, what = 15;           // halo node of this lane, what it loads
    if (wl < 9 * kNH) {
      hn = wl / 9;
      what = wl % 9 + 1;
    } else if (wl < 10 * kNH) {
      hn = wl - 9 * kNH;
      what = 0;
    } else if (kR1 && wl < 10 * kNH + 4) {
      hn = kHalo - 1 + (wl - 10 * kNH) / 2;
      what = 10 + (wl - 10 * kNH) % 2;
    }
    if (hn >= 0) {
      int hxc = (hn < kHalo ? sd.x0 - kHalo + hn : sd.x1 + hn - kHalo) % nx;
      if (hxc < 0) hxc += nx;
      hdesc = (uint32_t)hxc | ((uint32_t)what << 27);
    }
  }
  auto halo_pull = [&](int m, Real (&hv)[kHP]) {
    if constexpr (kIL) {
      const int yp = phys_row(row_of(m));
      // decode here, not once outside the march (the mixed scheme at N = 5
      // needs those registers): the empty asm makes dsc depend on the row
      // (no side effects, so loads still move across it)
      uint32_t dsc = hdesc;
      asm("" : "+v"(dsc) : "s"(m));
      const uint32_t hkp = dsc >> 27, hxc = dsc & ((1u << 27) - 1);
      // source node and direction hkp - 1 (bounce-back beyond a wall), as
      // src_of
      int sy = yp, sx = (int)hxc, kk = (int)hkp - 1;
      if (hkp >= 2 && hkp <= 9) {
        const int k = (int)hkp - 1;
        const int cx = cxk(k), cy = cyk(k);
        const int ys = yp - cy;
        if (wall && (ys < 0 || ys >= ny)) {
          kk = oppk(k);
        } else {
          sy = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
          sx -= cx;
          sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
        }
      }
      typedef const __attribute__((address_space(1))) char GC;
      const bool pop = hkp >= 1 && hkp <= 9;
      GC *base = pop ? (GC *)hs + (size_t)sy * rbh + (size_t)sx * SZ
                     : (GC *)pvs + (size_t)yp * rbp + (size_t)hxc * SZ;
      typedef const __attribute__((address_space(1))) Real GR;
      if (hkp <= 9) {
#pragma unroll
        for (int q = 0; q < kHP; ++q) {
          const int i = wv + q * kNW;
          if (i < M) {
            const uint32_t plane = pop ? (uint32_t)(i * 9 + kk) : (uint32_t)i;
            hv[q] = *(GR *)(base + (size_t)plane * pb);
          }
        }
      } else if (kR1 && hkp <= 11 && wv == 0) {
        hv[0] = *(GR *)(base + (size_t)(M + hkp - 10) * pb);
      }
    }
  };
  auto halo_phi = [&](int mA, const Real (&hv)[kHP]) {
    if constexpr (kIL) {
      const int slot = ring<kPR>(mA);
      const int wl = threadIdx.x & 63;
      Real *sh = shalo[ry * kNW + wv];
#pragma unroll
      for (int q = 0; q < kHP; ++q) {
        const int i = wv + q * kNW;
        if (i < M) {
          if (wl < 10 * kNH) sh[wl] = hv[q];
          if (wl < kNH) {
            Real lo = sh[9 * wl];
#pragma unroll
            for (int k = 1; k < 9; ++k) lo += sh[9 * wl + k];
            sphi[slot][i][wl < kHalo ? wl : ncol + wl] = sh[9 * kNH + wl] + lo;  // eq:N28
          }
        }
      }
      if constexpr (kR1) {
        // previous u of the halo nodes x0 - 1 and x1 (ring columns kHalo - 1
        // and ncol + kHalo)
        const int t = wl - 10 * kNH;
        if (wv == 0 && t >= 0 && t < 4)
          sU[ring<kUR>(mA)][t & 1][t < 2 ? kHalo - 1 : ncol + kHalo] = hv[0];
      }
    }
  };

  // ---- stage B: chemical potentials for march index mB -> LDS ----
  // C is needed on the interior columns and one (central) or two (mixed,
  // Remark 1) columns either side.  Next to a wall, C of a ghost row is the
  // mirror of C inside.  The central scheme reads it from the row it
  // mirrors (C(-1) = C(0)).  The other two evaluate ghost rows on the
  // mirrored phi rows the ring holds, which gives the same values (the
  // stencil is mirror-symmetric): the mixed scheme needs two ghost rows,
  // C(-2) = C(1) being ahead of the march, and Remark 1 needs the ghost C
  // for J~ on the wall row, which a strip marching away from the wall may
  // hold in its ramp; there the row it mirrors can be one whose phi
  // neighbour the march has not pulled yet (a strip starting one row
  // inside the wall).
  auto stageB = [&](int mB) {
    int me = mB;
    if (kGS == 0 && wall) {
      const int r = row_of(mB);
      if (r < 0) me = mB + dir;          // ghost below row 0: C(-1) = C(0)
      else if (r >= ny) me = mB - dir;   // ghost above row ny-1
    }
    const int s0 = ring<kPR>(me), s1 = ring<kPR>(me + 1), s2 = ring<kPR>(me - 1);
    const int sc = ring<kCR>(mB);
    // C at ring column x
    auto chem = [&](int x) {
      Real phi[M], lap[M];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const Real c = sphi[s0][i][x];
        const Real e = sphi[s0][i][x + 1], w = sphi[s0][i][x - 1];
        const Real n = sphi[s1][i][x], s = sphi[s2][i][x];
        const Real ne = sphi[s1][i][x + 1], nw = sphi[s1][i][x - 1];
        const Real se = sphi[s2][i][x + 1], sw = sphi[s2][i][x - 1];
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
#pragma unroll
      for (int i = 0; i < M; ++i) {
        Real Ci = Real(0);
#pragma unroll
        for (int j = 0; j < M; ++j) Ci -= K.lam[i][j] * lap[j];
#pragma unroll
        for (int k = 0; k < N; ++k) Ci += K.KH[k][i] * wv[k];
        sC[sc][i][x] = Ci;
      }
    };
    if constexpr (kIL) {
      // ring columns 1 .. ncol + 2 kHalo - 2: lane l takes l + 1, and the
      // first lanes also the last 2 kHalo - 2 of a full-width strip
      for (int x = lane + 1; x <= ncol + 2 * kHalo - 2; x += kBW) chem(x);
    } else {
      if (lane >= 1 && lane <= ncol + 2 * kHalo - 2) chem(pos);
    }
  };

  // ---- stage J (Remark 1 scheme): J~ and the products J~_b u_a ----
  // J~ (eq:N18 line 4) from the eq:N31a gradients of C, on the interior
  // columns and one either side, times the stored previous u.  Ghost rows
  // beyond a wall are not evaluated: stage C reads the mirrored row, the
  // same values (the ghost of a field is its mirror image).
  auto stageJ = [&](int mJ) {
    if (wall) {
      const int r = row_of(mJ);
      if (r < 0 || r >= ny) return;
    }
    const int q0 = ring<kCR>(mJ), qN = ring<kCR>(mJ + dir), qS = ring<kCR>(mJ - dir);
    const int su = ring<kUR>(mJ), sq = ring<kQR>(mJ);
    // at ring column x (2 .. ncol + 2 kHalo - 3)
    auto prod = [&](int x) {
      Real Jx = Real(0), Jy = Real(0);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const Real e = sC[q0][i][x + 1], w = sC[q0][i][x - 1];
        const Real n = sC[qN][i][x], s = sC[qS][i][x];
        const Real ne = sC[qN][i][x + 1], nw = sC[qN][i][x - 1];
        const Real se = sC[qS][i][x + 1], sw = sC[qS][i][x - 1];
        const Real gx = (Real(4) * (e - w) + ((ne - nw) + (se - sw))) * (Real(1) / Real(12));
        const Real gy = (Real(4) * (n - s) + ((ne + nw) - (se + sw))) * (Real(1) / Real(12));
        Jx += K.Jc[i] * gx;
        Jy += K.Jc[i] * gy;
      }
      const Real ux = sU[su][0][x], uy = sU[su][1][x];
      sQ[sq][0][x] = Jx * ux;
      sQ[sq][1][x] = Jy * ux;
      sQ[sq][2][x] = Jx * uy;
      sQ[sq][3][x] = Jy * uy;
    };
    if constexpr (kIL) {
      // lane l takes column l + 2, and the first lanes also the last two
      for (int x = lane + 2; x <= ncol + 2 * kHalo - 3; x += kBW) prod(x);
    } else {
      if (lane >= 2 && lane <= ncol + 2 * kHalo - 3) prod(pos);
    }
  };

  // ---- stage G (mixed scheme): the phi gradients of march index mC ----
  // eq:N40 below; phi is on the ring up to row mC + 4 once the first barrier
  // of the iteration is passed, so these terms are summed before stage B:
  // the two-hop stencils then do not share the registers of stage C with
  // the NS arithmetic (with them in stage C, three register sets spilled
  // 172 B per lane at N = 5 in FP32).  The sums are the ones stage C forms
  // for the other schemes, over the phases in the same order.
  struct PhiGrad {
    Real grs, gys, Fxs, Fys;  // sum_i rA_i grad phi_i, sum_i C_i grad phi_i
  };
  auto grad2 = [&](const Real (*f)[M][kRW], int r0, int rN, int rS, int rN2, int rS2, int i,
                   Real &gx, Real &gy) {
    // eq:N40 summed over the D2Q9 directions.  Per direction c the
    // difference is -z(x+2c) + 5 z(x+c) - 3 z(x) - z(x-c); with w_c, c_x
    // and 1/(4 c_s^2) the z(x) terms cancel and opposite directions pair:
    //   d/dx = [24 (E - W) - 4 (E2 - W2) + 6 (NE - NW + SE - SW)
    //           - (NE2 - NW2 + SE2 - SW2)] / 48
    // (E2 = z(x+2, y), NE2 = z(x+2, y+2), ...), and likewise d/dy.
    const Real e = f[r0][i][pos + 1], w = f[r0][i][pos - 1];
    const Real e2 = f[r0][i][pos + 2], w2 = f[r0][i][pos - 2];
    const Real n = f[rN][i][pos], s = f[rS][i][pos];
    const Real n2 = f[rN2][i][pos], s2 = f[rS2][i][pos];
    const Real ne = f[rN][i][pos + 1], nw = f[rN][i][pos - 1];
    const Real se = f[rS][i][pos + 1], sw = f[rS][i][pos - 1];
    const Real ne2 = f[rN2][i][pos + 2], nw2 = f[rN2][i][pos - 2];
    const Real se2 = f[rS2][i][pos + 2], sw2 = f[rS2][i][pos - 2];
    gx = (Real(24) * (e - w) - Real(4) * (e2 - w2) + Real(6) * ((ne - nw) + (se - sw)) -
          ((ne2 - nw2) + (se2 - sw2))) *
         (Real(1) / Real(48));
    gy = (Real(24) * (n - s) - Real(4) * (n2 - s2) + Real(6) * ((ne + nw) - (se + sw)) -
          ((ne2 + nw2) - (se2 + sw2))) *
         (Real(1) / Real(48));
  };
  auto stageG = [&](int mC) {
    PhiGrad G{Real(0), Real(0), Real(0), Real(0)};
    if constexpr (kTwoHop) {
      if (!interior || mC < 0 || mC >= H) return G;
      const int p0 = ring<kPR>(mC), pN = ring<kPR>(mC + dir), pS = ring<kPR>(mC - dir);
      const int pN2 = ring<kPR>(mC + 2 * dir), pS2 = ring<kPR>(mC - 2 * dir);
      const int q0 = ring<kCR>(mC);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        Real gx, gy;
        grad2(sphi, p0, pN, pS, pN2, pS2, i, gx, gy);
        const Real Ci = sC[q0][i][pos];
        G.grs += K.rA[i] * gx;
        G.gys += K.rA[i] * gy;
        G.Fxs += Ci * gx;
        G.Fys += Ci * gy;
      }
    }
    return G;
  };

  // ---- stage C: collide march index mC with what was pulled for it ----
  auto stageC = [&](int mC, const Pulled<M, Real> &P, const PulledNS<Real> &Q,
                    const PhiGrad &G) {
    if (!interior || mC < 0 || mC >= H) return;
    const int yp = row_of(mC);
    const int p0 = ring<kPR>(mC), pN = ring<kPR>(mC + dir), pS = ring<kPR>(mC - dir);
    const int q0 = ring<kCR>(mC), qN = ring<kCR>(mC + dir), qS = ring<kCR>(mC - dir);
    Real phi[M], Cv[M], gpx[M], gpy[M], gCx[M], gCy[M];
    if constexpr (!kTwoHop) {
      // eq:N31a on D2Q9: d/dx = [4 (E - W) + (NE - NW + SE - SW)] / 12
      auto grad = [&](const Real (*f)[M][kRW], int r0, int rN, int rS, int i, Real &gx,
                      Real &gy) {
        const Real e = f[r0][i][pos + 1], w = f[r0][i][pos - 1];
        const Real n = f[rN][i][pos], s = f[rS][i][pos];
        const Real ne = f[rN][i][pos + 1], nw = f[rN][i][pos - 1];
        const Real se = f[rS][i][pos + 1], sw = f[rS][i][pos - 1];
        gx = (Real(4) * (e - w) + ((ne - nw) + (se - sw))) * (Real(1) / Real(12));
        gy = (Real(4) * (n - s) + ((ne + nw) - (se + sw))) * (Real(1) / Real(12));
      };
#pragma unroll
      for (int i = 0; i < M; ++i) {
        phi[i] = sphi[p0][i][pos];
        Cv[i] = sC[q0][i][pos];
        grad(sphi, p0, pN, pS, i, gpx[i], gpy[i]);
        if constexpr (!kR1) grad(sC, q0, qN, qS, i, gCx[i], gCy[i]);
      }
    } else {
      // the C gradients (eq:N40) here; the phi gradients came from stage G
      const int qN2 = ring<kCR>(mC + 2 * dir), qS2 = ring<kCR>(mC - 2 * dir);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        phi[i] = sphi[p0][i][pos];
        Cv[i] = sC[q0][i][pos];
        grad2(sC, q0, qN, qS, qN2, qS2, i, gCx[i], gCy[i]);
      }
    }
    // density, relaxation, forces
    // (the sums over phases of the gradient terms stay in the state type:
    // measured, FP64 there changes nothing)
    Acc rho = KD.ra;
    Real grs = Real(0), gys = Real(0), Fxs = Real(0), Fys = Real(0), Jxs = Real(0), Jys = Real(0);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      rho += KD.rA[i] * phi[i];
      if constexpr (!kTwoHop) {
        grs += K.rA[i] * gpx[i];
        gys += K.rA[i] * gpy[i];
        Fxs += Cv[i] * gpx[i];
        Fys += Cv[i] * gpy[i];
      }
      if constexpr (!kR1) {
        Jxs += K.Jc[i] * gCx[i];
        Jys += K.Jc[i] * gCy[i];
      }
    }
    if constexpr (kTwoHop) {
      grs = G.grs;
      gys = G.gys;
      Fxs = G.Fxs;
      Fys = G.Fys;
    }
    const Acc grx = grs, gry = gys, Jx = Jxs, Jy = Jys;
    Acc Fx = Fxs, Fy = Fys;
    Fx += rho * KD.gx;
    Fy += rho * KD.gy;
    if constexpr (kR1) {
      // Remark 1: F -= div(J~ u), (div)_x = d_x q0 + d_y q1,
      // (div)_y = d_x q2 + d_y q3, eq:N31a on the product ring; a row
      // beyond a wall is its mirror, the collision row itself
      auto ghost = [&](int m) {
        const int r = row_of(m);
        return wall && (r < 0 || r >= ny);
      };
      const int s0 = ring<kQR>(mC);
      const int sN = ghost(mC + dir) ? s0 : ring<kQR>(mC + dir);
      const int sS = ghost(mC - dir) ? s0 : ring<kQR>(mC - dir);
      auto ddx = [&](int c) {
        return (Acc(4) * (sQ[s0][c][pos + 1] - sQ[s0][c][pos - 1]) +
                ((sQ[sN][c][pos + 1] - sQ[sN][c][pos - 1]) +
                 (sQ[sS][c][pos + 1] - sQ[sS][c][pos - 1]))) *
               (Acc(1) / Acc(12));
      };
      auto ddy = [&](int c) {
        return (Acc(4) * (sQ[sN][c][pos] - sQ[sS][c][pos]) +
                ((sQ[sN][c][pos + 1] + sQ[sN][c][pos - 1]) -
                 (sQ[sS][c][pos + 1] + sQ[sS][c][pos - 1]))) *
               (Acc(1) / Acc(12));
      };
      Fx -= ddx(0) + ddy(1);
      Fy -= ddx(2) + ddy(3);
    }
    Acc itau, srcg, theta;
    if (KD.const_tau) {
      itau = KD.itau_g;
      srcg = KD.src_g;
      theta = KD.theta_g;
    } else {
      Acc mu = KD.ma;
#pragma unroll
      for (int i = 0; i < M; ++i) mu += KD.mA[i] * phi[i];
      // tau_g = 1/2 + mu / (rho c_s^2)  (eq:N21_1 with nu = mu / rho)
      const Acc tm = Acc(3) * mu / rho;  // tau_g - 1/2
      itau = Acc(1) / (Acc(0.5) + tm);
      srcg = Acc(1) - Acc(0.5) * itau;
      theta = Acc(1) / tm;
    }
    Acc g[9];
#pragma unroll
    for (int k = 1; k < 9; ++k) g[k] = Q.g[k];
    const Acc irho = Acc(1) / rho;
    const Acc mx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const Acc my = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const Acc ux = (mx + Acc(0.5) * Fx) * irho;  // eq:N22_1
    const Acc uy = (my + Acc(0.5) * Fy) * irho;
    Acc sumg = g[1];
#pragma unroll
    for (int k = 2; k < 9; ++k) sumg += g[k];
    const Acc usq = ux * ux + uy * uy;
    const Acc udr = ux * grx + uy * gry;
    // eq:N23: p = c_s^2 / (1 - w_0) [sum_{k!=0} g_k + u.grad(rho)/2 + rho s_0(u)]
    const Acc p = Acc(0.6) * (sumg + Acc(0.5) * udr - Acc(2) / Acc(3) * rho * usq);
    const Acc uF = ux * Fx + uy * Fy;
    const Acc Ju = Jx * ux + Jy * uy;
    // isotropic part of eq:N20_1: u.grad(rho) - tr(T) / (2 c_s^2)
    const Acc gbase =
        udr - Acc(1.5) * (Acc(2) * uF + Acc(2) / Acc(3) * udr + (kR1 ? Acc(0) : theta * Ju));
    const Rsrc wh = row_rsrc(hd, rbh, yp), wg = row_rsrc(gd, rbg, yp),
               wp = row_rsrc(pvd, rbp, yp);
    // g* = (1 - 1/tau) g + g^eq / tau + (1 - 1/(2 tau)) G (eq:24), with
    // g^eq (eq:25) and G (eq:N20_1) split into the parts even and odd in
    // c_k: opposite directions share the even part and negate the odd one,
    // so each pair is evaluated once
    const Acc keep = Acc(1) - itau;
    const Acc e0 = Acc(3) * p - Acc(1.5) * rho * usq;
#pragma unroll
    for (int k = 1; k < 9; ++k) {
      if (oppk(k) < k) continue;
      const int ko = oppk(k);
      const Acc cx = Acc(cxk(k)), cy = Acc(cyk(k));
      const Acc w = wk<Acc>(k);
      const Acc cu = cx * ux + cy * uy;
      const Acc cF = cx * Fx + cy * Fy;
      const Acc cr = cx * grx + cy * gry;
      const Acc cJ = cx * Jx + cy * Jy;
      const Acc ev =
          w * (itau * (e0 + Acc(4.5) * rho * cu * cu) +
               srcg * (gbase + Acc(4.5) * cu *
                                   (Acc(2) * cF + Acc(2) / Acc(3) * cr +
                                    (kR1 ? Acc(0) : theta * cJ))));
      const Acc od = w * Acc(3) * (itau * rho * cu + srcg * cF);
      bst<Real, kNTS>(wg, xcu, (uint32_t)(k - 1) * pb, keep * g[k] + ev + od);
      bst<Real, kNTS>(wg, xcu, (uint32_t)(ko - 1) * pb, keep * g[ko] + ev - od);
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
      // h* = (1 - 1/tau_i) h + h^eq / tau_i + R_k with h^eq (eq:N25) and R_k
      // (eq:N26) split into the parts even and odd in c_k, per pair of
      // opposite directions
      const Real keep = Real(1) - it;
      Real hsum = Real(0);
#pragma unroll
      for (int k = 1; k < 9; ++k) {
        if (oppk(k) < k) continue;
        const int ko = oppk(k);
        const Real cx = Real(cxk(k)), cy = Real(cyk(k));
        const Real w = wk<Real>(k);
        const Real ev = it * w * ec;
        const Real od = w * Real(3) * (it * (cx * psx + cy * psy) + sr * (cx * dx + cy * dy));
        const Real hn = keep * P.h[i][k] + ev + od;
        const Real ho = keep * P.h[i][ko] + ev - od;
        hsum += hn + ho;
        bst<Real, kNTS>(wh, xcu, (uint32_t)(i * 9 + k) * pb, hn);
        bst<Real, kNTS>(wh, xcu, (uint32_t)(i * 9 + ko) * pb, ho);
      }
      // phi_i = hi + lo exactly; phi[i] = fl(hi + lo) is stored as the new
      // previous phi and the k = 0 slot keeps (hi + lo - phi[i]) - sum h_k
      // (error-free two-sum for the rounding part).
      const Real lo = lo_sum(P.h[i]);
      const Real bb = phi[i] - pp;
      const Real err = (pp - (phi[i] - bb)) + (lo - bb);
      bst<Real, kNTS>(wh, xcu, (uint32_t)(i * 9) * pb, err - hsum);
      bst<Real, kNTS>(wp, xcu, (uint32_t)i * pb, phi[i]);
    }
    bst<Real, kNTS>(wp, xcu, (uint32_t)M * pb, ux);
    bst<Real, kNTS>(wp, xcu, (uint32_t)(M + 1) * pb, uy);
  };

  // March over iterations j (march index mA = 2j - kRamp + row).  Each does
  //   phi(mA) -> LDS | barrier | NS pulls of mA - kLag | C(mA - 1) |
  //   barrier | collide mA - kLag
  // with the CH pulls of row mA held in registers until their collision
  // kLag / 2 iterations later.
  //  - central, FP32, N <= 5: the registers allow pipelining one more set:
  //    the CH pulls of mA + 2 (and the x-halo values of that row) are
  //    issued right after the first barrier, so they are in flight during
  //    stages B and C (three sets rotate: cur = mA, next = mA + 2, held =
  //    mA - 2);
  //  - central otherwise: two sets (cur, held = mA - 2); three would halve
  //    the occupancy or spill;
  //  - mixed and Remark 1, N <= 5: three sets (cur, mA - 2, mA - 4); the
  //    Remark 1 scheme runs stage J on rows mA - 2 behind a third barrier
  //    before the collision.  At N = 5 the three sets fit: in FP32 in two waves per SIMD once
  //    the mixed scheme's phi gradients are summed in stage G (245 VGPRs;
  //    Remark 1 229), in FP64 in one wave per SIMD with AGPRs (mixed 436
  //    registers, Remark 1 412, no spill).  Measured on the 2048^2 N = 5
  //    workload against pulling the collision row a second time: mixed FP32
  //    55.0% against 45.9% of the HBM roofline with 256-thread rows (58.2%
  //    with 128-thread rows), mixed FP64 63.6% against 50.8%, Remark 1 FP64
  //    63.9% against 49.8%.  Keeping the set pulled one
  //    iteration earlier in LDS instead of registers measured 59.7% (mixed
  //    FP64);
  //  - mixed and Remark 1, N >= 6: the collision row's CH populations are
  //    pulled a second time (from L2 / MALL, 2 iterations after the first
  //    pull) and one set suffices (the re-read costs the central scheme 13
  //    points of the HBM roofline).
  constexpr int kRamp = S::kRamp, kLag = S::kLag;
  constexpr bool kRepull = kGS != 0 && N >= 6;
  const int J = (H + kRamp + kLag + 1) / 2;
  PulledNS<Real> ns;
  constexpr bool kPipeline = kGS == 0 && sizeof(Real) == 4 && N <= 5;
  if constexpr (kRepull) {
    // one register set: the CH populations of the collision row are loaded
    // again (from L2 / MALL) right after the first barrier
    Pulled<M, Real> buf;
    for (int j = 0; j < J; ++j) {
      const int mA = 2 * j - kRamp + ry;
      pull_ch(mA, buf);
      stageA(mA, buf);
      __syncthreads();
      pull_ns(mA - kLag, ns);
      const PhiGrad g1 = stageG(mA - kLag);
      pull_ch(mA - kLag, buf);
      stageB(mA - 1);
      __syncthreads();
      if constexpr (kR1) {
        stageJ(mA - 2);
        __syncthreads();
      }
      stageC(mA - kLag, buf, ns, g1);
    }
  } else if constexpr (kGS != 0) {
    Pulled<M, Real> bufA, bufB, bufC;
    Real hv[kHP];
    auto iteration = [&](int j, Pulled<M, Real> &cur, const Pulled<M, Real> &held) {
      const int mA = 2 * j - kRamp + ry;
      pull_ch(mA, cur);
      halo_pull(mA, hv);
      stageA(mA, cur);
      halo_phi(mA, hv);
      __syncthreads();
      pull_ns(mA - kLag, ns);
      const PhiGrad g1 = stageG(mA - kLag);
      stageB(mA - 1);
      __syncthreads();
      if constexpr (kR1) {
        stageJ(mA - 2);
        __syncthreads();
      }
      stageC(mA - kLag, held, ns, g1);
    };
    for (int j = 0; j < J; j += 3) {  // j is uniform over the block
      iteration(j, bufA, bufB);       // bufB holds the pulls of iteration j - 2
      if (j + 1 < J) iteration(j + 1, bufB, bufC);
      if (j + 2 < J) iteration(j + 2, bufC, bufA);
    }
  } else if constexpr (kPipeline) {
    Pulled<M, Real> bufA, bufB, bufC;
    Real hv[kHP];  // halo values of row mA, pulled with its CH populations
    auto iteration = [&](int j, const Pulled<M, Real> &cur, Pulled<M, Real> &next,
                         const Pulled<M, Real> &held) {
      const int mA = 2 * j - kRamp + ry;
      stageA(mA, cur);
      halo_phi(mA, hv);
      __syncthreads();
      pull_ns(mA - kLag, ns);
      const PhiGrad g1 = stageG(mA - kLag);
      pull_ch(mA + 2, next);
      halo_pull(mA + 2, hv);
      stageB(mA - 1);
      __syncthreads();
      stageC(mA - kLag, held, ns, g1);
    };
    pull_ch(ry - kRamp, bufA);
    halo_pull(ry - kRamp, hv);
    for (int j = 0; j < J; j += 3) {  // j is uniform over the block
      iteration(j, bufA, bufB, bufC);
      if (j + 1 < J) iteration(j + 1, bufB, bufC, bufA);
      if (j + 2 < J) iteration(j + 2, bufC, bufA, bufB);
    }
  } else {
    Pulled<M, Real> bufA, bufB;  // pulled for mA (cur) and for mA - 2 (held)
    Real hv[kHP];
    auto iteration = [&](int j, Pulled<M, Real> &cur, const Pulled<M, Real> &held) {
      const int mA = 2 * j - kRamp + ry;
      pull_ch(mA, cur);
      halo_pull(mA, hv);
      stageA(mA, cur);
      halo_phi(mA, hv);
      __syncthreads();
      pull_ns(mA - kLag, ns);
      const PhiGrad g1 = stageG(mA - kLag);
      stageB(mA - 1);
      __syncthreads();
      stageC(mA - kLag, held, ns, g1);
    };
    for (int j = 0; j < J; j += 2) {  // j is uniform over the block
      iteration(j, bufA, bufB);
      if (j + 1 < J) iteration(j + 1, bufB, bufA);
    }
  }
}

// This translation unit instantiates the kernel for one scheme, NPL_GS (0
// central, 1 mixed, 2 Remark 1; step_kernel_mixed.hip and
// step_kernel_remark1.hip build the last two), so the three sets of
// instantiations compile in parallel.
#ifndef NPL_GS
#define NPL_GS 0
#endif

// LDS of one workgroup: the phi and C rings of (N-1) x row-width values
// (rows of interior lanes have kBW + 4 columns), plus the product and
// velocity rings of the Remark 1 scheme
constexpr int lds_bytes(int N, int bytes, int bw, int gs) {
  return ((gs == 1 ? Scheme<1>::kPR + Scheme<1>::kCR
                   : (gs == 2 ? Scheme<2>::kPR + Scheme<2>::kCR : Scheme<0>::kPR + Scheme<0>::kCR)) *
              (N - 1) +
          (gs == 2 ? 4 * kQR + 2 * kUR : 0)) *
         (interior_lanes(N, bytes, gs) ? bw + 2 * (gs ? Scheme<1>::kHalo : Scheme<0>::kHalo) : bw) *
         bytes;
}
// LDS budget of a workgroup: 64 KiB for the central scheme; 80 KiB for the
// others (gfx950 has 160 KiB per CU, so two such workgroups still fit)
constexpr int lds_budget(int gs) { return gs ? 80 * 1024 : 64 * 1024; }
// the widest row a (N, precision, scheme) is built for
constexpr int max_bw(int N, int bytes, int gs) {
  return lds_bytes(N, bytes, 256, gs) <= lds_budget(gs)
             ? 256
             : (lds_bytes(N, bytes, 128, gs) <= lds_budget(gs) ? 128 : 64);
}

#if NPL_GS == 0
int step_max_bw(int N, int precision, int scheme) {
  return max_bw(N, precision == 64 ? 8 : 4, scheme);
}
#endif

namespace {

template <int N, int BW>
hipError_t launch_nb(int precision, const StepArgs &a, int nblocks, hipStream_t st) {
  if (precision == 64) {
    if constexpr (BW <= max_bw(N, 8, NPL_GS))
      hipLaunchKernelGGL((k_step<N, double, BW, NPL_GS>), dim3(nblocks), dim3(BW * kRows), 0,
                         st, a);
    else
      return hipErrorInvalidValue;
  } else {
    if constexpr (BW <= max_bw(N, 4, NPL_GS))
      hipLaunchKernelGGL((k_step<N, float, BW, NPL_GS>), dim3(nblocks), dim3(BW * kRows), 0,
                         st, a);
    else
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N>
hipError_t launch_n(int precision, int bw, const StepArgs &a, int nblocks, hipStream_t st) {
  return bw == 256   ? launch_nb<N, 256>(precision, a, nblocks, st)
         : bw == 128 ? launch_nb<N, 128>(precision, a, nblocks, st)
                     : launch_nb<N, 64>(precision, a, nblocks, st);
}

template <int N, int BW>
int occ_nb(int precision) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  if (precision == 64) {
    if constexpr (BW <= max_bw(N, 8, NPL_GS))
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step<N, double, BW, NPL_GS>,
                                                       BW * kRows, 0);
  } else {
    if constexpr (BW <= max_bw(N, 4, NPL_GS))
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step<N, float, BW, NPL_GS>,
                                                       BW * kRows, 0);
  }
  return e == hipSuccess ? nb : 0;
}

template <int N>
int occ_n(int precision, int bw) {
  return bw == 256 ? occ_nb<N, 256>(precision)
                   : (bw == 128 ? occ_nb<N, 128>(precision) : occ_nb<N, 64>(precision));
}

}  // namespace

#if NPL_GS == 0
#define NPL_SCHEME_FN(name) name##_central
#elif NPL_GS == 1
#define NPL_SCHEME_FN(name) name##_mixed
#else
#define NPL_SCHEME_FN(name) name##_remark1
#endif

int NPL_SCHEME_FN(step_blocks_per_cu)(int N, int precision, int bw) {
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

hipError_t NPL_SCHEME_FN(launch_step)(int N, int precision, int bw, const StepArgs &a,
                                      int nblocks, hipStream_t st) {
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

#if NPL_GS == 0
int step_blocks_per_cu(int N, int precision, int scheme, int bw) {
  return scheme == kSchemeMixed     ? step_blocks_per_cu_mixed(N, precision, bw)
         : scheme == kSchemeRemark1 ? step_blocks_per_cu_remark1(N, precision, bw)
                                    : step_blocks_per_cu_central(N, precision, bw);
}

hipError_t launch_step(int N, int precision, int scheme, int bw, const StepArgs &a, int nblocks,
                       hipStream_t st) {
  return scheme == kSchemeMixed     ? launch_step_mixed(N, precision, bw, a, nblocks, st)
         : scheme == kSchemeRemark1 ? launch_step_remark1(N, precision, bw, a, nblocks, st)
                                    : launch_step_central(N, precision, bw, a, nblocks, st);
}
#endif

}  // namespace nplbm

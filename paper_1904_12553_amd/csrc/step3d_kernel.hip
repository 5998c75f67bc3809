// step3d_kernel.hip -- one time step of the N-phase phase-field LB model
// (arXiv:1904.12553) on the D3Q15 lattice of Sec. 3.1, for gfx950.
//
// The arithmetic per node is that of the 2-D kernel (step_kernel.hip) with
// three velocity components: pull streaming, phi_i by eq:N28 (the stored
// k = 0 value is the deviation h_0 - phi_prev, phi carried as the unevaluated
// sum phi_prev + (d + sum h_k)), closure eq:N18, C_i with the eq:N31b
// Laplacian, F and J~ from the eq:N31a gradients, u by eq:N22_1, p by
// eq:N23, NS collision eq:24 / eq:25 / eq:N20_1, CH collisions
// eq:N24-N27.  Only eq:N31a's central stencils and eq:N20_1 are built in 3-D.
//
// Two passes per step.  The phi pass (k_phi3) pulls the CH populations of
// every node once -- streaming fused into the load, bounce-back at z walls
// -- and writes phi_i to a dense array.  The step pass (k_step3) then owns
// a tile of interior nodes [x0, x1) x [y0, y1) (at most 64 x TY, x0 a
// multiple of 64, so loads and stores are whole cache lines) and marches
// through the planes [z0, z1) with one 64-lane wave per interior row; four
// lanes of each row bring in the 2-column x-halos and four waves the 2-row
// y-halos, so every wave collides.  Each iteration copies phi of plane mA
// from the array into a 5-plane LDS ring (all threads; the next plane's
// values are loaded right after, so they are in flight during the rest of
// the iteration); computes C of plane mA - 1 on the tile plus a ring of one
// into a 4-plane ring; and collides plane mA - 2 on the interior with the
// populations it pulls for that node, issued at the start of the iteration.
// The halo rings thus cost (N - 1) reads per node of the phi array (mostly
// from the 256 MB MALL, where the phi pass left it) instead of 16 (N - 1)
// population reads, and no population is read twice by the step pass.
// D3Q15 stencils reach the six faces and eight corners of a node, so the
// halo is two nodes for phi and one for C, as in 2-D.
//
// Stencils on D3Q15 (eq:N31 with the weights 1/9 and 1/72, c_s^2 = 1/3):
//   lap   = (8 sum_faces + sum_corners - 56 zeta) / 12
//   d/dx  = (8 (E - W) + sum_corners c_x zeta) / 24     (likewise y, z)
#include <cstdlib>
#include <type_traits>

#include "buffer_io.h"
#include "lattice3.h"
#include "nplbm_internal.h"

namespace nplbm {

#define NPL_CONST __attribute__((address_space(4)))

namespace {

constexpr int k3W = 64;   // threads per tile row (one wave) = interior columns of a tile
constexpr int k3L = 68;   // LDS row: the 64 columns plus 2 halo columns each side
constexpr int k3PR = 5;   // phi ring planes
constexpr int k3CR = 4;   // C ring planes

template <typename Real>
__device__ __forceinline__ const NPL_CONST Consts<Real> *consts3(const NPL_CONST DomDesc *d);
template <>
__device__ __forceinline__ const NPL_CONST Consts<double> *consts3<double>(
    const NPL_CONST DomDesc *d) {
  return &d->cd;
}
template <>
__device__ __forceinline__ const NPL_CONST Consts<float> *consts3<float>(
    const NPL_CONST DomDesc *d) {
  return &d->cf;
}

// what the collision of one node reads: CH populations pulled (k = 0: the
// stored deviation), stored previous phi, NS populations k = 1..14 pulled,
// stored previous u
template <int M, typename Real>
struct Col3 {
  Real h[M][15];
  Real hi[M];
  Real g[15];
  Real pu[3];
};

__device__ __forceinline__ int wrap_i(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

template <int N, typename Real, int TY>
__global__ void __launch_bounds__(k3W * TY) k_step3(StepArgs a) {
  constexpr int M = N - 1;
  // FP64 at N = 4 on 8-row tiles: the LDS rings (163 200 B) leave room for
  // one 8-wave workgroup per CU, two waves per SIMD, if the registers fit in
  // 256.  To get there this variant keeps fewer values live: each phase's
  // previous phi is loaded with its CH pulls, the collision re-reads phi_i
  // and C_i from LDS rather than holding them, the chemical-potential
  // stencil is one inline copy, and the next plane's phi values are loaded
  // after the collision rather than held through it.  Three moving spheres
  // at 192^3: 2.04 ms (45.0% of the HBM roofline) against 2.26 ms (40.7%)
  // on 4-row tiles at one wave per SIMD.  The same changes measured slower
  // on every other variant (up to 9%), which keep the plain code.
  constexpr bool kLean = sizeof(Real) == 8 && N == 4 && TY == 8;
  const NPL_CONST TileDesc3 *tp = (const NPL_CONST TileDesc3 *)a.strips + blockIdx.x;
  const int dom = tp->dom;
  if (dom < 0) return;
  const int x0 = tp->x0, x1 = tp->x1, y0 = tp->y0, y1 = tp->y1, z0 = tp->z0, z1 = tp->z1;
  const int dir = tp->dir;
  const NPL_CONST DomDesc *D = (const NPL_CONST DomDesc *)a.doms + dom;
  if (a.substep >= D->steps_left) return;
  const int par = (a.substep + D->parity0) & 1;
  const void *hs = D->h[par], *hd = D->h[par ^ 1];
  const void *gs = D->g[par], *gd = D->g[par ^ 1];
  const void *pvs = D->prev[par], *pvd = D->prev[par ^ 1];
  const NPL_CONST Consts<Real> &K = *consts3<Real>(D);
  // the NS part of the collision in FP64 arithmetic in both modes (FP32
  // populations stay FP32): FP32 rounding there biases each node's momentum
  // in the same direction wherever the flow state repeats
  using Acc = double;
  const NPL_CONST Consts<double> &KD = *consts3<double>(D);
  const int nx = D->nx, ny = D->ny, nz = D->nz;
  const bool wall = D->wall != 0;
  constexpr uint32_t SZ = sizeof(Real);
  const uint32_t pb = (uint32_t)D->ps[0] * SZ;
  const uint32_t rbh = (uint32_t)D->rs[0] * SZ, rbg = (uint32_t)D->rs[1] * SZ,
                 rbp = (uint32_t)D->rs[2] * SZ;

  // rows of the rings: phi on the TY interior rows and 2 halo rows each
  // side, C on the interior rows and 1 each side
  constexpr int kPRows = TY + 4, kCRows = TY + 2;
  __shared__ Real sphi[k3PR][M][kPRows][k3L];
  __shared__ Real sC[k3CR][M][kCRows][k3L];

  const int lane = threadIdx.x & (k3W - 1);
  const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x / k3W);  // uniform
  const int nxi = x1 - x0, nyi = y1 - y0;
  // Columns: lane l owns interior column x0 + l (tiles start on whole
  // cache lines, so every row of loads and stores is line-aligned) at LDS
  // column l + 2; lanes 0..3 also bring the halo columns x0 - 2, x0 - 1,
  // x0 + 64, x0 + 65 (LDS columns 0, 1, 66, 67) into the phi ring.
  const int xc = wrap_i(x0 + lane, nx);
  const int col = lane + 2;
  const int hcol = lane < 2 ? lane : 64 + lane;  // halo LDS column (lanes < 4)
  const uint32_t xh = (uint32_t)wrap_i(lane < 2 ? x0 - 2 + lane : x0 + 62 + lane, nx) * SZ;
  const uint32_t xcu = (uint32_t)xc * SZ;
  const uint32_t xw = (uint32_t)(xc == 0 ? nx - 1 : xc - 1) * SZ;  // x - 1
  const uint32_t xe = (uint32_t)(xc == nx - 1 ? 0 : xc + 1) * SZ;  // x + 1
  // Rows: wave w owns interior row y0 + w (phi ring row w + 2, C ring row
  // w + 1); waves 0..3 also bring the halo rows y0 - 2, y0 - 1, y0 + TY,
  // y0 + TY + 1 (phi ring rows 0, 1, TY + 2, TY + 3), and waves 0, 1
  // compute C of rows y0 - 1 and y0 + TY.  In a ragged tile (nyi < TY) the
  // waves past the interior hold the halo rows below it, as the lanes past
  // a ragged x end do.
  const int yc = wrap_i(y0 + ty, ny);                                // uniform
  const int yS = yc == 0 ? ny - 1 : yc - 1, yN = yc == ny - 1 ? 0 : yc + 1;
  const int pr = ty + 2, cr = ty + 1;                                // ring rows
  const bool lane_int = lane < nxi;
  const bool row_int = ty < nyi;                                     // uniform
  const bool hrow = ty < 4;                                          // uniform
  const int yh = wrap_i(ty < 2 ? y0 - 2 + ty : y0 + TY - 2 + ty, ny);
  const int prh = ty < 2 ? ty : TY + ty;                             // its ring row
  const int H = z1 - z0;

  auto plane_of = [&](int m) { return dir > 0 ? z0 + m : z1 - 1 - m; };
  // physical plane of a (possibly ghost) plane index: mirror beyond a wall,
  // periodic otherwise
  auto phys_plane = [&](int z) {
    if (wall) {
      if (z < 0) z = -1 - z;
      if (z >= nz) z = 2 * nz - 1 - z;
      z = z < 0 ? 0 : (z >= nz ? nz - 1 : z);
    } else {
      z = wrap_i(z, nz);
    }
    return z;
  };
  auto ring5 = [](int m) { return (m + 16 * k3PR) % k3PR; };
  auto ring4 = [](int m) { return (m + 16 * k3CR) % k3CR; };

  // Addressing.  A buffer resource spans one plane block of a group (its ny
  // row blocks); the row is a scalar byte offset fixed for the whole march
  // (the tile's rows do not change), the plane offset another scalar, and
  // the column the per-lane offset.
  const uint32_t ybh[3] = {(uint32_t)yS * rbh, (uint32_t)yc * rbh, (uint32_t)yN * rbh};
  const uint32_t ybg[3] = {(uint32_t)yS * rbg, (uint32_t)yc * rbg, (uint32_t)yN * rbg};
  const uint32_t ybp = (uint32_t)yc * rbp;
  const uint32_t plh = (uint32_t)ny * rbh, plg = (uint32_t)ny * rbg, plp = (uint32_t)ny * rbp;

  // Sources of the populations arriving at plane zp: plane zp - c_z, or the
  // node itself with the opposite direction when that plane lies beyond a
  // wall (bounce-back).  Index 0 / 1 / 2 = plane zp - 1 / zp / zp + 1.
  struct Planes {
    Rsrc r[3];
    bool bS, bN;  // bounce for c_z = +1 / c_z = -1
  };
  auto planes_of = [&](const void *base, uint32_t pl, int zp) {
    Planes P;
    P.bS = wall && zp == 0;
    P.bN = wall && zp == nz - 1;
    P.r[0] = row_rsrc(base, pl, zp == 0 ? nz - 1 : zp - 1);
    P.r[1] = row_rsrc(base, pl, zp);
    P.r[2] = row_rsrc(base, pl, zp == nz - 1 ? 0 : zp + 1);
    return P;
  };
  // load plane q0 + kk of direction k (kk = k, or its opposite when
  // bounced).  Bounce-back happens only on the two planes next to a wall,
  // so the callers take a branch-free path (kWall false) everywhere else.
  auto pull = [&](const Planes &P, const uint32_t (&yb)[3], int k, int q0, auto kWall) {
    const int cx = ex3(k), cy = ey3(k), cz = ez3(k);
    const uint32_t col = cx == 1 ? xw : (cx == -1 ? xe : xcu);
    if (!decltype(kWall)::value || cz == 0)
      return bld<Real>(P.r[1 - cz], col, yb[1 - cy] + (uint32_t)(q0 + k) * pb);
    const bool b = cz == 1 ? P.bS : P.bN;
    const Rsrc r = b ? P.r[1] : P.r[cz == 1 ? 0 : 2];
    const uint32_t so = b ? yb[1] + (uint32_t)(q0 + opp3(k)) * pb
                          : yb[1 - cy] + (uint32_t)(q0 + k) * pb;
    return bld<Real>(r, b ? xcu : col, so);
  };
  // run f(kWall) with kWall a compile-time flag: does plane zp border a wall?
  auto by_wall = [&](const Planes &P, auto f) {
    if (P.bS || P.bN)
      f(std::true_type());
    else
      f(std::false_type());
  };

  // ---- pull what the collision of march index m reads ----
  // CH populations of phase i
  auto pull_phase = [&](int m, int i, Col3<M, Real> &C) {
    const Planes P = planes_of(hs, plh, phys_plane(plane_of(m)));
    by_wall(P, [&](auto kWall) {
#pragma unroll
      for (int k = 0; k < 15; ++k) C.h[i][k] = pull(P, ybh, k, i * 15, kWall);
    });
    if constexpr (kLean)
      C.hi[i] = bld<Real>(row_rsrc(pvs, plp, phys_plane(plane_of(m))), xcu,
                          ybp + (uint32_t)i * pb);
  };
  // NS populations (planes k - 1), stored previous phi and u
  auto pull_ns = [&](int m, Col3<M, Real> &C) {
    const int zp = phys_plane(plane_of(m));
    const Planes P = planes_of(gs, plg, zp);
    by_wall(P, [&](auto kWall) {
#pragma unroll
      for (int k = 1; k < 15; ++k) C.g[k] = pull(P, ybg, k, -1, kWall);
    });
    const Rsrc rp = row_rsrc(pvs, plp, zp);
    if constexpr (!kLean)
#pragma unroll
      for (int i = 0; i < M; ++i) C.hi[i] = bld<Real>(rp, xcu, ybp + (uint32_t)i * pb);
#pragma unroll
    for (int d = 0; d < 3; ++d) C.pu[d] = bld<Real>(rp, xcu, ybp + (uint32_t)(M + d) * pb);
  };
  auto pull_col = [&](int m, Col3<M, Real> &C) {
#pragma unroll
    for (int i = 0; i < M; ++i) pull_phase(m, i, C);
    pull_ns(m, C);
  };

  // ---- stage A: phi of march index mA (from the phi pass) -> LDS ----
  // all threads; the values of plane mA + 1 are loaded right after, so they
  // are in flight during the rest of the iteration
  const uint32_t rbf = (uint32_t)D->rsf * SZ, plf = (uint32_t)ny * rbf;
  const uint32_t ybf = (uint32_t)yc * rbf, ybfh = (uint32_t)yh * rbf;
  const void *phi3 = D->phi3;
  // the values of the own row (f: column, fh: x-halo column of lanes < 4)
  // and of the halo row of waves 0..3 (g, gh)
  struct PhiRow {
    Real f[M], fh[M], g[M], gh[M];
  };
  auto load_phi = [&](int mA, PhiRow &F) {
    const Rsrc r = row_rsrc(phi3, plf, phys_plane(plane_of(mA)));
#pragma unroll
    for (int i = 0; i < M; ++i) {
      F.f[i] = bld<Real>(r, xcu, ybf + (uint32_t)i * pb);
      F.fh[i] = bld<Real>(r, xh, ybf + (uint32_t)i * pb);
    }
    if (hrow)
#pragma unroll
      for (int i = 0; i < M; ++i) {
        F.g[i] = bld<Real>(r, xcu, ybfh + (uint32_t)i * pb);
        F.gh[i] = bld<Real>(r, xh, ybfh + (uint32_t)i * pb);
      }
  };
  auto stageA = [&](int mA, const PhiRow &F) {
    const int slot = ring5(mA);
#pragma unroll
    for (int i = 0; i < M; ++i) sphi[slot][i][pr][col] = F.f[i];
    if (lane < 4)
#pragma unroll
      for (int i = 0; i < M; ++i) sphi[slot][i][pr][hcol] = F.fh[i];
    if (hrow) {
#pragma unroll
      for (int i = 0; i < M; ++i) sphi[slot][i][prh][col] = F.g[i];
      if (lane < 4)
#pragma unroll
        for (int i = 0; i < M; ++i) sphi[slot][i][prh][hcol] = F.gh[i];
    }
  };

  // ---- stage B: chemical potentials of march index mB -> LDS ----
  // On the tile plus a ring of one: LDS columns 1 .. nxi + 2, taken as
  // lane + 1 and, for the last two, 65 + lane.  Planes beyond a wall are
  // skipped: the collision next to the wall reads its own plane for the
  // mirror ghost.
  constexpr bool kOneCopy = N >= 5 || kLean;
  auto chem_at = [&](int q, int c, int s0, int sU, int sD, int sc) {
    const int ty = q + 1;  // phi ring row of C ring row q
    Real phi[M], lap[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const Real v = sphi[s0][i][ty][c];
      const Real faces = (sphi[s0][i][ty][c + 1] + sphi[s0][i][ty][c - 1]) +
                         (sphi[s0][i][ty + 1][c] + sphi[s0][i][ty - 1][c]) +
                         (sphi[sU][i][ty][c] + sphi[sD][i][ty][c]);
      const Real corners =
          ((sphi[sU][i][ty + 1][c + 1] + sphi[sU][i][ty + 1][c - 1]) +
           (sphi[sU][i][ty - 1][c + 1] + sphi[sU][i][ty - 1][c - 1])) +
          ((sphi[sD][i][ty + 1][c + 1] + sphi[sD][i][ty + 1][c - 1]) +
           (sphi[sD][i][ty - 1][c + 1] + sphi[sD][i][ty - 1][c - 1]));
      lap[i] = (Real(8) * faces + corners - Real(56) * v) * (Real(1) / Real(12));  // eq:N31b
      phi[i] = v;
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
      sC[sc][i][q][c] = Ci;
    }
  };
  // the C ring rows of a wave: its own (row y0 + w) while w <= nyi, and for
  // waves 0 / 1 rows y0 - 1 / y0 + TY
  //
  // At N = 5 the stencil code is kept to one inline copy (loops over the
  // rows and columns to evaluate): left to itself the compiler called it
  // out of line, and the call and its stack frame cost 16% of the step
  // (256^3 FP32: 3.56 against 3.00 ms).  Smaller N inline three copies.
  auto chem_row = [&](int q, int s0, int sU, int sD, int sc) __attribute__((always_inline)) {
    if constexpr (kOneCopy) {
#pragma unroll 1
      for (int pass = 0; pass < 2; ++pass) {
        const int c = pass == 0 ? lane + 1 : 65 + lane;
        if (c <= nxi + 2 && (pass == 0 || lane < 2)) chem_at(q, c, s0, sU, sD, sc);
      }
    } else {
      if (lane + 1 <= nxi + 2) chem_at(q, lane + 1, s0, sU, sD, sc);
      if (lane < 2 && 65 + lane <= nxi + 2) chem_at(q, 65 + lane, s0, sU, sD, sc);
    }
  };
  auto stageB = [&](int mB) {
    if (wall) {
      const int z = plane_of(mB);
      if (z < 0 || z >= nz) return;
    }
    const int s0 = ring5(mB), sU = ring5(mB + dir), sD = ring5(mB - dir), sc = ring4(mB);
    if constexpr (kOneCopy) {
      // this wave's C rows: its own while it has one, and a halo row for
      // waves 0 and 1 (uniform over the wave)
      const int qa = ty <= nyi ? cr : -1;
      const int qb = ty == 0 ? 0 : (ty == 1 && nyi == TY ? TY + 1 : -1);
#pragma unroll 1
      for (int pass = 0; pass < 2; ++pass) {
        const int q = pass == 0 ? qa : qb;
        if (q >= 0) chem_row(q, s0, sU, sD, sc);
      }
    } else {
      if (ty <= nyi) chem_row(cr, s0, sU, sD, sc);
      if (ty == 0) chem_row(0, s0, sU, sD, sc);
      if (ty == 1 && nyi == TY) chem_row(TY + 1, s0, sU, sD, sc);
    }
  };

  // eq:N31a on D3Q15 from an LDS ring: planes s0 (own), sU (z + 1), sD (z - 1)
  // around LDS column `lane` (2 .. 65)
  auto grad3 = [&](auto f, int ty, int lane, int s0, int sU, int sD, int i, Real &gx, Real &gy,
                   Real &gz) {
    const Real upp = f[sU][i][ty + 1][lane + 1], upm = f[sU][i][ty + 1][lane - 1];
    const Real ump = f[sU][i][ty - 1][lane + 1], umm = f[sU][i][ty - 1][lane - 1];
    const Real dpp = f[sD][i][ty + 1][lane + 1], dpm = f[sD][i][ty + 1][lane - 1];
    const Real dmp = f[sD][i][ty - 1][lane + 1], dmm = f[sD][i][ty - 1][lane - 1];
    const Real cx = ((upp - upm) + (ump - umm)) + ((dpp - dpm) + (dmp - dmm));
    const Real cy = ((upp + upm) - (ump + umm)) + ((dpp + dpm) - (dmp + dmm));
    const Real cz = ((upp + upm) + (ump + umm)) - ((dpp + dpm) + (dmp + dmm));
    gx = (Real(8) * (f[s0][i][ty][lane + 1] - f[s0][i][ty][lane - 1]) + cx) * (Real(1) / Real(24));
    gy = (Real(8) * (f[s0][i][ty + 1][lane] - f[s0][i][ty - 1][lane]) + cy) * (Real(1) / Real(24));
    gz = (Real(8) * (f[sU][i][ty][lane] - f[sD][i][ty][lane]) + cz) * (Real(1) / Real(24));
  };

  // ---- stage C: collide march index mC (interior rows) ----
  // With kLate the NS pulls are issued here and the CH populations of each
  // phase right before its collision, behind a compiler barrier, so only one
  // phase's populations are live at a time.
  auto stageC = [&](int mC, Col3<M, Real> &P, auto kLate) {
    if constexpr (decltype(kLate)::value) pull_ns(mC, P);
    const int zp = plane_of(mC);
    // ghost planes beyond a wall mirror the boundary plane, which is the
    // collision plane itself; march index mC + dir is plane zp + 1
    const bool gU = wall && zp + 1 >= nz, gD = wall && zp - 1 < 0;
    const int s0 = ring5(mC), c0 = ring4(mC);
    const int sU = gU ? s0 : ring5(mC + dir), sD = gD ? s0 : ring5(mC - dir);
    const int cU = gU ? c0 : ring4(mC + dir), cD = gD ? c0 : ring4(mC - dir);
    // lanes past a ragged tile end compute on their (valid) columns and do
    // not store
    const int ln = col;
    Real phi[M], Cv[M];
    // (the sums over phases of the gradient terms stay in the state type)
    Acc rho = KD.ra;
    Real grs[3] = {Real(0), Real(0), Real(0)}, Fs[3] = {Real(0), Real(0), Real(0)},
         Js[3] = {Real(0), Real(0), Real(0)};
#pragma unroll
    for (int i = 0; i < M; ++i) {
      phi[i] = sphi[s0][i][pr][ln];
      Cv[i] = sC[c0][i][cr][ln];
      Real gp[3], gc[3];
      grad3(sphi, pr, ln, s0, sU, sD, i, gp[0], gp[1], gp[2]);
      grad3(sC, cr, ln, c0, cU, cD, i, gc[0], gc[1], gc[2]);
      rho += KD.rA[i] * phi[i];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        grs[d] += K.rA[i] * gp[d];
        Fs[d] += Cv[i] * gp[d];
        Js[d] += K.Jc[i] * gc[d];
      }
    }
    const Acc gr[3] = {grs[0], grs[1], grs[2]}, J[3] = {Js[0], Js[1], Js[2]};
    Acc F[3] = {Fs[0], Fs[1], Fs[2]};
    F[0] += rho * KD.gx;
    F[1] += rho * KD.gy;
    F[2] += rho * KD.gz;
    Acc itau, srcg, theta;
    if (KD.const_tau) {
      itau = KD.itau_g;
      srcg = KD.src_g;
      theta = KD.theta_g;
    } else {
      Acc mu = KD.ma;
#pragma unroll
      for (int i = 0; i < M; ++i) mu += KD.mA[i] * phi[i];
      const Acc tm = Acc(3) * mu / rho;  // tau_g - 1/2 (eq:N21_1)
      itau = Acc(1) / (Acc(0.5) + tm);
      srcg = Acc(1) - Acc(0.5) * itau;
      theta = Acc(1) / tm;
    }
    const Real(&g)[15] = P.g;  // every use below is promoted to Acc
    Acc m[3] = {Acc(0), Acc(0), Acc(0)}, sumg = Acc(0);
#pragma unroll
    for (int k = 1; k < 15; ++k) {
      if (ex3(k)) m[0] += Acc(ex3(k)) * g[k];
      if (ey3(k)) m[1] += Acc(ey3(k)) * g[k];
      if (ez3(k)) m[2] += Acc(ez3(k)) * g[k];
      sumg += g[k];
    }
    const Acc irho = Acc(1) / rho;
    Acc u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = (m[d] + Acc(0.5) * F[d]) * irho;  // eq:N22_1
    const Acc usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const Acc udr = u[0] * gr[0] + u[1] * gr[1] + u[2] * gr[2];
    // eq:N23 with w_0 = 2/9: c_s^2 / (1 - w_0) = 3/7, rho s_0 = -(1/3) rho |u|^2
    const Acc p = Acc(3) / Acc(7) * (sumg + Acc(0.5) * udr - Acc(1) / Acc(3) * rho * usq);
    const Acc uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    const Acc Ju = J[0] * u[0] + J[1] * u[1] + J[2] * u[2];
    // isotropic part of eq:N20_1: u.grad(rho) - tr(T) / (2 c_s^2)
    const Acc gbase = udr - Acc(1.5) * (Acc(2) * uF + Acc(2) / Acc(3) * udr + theta * Ju);
    if (!lane_int) return;
    const Rsrc wh = row_rsrc(hd, plh, zp), wg = row_rsrc(gd, plg, zp),
               wp = row_rsrc(pvd, plp, zp);
    // eq:24 with g^eq and G split into the parts even and odd in c_k, each
    // pair of opposite directions evaluated once
    const Acc keep = Acc(1) - itau;
    const Acc e0 = Acc(3) * p - Acc(1.5) * rho * usq;
#pragma unroll
    for (int k = 1; k < 15; ++k) {
      if (opp3(k) < k) continue;
      const int ko = opp3(k);
      const Acc cx = Acc(ex3(k)), cy = Acc(ey3(k)), cz = Acc(ez3(k));
      const Acc w = w3<Acc>(k);
      const Acc cu = cx * u[0] + cy * u[1] + cz * u[2];
      const Acc cF = cx * F[0] + cy * F[1] + cz * F[2];
      const Acc cr = cx * gr[0] + cy * gr[1] + cz * gr[2];
      const Acc cJ = cx * J[0] + cy * J[1] + cz * J[2];
      const Acc ev =
          w * (itau * (e0 + Acc(4.5) * rho * cu * cu) +
               srcg * (gbase + Acc(4.5) * cu * (Acc(2) * cF + Acc(2) / Acc(3) * cr + theta * cJ)));
      const Acc od = w * Acc(3) * (itau * rho * cu + srcg * cF);
      bst<Real, true>(wg, xcu, ybg[1] + (uint32_t)(k - 1) * pb, keep * g[k] + ev + od);
      bst<Real, true>(wg, xcu, ybg[1] + (uint32_t)(ko - 1) * pb, keep * g[ko] + ev - od);
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
      Real phii = phi[i], Cvi = Cv[i];
      if constexpr (decltype(kLate)::value) {
        asm volatile("" ::: "memory");
        pull_phase(mC, i, P);
        // plane mC's slots of the phi and C rings are rewritten only two
        // iterations later, so these are the values read above
        if constexpr (kLean) {
          phii = sphi[s0][i][pr][ln];
          Cvi = sC[c0][i][cr][ln];
        }
      }
      const Real pp = P.hi[i];
      Real ps[3], dd[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        ps[d] = phii * u[d];
        dd[d] = ps[d] - pp * P.pu[d];  // eq:N27
      }
      const Real ec = K.eta_i[i] * Cvi;
      const Real it = K.itau_i[i], sr = K.src_i[i];
      // eq:N24 with h^eq (eq:N25) and R_k (eq:N26) split into the parts
      // even and odd in c_k, per pair of opposite directions
      const Real keep = Real(1) - it;
      Real hsum = Real(0);
#pragma unroll
      for (int k = 1; k < 15; ++k) {
        if (opp3(k) < k) continue;
        const int ko = opp3(k);
        const Real cx = Real(ex3(k)), cy = Real(ey3(k)), cz = Real(ez3(k));
        const Real w = w3<Real>(k);
        const Real ev = it * w * ec;
        const Real od = w * Real(3) *
                        (it * (cx * ps[0] + cy * ps[1] + cz * ps[2]) +
                         sr * (cx * dd[0] + cy * dd[1] + cz * dd[2]));
        const Real hn = keep * P.h[i][k] + ev + od;
        const Real ho = keep * P.h[i][ko] + ev - od;
        hsum += hn + ho;
        bst<Real, true>(wh, xcu, ybh[1] + (uint32_t)(i * 15 + k) * pb, hn);
        bst<Real, true>(wh, xcu, ybh[1] + (uint32_t)(i * 15 + ko) * pb, ho);
      }
      // phi_i = pp + lo exactly; fl(phi_i) is stored as the new previous
      // phi and the k = 0 slot keeps (pp + lo - fl(phi_i)) - sum h_k
      Real lo = P.h[i][0];
#pragma unroll
      for (int k = 1; k < 15; ++k) lo += P.h[i][k];
      const Real bb = phii - pp;
      const Real err = (pp - (phii - bb)) + (lo - bb);
      bst<Real, true>(wh, xcu, ybh[1] + (uint32_t)(i * 15) * pb, err - hsum);
      bst<Real, true>(wp, xcu, ybp + (uint32_t)i * pb, phii);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) bst<Real, true>(wp, xcu, ybp + (uint32_t)(M + d) * pb, u[d]);
  };

  // March: iteration j pulls plane mA = j - 2, computes C of mA - 1 and
  // collides mA - 2, so J = H + 4 iterations cover the interior planes.
  // The collision's own pulls are issued before stage A where the registers
  // allow it (held through two barriers); FP64 with N >= 3 spills that way,
  // so there they are issued at the collision (256^3 N = 3 FP64: 49.9%
  // against 44.9% of the HBM roofline; FP32 measured slower late).
  constexpr bool kEarly = !(sizeof(Real) == 8 && N >= 3);
  const int J = H + 4;
  PhiRow fr;
  load_phi(-2, fr);
  for (int j = 0; j < J; ++j) {  // j is uniform over the block
    const int mA = j - 2;
    const int mC = mA - 2;
    const bool collide = row_int && mC >= 0 && mC < H;  // uniform
    Col3<M, Real> col;
    if constexpr (kEarly)
      if (collide) pull_col(mC, col);
    stageA(mA, fr);
    if constexpr (!kLean) load_phi(mA + 1, fr);
    __syncthreads();
    stageB(mA - 1);
    __syncthreads();
    if (collide) stageC(mC, col, std::integral_constant<bool, !kEarly>());
    if constexpr (kLean) load_phi(mA + 1, fr);
  }
}

// The phi pass: phi_i = phi_prev + (d + sum_{k>=1} h_k) (eq:N28, the
// pulled populations and the stored deviation of h_0) of every node of the
// domain into the phi array.  One 64-lane wave per row segment of 64 nodes,
// four rows per workgroup; no halo, so every population is read once.
//
// Blocks are numbered for the 8 XCDs: hardware block b runs on XCD b % 8,
// and XCD x takes the x-th contiguous eighth of the (x, y, z)-ordered block
// list, in order.  Blocks next to each other in x then run on one XCD at
// about the same time, so the cache line that two of them pull from (the
// one holding the column left or right of a 64-column segment) comes from
// that XCD's L2 the second time.
template <int N, typename Real>
__global__ void __launch_bounds__(256) k_phi3(StepArgs a) {
  constexpr int M = N - 1;
  const NPL_CONST DomDesc *D = (const NPL_CONST DomDesc *)a.doms;
  if (a.substep >= D->steps_left) return;
  const int par = (a.substep + D->parity0) & 1;
  const void *hs = D->h[par], *pvs = D->prev[par];
  const int nx = D->nx, ny = D->ny, nz = D->nz;
  const bool wall = D->wall != 0;
  constexpr uint32_t SZ = sizeof(Real);
  const uint32_t pb = (uint32_t)D->ps[0] * SZ;
  const uint32_t rbh = (uint32_t)D->rs[0] * SZ, rbp = (uint32_t)D->rs[2] * SZ,
                 rbf = (uint32_t)D->rsf * SZ;
  const int gx = (nx + k3W - 1) / k3W, gy = (ny + 3) / 4;
  const int nblk = gx * gy * nz, per = (nblk + 7) / 8;
  const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (t >= nblk) return;
  const int bx = t % gx, by = (t / gx) % gy;
  const int lane = threadIdx.x & (k3W - 1);
  const int y = by * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / k3W);  // uniform
  const int z = t / (gx * gy);
  const int x = bx * k3W + lane;
  if (y >= ny || x >= nx) return;
  const uint32_t xcu = (uint32_t)x * SZ;
  const uint32_t xw = (uint32_t)(x == 0 ? nx - 1 : x - 1) * SZ;
  const uint32_t xe = (uint32_t)(x == nx - 1 ? 0 : x + 1) * SZ;
  const int yS = y == 0 ? ny - 1 : y - 1, yN = y == ny - 1 ? 0 : y + 1;
  const uint32_t yb[3] = {(uint32_t)yS * rbh, (uint32_t)y * rbh, (uint32_t)yN * rbh};
  const uint32_t plh = (uint32_t)ny * rbh;
  const bool bS = wall && z == 0, bN = wall && z == nz - 1;
  const Rsrc r0 = row_rsrc(hs, plh, z == 0 ? nz - 1 : z - 1);
  const Rsrc r1 = row_rsrc(hs, plh, z);
  const Rsrc r2 = row_rsrc(hs, plh, z == nz - 1 ? 0 : z + 1);
  const Rsrc rp = row_rsrc(pvs, (uint32_t)ny * rbp, z);
  Real f[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    Real lo = Real(0);
#pragma unroll
    for (int k = 0; k < 15; ++k) {
      const int cx = ex3(k), cy = ey3(k), cz = ez3(k);
      const bool b = (cz == 1 && bS) || (cz == -1 && bN);
      const Rsrc r = b ? r1 : (cz == 1 ? r0 : (cz == -1 ? r2 : r1));
      const uint32_t col = b ? xcu : (cx == 1 ? xw : (cx == -1 ? xe : xcu));
      const uint32_t so = b ? yb[1] + (uint32_t)(i * 15 + opp3(k)) * pb
                            : yb[1 - cy] + (uint32_t)(i * 15 + k) * pb;
      lo += bld<Real>(r, col, so);
    }
    f[i] = bld<Real>(rp, xcu, (uint32_t)y * rbp + (uint32_t)i * pb) + lo;
  }
  const Rsrc wf = row_rsrc(D->phi3, (uint32_t)ny * rbf, z);
#pragma unroll
  for (int i = 0; i < M; ++i) bst<Real, true>(wf, xcu, (uint32_t)y * rbf + (uint32_t)i * pb, f[i]);
}

template <int N, int TY>
constexpr int lds3_bytes(int bytes) {
  return (k3PR * (TY + 4) + k3CR * (TY + 2)) * (N - 1) * k3L * bytes;
}

template <int N>
hipError_t launch_phi3(int precision, const StepArgs &a, dim3 grid, hipStream_t st) {
  if (precision == 64)
    hipLaunchKernelGGL((k_phi3<N, double>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_phi3<N, float>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int N, int TY>
hipError_t launch3(int precision, const StepArgs &a, int nblocks, hipStream_t st) {
  if (precision == 64) {
    if constexpr (lds3_bytes<N, TY>(8) <= 160 * 1024)
      hipLaunchKernelGGL((k_step3<N, double, TY>), dim3(nblocks), dim3(k3W * TY), 0, st, a);
    else
      return hipErrorInvalidValue;
  } else {
    if constexpr (lds3_bytes<N, TY>(4) <= 160 * 1024)
      hipLaunchKernelGGL((k_step3<N, float, TY>), dim3(nblocks), dim3(k3W * TY), 0, st, a);
    else
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N, int TY>
int occ3(int precision) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  if (precision == 64) {
    if constexpr (lds3_bytes<N, TY>(8) <= 160 * 1024)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step3<N, double, TY>, k3W * TY, 0);
  } else {
    if constexpr (lds3_bytes<N, TY>(4) <= 160 * 1024)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step3<N, float, TY>, k3W * TY, 0);
  }
  return e == hipSuccess ? nb : 0;
}

}  // namespace

// Interior rows of a tile = waves of a workgroup: 4 in FP32, where two or
// more 4-row workgroups per CU measured faster than one of 8 (256^3: N = 3
// 48.3% against 44.9% of the HBM roofline, N = 5 38.2% against 35.6%); in
// FP64 8 for N <= 4 (N = 3: 44.9% against 43.9%; N = 4, with the leaner
// register use of that variant: 45.0% against 40.7%) and 4 for N = 5, where
// FP64 rings of 8 rows would not fit in LDS.  NPLBM_TY3 = 4 or 8 overrides.
int step3_ty(int N, int precision) {
  if (const char *e = std::getenv("NPLBM_TY3")) {
    const int t = std::atoi(e);
    const int bytes = precision == 64 ? 8 : 4;
    const int lds = (k3PR * (t + 4) + k3CR * (t + 2)) * (N - 1) * k3L * bytes;
    if (t == 4 || (t == 8 && lds <= 160 * 1024)) return t;
  }
  return precision == 64 && N <= 4 ? 8 : 4;
}

hipError_t launch_step3(int N, int precision, int ty, const StepArgs &a, int nblocks, int nx,
                        int ny, int nz, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  // one block per 64 x 4 row segments of a plane, in a 1-D grid whose
  // size is a multiple of 8 (the phi pass maps block numbers to XCDs)
  const int64_t nphi = (int64_t)((nx + k3W - 1) / k3W) * ((ny + 3) / 4) * nz;
  if (nphi > (int64_t)1 << 30) return hipErrorInvalidValue;
  const dim3 pg((unsigned)((nphi + 7) / 8 * 8));
  hipError_t e;
  switch (N) {
    case 2: e = launch_phi3<2>(precision, a, pg, st); break;
    case 3: e = launch_phi3<3>(precision, a, pg, st); break;
    case 4: e = launch_phi3<4>(precision, a, pg, st); break;
    case 5: e = launch_phi3<5>(precision, a, pg, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (ty == 4) {
    switch (N) {
      case 2: return launch3<2, 4>(precision, a, nblocks, st);
      case 3: return launch3<3, 4>(precision, a, nblocks, st);
      case 4: return launch3<4, 4>(precision, a, nblocks, st);
      case 5: return launch3<5, 4>(precision, a, nblocks, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (N) {
    case 2: return launch3<2, 8>(precision, a, nblocks, st);
    case 3: return launch3<3, 8>(precision, a, nblocks, st);
    case 4: return launch3<4, 8>(precision, a, nblocks, st);
    case 5: return launch3<5, 8>(precision, a, nblocks, st);
    default: return hipErrorInvalidValue;
  }
}

int step3_blocks_per_cu(int N, int precision, int ty) {
  if (ty == 4) {
    switch (N) {
      case 2: return occ3<2, 4>(precision);
      case 3: return occ3<3, 4>(precision);
      case 4: return occ3<4, 4>(precision);
      case 5: return occ3<5, 4>(precision);
      default: return 0;
    }
  }
  switch (N) {
    case 2: return occ3<2, 8>(precision);
    case 3: return occ3<3, 8>(precision);
    case 4: return occ3<4, 8>(precision);
    case 5: return occ3<5, 8>(precision);
    default: return 0;
  }
}

}  // namespace nplbm

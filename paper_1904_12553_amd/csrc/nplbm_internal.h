// nplbm_internal.h -- device-side data structures shared by the host
// library and the gfx950 kernels (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nplbm {

constexpr int kMaxN = 8;          // phases
constexpr int kMaxM = kMaxN - 1;  // order parameters
constexpr int kRows = 2;  // rows per marching iteration (one or more waves per row)
// Row width of a step workgroup in threads (a multiple of the 64-lane wave):
// each row covers the strip's interior columns plus a halo of `halo` columns
// on each side (2 for the central gradients of eq:N31a, 3 for the two-hop
// gradients of eq:N40); lanes beyond that stay idle.
struct StepGeom {
  int bw;    // threads per row (64, 128 or 256)
  int tx;    // maximum interior columns per strip (<= bw, or bw - 2 halo when the rows hold their halo)
  int unit;  // strip widths are multiples of this many columns (one cache line)
  int halo;  // halo columns on each side
};
// Gradient schemes (nplbm_params.grad_scheme): central isotropic (eq:N31a)
// or the isotropic mixed scheme of eq:N40 (sign of its two-hop term read as
// negative).
constexpr int kGradCentral = 0;
constexpr int kGradMixed = 1;
// Step-kernel schemes: central stencils with eq:N20_1, mixed stencils with
// eq:N20_1, central stencils with the force distribution of Remark 1.
constexpr int kSchemeCentral = 0;
constexpr int kSchemeMixed = 1;
constexpr int kSchemeRemark1 = 2;
// Whether every lane of a step-kernel row owns an interior column (the
// x-halo phi then comes from lanes that each pull one population of a halo
// node): the central scheme in FP32 for N <= 5 and in FP64 for N <= 3, the
// mixed and Remark 1 schemes in FP32 for N <= 5.  Elsewhere the rows hold
// their halo columns: with more phases, or in FP64 with the two-hop
// schemes, the extra registers of the halo pull cost more than the wider
// strips gain (FP64 N = 7 spilled).
constexpr bool interior_lanes(int N, int bytes, int scheme) {
  return (scheme == kSchemeCentral && N <= (bytes == 4 ? 5 : 3)) ||
         (scheme != kSchemeCentral && bytes == 4 && N <= 5);
}
// Geometry used for N phases at a precision (32 / 64) and scheme;
// NPLBM_BW and NPLBM_TX override.
StepGeom step_geom(int N, int precision, int scheme);
// widest row width the step kernel is built with for (N, precision, scheme)
int step_max_bw(int N, int precision, int scheme);

// Per-domain constants, folded on the host from the paper's closure so that
// every per-node quantity is an affine map or a short dot product:
//   c_k   = ca[k]  + sum_i cA[k][i] phi_i        (eq:N18, lines 1-2)
//   rho   = ra     + sum_i rA[i]    phi_i        (eq:N18 line 5 / eq:N29)
//   mu    = ma     + sum_i mA[i]    phi_i        (mu = sum_k mu~_k c_k)
//   C_i   = -sum_j lam[i][j] lap phi_j + sum_k KH[k][i] w_k,
//           w_k = c_k (1 - c_k) (1 - 2 c_k)       (eq:N18 line 3 with eq:N17)
//   grad rho = sum_i rA[i] grad phi_i             (linearity of eq:N31a)
//   J~    = sum_i Jc[i] grad C_i                  (eq:N18 line 4)
template <typename Real>
struct Consts {
  Real ca[kMaxN];
  Real cA[kMaxN][kMaxM];
  Real ra, ma;
  Real rA[kMaxM];
  Real mA[kMaxM];
  Real lam[kMaxM][kMaxM];
  Real KH[kMaxN][kMaxM];
  Real Jc[kMaxM];
  Real eta_i[kMaxM];     // eq:N30
  Real itau_i[kMaxM];    // 1 / tau_i
  Real src_i[kMaxM];     // 1 - 1 / (2 tau_i), eq:N26
  Real gx, gy, gz;
  Real itau_g, src_g, theta_g;  // used when tau_g is constant
  int32_t const_tau;
  int32_t pad_;
};

// One resident domain as the kernels see it.
struct DomDesc {
  void *h[2];        // CH populations, [(N-1)][9][ny][pitch], ping-pong; the
                     // k = 0 plane holds h_0 - phi_prev (see below)
  void *g[2];        // NS populations k = 1..8, [8][ny][pitch], ping-pong
  void *prev[2];     // previous-step phi_i (N-1 planes) and u (2 planes), ping-pong
  // Element (plane p, row y, column x) of group G (0: h, 1: g, 2: prev) is at
  // base + p * ps[G] + y * rs[G] + x.  The default layout interleaves planes
  // by row (ps = row pitch, rs = planes x pitch), so the populations one row
  // of nodes needs are one contiguous block.
  int64_t ps[3], rs[3];
  int32_t nx, ny, pitch, wall;
  int32_t N;
  int32_t parity0;   // buffer holding the current state at substep 0
  int32_t steps_left;  // substeps >= steps_left do nothing
  int32_t scheme;      // step-kernel scheme (kSchemeCentral / Mixed / Remark1)
  // Three-dimensional (D3Q15) domains: nz > 1.  Rows are then the (z, y)
  // lines of nodes, row index z * ny + y; groups hold 15 (N-1) CH planes,
  // 14 NS planes (k = 1..14) and (N-1) + 3 previous-step planes; `wall`
  // means halfway bounce-back walls below plane 0 and above plane nz - 1.
  int32_t nz;
  // 3-D: elements per row block of the phi array (M * pitch); the array
  // holds phi_i of the current state, [(z * ny + y)][i][pitch], written by
  // the phi pass and read by the step pass of the same time step
  int32_t rsf;
  void *phi3;
  Consts<double> cd;
  Consts<float> cf;
};

// One strip of the marching step kernel: interior columns [x0, x0 + kTX)
// clipped to nx, interior rows [y0, y1), marched upward (dir = +1) or
// downward (dir = -1).  dom < 0 marks an empty slot.
struct StripDesc {
  int32_t dom;
  int32_t x0, y0, y1;
  int32_t dir;
  int32_t x1;  // end of the interior columns (exclusive, <= nx)
  int32_t pad_[2];
};

// One tile of the 3-D marching step kernel: interior columns [x0, x1),
// interior rows [y0, y1), interior planes [z0, z1) marched upward (dir = +1)
// or downward (dir = -1).  dom < 0 marks an empty slot.  Same size as
// StripDesc, so both live in the same table storage.
struct TileDesc3 {
  int32_t dom;
  int32_t x0, x1, y0, y1, z0, z1;
  int32_t dir;
};
static_assert(sizeof(TileDesc3) == sizeof(StripDesc), "tile and strip records differ");

struct StepArgs {
  const StripDesc *strips;
  const DomDesc *doms;
  int32_t substep;
  int32_t pad_;
};

// Launchers (defined in the .hip files).  All are asynchronous on `st`.
hipError_t launch_step(int N, int precision, int scheme, int bw, const StepArgs &a,
                       int nblocks, hipStream_t st);
// resident step-kernel workgroups per compute unit (0 if unknown)
int step_blocks_per_cu(int N, int precision, int scheme, int bw);
// the same for one scheme (one translation unit each)
hipError_t launch_step_central(int N, int precision, int bw, const StepArgs &a, int nblocks,
                               hipStream_t st);
hipError_t launch_step_mixed(int N, int precision, int bw, const StepArgs &a, int nblocks,
                             hipStream_t st);
hipError_t launch_step_remark1(int N, int precision, int bw, const StepArgs &a, int nblocks,
                               hipStream_t st);
int step_blocks_per_cu_central(int N, int precision, int bw);
int step_blocks_per_cu_mixed(int N, int precision, int bw);
int step_blocks_per_cu_remark1(int N, int precision, int bw);

// The 3-D (D3Q15) step kernel: tiles of (64 - 4) x (ty - 4) interior nodes,
// ty rows of one 64-lane wave each (ty = 8 or 16).
int step3_ty(int N, int precision);
// One 3-D time step: the phi pass over all nx * ny * nz nodes of domain 0
// of a.doms, then the tiled step pass over nblocks tiles.
hipError_t launch_step3(int N, int precision, int ty, const StepArgs &a, int nblocks, int nx,
                        int ny, int nz, hipStream_t st);
int step3_blocks_per_cu(int N, int precision, int ty);
// 3-D initialisation and read-back, the counterparts of launch_init /
// launch_macro below on dense (nz * ny * nx) planes; u has 3 planes.
hipError_t launch_init3(const DomDesc *dd_dev, const DomDesc &dd, int precision,
                        const double *P1, const double *PN, const double *P0,
                        const double *c_dev, const double *u_dev, double *phi_tmp,
                        double *C_tmp, hipStream_t st);
hipError_t launch_macro3(const DomDesc *dd_dev, const DomDesc &dd, int precision, int parity,
                         double *phi, double *rho, double *C, double *c_out, double *u_out,
                         double *p_out, hipStream_t st);

// Initialisation: phi (double, (N-1) planes of nx*ny) is computed from c,
// then C from phi, then h^eq / g^eq written in pull layout.
// phi_i = P1[i] c_i + PN[i] c_N + P0[i] (eq:N12 inverted).
hipError_t launch_init(const DomDesc *dd_dev, const DomDesc &dd, int precision,
                       const double *P1, const double *PN, const double *P0,
                       const double *c_dev, const double *u_dev, double *phi_tmp,
                       double *C_tmp, hipStream_t st);

// Macroscopic fields in FP64 from the current state: phi (N-1), c (N), rho,
// C (N-1), u (2), p.  Any output plane pointer group may be null.
// Dense planes (nx*ny); u/p need the C scratch, and with the Remark 1
// scheme 4 more planes q for the products J~_b u_a.
hipError_t launch_macro(const DomDesc *dd_dev, const DomDesc &dd, int precision, int parity,
                        double *phi, double *rho, double *C, double *c_out, double *u_out,
                        double *p_out, double *q, hipStream_t st);

// FP64 reductions over the c fields (N planes): per-phase sums, max
// |sum c - 1|, non-finite count.  partials must hold nblk*(N+2) doubles.
int diag_blocks(int64_t n);
// Doubles in the static device scratch of the allocation-free diagnostics:
// the partial records of the most blocks diag_blocks() returns, plus the
// final record, at the largest N.
constexpr int kStaticDiagPartials = 1024 * (kMaxN + 2);
constexpr int kStaticDiagDoubles = kStaticDiagPartials + 16;
// Device address of that scratch on the current device (looked up once per
// device with that device current).
hipError_t static_diag_scratch(double **out);
hipError_t launch_diag(const double *c, int N, int64_t n, double *partials, int nblk,
                       double *out, hipStream_t st);
// Laplace jump on a dense FP64 p field of nx * ny * nz nodes (nz = 1 in
// 2-D): mean of p within distance r_in of (xc, yc, zc) minus the mean at
// distance >= r_out.
hipError_t launch_laplace(const double *p, int nx, int ny, int nz, double xc, double yc,
                          double zc, double r_in, double r_out, double *partials, int nblk,
                          double *out, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, size_t nbytes, hipStream_t st);

}  // namespace nplbm

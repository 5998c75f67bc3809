// host_internal.h -- host-side helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "nplbm.h"
#include "nplbm_internal.h"

namespace nplbm {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
void clear_error();
const char *last_error();

// Everything derived on the host from nplbm_params.
struct Derived {
  int N = 0;
  double eta = 0, beta2 = 0, K = 0;
  std::vector<double> lam;         // (N-1) x (N-1)
  double P1[kMaxM] = {0}, PN[kMaxM] = {0}, P0[kMaxM] = {0};  // eq:N12 inverse
  Consts<double> cd;
  Consts<float> cf;
};
int derive(const nplbm_params *p, Derived &d);
// 3-D (D3Q15) domain: nz >= 4; planes in z (1 for a 2-D domain)
inline bool is3d(const nplbm_params *p) { return p->nz > 1; }
inline int dom_nz(const nplbm_params *p) { return p->nz > 1 ? p->nz : 1; }

// Byte offsets of every device buffer of one domain inside its allocation.
struct Layout {
  int pitch = 0;
  int64_t ps[3] = {0, 0, 0}, rs[3] = {0, 0, 0};  // element strides (see DomDesc)
  size_t gbytes[3] = {0, 0, 0};                  // bytes of one copy of each group
  size_t h[2] = {0, 0}, g[2] = {0, 0}, prev[2] = {0, 0}, state_end = 0;
  size_t desc = 0, strips = 0;
  int nstrips = 0;
  size_t phi = 0, rho = 0, C = 0, c = 0, u = 0, p = 0, q = 0;
  size_t phi3 = 0;  // 3-D: phi array of the step (state precision)
  int nblk = 0;
  size_t partials = 0, out = 0;
  size_t total = 0;
};
Layout plan_layout(const nplbm_params *p);
int single_domain_target(const nplbm_params *p);

// default padding of every population plane (64 elements of 4 bytes)
constexpr size_t kPlanePadBytes = 256;
int64_t plane_pad(size_t elem);
// default padding of every row block of the row-interleaved layout
constexpr size_t kRowPadBytes = 0;
int64_t row_pad(size_t elem);
// elements between the planes of one lattice row (the padded row pitch)
int64_t state_pitch(const nplbm_params *p);
// step-kernel scheme (kSchemeCentral / kSchemeMixed / kSchemeRemark1) of a
// validated parameter set
int step_scheme(const nplbm_params *p);
int resident_step_blocks(int N, int precision, int scheme);
void build_strips(int nx, int ny, int dom, const StepGeom &geom, std::vector<StripDesc> &out,
                  int target = 0);
void xcd_order(std::vector<StripDesc> &s);
// tiles of the 3-D step kernel, stored as TileDesc3 records
void build_tiles3(int nx, int ny, int nz, int dom, int ty, int target,
                  std::vector<StripDesc> &out);

}  // namespace nplbm

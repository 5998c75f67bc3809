// lattice.h -- the D2Q9 lattice of Sec. 3.1 as compile-time functions, so
// that every per-direction expression folds to constants after unrolling.
#pragma once

namespace nplbm {

// velocities c_k in the paper's order k = 0..8:
// (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
__host__ __device__ constexpr int cxk(int k) {
  return (k == 1 || k == 5 || k == 8) ? 1 : ((k == 3 || k == 6 || k == 7) ? -1 : 0);
}
__host__ __device__ constexpr int cyk(int k) {
  return (k == 2 || k == 5 || k == 6) ? 1 : ((k == 4 || k == 7 || k == 8) ? -1 : 0);
}
// opposite direction: 1<->3, 2<->4, 5<->7, 6<->8
__host__ __device__ constexpr int oppk(int k) {
  return k == 0 ? 0 : (k <= 4 ? ((k + 1) % 4) + 1 : ((k - 3) % 4) + 5);
}
// weights omega_k: 4/9, 1/9 (axis), 1/36 (diagonal)
template <typename Real>
__host__ __device__ constexpr Real wk(int k) {
  return k == 0 ? Real(4) / Real(9) : (k <= 4 ? Real(1) / Real(9) : Real(1) / Real(36));
}

}  // namespace nplbm

// lattice3.h -- the D3Q15 lattice of Sec. 3.1 as compile-time functions, so
// that every per-direction expression folds to constants after unrolling.
#pragma once

namespace nplbm {

// velocities c_k in the paper's order k = 0..14: rest; +x, +y, +z, -x, -y,
// -z; then the corners (1,1,1) (1,1,-1) (1,-1,1) (-1,1,1) (-1,-1,-1)
// (-1,-1,1) (-1,1,-1) (1,-1,-1)
__host__ __device__ constexpr int ex3(int k) {
  return (k == 1 || k == 7 || k == 8 || k == 9 || k == 14)
             ? 1
             : ((k == 4 || k == 10 || k == 11 || k == 12 || k == 13) ? -1 : 0);
}
__host__ __device__ constexpr int ey3(int k) {
  return (k == 2 || k == 7 || k == 8 || k == 10 || k == 13)
             ? 1
             : ((k == 5 || k == 9 || k == 11 || k == 12 || k == 14) ? -1 : 0);
}
__host__ __device__ constexpr int ez3(int k) {
  return (k == 3 || k == 7 || k == 9 || k == 10 || k == 12)
             ? 1
             : ((k == 6 || k == 8 || k == 11 || k == 13 || k == 14) ? -1 : 0);
}
// opposite direction: the k' with c_k' = -c_k
__host__ __device__ constexpr int opp3(int k) {
  return k == 0 ? 0 : (k <= 3 ? k + 3 : (k <= 6 ? k - 3 : (k <= 10 ? k + 4 : k - 4)));
}
// weights omega_k: 2/9 (rest), 1/9 (faces), 1/72 (corners)
template <typename Real>
__host__ __device__ constexpr Real w3(int k) {
  return k == 0 ? Real(2) / Real(9) : (k <= 6 ? Real(1) / Real(9) : Real(1) / Real(72));
}

}  // namespace nplbm

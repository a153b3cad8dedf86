// common.h -- device-side constants and helpers of the gfx950 library.
//
// Lattice tables follow Sec. 3.1 (D2Q9 velocities and weights in the order
// the paper prints them) and the standard D3Q19 set for the 3D extension the
// paper calls direct.  c_s^2 = 1/3 throughout (normalisation of Sec. 3.1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define LB_HOST_DEVICE __host__ __device__ __forceinline__

// fixed-point scale of the integer accumulators used for every force that is
// summed from many contributions (spreading, coupling force): sums of int64
// are exact and order independent, so the result is bitwise deterministic.
#define FIX_SCALE 281474976710656.0        /* 2^48 */
#define FIX_INV (1.0 / 281474976710656.0)
#define FIX_LIMIT 16384.0                  /* |value| above this is an error */

namespace lb {

template <int Q> struct Lattice;

template <> struct Lattice<9> {
  static constexpr int D = 2;
  static constexpr int cx[9] = {0, 1, -1, 0, 0, 1, -1, -1, 1};
  static constexpr int cy[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
  static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int opp[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
  LB_HOST_DEVICE static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

// D3Q19: rest, faces +-x +-y +-z, edges in the xy, xz, yz planes
template <> struct Lattice<19> {
  static constexpr int D = 3;
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  LB_HOST_DEVICE static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

// Peskin's four-point kernel, eq. DiscreteDirac
LB_HOST_DEVICE double peskin(double r) {
  double a = fabs(r);
  if (a < 1.0) return 0.125 * (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a));
  if (a < 2.0) return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
  return 0.0;
}

LB_HOST_DEVICE int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// wrap(v, n) for a uniform index: one that is at most one period off is
// corrected without a division
LB_HOST_DEVICE int wrap_near(int v, int n) {
  if (v < 0)
    v += n;
  else if (v >= n)
    v -= n;
  return v >= 0 && v < n ? v : wrap(v, n);
}

// row index for finite differences: periodic wrap, or the mirror ghost of a
// wall at -1/2 / n-1/2 (zero normal gradient, eq. NaturalBCs)
LB_HOST_DEVICE int fd_row(int v, int n, int wall) {
  if (!wall) return wrap(v, n);
  if (v < 0) return -1 - v;
  if (v >= n) return 2 * n - 1 - v;
  return v;
}

// fd_row for a row index that is the same across a wavefront
LB_HOST_DEVICE int fd_row_near(int v, int n, int wall) {
  if (!wall) return wrap_near(v, n);
  if (v < 0) return -1 - v;
  if (v >= n) return 2 * n - 1 - v;
  return v;
}

__device__ __forceinline__ long long to_fix(double v) { return __double2ll_rn(v * FIX_SCALE); }
__device__ __forceinline__ double from_fix(long long v) { return (double)v * FIX_INV; }

}  // namespace lb

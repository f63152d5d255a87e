// k_common.h -- small device helpers shared by the kernels of libsedimi.
#pragma once

#include <hip/hip_runtime.h>

#include "sedimi_internal.h"

namespace sedimi {

__device__ __forceinline__ double min_image(double d, double L, double hL) {
  if (d > hL) {
    d -= L;
  } else if (d < -hL) {
    d += L;
  }
  return d;
}

// Squared centre distance and pair range in the exact FP64 association that
// defines the pair set: s = (dx*dx + dy*dy) + dz*dz, R = rs + f*rs, pair iff
// s < R*R.  Contraction into FMAs is switched off here so that the decision
// is bit-identical to a plain IEEE evaluation.
__device__ __forceinline__ double pair_s(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}
__device__ __forceinline__ bool pair_in_range(double s, double rs, double f) {
#pragma clang fp contract(off)
  double R = rs + f * rs;
  return s < R * R;
}

// Bin coordinate of a position (clamped into the grid).
__device__ __forceinline__ int bin_coord(double x, double h, int n) {
  int b = (int)floor(x / h);
  return b < 0 ? 0 : (b >= n ? n - 1 : b);
}

__device__ __forceinline__ int bin_of(const DevParams& P, double x, double y, double z) {
  int bx = bin_coord(x, P.hbx, P.nbx), by = bin_coord(y, P.hby, P.nby),
      bz = bin_coord(z, P.hbz, P.nbz);
  return (bz * P.nby + by) * P.nbx + bx;
}

template <typename T>
struct V3 {
  T x, y, z;
};

template <typename T>
__device__ __forceinline__ V3<T> mk(T a, T b, T c) {
  return V3<T>{a, b, c};
}
template <typename T>
__device__ __forceinline__ T dot(V3<T> a, V3<T> b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
__device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
  return V3<T>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) {
  return V3<T>{a.x + b.x, a.y + b.y, a.z + b.z};
}
template <typename T>
__device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) {
  return V3<T>{a.x - b.x, a.y - b.y, a.z - b.z};
}
template <typename T>
__device__ __forceinline__ V3<T> operator-(V3<T> a) {
  return V3<T>{-a.x, -a.y, -a.z};
}
template <typename T>
__device__ __forceinline__ V3<T> operator*(T s, V3<T> a) {
  return V3<T>{s * a.x, s * a.y, s * a.z};
}

}  // namespace sedimi

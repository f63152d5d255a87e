// k_common.h -- small device helpers shared by the kernels of libsedimi.
#pragma once

#include <hip/hip_runtime.h>

#include "sedimi_internal.h"

namespace sedimi {

// Nearest periodic image of a coordinate difference (selects, no branches).
__device__ __forceinline__ double min_image(double d, double L, double hL) {
  const double lo = d - L, hi = d + L;
  return d > hL ? lo : (d < -hL ? hi : d);
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

// Second half kick of velocity Verlet (explicit FMA, see kick_drift_one).
__device__ __forceinline__ double4 half_kick(double4 v, double4 a, double hdt, double vw) {
  return make_double4(fma(hdt, a.x, v.x), fma(hdt, a.y, v.y), fma(hdt, a.z, v.z), vw);
}

// First half kick and drift of velocity Verlet for one particle: v, w at
// the start of the step in, half-step values out; x drifts with the new v
// and is wrapped on the periodic axes.  Raises the escape / non-finite flags
// and, when the particle has moved more than half the skin since the last
// list build (minimum image), the rebuild flag *rb.
__device__ __forceinline__ void kick_drift_one(const DevParams& P, const DevArrays& A, int q,
                                               double4& x, double4& v, double4& w,
                                               const double4& a, const double4& al, int* rb) {
  // explicit FMAs: the same bits whichever kernel this is inlined into
  const double hdt = 0.5 * P.dt;
  v.x = fma(hdt, a.x, v.x);
  v.y = fma(hdt, a.y, v.y);
  v.z = fma(hdt, a.z, v.z);
  w.x = fma(hdt, al.x, w.x);
  w.y = fma(hdt, al.y, w.y);
  w.z = fma(hdt, al.z, w.z);
  x.x = fma(P.dt, v.x, x.x);
  x.y = fma(P.dt, v.y, x.y);
  x.z = fma(P.dt, v.z, x.z);
  if (x.x >= P.Lx) x.x -= P.Lx;
  if (x.x < 0.0) x.x += P.Lx;
  if (x.x >= P.Lx) x.x = 0.0;
  if (x.y >= P.Ly) x.y -= P.Ly;
  if (x.y < 0.0) x.y += P.Ly;
  if (x.y >= P.Ly) x.y = 0.0;
  int fl = 0;
  if (!(x.z >= 0.0 && x.z <= P.Lz)) fl |= kFlagEscape;
  if (!(isfinite(x.x) && isfinite(x.y) && isfinite(x.z) && isfinite(v.x) && isfinite(v.y) &&
        isfinite(v.z)))
    fl |= kFlagNonFinite;
  if (fl) atomicOr(&A.ctl->flags, fl);
  const double4 b = A.xb[q];
  const double dx = min_image(x.x - b.x, P.Lx, P.hLx), dy = min_image(x.y - b.y, P.Ly, P.hLy),
               dz = x.z - b.z;
  // many particles can cross the half skin in one step: one atomic per wave
  const unsigned long long over = __ballot(dx * dx + dy * dy + dz * dz > P.half_skin2);
  if (over && __lane_id() == __ffsll((long long)over) - 1) atomicOr(rb, 1);
}

// Counting-sort ranks for a whole wave (every lane calls it): each valid lane
// gets a slot among the members of its key, counts[key] growing by the
// number of lanes with that key.  The lanes are grouped by key first (ballots
// only), then every group's first lane adds its group's size with one atomic,
// all groups at once, so a wave waits for one atomic round trip, not one per
// key.  Which slots a key's lanes get depends on the order the atomics of
// different waves land in; the callers order each key's members afterwards.
__device__ __forceinline__ int wave_ranks(int* counts, int key, bool valid) {
  unsigned long long active = __ballot(valid);
  const int lane = __lane_id();
  int leader = lane, within = 0, size = 0;
  while (active) {
    const int l = __ffsll((long long)active) - 1;
    const int kl = __shfl(key, l);
    const unsigned long long grp = __ballot(valid && key == kl) & active;
    if ((grp >> lane) & 1ull) {
      leader = l;
      within = (int)__popcll(grp & ((1ull << lane) - 1ull));
      size = (int)__popcll(grp);
    }
    active &= ~grp;
  }
  int base = 0;
  if (valid && leader == lane) base = atomicAdd(&counts[key], size);
  base = __shfl(base, leader);
  return base + within;
}

// Cell of height z on a graded mesh with faces zf[0..nz]: the k with
// zf[k] <= z < zf[k + 1] (a point on a face belongs to the upper cell);
// below the mesh (or NaN) the first cell, at or above the top the last.
__device__ __forceinline__ int z_cell(const double* __restrict__ zf, int nz, double z) {
  if (!(z >= zf[0])) return 0;
  if (z >= zf[nz]) return nz - 1;
  int lo = 0, hi = nz;  // zf[lo] <= z < zf[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (zf[mid] <= z)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Index of the grid interval of width h holding x, clamped into [0, n - 1]
// before the conversion to int, so that huge and non-finite coordinates
// (NaN goes to 0) give a valid index.
__device__ __forceinline__ int grid_coord(double x, double h, int n) {
  const double f = floor(x / h);
  return f >= 0.0 ? (f < (double)n ? (int)f : n - 1) : 0;
}

// Bin coordinate of a position (clamped into the grid).
__device__ __forceinline__ int bin_coord(double x, double h, int n) { return grid_coord(x, h, n); }

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

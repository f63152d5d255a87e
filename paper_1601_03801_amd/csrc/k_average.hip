// k_average.hip -- particle-to-mesh averaging (Section 2.4).
//
// Deposition (Eq. 11): particles are counting-sorted by mesh cell (integer
// atomics for the counts only), each cell's members are ordered by particle
// ID, and one lane per cell sums volume and drag in that order: a segmented
// reduction with no floating-point atomics, bit-reproducible, and in the
// same summation order as a plain loop over particle IDs.
//
// Diffusion (Eq. 12): avg_ntau backward-Euler pseudo-time steps of unit
// diffusivity up to tau = b^2/4; each step solves (I - dtau L_h) x = b with
// the second-order finite-volume Laplacian (periodic x, y; zero-flux walls).
// The solver is Chebyshev iteration preconditioned by the exact z-line
// (tridiagonal) part of the operator: on a uniform mesh the spectrum of the
// preconditioned operator is known in closed form, so the iteration needs no
// inner products, every iteration is one fused column sweep, and the number
// of iterations that guarantees the residual tolerance is known in advance.
// The final residual of every pseudo-time step is then measured with an FP64
// reduction (fixed-order block trees, summed on the host in fixed order).
#include <math.h>

#include <type_traits>
#include <vector>

#include "k_common.h"

namespace sedimi {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Cell of each particle and its rank among the cell's members.  Sorted
// particles that share a cell mostly sit in the same wave: each group of
// lanes with one cell takes its ranks with a single atomic add
// (wave_ranks).
__global__ void k_cellkey(DevParams P, DevArrays A) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = q < P.n;
  int k = -1;
  if (valid) {
    const double4 x = A.pos[q];
    const int a = grid_coord(x.x, P.hx, P.nx), b = grid_coord(x.y, P.hy, P.ny),
              c = P.graded ? z_cell(A.zgeo + zgeo_faces(P.nz), P.nz, x.z)
                           : grid_coord(x.z, P.hz, P.nz);
    k = (c * P.ny + b) * P.nx + a;
    A.key[q] = k;
  }
  // every lane of the wave is still active here (no early return above)
  const int rank = wave_ranks(A.cell_count, k, valid);
  if (valid) A.rank[q] = rank;
}

__global__ void k_cellscatter(DevParams P, DevArrays A) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P.n) return;
  A.cperm[A.cell_start[A.key[q]] + A.rank[q]] =
      ((unsigned long long)(unsigned)A.id[q] << 32) | (unsigned)q;
}

// One lane per cell: order the members by particle ID (the high half of each
// (ID, index) key): a cell of up to kSortRegs members is sorted in registers
// by a bitonic network (padded with keys above every real one) and written
// back, a larger one by insertion in place.  Then the block's cells, which
// own one contiguous range of the sorted keys, gather their members' volume
// and drag into LDS together, kDepChunk members at a time (many gathers in
// flight instead of a few per lane), and each lane sums its cell's members
// from there in ID order.
constexpr int kSortRegs = 32;
constexpr int kDepChunk = 512;

__global__ __launch_bounds__(kBlock) void k_cellsum(DevParams P, DevArrays A) {
#pragma clang fp contract(off)
  __shared__ double sv[kDepChunk], sfx[kDepChunk], sfy[kDepChunk], sfz[kDepChunk];
  __shared__ double sqx[kDepChunk], sqy[kDepChunk], sqz[kDepChunk];
  const int c0 = blockIdx.x * kBlock;
  const int c = c0 + threadIdx.x;
  const bool valid = c < P.ncell;
  const bool flux = P.nch_avg == 7;
  int s = 0, e = 0;
  if (valid) {
    s = A.cell_start[c];
    e = A.cell_start[c + 1];
  }
  const int m = e - s;
  if (m > 0 && m <= kSortRegs) {
    // unconditional loads (clamped to the last member), padded after it
    unsigned long long key[kSortRegs];
#pragma unroll
    for (int t = 0; t < kSortRegs; ++t) {
      const unsigned long long k = A.cperm[s + (t < m ? t : m - 1)];
      key[t] = t < m ? k : ~0ull;
    }
#pragma unroll
    for (int k = 2; k <= kSortRegs; k <<= 1)
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
        for (int i = 0; i < kSortRegs; ++i) {
          const int l = i ^ j;
          if (l > i) {
            const unsigned long long a = key[i], b = key[l];
            const bool swap = (i & k) == 0 ? a > b : a < b;
            key[i] = swap ? b : a;
            key[l] = swap ? a : b;
          }
        }
#pragma unroll
    for (int t = 0; t < kSortRegs; ++t)
      if (t < m) A.cperm[s + t] = key[t];
  } else if (m > kSortRegs) {
    // a crowded cell is summed unsorted (order not reproducible) and flagged
    const bool sorted = m <= kMaxCellMembers;
    if (!sorted) atomicOr(&A.ctl->flags, kFlagCrowded);
    for (int i = s + 1; sorted && i < e; ++i) {
      const unsigned long long key = A.cperm[i];
      int j = i - 1;
      while (j >= s && A.cperm[j] > key) {
        A.cperm[j + 1] = A.cperm[j];
        --j;
      }
      A.cperm[j + 1] = key;
    }
  }
  // the block's range of sorted keys (written above by its own lanes)
  const int cl = c0 + kBlock < P.ncell ? c0 + kBlock : P.ncell;
  const int seg0 = A.cell_start[c0], seg1 = A.cell_start[cl];
  __syncthreads();
  double v = 0.0, fx = 0.0, fy = 0.0, fz = 0.0, qx = 0.0, qy = 0.0, qz = 0.0;
  for (int base = seg0; base < seg1; base += kDepChunk) {
    const int cnt = seg1 - base < kDepChunk ? seg1 - base : kDepChunk;
    for (int t = threadIdx.x; t < cnt; t += kBlock) {
      const int q = (int)(unsigned)(A.cperm[base + t] & 0xffffffffull);
      const double d = 2.0 * A.pos[q].w;
      const double V = (kPi / 6.0) * d * d * d;
      const double4 f = A.fdr[q];
      sv[t] = V;
      sfx[t] = f.x;
      sfy[t] = f.y;
      sfz[t] = f.z;
      if (flux) {
        const double4 u = A.vel[q];
        sqx[t] = V * u.x;
        sqy[t] = V * u.y;
        sqz[t] = V * u.z;
      }
    }
    __syncthreads();
    // this cell's members in the chunk, in ID order
    const int lo = s > base ? s : base, hi = e < base + cnt ? e : base + cnt;
    for (int i = lo - base; i < hi - base; ++i) {
      v += sv[i];
      fx += sfx[i];
      fy += sfy[i];
      fz += sfz[i];
      if (flux) {
        qx += sqx[i];
        qy += sqy[i];
        qz += sqz[i];
      }
    }
    __syncthreads();
  }
  if (!valid) return;
  const size_t nc = (size_t)P.ncell;
  // each cell divides by its own volume (one per plane on a graded mesh)
  const double Vc = P.graded ? A.zgeo[zgeo_volumes(P.nz) + c / (P.nx * P.ny)] : P.Vc;
  A.raw[c] = v / Vc;
  A.raw[nc + c] = fx / Vc;
  A.raw[2 * nc + c] = fy / Vc;
  A.raw[3 * nc + c] = fz / Vc;
  if (flux) {
    A.raw[4 * nc + c] = qx / Vc;
    A.raw[5 * nc + c] = qy / Vc;
    A.raw[6 * nc + c] = qz / Vc;
  }
}

// Solid velocity: the smoothed volume flux over the smoothed solid fraction,
// 0 where the fraction is at rounding level.
__global__ void k_solid_velocity(DevParams P, DevArrays A) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.ncell) return;
  const size_t nc = (size_t)P.ncell;
  const double es = A.smooth[c];
  const bool solid = es > kSolidEpsMin;
#pragma unroll
  for (int e = 0; e < 3; ++e) A.us[e * nc + c] = solid ? A.smooth[(4 + e) * nc + c] / es : 0.0;
}

// The operator I - dtau L_h.  Along z, a uniform mesh couples a plane to its
// neighbours with cz = dtau kz / hz^2; a graded mesh (gz set) with
// cz gz[2k] to the plane above and cz gz[2k + 1] to the one below (cz =
// dtau there): the flux through each face over the centre distance, per
// unit cell height.
struct Stencil {
  int nx, ny, nz, ncell;
  double cx, cy, cz;
  const double* gz;
};

// dtau L_z contribution at plane k from up = x_{k+1} - x_k and dn =
// x_{k-1} - x_k (each 0 where the plane has no such neighbour).
__device__ __forceinline__ double z_term(const Stencil& S, int k, double up, double dn) {
  if (S.gz) return S.cz * (S.gz[2 * k] * up + S.gz[2 * k + 1] * dn);
  return S.cz * (up + dn);
}
// dtau times the coupling of plane k to the plane below (the negated
// sub-diagonal of I - dtau L_z in row k).
__device__ __forceinline__ double z_down(const Stencil& S, int k) {
  return S.gz ? S.cz * S.gz[2 * k + 1] : S.cz;
}

Stencil make_stencil(const DevParams& P, const DevArrays& A, double dt) {
  Stencil S;
  S.nx = P.nx, S.ny = P.ny, S.nz = P.nz, S.ncell = P.ncell;
  S.cx = dt / (P.hx * P.hx);
  S.cy = dt / (P.hy * P.hy);
  S.cz = P.graded ? dt : dt * P.kz_diff / (P.hz * P.hz);
  S.gz = P.graded ? A.zgeo + zgeo_coupling(P.nz) : nullptr;
  return S;
}

// y = (I - dtau L_h) x at cell c (channel offset already applied to x).
template <typename T>
__device__ __forceinline__ double apply_A(const Stencil& S, const T* __restrict__ x, int c) {
  int i = c % S.nx;
  int jk = c / S.nx;
  int j = jk % S.ny;
  int k = jk / S.ny;
  double xc = (double)x[c];
  int ip = i + 1 == S.nx ? c - i : c + 1;
  int im = i == 0 ? c + S.nx - 1 : c - 1;
  int rowy = S.nx;
  int jp = j + 1 == S.ny ? c - j * rowy : c + rowy;
  int jm = j == 0 ? c + (S.ny - 1) * rowy : c - rowy;
  double lx = ((double)x[ip] - xc) + ((double)x[im] - xc);
  double ly = ((double)x[jp] - xc) + ((double)x[jm] - xc);
  int plane = S.nx * S.ny;
  const double up = k + 1 < S.nz ? (double)x[c + plane] - xc : 0.0;
  const double dn = k > 0 ? (double)x[c - plane] - xc : 0.0;
  return xc - (S.cx * lx + S.cy * ly + z_term(S, k, up, dn));
}

// Preconditioned Chebyshev iteration for (I - dtau L_h) x = b, preconditioner
// M = I - dtau L_z (the z-part of the operator, exact tridiagonal solve per
// column by the Thomas algorithm).  On a uniform mesh every Fourier x DCT
// mode is an eigenvector of both, so the spectrum of M^-1 A is
// (1 + a + c)/(1 + c) with a in [0, 4 (cx + cy)], c in [0, 4 cz]: it lies in
// [1, 1 + 4 (cx + cy)], free of the stiff z coupling.  One lane per
// (x, y) column and channel walks up the column (stencil, update, forward
// elimination) and back down (back substitution, new direction).
//
// ztab: inv_m[k] (reciprocal pivots) then cp[k] (modified super-diagonal).
template <typename T>
__device__ __forceinline__ double ld(const T* p, size_t o) {
  return (double)p[o];
}

// z-window stencil: A v at level k of column (i, j) given v_{k-1}, v_k,
// v_{k+1} (the caller passes 0-weighted neighbours outside the mesh).
template <typename T>
__device__ __forceinline__ double A_col(const Stencil& S, const T* __restrict__ v, size_t c,
                                        int i, int j, int k, double vm, double v0, double vp) {
  size_t ip = i + 1 == S.nx ? c - i : c + 1;
  size_t im = i == 0 ? c + S.nx - 1 : c - 1;
  size_t row = (size_t)S.nx;
  size_t jp = j + 1 == S.ny ? c - (size_t)j * row : c + row;
  size_t jm = j == 0 ? c + (size_t)(S.ny - 1) * row : c - row;
  double lx = (ld(v, ip) - v0) + (ld(v, im) - v0);
  double ly = (ld(v, jp) - v0) + (ld(v, jm) - v0);
  const double up = k + 1 < S.nz ? vp - v0 : 0.0;
  const double dn = k > 0 ? vm - v0 : 0.0;
  return v0 - (S.cx * lx + S.cy * ly + z_term(S, k, up, dn));
}

// Start of a pseudo-time step with b = x (x unchanged): r = b - A b,
// z = M^-1 r, d = z / theta; b saved for the residual check.
template <typename T>
__global__ void k_pcheb_init(Stencil S, const T* __restrict__ x, T* __restrict__ r,
                             T* __restrict__ d, T* __restrict__ bsave, T* __restrict__ tmp,
                             const double* __restrict__ ztab, double inv_theta) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int plane = S.nx * S.ny;
  if (col >= plane) return;
  const size_t off = (size_t)blockIdx.y * S.ncell;
  const T* xv = x + off;
  const int i = col % S.nx, j = col / S.nx;
  const double* inv_m = ztab;
  const double* cp = ztab + S.nz;
  double vm = 0.0, v0 = ld(xv, col), vp = S.nz > 1 ? ld(xv, (size_t)col + plane) : 0.0;
  double yp = 0.0;
  for (int k = 0; k < S.nz; ++k) {
    const size_t c = (size_t)k * plane + col;
    const double Ab = A_col<T>(S, xv, c, i, j, k, vm, v0, vp);
    const double rr = v0 - Ab;
    r[off + c] = (T)rr;
    bsave[off + c] = (T)v0;
    yp = (rr + z_down(S, k) * yp) * inv_m[k];
    tmp[off + c] = (T)yp;
    vm = v0;
    v0 = vp;
    vp = k + 2 < S.nz ? ld(xv, c + 2 * (size_t)plane) : 0.0;
  }
  double z = 0.0;
  for (int k = S.nz - 1; k >= 0; --k) {
    const size_t c = (size_t)k * plane + col;
    z = ld(tmp, off + c) - cp[k] * z;
    d[off + c] = (T)(z * inv_theta);
  }
}

// One iteration: x += d; r -= A d; z = M^-1 r; d' = c1 d + c2 z.
template <typename T>
__global__ void k_pcheb_iter(Stencil S, const T* __restrict__ d, T* __restrict__ x,
                             T* __restrict__ r, T* __restrict__ dn, T* __restrict__ tmp,
                             const double* __restrict__ ztab, double c1, double c2) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int plane = S.nx * S.ny;
  if (col >= plane) return;
  const size_t off = (size_t)blockIdx.y * S.ncell;
  const T* dv = d + off;
  const int i = col % S.nx, j = col / S.nx;
  const double* inv_m = ztab;
  const double* cp = ztab + S.nz;
  double vm = 0.0, v0 = ld(dv, col), vp = S.nz > 1 ? ld(dv, (size_t)col + plane) : 0.0;
  double yp = 0.0;
  for (int k = 0; k < S.nz; ++k) {
    const size_t c = (size_t)k * plane + col;
    const double Ad = A_col<T>(S, dv, c, i, j, k, vm, v0, vp);
    x[off + c] = (T)(ld(x, off + c) + v0);
    const double rr = ld(r, off + c) - Ad;
    r[off + c] = (T)rr;
    yp = (rr + z_down(S, k) * yp) * inv_m[k];
    tmp[off + c] = (T)yp;
    vm = v0;
    v0 = vp;
    vp = k + 2 < S.nz ? ld(dv, c + 2 * (size_t)plane) : 0.0;
  }
  double z = 0.0;
  for (int k = S.nz - 1; k >= 0; --k) {
    const size_t c = (size_t)k * plane + col;
    z = ld(tmp, off + c) - cp[k] * z;
    dn[off + c] = (T)(c1 * ld(dv, c) + c2 * z);
  }
}

// Unpreconditioned variant, one lane per cell (better when the mesh has few
// columns): x += d; r -= A d; d' = c1 d + c2 r.
template <typename T>
__global__ void k_cheb_init(Stencil S, const T* __restrict__ x, T* __restrict__ r,
                            T* __restrict__ d, T* __restrict__ bsave, double inv_theta) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= S.ncell) return;
  size_t off = (size_t)blockIdx.y * S.ncell;
  double b = (double)x[off + c];
  double rr = b - apply_A<T>(S, x + off, c);
  bsave[off + c] = (T)b;
  r[off + c] = (T)rr;
  d[off + c] = (T)(rr * inv_theta);
}

template <typename T>
__global__ void k_cheb_iter(Stencil S, const T* __restrict__ d, T* __restrict__ x,
                            T* __restrict__ r, T* __restrict__ dn, double c1, double c2) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= S.ncell) return;
  size_t off = (size_t)blockIdx.y * S.ncell;
  double dc = (double)d[off + c];
  double Ad = apply_A<T>(S, d + off, c);
  double rn = (double)r[off + c] - Ad;
  x[off + c] = (T)((double)x[off + c] + dc);
  r[off + c] = (T)rn;
  dn[off + c] = (T)(c1 * dc + c2 * rn);
}

template <typename A_, typename B_>
__global__ void k_convert(size_t n, const A_* __restrict__ in, B_* __restrict__ out) {
  size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = (B_)in[k];
}

// Per-block FP64 sums of (b - A x)^2 and b^2 for each channel.
template <typename T>
__global__ void k_residual(Stencil S, const T* __restrict__ b, const T* __restrict__ x,
                           double* __restrict__ part) {
  __shared__ double s1[kBlock], s2[kBlock];
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  size_t off = (size_t)blockIdx.y * S.ncell;
  double rr = 0.0, bb = 0.0;
  if (c < S.ncell) {
    double bv = (double)b[off + c];
    double r = bv - apply_A<T>(S, x + off, c);
    rr = r * r;
    bb = bv * bv;
  }
  s1[threadIdx.x] = rr;
  s2[threadIdx.x] = bb;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    size_t base = (size_t)blockIdx.y * gridDim.x * 2;
    part[base + blockIdx.x] = s1[0];
    part[base + gridDim.x + blockIdx.x] = s2[0];
  }
}

// out = A in for every channel (blockIdx.z), one x-row per block row: the
// row's (j, k) is uniform across the block, so no lane divides its index.
// COMB: out = alpha A in + beta in + gamma other instead.
template <bool COMB>
__global__ void k_applyA(Stencil S, const double* __restrict__ in, double* __restrict__ out,
                         double alpha, double beta, double gamma,
                         const double* __restrict__ other) {
  // one lane per cell over the flat index (full waves whatever n_x is);
  // the channel is blockIdx.z
  const size_t off = (size_t)blockIdx.z * S.ncell;
  const double* x = in + off;
  const int plane = S.nx * S.ny;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < S.ncell;
       c += gridDim.x * blockDim.x) {
    const int i = c % S.nx, jk = c / S.nx;
    const int j = jk % S.ny, k = jk / S.ny;
    const double xc = x[c];
    const int ip = i + 1 == S.nx ? c - i : c + 1;
    const int im = i == 0 ? c + S.nx - 1 : c - 1;
    const int jp = j + 1 == S.ny ? c - j * S.nx : c + S.nx;
    const int jm = j == 0 ? c + (S.ny - 1) * S.nx : c - S.nx;
    const double lx = (x[ip] - xc) + (x[im] - xc);
    const double ly = (x[jp] - xc) + (x[jm] - xc);
    const double up = k + 1 < S.nz ? x[c + plane] - xc : 0.0;
    const double dn = k > 0 ? x[c - plane] - xc : 0.0;
    const double ax = xc - (S.cx * lx + S.cy * ly + z_term(S, k, up, dn));
    if (COMB) {
      double v = alpha * ax + beta * xc;
      if (other) v += gamma * other[off + c];
      out[off + c] = v;
    } else {
      out[off + c] = ax;
    }
  }
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Residual of a smoothed field y against the deposited field on a seeded
// sample of cells: r = Ay - raw with Ay = A^ntau y.  Per-block FP64 sums of
// r^2 (first nch values) and y^2 (next nch) for each of the nch <= 7
// channels.
constexpr int kMaxCh = 7;
__global__ void k_check(int ncell, int nch, const double* __restrict__ Ay,
                        const double* __restrict__ raw, const double* __restrict__ y,
                        uint64_t seed, uint64_t thresh, double* __restrict__ part) {
  __shared__ double s[kBlock / 64][2 * kMaxCh];
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  double v[2 * kMaxCh];
#pragma unroll
  for (int q = 0; q < 2 * kMaxCh; ++q) v[q] = 0.0;
  if (c < ncell && splitmix64(seed ^ (uint64_t)c) < thresh) {
#pragma unroll
    for (int ch = 0; ch < kMaxCh; ++ch) {
      if (ch >= nch) break;
      size_t o = (size_t)ch * ncell + c;
      double r = Ay[o] - raw[o];
      v[ch] = r * r;
      v[kMaxCh + ch] = y[o] * y[o];
    }
  }
  // butterfly within each wave, then the waves' sums in wave order: a fixed
  // order, so the partials are reproducible
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 2 * kMaxCh; ++q) {
    if ((q < kMaxCh ? q : q - kMaxCh) >= nch) continue;
    double x = v[q];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) s[wid][q] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int ch = 0; ch < nch; ++ch) {
      double r = 0.0, yy = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) {
        r += s[w][ch];
        yy += s[w][kMaxCh + ch];
      }
      part[(size_t)blockIdx.x * 2 * nch + ch] = r;
      part[(size_t)blockIdx.x * 2 * nch + nch + ch] = yy;
    }
}

// Error of a smoothed field y against the plain solution, estimated on whole
// z-columns: the plain solution at a cell is the Green's function of all
// N_tau implicit steps applied to the deposited field, G * raw, taken here
// over a window of (2 rx + 1) x (2 ry + 1) x (2 rz + 1) cells (periodic in x
// and y; reflected about the wall faces in z, which gives the zero-flux
// walls' image terms).  The window is chosen to hold all but a small share
// of G's mass, which bounds the estimate's own error by that share of the
// field's largest value.  One block per sampled column; the column's window
// of one channel is staged in LDS kGreenKz output planes at a time.
// Per-block FP64 sums of (y - G * raw)^2 (first 4 values) and (G * raw)^2
// (next 4).
constexpr int kGreenKz = 64;            // output planes per stage
constexpr int kGreenMaxRxy = 4;
constexpr int kGreenMaxCols = (2 * kGreenMaxRxy + 1) * (2 * kGreenMaxRxy + 1);
constexpr int kGreenMaxRz = 32;
__global__ __launch_bounds__(256) void k_green_check(
    int nx, int ny, int nz, const int* __restrict__ cols, const double* __restrict__ gtab, int rx,
    int ry, int rz, const double* __restrict__ raw, const double* __restrict__ y,
    double* __restrict__ part) {
  __shared__ double win[kGreenMaxCols][kGreenKz + 2 * kGreenMaxRz + 1];  // +1: rows on other banks
  __shared__ double gs[kGreenMaxCols * (2 * kGreenMaxRz + 1)];
  __shared__ double red[8][4];
  const int col = cols[blockIdx.x];
  const int ci = col % nx, cj = col / nx;
  const int wx = 2 * rx + 1, wy = 2 * ry + 1, ncol = wx * wy, wz = 2 * rz + 1;
  const int64_t plane = (int64_t)nx * ny, ncell = plane * nz;
  for (int q = threadIdx.x; q < ncol * wz; q += blockDim.x) gs[q] = gtab[q];
  // each output (plane z, channel) is summed by 4 lanes, each over a quarter
  // of the window's columns; 64 outputs per pass
  const int sub = threadIdx.x & 3, oz = threadIdx.x >> 2;
  double e2[4] = {0, 0, 0, 0}, p2[4] = {0, 0, 0, 0};
  for (int ch = 0; ch < 4; ++ch) {
    for (int z0 = 0; z0 < nz; z0 += kGreenKz) {
      const int nzo = min(kGreenKz, nz - z0), nzs = nzo + 2 * rz;
      __syncthreads();  // the previous stage is no longer read
      for (int q = threadIdx.x; q < ncol * nzs; q += blockDim.x) {
        const int wc = q / nzs, zz = q % nzs;
        const int dx = wc % wx - rx, dy = wc / wx - ry;
        int ii = (ci + dx) % nx;
        ii = ii < 0 ? ii + nx : ii;
        int jj = (cj + dy) % ny;
        jj = jj < 0 ? jj + ny : jj;
        int kk = (z0 + zz - rz) % (2 * nz);  // reflection about the wall faces
        kk = kk < 0 ? kk + 2 * nz : kk;
        kk = kk < nz ? kk : 2 * nz - 1 - kk;
        win[wc][zz] = raw[(size_t)ch * ncell + (kk * plane + (int64_t)jj * nx + ii)];
      }
      __syncthreads();
      double acc = 0.0;
      if (oz < nzo) {
        for (int wc = sub; wc < ncol; wc += 4) {
          const double* g = gs + wc * wz;
          const double* w = &win[wc][oz];
          for (int t = 0; t < wz; ++t) acc += g[t] * w[t];
        }
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      if (sub == 0 && oz < nzo) {
        const int64_t c = (int64_t)(z0 + oz) * plane + (int64_t)cj * nx + ci;
        const double d = y[(size_t)ch * ncell + c] - acc;
        e2[ch] += d * d;
        p2[ch] += acc * acc;
      }
    }
  }
  // block sums: lanes of a wave, then the 4 waves
  for (int ch = 0; ch < 4; ++ch) {
    for (int o = 32; o > 0; o >>= 1) {
      e2[ch] += __shfl_xor(e2[ch], o, 64);
      p2[ch] += __shfl_xor(p2[ch], o, 64);
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
    for (int ch = 0; ch < 4; ++ch) red[wave][ch] = e2[ch], red[4 + wave][ch] = p2[ch];
  __syncthreads();
  if (threadIdx.x < 8) {
    const int ch = threadIdx.x & 3, which = threadIdx.x >> 2;
    const double v = red[4 * which + 0][ch] + red[4 * which + 1][ch] + red[4 * which + 2][ch] +
                     red[4 * which + 3][ch];
    part[(size_t)blockIdx.x * 8 + 4 * which + ch] = v;
  }
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int launch_green_check(const DevParams& P, const double* raw, const double* y, const int* cols,
                       int ncols, const double* gtab, int rx, int ry, int rz, double* part,
                       hipStream_t s) {
  if (ncols <= 0 || rx < 0 || ry < 0 || rz < 0 || rx > kGreenMaxRxy || ry > kGreenMaxRxy ||
      rz > kGreenMaxRz)
    return 0;
  hipLaunchKernelGGL(k_green_check, dim3(ncols), dim3(256), 0, s, P.nx, P.ny, P.nz, cols, gtab,
                     rx, ry, rz, raw, y, part);
  return ncols;
}

const double* apply_An(const DevParams& P, DevArrays& A, const double* y, int nch, int ntau,
                       double tau, hipStream_t s) {
  double dtau = tau / (ntau > 0 ? ntau : 1);
  const Stencil S = make_stencil(P, A, dtau);
  const dim3 grid(nblk(P.ncell), 1, nch);
  const double* cur = y;
  double* bufs[2] = {A.sd0, A.sd1};
  for (int m = 0; m < ntau; ++m) {
    hipLaunchKernelGGL(k_applyA<false>, grid, dim3(kBlock), 0, s, S, cur, bufs[m & 1], 1.0,
                       0.0, 0.0, nullptr);
    cur = bufs[m & 1];
  }
  return cur;
}

int launch_check(const DevParams& P, DevArrays& A, const double* y, int nch, int ntau,
                 double tau, uint64_t seed, double frac, hipStream_t s) {
  const double* cur = apply_An(P, A, y, nch, ntau, tau, s);
  double f = frac < 0.0 ? 0.0 : (frac > 1.0 ? 1.0 : frac);
  uint64_t thresh = f >= 1.0 ? ~0ull : (uint64_t)(f * 18446744073709551616.0);
  hipLaunchKernelGGL(k_check, dim3(nblk(P.ncell)), dim3(kBlock), 0, s, P.ncell, nch, cur, A.raw,
                     y, seed, thresh, A.red);
  return (int)nblk(P.ncell);
}

int read_check(DevArrays& A, int nblocks, int nch, double* rel, hipStream_t s) {
  return read_partials(A.red, nblocks, nch, rel, s);
}

int read_partials(const double* part, int nblocks, int nch, double* rel, hipStream_t s) {
  std::vector<double> h((size_t)nblocks * 2 * nch);
  if (hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return -1;
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  for (int ch = 0; ch < nch; ++ch) {
    double rr = 0.0, yy = 0.0;
    for (int b = 0; b < nblocks; ++b) {
      rr += h[(size_t)b * 2 * nch + ch];
      yy += h[(size_t)b * 2 * nch + nch + ch];
    }
    rel[ch] = yy > 0.0 ? sqrt(rr / yy) : sqrt(rr);
  }
  return 0;
}

int launch_check_bdf2(const DevParams& P, DevArrays& A, int nch, int ntau, double tau,
                      hipStream_t s) {
  const int N = ntau > 0 ? ntau : 1;
  const double dtau = tau / N;
  const Stencil S = make_stencil(P, A, dtau);
  const dim3 grid(nblk(P.ncell), 1, nch);
  // A = I + M, so (3 + 2M) x = 2 A x + x
  auto comb = [&](const double* in, double* out, double al, double be, double ga,
                  const double* other) {
    hipLaunchKernelGGL(k_applyA<true>, grid, dim3(kBlock), 0, s, S, in, out, al, be, ga, other);
  };
  // q_N(M) y: N - 1 factors (3 + 2M), then (1 + M)
  const double* qy = A.smooth;
  double* qb[2] = {A.sd0, A.sd1};
  for (int m = 0; m < N; ++m) {
    if (m + 1 < N)
      comb(qy, qb[m & 1], 2.0, 1.0, 0.0, nullptr);
    else
      comb(qy, qb[m & 1], 1.0, 0.0, 0.0, nullptr);
    qy = qb[m & 1];
  }
  // p_N(M) raw: p_1 = raw, p_2 = 3 raw - M raw = 4 raw - A raw,
  // p_{n+1} = 4 p_n - (2 A p_{n-1} + p_{n-1})
  const double* prev = A.raw;
  const double* cur = A.raw;
  double* pool[3] = {A.sx, A.sr, A.stmp};
  for (int n = 1; n < N; ++n) {
    double* next = pool[n % 3];
    if (n == 1)
      comb(A.raw, next, -1.0, 0.0, 4.0, A.raw);
    else
      comb(prev, next, -2.0, -1.0, 4.0, cur);
    prev = cur;
    cur = next;
  }
  hipLaunchKernelGGL(k_check, dim3(nblk(P.ncell)), dim3(kBlock), 0, s, P.ncell, nch, qy, cur,
                     (const double*)A.smooth, (uint64_t)0, ~0ull, A.red);
  return (int)nblk(P.ncell);
}

void launch_solid_velocity(const DevParams& P, DevArrays& A, hipStream_t s) {
  hipLaunchKernelGGL(k_solid_velocity, dim3(nblk(P.ncell)), dim3(kBlock), 0, s, P, A);
}

void launch_deposit(const DevParams& P, DevArrays& A, hipStream_t s) {
  launch_zero_ints(A.cell_count, P.ncell, false, A.rb, s);
  if (P.n > 0) {
    hipLaunchKernelGGL(k_cellkey, dim3(nblk(P.n)), dim3(kBlock), 0, s, P, A);
  }
  launch_exclusive_scan(A.cell_count, A.cell_start, P.ncell, A.scan_tmp, false, A.rb, s);
  if (P.n > 0) {
    hipLaunchKernelGGL(k_cellscatter, dim3(nblk(P.n)), dim3(kBlock), 0, s, P, A);
  }
  hipLaunchKernelGGL(k_cellsum, dim3(nblk(P.ncell)), dim3(kBlock), 0, s, P, A);
}

size_t smooth_red_doubles(int ncell, int nch, int ntau) {
  return (size_t)((ncell + kBlock - 1) / kBlock) * 2 * nch * (ntau > 0 ? ntau : 1);
}

void smooth_ztab(const DevParams& P, const double* zcoup, int ntau, double tau,
                 double* host_tab) {
  // Thomas factors of I - dtau L_z: row k has diagonal 1 + up_k + dn_k,
  // -dn_k below it and -up_k above it (uniform: up = dn = cz inside)
  double dtau = tau / (ntau > 0 ? ntau : 1);
  double cz = dtau * P.kz_diff / (P.hz * P.hz);
  double prev_cp = 0.0;
  for (int k = 0; k < P.nz; ++k) {
    double up, dn;
    if (P.graded) {
      up = dtau * zcoup[2 * k];
      dn = dtau * zcoup[2 * k + 1];
    } else {
      up = k + 1 < P.nz ? cz : 0.0;
      dn = k > 0 ? cz : 0.0;
    }
    double diag = 1.0 + up + dn;
    double m = k == 0 ? diag : diag + dn * prev_cp;
    double cp = -up / m;
    host_tab[k] = 1.0 / m;
    host_tab[P.nz + k] = cp;
    prev_cp = cp;
  }
}

// Chebyshev iteration count for the residual bound: |r_k| <= pre * 2 rho^k |b|.
static int cheb_iters(double kappa, double pre, double rtol) {
  if (kappa <= 1.0 + 1e-12) return 1;
  double rho = (sqrt(kappa) - 1.0) / (sqrt(kappa) + 1.0);
  int k = (int)ceil(log(rtol / (2.0 * pre)) / log(rho)) + 1;
  return k < 1 ? 1 : k;
}

// BDF2 right-hand side in place: x <- (4 x - prev) / 3, prev <- old x.
template <typename T>
__global__ void k_bdf2_rhs(size_t n, T* __restrict__ x, T* __restrict__ prev) {
  size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double t = (double)x[k];
  x[k] = (T)((4.0 * t - (double)prev[k]) / 3.0);
  prev[k] = (T)t;
}

// Chebyshev set-up for (I - dt L_h) at one pseudo-time step size dt.
struct ChebPlan {
  Stencil S;
  bool line;
  int kiter;
  double theta, delta;
};

static ChebPlan cheb_plan(const DevParams& P, const DevArrays& A, int nch, double dt,
                          double rtol) {
  ChebPlan p;
  p.S = make_stencil(P, A, dt);
  const Stencil& S = p.S;
  const double axy = 4.0 * ((P.nx > 1 ? S.cx : 0.0) + (P.ny > 1 ? S.cy : 0.0));
  const double az = P.nz > 1 ? dt * P.zlam : 0.0;
  const double kappaA = 1.0 + axy + az;
  // A graded mesh's operator is not symmetric but similar to a symmetric one
  // through the square roots of the cell heights: its residual norms carry
  // that similarity's condition number, zskew, on top of the bounds below.
  // plain Chebyshev on A: spectrum [1, kappaA], |r_0| <= (kappaA - 1) |b|
  const int k_plain = cheb_iters(kappaA, P.zskew * (kappaA - 1.0), rtol);
  // z-line preconditioned: L_xy and L_z commute (the z coupling is the same
  // in every column), so the spectrum of M^-1 A lies in [1, 1 + axy]; the
  // bound picks up sqrt(cond M) = sqrt(1 + az)
  const int k_line = cheb_iters(1.0 + axy, P.zskew * sqrt(1.0 + az) * (kappaA - 1.0), rtol);
  // cost model from measurements on MI355X: the per-cell sweep moves 6
  // vectors at ~5 TB/s; the column sweep moves 9 and reaches ~3.6 TB/s with
  // >= 128k column lanes, ~2 TB/s with fewer (latency bound)
  const double lanes = (double)P.nx * P.ny * nch;
  const double t_plain = k_plain * 6.0 / 5.0;
  const double t_line = k_line * 9.0 / (lanes >= 131072.0 ? 3.6 : 2.0);
  p.line = t_line < t_plain;
  const double lmin = 1.0, lmax = p.line ? 1.0 + axy : kappaA;
  p.kiter = p.line ? k_line : k_plain;
  p.theta = 0.5 * (lmax + lmin);
  p.delta = 0.5 * (lmax - lmin);
  return p;
}

template <typename T>
static int64_t smooth_impl(const DevParams& P, DevArrays& A, int nch, int ntau, double tau,
                           double rtol, bool bdf2, hipStream_t s) {
  const double dtau = tau / ntau;
  // backward Euler (and BDF2's first step) at dtau; later BDF2 steps solve
  // (I - 2/3 dtau L_h) with the second z-line table
  const ChebPlan plans[2] = {cheb_plan(P, A, nch, dtau, rtol),
                             cheb_plan(P, A, nch, (2.0 / 3.0) * dtau, rtol)};
  const size_t nall = (size_t)nch * P.ncell;
  const unsigned gall = (unsigned)((nall + kBlock - 1) / kBlock);
  T* x = std::is_same<T, double>::value ? (T*)A.smooth : (T*)A.sxf;
  T* r = (T*)A.sr;
  T* d0 = (T*)A.sd0;
  T* d1 = (T*)A.sd1;
  T* tmp = (T*)A.stmp;
  T* bsave = (T*)A.sx;
  T* prev = (T*)A.sprev;
  hipLaunchKernelGGL((k_convert<double, T>), dim3(gall), dim3(kBlock), 0, s, nall,
                     (const double*)A.raw, x);
  dim3 cgrid(nblk((int64_t)P.nx * P.ny), nch);
  dim3 grid(nblk(P.ncell), nch);
  const size_t nred = (size_t)grid.x * 2 * nch;
  int64_t total = 0;
  for (int m = 0; m < ntau; ++m) {
    const bool second = bdf2 && m > 0;
    if (bdf2) {
      // the step's right-hand side becomes x (and its starting guess)
      if (m == 0)
        hipLaunchKernelGGL((k_convert<T, T>), dim3(gall), dim3(kBlock), 0, s, nall,
                           (const T*)x, prev);
      else
        hipLaunchKernelGGL(k_bdf2_rhs<T>, dim3(gall), dim3(kBlock), 0, s, nall, x, prev);
    }
    const ChebPlan& pl = plans[second ? 1 : 0];
    const Stencil& S = pl.S;
    const double* ztab = A.ztab + (second ? 2 * (size_t)P.nz : 0);
    const double theta = pl.theta, delta = pl.delta;
    const double inv_theta = delta > 0.0 ? 1.0 / theta : 1.0;
    if (pl.line)
      hipLaunchKernelGGL((k_pcheb_init<T>), cgrid, dim3(kBlock), 0, s, S, x, r, d0, bsave, tmp,
                         ztab, inv_theta);
    else
      hipLaunchKernelGGL((k_cheb_init<T>), grid, dim3(kBlock), 0, s, S, x, r, d0, bsave,
                         inv_theta);
    double sigma1 = delta > 0.0 ? theta / delta : 1.0;
    double rho_k = 1.0 / sigma1;
    T* dcur = d0;
    T* dnext = d1;
    for (int it = 0; it < pl.kiter; ++it) {
      double c1 = 0.0, c2 = 0.0;
      if (delta > 0.0) {
        double rho_n = 1.0 / (2.0 * sigma1 - rho_k);
        c1 = rho_n * rho_k;
        c2 = 2.0 * rho_n / delta;
        rho_k = rho_n;
      }
      if (pl.line)
        hipLaunchKernelGGL((k_pcheb_iter<T>), cgrid, dim3(kBlock), 0, s, S, dcur, x, r, dnext,
                           tmp, ztab, c1, c2);
      else
        hipLaunchKernelGGL((k_cheb_iter<T>), grid, dim3(kBlock), 0, s, S, dcur, x, r, dnext,
                           c1, c2);
      T* t = dcur;
      dcur = dnext;
      dnext = t;
    }
    hipLaunchKernelGGL(k_residual<T>, grid, dim3(kBlock), 0, s, S, bsave, x,
                       A.red + (size_t)m * nred);
    total += pl.kiter;
  }
  if (!std::is_same<T, double>::value)
    hipLaunchKernelGGL((k_convert<T, double>), dim3(gall), dim3(kBlock), 0, s, nall, x,
                       A.smooth);
  return total;
}

int64_t launch_smooth(const DevParams& P, DevArrays& A, int nch, int ntau, double tau,
                      double rtol, bool mixed, bool bdf2, hipStream_t s) {
  if (ntau <= 0) {
    (void)hipMemcpyAsync(A.smooth, A.raw, sizeof(double) * nch * P.ncell,
                         hipMemcpyDeviceToDevice, s);
    return 0;
  }
  if (mixed) return smooth_impl<float>(P, A, nch, ntau, tau, rtol, bdf2, s);
  return smooth_impl<double>(P, A, nch, ntau, tau, rtol, bdf2, s);
}

double read_smooth_residual(const DevParams& P, DevArrays& A, int nch, int ntau,
                            hipStream_t s) {
  if (ntau <= 0) return 0.0;
  unsigned nb = nblk(P.ncell);
  const size_t nred = (size_t)nb * 2 * nch;
  std::vector<double> h((size_t)ntau * nred);
  if (hipMemcpyAsync(h.data(), A.red, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return -1.0;
  if (hipStreamSynchronize(s) != hipSuccess) return -1.0;
  double worst = 0.0;
  for (int m = 0; m < ntau; ++m) {
    for (int ch = 0; ch < nch; ++ch) {
      const double* p = h.data() + (size_t)m * nred + (size_t)ch * nb * 2;
      double rr = 0.0, bb = 0.0;
      for (unsigned b = 0; b < nb; ++b) {
        rr += p[b];
        bb += p[nb + b];
      }
      double rel = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
      if (rel > worst) worst = rel;
    }
  }
  return worst;
}

}  // namespace sedimi

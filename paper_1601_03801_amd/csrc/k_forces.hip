// k_forces.hip -- fused force evaluation and second half kick.
//
// One lane per particle (bin-sorted order) walks its full neighbour list.
// Every pair is evaluated on both of its sides in the frame of its lower-ID
// particle, with operations whose IEEE results do not depend on which side
// computes them, so both sides get bit-identical pair forces and tangential
// histories: the pair forces are exactly antisymmetric and no atomics are
// needed.  Per pair (Sections 2.1, 2.5):
//   - pair set: s = |dx|^2 < ((r_i + r_j)(1 + f_out))^2, exact FP64 test;
//   - lubrication (the force of the fluid squeezed out of the gap) for every
//     pair in the set:
//     F = -6 pi mu a_eff^2 u_n / max(h, h_in) n;
//   - contact when the overlap delta > 0: linear spring-dashpot normal force
//     -(k_n delta + gamma_n u_n) n, tangential history spring with Coulomb
//     cap mu |F_n|, torque r n x F_t;
// then the flat walls at z = 0 / Lz (same models, infinite wall mass), and
// the fluid-particle forces at the particle centre (Section 2.3): Di Felice
// (or Stokes) drag towards the interpolated fluid velocity, -V grad p, and
// added mass C_add rho_f V (DU_f/Dt - a_prev) with a_prev the acceleration of
// the previous step.  Translational and angular accelerations follow from
// Eq. (1a)-(1b).
//
// Precision: geometry (centre differences, distances, overlaps, normals) is
// always FP64; with R = float the force arithmetic, the history and the sums
// are FP32 and only the state update is FP64.
#include "k_common.h"

namespace sedimi {

namespace {

constexpr double kPi = 3.14159265358979323846;

template <typename R>
__device__ __forceinline__ V3<R> cvt(double a, double b, double c) {
  return V3<R>{(R)a, (R)b, (R)c};
}

// 1/x and 1/sqrt(x) of a positive operand.  FP64: the hardware estimate
// refined by two Newton steps, to within about an ulp in a third of the
// instructions of an IEEE division (the operands, squared lengths and sums of
// radii and masses, are never below the FP64 normal range here; the estimate
// does not take denormals).  FP32: IEEE division, since squared lengths of
// tiny tangential histories and forces do reach FP32 denormals.  Used where
// the quotient feeds a force continuously; the contact decision (the overlap
// from the correctly rounded centre distance) does not go through them.
// Both sides of a pair run the same sequence on the same operands, so pair
// forces stay exactly antisymmetric.
template <typename R>
__device__ __forceinline__ R recip(R x);
template <>
__device__ __forceinline__ double recip<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
template <>
__device__ __forceinline__ float recip<float>(float x) {
  return 1.0f / x;
}
// a / b: a * recip(b) in FP64; the plain quotient in FP32, where 1/b alone
// can overflow (b near the denormal range) while a / b does not.
__device__ __forceinline__ double quot(double a, double b) { return a * recip(b); }
__device__ __forceinline__ float quot(float a, float b) { return a / b; }
template <typename R>
__device__ __forceinline__ R rsqrt_of(R x);
template <>
__device__ __forceinline__ double rsqrt_of<double>(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  return r * fma(-h * r, r, 1.5);
}
template <>
__device__ __forceinline__ float rsqrt_of<float>(float x) {
  return 1.0f / sqrtf(x);
}

// Tangential spring: rotate the old history into the tangent plane keeping
// its length, add v_t dt, F_t = -k_t xi - gamma_t v_t, Coulomb cap mu |F_n|
// (history reset to the capped force when sliding).
template <typename R>
__device__ __forceinline__ V3<R> tangential(R kt, R gt, R mu, R dt, V3<R> n, V3<R> vrel,
                                            R un, R Fn, V3<R>& xi) {
  V3<R> vt = vrel - un * n;
  R old2 = dot(xi, xi);
  R xn = dot(xi, n);
  V3<R> xp = xi - xn * n;
  R pm2 = dot(xp, xp);
  if (pm2 > (R)0) {
    xp = sqrt(quot(old2, pm2)) * xp;
  } else {
    xp = V3<R>{0, 0, 0};
  }
  xi = xp + dt * vt;
  V3<R> ft = (-kt) * xi - gt * vt;
  R fm2 = dot(ft, ft);
  R cap = mu * Fn;
  if (fm2 > cap * cap) {
    ft = (sizeof(R) == 8 ? cap * rsqrt_of(fm2) : cap / sqrt(fm2)) * ft;
    if (kt > (R)0) xi = quot((R)-1, kt) * (ft + gt * vt);
  }
  return ft;
}

// Drag force per unit slip velocity w (F = drag_coef * w) for the selected
// law (Section 2.3).
template <typename R>
__device__ __forceinline__ R drag_coef(const DevParams& P, R d, R eps_f, R wm) {
  if (P.drag_law == SEDIMI_DRAG_STOKES) return (R)(3.0 * kPi * P.mu_f) * d;
  if (P.drag_law == SEDIMI_DRAG_SYAMLAL) {
    // (3/4) V_p C_d rho_f |w| / (V_r^2 d) = (pi/8) d^2 C_d rho_f |w| / V_r^2
    const R Re = (R)P.rho_f * d * wm / (R)P.mu_f;
    if (!(Re >= (R)1e-12)) return (R)0;
    const R A1 = pow(eps_f, (R)4.14);
    const R A2 = eps_f <= (R)0.85 ? (R)0.8 * pow(eps_f, (R)1.28) : pow(eps_f, (R)2.65);
    const R a = (R)0.06 * Re;
    const R Vr = (R)0.5 * (A1 - a + sqrt(a * a + (R)0.12 * Re * ((R)2 * A2 - A1) + A1 * A1));
    R cd = (R)0.63 + (R)4.8 * sqrt(Vr / Re);
    cd = cd * cd;
    return (R)(0.125 * kPi) * d * d * cd * (R)P.rho_f * wm / (Vr * Vr);
  }
  if (P.drag_law != SEDIMI_DRAG_DIFELICE) return (R)0;
  R Re = (R)P.rho_f * d * eps_f * wm / (R)P.mu_f;
  if (!(Re >= (R)1e-12)) return (R)0;
  R cd = (R)0.63 + (R)4.8 / sqrt(Re);
  cd = cd * cd;
  R lg = (R)1.5 - log10(Re);
  R chi = (R)3.7 - (R)0.65 * exp((R)-0.5 * lg * lg);
  R area = (R)(0.25 * kPi) * d * d;
  return (R)0.5 * cd * (R)P.rho_f * area * pow(eps_f, (R)2 - chi) * wm;
}

// Trilinear interpolation of the cell-centred mesh fields at (x, y, z):
// periodic in x and y, clamped to the first / last cell centre in z (on a
// graded mesh, between the centres' own heights).  The
// eight corners are visited as four x-rows (y then z), two cells each, in a
// loop that is not unrolled: unrolled, the sixteen in-flight double4 loads
// set the kernel's register peak and halve its occupancy.
struct FluidAt {
  double Ux, Uy, Uz, es;  // fluid velocity, solid fraction
  double gx, gy, gz;      // step modes: G; evaluation mode: grad p
  double dx, dy, dz;      // evaluation mode: DU/Dt
};

// The cell-centre corners around (x, y, z) and the fractional offsets.
struct Corners {
  int i0, i1, j0, j1, k0, k1;
  double fx, fy, fz;
};

__device__ __forceinline__ Corners corners_at(const DevParams& P, const double* __restrict__ zc,
                                              double x, double y, double z) {
  double sx = x / P.hx - 0.5, sy = y / P.hy - 0.5, sz = z / P.hz - 0.5;
  // keep indices in range even for non-finite positions (flagged elsewhere)
  if (!(sx >= -1.0 && sx <= (double)P.nx)) sx = 0.0;
  if (!(sy >= -1.0 && sy <= (double)P.ny)) sy = 0.0;
  const double fx0 = floor(sx), fy0 = floor(sy);
  Corners q;
  q.fx = sx - fx0;
  q.fy = sy - fy0;
  q.i0 = (((int)fx0 % P.nx) + P.nx) % P.nx;
  q.i1 = q.i0 + 1 == P.nx ? 0 : q.i0 + 1;
  q.j0 = (((int)fy0 % P.ny) + P.ny) % P.ny;
  q.j1 = q.j0 + 1 == P.ny ? 0 : q.j0 + 1;
  if (P.nz == 1) {
    q.k0 = q.k1 = 0;
    q.fz = 0.0;
  } else if (P.graded) {
    // linear between the two cell centres around z (zc: the centres'
    // heights), clamped to the first / last centre
    if (!(z > zc[0])) {
      q.k0 = 0;
      q.fz = 0.0;
    } else if (z >= zc[P.nz - 1]) {
      q.k0 = P.nz - 2;
      q.fz = 1.0;
    } else {
      int lo = 0, hi = P.nz - 1;  // zc[lo] <= z < zc[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (zc[mid] <= z)
          lo = mid;
        else
          hi = mid;
      }
      q.k0 = lo;
      q.fz = (z - zc[lo]) / (zc[lo + 1] - zc[lo]);
    }
    q.k1 = q.k0 + 1;
  } else {
    sz = sz >= 0.0 ? (sz > P.nz - 1 ? (double)(P.nz - 1) : sz) : 0.0;
    q.k0 = (int)floor(sz);
    if (q.k0 > P.nz - 2) q.k0 = P.nz - 2;
    q.k1 = q.k0 + 1;
    q.fz = sz - (double)q.k0;
  }
  return q;
}

template <int MODE>
__device__ __forceinline__ FluidAt fluid_at(const DevParams& P, const DevArrays& A, double x,
                                            double y, double z) {
  const Corners q = corners_at(P, A.zgeo + zgeo_centres(P.nz), x, y, z);
  const int i0 = q.i0, i1 = q.i1, j0 = q.j0, j1 = q.j1, k0 = q.k0, k1 = q.k1;
  const double fx = q.fx, fy = q.fy, fz = q.fz;
  FluidAt f{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
  for (int r = 0; r < 4; ++r) {
    const int jj = (r & 1) ? j1 : j0, kk = (r & 2) ? k1 : k0;
    const double wy = (r & 1) ? fy : 1.0 - fy, wz = (r & 2) ? fz : 1.0 - fz;
    const int row = (kk * P.ny + jj) * P.nx;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int c = row + (a ? i1 : i0);
      const double w = (a ? fx : 1.0 - fx) * wy * wz;
      const double4 u = A.U[c];
      f.Ux += w * u.x;
      f.Uy += w * u.y;
      f.Uz += w * u.z;
      f.es += w * u.w;
      if (P.fluid_forces) {
        if (MODE != 1) {
          const double4 g = A.G[c];
          f.gx += w * g.x;
          f.gy += w * g.y;
          f.gz += w * g.z;
        } else {
          const double4 g = A.gp[c], m = A.du[c];
          f.gx += w * g.x;
          f.gy += w * g.y;
          f.gz += w * g.z;
          f.dx += w * m.x;
          f.dy += w * m.y;
          f.dz += w * m.z;
        }
      }
    }
  }
  return f;
}

// Trilinear interpolation of the cell-centred vorticity W (the lift only).
__device__ __forceinline__ double3 vorticity_at(const DevParams& P, const DevArrays& A, double x,
                                             double y, double z) {
  const Corners q = corners_at(P, A.zgeo + zgeo_centres(P.nz), x, y, z);
  double3 o = make_double3(0.0, 0.0, 0.0);
#pragma unroll 1
  for (int r = 0; r < 8; ++r) {
    const int ii = (r & 1) ? q.i1 : q.i0, jj = (r & 2) ? q.j1 : q.j0, kk = (r & 4) ? q.k1 : q.k0;
    const double w = ((r & 1) ? q.fx : 1.0 - q.fx) * ((r & 2) ? q.fy : 1.0 - q.fy) *
                     ((r & 4) ? q.fz : 1.0 - q.fz);
    const double4 v = A.W[(kk * P.ny + jj) * P.nx + ii];
    o.x += w * v.x;
    o.y += w * v.y;
    o.z += w * v.z;
  }
  return o;
}

// One wall of particle i: side -1 bottom (n = -z), +1 top (n = +z).  The
// wall's history record is touched only when the particle is within the
// lubrication range of the wall or its history is active (mask bit).
template <typename R>
__device__ __forceinline__ void wall(const DevParams& P, int side, double dist, double r,
                                     double m, V3<R> v, V3<R> rw, double4* hist, bool active,
                                     bool update, unsigned bit, unsigned& mask_new, V3<R>& Fc,
                                     V3<R>& Fl, V3<R>& T) {
  double dfull = 2.0 * r;
  double h = dist - r;
  if (!(h < P.lub_out * dfull)) {
    if (update && active) hist->w = 0.0;
    return;
  }
  V3<R> n{(R)0, (R)0, (R)side};
  V3<R> vrel = v + cross(rw, n);
  R un = dot(vrel, n);
  if (P.lubrication) {
    double hin = P.lub_in * dfull;
    R hh = (R)(h > hin ? h : hin);
    R Flub = quot((R)(6.0 * kPi * P.mu_f) * (R)(r * r) * un, hh);
    Fl = Fl - Flub * n;
  }
  double delta = r - dist;
  if (delta > 0.0) {
    R gn = (R)(2.0 * P.zeta) * sqrt((R)m * (R)P.kn);
    R gt = (R)P.gt_over_gn * gn;
    R Frep = (R)P.kn * (R)delta + gn * un;
    V3<R> xi{0, 0, 0};
    if (active) {
      const double4 h0 = *hist;
      xi = cvt<R>(h0.x, h0.y, h0.z);
    }
    V3<R> ft = tangential<R>((R)P.kt, gt, (R)P.mu, (R)P.dt, n, vrel, un, fabs(Frep), xi);
    Fc = Fc + (ft - Frep * n);
    T = T + (R)r * cross(n, ft);
    if (update) {
      *hist = make_double4((double)xi.x, (double)xi.y, (double)xi.z, 1.0);
      mask_new |= bit;
    }
  } else if (update && active) {
    hist->w = 0.0;
  }
}

// r_i w_i + r_j w_j with each product rounded on its own (no fused
// multiply-add), so that both sides of a pair get the same bits.
template <typename R>
__device__ __forceinline__ V3<R> sym_rw(double ri, const double4& wi, double rj,
                                        const double4& wj);
template <>
__device__ __forceinline__ V3<double> sym_rw<double>(double ri, const double4& wi, double rj,
                                                     const double4& wj) {
  return V3<double>{__dadd_rn(__dmul_rn(ri, wi.x), __dmul_rn(rj, wj.x)),
                    __dadd_rn(__dmul_rn(ri, wi.y), __dmul_rn(rj, wj.y)),
                    __dadd_rn(__dmul_rn(ri, wi.z), __dmul_rn(rj, wj.z))};
}
template <>
__device__ __forceinline__ V3<float> sym_rw<float>(double ri, const double4& wi, double rj,
                                                   const double4& wj) {
  const float a = (float)ri, b = (float)rj;
  return V3<float>{__fadd_rn(__fmul_rn(a, (float)wi.x), __fmul_rn(b, (float)wj.x)),
                   __fadd_rn(__fmul_rn(a, (float)wi.y), __fmul_rn(b, (float)wj.y)),
                   __fadd_rn(__fmul_rn(a, (float)wi.z), __fmul_rn(b, (float)wj.z))};
}

// One pair (i, slot k, partner state pj / vj / wj, partner ID idj,
// minimum-image offset (dx, dy, dz), squared distance s) already known to be
// in the pair set: its lubrication and contact forces on i and the contact
// torque on i.  The pair is computed in the frame of its lower-ID particle
// (normal from lower to higher ID) using only sign-symmetric and commutative
// steps, so both sides of the pair compute the same bits; the result is added
// with the sign of i's side.  xi is slot k's tangential history at the start
// of the step (zero if the slot held no contact); the updated history is
// stored back into slot k.
template <typename R>
__device__ __forceinline__ void pair_force(const DevParams& P, const DevArrays& A, int N, int i,
                                           int k, const double4& pi, const double4& pj,
                                           const double4& vj, const double4& wj, int idj,
                                           double dx, double dy, double dz, double s,
                                           const double4& vi, const double4& wi, int idi,
                                           V3<R> xi, bool upd, V3<R>& Fc, V3<R>& Fl,
                                           V3<R>& T, unsigned& mask_new) {
  const double ri = pi.w, mi = vi.w;
  const double rs = ri + pj.w;
  const R kn = (R)P.kn, kt = (R)P.kt, mu = (R)P.mu, dtR = (R)P.dt;
  R* hx = (R*)A.hxi;
  R* hy = hx + (size_t)P.maxn * N;
  R* hz = hy + (size_t)P.maxn * N;
  const bool lo = idi < idj;
  // canonical orientation: from the lower to the higher particle ID
  const double sg = lo ? 1.0 : -1.0;
  dx *= sg;
  dy *= sg;
  dz *= sg;
  const double dist = sqrt(s);
  const double inv = recip(dist);
  const V3<R> n = cvt<R>(dx * inv, dy * inv, dz * inv);
  // Quantities of the lower-ID side computed without selecting operands:
  // sg (v_i - v_j) is exactly v_lo - v_hi (IEEE subtraction is sign
  // symmetric), and r_i w_i + r_j w_j with separately rounded products is the
  // same on both sides (IEEE addition and multiplication commute).
  const V3<R> dv = cvt<R>(sg * (vi.x - vj.x), sg * (vi.y - vj.y), sg * (vi.z - vj.z));
  const V3<R> rw = sym_rw<R>(ri, wi, pj.w, wj);
  const V3<R> vrel = dv + cross(rw, n);
  const R un = dot(vrel, n);
  V3<R> Fpl{0, 0, 0}, Fpc{0, 0, 0};
  if (P.lubrication) {
    const double h = dist - rs, hin = P.lub_in * rs;
    const R hh = (R)(h > hin ? h : hin);
    const R aeff = (R)(ri * pj.w * recip(rs));
    const R Flub = quot((R)(6.0 * kPi * P.mu_f) * aeff * aeff * un, hh);
    Fpl = (-Flub) * n;
  }
  const double delta = rs - dist;
  V3<R> Tp{0, 0, 0};
  if (delta > 0.0) {
    const R meff = (R)(mi * vj.w * recip(mi + vj.w));
    const R gn = (R)(2.0 * P.zeta) * sqrt(meff * kn);
    const R gt = (R)P.gt_over_gn * gn;
    const R Frep = kn * (R)delta + gn * un;
    const size_t o = (size_t)k * N + i;
    const V3<R> ft = tangential<R>(kt, gt, mu, dtR, n, vrel, un, fabs(Frep), xi);
    Fpc = ft - Frep * n;
    Tp = (R)ri * cross(n, ft);
    if (upd) {
      hx[o] = xi.x;
      hy[o] = xi.y;
      hz[o] = xi.z;
      mask_new |= 1u << k;
    }
  }
  // back to i's side (multiplying by +-1 is exact)
  Fc = Fc + (R)sg * Fpc;
  Fl = Fl + (R)sg * Fpl;
  T = T + Tp;
}

// Neighbours of a block's particles lie mostly near them in the sorted order
// (bins in Morton order): the block stages the state of its own particles
// (and of kWin particles on each side) in LDS and reads a neighbour's state
// from there when it falls in that window, from global memory otherwise.  On
// a deposited bed 73% of neighbour reads fall in a 256-particle block itself;
// windows of +-64 / +-128 (80% / 82%, staging up to twice the block) measured
// no faster, while 512-particle blocks, which stage only their own particles,
// are 0.7% faster in FP64 (1024 no faster again).
constexpr int kWin = 0;
// particles per block: 512 in FP64 (4 waves per SIMD either way: two blocks
// of 48 KB per CU), 256 in FP32 (which runs 5 waves per SIMD)
template <typename R>
constexpr int force_block() {
  return sizeof(R) == 8 ? 512 : 256;
}
template <int NS>
struct Staged {
  double4 pos[NS];
  double4 vel[NS];
  double4 omg[NS];  // .w = particle ID
};

// Occupancy: the kernel is bound by the memory latency each SIMD can hide,
// so waves count.  With FP32 pair arithmetic the step kernel fits 5 waves per
// SIMD (95 VGPRs, a 20 B/lane spill outside the pair loop; 3% faster than 4
// waves on the 10M-sphere bed); the FP64 kernels keep the compiler's choice
// (4 waves: forcing 5 spills inside the loop).
template <typename R, int MODE>
__global__ __launch_bounds__(force_block<R>()) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 5 : 1)))
void k_forces(DevParams P, DevArrays A, int update_history) {
  constexpr int kFB = force_block<R>();
  constexpr int kStage = kFB + 2 * kWin;
  __shared__ Staged<kStage> S;
  const int base = xcd_block(blockIdx.x, gridDim.x) * kFB;
  const int i = base + threadIdx.x;
  if (i == 0 && *A.rb) {
    A.ctl->rebuilds += 1;
    *A.rb = 0;
  }
  const int N = P.n;
  const int wlo = base - kWin;
  for (int t = threadIdx.x; t < kStage; t += kFB) {
    const int g = wlo + t;
    if (g >= 0 && g < N) {
      S.pos[t] = A.pos[g];
      S.vel[t] = A.vel[g];
      double4 w = A.omg[g];
      w.w = (double)A.id[g];
      S.omg[t] = w;
    }
  }
  __syncthreads();
  if (i >= N) return;
  const bool upd = update_history != 0;
  const int ti = kWin + threadIdx.x;
  const int idi = (int)S.omg[ti].w;
  const double ri = S.pos[ti].w, mi = S.vel[ti].w;
  V3<R> Fc{0, 0, 0}, Fl{0, 0, 0}, T{0, 0, 0};
  // the step modes need only the sum of contact and lubrication forces:
  // one accumulator for both saves registers
  V3<R>& Flub = MODE == 1 ? Fl : Fc;
  const unsigned mask_old = A.hmask[i];
  unsigned mask_new = 0;
  const int cnt = A.ncnt[i];

  const R* hx = (const R*)A.hxi;
  const R* hy = hx + (size_t)P.maxn * N;
  const R* hz = hy + (size_t)P.maxn * N;
  for (int k = 0; k < cnt; ++k) {
    const int j = A.nbr[(size_t)k * N + i];
    // FP64: the particle's own state is read from LDS in every slot, through
    // an index the compiler cannot hoist, instead of occupying 24 registers
    // across the loop (2% faster at 4 waves per SIMD).  FP32, which runs 5
    // waves, keeps it in registers (the loads are hoisted).
    int tl = ti;
    if (sizeof(R) == 8) asm volatile("" : "+v"(tl));
    const double4 pi = S.pos[tl], vi = S.vel[tl];
    double4 wi = S.omg[tl];
    wi.w = 0.0;
    // The slot's tangential history and the partner's whole state are
    // loaded together, before the range test: a wait for a load also waits
    // for every earlier store (the previous slot's history), so fewer,
    // larger groups of loads per slot pay that wait fewer times.
    V3<R> xi{0, 0, 0};
    if (mask_old & (1u << k)) {
      const size_t o = (size_t)k * N + i;
      xi = V3<R>{hx[o], hy[o], hz[o]};
    }
    const int t = j - wlo;
    const bool staged = (unsigned)t < (unsigned)kStage;
    double4 pj, vj, wj;
    int idj;
    if (staged) {
      pj = S.pos[t];
      vj = S.vel[t];
      wj = S.omg[t];
      idj = (int)wj.w;
    } else {
      pj = A.pos[j];
      vj = A.vel[j];
      wj = A.omg[j];
      idj = A.id[j];
    }
    const double dx = min_image(pj.x - pi.x, P.Lx, P.hLx);
    const double dy = min_image(pj.y - pi.y, P.Ly, P.hLy);
    const double dz = pj.z - pi.z;
    const double s = pair_s(dx, dy, dz);
    if (!pair_in_range(s, ri + pj.w, P.lub_out)) continue;
    pair_force<R>(P, A, N, i, k, pi, pj, vj, wj, idj, dx, dy, dz, s, vi, wi, idi, xi, upd,
                  Fc, Flub, T, mask_new);
  }
  const double4 ai = A.acc[i];  // loaded after the pair loop: not live across it
  const double4 pi = S.pos[ti], vi = S.vel[ti];
  double4 wi = S.omg[ti];
  wi.w = 0.0;
  // flat walls (history validity in mask bits 30 / 31)
  {
    const V3<R> v = cvt<R>(vi.x, vi.y, vi.z);
    const V3<R> rw = (R)ri * cvt<R>(wi.x, wi.y, wi.z);
    if (P.bottom_wall)
      wall<R>(P, -1, pi.z, ri, mi, v, rw, A.wxi + i, (mask_old >> 30) & 1u, upd, 1u << 30,
              mask_new, Fc, Flub, T);
    if (P.top_wall)
      wall<R>(P, 1, P.Lz - pi.z, ri, mi, v, rw, A.wxi + (size_t)N + i, (mask_old >> 31) & 1u,
              upd, 1u << 31, mask_new, Fc, Flub, T);
  }
  if (upd) A.hmask[i] = mask_new;

  // fluid-particle forces at the particle centre; U.w carries the averaged
  // solid fraction; the step kernel reads the pressure-gradient and added-mass
  // fields pre-combined as G = -grad p + C_add rho_f DU/Dt (both enter
  // linearly with the particle volume).
  const double d = 2.0 * ri;
  const double Vp = (kPi / 6.0) * d * d * d;
  const FluidAt fl = fluid_at<MODE>(P, A, pi.x, pi.y, pi.z);
  const double Ux = fl.Ux, Uy = fl.Uy, Uz = fl.Uz;
  const double gpx = fl.gx, gpy = fl.gy, gpz = fl.gz, dux = fl.dx, duy = fl.dy, duz = fl.dz;
  double es = fl.es;
  es = es < 0.0 ? 0.0 : (es > P.eps_s_max ? P.eps_s_max : es);
  const V3<R> wrel = cvt<R>(Ux - vi.x, Uy - vi.y, Uz - vi.z);
  const R wm = sqrt(dot(wrel, wrel));
  const V3<R> Fd = drag_coef<R>(P, (R)d, (R)(1.0 - es), wm) * wrel;
  V3<R> Fp{0, 0, 0}, Fa{0, 0, 0};
  if (P.fluid_forces) {
    const double ca = P.c_add * P.rho_f * Vp;
    if (MODE != 1) {
      // pressure gradient + added mass together
      Fp = cvt<R>(Vp * gpx - ca * ai.x, Vp * gpy - ca * ai.y, Vp * gpz - ca * ai.z);
    } else {
      Fp = cvt<R>(-Vp * gpx, -Vp * gpy, -Vp * gpz);
      Fa = cvt<R>(ca * (dux - ai.x), ca * (duy - ai.y), ca * (duz - ai.z));
    }
  }
  // shear lift C_l rho_f nu^(1/2) d^2 |omega|^(-1/2) (U_f - u_p) x omega
  V3<R> Fy{0, 0, 0};
  if (P.lift_c > 0.0) {
    const double3 om = vorticity_at(P, A, pi.x, pi.y, pi.z);
    const double on = sqrt(om.x * om.x + om.y * om.y + om.z * om.z);
    if (on > 0.0) {
      const double cl = P.lift_c * d * d / sqrt(on);
      const double sx = Ux - vi.x, sy = Uy - vi.y, sz = Uz - vi.z;
      Fy = cvt<R>(cl * (sy * om.z - sz * om.y), cl * (sz * om.x - sx * om.z),
                  cl * (sx * om.y - sy * om.x));
    }
  }
  const V3<R> F = Fc + Fl + Fd + Fp + Fa + Fy;
  const double im = 1.0 / mi;
  const double II = 0.4 * mi * ri * ri;
  const double4 an = make_double4((double)F.x * im + P.gx, (double)F.y * im + P.gy,
                                  (double)F.z * im + P.gz, 0.0);
  const double4 al = make_double4((double)T.x / II, (double)T.y / II, (double)T.z / II, 0.0);
  A.acc[i] = an;
  if (MODE == 2) {
    // second half kick, then the first half kick and drift of the next step
    // (the arithmetic of the separate kick-drift kernel); alpha and the drag
    // are consumed only by a separate kick-drift or a deposition, which never
    // follow this mode directly
    const double hdt = 0.5 * P.dt;
    double4 v = half_kick(vi, an, hdt, mi);
    double4 w = half_kick(wi, al, hdt, 0.0);
    double4 x = pi;
    kick_drift_one(P, A, i, x, v, w, an, al, A.rb_next);
    A.pos_t[i] = x;
    A.vel_t[i] = v;
    A.omg_t[i] = w;
    return;
  }
  A.alp[i] = al;
  A.fdr[i] = make_double4((double)Fd.x, (double)Fd.y, (double)Fd.z, 0.0);
  if (MODE == 0) {
    const double hdt = 0.5 * P.dt;
    A.vel_t[i] = half_kick(vi, an, hdt, mi);
    A.omg_t[i] = half_kick(wi, al, hdt, 0.0);
  } else {
    double4* c = A.comp;
    c[(size_t)0 * N + i] = make_double4(Fc.x, Fc.y, Fc.z, 0.0);
    c[(size_t)1 * N + i] = make_double4(Fl.x, Fl.y, Fl.z, 0.0);
    c[(size_t)2 * N + i] = make_double4(Fd.x, Fd.y, Fd.z, 0.0);
    c[(size_t)3 * N + i] = make_double4(Fp.x, Fp.y, Fp.z, 0.0);
    c[(size_t)4 * N + i] = make_double4(Fa.x, Fa.y, Fa.z, 0.0);
    c[(size_t)5 * N + i] = make_double4((double)F.x + mi * P.gx, (double)F.y + mi * P.gy,
                                        (double)F.z + mi * P.gz, 0.0);
    c[(size_t)6 * N + i] = make_double4(T.x, T.y, T.z, 0.0);
    c[(size_t)7 * N + i] = make_double4(Fy.x, Fy.y, Fy.z, 0.0);
  }
}

// Solid fraction of the last averaging into U.w, where the force kernel reads it.
__global__ void k_pack_eps(DevParams P, DevArrays A) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.ncell) return;
  A.U[c].w = A.smooth[c];
}

}  // namespace

void launch_forces(const DevParams& P, DevArrays& A, int mode, bool update_history,
                   bool mixed, hipStream_t s) {
  if (P.n <= 0) return;
  int u = update_history ? 1 : 0;
  if (mixed) {
    constexpr int fb = force_block<float>();
    const unsigned g = xcd_grid((P.n + fb - 1) / fb);
    if (mode == 0)
      hipLaunchKernelGGL((k_forces<float, 0>), dim3(g), dim3(fb), 0, s, P, A, u);
    else if (mode == 2)
      hipLaunchKernelGGL((k_forces<float, 2>), dim3(g), dim3(fb), 0, s, P, A, u);
    else
      hipLaunchKernelGGL((k_forces<float, 1>), dim3(g), dim3(fb), 0, s, P, A, u);
  } else {
    constexpr int fb = force_block<double>();
    const unsigned g = xcd_grid((P.n + fb - 1) / fb);
    if (mode == 0)
      hipLaunchKernelGGL((k_forces<double, 0>), dim3(g), dim3(fb), 0, s, P, A, u);
    else if (mode == 2)
      hipLaunchKernelGGL((k_forces<double, 2>), dim3(g), dim3(fb), 0, s, P, A, u);
    else
      hipLaunchKernelGGL((k_forces<double, 1>), dim3(g), dim3(fb), 0, s, P, A, u);
  }
}

void launch_pack_eps(const DevParams& P, DevArrays& A, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_eps, dim3((P.ncell + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P,
                     A);
}

}  // namespace sedimi

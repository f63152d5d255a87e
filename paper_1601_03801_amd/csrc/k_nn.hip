// k_nn.hip -- learned stand-in for the diffusion averaging: a 6-layer 3-D
// convolutional network (3x3x3 taps, z dilations 1,2,4,4,2,1, 32 channels,
// residual layers, leaky ReLU, global residual) with BF16 weights and
// activations, FP32 accumulation on the MFMA units, FP32 output.
//
// Convolution as an implicit GEMM on v_mfma_f32_16x16x32_bf16: each MFMA
// computes 16 consecutive cells (M) by 16 output channels (N); K runs over
// (tap, input channel); a wave works on 4 such cell tiles at once.
// Activations are stored channel-last, so the A fragment of a tap (8
// consecutive input channels of one neighbour cell per lane) is 16 contiguous
// bytes; the layer's weights sit in LDS in the order the B fragments are read.
//   - 32 input channels (k_conv_tiled): one tap is one K step; the input is
//     staged through LDS one z-plane of a 64 x 16-cell tile at a time.
//   - 4 input channels (k_conv): two taps share a lane group, K is padded
//     from 108 to 128, and the fragments are gathered directly.
// Both write their outputs through LDS so that the epilogue's loads and
// stores are 8-byte pieces of consecutive channels.
//
// The data gradient of a convolution is the same kernel run with the tap
// offsets negated and the weights transposed; the weight gradient is a GEMM
// over cells (K = cells) whose operands come from LDS through transpose
// reads, with per-block partial sums reduced in a fixed order.
#include <math.h>

#include <algorithm>

#include "k_nn.h"

namespace sedimi {

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float leaky(float z, float a) { return z > 0.0f ? z : a * z; }
__device__ __forceinline__ float dleaky(float z, float a) { return z > 0.0f ? 1.0f : a; }
__device__ __forceinline__ float bf(float v) { return (float)(__bf16)v; }

// z source planes of output plane k for the z-tap offset dz (in taps, not
// scaled by the dilation).  The field is extended along z by reflection about
// the wall faces (mirror padding, period 2 nz).  The forward convolution
// (neg = 0) reads the one plane R(k + dil dz): `which` 0.  Its adjoint
// (neg = 1) gathers every plane k' with R(k' + dil dz) = k: the direct one,
// k' = k - dil dz (`which` 0), and the mirror image, k' = -k - 1 - dil dz
// below the bottom face or 2 nz - 1 - k - dil dz above the top one (`which`
// 1); each exists only when it lies inside the mesh.  -1: no such plane.
template <bool ADJ>
__device__ __forceinline__ int zsrc(const ConvGeom& g, int k, int dz, int which) {
  const int nz = g.nz, nz2 = 2 * nz, lo = g.dil * dz;
  if (!ADJ) {
    if (which) return -1;
    int j = k + lo;
    if (nz >= g.dil) return j < 0 ? -j - 1 : (j >= nz ? nz2 - 1 - j : j);  // one reflection
    j %= nz2;
    j = j < 0 ? j + nz2 : j;
    return j < nz ? j : nz2 - 1 - j;
  }
  int m = which ? -k - 1 - lo : k - lo;
  if (nz >= g.dil) {  // m lies in [-nz - dil, nz + dil): at most one period away
    m = m < 0 ? m + nz2 : (m >= nz2 ? m - nz2 : m);
    return m < nz ? m : -1;
  }
  m %= nz2;
  m = m < 0 ? m + nz2 : m;
  return m < nz ? m : -1;
}

// Neighbour cell of (i, j, k) for tap t and z source `which` (x and y offsets
// negated when neg != 0); -1 when that z source does not exist; periodic in x
// and y.
template <bool ADJ>
__device__ __forceinline__ int tap_cell(const ConvGeom& g, int i, int j, int k, int t,
                                        int which) {
  int dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  if (ADJ) dy = -dy, dx = -dx;
  const int kk = zsrc<ADJ>(g, k, t / 9 - 1, which);
  if (kk < 0) return -1;
  int ii = i + dx;
  ii = ii < 0 ? ii + g.nx : (ii >= g.nx ? ii - g.nx : ii);
  int jj = j + dy;
  jj = jj < 0 ? jj + g.ny : (jj >= g.ny ? jj - g.ny : jj);
  return (kk * g.ny + jj) * g.nx + ii;
}

// Output element o = cell * COUT + n (channel n) of the layer from its
// accumulated convolution v.
template <int EPI>
__device__ __forceinline__ void epilogue(const EpiArgs& e, const float* __restrict__ bias,
                                         size_t o, int n, float v) {
  if (EPI == EPI_FIRST || EPI == EPI_RES) {
    const float zb = bf(v + bias[n]);
    if (e.zout) e.zout[o] = (__bf16)zb;
    float h = leaky(zb, e.alpha);
    if (EPI == EPI_RES) h += (float)e.hin[o];
    e.hout[o] = (__bf16)h;
  } else if (EPI == EPI_LAST) {
    e.yout[o] = e.xres[o] + v + bias[n];
  } else {  // EPI_BWD: dh = acc (+ dh of the layer above); dz = dh * phi'(z)
    float gsum = v + (e.hin ? (float)e.hin[o] : 0.0f);
    const float gb = bf(gsum);
    if (e.hout) e.hout[o] = (__bf16)gb;
    if (e.zout) e.zout[o] = (__bf16)(gb * dleaky((float)e.zin[o], e.alpha));
  }
}

// The same for channels n0 .. n0+3 of one cell (o = cell * 32 + n0): 8-byte
// loads and stores, the same roundings as epilogue().  hres, when given, is
// the residual input of these channels (EPI_RES), already loaded.
template <int EPI>
__device__ __forceinline__ void epilogue4(const EpiArgs& e, const float* __restrict__ bias,
                                          size_t o, int n0, const float4& v4,
                                          const v4bf* hres = nullptr) {
  const float v[4] = {v4.x, v4.y, v4.z, v4.w};
  if (EPI == EPI_FIRST || EPI == EPI_RES) {
    v4bf hin4 = {};
    if (EPI == EPI_RES) hin4 = hres ? *hres : *reinterpret_cast<const v4bf*>(e.hin + o);
    v4bf zb4, h4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float zb = bf(v[q] + bias[n0 + q]);
      zb4[q] = (__bf16)zb;
      float h = leaky(zb, e.alpha);
      if (EPI == EPI_RES) h += (float)hin4[q];
      h4[q] = (__bf16)h;
    }
    if (e.zout) *reinterpret_cast<v4bf*>(e.zout + o) = zb4;
    *reinterpret_cast<v4bf*>(e.hout + o) = h4;
  } else if (EPI == EPI_BWD) {
    v4bf hin4 = {}, zin4 = {};
    if (e.hin) hin4 = *reinterpret_cast<const v4bf*>(e.hin + o);
    if (e.zout) zin4 = *reinterpret_cast<const v4bf*>(e.zin + o);
    v4bf gb4, dz4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float gb = bf(v[q] + (e.hin ? (float)hin4[q] : 0.0f));
      gb4[q] = (__bf16)gb;
      dz4[q] = (__bf16)(gb * dleaky((float)zin4[q], e.alpha));
    }
    if (e.hout) *reinterpret_cast<v4bf*>(e.hout + o) = gb4;
    if (e.zout) *reinterpret_cast<v4bf*>(e.zout + o) = dz4;
  }
}

// Weights in LDS, layout for CIN = 32: [27][NT*16][32]; for CIN = 4:
// [NT*16][128] with k = tap*4 + channel (zero beyond 108).
template <int CIN, int COUT>
struct WShape {
  static constexpr int NT = (COUT + 15) / 16;
  static constexpr int elems = CIN == 32 ? 27 * NT * 16 * 32 : NT * 16 * 128;
};

// Each wave computes TM tiles of 16 cells at once, so per tap it has TM
// independent neighbour loads in flight and reuses each B fragment TM times.
constexpr int TM = 4;

constexpr int kConvThreads = 512;

template <int CIN, int COUT, int EPI>
__global__ __launch_bounds__(kConvThreads) void k_conv(ConvGeom g, const __bf16* __restrict__ in,
                                              const __bf16* __restrict__ wpk,
                                              const float* __restrict__ bias, EpiArgs e) {
  static_assert(CIN == 4 && COUT == 32, "k_conv serves the 4 -> 32 channel convolutions");
  constexpr int NT = WShape<CIN, COUT>::NT;
  constexpr int WE = WShape<CIN, COUT>::elems;
  constexpr int kOS = 36;  // epilogue staging: cell stride in floats
  __shared__ __attribute__((aligned(16))) __bf16 sw[WE];
  __shared__ __attribute__((aligned(16))) float ep[kConvThreads / 64][32 * kOS];
  for (int q = threadIdx.x; q < WE / 8; q += blockDim.x)
    reinterpret_cast<uint4*>(sw)[q] = reinterpret_cast<const uint4*>(wpk)[q];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, grp = lane >> 4;
  const int ngroups = (g.ncell + 16 * TM - 1) / (16 * TM);
  const int wpb = blockDim.x / 64;
  float* wreg = &ep[wave][0];
  for (int tg = blockIdx.x * wpb + wave; tg < ngroups; tg += gridDim.x * wpb) {
    int ci[TM], cj[TM], ck[TM];
    bool valid[TM];
#pragma unroll
    for (int m = 0; m < TM; ++m) {
      const int c = (tg * TM + m) * 16 + row;
      valid[m] = c < g.ncell;
      ci[m] = valid[m] ? c % g.nx : 0;
      cj[m] = valid[m] ? (c / g.nx) % g.ny : 0;
      ck[m] = valid[m] ? c / (g.nx * g.ny) : 0;
    }
    v4f acc[TM][NT];
#pragma unroll
    for (int m = 0; m < TM; ++m)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[m][nt] = v4f{0.f, 0.f, 0.f, 0.f};
    // 4 input channels: two taps share a lane group, K padded from 108 to 128.
    // Pass 0 takes each tap's direct z source; the adjoint then takes a
    // second pass over the mirror-image sources, needed only by waves with a
    // cell within one dilation of a wall (each product accumulates in FP32,
    // as for any other tap).
    constexpr bool kAdj = EPI == EPI_BWD;  // the data gradient: negated offsets
    int npass = 1;
    if (kAdj) {
      bool near = false;
#pragma unroll
      for (int m = 0; m < TM; ++m)
        near |= valid[m] && (ck[m] < g.dil || ck[m] >= g.nz - g.dil);
      npass = __ballot(near) ? 2 : 1;
    }
#pragma unroll 1
    for (int which = 0; which < npass; ++which) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int t0 = 8 * s + 2 * grp, t1 = t0 + 1;
        v8bf a[TM];
#pragma unroll
        for (int m = 0; m < TM; ++m) {
          v4bf lo = {}, hi = {};
          if (valid[m] && t0 < 27) {
            const int q = tap_cell<kAdj>(g, ci[m], cj[m], ck[m], t0, which);
            if (q >= 0) lo = *reinterpret_cast<const v4bf*>(in + (size_t)q * 4);
          }
          if (valid[m] && t1 < 27) {
            const int q = tap_cell<kAdj>(g, ci[m], cj[m], ck[m], t1, which);
            if (q >= 0) hi = *reinterpret_cast<const v4bf*>(in + (size_t)q * 4);
          }
          a[m] = v8bf{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const v8bf b = *reinterpret_cast<const v8bf*>(sw + (nt * 16 + row) * 128 + 32 * s + grp * 8);
#pragma unroll
          for (int m = 0; m < TM; ++m)
            acc[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b, acc[m][nt], 0, 0, 0);
        }
      }
    }
    // acc[m][nt][r] = output (cell (tg*TM + m)*16 + 4*grp + r, channel nt*16 + row).
    // Through the wave's own LDS region, 32 cells at a time, so that each
    // lane then handles 4 consecutive channels of a cell (as in
    // k_conv_tiled).  Only this wave touches its region; the fences keep the
    // compiler from moving the lanes' reads above the other lanes' writes
    // (the LDS executes one wave's accesses in order).
    const int c0 = tg * TM * 16;
#pragma unroll
    for (int ps = 0; ps < 2; ++ps) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int mm = 0; mm < 2; ++mm)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            wreg[(16 * mm + 4 * grp + r) * kOS + nt * 16 + row] = acc[2 * ps + mm][nt][r];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int id = lane + 64 * j;
        const int cl = id >> 3, n0 = 4 * (id & 7);
        const int co = c0 + 32 * ps + cl;
        if (co >= g.ncell) continue;
        const float4 v4 = *reinterpret_cast<const float4*>(wreg + cl * kOS + n0);
        epilogue4<EPI>(e, bias, (size_t)co * 32 + n0, n0, v4);
      }
    }
  }
}

// Convolutions with 32 input channels, tiled through LDS.  A block of 16
// waves owns an output tile of 64 (x) by 16 (y) cells in one z-plane; wave w
// computes row w of it as 4 MFMA tiles of 16 cells.  The taps are taken one
// z-plane at a time: the block copies the input plane (the tile plus a
// one-cell halo in x and y, periodic) into LDS with coalesced 16-byte loads,
// then every wave reads the A fragments of the plane's 9 taps from LDS,
// where 16 consecutive cells of one row are 1 KB of contiguous LDS (no bank
// conflicts).  Each input cell is thus read from memory about 1.3 times per
// plane (halo) instead of once per tap through L1.  The next plane is loaded
// into registers while the current one feeds the matrix cores.
//
// The planes of a tile are jobs (z-tap p, source plane): the forward takes
// one source per z-tap (mirror padding, zsrc), the adjoint one or two (a
// direct plane and a mirror image), and some z-taps of its planes next to a
// wall have none.  Job j = 2 pi + which for pi = 0..2 in the tap order below.
constexpr int kTileX = 64, kTileY = 16;
constexpr int kTiledThreads = 64 * kTileY;
constexpr int kHaloX = kTileX + 2, kHaloY = kTileY + 2;
constexpr int kPlaneUnits = kHaloY * kHaloX * 4;  // 16-byte units of a staged plane
constexpr int kUnitsPerThread = (kPlaneUnits + kTiledThreads - 1) / kTiledThreads;

template <int COUT, int EPI>
__global__ __launch_bounds__(kTiledThreads) void k_conv_tiled(ConvGeom g,
                                                              const __bf16* __restrict__ in,
                                                              const __bf16* __restrict__ wpk,
                                                              const float* __restrict__ bias,
                                                              EpiArgs e) {
  constexpr int NT = WShape<32, COUT>::NT;
  constexpr int WE = WShape<32, COUT>::elems;
  __shared__ __attribute__((aligned(16))) __bf16 sw[WE];
  __shared__ __attribute__((aligned(16))) __bf16 sp[kHaloY][kHaloX][32];
  for (int q = threadIdx.x; q < WE / 8; q += blockDim.x)
    reinterpret_cast<uint4*>(sw)[q] = reinterpret_cast<const uint4*>(wpk)[q];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, grp = lane >> 4;
  const int ntx = (g.nx + kTileX - 1) / kTileX, nty = (g.ny + kTileY - 1) / kTileY;
  const int ntiles = ntx * nty * g.nz;
  constexpr bool kAdj = EPI == EPI_BWD;  // the data gradient: negated offsets
  const int sgn = kAdj ? -1 : 1;
  // Residual layers take the centre z-tap last: it then stays in LDS for the
  // epilogue, which reads the residual input h_in (the layer's own input,
  // plane z itself) from there instead of from memory.
  constexpr bool kCentreLast = EPI == EPI_RES;
  auto phase = [](int i) { return kCentreLast ? (i == 0 ? 0 : (i == 1 ? 2 : 1)) : i; };
  // source plane of job j of output plane tz (-1: none); z-tap p covers the
  // forward offset dz = p - 1
  auto job_src = [&](int tz, int j) { return zsrc<kAdj>(g, tz, phase(j >> 1) - 1, j & 1); };
  // the tile's jobs as a bit mask (bit j: job j has a source plane)
  auto jobs_of = [&](int tz) {
    unsigned m = 0;
    for (int j = 0; j < 6; ++j)
      if (!(j & 1) || kAdj) m |= (job_src(tz, j) >= 0 ? 1u : 0u) << j;
    return m;
  };
  auto lowest = [](unsigned m) { return __builtin_ctz(m); };
  // Plane of (tile, job) -> registers.  The loads are unconditional (clamped
  // to valid addresses): conditional loads would make the compiler merge and
  // copy the registers, which waits for the loads right away.
  uint4 st[kUnitsPerThread];
  // (kc is computed at the call sites, so that the lambda stays small, is
  // inlined, and st stays in registers)
  auto fetch = [&](int tile, int kc) __attribute__((always_inline)) {
    const int tx = tile % ntx, ty = (tile / ntx) % nty;
#pragma unroll
    for (int q = 0; q < kUnitsPerThread; ++q) {
      int u = threadIdx.x + q * kTiledThreads;
      u = u < kPlaneUnits ? u : kPlaneUnits - 1;
      const int ry = u / (kHaloX * 4), rem = u % (kHaloX * 4);
      const int px = rem / 4, part = rem % 4;
      int ii = (tx * kTileX - 1 + px) % g.nx;
      ii = ii < 0 ? ii + g.nx : ii;
      int jj = (ty * kTileY - 1 + ry) % g.ny;
      jj = jj < 0 ? jj + g.ny : jj;
      const size_t c = ((size_t)kc * g.ny + jj) * g.nx + ii;
      st[q] = *reinterpret_cast<const uint4*>(in + c * 32 + part * 8);
    }
  };
  int tile = blockIdx.x;
  // every plane has at least one job: the centre z-tap's direct source
  unsigned jobs = tile < ntiles ? jobs_of(tile / (ntx * nty)) : 0u;
  if (tile < ntiles) fetch(tile, job_src(tile / (ntx * nty), lowest(jobs)));
  for (; tile < ntiles; tile += gridDim.x) {
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int next = tile + (int)gridDim.x < ntiles ? tile + (int)gridDim.x : tile;
    const unsigned next_jobs = jobs_of(next / (ntx * nty));
    v4f acc[TM][NT];
#pragma unroll
    for (int m = 0; m < TM; ++m)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[m][nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (unsigned left = jobs; left; left &= left - 1) {
      const int j = lowest(left);
      const int p = phase(j >> 1);
      __syncthreads();  // every wave is done with the previous plane
#pragma unroll
      for (int q = 0; q < kUnitsPerThread; ++q) {
        const int u = threadIdx.x + q * kTiledThreads;
        // member by member: a whole-struct copy of the vector type keeps st
        // out of registers (it is then spilled to scratch between loads)
        if (u < kPlaneUnits)
          reinterpret_cast<uint4*>(&sp[0][0][0])[u] = make_uint4(st[q].x, st[q].y, st[q].z, st[q].w);
      }
      __syncthreads();
      // the next plane (of this tile, else the first of the next tile; the
      // last tile refetches its own first plane) is in flight during the MFMAs
      // (one call site: loads in two branches would be waited for at the join)
      const unsigned rest = left & (left - 1);
      const int ft = rest ? tile : next;
      fetch(ft, job_src(ft / (ntx * nty), rest ? lowest(rest) : lowest(next_jobs)));
#pragma unroll 1
      for (int t9 = 0; t9 < 9; ++t9) {
        const int t = p * 9 + t9;
        const int ly = wave + 1 + sgn * (t9 / 3 - 1);
        const int lx = row + 1 + sgn * (t9 % 3 - 1);
        v8bf a[TM];
#pragma unroll
        for (int m = 0; m < TM; ++m)
          a[m] = *reinterpret_cast<const v8bf*>(&sp[ly][lx + 16 * m][grp * 8]);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const v8bf b = *reinterpret_cast<const v8bf*>(sw + ((t * NT + nt) * 16 + row) * 32 + grp * 8);
#pragma unroll
          for (int m = 0; m < TM; ++m)
            acc[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b, acc[m][nt], 0, 0, 0);
        }
      }
    }
    // acc[m][nt][r] = output (x = tile x0 + 16 m + 4 grp + r, y = y0 + wave, channel nt*16 + row)
    const int cy = ty * kTileY + wave;
    if (COUT == 32) {
      // Through LDS, half a row (32 cells x 32 channels, FP32) per wave and
      // pass, into the wave's own region of the plane buffer (cell stride 36
      // floats: the 64 lanes of a write hit 64 different banks).  Then each
      // lane takes 4 consecutive channels of a cell, so consecutive lanes
      // cover consecutive 8-byte pieces of the channel-last outputs.
      constexpr int kOS = 36;
      static_assert(kTileY * 32 * kOS * 4 <= (int)sizeof(sp), "epilogue staging exceeds the plane buffer");
      // h_in of this lane's output pieces, from the centre plane still in LDS
      v4bf hres[2][4];
      if (kCentreLast) {
#pragma unroll
        for (int ps = 0; ps < 2; ++ps)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int id = lane + 64 * j;
            const int cl = id >> 3, n0 = 4 * (id & 7);
            hres[ps][j] = *reinterpret_cast<const v4bf*>(&sp[wave + 1][32 * ps + cl + 1][n0]);
          }
      }
      float* wreg = reinterpret_cast<float*>(&sp[0][0][0]) + wave * 32 * kOS;
#pragma unroll
      for (int ps = 0; ps < 2; ++ps) {
        __syncthreads();  // the plane (or the previous pass) is no longer read
#pragma unroll
        for (int mm = 0; mm < 2; ++mm)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              wreg[(16 * mm + 4 * grp + r) * kOS + nt * 16 + row] = acc[2 * ps + mm][nt][r];
        __syncthreads();
        if (cy < g.ny) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int id = lane + 64 * j;
            const int cl = id >> 3, n0 = 4 * (id & 7);
            const int cx = tx * kTileX + 32 * ps + cl;
            if (cx >= g.nx) continue;
            const float4 v4 = *reinterpret_cast<const float4*>(wreg + cl * kOS + n0);
            const size_t co = ((size_t)tz * g.ny + cy) * g.nx + cx;
            epilogue4<EPI>(e, bias, co * 32 + n0, n0, v4, kCentreLast ? &hres[ps][j] : nullptr);
          }
        }
      }
    } else if (cy < g.ny) {
#pragma unroll
      for (int m = 0; m < TM; ++m)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int n = nt * 16 + row;
          if (n >= COUT) continue;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int cx = tx * kTileX + 16 * m + 4 * grp + r;
            if (cx >= g.nx) continue;
            const size_t co = ((size_t)tz * g.ny + cy) * g.nx + cx;
            epilogue<EPI>(e, bias, co * COUT + n, n, acc[m][nt][r]);
          }
        }
    }
    jobs = next_jobs;
  }
}

// Weight and bias gradients of one convolution: dW[t][i][o] = sum_cells
// x[nb(c,t)][i] dy[c][o], as per-block partials.  K of the GEMM runs over
// cells, so both MFMA operands need 8 consecutive cells of one channel per
// lane while the activations are channel-last.  A chunk is 32 consecutive
// cells of kDwRows consecutive x-rows of one z-plane; its dy and the input
// row segments it touches (3 z-planes x (kDwRows + 2) rows, 34 cells each,
// shared by the x-taps and by neighbouring rows) are copied into LDS
// unchanged, and the operands are read with the LDS transpose read
// (ds_read_b64_tr_b16): within each 16-lane group, lane 4b+a receives element
// a of the 4-element rows addressed by lanes b, b+4, b+8, b+12.  If lane r
// addresses cell base + r/4, channels 4(r%4) .. 4(r%4)+3, lane t receives
// cells base..base+3 of channel t.  Wave w owns taps w, w+8, ...; each row of
// the chunk is one K step.  The next chunk is loaded into registers while the
// current one feeds the matrix cores.
typedef short v4s __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4s lds_v4s;

__device__ __forceinline__ v8bf tr_pair(const __bf16* p0, const __bf16* p1) {
  v4s a = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)p0);
  v4s b = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)p1);
  v8bf r;
  __builtin_memcpy(&r, &a, 8);
  __builtin_memcpy(reinterpret_cast<char*>(&r) + 8, &b, 8);
  return r;
}

constexpr int kDwThreads = 512;
constexpr int kDwRows = 4;

template <int CIN, int COUT>
__global__ __launch_bounds__(kDwThreads) void k_conv_dw(ConvGeom g, const __bf16* __restrict__ x,
                                                        const __bf16* __restrict__ dy,
                                                        float* __restrict__ part,
                                                        float* __restrict__ part_b) {
  constexpr int CP = CIN < 16 ? 16 : CIN;    // padded input channels (M)
  constexpr int OP = COUT < 16 ? 16 : COUT;  // padded output channels (N)
  constexpr int MT = CP / 16, NT = OP / 16;
  constexpr int NW = kDwThreads / 64;
  constexpr int SLOTS = (27 + NW - 1) / NW;  // taps per wave
  constexpr int SEG = 34;                    // row segment: cells x0-1 .. x0+32
  constexpr int XR = kDwRows + 2;            // staged rows per z-plane
  constexpr int XU = CIN / 4;                // 8-byte units per cell of x
  constexpr int YU = COUT / 4;               // 8-byte units per cell of dy
  constexpr int XUNITS = 3 * XR * SEG * XU, YUNITS = kDwRows * 32 * YU;
  constexpr int XPT = (XUNITS + kDwThreads - 1) / kDwThreads;
  constexpr int YPT = (YUNITS + kDwThreads - 1) / kDwThreads;
  static_assert(kDwThreads % YU == 0, "each thread must keep one dy channel block");
  __shared__ __attribute__((aligned(16))) __bf16 xs[3][XR][SEG][CP];
  __shared__ __attribute__((aligned(16))) __bf16 dys[kDwRows][32][OP];
  __shared__ float bsum[kDwThreads][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t16 = lane & 15, grp = lane >> 4;
  // zero the padding channels once (never overwritten)
  for (int q = threadIdx.x; q < 3 * XR * SEG * CP; q += kDwThreads) (&xs[0][0][0][0])[q] = (__bf16)0.0f;
  for (int q = threadIdx.x; q < kDwRows * 32 * OP; q += kDwThreads) (&dys[0][0][0])[q] = (__bf16)0.0f;
  v4f acc[SLOTS][MT][NT];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s)
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int b = 0; b < NT; ++b) acc[s][a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  float bacc[4] = {0, 0, 0, 0};
  const int nseg = (g.nx + 31) / 32, nrow = (g.ny + kDwRows - 1) / kDwRows;
  const int nchunks = nseg * nrow * g.nz;
  // Chunk -> registers.  Loads are unconditional (clamped to valid cells);
  // the x planes are mirrored into the mesh along z, and the dy cells beyond
  // a ragged row end are zeroed when the registers are written to LDS, from
  // the bit masks: conditional loads would make the compiler copy the
  // registers and wait for the loads at once.
  uint2 rx[XPT], ry[YPT];
  unsigned mx = 0, my = 0;  // bit q: unit q holds data
  auto fetch = [&](int ch) {
    const int seg = ch % nseg, rb = (ch / nseg) % nrow, ck = ch / (nseg * nrow);
    const int x0 = seg * 32, y0 = rb * kDwRows;
    mx = 0;
    my = 0;
#pragma unroll
    for (int q = 0; q < YPT; ++q) {
      const int u = threadIdx.x + q * kDwThreads;
      const int rr = u / (32 * YU), rem = u % (32 * YU);
      const int cl = rem / YU, blk = rem % YU;
      const int yy = y0 + rr, xx = x0 + cl;
      const bool ok = u < YUNITS && yy < g.ny && xx < g.nx;
      const size_t c = ok ? ((size_t)ck * g.ny + yy) * g.nx + xx : 0;
      ry[q] = *reinterpret_cast<const uint2*>(dy + c * COUT + blk * 4);
      my |= (ok ? 1u : 0u) << q;
    }
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int u = threadIdx.x + q * kDwThreads;
      const int pz = u / (XR * SEG * XU), rem = u % (XR * SEG * XU);
      const int pr = rem / (SEG * XU), rem2 = rem % (SEG * XU);
      const int pc = rem2 / XU, blk = rem2 % XU;
      int kk = (ck + g.dil * (pz - 1)) % (2 * g.nz);  // mirror padding in z
      kk = kk < 0 ? kk + 2 * g.nz : kk;
      kk = kk < g.nz ? kk : 2 * g.nz - 1 - kk;
      const bool ok = u < XUNITS;
      int jj = (y0 - 1 + pr) % g.ny;
      jj = jj < 0 ? jj + g.ny : jj;
      int ii = (x0 - 1 + pc) % g.nx;
      ii = ii < 0 ? ii + g.nx : ii;
      const size_t c = ok ? ((size_t)kk * g.ny + jj) * g.nx + ii : 0;
      rx[q] = *reinterpret_cast<const uint2*>(x + c * CIN + blk * 4);
      mx |= (ok ? 1u : 0u) << q;
    }
  };
  int ch = blockIdx.x;
  if (ch < nchunks) fetch(ch);
  __syncthreads();
  for (; ch < nchunks; ch += gridDim.x) {
#pragma unroll
    for (int q = 0; q < YPT; ++q) {
      const int u = threadIdx.x + q * kDwThreads;
      if (u >= YUNITS) continue;
      const unsigned keep = ((my >> q) & 1u) ? ~0u : 0u;
      const uint2 v = make_uint2(ry[q].x & keep, ry[q].y & keep);
      const int rr = u / (32 * YU), rem = u % (32 * YU);
      const int cl = rem / YU, blk = rem % YU;
      *reinterpret_cast<uint2*>(&dys[rr][cl][blk * 4]) = v;
      const __bf16* e = reinterpret_cast<const __bf16*>(&v);
#pragma unroll
      for (int k = 0; k < 4; ++k) bacc[k] += (float)e[k];
    }
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int u = threadIdx.x + q * kDwThreads;
      if (u >= XUNITS) continue;
      const unsigned keep = ((mx >> q) & 1u) ? ~0u : 0u;
      const int pz = u / (XR * SEG * XU), rem = u % (XR * SEG * XU);
      const int pr = rem / (SEG * XU), rem2 = rem % (SEG * XU);
      const int pc = rem2 / XU, blk = rem2 % XU;
      *reinterpret_cast<uint2*>(&xs[pz][pr][pc][blk * 4]) =
          make_uint2(rx[q].x & keep, rx[q].y & keep);
    }
    __syncthreads();
    // the next chunk (the last one refetches itself) is in flight meanwhile
    fetch(ch + (int)gridDim.x < nchunks ? ch + (int)gridDim.x : ch);
#pragma unroll
    for (int slot = 0; slot < SLOTS; ++slot) {
      const int t = wave + NW * slot;
      if (t < 27) {
        const int pz = t / 9, dyi = (t / 3) % 3, dxi = t % 3;  // z-plane, row and x shift + 1
#pragma unroll 1
        for (int rr = 0; rr < kDwRows; ++rr) {
#pragma unroll
          for (int a = 0; a < MT; ++a) {
            const __bf16* pa = &xs[pz][rr + dyi][8 * grp + (t16 >> 2) + dxi][16 * a + 4 * (t16 & 3)];
            const v8bf A = tr_pair(pa, pa + 4 * CP);
#pragma unroll
            for (int b = 0; b < NT; ++b) {
              const __bf16* pb = &dys[rr][8 * grp + (t16 >> 2)][16 * b + 4 * (t16 & 3)];
              const v8bf B = tr_pair(pb, pb + 4 * OP);
              acc[slot][a][b] =
                  __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[slot][a][b], 0, 0, 0);
            }
          }
        }
      }
    }
    __syncthreads();
  }
  // partials: C rows m = a*16 + 4*grp + q (input channel), col n = b*16 + t16
  float* pb = part + (size_t)blockIdx.x * 27 * CIN * COUT;
#pragma unroll
  for (int slot = 0; slot < SLOTS; ++slot) {
    const int t = wave + NW * slot;
    if (t >= 27) continue;
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int b = 0; b < NT; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int m = a * 16 + 4 * grp + q, n = b * 16 + t16;
          if (m < CIN && n < COUT) pb[((size_t)t * CIN + m) * COUT + n] = acc[slot][a][b][q];
        }
  }
  // bias: thread u always loaded dy channel block u % YU (kDwThreads % YU == 0)
  for (int q = 0; q < 4; ++q) bsum[threadIdx.x][q] = bacc[q];
  __syncthreads();
  if ((int)threadIdx.x < COUT) {
    const int blk = threadIdx.x / 4, q = threadIdx.x % 4;
    float s2 = 0.0f;
    for (int u = blk; u < kDwThreads; u += YU) s2 += bsum[u][q];
    part_b[(size_t)blockIdx.x * COUT + threadIdx.x] = s2;
  }
}

// out[k] = sum over blocks of part[b][k] in a fixed order: the blocks in four
// contiguous segments (one wave each, 64 outputs per workgroup), each summed
// with four interleaved accumulators so that four loads are in flight, then
// the partial sums added pairwise.
__global__ __launch_bounds__(256) void k_reduce_parts(const float* __restrict__ part,
                                                      int nblocks, int len,
                                                      float* __restrict__ out) {
  __shared__ float seg[4][64];
  const int kk = threadIdx.x & 63, sgi = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + kk;
  float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
  if (k < len) {
    const int b1 = (int)((int64_t)(sgi + 1) * nblocks / 4);
    int b = (int)((int64_t)sgi * nblocks / 4);
    for (; b + 3 < b1; b += 4) {
      a0 += part[(size_t)b * len + k];
      a1 += part[(size_t)(b + 1) * len + k];
      a2 += part[(size_t)(b + 2) * len + k];
      a3 += part[(size_t)(b + 3) * len + k];
    }
    for (; b < b1; ++b) a0 += part[(size_t)b * len + k];
  }
  seg[sgi][kk] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (sgi == 0 && k < len) out[k] = (seg[0][kk] + seg[1][kk]) + (seg[2][kk] + seg[3][kk]);
}

// Normalised input: xf [c][4] = (raw[ch][c] - mean) / std, and its BF16 copy.
__global__ void k_nn_prep(int ncell, const double* __restrict__ raw, NNNorm nm,
                          float* __restrict__ xf, __bf16* __restrict__ xb) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  for (int ch = 0; ch < 4; ++ch) {
    float v = (float)((raw[(size_t)ch * ncell + c] - nm.mean[ch]) / nm.std[ch]);
    xf[(size_t)c * 4 + ch] = v;
    xb[(size_t)c * 4 + ch] = (__bf16)v;
  }
}

// The network's input: what the skip leaves behind, x - S x, in BF16.
__global__ void k_nn_highpass(int64_t n4, const float* __restrict__ xf,
                              const float* __restrict__ xs, __bf16* __restrict__ xb) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4;
       q += (int64_t)gridDim.x * blockDim.x)
    xb[q] = (__bf16)(xf[q] - xs[q]);
}

// Network output back to the smoothed field: smooth[ch][c] = y*std + mean.
__global__ void k_nn_out(int ncell, const float* __restrict__ y, NNNorm nm,
                         double* __restrict__ smooth) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  for (int ch = 0; ch < 4; ++ch)
    smooth[(size_t)ch * ncell + c] = (double)y[(size_t)c * 4 + ch] * nm.std[ch] + nm.mean[ch];
}

// Loss gradient: target t = (smooth - mean)/std; with the channel weight w,
// dy = (2 w / (4 n)) (y - t) in BF16 (the factor 2 w / (4 n) formed in FP32);
// per-block FP64 partial sums of w (y - t)^2.
__global__ void k_nn_loss(int ncell, const float* __restrict__ y,
                          const double* __restrict__ smooth, NNNorm nm,
                          __bf16* __restrict__ dy, double* __restrict__ part) {
  __shared__ double s[256];
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (c < ncell) {
    const float scale = 2.0f / (4.0f * (float)ncell);
    for (int ch = 0; ch < 4; ++ch) {
      float t = (float)((smooth[(size_t)ch * ncell + c] - nm.mean[ch]) / nm.std[ch]);
      float d = y[(size_t)c * 4 + ch] - t;
      acc += nm.lw[ch] * ((double)d * (double)d);
      const float sw = scale * (float)nm.lw[ch];
      dy[(size_t)c * 4 + ch] = (__bf16)(sw * d);
    }
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// Adam on the FP32 master parameters.
__global__ void k_adam(int64_t n, float* __restrict__ w, float* __restrict__ m,
                       float* __restrict__ v, const float* __restrict__ gr, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float g = gr[k];
  float mm = b1 * m[k] + (1.0f - b1) * g;
  float vv = b2 * v[k] + (1.0f - b2) * g * g;
  m[k] = mm;
  v[k] = vv;
  w[k] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Zero the entries of one layer's weights a[27][cin][cout] that join two
// different channel groups.  A side with 4 channels has one field per group;
// a wider side splits into 4 equal groups of consecutive channels.
__global__ void k_group_mask(float* __restrict__ a, int cin, int cout) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 27 * cin * cout) return;
  const int i = (q / cout) % cin, o = q % cout;
  const int gi = cin == 4 ? i : i / (cin / 4), go = cout == 4 ? o : o / (cout / 4);
  if (gi != go) a[q] = 0.0f;
}

// Pack one layer's FP32 weights w[27][cin][cout] into the BF16 layouts the
// convolution kernel reads: forward and (for layers > 1) the transposed
// adjoint used by the data gradient.
__global__ void k_pack(const float* __restrict__ w, int cin, int cout,
                       __bf16* __restrict__ fwd, __bf16* __restrict__ adj) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 27 * cin * cout) return;
  const int t = q / (cin * cout), i = (q / cout) % cin, o = q % cout;
  const __bf16 v = (__bf16)w[q];
  // forward: input channels i, output channels o
  if (cin == 32) {
    const int ntp = ((cout + 15) / 16) * 16;
    fwd[((size_t)t * ntp + o) * 32 + i] = v;
  } else {
    fwd[(size_t)o * 128 + t * 4 + i] = v;
  }
  // adjoint: input channels o, output channels i (offsets negated at run time)
  if (adj) {
    if (cout == 32) {
      const int ntp = ((cin + 15) / 16) * 16;
      adj[((size_t)t * ntp + i) * 32 + o] = v;
    } else {
      adj[(size_t)i * 128 + t * 4 + o] = v;
    }
  }
}

// ---- the network's skip S: the diffusion split by axis ----
// out = S_a in along one periodic axis (a = x: stride 1, length nx; a = y:
// stride nx, length ny) as a circulant: out[i] = sum_t tap[t] in[i + off0 + t]
// (wrapped), FP64 sums of the FP32 channel-last cells.
__global__ void k_split_line(int nx, int ny, int nz, int axis, int off0, int ntap,
                             const double* __restrict__ tap, const float4* __restrict__ in,
                             float4* __restrict__ out) {
  const int64_t ncell = (int64_t)nx * ny * nz;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % nx), j = (int)((c / nx) % ny);
    const int n = axis == 0 ? nx : ny;
    const int pos = axis == 0 ? i : j;
    const int64_t stride = axis == 0 ? 1 : nx;
    const int64_t base = c - (int64_t)pos * stride;
    int q = (pos + off0) % n;
    q = q < 0 ? q + n : q;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int t = 0; t < ntap; ++t) {
      const float4 v = in[base + (int64_t)q * stride];
      const double w = tap[t];
      a0 += w * v.x, a1 += w * v.y, a2 += w * v.z, a3 += w * v.w;
      q = q + 1 == n ? 0 : q + 1;
    }
    out[c] = make_float4((float)a0, (float)a1, (float)a2, (float)a3);
  }
}

// The same circulant with the lines staged in LDS, so that each cell is read
// from memory once and its ntap reads come from LDS: along x a block holds
// whole x-lines, along y a tile of kSplitTX consecutive x-columns of one
// z-plane over the whole y-line.  Same taps and FP64 sums in the same order,
// so the same bits as k_split_line.
constexpr int kSplitTX = 16;
__global__ __launch_bounds__(256) void k_split_x_lds(int nx, int ny, int nz, int off0, int ntap,
                                                     const double* __restrict__ tap,
                                                     const float4* __restrict__ in,
                                                     float4* __restrict__ out) {
  extern __shared__ float4 line[];  // [nx]
  const int64_t nlines = (int64_t)ny * nz;
  for (int64_t l = blockIdx.x; l < nlines; l += gridDim.x) {
    const int64_t base = l * nx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) line[i] = in[base + i];
    __syncthreads();
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
      int q = (i + off0) % nx;
      q = q < 0 ? q + nx : q;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      for (int t = 0; t < ntap; ++t) {
        const float4 v = line[q];
        const double w = tap[t];
        a0 += w * v.x, a1 += w * v.y, a2 += w * v.z, a3 += w * v.w;
        q = q + 1 == nx ? 0 : q + 1;
      }
      out[base + i] = make_float4((float)a0, (float)a1, (float)a2, (float)a3);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_split_y_lds(int nx, int ny, int nz, int off0, int ntap,
                                                     const double* __restrict__ tap,
                                                     const float4* __restrict__ in,
                                                     float4* __restrict__ out) {
  extern __shared__ float4 tile[];  // [ny][kSplitTX]
  const int ntx = (nx + kSplitTX - 1) / kSplitTX;
  const int64_t ntiles = (int64_t)ntx * nz;
  for (int64_t b = blockIdx.x; b < ntiles; b += gridDim.x) {
    const int k = (int)(b / ntx), x0 = (int)(b % ntx) * kSplitTX;
    const int tw = nx - x0 < kSplitTX ? nx - x0 : kSplitTX;
    const int64_t plane = (int64_t)k * ny * nx;
    for (int e = threadIdx.x; e < ny * kSplitTX; e += blockDim.x) {
      const int y = e / kSplitTX, x = e % kSplitTX;
      if (x < tw) tile[e] = in[plane + (int64_t)y * nx + x0 + x];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ny * kSplitTX; e += blockDim.x) {
      const int y = e / kSplitTX, x = e % kSplitTX;
      if (x >= tw) continue;
      int q = (y + off0) % ny;
      q = q < 0 ? q + ny : q;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      for (int t = 0; t < ntap; ++t) {
        const float4 v = tile[q * kSplitTX + x];
        const double w = tap[t];
        a0 += w * v.x, a1 += w * v.y, a2 += w * v.z, a3 += w * v.w;
        q = q + 1 == ny ? 0 : q + 1;
      }
      out[plane + (int64_t)y * nx + x0 + x] = make_float4((float)a0, (float)a1, (float)a2, (float)a3);
    }
    __syncthreads();
  }
}

// S_z: ntau backward-Euler steps along z with zero-flux walls, in place.  A
// block of 64 lanes takes kSplitCols consecutive columns, one lane per
// (column, channel) pair, the columns held in LDS as FP32 (FP64 sums):
// 16 columns x nz planes x 4 channels, 32 KB at nz = 128, so several blocks
// share a CU.  tab: reciprocal pivots [nz] then the Thomas multipliers [nz]
// of the tridiagonal (1 + c n_k) u_k - c u_{k-1} - c u_{k+1}, n_k the number
// of neighbours of plane k.
constexpr int kSplitCols = 16;
__global__ __launch_bounds__(64) void k_split_z(int nx, int ny, int nz, int ntau, double c,
                                                const double* __restrict__ tab,
                                                float4* __restrict__ f4) {
  extern __shared__ float col[];  // [nz][kSplitCols * 4]
  constexpr int W = kSplitCols * 4;
  float* f = reinterpret_cast<float*>(f4);
  const int64_t plane = (int64_t)nx * ny;
  const int64_t c0 = (int64_t)blockIdx.x * kSplitCols;
  const int t = threadIdx.x;  // column c0 + t / 4, channel t % 4
  const bool live = c0 + t / 4 < plane;
  for (int k = 0; k < nz; ++k)
    if (live) col[k * W + t] = f[(k * plane + c0) * 4 + t];
  if (live && nz > 1) {
    const double* ib = tab;       // 1 / pivot
    const double* gm = tab + nz;  // multiplier of the back substitution
    for (int s = 0; s < ntau; ++s) {
      // forward sweep: u_k = (f_k + c u_{k-1}) / pivot_k
      double p = col[t] * ib[0];
      col[t] = (float)p;
      for (int k = 1; k < nz; ++k) {
        p = (col[k * W + t] + c * p) * ib[k];
        col[k * W + t] = (float)p;
      }
      // back substitution: u_k -= gamma_{k+1} u_{k+1}, carried in FP64
      for (int k = nz - 2; k >= 0; --k) {
        p = col[k * W + t] - gm[k + 1] * p;
        col[k * W + t] = (float)p;
      }
    }
  }
  for (int k = 0; k < nz; ++k)
    if (live) f[(k * plane + c0) * 4 + t] = col[k * W + t];
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

size_t split_lds_bytes(int nz) { return (size_t)nz * kSplitCols * 4 * sizeof(float); }

void launch_split(int nx, int ny, int nz, int ntau, const SplitTabs& st, const float* in,
                  float* tmp, float* out, hipStream_t s) {
  const int64_t ncell = (int64_t)nx * ny * nz;
  const unsigned g = (unsigned)std::min<int64_t>((ncell + 255) / 256, 4096);
  // LDS-staged lines when a line (x) or a y-tile fits in 32 KB
  constexpr size_t kSplitLds = 32768;
  const size_t bx = (size_t)nx * sizeof(float4), by = (size_t)ny * kSplitTX * sizeof(float4);
  const int64_t nxl = (int64_t)ny * nz, nyt = (int64_t)((nx + kSplitTX - 1) / kSplitTX) * nz;
  if (bx <= kSplitLds)
    hipLaunchKernelGGL(k_split_x_lds, dim3((unsigned)std::min<int64_t>(nxl, 8192)), dim3(256), bx,
                       s, nx, ny, nz, st.off0x, st.ntapx, st.tapx, (const float4*)in,
                       (float4*)tmp);
  else
    hipLaunchKernelGGL(k_split_line, dim3(g), dim3(256), 0, s, nx, ny, nz, 0, st.off0x, st.ntapx,
                       st.tapx, (const float4*)in, (float4*)tmp);
  if (by <= kSplitLds)
    hipLaunchKernelGGL(k_split_y_lds, dim3((unsigned)std::min<int64_t>(nyt, 8192)), dim3(256), by,
                       s, nx, ny, nz, st.off0y, st.ntapy, st.tapy, (const float4*)tmp,
                       (float4*)out);
  else
    hipLaunchKernelGGL(k_split_line, dim3(g), dim3(256), 0, s, nx, ny, nz, 1, st.off0y, st.ntapy,
                       st.tapy, (const float4*)tmp, (float4*)out);
  const int64_t plane = (int64_t)nx * ny;
  hipLaunchKernelGGL(k_split_z, dim3((unsigned)((plane + kSplitCols - 1) / kSplitCols)),
                     dim3(kSplitCols * 4), split_lds_bytes(nz), s, nx, ny, nz, ntau, st.cz,
                     st.ztab, (float4*)out);
}

size_t nn_packed_elems(int cin, int cout) {
  int nt = (cout + 15) / 16;
  return cin == 32 ? (size_t)27 * nt * 16 * 32 : (size_t)nt * 16 * 128;
}

void launch_conv(int cin, int cout, int epi, const ConvGeom& g, const __bf16* in,
                 const __bf16* wpk, const float* bias, const EpiArgs& e, hipStream_t s) {
  if (cin == 32) {
    const int64_t ntiles = (int64_t)((g.nx + kTileX - 1) / kTileX) *
                           ((g.ny + kTileY - 1) / kTileY) * g.nz;
    if (ntiles == 0) return;
    // one block of 16 waves per CU, persistent over the tiles
    const unsigned grid = (unsigned)(ntiles < 256 ? ntiles : 256);
#define SEDIMI_CONV_T(CO, EP)                                                           \
    if (cout == CO && epi == EP) {                                                      \
      hipLaunchKernelGGL((k_conv_tiled<CO, EP>), dim3(grid), dim3(kTiledThreads), 0, s, g, in, \
                         wpk, bias, e);                                                 \
      return;                                                                           \
    }
    SEDIMI_CONV_T(32, EPI_RES)
    SEDIMI_CONV_T(4, EPI_LAST)
    SEDIMI_CONV_T(32, EPI_BWD)
#undef SEDIMI_CONV_T
    return;
  }
  int ngroups = (g.ncell + 16 * TM - 1) / (16 * TM);
  const int wpb = kConvThreads / 64;
  unsigned grid = (unsigned)((ngroups + wpb - 1) / wpb);
  if (grid > 1024) grid = 1024;
  if (grid == 0) return;
#define SEDIMI_CONV(CI, CO, EP)                                                             \
  if (cin == CI && cout == CO && epi == EP) {                                             \
    hipLaunchKernelGGL((k_conv<CI, CO, EP>), dim3(grid), dim3(kConvThreads), 0, s, g, in, wpk, bias, e); \
    return;                                                                               \
  }
  SEDIMI_CONV(4, 32, EPI_FIRST)
  SEDIMI_CONV(4, 32, EPI_BWD)
#undef SEDIMI_CONV
}

int launch_conv_dw(int cin, int cout, const ConvGeom& g, const __bf16* x, const __bf16* dy,
                   float* part, float* part_b, float* dw, float* db, int nblocks,
                   hipStream_t s) {
  if (cin == 32 && cout == 32)
    hipLaunchKernelGGL((k_conv_dw<32, 32>), dim3(nblocks), dim3(kDwThreads), 0, s, g, x, dy, part, part_b);
  else if (cin == 4 && cout == 32)
    hipLaunchKernelGGL((k_conv_dw<4, 32>), dim3(nblocks), dim3(kDwThreads), 0, s, g, x, dy, part, part_b);
  else if (cin == 32 && cout == 4)
    hipLaunchKernelGGL((k_conv_dw<32, 4>), dim3(nblocks), dim3(kDwThreads), 0, s, g, x, dy, part, part_b);
  else
    return -1;
  int len = 27 * cin * cout;
  hipLaunchKernelGGL(k_reduce_parts, dim3((len + 63) / 64), dim3(256), 0, s, part, nblocks, len, dw);
  hipLaunchKernelGGL(k_reduce_parts, dim3((cout + 63) / 64), dim3(256), 0, s, part_b, nblocks, cout,
                     db);
  return 0;
}

void launch_nn_prep(int ncell, const double* raw, const NNNorm& nm, float* xf, __bf16* xb,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_nn_prep, dim3(nblk(ncell)), dim3(256), 0, s, ncell, raw, nm, xf, xb);
}
void launch_nn_highpass(int ncell, const float* xf, const float* xs, __bf16* xb, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_highpass, dim3(2048), dim3(256), 0, s, (int64_t)ncell * 4, xf, xs, xb);
}
void launch_nn_out(int ncell, const float* y, const NNNorm& nm, double* smooth, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_out, dim3(nblk(ncell)), dim3(256), 0, s, ncell, y, nm, smooth);
}
unsigned launch_nn_loss(int ncell, const float* y, const double* smooth, const NNNorm& nm,
                        __bf16* dy, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_loss, dim3(nblk(ncell)), dim3(256), 0, s, ncell, y, smooth, nm, dy, part);
  return nblk(ncell);
}
void launch_adam(int64_t n, float* w, float* m, float* v, const float* g, float lr, float b1,
                 float b2, float eps, int64_t t, hipStream_t s) {
  float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, s, n, w, m, v, g, lr, b1, b2, eps, c1, c2);
}
void launch_group_mask(float* a, int cin, int cout, hipStream_t s) {
  hipLaunchKernelGGL(k_group_mask, dim3(nblk(27 * cin * cout)), dim3(256), 0, s, a, cin, cout);
}
void launch_pack(const float* w, int cin, int cout, __bf16* fwd, __bf16* adj, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(nblk(27 * cin * cout)), dim3(256), 0, s, w, cin, cout, fwd, adj);
}

}  // namespace sedimi

// k_neighbors.hip -- drift, binning, stable re-sort and neighbour-list build
// (link-cell binning with neighbour lists, Section 2.5).
//
// A rebuild runs only when some particle has moved more than half the skin
// since the last build (decided on the device in k_kick_drift); every
// rebuild kernel reads that flag and returns at once when it is clear, so the
// host can enqueue the whole chain every step without a round trip.
//
// Re-sort: counting sort by bin, the bins taken in Morton (Z-curve) order of
// their 3-D coordinates so that spatial neighbours are also near in memory
// (integer atomics give the counts; the order inside a bin is then fixed by
// sorting its few members by particle ID), so
// the sorted order, the neighbour order and hence all force sums are
// deterministic.  The tangential history survives a re-sort as (partner ID,
// xi) rows and is matched back onto the new list slots by partner ID.
#include "k_common.h"

namespace sedimi {

namespace {

__device__ __forceinline__ bool gate(const int* flag) { return *flag != 0; }

// exclusive scans of int counts: 1024 items per block
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__global__ void k_zero_ints(int* p, int64_t n, int gated, const int* flag) {
  if (gated && !gate(flag)) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// First half kick and drift of velocity Verlet; wrap on the periodic axes;
// escape / non-finite checks; skin test against the positions of the last
// build (minimum image).
__global__ void k_kick_drift(DevParams P, DevArrays A) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P.n) return;
  double4 x = A.pos[q], v = A.vel[q], w = A.omg[q];
  const double4 a = A.acc[q], al = A.alp[q];
  kick_drift_one(P, A, q, x, v, w, a, al, A.rb);
  A.pos[q] = x;
  A.vel[q] = v;
  A.omg[q] = w;
}

// Active slot history -> (partner ID, xi) rows of particle p, before the re-sort.
template <typename H>
__device__ __forceinline__ void compact_one(const DevParams& P, const DevArrays& A, int p) {
  const int N = P.n;
  unsigned m = A.hmask[p];
  int cnt = A.ncnt[p];
  const H* hx = (const H*)A.hxi;
  const H* hy = hx + (size_t)P.maxn * N;
  const H* hz = hy + (size_t)P.maxn * N;
  int c = 0;
  for (int k = 0; k < cnt; ++k) {
    if (!(m & (1u << k))) continue;
    if (c >= kMaxContacts) {
      atomicOr(&A.ctl->flags, kFlagOverflow);
      break;
    }
    int j = A.nbr[(size_t)k * N + p];
    A.cid[(size_t)c * N + p] = A.id[j];
    A.cxi[((size_t)0 * kMaxContacts + c) * N + p] = (double)hx[(size_t)k * N + p];
    A.cxi[((size_t)1 * kMaxContacts + c) * N + p] = (double)hy[(size_t)k * N + p];
    A.cxi[((size_t)2 * kMaxContacts + c) * N + p] = (double)hz[(size_t)k * N + p];
    ++c;
  }
  A.ccnt[p] = c;
}

// Bin key of particle p (bins in Morton order) and its rank among the bin's
// members (any order: k_permute orders each bin by ID).  Particles still in
// the last sorted order mostly share a bin with their wave neighbours: each
// group of lanes with one bin takes its ranks with a single atomic add.
// Every lane of the wave calls this (valid says whether p is a particle).
__device__ __forceinline__ void keys_one(const DevParams& P, const DevArrays& A, int p,
                                         bool valid) {
  int b = -1;
  if (valid) {
    const double4 x = A.pos[p];
    b = A.bin_rank[bin_of(P, x.x, x.y, x.z)];
    A.key[p] = b;
  }
  const int rank = wave_ranks(A.bin_count, b, valid);
  if (valid) A.rank[p] = rank;
}

// First kernel of a rebuild: history rows (when the list slots carry
// history) and bin keys, one pass over the particles.  The loop runs while
// any lane of the block has a particle, so whole waves reach keys_one.
template <typename H, bool SLOTS>
__global__ void k_compact_keys(DevParams P, DevArrays A) {
  if (!gate(A.rb)) return;
  const int stride = gridDim.x * blockDim.x;
  for (int p0 = blockIdx.x * blockDim.x; p0 < P.n; p0 += stride) {
    const int p = p0 + threadIdx.x;
    const bool valid = p < P.n;
    if (SLOTS && valid) compact_one<H>(P, A, p);
    keys_one(P, A, p, valid);
  }
}


// Scatter by bin, finishing the bin scan on the way: bin_count holds each
// bin's exclusive prefix within its scan tile and scan_tmp the exclusive
// offsets of the tiles, the total last (k_scan_bins).  A particle's slot is
// its bin's start plus its rank; the blocks also write the final bin starts.
__global__ void k_scatter(DevParams P, DevArrays A) {
  if (!gate(A.rb)) return;
  const int* toff = A.scan_tmp;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P.n;
       p += gridDim.x * blockDim.x) {
    const int b = A.key[p];
    A.perm[A.bin_count[b] + toff[b / kScanTile] + A.rank[p]] = p;
  }
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < P.nbins;
       b += gridDim.x * blockDim.x)
    A.bin_start[b] = A.bin_count[b] + toff[b / kScanTile];
  if (blockIdx.x == 0 && threadIdx.x == 0)
    A.bin_start[P.nbins] = toff[(P.nbins + kScanTile - 1) / kScanTile];
}

// Second half of the re-sort: k_scatter left each bin's members in arbitrary
// order; every element takes its rank by particle ID among its bin's members
// (bins hold a handful of particles, so each counts them all) and copies its
// state into the spare copies at that place.  The sorted permutation goes to
// A.rank, free once k_scatter has run, for the list build.  A crowded bin
// keeps the scatter order and raises kFlagCrowded.
__global__ void k_permute(DevParams P, DevArrays A) {
  if (!gate(A.rb)) return;
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < P.n;
       m += gridDim.x * blockDim.x) {
    const int p = A.perm[m];
    const int b = A.key[p];
    const int s = A.bin_start[b], e = A.bin_start[b + 1];
    int q = m;
    if (e - s > kMaxBinMembers) {
      if (m == s) atomicOr(&A.ctl->flags, kFlagCrowded);
    } else {
      const int idp = A.id[p];
      int r = 0;
      for (int t = s; t < e; ++t) r += A.id[A.perm[t]] < idp;
      q = s + r;
    }
    A.rank[q] = p;
    A.pos_t[q] = A.pos[p];
    A.vel_t[q] = A.vel[p];
    A.omg_t[q] = A.omg[p];
    A.acc_t[q] = A.acc[p];
    A.alp_t[q] = A.alp[p];
    A.fdr_t[q] = A.fdr[p];
    A.wxi_t[q] = A.wxi[p];
    A.wxi_t[(size_t)P.n + q] = A.wxi[(size_t)P.n + p];
    A.id_t[q] = A.id[p];
  }
}

// Neighbour list of particle q: every particle in the 27 surrounding bins
// within (pair range + skin), ordered by class: overlapping (in contact)
// first, then within the lubrication range, then the rest; in bin-scan order
// within a class.  The force kernel walks the slots of a wave's particles in
// lockstep and runs the contact and lubrication code for a slot when any lane
// needs it, so putting each list's contacts first about halves the slots
// that run the contact code (and touch the tangential history).
// One pass over the bins, a row of three (consecutive x) at a time: while a
// row is tested, the member ranges of the next row and the bin ranks of the
// one after are loaded; a row's three ranges are joined into one run of
// candidates, whose positions are loaded kBuildBatch at a time (a lane waits
// on one memory round trip per batch, not per candidate or per bin).
// Candidates are tested in bin-scan order and parked with their class in the
// lane's row of LDS.  The list is then written class by class, and each
// slot's tangential history is matched by partner ID against the contact
// rows of q's pre-sort position, whose IDs are held in registers.
// WRAP (at least 5 bins on each periodic axis): a candidate's periodic image
// is known from its bin alone.  A neighbour bin reached without wrapping lies
// within 2 bins, i.e. within L/2, where the minimum image is the plain
// difference; one reached across the seam lies beyond L/2, where it is the
// difference -/+ L.  Adding that per-bin shift is the very operation the
// minimum-image selection would pick, so the distances, and the lists, are
// bit-identical, for a fifth of the instructions per candidate.
constexpr int kBuildStride = 31;  // LDS row of a lane: >= max_neighbors, odd (no bank conflicts)
static_assert(kBuildStride >= 30, "a lane's LDS row must hold max_neighbors (<= 30) slots");
constexpr int kWrapMinBins = 5;
constexpr int kBuildBatch = 6;  // candidate loads in flight per lane
template <typename H, bool WRAP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_build(DevParams P, DevArrays A) {
  if (!gate(A.rb)) return;
  __shared__ int park[kBlock * kBuildStride];
  int* row = park + threadIdx.x * kBuildStride;
  int most = 0;  // the lane's largest list
  // each XCD works through one contiguous range of particles, whose
  // neighbours' positions then stay in that XCD's L2
  for (int q = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; q < P.n;
       q += gridDim.x * blockDim.x) {
    const int N = P.n;
    // the re-sorted state is still in the _t copies: the build reads
    // positions, IDs and wall histories there and copies particle q back
    const double4 xi = A.pos_t[q];
    const int bx = bin_coord(xi.x, P.hbx, P.nbx), by = bin_coord(xi.y, P.hby, P.nby),
              bz = bin_coord(xi.z, P.hbz, P.nbz);
    const int cxm = bx == 0 ? P.nbx - 1 : bx - 1, cxp = bx + 1 == P.nbx ? 0 : bx + 1;
    // the scan tests every candidate (no early stop, so consecutive
    // candidates' loads do not wait on each other); the first maxn are kept
    // and more than maxn overflow the list
    int seen = 0;
    unsigned long long cls = 0;  // 2 bits of class per kept candidate
    // bin ranks of a row (all -1 when the row lies outside the grid in z) and
    // the bounds of its three member ranges: a row's ranges are loaded while
    // the row before it is tested, and its ranks one row earlier still
    auto row_ranks = [&](int r, int (&rk)[3]) {
      const int cz = bz + r / 3 - 1;
      rk[0] = rk[1] = rk[2] = -1;
      if (r < 9 && cz >= 0 && cz < P.nbz) {
        int cy = by + r % 3 - 1;
        cy = cy < 0 ? cy + P.nby : (cy >= P.nby ? cy - P.nby : cy);
        const int base = (cz * P.nby + cy) * P.nbx;
        rk[0] = A.bin_rank[base + cxm];
        rk[1] = A.bin_rank[base + bx];
        rk[2] = A.bin_rank[base + cxp];
      }
    };
    auto row_bounds = [&](const int (&rk)[3], int (&lo)[3], int (&hi)[3]) {
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        lo[t] = rk[0] >= 0 ? A.bin_start[rk[t]] : 0;
        hi[t] = rk[0] >= 0 ? A.bin_start[rk[t] + 1] : 0;
      }
    };
    int rk_next[3], lo[3], hi[3];
    row_ranks(0, rk_next);
    row_bounds(rk_next, lo, hi);
    row_ranks(1, rk_next);
    const double sx0 = bx == 0 ? -P.Lx : 0.0, sx2 = bx + 1 == P.nbx ? P.Lx : 0.0;
#pragma unroll 1
    for (int r = 0; r < 9; ++r) {
      int lo_next[3], hi_next[3];
      row_bounds(rk_next, lo_next, hi_next);
      row_ranks(r + 2, rk_next);
      {
        const int cyr = by + r % 3 - 1;
        const double sy = cyr < 0 ? -P.Ly : (cyr >= P.nby ? P.Ly : 0.0);
        // the row's three member ranges as one run of candidates (a crowded
        // bin, flagged by k_permute, counts as empty; a row outside the grid
        // has none)
        const int s0 = lo[0], s1 = lo[1], s2 = lo[2];
        int n0 = hi[0] - s0, n1 = hi[1] - s1, n2 = hi[2] - s2;
        n0 = n0 > kMaxBinMembers ? 0 : n0;
        n1 = n1 > kMaxBinMembers ? 0 : n1;
        n2 = n2 > kMaxBinMembers ? 0 : n2;
        const int n01 = n0 + n1, nrow = n01 + n2;
        // kBuildBatch candidates' loads in flight at once, then tested in
        // scan order
        for (int c0 = 0; c0 < nrow; c0 += kBuildBatch) {
          int js[kBuildBatch];
          double4 xs[kBuildBatch];
#pragma unroll
          for (int u = 0; u < kBuildBatch; ++u) {
            const int c = c0 + u;
            js[u] = c < n0 ? s0 + c : (c < n01 ? s1 + (c - n0) : s2 + (c - n01));
            xs[u] = c < nrow ? A.pos_t[js[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
          }
#pragma unroll
          for (int u = 0; u < kBuildBatch; ++u) {
            const int c = c0 + u;
            const int j = js[u];
            if (c >= nrow || j == q) continue;
            const double4 xj = xs[u];
            const double sx = c < n0 ? sx0 : (c < n01 ? 0.0 : sx2);
            const double ddx = WRAP ? (xj.x - xi.x) + sx : min_image(xj.x - xi.x, P.Lx, P.hLx);
            const double ddy = WRAP ? (xj.y - xi.y) + sy : min_image(xj.y - xi.y, P.Ly, P.hLy);
            const double ddz = xj.z - xi.z;
            const double s2 = ddx * ddx + ddy * ddy + ddz * ddz;
            const double rs = xi.w + xj.w;
            const double Rl = rs + P.lub_out * rs + P.skin;
            if (!(s2 < Rl * Rl * (1.0 + 1e-9))) continue;
            const double Rp = rs + P.lub_out * rs;
            const unsigned long long k = s2 < rs * rs ? 0 : (s2 < Rp * Rp ? 1 : 2);
            if (seen < P.maxn) {
              row[seen] = j;
              cls |= k << (2 * seen);
            }
            ++seen;
          }
        }
      }
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        lo[t] = lo_next[t];
        hi[t] = hi_next[t];
      }
    }
    int cnt = seen;
    if (cnt > P.maxn) {
      atomicOr(&A.ctl->flags, kFlagOverflow);
      cnt = P.maxn;
    }
    most = cnt > most ? cnt : most;
    A.ncnt[q] = cnt;
    A.xb[q] = xi;
    // contact rows of the pre-sort position p (the sorted permutation that
    // k_permute left in A.rank): partner IDs in registers
    const int p = A.rank[q];
    const int nc = A.ccnt[p];
    int cid[kMaxContacts];
#pragma unroll
    for (int c = 0; c < kMaxContacts; ++c) cid[c] = c < nc ? A.cid[(size_t)c * N + p] : -1;
    H* hx = (H*)A.hxi;
    H* hy = hx + (size_t)P.maxn * N;
    H* hz = hy + (size_t)P.maxn * N;
    unsigned mask = 0;
    int matched = 0;
    int w0 = 0, w1 = 0, w2 = 0;
    for (int k = 0; k < cnt; ++k) {
      const int c = (int)((cls >> (2 * k)) & 3ull);
      w1 += c == 0;
      w2 += c != 2;
    }
    // slots kBuildBatch at a time: the partners' IDs are gathered together,
    // then the matched history rows, so a lane waits on two memory round
    // trips per batch rather than on one or two per slot
#pragma unroll 1
    for (int k0 = 0; k0 < cnt; k0 += kBuildBatch) {
      int jj[kBuildBatch], pid[kBuildBatch];
#pragma unroll
      for (int u = 0; u < kBuildBatch; ++u) {
        const int k = k0 + u;
        jj[u] = k < cnt ? row[k] : 0;
        pid[u] = (k < cnt && nc > 0) ? A.id_t[jj[u]] : -1;
      }
      int hw[kBuildBatch], hr[kBuildBatch];
#pragma unroll
      for (int u = 0; u < kBuildBatch; ++u) {
        const int k = k0 + u;
        hw[u] = 0;
        hr[u] = -1;
        if (k < cnt) {
          const int c = (int)((cls >> (2 * k)) & 3ull);
          const int w = c == 0 ? w0++ : (c == 1 ? w1++ : w2++);
          A.nbr[(size_t)w * N + q] = jj[u];
          // partner IDs in a list are distinct: at most one row matches
          int hit = -1;
#pragma unroll
          for (int r = 0; r < kMaxContacts; ++r) hit = pid[u] >= 0 && cid[r] == pid[u] ? r : hit;
          hw[u] = w;
          hr[u] = hit;
        }
      }
      double gx[kBuildBatch], gy[kBuildBatch], gz[kBuildBatch];
#pragma unroll
      for (int u = 0; u < kBuildBatch; ++u) {
        gx[u] = gy[u] = gz[u] = 0.0;
        if (hr[u] >= 0) {
          gx[u] = A.cxi[((size_t)0 * kMaxContacts + hr[u]) * N + p];
          gy[u] = A.cxi[((size_t)1 * kMaxContacts + hr[u]) * N + p];
          gz[u] = A.cxi[((size_t)2 * kMaxContacts + hr[u]) * N + p];
        }
      }
#pragma unroll
      for (int u = 0; u < kBuildBatch; ++u) {
        if (hr[u] < 0) continue;
        hx[(size_t)hw[u] * N + q] = (H)gx[u];
        hy[(size_t)hw[u] * N + q] = (H)gy[u];
        hz[(size_t)hw[u] * N + q] = (H)gz[u];
        mask |= 1u << hw[u];
        ++matched;
      }
    }
    const double4 wall0 = A.wxi_t[q], wall1 = A.wxi_t[(size_t)N + q];
    if (wall0.w != 0.0) mask |= 1u << 30;
    if (wall1.w != 0.0) mask |= 1u << 31;
    A.hmask[q] = mask;
    if (matched != nc) atomicOr(&A.ctl->flags, kFlagLost);
    A.pos[q] = xi;
    A.vel[q] = A.vel_t[q];
    A.omg[q] = A.omg_t[q];
    A.acc[q] = A.acc_t[q];
    A.alp[q] = A.alp_t[q];
    A.fdr[q] = A.fdr_t[q];
    A.wxi[q] = wall0;
    A.wxi[(size_t)N + q] = wall1;
    A.id[q] = A.id_t[q];
  }
  // the bin counts are no longer needed: clear them for the next rebuild
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < P.nbins; b += gridDim.x * blockDim.x)
    A.bin_count[b] = 0;
  // the largest list: one atomic per wave, not per particle (all lanes of
  // the wave are back together here)
  for (int o = 32; o > 0; o >>= 1) {
    const int other = __shfl_xor(most, o, 64);
    most = other > most ? other : most;
  }
  if ((threadIdx.x & 63) == 0 && most > 0) atomicMax(&A.ctl->max_nbr, most);
}

// ---- exclusive scan of int counts (2 passes, 1024 items per block) ----

__device__ int block_exclusive(int v, int* lds, int* total) {
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  int off = 0, tot = 0;
  for (int w = 0; w < kBlock / 64; ++w) {
    int s = lds[w];
    if (w < wid) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ void k_scan_tiles(const int* cnt, int* start, int n, int* tile_sums, int gated,
                             const int* flag) {
  if (gated && !gate(flag)) return;
  __shared__ int lds[kBlock / 64];
  int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int sum = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? cnt[base + k] : 0;
    sum += v[k];
  }
  int tot;
  int ex = block_exclusive(sum, lds, &tot);
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) start[base + k] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}


// Second pass: each tile adds the sum of all tiles before it (read and
// reduced by the tile's own block, so no third pass is needed); the last
// tile also writes the total to start[n].
__global__ void k_scan_add(int* start, int n, const int* tile_sums, int ntiles, int gated,
                           const int* flag) {
  if (gated && !gate(flag)) return;
  __shared__ int lds[kBlock / 64];
  const int b = blockIdx.x;
  int part = 0;
  for (int t = threadIdx.x; t < b; t += kBlock) part += tile_sums[t];
  int off;
  (void)block_exclusive(part, lds, &off);
  const int base = b * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += kBlock)
    if (base + k < n) start[base + k] += off;
  if (b == ntiles - 1 && threadIdx.x == 0) start[n] = off + tile_sums[b];
}

// The bin scan in one launch: each block turns its tile of counts in place
// into exclusive prefixes within the tile and publishes the tile's total;
// the block that finishes last (one atomic counter, nobody waits) turns the
// totals into exclusive tile offsets, with the grand total after them, and
// resets the counter.  k_scatter adds the offsets.  One block per tile.
__global__ void k_scan_bins(int* cnt, int n, int* tiles, int* done, const int* flag) {
  if (!gate(flag)) return;
  __shared__ int lds[kBlock / 64];
  __shared__ int last;
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int sum = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? cnt[base + k] : 0;
    sum += v[k];
  }
  int tot;
  int ex = block_exclusive(sum, lds, &tot);
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) cnt[base + k] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) {
    tiles[blockIdx.x] = tot;
    __threadfence();
    last = atomicAdd(done, 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  const int nt = gridDim.x;
  const int per = (nt + kBlock - 1) / kBlock;
  const int t0 = threadIdx.x * per, t1 = t0 + per < nt ? t0 + per : nt;
  int part = 0;
  for (int t = t0; t < t1; ++t)
    part += __hip_atomic_load(&tiles[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int total;
  int off = block_exclusive(part, lds, &total);
  for (int t = t0; t < t1; ++t) {
    const int x = __hip_atomic_load(&tiles[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tiles[t] = off;
    off += x;
  }
  if (threadIdx.x == 0) {
    tiles[nt] = total;
    *done = 0;
  }
}

// Which neighbour slots of each particle are in the pair set right now (the
// same exact test the force kernel applies); bit k of out[q] = slot k.
__global__ void k_pairmask(DevParams P, DevArrays A, unsigned* out) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P.n) return;
  const int N = P.n;
  double4 pi = A.pos[q];
  unsigned m = 0;
  for (int k = 0; k < A.ncnt[q]; ++k) {
    double4 pj = A.pos[A.nbr[(size_t)k * N + q]];
    double dx = min_image(pj.x - pi.x, P.Lx, P.hLx);
    double dy = min_image(pj.y - pi.y, P.Ly, P.hLy);
    double dz = pj.z - pi.z;
    if (pair_in_range(pair_s(dx, dy, dz), pi.w + pj.w, P.lub_out)) m |= 1u << k;
  }
  out[q] = m;
}

// Periodic translation of positions and of the last-build positions.
__global__ void k_translate(DevParams P, DevArrays A, double dx, double dy) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P.n) return;
  double4 x = A.pos[q], b = A.xb[q];
  double nx = fmod(x.x + dx, P.Lx), ny = fmod(x.y + dy, P.Ly);
  if (nx < 0.0) nx += P.Lx;
  if (ny < 0.0) ny += P.Ly;
  if (nx >= P.Lx) nx = 0.0;
  if (ny >= P.Ly) ny = 0.0;
  b.x += nx - x.x;
  b.y += ny - x.y;
  x.x = nx;
  x.y = ny;
  A.pos[q] = x;
  A.xb[q] = b;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
// Grid of the rebuild-chain kernels: they loop over their range, so a few
// blocks per CU suffice when a rebuild runs, and when it does not (most
// steps) each launch only dispatches these blocks, which read the flag and
// return.
constexpr unsigned kGatedBlocks = 1024;
inline unsigned gated_grid(int64_t n) {
  const unsigned b = nblk(n);
  return b < kGatedBlocks ? (b > 0 ? b : 1) : kGatedBlocks;
}

}  // namespace

void launch_translate(const DevParams& P, DevArrays& A, double dx, double dy, hipStream_t s) {
  if (P.n <= 0) return;
  hipLaunchKernelGGL(k_translate, dim3(nblk(P.n)), dim3(kBlock), 0, s, P, A, dx, dy);
}

void launch_pairmask(const DevParams& P, DevArrays& A, unsigned* out, hipStream_t s) {
  if (P.n <= 0) return;
  hipLaunchKernelGGL(k_pairmask, dim3(nblk(P.n)), dim3(kBlock), 0, s, P, A, out);
}

void launch_zero_ints(int* p, int64_t n, bool gated, const int* flag, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero_ints, dim3(gated_grid(n)), dim3(kBlock), 0, s, p, n, gated ? 1 : 0,
                     flag);
}

void launch_exclusive_scan(int* cnt, int* start, int n, int* tmp, bool gated, const int* flag,
                           hipStream_t s) {
  int ntiles = (n + kScanTile - 1) / kScanTile;
  if (ntiles == 0) ntiles = 1;
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kBlock), 0, s, cnt, start, n, tmp,
                     gated ? 1 : 0, flag);
  hipLaunchKernelGGL(k_scan_add, dim3(ntiles), dim3(kBlock), 0, s, start, n, tmp, ntiles,
                     gated ? 1 : 0, flag);
}

void launch_kick_drift(const DevParams& P, DevArrays& A, hipStream_t s) {
  if (P.n <= 0) return;
  hipLaunchKernelGGL(k_kick_drift, dim3(nblk(P.n)), dim3(kBlock), 0, s, P, A);
}

void launch_rebuild(const DevParams& P, DevArrays& A, bool from_slots, bool mixed,
                    hipStream_t s) {
  if (P.n <= 0) return;
  unsigned g = gated_grid(P.n);
  // the bin counts are zero here: set_particles clears them and every
  // rebuild clears them again in k_build
  if (!from_slots)
    hipLaunchKernelGGL((k_compact_keys<double, false>), dim3(g), dim3(kBlock), 0, s, P, A);
  else if (mixed)
    hipLaunchKernelGGL((k_compact_keys<float, true>), dim3(g), dim3(kBlock), 0, s, P, A);
  else
    hipLaunchKernelGGL((k_compact_keys<double, true>), dim3(g), dim3(kBlock), 0, s, P, A);
  hipLaunchKernelGGL(k_scan_bins, dim3((P.nbins + kScanTile - 1) / kScanTile), dim3(kBlock), 0, s,
                     A.bin_count, P.nbins, A.scan_tmp, &A.ctl->scan_done, A.rb);
  hipLaunchKernelGGL(k_scatter, dim3(g), dim3(kBlock), 0, s, P, A);
  hipLaunchKernelGGL(k_permute, dim3(g), dim3(kBlock), 0, s, P, A);
  // the list build is latency bound: every particle gets its own lane (the
  // grid a multiple of the XCD count for the block renumbering)
  const unsigned gb = xcd_grid(nblk(P.n) < 8192 ? nblk(P.n) : 8192);
  const bool wrap = P.nbx >= kWrapMinBins && P.nby >= kWrapMinBins;
  if (mixed && wrap)
    hipLaunchKernelGGL((k_build<float, true>), dim3(gb), dim3(kBlock), 0, s, P, A);
  else if (mixed)
    hipLaunchKernelGGL((k_build<float, false>), dim3(gb), dim3(kBlock), 0, s, P, A);
  else if (wrap)
    hipLaunchKernelGGL((k_build<double, true>), dim3(gb), dim3(kBlock), 0, s, P, A);
  else
    hipLaunchKernelGGL((k_build<double, false>), dim3(gb), dim3(kBlock), 0, s, P, A);
}

}  // namespace sedimi

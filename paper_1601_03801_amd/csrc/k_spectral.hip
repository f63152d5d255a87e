// k_spectral.hip -- direct solve of the implicit diffusion averaging.
//
// Each pseudo-time step of the averaging (Eq. 12, backward Euler with
// Delta tau = tau / N_tau) solves (I - Delta tau L_h) e_{m+1} = e_m with L_h
// the 7-point finite-volume Laplacian: periodic in x and y, zero-flux faces
// at z = 0 and Lz.  On a uniform mesh that operator is diagonalised by a
// real orthogonal basis: the discrete Hartley transform along the periodic
// axes (cas(2 pi p q / n), an eigenvector of every symmetric circulant with
// eigenvalue (2 - 2 cos(2 pi p / n)) / h^2) and the DCT-II along z
// (cos(pi m (k + 1/2) / n), eigenvalue (2 - 2 cos(pi m / n)) / h^2).  All
// N_tau steps together are then
//   smooth = T^-1 diag((1 + Delta tau lambda)^-N_tau) T raw,
// with T = H_x (x) H_y (x) C_z applied one axis at a time.  Every axis
// transform is a small dense real matrix product over the field, done here
// as a tiled FP64 GEMM; the spectral factor is applied in the epilogue of the
// forward z pass.  Six passes over
// the field replace the tens of stencil sweeps of an iterative solve.
//
// On a z mesh graded towards the bottom wall (Section 4's channel case) the
// z operator is the finite-volume one (face flux over the centre distance,
// per unit cell height), not a DCT-diagonal matrix; it is similar to a
// symmetric tridiagonal matrix through the square roots of the cell
// heights, whose eigenvectors (computed once on the host) replace C_z and
// its inverse.  The x and y transforms and the passes are unchanged.
//
// The GEMM runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64): a block
// computes a 64 x 64 tile of C with four waves of 32 x 32 (2 x 2 MFMA tiles);
// K is staged through LDS 16 at a time.  Per MFMA a lane reads one double of
// A and one of B, against eight LDS reads per 16 FMAs for a 4 x 4 outer
// product on the vector units.
#include <algorithm>
#include <mutex>
#include <vector>
#include <string>

#include "k_common.h"

namespace sedimi {

namespace {

constexpr int kTN = 64, kTK = 16;

// C[b] = alpha * A[b] * B[b] (row-major, FP64), optional spectral epilogue:
// with a = dtau (lam_m[m] + lam_x[j % nx] + lam_y[j / nx]), C[m][j] is scaled
// by (1 + a)^-ntau (backward Euler) or by the BDF2 factor g_ntau(a) of the
// recurrence g_0 = 1, g_1 = 1 / (1 + a), g_{n+1} = (4 g_n - g_{n-1}) / (3 + 2a).
struct Gemm {
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  int64_t lda, ldb, ldc;
  int64_t sa, sb, sc;  // batch strides (0: shared)
  double alpha;
  const double* lam_m;
  const double* lam_x;
  const double* lam_y;
  int nx;
  int ntau;
  double dtau;
  int bdf2;
};

typedef double v4d __attribute__((ext_vector_type(4)));

// TM rows x kTN columns per block; each of the 4 waves computes a
// (TM / 2) x 32 quarter as MI x 2 MFMA tiles of 16 x 16.
template <bool SPECTRAL, int TM>
__global__ __launch_bounds__(256) void k_gemm64(Gemm g) {
  constexpr int MI = TM / 32;
  __shared__ double As[kTK][TM + 1];
  __shared__ double Bs[kTK][kTN];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // the wave's quarter of the tile
  const int lr = lane & 15, lk = lane >> 4;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * kTN;
  const int64_t b = blockIdx.z;
  const double* A = g.A + b * g.sa;
  const double* B = g.B + b * g.sb;
  double* C = g.C + b * g.sc;
  v4d acc[MI][2];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  // The next K chunk is loaded into registers while the current one, already
  // in LDS, feeds the matrix cores.
  double ra[TM / 16], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int s = 0; s < TM / 16; ++s) {
      // A: TM rows x 16 k, read along k (contiguous)
      const int r = (tid >> 4) + 16 * s, c = tid & 15;
      const int m = m0 + r, k = k0 + c;
      ra[s] = (m < g.M && k < g.K) ? A[(int64_t)m * g.lda + k] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      // B: 16 k x 64 columns, read along the columns (contiguous)
      const int idx = tid + 256 * s;
      const int rr = idx >> 6, cc = idx & 63;
      const int kb = k0 + rr, n = n0 + cc;
      rb[s] = (kb < g.K && n < g.N) ? B[(int64_t)kb * g.ldb + n] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < g.K; k0 += kTK) {
#pragma unroll
    for (int s = 0; s < TM / 16; ++s) As[tid & 15][(tid >> 4) + 16 * s] = ra[s];  // k-major
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int idx = tid + 256 * s;
      Bs[idx >> 6][idx & 63] = rb[s];
    }
    __syncthreads();
    if (k0 + kTK < g.K) fetch(k0 + kTK);
    // MFMA operands: lane (lr, lk) holds A[m = lr][k = lk] and B[k = lk][n = lr]
    // of each 16 x 4 / 4 x 16 fragment
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 4) {
      double a[MI], bb[2];
#pragma unroll
      for (int i = 0; i < MI; ++i) a[i] = As[kk + lk][wm * (TM / 2) + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) bb[j] = Bs[kk + lk][wn * 32 + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // result layout (checked on the device): element r of lane (lr, lk) is row
  // lk + 4 r, column lr of each 16 x 16 tile
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * (TM / 2) + i * 16 + lk + 4 * r;
      const int n = n0 + wn * 32 + j * 16 + lr;
      if (m >= g.M || n >= g.N) continue;
      double v = g.alpha * acc[i][j][r];
      if (SPECTRAL) {
        const double lam = g.lam_m[m] + g.lam_x[n % g.nx] + g.lam_y[n / g.nx];
        const double f = 1.0 / (1.0 + g.dtau * lam);
        double p = 1.0;
        if (g.bdf2) {
          const double r = 1.0 / (3.0 + 2.0 * g.dtau * lam);
          double g0 = 1.0;
          p = f;
          for (int q = 1; q < g.ntau; ++q) {
            const double g2 = (4.0 * p - g0) * r;
            g0 = p;
            p = g2;
          }
        } else {
          for (int q = 0; q < g.ntau; ++q) p *= f;
        }
        v *= p;
      }
      C[(int64_t)m * g.ldc + n] = v;
    }
}

// Row tile: 64 when that already gives the chip thousands of blocks (the
// larger tile reuses its B operand twice as often), 32 on smaller fields,
// where twice the blocks (more waves per SIMD to cover the memory latency)
// win over that reuse.
constexpr int64_t kGemmBlocksFor64 = 1024;
template <int TM>
void gemm_tm(const Gemm& g, int batch, bool spectral, hipStream_t s) {
  dim3 grid((unsigned)((g.N + kTN - 1) / kTN), (unsigned)((g.M + TM - 1) / TM), (unsigned)batch);
  if (spectral)
    hipLaunchKernelGGL((k_gemm64<true, TM>), grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL((k_gemm64<false, TM>), grid, dim3(256), 0, s, g);
}
void gemm(const Gemm& g, int batch, bool spectral, hipStream_t s) {
  const int64_t blocks64 = (int64_t)((g.N + kTN - 1) / kTN) * ((g.M + 63) / 64) * batch;
  if (blocks64 >= kGemmBlocksFor64)
    gemm_tm<64>(g, batch, spectral, s);
  else
    gemm_tm<32>(g, batch, spectral, s);
}

}  // namespace

size_t spectral_table_doubles(const DevParams& P) {
  const size_t nx = P.nx, ny = P.ny, nz = P.nz;
  return nx * nx + ny * ny + 2 * nz * nz + nx + ny + nz;
}

// Eigen-decomposition of a real symmetric tridiagonal matrix (diagonal d,
// off-diagonal e[i] = T[i][i + 1], e[n - 1] unused) by the implicit QL
// iteration with Wilkinson's shift: each sweep chases a bulge up from the
// first negligible off-diagonal element below l with plane rotations, which
// are accumulated into the columns of z (row-major n x n, identity on entry).
// On return d holds the eigenvalues and column j of z the unit eigenvector
// of d[j].  Returns false if an eigenvalue needs more than 64 sweeps.
static bool tridiagonal_eigen(int n, double* d, double* e, double* z) {
  const double eps = 2.220446049250313e-16;
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    for (int sweep = 0;; ++sweep) {
      int m = l;
      while (m < n - 1 && fabs(e[m]) > eps * (fabs(d[m]) + fabs(d[m + 1]))) ++m;
      if (m == l) break;
      if (sweep == 64) return false;
      // shift: the eigenvalue of the leading 2 x 2 block nearer to d[l]
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double sn = 1.0, cs = 1.0, shift = 0.0;
      bool split = false;
      for (int i = m - 1; i >= l; --i) {
        const double f = sn * e[i], b = cs * e[i];
        r = hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {  // the matrix splits here: restart on the smaller block
          d[i + 1] -= shift;
          e[m] = 0.0;
          split = true;
          break;
        }
        sn = f / r;
        cs = g / r;
        g = d[i + 1] - shift;
        r = (d[i] - g) * sn + 2.0 * cs * b;
        shift = sn * r;
        d[i + 1] = g + shift;
        g = cs * r - b;
        for (int k = 0; k < n; ++k) {
          const double a = z[(size_t)k * n + i], c = z[(size_t)k * n + i + 1];
          z[(size_t)k * n + i + 1] = sn * a + cs * c;
          z[(size_t)k * n + i] = cs * a - sn * c;
        }
      }
      if (split) continue;
      d[l] -= shift;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

// The graded z operator: -L_z = H^-1 S with H the cell heights and S
// symmetric tridiagonal (S_kk = u_k + d_k, S_k,k+1 = -u_k in units of the
// coupling times the height of cell k).  B = H^-1/2 S H^-1/2 = Q diag(lam) Q^T
// is symmetric, so -L_z = (H^-1/2 Q) diag(lam) (Q^T H^1/2): the forward
// transform is Q^T H^1/2, the inverse H^-1/2 Q.
int graded_z_transform(int nz, const double* zgeo, double* out) {
  const double* zf = zgeo + zgeo_faces(nz);
  const double* cp = zgeo + zgeo_coupling(nz);
  std::vector<double> h(nz), d(nz), e(nz, 0.0), q((size_t)nz * nz, 0.0);
  for (int k = 0; k < nz; ++k) h[k] = zf[k + 1] - zf[k];
  for (int k = 0; k < nz; ++k) {
    d[k] = cp[2 * k] + cp[2 * k + 1];  // (H^-1 S)_kk = S_kk / h_k
    // S_k,k+1 = -h_k u_k (= -h_{k+1} d_{k+1}); B_k,k+1 = S_k,k+1 / sqrt(h_k h_k+1)
    if (k + 1 < nz) e[k] = -h[k] * cp[2 * k] / sqrt(h[k] * h[k + 1]);
  }
  for (int k = 0; k < nz; ++k) q[(size_t)k * nz + k] = 1.0;
  if (!tridiagonal_eigen(nz, d.data(), e.data(), q.data())) return -1;
  // the columns must be orthonormal to rounding
  double worst = 0.0;
  for (int a = 0; a < nz; ++a)
    for (int b = a; b < nz; ++b) {
      double dot = 0.0;
      for (int k = 0; k < nz; ++k) dot += q[(size_t)k * nz + a] * q[(size_t)k * nz + b];
      worst = std::max(worst, fabs(dot - (a == b ? 1.0 : 0.0)));
    }
  if (!(worst <= 1e-13 * nz)) return -1;
  double* fwd = out;
  double* inv = out + (size_t)nz * nz;
  double* lam = inv + (size_t)nz * nz;
  for (int m = 0; m < nz; ++m) {
    lam[m] = d[m] > 0.0 ? d[m] : 0.0;  // -L_z is positive semi-definite
    for (int k = 0; k < nz; ++k) {
      const double v = q[(size_t)k * nz + m];
      fwd[(size_t)m * nz + k] = v * sqrt(h[k]);
      inv[(size_t)k * nz + m] = v / sqrt(h[k]);
    }
  }
  return 0;
}

// Host tables: H_x, H_y (symmetric, H H = n I), C_z, its inverse, and the
// eigenvalues of -L_h per axis.  Angles are reduced exactly in integers
// before the cosine so that large p q stay accurate.  On a graded mesh the
// z transform, its inverse and eigenvalues are zdiag's.
void spectral_tables(const DevParams& P, const double* zdiag, double* t) {
  const double pi = 3.14159265358979323846;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  double* hx = t;
  double* hy = hx + (size_t)nx * nx;
  double* cz = hy + (size_t)ny * ny;
  double* czi = cz + (size_t)nz * nz;
  double* lx = czi + (size_t)nz * nz;
  double* ly = lx + nx;
  double* lz = ly + ny;
  auto cas_table = [&](double* h, int n) {
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        const double a = 2.0 * pi * (double)(((int64_t)p * q) % n) / n;
        h[(size_t)p * n + q] = cos(a) + sin(a);
      }
  };
  cas_table(hx, nx);
  cas_table(hy, ny);
  for (int m = 0; zdiag == nullptr && m < nz; ++m)
    for (int k = 0; k < nz; ++k) {
      // cos(pi m (2k + 1) / (2 nz)), angle reduced modulo 4 nz
      const int64_t r = ((int64_t)m * (2 * k + 1)) % (4 * (int64_t)nz);
      const double c = cos(pi * (double)r / (2.0 * nz));
      cz[(size_t)m * nz + k] = c;
      czi[(size_t)k * nz + m] = (m == 0 ? 1.0 : 2.0) / nz * c;
    }
  for (int p = 0; p < nx; ++p)
    lx[p] = (2.0 - 2.0 * cos(2.0 * pi * p / nx)) / (P.hx * P.hx);
  for (int p = 0; p < ny; ++p)
    ly[p] = (2.0 - 2.0 * cos(2.0 * pi * p / ny)) / (P.hy * P.hy);
  for (int m = 0; zdiag == nullptr && m < nz; ++m)
    lz[m] = P.kz_diff * (2.0 - 2.0 * cos(pi * m / nz)) / (P.hz * P.hz);  // z diffusivity
  if (zdiag) {
    std::copy(zdiag, zdiag + 2 * (size_t)nz * nz, cz);  // forward, then inverse
    std::copy(zdiag + 2 * (size_t)nz * nz, zdiag + 2 * (size_t)nz * nz + nz, lz);
  }
}

namespace {

// The six axis passes of the direct solve: in -> t -> out -> t -> out -> t ->
// out (t is scratch; in, t and out must not overlap).  tab holds the tables
// in spectral_tables' order.
void spectral_passes(int nx, int ny, int nz, const double* tab, const double* in, double* t,
                     double* out, int nch, int ntau, double tau, bool bdf2, hipStream_t s) {
  const int64_t plane = (int64_t)nx * ny, nc = plane * nz;
  const double* hx = tab;
  const double* hy = hx + (size_t)nx * nx;
  const double* cz = hy + (size_t)ny * ny;
  const double* czi = cz + (size_t)nz * nz;
  const double* lx = czi + (size_t)nz * nz;
  const double* ly = lx + nx;
  const double* lz = ly + ny;
  auto xpass = [&](const double* a, double* c, double alpha) {
    // lines along x: c[l][p] = alpha sum_q a[l][q] H_x[q][p]
    Gemm g{};
    g.A = a, g.B = hx, g.C = c;
    g.M = (int)((int64_t)nch * nz * ny), g.N = nx, g.K = nx;
    g.lda = nx, g.ldb = nx, g.ldc = nx;
    g.alpha = alpha;
    gemm(g, 1, false, s);
  };
  auto ypass = [&](const double* a, double* c, double alpha) {
    Gemm g{};
    g.A = hy, g.B = a, g.C = c;
    g.M = ny, g.N = nx, g.K = ny;
    g.lda = ny, g.ldb = nx, g.ldc = nx;
    g.sa = 0, g.sb = plane, g.sc = plane;
    g.alpha = alpha;
    gemm(g, nch * nz, false, s);
  };
  auto zpass = [&](const double* a, double* c, const double* mat, bool spectral) {
    Gemm g{};
    g.A = mat, g.B = a, g.C = c;
    g.M = nz, g.N = (int)plane, g.K = nz;
    g.lda = nz, g.ldb = plane, g.ldc = plane;
    g.sa = 0, g.sb = nc, g.sc = nc;
    g.alpha = 1.0;
    g.lam_m = lz, g.lam_x = lx, g.lam_y = ly, g.nx = nx;
    g.ntau = ntau, g.dtau = tau / ntau;
    g.bdf2 = bdf2 ? 1 : 0;
    gemm(g, nch, spectral, s);
  };
  xpass(in, t, 1.0);
  ypass(t, out, 1.0);
  zpass(out, t, cz, true);
  zpass(t, out, czi, false);
  ypass(out, t, 1.0 / ny);
  xpass(t, out, 1.0 / nx);
}

// ---- the direct solve without a workspace ----
// Its tables and intermediate field live in this static device array; each
// GPU the library runs on holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in): it uses the device address looked up once per device.
static __device__ __align__(256) unsigned char scratch[SEDIMI_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up at the first
// call on each device, with that device current).
hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// The tables of spectral_tables, computed on the device (the same integer
// angle reduction; cosines and sines from the device's FP64 library).
__global__ void k_spectral_tables(int nx, int ny, int nz, double hx, double hy, double hz,
                                  double kz_diff, double* __restrict__ t) {
  const double pi = 3.14159265358979323846;
  const int64_t sx = (int64_t)nx * nx, sy = (int64_t)ny * ny, sz = (int64_t)nz * nz;
  const int64_t total = sx + sy + 2 * sz + nx + ny + nz;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    double v;
    if (q < sx + sy) {
      const int n = q < sx ? nx : ny;
      const int64_t r = q < sx ? q : q - sx;
      const int64_t p = r / n, k = r % n;
      const double a = 2.0 * pi * (double)((p * k) % n) / n;
      v = cos(a) + sin(a);
    } else if (q < sx + sy + 2 * sz) {
      // C_z[m][k] = cos(pi m (2k + 1) / (2 nz)); C_z^-1[k][m] = (1 or 2)/nz C_z[m][k]
      const int64_t r = q - sx - sy;
      const bool inv = r >= sz;
      const int64_t rr = inv ? r - sz : r;
      const int64_t m = inv ? rr % nz : rr / nz, k = inv ? rr / nz : rr % nz;
      const int64_t ang = (m * (2 * k + 1)) % (4 * (int64_t)nz);
      const double c = cos(pi * (double)ang / (2.0 * nz));
      v = inv ? (m == 0 ? 1.0 : 2.0) / nz * c : c;
    } else {
      const int64_t r = q - sx - sy - 2 * sz;
      if (r < nx) {
        v = (2.0 - 2.0 * cos(2.0 * pi * r / nx)) / (hx * hx);
      } else if (r < nx + ny) {
        v = (2.0 - 2.0 * cos(2.0 * pi * (r - nx) / ny)) / (hy * hy);
      } else {
        v = kz_diff * (2.0 - 2.0 * cos(pi * (r - nx - ny) / nz)) / (hz * hz);
      }
    }
    t[q] = v;
  }
}

__global__ void k_copy_field(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    b[q] = a[q];
}

}  // namespace

// raw (nch channels) -> smooth, through A.sr.
void launch_spectral(const DevParams& P, DevArrays& A, int nch, int ntau, double tau,
                     bool bdf2, hipStream_t s) {
  spectral_passes(P.nx, P.ny, P.nz, A.spec, A.raw, A.sr, A.smooth, nch, ntau, tau, bdf2, s);
}

size_t spectral_static_bytes(int nx, int ny, int nz, int nch) {
  const size_t tab = (size_t)nx * nx + (size_t)ny * ny + 2 * (size_t)nz * nz + nx + ny + nz;
  return ((tab * sizeof(double) + 255) & ~(size_t)255) +
         (size_t)nch * nx * ny * nz * sizeof(double);
}

int spectral_static(int nx, int ny, int nz, double hx, double hy, double hz, double kz_diff,
                    int nch, int ntau, double tau, bool bdf2, const double* raw, double* out,
                    hipStream_t s, std::string* err) {
  const size_t need = spectral_static_bytes(nx, ny, nz, nch);
  if (need > (size_t)SEDIMI_STATIC_SCRATCH_BYTES) {
    *err = "problem needs " + std::to_string(need) + " bytes of static scratch, more than the " +
           std::to_string((size_t)SEDIMI_STATIC_SCRATCH_BYTES) + " available";
    return SEDIMI_ENOMEM;
  }
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) {
    *err = std::string("looking up the static scratch: ") + hipGetErrorString(e);
    return SEDIMI_EDEVICE;
  }
  const int64_t n = (int64_t)nch * nx * ny * nz;
  if (ntau == 0) {  // no pseudo-time step: the field unchanged
    hipLaunchKernelGGL(k_copy_field, dim3(1024), dim3(256), 0, s, n, raw, out);
  } else {
    double* tab = (double*)base;
    const size_t ntab = (size_t)nx * nx + (size_t)ny * ny + 2 * (size_t)nz * nz + nx + ny + nz;
    double* t = (double*)((char*)base + ((ntab * sizeof(double) + 255) & ~(size_t)255));
    hipLaunchKernelGGL(k_spectral_tables, dim3(1024), dim3(256), 0, s, nx, ny, nz, hx, hy, hz,
                       kz_diff, tab);
    spectral_passes(nx, ny, nz, tab, raw, t, out, nch, ntau, tau, bdf2, s);
  }
  e = hipGetLastError();
  if (e != hipSuccess) {
    *err = std::string("launching the direct solve: ") + hipGetErrorString(e);
    return SEDIMI_EDEVICE;
  }
  return SEDIMI_OK;
}

}  // namespace sedimi

// k_spectral.hip -- direct solve of the implicit diffusion averaging on the
// uniform mesh.
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
// The GEMM runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64): a block
// computes a 64 x 64 tile of C with four waves of 32 x 32 (2 x 2 MFMA tiles);
// K is staged through LDS 16 at a time.  Per MFMA a lane reads one double of
// A and one of B, against eight LDS reads per 16 FMAs for a 4 x 4 outer
// product on the vector units.
#include "k_common.h"

namespace sedimi {

namespace {

constexpr int kTM = 64, kTN = 64, kTK = 16;

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

template <bool SPECTRAL>
__global__ __launch_bounds__(256) void k_gemm64(Gemm g) {
  __shared__ double As[kTK][kTM + 1];
  __shared__ double Bs[kTK][kTN];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // the wave's 32 x 32 quarter of the tile
  const int lr = lane & 15, lk = lane >> 4;
  const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
  const int64_t b = blockIdx.z;
  const double* A = g.A + b * g.sa;
  const double* B = g.B + b * g.sb;
  double* C = g.C + b * g.sc;
  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  // The next K chunk is loaded into registers while the current one, already
  // in LDS, feeds the matrix cores.
  double ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      // A: 64 rows x 16 k, read along k (contiguous)
      const int r = (tid >> 4) + 16 * s, c = tid & 15;
      const int m = m0 + r, k = k0 + c;
      ra[s] = (m < g.M && k < g.K) ? A[(int64_t)m * g.lda + k] : 0.0;
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
    for (int s = 0; s < 4; ++s) {
      As[tid & 15][(tid >> 4) + 16 * s] = ra[s];  // stored k-major
      const int idx = tid + 256 * s;
      Bs[idx >> 6][idx & 63] = rb[s];
    }
    __syncthreads();
    if (k0 + kTK < g.K) fetch(k0 + kTK);
    // MFMA operands: lane (lr, lk) holds A[m = lr][k = lk] and B[k = lk][n = lr]
    // of each 16 x 4 / 4 x 16 fragment
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 4) {
      double a[2], bb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + lk][wm * 32 + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) bb[j] = Bs[kk + lk][wn * 32 + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // result layout (checked on the device): element r of lane (lr, lk) is row
  // lk + 4 r, column lr of each 16 x 16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * 32 + i * 16 + lk + 4 * r;
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

void gemm(const Gemm& g, int batch, bool spectral, hipStream_t s) {
  dim3 grid((unsigned)((g.N + kTN - 1) / kTN), (unsigned)((g.M + kTM - 1) / kTM),
            (unsigned)batch);
  if (spectral)
    hipLaunchKernelGGL(k_gemm64<true>, grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(k_gemm64<false>, grid, dim3(256), 0, s, g);
}

}  // namespace

size_t spectral_table_doubles(const DevParams& P) {
  const size_t nx = P.nx, ny = P.ny, nz = P.nz;
  return nx * nx + ny * ny + 2 * nz * nz + nx + ny + nz;
}

// Host tables: H_x, H_y (symmetric, H H = n I), C_z, its inverse, and the
// eigenvalues of -L_h per axis.  Angles are reduced exactly in integers
// before the cosine so that large p q stay accurate.
void spectral_tables(const DevParams& P, double* t) {
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
  for (int m = 0; m < nz; ++m)
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
  for (int m = 0; m < nz; ++m)
    lz[m] = P.kz_diff * (2.0 - 2.0 * cos(pi * m / nz)) / (P.hz * P.hz);  // z diffusivity
}

// raw (nch channels) -> smooth, through A.sr / A.stmp.
void launch_spectral(const DevParams& P, DevArrays& A, int nch, int ntau, double tau,
                     bool bdf2, hipStream_t s) {
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int64_t nc = P.ncell, plane = (int64_t)nx * ny;
  const double* hx = A.spec;
  const double* hy = hx + (size_t)nx * nx;
  const double* cz = hy + (size_t)ny * ny;
  const double* czi = cz + (size_t)nz * nz;
  const double* lx = czi + (size_t)nz * nz;
  const double* ly = lx + nx;
  const double* lz = ly + ny;
  double* t0 = A.sr;
  double* t1 = A.stmp;
  auto xpass = [&](const double* in, double* out, double alpha) {
    // lines along x: out[l][p] = alpha sum_q in[l][q] H_x[q][p]
    Gemm g{};
    g.A = in, g.B = hx, g.C = out;
    g.M = (int)((int64_t)nch * nz * ny), g.N = nx, g.K = nx;
    g.lda = nx, g.ldb = nx, g.ldc = nx;
    g.alpha = alpha;
    gemm(g, 1, false, s);
  };
  auto ypass = [&](const double* in, double* out, double alpha) {
    Gemm g{};
    g.A = hy, g.B = in, g.C = out;
    g.M = ny, g.N = nx, g.K = ny;
    g.lda = ny, g.ldb = nx, g.ldc = nx;
    g.sa = 0, g.sb = plane, g.sc = plane;
    g.alpha = alpha;
    gemm(g, nch * nz, false, s);
  };
  auto zpass = [&](const double* in, double* out, const double* mat, bool spectral) {
    Gemm g{};
    g.A = mat, g.B = in, g.C = out;
    g.M = nz, g.N = (int)plane, g.K = nz;
    g.lda = nz, g.ldb = plane, g.ldc = plane;
    g.sa = 0, g.sb = nc, g.sc = nc;
    g.alpha = 1.0;
    g.lam_m = lz, g.lam_x = lx, g.lam_y = ly, g.nx = nx;
    g.ntau = ntau, g.dtau = tau / ntau;
    g.bdf2 = bdf2 ? 1 : 0;
    gemm(g, nch, spectral, s);
  };
  xpass(A.raw, t0, 1.0);
  ypass(t0, t1, 1.0);
  zpass(t1, t0, cz, true);
  zpass(t0, t1, czi, false);
  ypass(t1, t0, 1.0 / ny);
  xpass(t0, A.smooth, 1.0 / nx);
}

}  // namespace sedimi

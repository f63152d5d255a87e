// sedimi_api.cpp -- the C ABI of libsedimi (declared in include/sedimi.h):
// parameter checks, workspace layout, host<->device transfers, and the
// enqueueing of the kernel chains for one step and one averaging.
#include <hip/hip_runtime.h>
#include <math.h>

#include <cmath>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "k_nn.h"
#include "sedimi_internal.h"

using namespace sedimi;

namespace {
constexpr int kNNC = 32;                       // network width
constexpr int kNNDil[6] = {1, 2, 4, 4, 2, 1};  // z dilation per layer
constexpr int kDwBlocks = 512;                 // weight-gradient partial blocks

struct NNBufs {
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // parameters, moments, grads
  __bf16* fwd[6] = {};
  __bf16* adj[6] = {};
  float *xf = nullptr, *y = nullptr;
  __bf16 *xb = nullptr, *dy6 = nullptr;
  __bf16* z[5] = {};
  __bf16* h[5] = {};
  __bf16* dh[5] = {};  // gradient of the loss at h_l, z_l of layers 1..5 (kept for reading)
  __bf16* dz[5] = {};
  float *part = nullptr, *part_b = nullptr;
  // the check: Green's function window of the plain solve, sampled columns,
  // per-column partials
  double* gtab = nullptr;
  int* cols = nullptr;
  double* gpart = nullptr;
  // the skip S (the diffusion split by axis): S x and scratch, FP32 [ncell][4];
  // taps in x and y and the z-line table, FP64
  float *xs = nullptr, *xt = nullptr;
  double* stab = nullptr;
};

constexpr int kSplitMaxTaps = 129;  // circulant taps per periodic axis
constexpr int kSplitMaxNz = 150;    // z-column held in LDS by the split's z solve

// Window of the check's Green's function (host side).
struct GreenWindow {
  int rx = 0, ry = 0, rz = 0;
  double trunc = 1.0;  // mass of the Green's function outside the window
  std::vector<double> tab;  // [2ry+1][2rx+1][2rz+1]
};
constexpr int kGreenRxy = 4, kGreenRz = 32;
int nn_check_columns(const sedimi_params& p) {
  const int64_t ncol = (int64_t)p.nx * p.ny;
  const int64_t m = (int64_t)ceil(p.nn_sample * (double)ncol);
  return (int)std::max<int64_t>(1, std::min<int64_t>(ncol, m));
}

int nn_cin(int l) { return l == 0 ? 4 : kNNC; }
int nn_cout(int l) { return l == 5 ? 4 : kNNC; }
int64_t nn_woff(int l) {
  int64_t o = 0;
  for (int q = 0; q < l; ++q) o += 27LL * nn_cin(q) * nn_cout(q) + nn_cout(q);
  return o;
}
int64_t nn_count() { return nn_woff(6); }
}  // namespace

struct sedimi_ctx {
  sedimi_params prm;
  int avg_mode = SEDIMI_AVG_PLAIN;
  NNBufs nn;
  NNNorm norm{{0, 0, 0, 0}, {1, 1, 1, 1}, {1, 1, 1, 1}};
  int64_t adam_t = 0;
  int nn_groups = 1;  // 4: one channel group per field, cross-group weights held at zero
  int64_t nn_calls = 0, nn_fallbacks = 0;
  double nn_last_check = 0.0;
  int64_t cap = 0;
  int64_t n = 0;
  int64_t step = 0;
  size_t ws_bytes = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  DevParams P{};
  DevArrays A{};
  bool mixed = false;
  bool have_particles = false;
  int64_t last_iters = 0;
  double last_residual = 0.0;
  std::vector<double> zgeo;  // z geometry (zgeo_* layout), uploaded at bind
  std::vector<double> zdiag; // graded direct solve: z transform, inverse, eigenvalues
  bool direct = false;       // the implicit steps are solved by diagonalisation
  bool last_direct = false;  // the last plain solve was the direct one
  int check_blocks = 0;      // residual partials of the last direct solve
  GreenWindow green;         // the network check's Green's function window
  SplitTabs split{};         // the network's skip S (device tables)
  int green_cols = 0;        // sampled columns of the network check
  std::string err;
  // phase timing
  bool prof = false;
  struct Mark {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  double prof_ms[SEDIMI_NPHASES] = {0};
  int64_t prof_count[SEDIMI_NPHASES] = {0};
  // Replayed steps: sedimi_step's kernel sequence captured once into a HIP
  // graph and launched as one (about 1.6 us per kernel instead of 2.7 us).
  // An entry is keyed on everything the captured launches baked in.
  bool graphs_on = true;
  int64_t graph_steps = 0;           // calls run from a graph
  hipStream_t cap_stream = nullptr;  // capture needs a stream of its own
  struct StepGraph {
    std::vector<unsigned char> key;
    hipGraphExec_t exec = nullptr;
    DevArrays after{};  // the device-array pointers after the steps
    bool averaged = false, last_direct = false;
    int64_t last_iters = 0;
    int check_blocks = 0;
    uint64_t used = 0;
  };
  std::vector<StepGraph> graphs;
  uint64_t graph_clock = 0;
  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  ~sedimi_ctx() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& m : marks) pool.push_back(m.a), pool.push_back(m.b);
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

namespace {

constexpr double kPi = 3.14159265358979323846;

// splitmix64 (Steele, Lea & Flood): seeded weights and check samples
uint64_t mix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// last failure of a context-free call, per thread
thread_local std::string g_noctx_err = "null context";

int fail(sedimi_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, SEDIMI_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Largest axis of the direct diffusion solve (its transform tables grow as
// n^2 and its work per cell as n).
constexpr int kDirectMaxAxis = 2048;
// On a graded mesh the z transform comes from an eigen-decomposition on the
// host at context creation (cubic in nz): larger graded meshes are solved by
// the iterative solver.
constexpr int kGradedDirectMaxNz = 512;

bool graded_mesh(const sedimi_params& p) {
  return p.nz > 1 && p.z_grading > 0.0 && p.z_grading != 1.0;
}

// Faces, centres, cell volumes and z coupling of the diffusion operator in
// the zgeo_* layout.  Section 4's channel mesh is refined towards the bottom
// wall; the grading is read as cell heights growing geometrically, h_k =
// h_0 q^k with q^(nz - 1) = z_grading (the top cell's height over the bottom
// cell's), summed from the bottom in order and scaled to Lz.  The coupling
// of plane k to a neighbour is the flux through the shared face over the
// centre distance, per unit height of cell k: kz / (h_k dc).
std::vector<double> z_geometry(const sedimi_params& p, const DevParams& P) {
  const int nz = P.nz;
  std::vector<double> g(zgeo_doubles(nz), 0.0);
  double* zf = g.data() + zgeo_faces(nz);
  double* zc = g.data() + zgeo_centres(nz);
  double* vol = g.data() + zgeo_volumes(nz);
  double* cp = g.data() + zgeo_coupling(nz);
  zf[0] = 0.0;
  if (P.graded) {
    double sum = 0.0;
    for (int k = 0; k < nz; ++k) sum += pow(p.z_grading, (double)k / (nz - 1));
    const double scale = p.Lz / sum;
    for (int k = 1; k <= nz; ++k)
      zf[k] = zf[k - 1] + pow(p.z_grading, (double)(k - 1) / (nz - 1)) * scale;
    zf[nz] = p.Lz;
  } else {
    for (int k = 1; k <= nz; ++k) zf[k] = p.Lz * k / nz;
  }
  for (int k = 0; k < nz; ++k) {
    zc[k] = 0.5 * (zf[k] + zf[k + 1]);
    vol[k] = P.hx * P.hy * (zf[k + 1] - zf[k]);
  }
  for (int k = 0; k < nz; ++k) {
    const double h = zf[k + 1] - zf[k];
    cp[2 * k] = k + 1 < nz ? P.kz_diff / (h * (zc[k + 1] - zc[k])) : 0.0;
    cp[2 * k + 1] = k > 0 ? P.kz_diff / (h * (zc[k] - zc[k - 1])) : 0.0;
  }
  return g;
}

// Workspace carving: the same walk computes the size (base == nullptr) and
// assigns the pointers.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = align256(off);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (count > 0 ? count : 1);
    return p;
  }
};

size_t layout(const sedimi_ctx* c, char* base, DevArrays* A) {
  Carver w{base};
  const size_t N = (size_t)(c->cap > 0 ? c->cap : 1);
  const size_t maxn = (size_t)c->P.maxn;
  const size_t nb = (size_t)c->P.nbins + 1;
  const size_t nc = (size_t)c->P.ncell;
  DevArrays a{};
  a.pos = w.take<double4>(N);
  a.vel = w.take<double4>(N);
  a.omg = w.take<double4>(N);
  a.acc = w.take<double4>(N);
  a.alp = w.take<double4>(N);
  a.fdr = w.take<double4>(N);
  a.xb = w.take<double4>(N);
  a.wxi = w.take<double4>(2 * N);
  a.pos_t = w.take<double4>(N);
  a.vel_t = w.take<double4>(N);
  a.omg_t = w.take<double4>(N);
  a.acc_t = w.take<double4>(N);
  a.alp_t = w.take<double4>(N);
  a.fdr_t = w.take<double4>(N);
  a.wxi_t = w.take<double4>(2 * N);
  a.id = w.take<int>(N);
  a.id_t = w.take<int>(N);
  a.nbr = w.take<int>(maxn * N);
  a.ncnt = w.take<int>(N);
  a.hmask = w.take<unsigned>(N);
  a.hxi = w.take<double>(3 * maxn * N);
  a.cid = w.take<int>((size_t)kMaxContacts * N);
  a.cxi = w.take<double>(3 * (size_t)kMaxContacts * N);
  a.ccnt = w.take<int>(N);
  a.comp = w.take<double4>(8 * N);
  a.key = w.take<int>(N);
  a.rank = w.take<int>(N);
  a.perm = w.take<int>(N);
  a.cperm = w.take<unsigned long long>(N);
  a.bin_count = w.take<int>(nb);
  a.bin_start = w.take<int>(nb);
  size_t tiles = (std::max(nb, nc + 1) + 1023) / 1024 + 2;
  a.scan_tmp = w.take<int>(tiles);
  a.U = w.take<double4>(nc);
  a.gp = w.take<double4>(nc);
  a.du = w.take<double4>(nc);
  a.G = w.take<double4>(nc);
  a.W = w.take<double4>(c->prm.c_lift > 0 ? nc : 0);
  const size_t nch = c->prm.avg_solid_velocity ? 7 : 4;
  a.raw = w.take<double>(nch * nc);
  a.smooth = w.take<double>(nch * nc);
  a.sx = w.take<double>(nch * nc);
  a.sr = w.take<double>(nch * nc);
  a.sd0 = w.take<double>(nch * nc);
  a.sd1 = w.take<double>(nch * nc);
  a.sxf = w.take<double>(nch * nc);
  a.stmp = w.take<double>(nch * nc);
  a.us = w.take<double>(nch == 7 ? 3 * nc : 0);
  a.ztab = w.take<double>(4 * (size_t)c->P.nz);
  a.zgeo = w.take<double>(zgeo_doubles(c->P.nz));
  a.sprev = w.take<double>(c->prm.avg_scheme == SEDIMI_SCHEME_BDF2 && !c->direct ? nch * nc : 0);
  a.spec = w.take<double>(c->direct ? spectral_table_doubles(c->P) : 0);
  a.cell_count = w.take<int>(nc + 1);
  a.cell_start = w.take<int>(nc + 1);
  a.red = w.take<double>(smooth_red_doubles((int)nc, (int)nch, std::max(1, c->prm.avg_ntau)));
  // kept across sedimi_set_particles (which clears everything before U)
  a.bin_rank = w.take<int>(nb);
  a.ctl = w.take<Ctl>(1);
  a.rb = a.ctl ? &a.ctl->rebuild : nullptr;
  a.rb_next = a.ctl ? &a.ctl->rebuild_alt : nullptr;
  if (A) *A = a;
  if (c->prm.nn_enable) {
    NNBufs b;
    const size_t P = (size_t)nn_count();
    b.w = w.take<float>(P);
    b.m = w.take<float>(P);
    b.v = w.take<float>(P);
    b.g = w.take<float>(P);
    for (int l = 0; l < 6; ++l) {
      b.fwd[l] = w.take<__bf16>(nn_packed_elems(nn_cin(l), nn_cout(l)));
      if (l > 0) b.adj[l] = w.take<__bf16>(nn_packed_elems(nn_cout(l), nn_cin(l)));
    }
    b.xf = w.take<float>(4 * nc);
    b.y = w.take<float>(4 * nc);
    b.xb = w.take<__bf16>(4 * nc);
    b.dy6 = w.take<__bf16>(4 * nc);
    for (int l = 0; l < 5; ++l) b.z[l] = w.take<__bf16>(kNNC * nc);
    for (int l = 0; l < 5; ++l) b.h[l] = w.take<__bf16>(kNNC * nc);
    for (int l = 0; l < 5; ++l) b.dh[l] = w.take<__bf16>(kNNC * nc);
    for (int l = 0; l < 5; ++l) b.dz[l] = w.take<__bf16>(kNNC * nc);
    b.part = w.take<float>((size_t)kDwBlocks * 27 * kNNC * kNNC);
    b.part_b = w.take<float>((size_t)kDwBlocks * kNNC);
    b.xs = w.take<float>(4 * nc);
    b.xt = w.take<float>(4 * nc);
    b.stab = w.take<double>(2 * kSplitMaxTaps + 2 * (size_t)c->P.nz);
    b.gtab = w.take<double>((size_t)(2 * kGreenRxy + 1) * (2 * kGreenRxy + 1) * (2 * kGreenRz + 1));
    b.cols = w.take<int>((size_t)nn_check_columns(c->prm));
    b.gpart = w.take<double>(8 * (size_t)nn_check_columns(c->prm));
    if (base) const_cast<sedimi_ctx*>(c)->nn = b;
  }
  return align256(w.off);
}

// Green's function of all N_tau backward-Euler steps, (I - dtau L)^-N_tau
// delta, on the unbounded mesh with this mesh's spacings: the inverse cosine
// transform of (1 + sum_a c_a (2 - 2 cos k_a))^-N_tau (c_a = dtau D_a / h_a^2)
// over a periodic grid of 64 x 64 x 256 cells, far wider than the function
// (it decays exponentially), evaluated one axis at a time on the offsets
// |dx|, |dy| <= 4, |dz| <= 32.  The window is the smallest box whose mass
// (the function sums to 1) is within 1e-4 of 1, else the largest; the mass
// outside bounds the estimate's error by that share of the field's largest
// value.
GreenWindow green_window(const DevParams& P, int ntau, double tau) {
  constexpr int Mx = 64, My = 64, Mz = 256;
  constexpr int R = kGreenRz, Q = kGreenRxy;
  GreenWindow gw;
  const int N = ntau > 0 ? ntau : 1;
  const double dtau = tau / N;
  const double cx = dtau / (P.hx * P.hx), cy = dtau / (P.hy * P.hy);
  const double cz = dtau * P.kz_diff / (P.hz * P.hz);
  std::vector<double> ex(Mx), ey(My), ez(Mz), cosx(Mx * (Q + 1)), cosy(My * (Q + 1)),
      cosz(Mz * (R + 1));
  for (int k = 0; k < Mx; ++k) {
    ex[k] = cx * (2.0 - 2.0 * cos(2.0 * kPi * k / Mx));
    for (int d = 0; d <= Q; ++d) cosx[k * (Q + 1) + d] = cos(2.0 * kPi * (double)((k * d) % Mx) / Mx);
  }
  for (int k = 0; k < My; ++k) {
    ey[k] = cy * (2.0 - 2.0 * cos(2.0 * kPi * k / My));
    for (int d = 0; d <= Q; ++d) cosy[k * (Q + 1) + d] = cos(2.0 * kPi * (double)((k * d) % My) / My);
  }
  for (int k = 0; k < Mz; ++k) {
    ez[k] = cz * (2.0 - 2.0 * cos(2.0 * kPi * k / Mz));
    for (int d = 0; d <= R; ++d) cosz[k * (R + 1) + d] = cos(2.0 * kPi * (double)((k * d) % Mz) / Mz);
  }
  // T[kx][ky][dz] = sum_kz S cos(kz dz); U[kx][dy][dz] = sum_ky T cos(ky dy)
  std::vector<double> U((size_t)Mx * (Q + 1) * (R + 1), 0.0), T(R + 1);
  for (int kx = 0; kx < Mx; ++kx)
    for (int ky = 0; ky < My; ++ky) {
      std::fill(T.begin(), T.end(), 0.0);
      for (int kz = 0; kz < Mz; ++kz) {
        const double S = pow(1.0 + ex[kx] + ey[ky] + ez[kz], -(double)N);
        const double* cz_ = &cosz[kz * (R + 1)];
        for (int d = 0; d <= R; ++d) T[d] += S * cz_[d];
      }
      for (int dy = 0; dy <= Q; ++dy) {
        const double c = cosy[ky * (Q + 1) + dy];
        double* u = &U[((size_t)kx * (Q + 1) + dy) * (R + 1)];
        for (int d = 0; d <= R; ++d) u[d] += c * T[d];
      }
    }
  // G[|dx|][|dy|][|dz|]
  std::vector<double> G((size_t)(Q + 1) * (Q + 1) * (R + 1), 0.0);
  const double norm = 1.0 / ((double)Mx * My * Mz);
  for (int dx = 0; dx <= Q; ++dx)
    for (int kx = 0; kx < Mx; ++kx) {
      const double c = cosx[kx * (Q + 1) + dx] * norm;
      for (int dy = 0; dy <= Q; ++dy)
        for (int d = 0; d <= R; ++d)
          G[((size_t)dx * (Q + 1) + dy) * (R + 1) + d] += c * U[((size_t)kx * (Q + 1) + dy) * (R + 1) + d];
    }
  auto g = [&](int dx, int dy, int dz) {
    return G[((size_t)std::abs(dx) * (Q + 1) + std::abs(dy)) * (R + 1) + std::abs(dz)];
  };
  auto mass = [&](int rx, int ry, int rz) {
    double m = 0.0;
    for (int dz = -rz; dz <= rz; ++dz)
      for (int dy = -ry; dy <= ry; ++dy)
        for (int dx = -rx; dx <= rx; ++dx) m += g(dx, dy, dz);
    return m;
  };
  int best = -1;
  for (int rx = 0; rx <= Q; ++rx)
    for (int ry = 0; ry <= Q; ++ry)
      for (int rz = 0; rz <= R; ++rz) {
        const int vol = (2 * rx + 1) * (2 * ry + 1) * (2 * rz + 1);
        if (best >= 0 && vol >= best) continue;
        if (1.0 - mass(rx, ry, rz) <= 1e-4) {
          best = vol;
          gw.rx = rx, gw.ry = ry, gw.rz = rz;
        }
      }
  if (best < 0) gw.rx = Q, gw.ry = Q, gw.rz = R;
  gw.trunc = 1.0 - mass(gw.rx, gw.ry, gw.rz);
  gw.tab.clear();  // [dy][dx][dz]: one z-run per window column
  for (int dy = -gw.ry; dy <= gw.ry; ++dy)
    for (int dx = -gw.rx; dx <= gw.rx; ++dx)
      for (int dz = -gw.rz; dz <= gw.rz; ++dz) gw.tab.push_back(g(dx, dy, dz));
  return gw;
}

// Circulant taps of N periodic one-dimensional implicit steps
// (1 - c D)^-N on n cells: g[m] = (1/n) sum_k cos(2 pi k m / n)
// (1 + c (2 - 2 cos(2 pi k / n)))^-N.  The offsets |m| <= R for the smallest
// R <= 64 whose tail sums below 1e-13, or all n offsets when those do not
// leave out any (2R + 1 >= n, n <= 129).
void split_taps(int n, double c, int N, std::vector<double>* taps, int* off0) {
  std::vector<double> g((size_t)n, 0.0);
  for (int m = 0; m < n; ++m) {
    double acc = 0.0;
    for (int k = 0; k < n; ++k) {
      const double lam = c * (2.0 - 2.0 * cos(2.0 * kPi * k / n));
      acc += cos(2.0 * kPi * (double)(((int64_t)k * m) % n) / n) * pow(1.0 + lam, -(double)N);
    }
    g[m] = acc / n;
  }
  taps->clear();
  int R = 64;
  for (int r = 0; r < 64 && 2 * r + 1 < n; ++r) {
    double tail = 0.0;
    for (int m = r + 1; m <= n - 1 - r; ++m) tail += fabs(g[m]);
    if (tail <= 1e-13) {
      R = r;
      break;
    }
  }
  if (2 * R + 1 >= n && n <= kSplitMaxTaps) {
    *taps = g;
    *off0 = 0;
    return;
  }
  for (int t = -R; t <= R; ++t) taps->push_back(g[(size_t)((t + n) % n)]);
  *off0 = -R;
}

int check_params(sedimi_ctx* c, const sedimi_params& p, int64_t cap) {
  if (cap < 0 || cap > (int64_t)INT32_MAX / 32)
    return fail(c, SEDIMI_EINVAL, "max_particles out of range");
  if (!(p.Lx > 0 && p.Ly > 0 && p.Lz > 0)) return fail(c, SEDIMI_EINVAL, "domain must be positive");
  if (p.nx < 1 || p.ny < 1 || p.nz < 1) return fail(c, SEDIMI_EINVAL, "mesh needs >= 1 cell per axis");
  if ((int64_t)p.nx * p.ny * p.nz > (int64_t)INT32_MAX / 8)
    return fail(c, SEDIMI_EINVAL, "mesh too large");
  if (!(p.kn > 0)) return fail(c, SEDIMI_EINVAL, "kn must be positive");
  if (!(p.restitution > 0 && p.restitution <= 1))
    return fail(c, SEDIMI_EINVAL, "restitution must be in (0, 1]");
  if (!(p.friction >= 0 && p.kt_over_kn >= 0 && p.gammat_over_gamman >= 0))
    return fail(c, SEDIMI_EINVAL, "friction / tangential ratios must be >= 0");
  if (!(p.lub_out_frac >= 0 && p.lub_in_frac > 0))
    return fail(c, SEDIMI_EINVAL, "lubrication gaps must be >= 0 (inner > 0)");
  if (!(p.rho_f >= 0 && p.mu_f > 0 && p.c_add >= 0))
    return fail(c, SEDIMI_EINVAL, "fluid properties out of range");
  if (!(p.dt > 0)) return fail(c, SEDIMI_EINVAL, "dt must be positive");
  if (p.drag_law < SEDIMI_DRAG_NONE || p.drag_law > SEDIMI_DRAG_SYAMLAL)
    return fail(c, SEDIMI_EINVAL, "unknown drag law");
  if (!(p.eps_s_max >= 0 && p.eps_s_max < 1)) return fail(c, SEDIMI_EINVAL, "eps_s_max in [0,1)");
  if (!(p.avg_bandwidth >= 0) || p.avg_ntau < 0 || !(p.avg_rtol > 0))
    return fail(c, SEDIMI_EINVAL, "averaging parameters out of range");
  if (p.precision != SEDIMI_FP64 && p.precision != SEDIMI_MIXED)
    return fail(c, SEDIMI_EINVAL, "precision must be SEDIMI_FP64 or SEDIMI_MIXED");
  if (!(p.d_max > 0)) return fail(c, SEDIMI_EINVAL, "d_max must be positive");
  if (!(p.skin >= 0)) return fail(c, SEDIMI_EINVAL, "skin must be >= 0");
  if (p.max_neighbors < 1 || p.max_neighbors > 30)
    return fail(c, SEDIMI_EINVAL, "max_neighbors must be in 1..30");
  if (p.nn_enable && !(p.nn_alpha >= 0 && p.nn_bound > 0 && p.nn_sample > 0 && p.nn_sample <= 1))
    return fail(c, SEDIMI_EINVAL, "surrogate parameters out of range");
  if (p.nn_enable && p.nz > kSplitMaxNz)
    return fail(c, SEDIMI_EINVAL, "the network needs nz <= 150 (its skip holds a z-column in LDS)");
  if (!(p.z_grading >= 0.0 && std::isfinite(p.z_grading)))
    return fail(c, SEDIMI_EINVAL, "z_grading must be finite and >= 0 (0 or 1: uniform)");
  if (graded_mesh(p) && p.nn_enable)
    return fail(c, SEDIMI_EINVAL, "the network needs a uniform z mesh (z_grading 0 or 1)");
  if (graded_mesh(p) && p.avg_solver == SEDIMI_SOLVE_DIRECT && p.nz > kGradedDirectMaxNz)
    return fail(c, SEDIMI_EINVAL, "direct averaging solve on a graded mesh needs nz <= 512");
  if (p.avg_scheme != SEDIMI_SCHEME_EULER && p.avg_scheme != SEDIMI_SCHEME_BDF2)
    return fail(c, SEDIMI_EINVAL, "unknown averaging scheme");
  if (p.avg_scheme == SEDIMI_SCHEME_BDF2 && p.nn_enable)
    return fail(c, SEDIMI_EINVAL, "BDF2 averaging needs the plain solve (nn_enable off)");
  if (p.avg_solid_velocity && p.nn_enable)
    return fail(c, SEDIMI_EINVAL, "avg_solid_velocity needs the plain solve (nn_enable off)");
  if (!(p.c_lift >= 0 && std::isfinite(p.c_lift)))
    return fail(c, SEDIMI_EINVAL, "c_lift must be finite and >= 0");
  if (!(p.avg_bandwidth_z >= 0 && std::isfinite(p.avg_bandwidth_z)))
    return fail(c, SEDIMI_EINVAL, "avg_bandwidth_z must be finite and >= 0");
  if (p.avg_solver < SEDIMI_SOLVE_AUTO || p.avg_solver > SEDIMI_SOLVE_ITERATIVE)
    return fail(c, SEDIMI_EINVAL, "unknown averaging solver");
  if (p.avg_solver == SEDIMI_SOLVE_DIRECT && std::max(p.nx, std::max(p.ny, p.nz)) > kDirectMaxAxis)
    return fail(c, SEDIMI_EINVAL, "direct averaging solve needs <= 2048 cells per axis");
  return SEDIMI_OK;
}

void fill_dev_params(sedimi_ctx* c) {
  const sedimi_params& p = c->prm;
  DevParams& P = c->P;
  P.Lx = p.Lx, P.Ly = p.Ly, P.Lz = p.Lz;
  P.hLx = 0.5 * p.Lx, P.hLy = 0.5 * p.Ly;
  P.nx = p.nx, P.ny = p.ny, P.nz = p.nz;
  P.ncell = p.nx * p.ny * p.nz;
  P.hx = p.Lx / p.nx, P.hy = p.Ly / p.ny, P.hz = p.Lz / p.nz;
  P.Vc = P.hx * P.hy * P.hz;
  P.kn = p.kn;
  if (p.restitution >= 1.0) {
    P.zeta = 0.0;
  } else {
    double le = log(p.restitution);
    P.zeta = -le / sqrt(kPi * kPi + le * le);
  }
  P.kt = p.kt_over_kn * p.kn;
  P.gt_over_gn = p.gammat_over_gamman;
  P.mu = p.friction;
  P.lub_out = p.lub_out_frac, P.lub_in = p.lub_in_frac;
  P.rho_f = p.rho_f, P.mu_f = p.mu_f, P.c_add = p.c_add;
  P.gx = p.gx, P.gy = p.gy, P.gz = p.gz, P.dt = p.dt;
  P.drag_law = p.drag_law, P.lubrication = p.lubrication ? 1 : 0;
  P.fluid_forces = p.fluid_forces ? 1 : 0;
  P.bottom_wall = p.bottom_wall ? 1 : 0, P.top_wall = p.top_wall ? 1 : 0;
  P.eps_s_max = p.eps_s_max;
  P.lift_c = p.c_lift > 0 ? p.c_lift * p.rho_f * sqrt(p.mu_f / p.rho_f) : 0.0;
  P.nch_avg = p.avg_solid_velocity ? 7 : 4;
  P.kz_diff = 1.0;
  if (p.avg_bandwidth_z > 0 && p.avg_bandwidth > 0) {
    const double r = p.avg_bandwidth_z / p.avg_bandwidth;
    P.kz_diff = r * r;
  }
  P.graded = graded_mesh(p) ? 1 : 0;
  P.zlam = p.nz > 1 ? 4.0 * P.kz_diff / (P.hz * P.hz) : 0.0;
  P.zskew = 1.0;
  c->zgeo = z_geometry(p, P);
  if (P.graded) {
    // Gershgorin bound of -L_z, and the cell heights' spread
    const double* zf = c->zgeo.data() + zgeo_faces(p.nz);
    const double* cp = c->zgeo.data() + zgeo_coupling(p.nz);
    double lam = 0.0, hmin = INFINITY, hmax = 0.0;
    for (int k = 0; k < p.nz; ++k) {
      lam = std::max(lam, 2.0 * (cp[2 * k] + cp[2 * k + 1]));
      hmin = std::min(hmin, zf[k + 1] - zf[k]);
      hmax = std::max(hmax, zf[k + 1] - zf[k]);
    }
    P.zlam = lam;
    P.zskew = sqrt(hmax / hmin);
  }
  // neighbour bins: no smaller than the largest pair range plus the skin
  double hb = p.d_max * (1.0 + p.lub_out_frac) + p.skin;
  P.nbx = std::max(1, (int)floor(p.Lx / hb));
  P.nby = std::max(1, (int)floor(p.Ly / hb));
  P.nbz = std::max(1, (int)floor(p.Lz / hb));
  P.nbins = P.nbx * P.nby * P.nbz;
  P.hbx = p.Lx / P.nbx, P.hby = p.Ly / P.nby, P.hbz = p.Lz / P.nbz;
  P.skin = p.skin;
  P.half_skin2 = 0.25 * p.skin * p.skin;
  P.maxn = p.max_neighbors;
  P.n = 0;
}

int need_ws(sedimi_ctx* c) {
  if (!c) return SEDIMI_EINVAL;
  if (!c->ws) return fail(c, SEDIMI_ENOMEM, "no workspace bound");
  return SEDIMI_OK;
}
int need_particles(sedimi_ctx* c) {
  int rc = need_ws(c);
  if (rc) return rc;
  if (!c->have_particles) return fail(c, SEDIMI_ESTATE, "no particles set");
  return SEDIMI_OK;
}

int read_ctl(sedimi_ctx* c, Ctl* out) {
  HIPCHK(c, hipMemcpyAsync(out, c->A.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int flags_to_rc(sedimi_ctx* c, int flags) {
  if (flags & kFlagNonFinite) return fail(c, SEDIMI_EUNSTABLE, "non-finite particle state");
  if (flags & kFlagEscape) return fail(c, SEDIMI_EESCAPE, "a particle left [0, Lz]");
  if (flags & kFlagCrowded)
    return fail(c, SEDIMI_EOVERFLOW,
                "a neighbour bin or mesh cell holds more particles than its sort allows");
  if (flags & kFlagOverflow) return fail(c, SEDIMI_EOVERFLOW, "neighbour or contact slots exceeded");
  if (flags & kFlagLost) return fail(c, SEDIMI_EOVERFLOW, "a contact fell out of the neighbour list");
  return SEDIMI_OK;
}

int set_rebuild_flag(sedimi_ctx* c) {
  int one = 1;
  HIPCHK(c, hipMemcpyAsync(c->A.rb, &one, sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

// Download a device array of `count` T's.
template <typename T>
int download(sedimi_ctx* c, std::vector<T>& h, const T* d, size_t count) {
  h.resize(count);
  if (count == 0) return SEDIMI_OK;
  HIPCHK(c, hipMemcpyAsync(h.data(), d, sizeof(T) * count, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

hipEvent_t take_event(sedimi_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Open / close a timed phase on the bound stream (no-ops unless profiling).
void phase_begin(sedimi_ctx* c, int phase) {
  if (!c->prof) return;
  sedimi_ctx::Mark m{phase, take_event(c), take_event(c)};
  if (m.a) (void)hipEventRecord(m.a, c->stream);
  c->marks.push_back(m);
}
void phase_end(sedimi_ctx* c) {
  if (!c->prof || c->marks.empty()) return;
  if (c->marks.back().b) (void)hipEventRecord(c->marks.back().b, c->stream);
}

void nn_run_forward(sedimi_ctx* c, bool keep);
int nn_check_smooth(sedimi_ctx* c, double rel[4]);

// Plain solve of channels [0, nch) of RAW into SMOOTH.  Returns the solver
// iterations (0 for the direct solve).  The direct solve is followed by the
// full-field residual r = A^N_tau y - raw (A = I - Delta tau L_h) for
// check_solve.
int64_t plain_solve(sedimi_ctx* c, int nch) {
  const int ntau = c->prm.avg_ntau;
  double tau = 0.25 * c->prm.avg_bandwidth * c->prm.avg_bandwidth;
  c->last_direct = c->direct && ntau > 0;
  int64_t it = 0;
  if (c->last_direct) {
    const bool bdf2 = c->prm.avg_scheme == SEDIMI_SCHEME_BDF2;
    launch_spectral(c->P, c->A, nch, ntau, tau, bdf2, c->stream);
    c->check_blocks = bdf2 ? launch_check_bdf2(c->P, c->A, nch, ntau, tau, c->stream)
                           : launch_check(c->P, c->A, c->A.smooth, nch, ntau, tau, 0, 1.0,
                                          c->stream);
  } else {
    const double rtol = c->mixed ? std::max(c->prm.avg_rtol, 1e-6) : c->prm.avg_rtol;
    it = launch_smooth(c->P, c->A, nch, ntau, tau, rtol, c->mixed,
                       c->prm.avg_scheme == SEDIMI_SCHEME_BDF2, c->stream);
  }
  // all channels smoothed: the solid velocity follows from the flux
  if (nch == 7) launch_solid_velocity(c->P, c->A, c->stream);
  return it;
}

int64_t do_average_plain(sedimi_ctx* c) { return plain_solve(c, c->P.nch_avg); }

// Residual bound of the direct solve: a backward-stable y has
// |A^N y - raw| <= c eps |A|^N |y| with |A| <= 1 + Delta tau lambda_max.
double direct_tol(const sedimi_ctx* c) {
  const DevParams& P = c->P;
  const int ntau = std::max(1, c->prm.avg_ntau);
  const double dtau = 0.25 * c->prm.avg_bandwidth * c->prm.avg_bandwidth / ntau;
  double lam = 0.0;
  if (P.nx > 1) lam += 4.0 / (P.hx * P.hx);
  if (P.ny > 1) lam += 4.0 / (P.hy * P.hy);
  if (P.nz > 1) lam += P.zlam;
  const double a = dtau * lam;
  // BDF2: the check multiplies y by (I + M)(3 I + 2 M)^(N-1), M = -dtau L
  const double amp = c->prm.avg_scheme == SEDIMI_SCHEME_BDF2
                         ? (1.0 + a) * pow(3.0 + 2.0 * a, (double)(ntau - 1))
                         : pow(1.0 + a, (double)ntau);
  return std::max(c->prm.avg_rtol, 1e-13 * amp);
}

// One averaging in the current mode.  Returns the solver iterations (0 when
// the network answered), or a negative SEDIMI_E* code.
int64_t do_average(sedimi_ctx* c, bool* used_plain) {
  phase_begin(c, 3);
  launch_deposit(c->P, c->A, c->stream);
  phase_end(c);
  phase_begin(c, 4);
  int64_t it = 0;
  bool plain = true;
  if (c->avg_mode != SEDIMI_AVG_PLAIN && c->prm.nn_enable) {
    nn_run_forward(c, false);
    ++c->nn_calls;
    plain = false;
    if (c->avg_mode == SEDIMI_AVG_SURROGATE_CHECKED) {
      double rel[4];  // the network's 4 channels
      int rc = nn_check_smooth(c, rel);
      if (rc) return rc;
      // the solid fraction decides: it is the field the particle step reads back
      const double worst = rel[0];
      c->nn_last_check = worst;
      if (!(worst <= c->prm.nn_bound)) {
        ++c->nn_fallbacks;
        plain = true;
      }
    }
  }
  if (plain) it = do_average_plain(c);
  launch_pack_eps(c->P, c->A, c->stream);
  phase_end(c);
  if (used_plain) *used_plain = plain;
  return it;
}

int check_solve(sedimi_ctx* c, int nch) {
  if (c->last_direct) {
    double rel[7];
    if (read_check(c->A, c->check_blocks, nch, rel, c->stream))
      return fail(c, SEDIMI_EDEVICE, "reading the solver residual failed");
    double res = 0.0;
    for (int ch = 0; ch < nch; ++ch) res = std::max(res, rel[ch]);
    c->last_residual = res;
    if (!(res <= direct_tol(c) * 10.0))
      return fail(c, SEDIMI_ENOCONV, "direct diffusion solve residual above its bound");
    return SEDIMI_OK;
  }
  double res = read_smooth_residual(c->P, c->A, nch, c->prm.avg_ntau, c->stream);
  if (res < 0) return fail(c, SEDIMI_EDEVICE, "reading the solver residual failed");
  c->last_residual = res;
  // FP32 working vectors cannot go below ~1e-6 relative
  const double tol = c->mixed ? std::max(c->prm.avg_rtol, 1e-6) : c->prm.avg_rtol;
  if (!(res <= tol * 10.0 + 1e-300))
    return fail(c, SEDIMI_ENOCONV, "diffusion solve residual above tolerance");
  return SEDIMI_OK;
}

}  // namespace

extern "C" {

int sedimi_create(const sedimi_params* p, int64_t max_particles, sedimi_ctx** out) {
  if (!p || !out) return SEDIMI_EINVAL;
  *out = nullptr;
  sedimi_ctx* c = new (std::nothrow) sedimi_ctx();
  if (!c) return SEDIMI_ENOMEM;
  int rc = check_params(c, *p, max_particles);
  c->prm = *p;
  c->cap = max_particles;
  c->mixed = p->precision == SEDIMI_MIXED;
  c->direct = p->avg_solver == SEDIMI_SOLVE_DIRECT ||
              (p->avg_solver == SEDIMI_SOLVE_AUTO &&
               std::max(p->nx, std::max(p->ny, p->nz)) <= kDirectMaxAxis &&
               (!graded_mesh(*p) || p->nz <= kGradedDirectMaxNz));
  if (rc == SEDIMI_OK) {
    fill_dev_params(c);
    if (c->direct && c->P.graded) {
      // the z transform of the graded operator (host eigen-decomposition)
      c->zdiag.assign(2 * (size_t)p->nz * p->nz + p->nz, 0.0);
      if (graded_z_transform(p->nz, c->zgeo.data(), c->zdiag.data()) != 0) {
        if (p->avg_solver == SEDIMI_SOLVE_DIRECT)
          rc = fail(c, SEDIMI_ENOCONV, "eigen-decomposition of the graded z operator failed");
        c->direct = false;
        c->zdiag.clear();
      }
    }
  }
  if (rc == SEDIMI_OK) {
    if (c->P.nbx < 3 || c->P.nby < 3)
      rc = fail(c, SEDIMI_EINVAL, "domain must span at least 3 neighbour bins in x and y");
    else if ((int64_t)c->P.nbins > (int64_t)INT32_MAX / 8)
      rc = fail(c, SEDIMI_EINVAL, "too many neighbour bins");
  }
  if (rc != SEDIMI_OK) {
    // keep the message reachable through a context-less error: print it
    fprintf(stderr, "sedimi_create: %s\n", c->err.c_str());
    delete c;
    return rc;
  }
  c->ws_bytes = layout(c, nullptr, nullptr);
  *out = c;
  return SEDIMI_OK;
}

void sedimi_destroy(sedimi_ctx* c) { delete c; }

const char* sedimi_last_error(const sedimi_ctx* c) {
  return c ? c->err.c_str() : g_noctx_err.c_str();
}

int sedimi_smooth_static(const sedimi_params* p, int nch, const double* raw, double* out,
                         void* stream) {
  auto bad = [](int code, const std::string& msg) {
    g_noctx_err = msg;
    return code;
  };
  if (!p) return bad(SEDIMI_EINVAL, "null parameters");
  if (!(p->Lx > 0 && p->Ly > 0 && p->Lz > 0) || p->nx < 1 || p->ny < 1 || p->nz < 1)
    return bad(SEDIMI_EINVAL, "domain and mesh must be positive");
  if (std::max(p->nx, std::max(p->ny, p->nz)) > kDirectMaxAxis)
    return bad(SEDIMI_EINVAL, "direct averaging solve needs <= 2048 cells per axis");
  if (graded_mesh(*p))
    return bad(SEDIMI_EINVAL, "the static solve needs a uniform z mesh (z_grading 0 or 1)");
  if (!(p->avg_bandwidth >= 0 && std::isfinite(p->avg_bandwidth)) ||
      !(p->avg_bandwidth_z >= 0 && std::isfinite(p->avg_bandwidth_z)) || p->avg_ntau < 0)
    return bad(SEDIMI_EINVAL, "averaging parameters out of range");
  if (p->avg_scheme != SEDIMI_SCHEME_EULER && p->avg_scheme != SEDIMI_SCHEME_BDF2)
    return bad(SEDIMI_EINVAL, "unknown averaging scheme");
  if (nch < 1 || nch > 7) return bad(SEDIMI_EINVAL, "nch must be 1..7");
  if (!raw || !out) return bad(SEDIMI_EINVAL, "null field");
  const size_t bytes = sizeof(double) * (size_t)nch * p->nx * p->ny * p->nz;
  if ((const char*)raw < (const char*)out + bytes && (const char*)out < (const char*)raw + bytes)
    return bad(SEDIMI_EINVAL, "raw and smooth fields overlap");
  double kz = 1.0;
  if (p->avg_bandwidth_z > 0 && p->avg_bandwidth > 0) {
    const double r = p->avg_bandwidth_z / p->avg_bandwidth;
    kz = r * r;
  }
  std::string err;
  const int rc = spectral_static(p->nx, p->ny, p->nz, p->Lx / p->nx, p->Ly / p->ny,
                                 p->Lz / p->nz, kz, nch, p->avg_ntau,
                                 0.25 * p->avg_bandwidth * p->avg_bandwidth,
                                 p->avg_scheme == SEDIMI_SCHEME_BDF2, raw, out,
                                 (hipStream_t)stream, &err);
  if (rc) return bad(rc, err);
  return SEDIMI_OK;
}

size_t sedimi_workspace_bytes(const sedimi_ctx* c) { return c ? c->ws_bytes : 0; }

int sedimi_bind_workspace(sedimi_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c) return SEDIMI_EINVAL;
  if (!dev_ptr || ((uintptr_t)dev_ptr & 255)) return fail(c, SEDIMI_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < c->ws_bytes) return fail(c, SEDIMI_ENOMEM, "workspace too small");
  c->ws = (char*)dev_ptr;
  layout(c, c->ws, &c->A);
  HIPCHK(c, hipMemsetAsync(c->ws, 0, c->ws_bytes, c->stream));
  {
    // Morton rank of every bin: interleave the bits of (bx, by, bz)
    const DevParams& P = c->P;
    std::vector<std::pair<uint64_t, int>> code((size_t)P.nbins);
    auto spread = [](uint64_t v) {
      uint64_t r = 0;
      for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
      return r;
    };
    for (int bz = 0; bz < P.nbz; ++bz)
      for (int by = 0; by < P.nby; ++by)
        for (int bx = 0; bx < P.nbx; ++bx) {
          int b = (bz * P.nby + by) * P.nbx + bx;
          code[b] = {spread(bx) | (spread(by) << 1) | (spread(bz) << 2), b};
        }
    std::sort(code.begin(), code.end());
    std::vector<int> rank((size_t)P.nbins);
    for (int r = 0; r < P.nbins; ++r) rank[code[r].second] = r;
    HIPCHK(c, hipMemcpyAsync(c->A.bin_rank, rank.data(), sizeof(int) * rank.size(),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->A.zgeo, c->zgeo.data(), sizeof(double) * c->zgeo.size(),
                             hipMemcpyHostToDevice, c->stream));
    std::vector<double> zt(4 * (size_t)P.nz);
    double tau = 0.25 * c->prm.avg_bandwidth * c->prm.avg_bandwidth;
    const double* zcoup = c->zgeo.data() + zgeo_coupling(P.nz);
    smooth_ztab(P, zcoup, std::max(1, c->prm.avg_ntau), tau, zt.data());
    smooth_ztab(P, zcoup, std::max(1, c->prm.avg_ntau), (2.0 / 3.0) * tau,
                zt.data() + 2 * P.nz);
    HIPCHK(c, hipMemcpyAsync(c->A.ztab, zt.data(), sizeof(double) * zt.size(),
                             hipMemcpyHostToDevice, c->stream));
    if (c->direct) {
      std::vector<double> st(spectral_table_doubles(P));
      spectral_tables(P, c->zdiag.empty() ? nullptr : c->zdiag.data(), st.data());
      HIPCHK(c, hipMemcpyAsync(c->A.spec, st.data(), sizeof(double) * st.size(),
                               hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (c->prm.nn_enable) {
      // the network's skip S: taps in x and y, the z-line Thomas table
      const int N = std::max(1, c->prm.avg_ntau);
      const double dtau = tau / N;
      std::vector<double> tx, ty;
      int ox = 0, oy = 0;
      split_taps(P.nx, dtau / (P.hx * P.hx), N, &tx, &ox);
      split_taps(P.ny, dtau / (P.hy * P.hy), N, &ty, &oy);
      const double cz = dtau * P.kz_diff / (P.hz * P.hz);
      std::vector<double> stab(2 * kSplitMaxTaps + 2 * (size_t)P.nz, 0.0);
      std::copy(tx.begin(), tx.end(), stab.begin());
      std::copy(ty.begin(), ty.end(), stab.begin() + kSplitMaxTaps);
      double* ib = stab.data() + 2 * kSplitMaxTaps;
      double* gm = ib + P.nz;
      // Thomas factors of (1 + c n_k) u_k - c u_{k-1} - c u_{k+1}: pivots and
      // the back-substitution multipliers
      double bet = 1.0 + cz * ((P.nz > 1) ? 1 : 0);
      ib[0] = 1.0 / bet;
      for (int k = 1; k < P.nz; ++k) {
        gm[k] = -cz / bet;
        const double diag = 1.0 + cz * (k == P.nz - 1 ? 1 : 2);
        bet = diag + cz * gm[k];
        ib[k] = 1.0 / bet;
      }
      HIPCHK(c, hipMemcpyAsync(c->nn.stab, stab.data(), sizeof(double) * stab.size(),
                               hipMemcpyHostToDevice, c->stream));
      c->split.tapx = c->nn.stab;
      c->split.tapy = c->nn.stab + kSplitMaxTaps;
      c->split.ztab = c->nn.stab + 2 * kSplitMaxTaps;
      c->split.off0x = ox, c->split.ntapx = (int)tx.size();
      c->split.off0y = oy, c->split.ntapy = (int)ty.size();
      c->split.cz = cz;
      // the network check: Green's function window and the sampled columns
      // (the nn_sample share of the columns with the smallest seeded hashes)
      c->green = green_window(P, c->prm.avg_ntau, tau);
      HIPCHK(c, hipMemcpyAsync(c->nn.gtab, c->green.tab.data(),
                               sizeof(double) * c->green.tab.size(), hipMemcpyHostToDevice,
                               c->stream));
      const int ncol = P.nx * P.ny;
      std::vector<std::pair<uint64_t, int>> h((size_t)ncol);
      uint64_t st = c->prm.nn_seed;
      for (int q = 0; q < ncol; ++q) {
        uint64_t s2 = st ^ (uint64_t)q;
        h[q] = {mix64(s2), q};
      }
      c->green_cols = nn_check_columns(c->prm);
      std::partial_sort(h.begin(), h.begin() + c->green_cols, h.end());
      std::vector<int> cols((size_t)c->green_cols);
      for (int q = 0; q < c->green_cols; ++q) cols[q] = h[q].second;
      std::sort(cols.begin(), cols.end());
      HIPCHK(c, hipMemcpyAsync(c->nn.cols, cols.data(), sizeof(int) * cols.size(),
                               hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->have_particles = false;
  return SEDIMI_OK;
}

int sedimi_set_stream(sedimi_ctx* c, void* s) {
  if (!c) return SEDIMI_EINVAL;
  c->stream = (hipStream_t)s;
  return SEDIMI_OK;
}

int sedimi_set_particles(sedimi_ctx* c, int64_t n, const double* x, const double* v,
                         const double* w, const double* d, const double* rho) {
  int rc = need_ws(c);
  if (rc) return rc;
  if (n < 0 || n > c->cap) return fail(c, SEDIMI_EINVAL, "particle count exceeds capacity");
  if (n > 0 && (!x || !v || !d || !rho)) return fail(c, SEDIMI_EINVAL, "null particle array");
  std::vector<double4> pos(n), vel(n), omg(n);
  std::vector<int> id(n);
  for (int64_t i = 0; i < n; ++i) {
    double di = d[i];
    if (!(di > 0 && di <= c->prm.d_max)) return fail(c, SEDIMI_EINVAL, "diameter outside (0, d_max]");
    if (!(rho[i] > 0)) return fail(c, SEDIMI_EINVAL, "density must be positive");
    double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
    if (!(xi >= 0 && xi < c->prm.Lx && yi >= 0 && yi < c->prm.Ly && zi >= 0 && zi <= c->prm.Lz))
      return fail(c, SEDIMI_EINVAL, "particle centre outside the domain");
    double V = (kPi / 6.0) * di * di * di;
    pos[i] = make_double4(xi, yi, zi, 0.5 * di);
    vel[i] = make_double4(v[3 * i], v[3 * i + 1], v[3 * i + 2], rho[i] * V);
    omg[i] = w ? make_double4(w[3 * i], w[3 * i + 1], w[3 * i + 2], 0.0) : make_double4(0, 0, 0, 0);
    id[i] = (int)i;
  }
  c->n = n;
  c->P.n = (int)n;
  c->step = 0;
  // clear the per-particle arrays (they precede the mesh arrays in the
  // layout) and the control block; mesh fields are kept
  HIPCHK(c, hipMemsetAsync(c->ws, 0, (size_t)((char*)c->A.U - c->ws), c->stream));
  HIPCHK(c, hipMemsetAsync(c->A.ctl, 0, sizeof(Ctl), c->stream));
  c->A.rb = &c->A.ctl->rebuild;
  c->A.rb_next = &c->A.ctl->rebuild_alt;
  if (n > 0) {
    HIPCHK(c, hipMemcpyAsync(c->A.pos, pos.data(), sizeof(double4) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->A.vel, vel.data(), sizeof(double4) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->A.omg, omg.data(), sizeof(double4) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->A.id, id.data(), sizeof(int) * n, hipMemcpyHostToDevice, c->stream));
  }
  rc = set_rebuild_flag(c);
  if (rc) return rc;
  launch_rebuild(c->P, c->A, false, c->mixed, c->stream);
  Ctl ctl;
  rc = read_ctl(c, &ctl);
  if (rc) return rc;
  c->have_particles = true;
  return flags_to_rc(c, ctl.flags);
}

int sedimi_set_fluid(sedimi_ctx* c, const double* U, const double* gp, const double* du) {
  int rc = need_ws(c);
  if (rc) return rc;
  const int nc = c->P.ncell;
  std::vector<double4> h(nc);
  const double* src[3] = {U, gp, du};
  double4* dst[3] = {c->A.U, c->A.gp, c->A.du};
  for (int f = 0; f < 3; ++f) {
    for (int k = 0; k < nc; ++k)
      h[k] = src[f] ? make_double4(src[f][3 * k], src[f][3 * k + 1], src[f][3 * k + 2], 0.0)
                    : make_double4(0, 0, 0, 0);
    HIPCHK(c, hipMemcpyAsync(dst[f], h.data(), sizeof(double4) * nc, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  // G = -grad p + C_add rho_f DU/Dt, the combination the step kernel reads
  const double ca = c->prm.c_add * c->prm.rho_f;
  for (int k = 0; k < nc; ++k) {
    double g[3], m[3];
    for (int a = 0; a < 3; ++a) {
      g[a] = gp ? gp[3 * k + a] : 0.0;
      m[a] = du ? du[3 * k + a] : 0.0;
    }
    h[k] = make_double4(-g[0] + ca * m[0], -g[1] + ca * m[1], -g[2] + ca * m[2], 0.0);
  }
  HIPCHK(c, hipMemcpyAsync(c->A.G, h.data(), sizeof(double4) * nc, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->prm.c_lift > 0) {
    // vorticity of the frozen flow at cell centres (central differences,
    // periodic in x and y, one-sided in the first and last z cell), read by
    // the shear lift
    const DevParams& P = c->P;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    auto u = [&](int i, int j, int k, int a) {
      return U ? U[3 * (((size_t)k * ny + j) * nx + i) + a] : 0.0;
    };
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          const int ip = (i + 1) % nx, im = (i + nx - 1) % nx;
          const int jp = (j + 1) % ny, jm = (j + ny - 1) % ny;
          const int kp = std::min(k + 1, nz - 1), km = std::max(k - 1, 0);
          double gx[3], gy[3], gz[3];
          for (int a = 0; a < 3; ++a) {
            gx[a] = (u(ip, j, k, a) - u(im, j, k, a)) / (2.0 * P.hx);
            gy[a] = (u(i, jp, k, a) - u(i, jm, k, a)) / (2.0 * P.hy);
            // z differences over the centre distance (graded meshes: the
            // centres' own heights)
            const double dzc = P.graded ? c->zgeo[zgeo_centres(nz) + kp] - c->zgeo[zgeo_centres(nz) + km]
                                        : (kp - km) * P.hz;
            gz[a] = kp > km ? (u(i, j, kp, a) - u(i, j, km, a)) / dzc : 0.0;
          }
          h[((size_t)k * ny + j) * nx + i] =
              make_double4(gy[2] - gz[1], gz[0] - gx[2], gx[1] - gy[0], 0.0);
        }
    HIPCHK(c, hipMemcpyAsync(c->A.W, h.data(), sizeof(double4) * nc, hipMemcpyHostToDevice, c->stream));
  }
  launch_pack_eps(c->P, c->A, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int sedimi_set_field(sedimi_ctx* c, int field, const double* in) {
  int rc = need_ws(c);
  if (rc) return rc;
  if (!in || (field != SEDIMI_FIELD_RAW && field != SEDIMI_FIELD_SMOOTH))
    return fail(c, SEDIMI_EINVAL, "bad field");
  double* dst = field == SEDIMI_FIELD_RAW ? c->A.raw : c->A.smooth;
  HIPCHK(c, hipMemcpyAsync(dst, in, sizeof(double) * c->P.nch_avg * c->P.ncell,
                           hipMemcpyHostToDevice, c->stream));
  if (field == SEDIMI_FIELD_SMOOTH) launch_pack_eps(c->P, c->A, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int sedimi_translate(sedimi_ctx* c, double dx, double dy) {
  int rc = need_particles(c);
  if (rc) return rc;
  if (!(std::isfinite(dx) && std::isfinite(dy))) return fail(c, SEDIMI_EINVAL, "non-finite shift");
  launch_translate(c->P, c->A, dx, dy, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int sedimi_set_accel(sedimi_ctx* c, const double* a, const double* alpha) {
  int rc = need_particles(c);
  if (rc) return rc;
  std::vector<int> id;
  rc = download(c, id, c->A.id, (size_t)c->n);
  if (rc) return rc;
  std::vector<double4> ha(c->n), hal(c->n);
  rc = download(c, ha, c->A.acc, (size_t)c->n);
  if (rc) return rc;
  rc = download(c, hal, c->A.alp, (size_t)c->n);
  if (rc) return rc;
  for (int64_t q = 0; q < c->n; ++q) {
    int i = id[q];
    if (a) ha[q] = make_double4(a[3 * i], a[3 * i + 1], a[3 * i + 2], 0.0);
    if (alpha) hal[q] = make_double4(alpha[3 * i], alpha[3 * i + 1], alpha[3 * i + 2], 0.0);
  }
  HIPCHK(c, hipMemcpyAsync(c->A.acc, ha.data(), sizeof(double4) * c->n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->A.alp, hal.data(), sizeof(double4) * c->n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int sedimi_compute_forces(sedimi_ctx* c, int update_history) {
  int rc = need_particles(c);
  if (rc) return rc;
  launch_forces(c->P, c->A, 1, update_history != 0, c->mixed, c->stream);
  HIPCHK(c, hipGetLastError());
  Ctl ctl;
  rc = read_ctl(c, &ctl);
  if (rc) return rc;
  return flags_to_rc(c, ctl.flags);
}

int sedimi_rebuild(sedimi_ctx* c) {
  int rc = need_particles(c);
  if (rc) return rc;
  if ((rc = set_rebuild_flag(c))) return rc;
  phase_begin(c, 1);
  launch_rebuild(c->P, c->A, true, c->mixed, c->stream);
  phase_end(c);
  HIPCHK(c, hipGetLastError());
  // the force kernel clears the flag and counts the rebuild; with no force
  // evaluation in this call, do both here so the next step does not rebuild
  // again
  Ctl ctl;
  if ((rc = read_ctl(c, &ctl))) return rc;
  ctl.rebuilds += 1;
  ctl.rebuild = ctl.rebuild_alt = 0;
  HIPCHK(c, hipMemcpyAsync(c->A.ctl, &ctl, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return flags_to_rc(c, ctl.flags);
}

}  // extern "C"

namespace {

// The kernel sequence of nsteps particle steps (with the averagings that
// fall in them), enqueued on c->stream; host bookkeeping (buffer swaps, the
// step counter, the solve's check state) advances as it goes.
int step_loop(sedimi_ctx* c, int nsteps, int average_every, bool* averaged_out) {
  bool averaged = false;
  // A step whose successor is in this call and is not preceded by an
  // averaging fuses the successor's half kick and drift into its force
  // kernel; the state between calls is always the end of a whole step.
  bool drifted = false;
  for (int s = 0; s < nsteps; ++s) {
    if (!drifted) {
      phase_begin(c, 0);
      launch_kick_drift(c->P, c->A, c->stream);
      phase_end(c);
    }
    phase_begin(c, 1);
    launch_rebuild(c->P, c->A, true, c->mixed, c->stream);
    phase_end(c);
    const bool avg_now = average_every > 0 && (c->step + 1) % average_every == 0;
    const bool fuse = s + 1 < nsteps && !avg_now;
    phase_begin(c, 2);
    launch_forces(c->P, c->A, fuse ? 2 : 0, true, c->mixed, c->stream);
    phase_end(c);
    std::swap(c->A.vel, c->A.vel_t);
    std::swap(c->A.omg, c->A.omg_t);
    if (fuse) {
      std::swap(c->A.pos, c->A.pos_t);
      std::swap(c->A.rb, c->A.rb_next);
    }
    drifted = fuse;
    ++c->step;
    if (avg_now) {
      bool plain = true;
      int64_t it = do_average(c, &plain);
      if (it < 0) return (int)it;
      c->last_iters = it;
      averaged = plain;  // residual partials of the last averaging (plain only)
    }
  }
  *averaged_out = averaged;
  return SEDIMI_OK;
}

// Whether a call's steps can be replayed from a graph: no read-back inside
// them, i.e. every averaging they contain is the plain direct solve.
bool step_graphable(const sedimi_ctx* c, int nsteps, int average_every) {
  if (!c->graphs_on || c->prof || nsteps <= 0 || c->n <= 0) return false;
  const bool avg_inside =
      average_every > 0 && (c->step % average_every) + nsteps >= average_every;
  if (!avg_inside) return true;
  const bool network = c->avg_mode != SEDIMI_AVG_PLAIN && c->prm.nn_enable;
  return !network && c->direct && c->prm.avg_ntau > 0;
}

void put_bytes(std::vector<unsigned char>& k, const void* v, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(v);
  k.insert(k.end(), b, b + n);
}

// Everything the captured launches depend on: the device parameters and
// array pointers passed by value, the parameters the host derives launch
// arguments from, the call's shape and where it starts in the averaging
// cycle.
std::vector<unsigned char> step_key(const sedimi_ctx* c, int nsteps, int average_every) {
  std::vector<unsigned char> k;
  const int32_t head[6] = {nsteps, average_every,
                           average_every > 0 ? (int32_t)(c->step % average_every) : 0,
                           c->avg_mode, c->direct ? 1 : 0, c->mixed ? 1 : 0};
  put_bytes(k, head, sizeof(head));
  put_bytes(k, &c->P, sizeof(c->P));
  put_bytes(k, &c->A, sizeof(c->A));
  put_bytes(k, &c->prm, sizeof(c->prm));
  return k;
}

constexpr size_t kMaxStepGraphs = 4;

int step_graph(sedimi_ctx* c, int nsteps, int average_every, bool* averaged) {
  std::vector<unsigned char> key = step_key(c, nsteps, average_every);
  for (auto& g : c->graphs) {
    if (g.key != key) continue;
    HIPCHK(c, hipGraphLaunch(g.exec, c->stream));
    c->A = g.after;
    c->step += nsteps;
    if (g.averaged) {
      c->last_iters = g.last_iters;
      c->last_direct = g.last_direct;
      c->check_blocks = g.check_blocks;
    }
    *averaged = g.averaged;
    g.used = ++c->graph_clock;
    ++c->graph_steps;
    return SEDIMI_OK;
  }
  if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  // capture records and runs nothing: keep the host state to restore if it fails
  const DevArrays A0 = c->A;
  const int64_t step0 = c->step, iters0 = c->last_iters;
  const bool direct0 = c->last_direct;
  const int blocks0 = c->check_blocks;
  hipStream_t user = c->stream;
  c->stream = c->cap_stream;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
  int rc = SEDIMI_OK;
  bool av = false;
  hipGraph_t graph = nullptr;
  if (e == hipSuccess) {
    rc = step_loop(c, nsteps, average_every, &av);
    const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
    if (e2 != hipSuccess) e = e2;
  }
  c->stream = user;
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess && rc == SEDIMI_OK && graph)
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess || rc != SEDIMI_OK || !exec) {
    // take these steps eagerly and do not try again on this context
    (void)hipGetLastError();
    c->A = A0, c->step = step0, c->last_iters = iters0;
    c->last_direct = direct0, c->check_blocks = blocks0;
    c->graphs_on = false;
    return step_loop(c, nsteps, average_every, averaged);
  }
  sedimi_ctx::StepGraph g;
  g.key = std::move(key);
  g.exec = exec;
  g.after = c->A;
  g.averaged = av;
  g.last_direct = c->last_direct;
  g.last_iters = c->last_iters;
  g.check_blocks = c->check_blocks;
  g.used = ++c->graph_clock;
  if (c->graphs.size() >= kMaxStepGraphs) {
    size_t lru = 0;
    for (size_t i = 1; i < c->graphs.size(); ++i)
      if (c->graphs[i].used < c->graphs[lru].used) lru = i;
    (void)hipGraphExecDestroy(c->graphs[lru].exec);
    c->graphs.erase(c->graphs.begin() + (long)lru);
  }
  c->graphs.push_back(std::move(g));
  HIPCHK(c, hipGraphLaunch(exec, c->stream));
  ++c->graph_steps;
  *averaged = av;
  return SEDIMI_OK;
}

}  // namespace

extern "C" {

int sedimi_step(sedimi_ctx* c, int nsteps, int average_every) {
  int rc = need_particles(c);
  if (rc) return rc;
  if (nsteps < 0) return fail(c, SEDIMI_EINVAL, "nsteps must be >= 0");
  bool averaged = false;
  rc = step_graphable(c, nsteps, average_every) ? step_graph(c, nsteps, average_every, &averaged)
                                                 : step_loop(c, nsteps, average_every, &averaged);
  if (rc) return rc;
  HIPCHK(c, hipGetLastError());
  Ctl ctl;
  rc = read_ctl(c, &ctl);
  if (rc) return rc;
  rc = flags_to_rc(c, ctl.flags);
  if (rc) return rc;
  if (averaged) return check_solve(c, c->P.nch_avg);
  return SEDIMI_OK;
}

int sedimi_set_step_graphs(sedimi_ctx* c, int enable) {
  if (!c) return SEDIMI_EINVAL;
  c->graphs_on = enable != 0;
  if (!c->graphs_on) c->drop_graphs();
  return SEDIMI_OK;
}

int sedimi_average(sedimi_ctx* c) {
  int rc = need_particles(c);
  if (rc) return rc;
  bool plain = true;
  int64_t it = do_average(c, &plain);
  if (it < 0) return (int)it;
  c->last_iters = it;
  HIPCHK(c, hipGetLastError());
  Ctl ctl;
  if ((rc = read_ctl(c, &ctl))) return rc;
  if ((rc = flags_to_rc(c, ctl.flags))) return rc;
  if (!plain) return SEDIMI_OK;
  return check_solve(c, c->P.nch_avg);
}

int sedimi_deposit(sedimi_ctx* c) {
  int rc = need_particles(c);
  if (rc) return rc;
  launch_deposit(c->P, c->A, c->stream);
  HIPCHK(c, hipGetLastError());
  Ctl ctl;
  if ((rc = read_ctl(c, &ctl))) return rc;
  return flags_to_rc(c, ctl.flags);
}

int sedimi_smooth(sedimi_ctx* c, int nch) {
  int rc = need_ws(c);
  if (rc) return rc;
  if (nch < 1 || nch > c->P.nch_avg)
    return fail(c, SEDIMI_EINVAL, "nch must be 1..4 (1..7 with avg_solid_velocity)");
  c->last_iters = plain_solve(c, nch);
  launch_pack_eps(c->P, c->A, c->stream);
  HIPCHK(c, hipGetLastError());
  return check_solve(c, nch);
}

int sedimi_get_particles(sedimi_ctx* c, double* x, double* v, double* w, double* a) {
  int rc = need_particles(c);
  if (rc) return rc;
  const size_t n = (size_t)c->n;
  std::vector<int> id;
  rc = download(c, id, c->A.id, n);
  if (rc) return rc;
  double* outs[4] = {x, v, w, a};
  const double4* srcs[4] = {c->A.pos, c->A.vel, c->A.omg, c->A.acc};
  std::vector<double4> h;
  for (int f = 0; f < 4; ++f) {
    if (!outs[f]) continue;
    rc = download(c, h, srcs[f], n);
    if (rc) return rc;
    for (size_t q = 0; q < n; ++q) {
      double* o = outs[f] + 3 * (size_t)id[q];
      o[0] = h[q].x, o[1] = h[q].y, o[2] = h[q].z;
    }
  }
  return SEDIMI_OK;
}

int sedimi_get_accel(sedimi_ctx* c, double* a, double* alpha) {
  int rc = need_particles(c);
  if (rc) return rc;
  const size_t n = (size_t)c->n;
  std::vector<int> id;
  rc = download(c, id, c->A.id, n);
  if (rc) return rc;
  double* outs[2] = {a, alpha};
  const double4* srcs[2] = {c->A.acc, c->A.alp};
  std::vector<double4> h;
  for (int f = 0; f < 2; ++f) {
    if (!outs[f]) continue;
    rc = download(c, h, srcs[f], n);
    if (rc) return rc;
    for (size_t q = 0; q < n; ++q) {
      double* o = outs[f] + 3 * (size_t)id[q];
      o[0] = h[q].x, o[1] = h[q].y, o[2] = h[q].z;
    }
  }
  return SEDIMI_OK;
}

int sedimi_get_forces(sedimi_ctx* c, int comp, double* f) {
  int rc = need_particles(c);
  if (rc) return rc;
  if (comp < 0 || comp > SEDIMI_F_LIFT || !f) return fail(c, SEDIMI_EINVAL, "bad force component");
  const size_t n = (size_t)c->n;
  std::vector<int> id;
  rc = download(c, id, c->A.id, n);
  if (rc) return rc;
  std::vector<double4> h;
  rc = download(c, h, c->A.comp + (size_t)comp * n, n);
  if (rc) return rc;
  for (size_t q = 0; q < n; ++q) {
    double* o = f + 3 * (size_t)id[q];
    o[0] = h[q].x, o[1] = h[q].y, o[2] = h[q].z;
  }
  return SEDIMI_OK;
}

int sedimi_get_field(sedimi_ctx* c, int field, double* out) {
  int rc = need_ws(c);
  if (rc) return rc;
  if (!out || field < SEDIMI_FIELD_RAW || field > SEDIMI_FIELD_US)
    return fail(c, SEDIMI_EINVAL, "bad field");
  if (field == SEDIMI_FIELD_US && c->P.nch_avg != 7)
    return fail(c, SEDIMI_EINVAL, "the solid velocity needs avg_solid_velocity");
  const double* src = field == SEDIMI_FIELD_RAW ? c->A.raw
                      : field == SEDIMI_FIELD_SMOOTH ? c->A.smooth : c->A.us;
  const size_t nch = field == SEDIMI_FIELD_US ? 3 : (size_t)c->P.nch_avg;
  HIPCHK(c, hipMemcpyAsync(out, src, sizeof(double) * nch * c->P.ncell, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int sedimi_get_pairs(sedimi_ctx* c, int64_t cap, int64_t* ij, int64_t* n_out) {
  int rc = need_particles(c);
  if (rc) return rc;
  if (!n_out) return fail(c, SEDIMI_EINVAL, "null n_out");
  const size_t n = (size_t)c->n;
  // the pair test runs on the device (the force kernel's exact predicate);
  // the key array serves as scratch for the slot masks
  launch_pairmask(c->P, c->A, (unsigned*)c->A.key, c->stream);
  HIPCHK(c, hipGetLastError());
  std::vector<unsigned> mask;
  std::vector<int> id, cnt, nbr;
  if ((rc = download(c, mask, (const unsigned*)c->A.key, n))) return rc;
  if ((rc = download(c, id, c->A.id, n))) return rc;
  if ((rc = download(c, cnt, c->A.ncnt, n))) return rc;
  if ((rc = download(c, nbr, c->A.nbr, (size_t)c->P.maxn * n))) return rc;
  std::vector<std::pair<int64_t, int64_t>> pairs;
  for (size_t q = 0; q < n; ++q) {
    for (int k = 0; k < cnt[q]; ++k) {
      if (!(mask[q] & (1u << k))) continue;
      int j = nbr[(size_t)k * n + q];
      if (id[q] < id[j]) pairs.emplace_back(id[q], id[j]);
    }
  }
  std::sort(pairs.begin(), pairs.end());
  *n_out = (int64_t)pairs.size();
  if ((int64_t)pairs.size() > cap) return fail(c, SEDIMI_EOVERFLOW, "pair buffer too small");
  for (size_t k = 0; k < pairs.size(); ++k) {
    ij[2 * k] = pairs[k].first;
    ij[2 * k + 1] = pairs[k].second;
  }
  return SEDIMI_OK;
}

struct HistRec {
  int64_t i, j;
  double xi[3];
};

int sedimi_get_history(sedimi_ctx* c, int64_t cap, void* records, int64_t* n_out) {
  int rc = need_particles(c);
  if (rc) return rc;
  if (!n_out) return fail(c, SEDIMI_EINVAL, "null n_out");
  const size_t n = (size_t)c->n, maxn = (size_t)c->P.maxn;
  std::vector<int> id, cnt, nbr;
  std::vector<unsigned> mask;
  std::vector<double4> wxi;
  if ((rc = download(c, id, c->A.id, n))) return rc;
  if ((rc = download(c, cnt, c->A.ncnt, n))) return rc;
  if ((rc = download(c, nbr, c->A.nbr, maxn * n))) return rc;
  if ((rc = download(c, mask, c->A.hmask, n))) return rc;
  if ((rc = download(c, wxi, c->A.wxi, 2 * n))) return rc;
  std::vector<double> hd;
  std::vector<float> hf;
  if (c->mixed) {
    if ((rc = download(c, hf, (const float*)c->A.hxi, 3 * maxn * n))) return rc;
  } else {
    if ((rc = download(c, hd, (const double*)c->A.hxi, 3 * maxn * n))) return rc;
  }
  auto hx = [&](int comp, size_t k, size_t q) -> double {
    size_t o = ((size_t)comp * maxn + k) * n + q;
    return c->mixed ? (double)hf[o] : hd[o];
  };
  std::vector<HistRec> out;
  for (size_t q = 0; q < n; ++q) {
    for (int k = 0; k < cnt[q]; ++k) {
      if (!(mask[q] & (1u << k))) continue;
      int j = nbr[(size_t)k * n + q];
      if (id[q] < id[j]) out.push_back({id[q], id[j], {hx(0, k, q), hx(1, k, q), hx(2, k, q)}});
    }
    for (int side = 0; side < 2; ++side) {
      const double4& h = wxi[(size_t)side * n + q];
      if (h.w != 0.0) out.push_back({id[q], side == 0 ? -1 : -2, {h.x, h.y, h.z}});
    }
  }
  std::sort(out.begin(), out.end(), [](const HistRec& a, const HistRec& b) {
    return a.i != b.i ? a.i < b.i : a.j < b.j;
  });
  *n_out = (int64_t)out.size();
  if ((int64_t)out.size() > cap) return fail(c, SEDIMI_EOVERFLOW, "history buffer too small");
  if (!out.empty()) memcpy(records, out.data(), sizeof(HistRec) * out.size());
  return SEDIMI_OK;
}

int sedimi_set_history(sedimi_ctx* c, int64_t nrec, const void* records) {
  int rc = need_particles(c);
  if (rc) return rc;
  if (nrec < 0 || (nrec > 0 && !records)) return fail(c, SEDIMI_EINVAL, "bad history records");
  const size_t n = (size_t)c->n;
  std::vector<int> id;
  if ((rc = download(c, id, c->A.id, n))) return rc;
  std::vector<int> where(n);
  for (size_t q = 0; q < n; ++q) where[id[q]] = (int)q;
  std::vector<int> cid((size_t)kMaxContacts * n, 0), ccnt(n, 0);
  std::vector<double> cxi(3 * (size_t)kMaxContacts * n, 0.0);
  std::vector<double4> wxi(2 * n, make_double4(0, 0, 0, 0));
  const HistRec* r = (const HistRec*)records;
  auto add = [&](int64_t self, int64_t partner, const double* xi) -> bool {
    size_t q = (size_t)where[self];
    int k = ccnt[q];
    if (k >= kMaxContacts) return false;
    cid[(size_t)k * n + q] = (int)partner;
    for (int a = 0; a < 3; ++a) cxi[((size_t)a * kMaxContacts + k) * n + q] = xi[a];
    ccnt[q] = k + 1;
    return true;
  };
  for (int64_t t = 0; t < nrec; ++t) {
    int64_t i = r[t].i, j = r[t].j;
    if (i < 0 || i >= c->n || j < -2 || j >= c->n || (j >= 0 && j <= i))
      return fail(c, SEDIMI_EINVAL, "history record has bad IDs");
    if (j < 0) {
      wxi[(size_t)(j == -1 ? 0 : 1) * n + where[i]] = make_double4(r[t].xi[0], r[t].xi[1], r[t].xi[2], 1.0);
    } else if (!add(i, j, r[t].xi) || !add(j, i, r[t].xi)) {
      return fail(c, SEDIMI_EOVERFLOW, "too many contacts for one particle");
    }
  }
  HIPCHK(c, hipMemcpyAsync(c->A.cid, cid.data(), sizeof(int) * cid.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->A.cxi, cxi.data(), sizeof(double) * cxi.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->A.ccnt, ccnt.data(), sizeof(int) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->A.wxi, wxi.data(), sizeof(double4) * 2 * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemsetAsync(c->A.ctl, 0, sizeof(int) * 4, c->stream));
  c->A.rb = &c->A.ctl->rebuild;
  c->A.rb_next = &c->A.ctl->rebuild_alt;
  rc = set_rebuild_flag(c);
  if (rc) return rc;
  launch_rebuild(c->P, c->A, false, c->mixed, c->stream);
  // the next force kernel clears the rebuild flag; do it here for a clean state
  int zero = 0;
  HIPCHK(c, hipMemcpyAsync(c->A.rb, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
  Ctl ctl;
  if ((rc = read_ctl(c, &ctl))) return rc;
  if (ctl.flags & kFlagLost)
    return fail(c, SEDIMI_EINVAL, "a history pair is not in the neighbour list");
  return flags_to_rc(c, ctl.flags);
}

}  // extern "C"

namespace {

// Header of a state blob; the workspace bytes follow it.
struct StateHeader {
  char magic[8];
  uint64_t header_bytes, ws_bytes;
  // layout: a restoring context must carve its workspace the same way
  int64_t cap;
  int32_t maxn, nbins, ncell, nch_avg, mixed, direct, nn_enable, pad0;
  // host-side state
  int64_t n, step, adam_t, nn_calls, nn_fallbacks, last_iters;
  double nn_last_check, last_residual;
  int32_t avg_mode, have_particles, last_direct, check_blocks;
  uint32_t swapped;  // double buffers in their second position: vel, omg, pos, rb
  int32_t nn_groups;
  NNNorm norm;
  // the device parameters (every physical parameter the kernels and the
  // workspace's derived tables and fields depend on), particle count zeroed
  DevParams P;
  // the averaging and network parameters that DevParams does not carry (the
  // z-line and spectral tables in the workspace derive from the bandwidths
  // and N_tau)
  struct AvgParams {
    double avg_bandwidth, avg_bandwidth_z, avg_rtol, nn_alpha, nn_bound, nn_sample, z_grading;
    uint64_t nn_seed;
    int32_t avg_ntau, avg_scheme, avg_solver, avg_solid_velocity;
  } avg;
};
constexpr char kStateMagic[8] = {'S', 'E', 'D', 'I', 'M', 'I', 'S', '1'};

// Field by field into a zeroed struct (no padding bytes are compared).
void state_avg_params(const sedimi_ctx* c, StateHeader::AvgParams* a) {
  memset(a, 0, sizeof(*a));
  const sedimi_params& p = c->prm;
  a->avg_bandwidth = p.avg_bandwidth;
  a->avg_bandwidth_z = p.avg_bandwidth_z;
  a->avg_rtol = p.avg_rtol;
  a->nn_alpha = p.nn_alpha;
  a->nn_bound = p.nn_bound;
  a->nn_sample = p.nn_sample;
  a->z_grading = p.z_grading;
  a->nn_seed = p.nn_seed;
  a->avg_ntau = p.avg_ntau;
  a->avg_scheme = p.avg_scheme;
  a->avg_solver = p.avg_solver;
  a->avg_solid_velocity = p.avg_solid_velocity;
}

void state_layout(const sedimi_ctx* c, StateHeader* h) {
  h->ws_bytes = c->ws_bytes;
  h->cap = c->cap;
  h->maxn = c->P.maxn;
  h->nbins = c->P.nbins;
  h->ncell = c->P.ncell;
  h->nch_avg = c->P.nch_avg;
  h->mixed = c->mixed ? 1 : 0;
  h->direct = c->direct ? 1 : 0;
  h->nn_enable = c->prm.nn_enable ? 1 : 0;
}

}  // namespace

extern "C" {

int sedimi_get_state(sedimi_ctx* c, void* buf, size_t cap, size_t* size_out) {
  int rc = need_ws(c);
  if (rc) return rc;
  const size_t total = sizeof(StateHeader) + c->ws_bytes;
  if (size_out) *size_out = total;
  if (!buf) return SEDIMI_OK;
  if (cap < total) return fail(c, SEDIMI_ENOMEM, "state buffer too small");
  StateHeader h{};
  memcpy(h.magic, kStateMagic, sizeof(kStateMagic));
  h.header_bytes = sizeof(StateHeader);
  state_layout(c, &h);
  h.n = c->n, h.step = c->step, h.adam_t = c->adam_t;
  h.nn_calls = c->nn_calls, h.nn_fallbacks = c->nn_fallbacks, h.last_iters = c->last_iters;
  h.nn_last_check = c->nn_last_check, h.last_residual = c->last_residual;
  h.avg_mode = c->avg_mode, h.have_particles = c->have_particles ? 1 : 0;
  h.last_direct = c->last_direct ? 1 : 0, h.check_blocks = c->check_blocks;
  h.nn_groups = c->nn_groups;
  h.norm = c->norm;
  memcpy(&h.P, &c->P, sizeof(DevParams));  // bytes, padding included
  h.P.n = 0;
  state_avg_params(c, &h.avg);
  DevArrays canon{};
  layout(c, c->ws, &canon);
  h.swapped = (c->A.vel != canon.vel ? 1u : 0u) | (c->A.omg != canon.omg ? 2u : 0u) |
              (c->A.pos != canon.pos ? 4u : 0u) | (c->A.rb != canon.rb ? 8u : 0u);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  memcpy(buf, &h, sizeof(h));
  HIPCHK(c, hipMemcpy((char*)buf + sizeof(h), c->ws, c->ws_bytes, hipMemcpyDeviceToHost));
  return SEDIMI_OK;
}

int sedimi_set_state(sedimi_ctx* c, const void* buf, size_t size) {
  int rc = need_ws(c);
  if (rc) return rc;
  if (!buf || size < sizeof(StateHeader)) return fail(c, SEDIMI_EINVAL, "state blob too short");
  StateHeader h;
  memcpy(&h, buf, sizeof(h));
  if (memcmp(h.magic, kStateMagic, sizeof(kStateMagic)) != 0 ||
      h.header_bytes != sizeof(StateHeader) || size != sizeof(StateHeader) + h.ws_bytes)
    return fail(c, SEDIMI_EINVAL, "not a state blob of this library");
  StateHeader mine{};
  state_layout(c, &mine);
  if (h.ws_bytes != mine.ws_bytes || h.cap != mine.cap || h.maxn != mine.maxn ||
      h.nbins != mine.nbins || h.ncell != mine.ncell || h.nch_avg != mine.nch_avg ||
      h.mixed != mine.mixed || h.direct != mine.direct || h.nn_enable != mine.nn_enable)
    return fail(c, SEDIMI_EINVAL, "state blob from a context of another layout");
  if (h.n < 0 || h.n > c->cap || h.swapped > 15u)
    return fail(c, SEDIMI_EINVAL, "state blob out of range");
  // c->P is value-initialised (zero padding) and both sides are copied as bytes
  DevParams here;
  memcpy(&here, &c->P, sizeof(DevParams));
  here.n = 0;
  StateHeader::AvgParams avg_here;
  state_avg_params(c, &avg_here);
  if (memcmp(&here, &h.P, sizeof(DevParams)) != 0 ||
      memcmp(&avg_here, &h.avg, sizeof(avg_here)) != 0)
    return fail(c, SEDIMI_EINVAL, "state blob from a context with other parameters");
  if (h.avg_mode < SEDIMI_AVG_PLAIN || h.avg_mode > SEDIMI_AVG_SURROGATE ||
      (h.avg_mode != SEDIMI_AVG_PLAIN && !c->prm.nn_enable) || h.check_blocks < 0 ||
      h.step < 0 || h.adam_t < 0 || (h.nn_groups != 1 && h.nn_groups != 4))
    return fail(c, SEDIMI_EINVAL, "state blob out of range");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->ws, (const char*)buf + sizeof(h), c->ws_bytes, hipMemcpyHostToDevice));
  layout(c, c->ws, &c->A);
  if (h.swapped & 1u) std::swap(c->A.vel, c->A.vel_t);
  if (h.swapped & 2u) std::swap(c->A.omg, c->A.omg_t);
  if (h.swapped & 4u) std::swap(c->A.pos, c->A.pos_t);
  if (h.swapped & 8u) std::swap(c->A.rb, c->A.rb_next);
  c->n = h.n;
  c->P.n = (int)h.n;
  c->step = h.step, c->adam_t = h.adam_t;
  c->nn_calls = h.nn_calls, c->nn_fallbacks = h.nn_fallbacks, c->last_iters = h.last_iters;
  c->nn_last_check = h.nn_last_check, c->last_residual = h.last_residual;
  c->avg_mode = h.avg_mode, c->have_particles = h.have_particles != 0;
  c->last_direct = h.last_direct != 0, c->check_blocks = h.check_blocks;
  c->nn_groups = h.nn_groups;
  c->norm = h.norm;
  return SEDIMI_OK;
}

int sedimi_get_stats(sedimi_ctx* c, sedimi_stats* out) {
  int rc = need_ws(c);
  if (rc) return rc;
  if (!out) return fail(c, SEDIMI_EINVAL, "null stats");
  Ctl ctl;
  if ((rc = read_ctl(c, &ctl))) return rc;
  out->steps = c->step;
  out->rebuilds = ctl.rebuilds;
  out->max_neighbors = ctl.max_nbr;
  out->flags = ctl.flags;
  out->solve_iters = c->last_iters;
  out->solve_residual = c->last_residual;
  out->mean_neighbors = 0.0;
  out->mean_contacts = 0.0;
  out->nn_calls = c->nn_calls;
  out->nn_fallbacks = c->nn_fallbacks;
  out->nn_last_check = c->nn_last_check;
  out->nn_check_trunc = c->prm.nn_enable ? c->green.trunc : 0.0;
  out->nn_check_window[0] = c->green.rx;
  out->nn_check_window[1] = c->green.ry;
  out->nn_check_window[2] = c->green.rz;
  out->nn_check_columns = c->green_cols;
  out->graph_steps = c->graph_steps;
  out->particles = c->n;
  if (c->have_particles && c->n > 0) {
    const size_t n = (size_t)c->n;
    std::vector<int> cnt;
    std::vector<unsigned> mask;
    std::vector<double4> wxi;
    if ((rc = download(c, cnt, c->A.ncnt, n))) return rc;
    if ((rc = download(c, mask, c->A.hmask, n))) return rc;
    if ((rc = download(c, wxi, c->A.wxi, 2 * n))) return rc;
    double sn = 0.0, sc = 0.0;
    for (size_t q = 0; q < n; ++q) {
      sn += cnt[q];
      sc += __builtin_popcount(mask[q]);  // list slots and the two wall bits
    }
    out->mean_neighbors = sn / n;
    out->mean_contacts = sc / n;
  }
  return SEDIMI_OK;
}

int sedimi_set_profiling(sedimi_ctx* c, int on) {
  if (!c) return SEDIMI_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& m : c->marks) c->pool.push_back(m.a), c->pool.push_back(m.b);
  c->marks.clear();
  for (int k = 0; k < SEDIMI_NPHASES; ++k) c->prof_ms[k] = 0.0, c->prof_count[k] = 0;
  c->prof = on != 0;
  return SEDIMI_OK;
}

int sedimi_get_profile(sedimi_ctx* c, sedimi_profile* out) {
  if (!c || !out) return SEDIMI_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& m : c->marks) {
    float ms = 0.0f;
    if (m.a && m.b && hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
      c->prof_ms[m.phase] += ms;
      c->prof_count[m.phase] += 1;
    }
    c->pool.push_back(m.a);
    c->pool.push_back(m.b);
  }
  c->marks.clear();
  for (int k = 0; k < SEDIMI_NPHASES; ++k) out->ms[k] = c->prof_ms[k], out->count[k] = c->prof_count[k];
  return SEDIMI_OK;
}

}  // extern "C"

namespace {

ConvGeom geom(const sedimi_ctx* c, int layer, int neg) {
  ConvGeom g;
  g.nx = c->P.nx, g.ny = c->P.ny, g.nz = c->P.nz, g.ncell = c->P.ncell;
  g.dil = kNNDil[layer];
  g.neg = neg;
  return g;
}

void nn_pack_all(sedimi_ctx* c) {
  for (int l = 0; l < 6; ++l)
    launch_pack(c->nn.w + nn_woff(l), nn_cin(l), nn_cout(l), c->nn.fwd[l], c->nn.adj[l],
                c->stream);
}

// Zero the cross-group entries of a parameter-shaped array (weights, their
// gradient or Adam moments); biases are per channel and stay.
void nn_mask_groups(sedimi_ctx* c, float* a) {
  for (int l = 0; l < 6; ++l) launch_group_mask(a + nn_woff(l), nn_cin(l), nn_cout(l), c->stream);
}

// Network forward on the RAW field into nn.y and the SMOOTH field.  keep:
// store the pre-activations needed by the backward pass.
void nn_run_forward(sedimi_ctx* c, bool keep) {
  NNBufs& b = c->nn;
  const int n = c->P.ncell;
  launch_nn_prep(n, c->A.raw, c->norm, b.xf, b.xb, c->stream);
  launch_split(c->P.nx, c->P.ny, c->P.nz, std::max(1, c->prm.avg_ntau), c->split, b.xf, b.xt,
               b.xs, c->stream);
  launch_nn_highpass(n, b.xf, b.xs, b.xb, c->stream);
  const float alpha = (float)c->prm.nn_alpha;
  for (int l = 0; l < 5; ++l) {
    EpiArgs e{};
    e.alpha = alpha;
    e.zout = keep ? b.z[l] : nullptr;
    e.hout = b.h[l];
    e.hin = l == 0 ? nullptr : b.h[l - 1];
    const float* bias = b.w + nn_woff(l) + 27LL * nn_cin(l) * nn_cout(l);
    launch_conv(nn_cin(l), nn_cout(l), l == 0 ? EPI_FIRST : EPI_RES, geom(c, l, 0),
                l == 0 ? b.xb : b.h[l - 1], b.fwd[l], bias, e, c->stream);
  }
  EpiArgs e{};
  e.alpha = alpha;
  e.xres = b.xs;
  e.yout = b.y;
  launch_conv(kNNC, 4, EPI_LAST, geom(c, 5, 0), b.h[4], b.fwd[5],
              b.w + nn_woff(5) + 27LL * kNNC * 4, e, c->stream);
  launch_nn_out(n, b.y, c->norm, c->A.smooth, c->stream);
}

int nn_check_smooth(sedimi_ctx* c, double rel[4]) {
  const GreenWindow& gw = c->green;
  int nb = launch_green_check(c->P, c->A.raw, c->A.smooth, c->nn.cols, c->green_cols,
                              c->nn.gtab, gw.rx, gw.ry, gw.rz, c->nn.gpart, c->stream);
  if (nb <= 0 || read_partials(c->nn.gpart, nb, 4, rel, c->stream) != 0)
    return fail(c, SEDIMI_EDEVICE, "reading the network check failed");
  return SEDIMI_OK;
}

int need_nn(sedimi_ctx* c) {
  int rc = need_ws(c);
  if (rc) return rc;
  if (!c->prm.nn_enable) return fail(c, SEDIMI_ESTATE, "context created without nn_enable");
  return SEDIMI_OK;
}


}  // namespace

extern "C" {

int sedimi_set_avg_mode(sedimi_ctx* c, int mode) {
  if (!c) return SEDIMI_EINVAL;
  if (mode < SEDIMI_AVG_PLAIN || mode > SEDIMI_AVG_SURROGATE)
    return fail(c, SEDIMI_EINVAL, "unknown averaging mode");
  if (mode != SEDIMI_AVG_PLAIN && !c->prm.nn_enable)
    return fail(c, SEDIMI_ESTATE, "surrogate modes need nn_enable");
  c->avg_mode = mode;
  return SEDIMI_OK;
}

int sedimi_nn_param_count(const sedimi_ctx* c, int64_t* n) {
  if (!c || !n) return SEDIMI_EINVAL;
  *n = nn_count();
  return SEDIMI_OK;
}

int sedimi_nn_init(sedimi_ctx* c, uint64_t seed) {
  int rc = need_nn(c);
  if (rc) return rc;
  const int64_t P = nn_count();
  std::vector<float> w((size_t)P, 0.0f);
  uint64_t s = seed;
  // Variance-preserving scale for a leaky ReLU of slope alpha (2 / (1 + alpha^2)
  // over the fan-in: 1 / fan-in for the linear network), and the four
  // residual branches at 1/sqrt(4) of it so that the residual stream's
  // variance stays within a small factor of the first layer's instead of
  // growing with depth.  The last layer starts at zero: output = skip.
  // With 4 channel groups a hidden channel's fan-in is its own group's share.
  const double a = c->prm.nn_alpha;
  for (int l = 0; l < 5; ++l) {
    const double fan = 27.0 * nn_cin(l) / c->nn_groups;
    const double sd = sqrt(2.0 / ((1.0 + a * a) * fan)) * (l >= 1 ? 0.5 : 1.0);
    const int64_t nw = 27LL * nn_cin(l) * nn_cout(l);
    for (int64_t k = 0; k < nw; k += 2) {
      double u1 = ((mix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
      double u2 = ((mix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
      double r = sqrt(-2.0 * log(u1));
      w[(size_t)(nn_woff(l) + k)] = (float)(sd * r * cos(2.0 * kPi * u2));
      if (k + 1 < nw) w[(size_t)(nn_woff(l) + k + 1)] = (float)(sd * r * sin(2.0 * kPi * u2));
    }
  }
  return sedimi_nn_set_params(c, w.data(), P);
}

int sedimi_nn_set_params(sedimi_ctx* c, const float* p, int64_t n) {
  int rc = need_nn(c);
  if (rc) return rc;
  const int64_t P = nn_count();
  if (!p || n != P) return fail(c, SEDIMI_EINVAL, "parameter vector has the wrong length");
  HIPCHK(c, hipMemcpyAsync(c->nn.w, p, sizeof(float) * P, hipMemcpyHostToDevice, c->stream));
  if (c->nn_groups == 4) nn_mask_groups(c, c->nn.w);
  HIPCHK(c, hipMemsetAsync(c->nn.m, 0, sizeof(float) * P, c->stream));
  HIPCHK(c, hipMemsetAsync(c->nn.v, 0, sizeof(float) * P, c->stream));
  for (int l = 0; l < 6; ++l) {
    HIPCHK(c, hipMemsetAsync(c->nn.fwd[l], 0, sizeof(__bf16) * nn_packed_elems(nn_cin(l), nn_cout(l)), c->stream));
    if (l > 0)
      HIPCHK(c, hipMemsetAsync(c->nn.adj[l], 0, sizeof(__bf16) * nn_packed_elems(nn_cout(l), nn_cin(l)), c->stream));
  }
  c->adam_t = 0;
  nn_pack_all(c);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int sedimi_nn_get_params(sedimi_ctx* c, float* p, int64_t n) {
  int rc = need_nn(c);
  if (rc) return rc;
  if (!p || n != nn_count()) return fail(c, SEDIMI_EINVAL, "parameter vector has the wrong length");
  HIPCHK(c, hipMemcpyAsync(p, c->nn.w, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

struct NNSaveHeader {
  char magic[8];
  int64_t count, adam_t, groups;
  double alpha;
  double mean[4], std[4], lw[4];
};
constexpr char kNNMagic[8] = {'S', 'E', 'D', 'I', 'N', 'N', '0', '2'};

int sedimi_nn_save(sedimi_ctx* c, void* buf, size_t cap, size_t* size_out) {
  int rc = need_nn(c);
  if (rc) return rc;
  const int64_t P = nn_count();
  const size_t total = sizeof(NNSaveHeader) + 3 * sizeof(float) * (size_t)P;
  if (size_out) *size_out = total;
  if (!buf) return SEDIMI_OK;
  if (cap < total) return fail(c, SEDIMI_ENOMEM, "network blob buffer too small");
  NNSaveHeader h;
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, kNNMagic, sizeof(h.magic));
  h.count = P, h.adam_t = c->adam_t, h.groups = c->nn_groups, h.alpha = c->prm.nn_alpha;
  for (int k = 0; k < 4; ++k)
    h.mean[k] = c->norm.mean[k], h.std[k] = c->norm.std[k], h.lw[k] = c->norm.lw[k];
  memcpy(buf, &h, sizeof(h));
  float* body = reinterpret_cast<float*>(static_cast<char*>(buf) + sizeof(h));
  const float* src[3] = {c->nn.w, c->nn.m, c->nn.v};
  for (int a = 0; a < 3; ++a)
    HIPCHK(c, hipMemcpyAsync(body + (size_t)a * P, src[a], sizeof(float) * P,
                             hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int sedimi_nn_load(sedimi_ctx* c, const void* buf, size_t size) {
  int rc = need_nn(c);
  if (rc) return rc;
  const int64_t P = nn_count();
  NNSaveHeader h;
  if (!buf || size < sizeof(h)) return fail(c, SEDIMI_EINVAL, "network blob too short");
  memcpy(&h, buf, sizeof(h));
  if (memcmp(h.magic, kNNMagic, sizeof(h.magic)) != 0 || h.count != P ||
      size != sizeof(h) + 3 * sizeof(float) * (size_t)P || h.adam_t < 0 ||
      (h.groups != 1 && h.groups != 4))
    return fail(c, SEDIMI_EINVAL, "not a network blob of this architecture");
  if (h.alpha != c->prm.nn_alpha)
    return fail(c, SEDIMI_EINVAL, "network blob trained with another leaky-ReLU slope");
  for (int k = 0; k < 4; ++k)
    if (!(h.std[k] != 0 && std::isfinite(h.std[k])) || !std::isfinite(h.mean[k]) || !(h.lw[k] >= 0))
      return fail(c, SEDIMI_EINVAL, "network blob with an invalid standardisation");
  const float* body = reinterpret_cast<const float*>(static_cast<const char*>(buf) + sizeof(h));
  c->nn_groups = (int)h.groups;
  rc = sedimi_nn_set_params(c, body, P);  // parameters, packed copies; zeroes the moments
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->nn.m, body + (size_t)P, sizeof(float) * P, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(c->nn.v, body + 2 * (size_t)P, sizeof(float) * P,
                           hipMemcpyHostToDevice, c->stream));
  c->adam_t = h.adam_t;
  for (int k = 0; k < 4; ++k)
    c->norm.mean[k] = h.mean[k], c->norm.std[k] = h.std[k], c->norm.lw[k] = h.lw[k];
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int sedimi_nn_get_grads(sedimi_ctx* c, float* g, int64_t n) {
  int rc = need_nn(c);
  if (rc) return rc;
  if (!g || n != nn_count()) return fail(c, SEDIMI_EINVAL, "gradient vector has the wrong length");
  HIPCHK(c, hipMemcpyAsync(g, c->nn.g, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int sedimi_nn_set_norm(sedimi_ctx* c, const double* mean4, const double* std4) {
  int rc = need_nn(c);
  if (rc) return rc;
  if (!mean4 || !std4) return fail(c, SEDIMI_EINVAL, "null normalisation");
  for (int k = 0; k < 4; ++k) {
    if (!(std4[k] != 0 && std::isfinite(std4[k]) && std::isfinite(mean4[k])))
      return fail(c, SEDIMI_EINVAL, "std must be finite and nonzero, mean finite");
    c->norm.mean[k] = mean4[k];
    c->norm.std[k] = std4[k];
  }
  return SEDIMI_OK;
}

int sedimi_nn_set_groups(sedimi_ctx* c, int groups) {
  int rc = need_nn(c);
  if (rc) return rc;
  if (groups != 1 && groups != 4) return fail(c, SEDIMI_EINVAL, "channel groups must be 1 or 4");
  c->nn_groups = groups;
  if (groups == 4) {
    nn_mask_groups(c, c->nn.w);
    nn_mask_groups(c, c->nn.m);
    nn_mask_groups(c, c->nn.v);
    nn_pack_all(c);
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int sedimi_nn_set_loss_weights(sedimi_ctx* c, const double* w4) {
  int rc = need_nn(c);
  if (rc) return rc;
  if (!w4) return fail(c, SEDIMI_EINVAL, "null loss weights");
  for (int k = 0; k < 4; ++k)
    if (!(w4[k] >= 0 && std::isfinite(w4[k]))) return fail(c, SEDIMI_EINVAL, "loss weights must be finite and >= 0");
  for (int k = 0; k < 4; ++k) c->norm.lw[k] = w4[k];
  return SEDIMI_OK;
}

int sedimi_nn_forward(sedimi_ctx* c) {
  int rc = need_nn(c);
  if (rc) return rc;
  phase_begin(c, 4);
  nn_run_forward(c, false);
  launch_pack_eps(c->P, c->A, c->stream);
  phase_end(c);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SEDIMI_OK;
}

int sedimi_nn_train_step(sedimi_ctx* c, double lr, double* loss) {
  int rc = need_nn(c);
  if (rc) return rc;
  if (!(lr >= 0)) return fail(c, SEDIMI_EINVAL, "learning rate must be >= 0");
  NNBufs& b = c->nn;
  const int n = c->P.ncell;
  const float alpha = (float)c->prm.nn_alpha;
  phase_begin(c, 5);
  // forward keeping activations; the network output goes to nn.y only (the
  // SMOOTH field holds the target and is not touched)
  launch_nn_prep(n, c->A.raw, c->norm, b.xf, b.xb, c->stream);
  launch_split(c->P.nx, c->P.ny, c->P.nz, std::max(1, c->prm.avg_ntau), c->split, b.xf, b.xt,
               b.xs, c->stream);
  launch_nn_highpass(n, b.xf, b.xs, b.xb, c->stream);
  for (int l = 0; l < 5; ++l) {
    EpiArgs e{};
    e.alpha = alpha;
    e.zout = b.z[l];
    e.hout = b.h[l];
    e.hin = l == 0 ? nullptr : b.h[l - 1];
    launch_conv(nn_cin(l), nn_cout(l), l == 0 ? EPI_FIRST : EPI_RES, geom(c, l, 0),
                l == 0 ? b.xb : b.h[l - 1], b.fwd[l],
                b.w + nn_woff(l) + 27LL * nn_cin(l) * nn_cout(l), e, c->stream);
  }
  {
    EpiArgs e{};
    e.alpha = alpha;
    e.xres = b.xs;
    e.yout = b.y;
    launch_conv(kNNC, 4, EPI_LAST, geom(c, 5, 0), b.h[4], b.fwd[5],
                b.w + nn_woff(5) + 27LL * kNNC * 4, e, c->stream);
  }
  unsigned nlb = launch_nn_loss(n, b.y, c->A.smooth, c->norm, b.dy6, c->A.red, c->stream);
  const int dwb = std::max(1, std::min(kDwBlocks, (n + 31) / 32));
  // layer 6
  launch_conv_dw(kNNC, 4, geom(c, 5, 0), b.h[4], b.dy6, b.part, b.part_b, b.g + nn_woff(5),
                 b.g + nn_woff(5) + 27LL * kNNC * 4, dwb, c->stream);
  {
    EpiArgs e{};
    e.alpha = alpha;
    e.zin = b.z[4];
    e.hout = b.dh[4];
    e.zout = b.dz[4];
    launch_conv(4, kNNC, EPI_BWD, geom(c, 5, 1), b.dy6, b.adj[5], nullptr, e, c->stream);
  }
  for (int l = 4; l >= 1; --l) {
    launch_conv_dw(kNNC, kNNC, geom(c, l, 0), b.h[l - 1], b.dz[l], b.part, b.part_b,
                   b.g + nn_woff(l), b.g + nn_woff(l) + 27LL * kNNC * kNNC, dwb, c->stream);
    EpiArgs e{};
    e.alpha = alpha;
    e.hin = b.dh[l];
    e.zin = b.z[l - 1];
    e.hout = b.dh[l - 1];
    e.zout = b.dz[l - 1];
    launch_conv(kNNC, kNNC, EPI_BWD, geom(c, l, 1), b.dz[l], b.adj[l], nullptr, e, c->stream);
  }
  launch_conv_dw(4, kNNC, geom(c, 0, 0), b.xb, b.dz[0], b.part, b.part_b, b.g + nn_woff(0),
                 b.g + nn_woff(0) + 27LL * 4 * kNNC, dwb, c->stream);
  const int64_t P = nn_count();
  if (c->nn_groups == 4) nn_mask_groups(c, b.g);
  c->adam_t += 1;
  launch_adam(P, b.w, b.m, b.v, b.g, (float)lr, 0.9f, 0.999f, 1e-8f, c->adam_t, c->stream);
  nn_pack_all(c);
  phase_end(c);
  HIPCHK(c, hipGetLastError());
  if (loss) {
    std::vector<double> h(nlb);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->A.red, sizeof(double) * nlb, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double sum = 0.0;
    for (unsigned k = 0; k < nlb; ++k) sum += h[k];
    *loss = sum / (4.0 * n);
  } else {
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return SEDIMI_OK;
}

int sedimi_nn_get_tensor(sedimi_ctx* c, int which, int layer, float* out, int64_t n) {
  int rc = need_nn(c);
  if (rc) return rc;
  const NNBufs& b = c->nn;
  const int64_t nc = c->P.ncell;
  const bool layered = which == SEDIMI_NN_Z || which == SEDIMI_NN_H || which == SEDIMI_NN_DH ||
                       which == SEDIMI_NN_DZ;
  if (which < SEDIMI_NN_X || which > SEDIMI_NN_DZ || (layered && (layer < 0 || layer > 4)) || !out)
    return fail(c, SEDIMI_EINVAL, "bad network tensor");
  const int64_t want = (layered ? kNNC : 4) * nc;
  if (n != want) return fail(c, SEDIMI_EINVAL, "network tensor has the wrong length");
  const float* f32 = which == SEDIMI_NN_X ? b.xf : which == SEDIMI_NN_SX ? b.xs
                     : which == SEDIMI_NN_Y ? b.y : nullptr;
  if (f32) {
    HIPCHK(c, hipMemcpyAsync(out, f32, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SEDIMI_OK;
  }
  const __bf16* h16 = which == SEDIMI_NN_XB ? b.xb : which == SEDIMI_NN_DY ? b.dy6
                      : which == SEDIMI_NN_Z ? b.z[layer] : which == SEDIMI_NN_H ? b.h[layer]
                      : which == SEDIMI_NN_DH ? b.dh[layer] : b.dz[layer];
  std::vector<uint16_t> h((size_t)n);
  HIPCHK(c, hipMemcpyAsync(h.data(), h16, sizeof(uint16_t) * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int64_t q = 0; q < n; ++q) {
    const uint32_t u = (uint32_t)h[q] << 16;  // a BF16 is the upper half of an FP32
    memcpy(out + q, &u, 4);
  }
  return SEDIMI_OK;
}

int sedimi_nn_check(sedimi_ctx* c, double* rel4) {
  int rc = need_nn(c);
  if (rc) return rc;
  if (!rel4) return fail(c, SEDIMI_EINVAL, "null output");
  return nn_check_smooth(c, rel4);
}

}  // extern "C"

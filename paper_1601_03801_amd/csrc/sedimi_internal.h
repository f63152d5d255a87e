// sedimi_internal.h -- device data layout and kernel launchers of libsedimi.
//
// Device layout (all in the caller's workspace, 256-byte aligned arrays):
//   particles, kept sorted by neighbour bin (x, then y, then z bin; IDs
//   ascending inside a bin) so that neighbours are near in memory:
//     pos   double4 (x, y, z, r)          vel double4 (vx, vy, vz, m)
//     omg   double4 (wx, wy, wz, -)       acc double4 (a^n), alp double4 (alpha^n)
//     fdr   double4 (drag of the last evaluation)
//     id    int32 original particle ID
//     xb    double4 positions at the last neighbour-list build
//     wxi   double4 [2][N] wall history (bottom, top); .w = 1 when active
//   neighbour list (full: each pair appears on both sides), slot-major so that
//   slot k of consecutive particles is contiguous:
//     nbr   int32 [maxn][N], ncnt int32 [N]
//     hmask uint32 [N]   bit k set = slot k carries tangential history;
//                        bits 30 / 31: bottom / top wall history active
//     hxi   3 x [maxn][N] history of slot k (double, or float in mixed mode),
//           oriented from the lower to the higher particle ID
//   compact history (partner ID + xi per contact) used across a re-sort:
//     cid int32 [maxc][N], cxi 3 x [maxc][N] double, ccnt int32 [N]
//   mesh: U, gp, du double4 [ncell]; raw, smooth 4 x [ncell] double; solver
//   vectors; sort scratch; a control block of flags and counters.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/sedimi.h"

namespace sedimi {

constexpr int kBlock = 256;
// smoothed solid fraction below which the solid velocity is set to 0
constexpr double kSolidEpsMin = 1e-9;
constexpr int kMaxContacts = 16;  // contacts per particle kept across a re-sort
// Members a neighbour bin / a mesh cell may hold: each is ordered by one
// thread (insertion sort), so a state that crowds many particles into one
// (a non-finite or runaway position is clamped into the grid) would otherwise
// cost that thread quadratic time.  Above the limit the bin or cell raises
// kFlagCrowded instead; physical packings stay far below it.
constexpr int kMaxBinMembers = 1024;
constexpr int kMaxCellMembers = 4096;
// Ctl::flags bits
constexpr int kFlagOverflow = 1;   // neighbour or contact slots exceeded
constexpr int kFlagLost = 2;       // a contact fell out of the neighbour list
constexpr int kFlagEscape = 4;     // a particle left [0, Lz]
constexpr int kFlagNonFinite = 8;  // non-finite position or velocity
constexpr int kFlagCrowded = 16;   // a bin or mesh cell above its member limit

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2).
// Renumber them so that every XCD works through one contiguous range of
// particles; launch grids rounded up to a multiple of 8.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nblocks8) {
  return (b % kXcds) * (nblocks8 / kXcds) + b / kXcds;
}
inline unsigned xcd_grid(int64_t nblocks) {
  return (unsigned)((nblocks + kXcds - 1) / kXcds * kXcds);
}

// Flags and counters living in device memory.
// rebuild / rebuild_alt are the two rebuild flags: DevArrays::rb points at
// the one of the current step, rb_next at the other.
struct Ctl {
  int rebuild;
  int flags;        // kFlag* bits
  int max_nbr;      // largest neighbour count at a build
  int rebuild_alt;
  long long rebuilds;
  int scan_done;    // tiles of the bin scan finished so far (0 between scans)
  int pad0;
  long long pad1[4];
};

// Offsets into DevArrays::zgeo for a mesh of nz planes.
__host__ __device__ inline size_t zgeo_faces(int) { return 0; }
__host__ __device__ inline size_t zgeo_centres(int nz) { return (size_t)nz + 1; }
__host__ __device__ inline size_t zgeo_volumes(int nz) { return 2 * (size_t)nz + 1; }
__host__ __device__ inline size_t zgeo_coupling(int nz) { return 3 * (size_t)nz + 1; }
__host__ __device__ inline size_t zgeo_doubles(int nz) { return 5 * (size_t)nz + 1; }

// Parameters copied by value into the kernels.
struct DevParams {
  double Lx, Ly, Lz, hLx, hLy;
  int nx, ny, nz, ncell;
  double hx, hy, hz, Vc;
  double kn, zeta, kt, gt_over_gn, mu;
  double lub_out, lub_in;
  double rho_f, mu_f, c_add;
  double gx, gy, gz, dt;
  int drag_law, lubrication, fluid_forces, bottom_wall, top_wall;
  double eps_s_max;
  double kz_diff;  // diffusivity of the averaging along z (1: isotropic)
  // z mesh: graded (geometric cell heights towards the bottom wall) or
  // uniform.  zlam bounds the eigenvalues of -L_z (z diffusivity included);
  // zskew = sqrt(largest / smallest cell height) (1 on a uniform mesh).
  double zlam, zskew;
  int graded, graded_pad;
  double lift_c;   // C_l rho_f nu^(1/2) of the shear lift (0: no lift)
  int nch_avg;     // averaged channels: 4, or 7 with the solid volume flux
  // neighbour bins
  int nbx, nby, nbz, nbins;
  double hbx, hby, hbz;
  double skin, half_skin2;
  int maxn, n;
};

// Device pointers of one context.
struct DevArrays {
  double4 *pos, *vel, *omg, *acc, *alp, *fdr, *xb, *wxi;  // primary
  double4 *pos_t, *vel_t, *omg_t, *acc_t, *alp_t, *fdr_t, *wxi_t;  // second buffers
  int *id, *id_t;
  int* nbr;
  int* ncnt;
  unsigned* hmask;
  void* hxi;  // 3 x [maxn][N] of double (FP64) or float (mixed)
  int* cid;
  double* cxi;
  int* ccnt;
  // force breakdown (diagnostic evaluation): 8 x double4 [N], SEDIMI_F_* order (lift last)
  double4* comp;
  // sort scratch
  int *key, *rank, *perm, *bin_count, *bin_start, *scan_tmp;
  int* bin_rank;  // Morton rank of each bin (bins are stored in this order)
  // mesh
  double4 *U, *gp, *du;  // U.w = averaged solid fraction
  double4* G;            // -grad p + C_add rho_f DU/Dt (step kernel)
  double4* W;            // curl U_f at cell centres (only with the lift)
  // z geometry (ZGEO_* offsets): faces [nz + 1], centres [nz], cell volumes
  // [nz], and per plane the z coupling of the diffusion operator to the plane
  // above and below ([nz][2], z diffusivity included, zero at the walls)
  double* zgeo;
  double *raw, *smooth, *sx, *sr, *sd0, *sd1;  // [nch_avg][ncell] each
  double* us;  // solid velocity [3][ncell] (only with the solid flux)
  double *sxf, *stmp;  // solver: FP32 iterate (mixed mode), column-sweep scratch
  double* ztab;        // z-line preconditioner: reciprocal pivots, super-diagonal, for
                       // dtau and (BDF2) for 2/3 dtau
  double* sprev;       // BDF2 iterative solve: the previous pseudo-time step
  double* spec;        // direct solve: H_x, H_y, C_z, C_z^-1, per-axis eigenvalues
  int *cell_count, *cell_start;
  unsigned long long* cperm;  // deposition: (particle ID << 32 | sorted index), by cell
  double* red;  // reduction partials
  Ctl* ctl;
  // Rebuild flags.  *rb: a rebuild is due before this step's forces (set by
  // the drift, read by every rebuild kernel, cleared by the force kernel).  A
  // force kernel that also drifts to the next step sets *rb_next instead; the
  // host then swaps the two pointers.
  int* rb;
  int* rb_next;
};

// ---- launchers (k_neighbors.hip) ----
void launch_zero_ints(int* p, int64_t n, bool gated, const int* flag, hipStream_t s);
void launch_kick_drift(const DevParams& P, DevArrays& A, hipStream_t s);
void launch_rebuild(const DevParams& P, DevArrays& A, bool from_slots, bool mixed,
                    hipStream_t s);
void launch_pairmask(const DevParams& P, DevArrays& A, unsigned* out, hipStream_t s);
void launch_translate(const DevParams& P, DevArrays& A, double dx, double dy, hipStream_t s);
void launch_exclusive_scan(int* in_out_count, int* start, int n, int* tmp, bool gated,
                           const int* flag, hipStream_t s);

// ---- launchers (k_forces.hip) ----
// mode: 0 = step (second half kick, writes vel_t/omg_t), 1 = evaluation with
// breakdown (writes comp, acc, alp), 2 = step fused with the first half kick
// and drift of the next step (writes pos_t/vel_t/omg_t/acc, sets *rb_next);
// update_history as in sedimi_compute_forces.
void launch_forces(const DevParams& P, DevArrays& A, int mode, bool update_history,
                   bool mixed, hipStream_t s);
// Copy channel 0 of the smoothed field (solid fraction) into U.w.
void launch_pack_eps(const DevParams& P, DevArrays& A, hipStream_t s);

// ---- launchers (k_average.hip) ----
void launch_deposit(const DevParams& P, DevArrays& A, hipStream_t s);
// Enqueue the smoothing of channels [0, nch) of raw into smooth (backward
// Euler, or BDF2 with A.sprev holding the previous step); returns the total
// number of solver iterations.  Each pseudo-time step's final residual
// partials are left in A.red for read_smooth_residual.
int64_t launch_smooth(const DevParams& P, DevArrays& A, int nch, int ntau, double tau,
                      double rtol, bool mixed, bool bdf2, hipStream_t s);
// Largest relative residual over channels and pseudo-time steps of the last
// launch_smooth (synchronises the stream); negative on a HIP error.
double read_smooth_residual(const DevParams& P, DevArrays& A, int nch, int ntau,
                            hipStream_t s);
size_t smooth_red_doubles(int ncell, int nch, int ntau);
// Thomas-algorithm table of the z-line preconditioner (2 * nz doubles).
// zcoup: the host copy of the z coupling table (graded meshes; may be null
// on a uniform mesh).
void smooth_ztab(const DevParams& P, const double* zcoup, int ntau, double tau,
                 double* host_tab);
// Residual check of a smoothed field y (nch channels) against raw on a seeded
// sample of cells (fraction frac): r = A^ntau y - raw.  Enqueues the work
// (partials in A.red, A.sd0/A.sd1 as scratch) and returns the block count;
// read_check then gives |r|/|y| per channel over the sample (synchronises).
int launch_check(const DevParams& P, DevArrays& A, const double* y, int nch, int ntau,
                 double tau, uint64_t seed, double frac, hipStream_t s);
int read_check(DevArrays& A, int nblocks, int nch, double* rel, hipStream_t s);
// The same from per-block partials part[b][2 nch] of any check kernel.
int read_partials(const double* part, int nblocks, int nch, double* rel, hipStream_t s);
// A^ntau y (A = I - dtau L_h) for channels [0, nch) into A.sd0 / A.sd1;
// returns the buffer holding it (y itself when ntau = 0).
const double* apply_An(const DevParams& P, DevArrays& A, const double* y, int nch, int ntau,
                       double tau, hipStream_t s);
// Error estimate of a smoothed 4-channel field y on whole sampled z-columns
// (cols: x + nx y): the plain solution there is taken as the Green's function
// of the ntau implicit steps (gtab [2ry+1][2rx+1][2rz+1], rx, ry <= 4,
// rz <= 32) applied to raw, with periodic x, y and mirror images about the
// walls.  Per-column partials part[col][8] = sum (y - G*raw)^2, sum (G*raw)^2
// per channel, in read_check's layout; returns the block count.
int launch_green_check(const DevParams& P, const double* raw, const double* y, const int* cols,
                       int ncols, const double* gtab, int rx, int ry, int rz, double* part,
                       hipStream_t s);
// The same check for BDF2 steps: y = g_N(M) raw with M = -dtau L and the
// per-mode BDF2 factor g_N = p_N / q_N, q_N = (1 + M)(3 + 2M)^(N-1),
// p_1 = 1, p_2 = 3 - M, p_{n+1} = 4 p_n - (3 + 2M) p_{n-1}; the residual is
// r = q_N(M) y - p_N(M) raw, from stencil products only (A.sx, A.sr, A.stmp,
// A.sd0, A.sd1 as scratch).
int launch_check_bdf2(const DevParams& P, DevArrays& A, int nch, int ntau, double tau,
                      hipStream_t s);
// U_s = smoothed flux / smoothed solid fraction (channels 4..6 over 0) into A.us.
void launch_solid_velocity(const DevParams& P, DevArrays& A, hipStream_t s);

// ---- launchers (k_spectral.hip) ----
// Direct solve of all N_tau implicit steps on the uniform mesh: channels
// [0, nch) of raw into smooth (A.sr and A.stmp as scratch).
void launch_spectral(const DevParams& P, DevArrays& A, int nch, int ntau, double tau,
                     bool bdf2, hipStream_t s);
size_t spectral_table_doubles(const DevParams& P);
// zdiag: on a graded mesh the z transform of graded_z_transform (null on a
// uniform mesh, which uses the DCT-II).
void spectral_tables(const DevParams& P, const double* zdiag, double* host_tab);
// The z transform that diagonalises -L_z on a graded mesh (zgeo: the z
// geometry in the zgeo_* layout): out = forward [nz][nz], inverse [nz][nz],
// eigenvalues [nz].  Returns 0, or -1 if the eigen-decomposition did not
// converge or its result fails the orthogonality check.
int graded_z_transform(int nz, const double* zgeo, double* out);
// The same solve of a caller's device field without a workspace: tables and
// the intermediate field in the library's static device scratch (see
// sedimi_smooth_static).  Enqueue only; SEDIMI_OK or an error code with *err.
size_t spectral_static_bytes(int nx, int ny, int nz, int nch);
int spectral_static(int nx, int ny, int nz, double hx, double hy, double hz, double kz_diff,
                    int nch, int ntau, double tau, bool bdf2, const double* raw, double* out,
                    hipStream_t s, std::string* err);

}  // namespace sedimi

/*
 * sedimi.h -- C ABI of the MI355X (gfx950) CFD-DEM particle step and
 * particle-to-mesh diffusion averaging of SediFoam (Sun & Xiao).
 *
 * The calls follow the paper's statement of the problem: particles with
 * diameter, density, position, velocity and angular velocity evolve under
 * Newton's equations (Eq. 1a-1b) with contact, lubrication and fluid-particle
 * forces (Sections 2.1, 2.3, 2.5); the fluid is given on an Eulerian mesh
 * (Section 2.2; frozen here: velocity, pressure gradient and material
 * derivative per cell); the particles' volume, drag and (optionally) volume
 * flux are averaged back onto the mesh by deposition (Eq. 11) and implicit
 * diffusion (Eq. 12).
 *
 * Conventions (SI units throughout):
 *   - axes: x streamwise and y spanwise, both periodic on [0, L); z
 *     wall-normal, with optional flat walls at z = 0 and z = Lz;
 *   - host particle arrays are in particle-ID order (ID = row index at
 *     sedimi_set_particles), vectors [n][3] row-major, scalars [n];
 *   - mesh cell (i, j, k) has index (k*ny + j)*nx + i; vector fields are
 *     [ncell][3], averaged fields are [4][ncell] (channel 0 = solid volume
 *     fraction, channels 1..3 = drag force density on the particles), or
 *     [7][ncell] with avg_solid_velocity (channels 4..6 = solid volume flux);
 *   - host arrays passed in are copied, never retained; host arrays passed
 *     out are filled before the call returns (those calls synchronise the
 *     bound stream);
 *   - all device memory lives in one caller-provided workspace (see
 *     sedimi_workspace_bytes / sedimi_bind_workspace); the library never
 *     allocates device memory itself;
 *   - device work is enqueued on the bound HIP stream (default: the null
 *     stream); a context is not thread-safe;
 *   - every call returns SEDIMI_OK (0) or a negative SEDIMI_E* code and never
 *     aborts; sedimi_last_error() gives a message for the last failure.
 */
#ifndef SEDIMI_H
#define SEDIMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define SEDIMI_OK 0
#define SEDIMI_EINVAL (-1)    /* bad argument or parameter */
#define SEDIMI_ENOMEM (-2)    /* workspace missing or too small, or host allocation failed */
#define SEDIMI_EDEVICE (-3)   /* a HIP runtime call failed */
#define SEDIMI_EOVERFLOW (-4) /* neighbour slots exceeded, a contact fell out of the list, or
                                 a neighbour bin / mesh cell too crowded to sort */
#define SEDIMI_EUNSTABLE (-5) /* non-finite state */
#define SEDIMI_EESCAPE (-6)   /* a particle left [0, Lz] through a wall plane */
#define SEDIMI_ENOCONV (-7)   /* diffusion solve above its residual tolerance */
#define SEDIMI_ESTATE (-8)    /* call out of order (e.g. no particles yet) */

/* drag laws (Section 2.3); w = U_f - u_p at the particle centre */
#define SEDIMI_DRAG_NONE 0
#define SEDIMI_DRAG_DIFELICE 1 /* 1/2 C_d rho_f (pi d^2/4) eps_f^(2-chi) |w| w */
#define SEDIMI_DRAG_STOKES 2   /* 3 pi mu d w */
#define SEDIMI_DRAG_SYAMLAL 3  /* Syamlal-O'Brien, Eqs. (beta-i)-(drag-A):
                                  (3/4) V_p C_d rho_f |w| w / (V_r^2 d),
                                  C_d = (0.63 + 4.8 sqrt(V_r/Re))^2,
                                  Re = rho_f d |w| / mu */

/* arithmetic of the force evaluation */
#define SEDIMI_FP64 0  /* everything in FP64 */
#define SEDIMI_MIXED 1 /* FP64 state, geometry and integration; FP32 force arithmetic,
                          FP32 tangential history; FP32 diffusion vectors with FP64
                          residual reduction */

/* force components for sedimi_get_forces */
#define SEDIMI_F_CONTACT 0  /* spring-dashpot + friction, particle and wall contacts */
#define SEDIMI_F_LUB 1      /* lubrication */
#define SEDIMI_F_DRAG 2     /* drag */
#define SEDIMI_F_PRESSURE 3 /* -V_p grad p */
#define SEDIMI_F_ADDED 4    /* added mass */
#define SEDIMI_F_TOTAL 5    /* sum of the forces (lift included) + m g */
#define SEDIMI_F_TORQUE 6   /* contact torque */
#define SEDIMI_F_LIFT 7     /* shear lift (zero unless c_lift > 0) */

/* mesh fields for sedimi_get_field / sedimi_set_field.  RAW and SMOOTH are
 * [nch][ncell] with nch = 4 (solid fraction, drag density x, y, z), or 7 when
 * avg_solid_velocity is set (channels 4..6: the solid volume flux
 * eps_s U_s = sum V_p u_p / V_c). */
#define SEDIMI_FIELD_RAW 0    /* deposited, before smoothing (Eq. 11) */
#define SEDIMI_FIELD_SMOOTH 1 /* after the diffusion solve (Eq. 12); channel 0
                                 is the solid fraction the drag reads */
#define SEDIMI_FIELD_US 2     /* get only, [3][ncell]: the solid velocity U_s,
                                 smoothed flux / smoothed eps_s where eps_s
                                 > 1e-9, else 0 (avg_solid_velocity only) */

typedef struct sedimi_ctx sedimi_ctx;

typedef struct {
  double Lx, Ly, Lz;         /* domain (m) */
  int nx, ny, nz;            /* mesh cells per axis (uniform spacing) */
  double kn;                 /* normal contact stiffness (N/m) */
  double restitution;        /* normal restitution e, 0 < e <= 1 */
  double friction;           /* Coulomb coefficient */
  double kt_over_kn;         /* tangential stiffness ratio */
  double gammat_over_gamman; /* tangential damping ratio */
  double lub_out_frac;       /* lubrication cut-off gap / mean diameter */
  double lub_in_frac;        /* lubrication gap floor / mean diameter */
  double rho_f, mu_f;        /* fluid density (kg/m^3), dynamic viscosity (Pa s) */
  double c_add;              /* added-mass coefficient */
  double gx, gy, gz;         /* gravity (m/s^2) */
  double dt;                 /* time step (s) */
  int drag_law;              /* SEDIMI_DRAG_* */
  int lubrication;           /* 0/1 */
  int fluid_forces;          /* 0/1: pressure gradient and added mass */
  int bottom_wall, top_wall; /* 0/1 */
  double eps_s_max;          /* clamp of the interpolated solid fraction in the drag */
  double avg_bandwidth;      /* averaging bandwidth b (m); pseudo-time b^2/4 */
  int avg_ntau;              /* implicit pseudo-time steps (0: no smoothing, SMOOTH = RAW) */
  double avg_rtol;           /* relative residual tolerance of each implicit step */
  int precision;             /* SEDIMI_FP64 or SEDIMI_MIXED */
  double d_max;              /* largest particle diameter the context will hold (m);
                                sets the neighbour-bin size */
  double skin;               /* neighbour-list skin (m); the list is rebuilt when any
                                particle has moved skin/2 since the last build */
  int max_neighbors;         /* neighbour slots per particle, 1..30 */
  /* learned stand-in for the diffusion averaging (not part of the paper) */
  int nn_enable;             /* 1: allocate the 6-layer, 32-channel 3-D CNN */
  double nn_alpha;           /* leaky-ReLU slope for negative arguments */
  double nn_bound;           /* fallback when the check's estimated relative error of the
                                solid fraction exceeds this */
  double nn_sample;          /* share of z-columns (so of cells) the check samples */
  uint64_t nn_seed;          /* seed of the residual sample */
  int avg_solver;            /* SEDIMI_SOLVE_*: how the implicit steps are solved */
  double avg_bandwidth_z;    /* averaging bandwidth across the bed, along z (m); 0: the
                                same as avg_bandwidth.  The z diffusivity is then
                                (avg_bandwidth_z / avg_bandwidth)^2, so each axis has
                                its own Gaussian width (Section 4's cases use 2d / d) */
  double c_lift;             /* lift coefficient C_l of Eq. (particleLift); 0: no lift.
                                Read as Saffman's shear lift
                                C_l rho_f nu^(1/2) d^2 |w|^(-1/2) (U_f - u_p) x w with
                                w = curl U_f, nu = mu_f / rho_f, the curl taken by
                                central differences at cell centres (periodic in x and
                                y, one-sided in the first and last z cell, zero with one
                                z cell) and interpolated like U_f; 1.6 approximates
                                Saffman's 1.615 */
  int avg_solid_velocity;    /* nonzero: the averaging also deposits and smooths
                                the particle volume flux and forms the solid
                                velocity U_s (Section 2.4); the SMOOTH field
                                then has 7 channels.  Not with nn_enable (the
                                network covers the 4 standard channels) */
  int avg_scheme;            /* pseudo-time scheme of the averaging (Section 2.4):
                                SEDIMI_SCHEME_EULER, or SEDIMI_SCHEME_BDF2 (either
                                solver; not with nn_enable) */
  double z_grading;          /* top / bottom cell height ratio of a z mesh graded
                                towards the bottom wall (Section 4's channel case):
                                cell heights grow geometrically from the bottom,
                                h_k = h_0 q^k with q^(nz-1) = z_grading, summed in
                                order and scaled to Lz.  0 or 1: uniform; finite
                                and >= 0, else EINVAL.  On a graded mesh the
                                deposition finds each particle's cell from the faces
                                and divides by that cell's volume, the diffusion is
                                the finite-volume operator (face flux over the
                                centre distance, per unit cell height), the fluid
                                fields and their curl are interpolated between the
                                centres' own heights.  The direct solve handles
                                nz <= 512 (its z transform is an eigen-decomposition
                                at sedimi_create); the network (nn_enable) and
                                sedimi_smooth_static need a uniform mesh (EINVAL) */
} sedimi_params;

/* avg_scheme: backward Euler, (I - dtau L) phi^{m+1} = phi^m; or the two-step
 * backward difference formula (I - 2/3 dtau L) phi^{m+1} = (4 phi^m - phi^{m-1})/3,
 * started by one backward-Euler step (the paper's second-order implicit
 * scheme) */
#define SEDIMI_SCHEME_EULER 0
#define SEDIMI_SCHEME_BDF2 1

/* solvers of the implicit diffusion steps (Eq. 12) */
#define SEDIMI_SOLVE_AUTO 0      /* direct when every axis has <= 2048 cells
                                    (graded z meshes: and nz <= 512) */
#define SEDIMI_SOLVE_DIRECT 1    /* exact diagonalisation: Hartley transforms
                                    in x and y, DCT-II in z (graded z meshes:
                                    the eigenvectors of the graded z operator);
                                    all N_tau steps in one pass; FP64 always */
#define SEDIMI_SOLVE_ITERATIVE 2 /* Chebyshev iteration per step to avg_rtol
                                    (FP32 vectors with FP64 residuals in mixed mode) */

/* averaging modes (sedimi_set_avg_mode) */
#define SEDIMI_AVG_PLAIN 0             /* deposition + implicit diffusion solve */
#define SEDIMI_AVG_SURROGATE_CHECKED 1 /* network, sampled error check, plain
                                          solve when the check fails */
#define SEDIMI_AVG_SURROGATE 2         /* network only */

typedef struct {
  int64_t steps;          /* steps taken since sedimi_set_particles */
  int64_t rebuilds;       /* neighbour-list rebuilds (re-sorts) */
  int32_t max_neighbors;  /* largest neighbour count seen at a rebuild */
  int32_t flags;          /* bit 0 slot overflow, 1 lost contact, 2 escape, 3 non-finite,
                             4 a neighbour bin (> 1024) or mesh cell (> 4096) too crowded
                             to sort */
  int64_t solve_iters;    /* iterations of the last diffusion solve (all steps) */
  double solve_residual;  /* largest final relative residual of the last solve */
  double mean_neighbors;  /* mean neighbour-list length per particle (now) */
  double mean_contacts;   /* mean tangential-history slots in use per particle,
                             walls included (now) */
  int64_t nn_calls;       /* averagings answered by the network (checked or not) */
  int64_t nn_fallbacks;   /* checked averagings that fell back to the plain solve */
  double nn_last_check;   /* estimated relative error of the solid fraction at the last
                             check */
  int64_t particles;      /* particles in the context */
  double nn_check_trunc;  /* mass of the check's Green's function outside its window */
  int32_t nn_check_window[3]; /* the window's half widths in cells (x, y, z) */
  int32_t nn_check_columns;   /* z-columns the check samples */
  int64_t graph_steps;        /* sedimi_step calls run from a captured graph (the
                                 capturing call included; see sedimi_set_step_graphs) */
} sedimi_stats;

/* Device time per phase of sedimi_step / sedimi_average, measured with HIP
 * events recorded on the bound stream around each phase while profiling is
 * on.  Phases: 0 half kick + drift, 1 neighbour-list rebuild chain (its
 * kernels return at once when no rebuild is due), 2 force kernel, 3
 * deposition, 4 diffusion solve (or network + check), 5 network training step. */
#define SEDIMI_NPHASES 6
typedef struct {
  double ms[SEDIMI_NPHASES];
  int64_t count[SEDIMI_NPHASES];
} sedimi_profile;

/* Create a context for up to max_particles particles.  Checks the parameters
 * (EINVAL with a message on failure).  No device memory is touched yet. */
int sedimi_create(const sedimi_params* p, int64_t max_particles, sedimi_ctx** out);
void sedimi_destroy(sedimi_ctx* ctx);
/* Message of the context's last failure; with NULL, of the calling thread's
 * last failed context-free call ("null context" before any). */
const char* sedimi_last_error(const sedimi_ctx* ctx);

/* Device bytes the context needs; bind a device allocation of at least that
 * size (256-byte aligned), owned and kept alive by the caller. */
size_t sedimi_workspace_bytes(const sedimi_ctx* ctx);
int sedimi_bind_workspace(sedimi_ctx* ctx, void* dev_ptr, size_t bytes);
/* Bind the HIP stream (hipStream_t passed as void*) all device work goes to. */
int sedimi_set_stream(sedimi_ctx* ctx, void* hip_stream);

/* Upload particles (host, ID order) and build the neighbour list.  Angular
 * velocity may be NULL (zero).  Resets accelerations, history and counters. */
int sedimi_set_particles(sedimi_ctx* ctx, int64_t n, const double* x, const double* v,
                         const double* omega, const double* diam, const double* rho_p);
/* Upload the frozen fluid fields (host, [ncell][3] each; NULL = zero). */
int sedimi_set_fluid(sedimi_ctx* ctx, const double* U, const double* gradp,
                     const double* dudt);
/* Overwrite the RAW or SMOOTH mesh field (host [nch][ncell]). */
int sedimi_set_field(sedimi_ctx* ctx, int field, const double* in);
/* Translate every particle by (dx, dy) on the periodic axes (positions
 * wrapped into [0, L)); relative positions, neighbour lists and contact
 * history are unchanged.  Used to draw shifted copies of a bed. */
int sedimi_translate(sedimi_ctx* ctx, double dx, double dy);
/* Overwrite the stored accelerations a^n (host [n][3], ID order; used by the
 * added-mass lag and the next half kick). */
int sedimi_set_accel(sedimi_ctx* ctx, const double* a, const double* alpha);

/* One force evaluation at the current state (no time integration): stores
 * the per-component breakdown for sedimi_get_forces and the accelerations
 * a = F/m + g, alpha = T/I (the previous a is the added-mass lag).  The
 * tangential history advances only if update_history != 0. */
int sedimi_compute_forces(sedimi_ctx* ctx, int update_history);
/* nsteps velocity-Verlet steps (half kick, drift, forces at the half-step
 * velocities, half kick).  If average_every > 0, the averaging runs after
 * every step whose global index is a multiple of average_every, and its
 * solid fraction feeds the drag of the following steps. */
int sedimi_step(sedimi_ctx* ctx, int nsteps, int average_every);
/* Replay of sedimi_step from HIP graphs (on by default).  When the steps of a
 * call contain no averaging other than the plain direct solve (so nothing is
 * read back inside them), the call's kernel sequence is captured once into a
 * graph on a stream of the context's own and later calls of the same shape
 * (same nsteps, average_every and place in the averaging cycle, unchanged
 * parameters, workspace and particle count) launch that graph on the
 * context's stream: fewer per-kernel launch costs, identical results.  Up to
 * 4 graphs are kept per context.  If a capture fails the call runs the
 * kernels directly and replay stays off for the context.  enable = 0 turns
 * replay off and frees the graphs. */
int sedimi_set_step_graphs(sedimi_ctx* ctx, int enable);
/* Rebuild the neighbour lists now, as sedimi_step does when a particle has
 * moved half the skin (Section 2.5's link-cell search): binning, the stable
 * re-sort by (bin, ID), the pair search and the carry-over of the tangential
 * history.  Positions, velocities and history are unchanged; later steps may
 * differ from an unforced run by the order of each particle's force sum only.
 * Errors: ESTATE before particles, EOVERFLOW as sedimi_step. */
int sedimi_rebuild(sedimi_ctx* ctx);
/* Deposition (Eq. 11) into the RAW field, then the diffusion solve (Eq. 12)
 * into the SMOOTH field.  Both use the particles' current positions and the
 * drag of the last force evaluation.  Like sedimi_step, returns the error of
 * any state flag raised since sedimi_set_particles (EOVERFLOW when a mesh
 * cell holds more than 4096 particles: its sum is then not in ID order). */
int sedimi_average(sedimi_ctx* ctx);
/* Deposition only (RAW field); flags as sedimi_average. */
int sedimi_deposit(sedimi_ctx* ctx);
/* Diffusion solve only: SMOOTH <- smoothed RAW, for channels [0, nch), nch at
 * most the field's channel count; with all 7 channels U_s is formed too. */
int sedimi_smooth(sedimi_ctx* ctx, int nch);

/* Read back, in ID order.  Any output pointer may be NULL. */
int sedimi_get_particles(sedimi_ctx* ctx, double* x, double* v, double* omega, double* a);
/* The accelerations a^n and angular accelerations alpha^n of the last force
 * evaluation (host [n][3], ID order), the counterpart of sedimi_set_accel: with
 * sedimi_get_particles, sedimi_get_history and the SMOOTH field they make a
 * checkpoint from which set_particles, set_field, set_accel and set_history
 * resume the run (Section 2.5's velocity Verlet needs a^n and alpha^n for the
 * next half kick). */
int sedimi_get_accel(sedimi_ctx* ctx, double* a, double* alpha);
/* Checkpoint of the whole context as one opaque blob: the device workspace
 * (particles in their sorted order, neighbour lists, contact history, mesh
 * fields, network) and the host-side counters.  A context created with the
 * same parameters and capacity restores it with sedimi_set_state and
 * continues the run bit for bit.
 * get: *size_out receives the blob size (about the workspace size); the blob
 * is written only if buf is non-NULL and cap >= that size, else ENOMEM when
 * buf is non-NULL.  set: EINVAL if the blob is malformed or from a context
 * with other parameters or capacity.  Both synchronise the stream; host
 * buffers are the caller's. */
int sedimi_get_state(sedimi_ctx* ctx, void* buf, size_t cap, size_t* size_out);
int sedimi_set_state(sedimi_ctx* ctx, const void* buf, size_t size);
int sedimi_get_forces(sedimi_ctx* ctx, int component, double* f);
int sedimi_get_field(sedimi_ctx* ctx, int field, double* out);
/* Current pair set (Section 2.5: particles interact, by contact or by
 * lubrication, when the centre distance is below the contact distance plus
 * the lubrication cut-off), as (i, j) ID pairs with i < j in ascending order,
 * host int64 [cap][2].  *n_out receives the count; returns EOVERFLOW if it
 * exceeds cap (nothing beyond cap is written). */
int sedimi_get_pairs(sedimi_ctx* ctx, int64_t cap, int64_t* ij, int64_t* n_out);
/* Tangential contact history (the tangential spring of the soft-sphere
 * contact model, Section 2.1) as records {int64 i, int64 j, double xi[3]}:
 * i < j particle IDs, or j = -1 (wall z = 0) / -2 (wall z = Lz); xi is the
 * spring displacement of i relative to j.  get: sorted by (i, j), host
 * records [cap], *n_out the count, EOVERFLOW beyond cap; set: replaces the
 * whole history (any order; pairs must be in the current neighbour list,
 * else EINVAL).  Both synchronise the stream. */
int sedimi_get_history(sedimi_ctx* ctx, int64_t cap, void* records, int64_t* n_out);
int sedimi_set_history(sedimi_ctx* ctx, int64_t n, const void* records);
/* Counters of the run (host struct, filled whole): steps, neighbour-list
 * rebuilds and the list statistics of the link-cell search (Section 2.5), the
 * iterations and residual of the last diffusion solve (Eq. 12, Section 2.4),
 * and the network's calls, fallbacks and check window.  Synchronises. */
int sedimi_get_stats(sedimi_ctx* ctx, sedimi_stats* out);
/* Averaging mode used by sedimi_average and by the averaging inside
 * sedimi_step (SEDIMI_AVG_*; the surrogate modes need nn_enable). */
int sedimi_set_avg_mode(sedimi_ctx* ctx, int mode);

/* ---- learned stand-in for the diffusion averaging ----
 * A 6-layer 3-D CNN (3x3x3 taps; z dilations 1, 2, 4, 4, 2, 1; 32 channels;
 * layer 1: 4 -> 32, layers 2-5: 32 -> 32 with identity skips, layer 6: 32 -> 4;
 * leaky ReLU) mapping the deposited fields x to the smoothed ones in
 * per-channel normalised units as y = S x + network(x - S x).  The skip S is
 * the diffusion of Eq. 12 split by axis: each implicit step replaced by the
 * product of the exact one-dimensional implicit steps along x, y and z
 * (FP32, computed from the mesh, the bandwidths and avg_ntau); it leaves only
 * the steps' small non-separable cross terms to the network, which reads the
 * part of the field S smooths away.  Periodic in x, y and mirror
 * padded in z (the field extended by reflection about the wall faces, as the
 * zero-flux walls of Eq. 12 reflect the diffusion).  BF16 weights and
 * activations, FP32 accumulation and output.
 * Parameters are a flat FP32 vector: per layer w[27][cin][cout] then b[cout],
 * tap t = (dz+1)*9 + (dy+1)*3 + (dx+1).  The plain solve stays the fallback
 * and the reference: a checked averaging estimates the network's error on a
 * seeded sample of whole z-columns (the nn_sample share of the columns, so of
 * the cells), where the plain solution is the Green's function G of all ntau
 * implicit steps of Eq. 12, (I - dtau L_h)^-ntau, applied to RAW: over a
 * window of at most 9 x 9 x 65 cells (periodic in x, y; the walls' mirror
 * images in z) that holds all but 1e-4 of G's mass where the mesh allows
 * (chosen at sedimi_bind_workspace; sedimi_get_stats reports it and the mass
 * outside, which bounds the estimate's own error by that share of the
 * field's largest value).  It accepts the network's field y if
 * |y - G*RAW| / |G*RAW| over the sample is <= nn_bound for the solid fraction
 * (channel 0, the field the particle step reads back); otherwise the plain
 * solve runs.  On meshes where G reaches beyond the window (cells coarse
 * against the bandwidth) the estimate cannot resolve small errors and the
 * check falls back.  Backward Euler only (the network is refused with
 * BDF2). */
int sedimi_nn_param_count(const sedimi_ctx* ctx, int64_t* n);
/* Seeded normal initial weights: standard deviation sqrt(2 / ((1 + a^2) fan_in))
 * for leaky-ReLU slope a (fan_in = 27 x input channels), halved on the four
 * residual layers; the last layer and all biases zero (the network starts as
 * its skip); Adam moments zero. */
int sedimi_nn_init(sedimi_ctx* ctx, uint64_t seed);
int sedimi_nn_set_params(sedimi_ctx* ctx, const float* p, int64_t n);
int sedimi_nn_get_params(sedimi_ctx* ctx, float* p, int64_t n);
/* The trained network as one host blob, so that training resumes exactly: a
 * header (magic, parameter count, Adam step count, channel groups, leaky-ReLU
 * slope, the per-channel standardisation and loss weights) followed by the FP32
 * parameters and Adam's first and second moments (3 x count floats).
 * save: *size_out receives the blob size; the blob is written only if buf is
 * non-NULL and cap >= that size, else ENOMEM when buf is non-NULL.
 * load: EINVAL if the blob is malformed, its parameter count differs or its
 * slope differs from the context's nn_alpha.  Both synchronise the stream;
 * the buffer is the caller's. */
int sedimi_nn_save(sedimi_ctx* ctx, void* buf, size_t cap, size_t* size_out);
int sedimi_nn_load(sedimi_ctx* ctx, const void* buf, size_t size);
/* Gradient of the loss from the last sedimi_nn_train_step (same layout). */
int sedimi_nn_get_grads(sedimi_ctx* ctx, float* g, int64_t n);
/* Per-channel normalisation x_n = (x - mean) / std of inputs and targets,
 * outputs mapped back by y * std + mean.  std: finite and nonzero; a negative
 * value flips the channel's sign.  The averaging is linear and acts on each
 * channel alone, so training with a random sign (and scale) per channel and
 * step keeps the network from tying one channel's output to another
 * channel's input.  EINVAL otherwise. */
int sedimi_nn_set_norm(sedimi_ctx* ctx, const double* mean4, const double* std4);
/* Channel groups of the network: 1 (default, every hidden channel sees every
 * field) or 4.  With 4, the 32 hidden channels split into 4 groups of 8 and
 * group k reads and writes field k only: every weight joining two groups is
 * zeroed now and held at zero (sedimi_nn_set_params and sedimi_nn_init zero
 * it, and each training step zeroes its gradient before Adam), so the output
 * for one field depends on that field's input alone, as the averaging of
 * Eq. 12 does (the diffusion acts on each field separately).  The setting
 * travels in the network blob and the state blob.  EINVAL for other values. */
int sedimi_nn_set_groups(sedimi_ctx* ctx, int groups);
/* Per-channel weights w of the training loss (default 1 each): the loss is
 * sum_ch w_ch mean over cells of (y - target)^2 / 4.  Weights that equalise
 * the channels' errors let a channel with a small error (the solid fraction)
 * be learned beside noisier ones. */
int sedimi_nn_set_loss_weights(sedimi_ctx* ctx, const double* w4);
/* SMOOTH <- network(RAW) (no check). */
int sedimi_nn_forward(sedimi_ctx* ctx);
/* One Adam step (lr; beta 0.9 / 0.999; eps 1e-8) on the weighted
 * mean-squared error between network(RAW) and SMOOTH in normalised units;
 * *loss (may be NULL) receives the loss before the step.  RAW and SMOOTH are
 * not modified. */
int sedimi_nn_train_step(sedimi_ctx* ctx, double lr, double* loss);
/* The network's tensors of the last sedimi_nn_train_step (its forward
 * keeps them all; sedimi_nn_forward refreshes X, XB, SX, H and Y only), for
 * inspection and element-wise tests, as FP32 (BF16 values are exact in FP32)
 * channel-last [ncell][channels]: n must be 4 ncell, or 32 ncell for the
 * per-layer tensors, layer 0..4 (the outputs of layers 1..5). */
#define SEDIMI_NN_X 0   /* normalised input, FP32 [ncell][4] */
#define SEDIMI_NN_XB 1  /* its BF16 copy, the first layer's input [ncell][4] */
#define SEDIMI_NN_SX 2  /* the skip S x, FP32 [ncell][4] */
#define SEDIMI_NN_Z 3   /* pre-activation z_l, BF16 [ncell][32] */
#define SEDIMI_NN_H 4   /* activation h_l, BF16 [ncell][32] */
#define SEDIMI_NN_Y 5   /* output S x + conv6(h_5) + b, FP32 [ncell][4] (normalised) */
#define SEDIMI_NN_DY 6  /* loss gradient at the output, BF16 [ncell][4] */
#define SEDIMI_NN_DH 7  /* loss gradient at h_l, BF16 [ncell][32] */
#define SEDIMI_NN_DZ 8  /* loss gradient at z_l, BF16 [ncell][32] */
int sedimi_nn_get_tensor(sedimi_ctx* ctx, int which, int layer, float* out, int64_t n);
/* The check's error estimate for SMOOTH, per channel (rel4[4]):
 * |SMOOTH - G*RAW| / |G*RAW| over the sampled columns. */
int sedimi_nn_check(sedimi_ctx* ctx, double* rel4);

/* ---- the direct solve without an allocation ----
 * For callers that cannot allocate device memory or bind a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same direct solve as sedimi_smooth (all avg_ntau implicit
 * steps, backward Euler or BDF2, uniform mesh) of channels [0, nch) of a
 * caller's device field raw_dev [nch][ncell] into smooth_dev [nch][ncell]
 * (caller-owned device memory on the current device, not overlapping),
 * enqueued on hip_stream (NULL: the null stream), with no context.
 * It reads the mesh (Lx, Ly, Lz, nx, ny, nz, z_grading), avg_bandwidth,
 * avg_bandwidth_z, avg_ntau and avg_scheme of p and ignores the rest; every
 * axis <= 2048 cells, a uniform z mesh (z_grading 0 or 1), nch 1..7.
 * Memory: the transform tables and one intermediate field live in a static
 * device array of SEDIMI_STATIC_SCRATCH_BYTES that each GPU the library runs
 * on holds until the process ends.  The call needs
 * 8 (nx^2 + ny^2 + 2 nz^2 + nx + ny + nz) bytes (rounded up to 256) plus
 * 8 nch nx ny nz bytes of it and refuses larger problems (ENOMEM).  Every
 * call on one GPU shares that array, so calls that overlap on one GPU (on
 * other streams or threads) race; calls on one stream are ordered.  It calls
 * no allocator: the first call on each device looks up the array's address
 * (not a stream operation).
 * Asynchronous: no residual check (sedimi_smooth's needs a read back) and no
 * synchronisation.  Errors (EINVAL, ENOMEM, EDEVICE) leave nothing enqueued;
 * sedimi_last_error(NULL) gives the calling thread's last message. */
#define SEDIMI_STATIC_SCRATCH_BYTES (64u << 20)
int sedimi_smooth_static(const sedimi_params* p, int nch, const double* raw_dev,
                         double* smooth_dev, void* hip_stream);

/* Turn phase timing on (1) or off (0); turning it on clears the totals. */
int sedimi_set_profiling(sedimi_ctx* ctx, int on);
/* Totals since profiling was turned on (synchronises the stream). */
int sedimi_get_profile(sedimi_ctx* ctx, sedimi_profile* out);

#ifdef __cplusplus
}
#endif
#endif /* SEDIMI_H */

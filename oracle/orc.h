/*
 * orc.h -- plain FP64 CPU oracle for the SediFoam CFD-DEM particle step and the
 * diffusion-based particle-to-mesh averaging (Sun & Xiao, SediFoam).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or constant with the
 * GPU path.  Every routine is written for clarity, not speed: pairs are
 * handled once each in ascending (i, j) order, sums run in particle-ID order,
 * and the linear solves are textbook conjugate gradients.  Loops whose
 * iterations are independent may run on OpenMP threads; the sums after
 * them keep that order.
 *
 * Conventions (all SI):
 *   axes x streamwise (periodic, [0, Lx)), y spanwise (periodic, [0, Ly)),
 *   z wall-normal with walls at z = 0 and z = Lz;
 *   particle arrays are [n][3] row-major for vectors and [n] for scalars,
 *   indexed by particle ID;
 *   mesh fields are cell-centred, cell (i, j, k) at index (k*ny + j)*nx + i,
 *   vectors [ncell][3]; averaged channel arrays are [channel][ncell].
 *
 * Readings of the paper that this oracle fixes (the paper names the models but
 * does not print them) are listed where each routine is defined in the C files.
 */
#ifndef ORC_H
#define ORC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_DRAG_NONE = 0, ORC_DRAG_DIFELICE = 1, ORC_DRAG_STOKES = 2, ORC_DRAG_SYAMLAL = 3 };
enum { ORC_WALL_BOTTOM = -1, ORC_WALL_TOP = -2 };

typedef struct {
  double Lx, Ly, Lz;         /* domain; periodic x, y; walls at z = 0 and Lz */
  int nx, ny, nz;            /* Eulerian mesh (uniform per axis) */
  double kn;                 /* normal spring stiffness (N/m) */
  double restitution;        /* normal restitution coefficient e */
  double friction;           /* Coulomb coefficient mu */
  double kt_over_kn;         /* tangential / normal stiffness */
  double gammat_over_gamman; /* tangential / normal damping */
  double lub_out_frac;       /* lubrication cut-off gap h_out = frac * (d_i + d_j)/2 */
  double lub_in_frac;        /* inner gap floor  h_in  = frac * (d_i + d_j)/2 */
  double rho_f, mu_f;        /* fluid density, dynamic viscosity */
  double c_add;              /* added-mass coefficient */
  double gx, gy, gz;         /* body acceleration */
  double dt;                 /* time step */
  int drag_law;              /* ORC_DRAG_* */
  int lubrication;           /* 0/1 */
  int fluid_forces;          /* 0/1: pressure-gradient and added-mass forces */
  int bottom_wall, top_wall; /* 0/1 */
  double eps_s_max;          /* clamp for the interpolated solid fraction in drag */
  double avg_bandwidth;      /* diffusion-averaging bandwidth b (m) */
  int avg_ntau;              /* number of implicit pseudo-time steps (0: no smoothing) */
  double cg_rtol;            /* CG relative residual tolerance */
  double avg_bandwidth_z;    /* bandwidth along z (m); 0: avg_bandwidth */
  double c_lift;             /* lift coefficient C_l of Eq. (particleLift); 0: no lift */
  int avg_scheme;            /* pseudo-time scheme: ORC_SCHEME_EULER or ORC_SCHEME_BDF2 */
  double z_grading;          /* top / bottom cell height ratio of a geometrically graded
                                z mesh; <= 0 or 1: uniform */
} orc_params;

/* ---- threads (orc_pairs.c) ----
 * The pair search, the per-pair and per-particle force evaluations and the
 * kick-drift loops run on OpenMP threads; every sum still runs in the order
 * written above, so the results are bit-identical for any thread count. */
void orc_set_threads(int nthreads);
int orc_get_threads(void);

/* ---- mesh geometry along z (orc_mesh.c) ---- */
int orc_graded(const orc_params* p);
/* faces zf[0..nz]: 0 = zf[0] < ... < zf[nz] = Lz */
void orc_z_faces(const orc_params* p, double* zf);
/* cell k with zf[k] <= z < zf[k+1], clamped to [0, nz - 1] */
int orc_z_cell(const double* zf, int nz, double z);

/* One tangential-history record.  Particle pairs carry i < j (IDs); a wall
 * contact carries j = ORC_WALL_BOTTOM or ORC_WALL_TOP.  xi is the tangential
 * spring displacement of i relative to j. */
typedef struct {
  int64_t i, j;
  double xi[3];
} orc_contact;

/* Frozen Eulerian fields interpolated to particles.  Any pointer may be NULL
 * (treated as zero).  eps_s is the averaged solid fraction [ncell]. */
typedef struct {
  const double* U;     /* fluid velocity      [ncell][3] */
  const double* gradp; /* pressure gradient   [ncell][3] */
  const double* dudt;  /* material derivative of U [ncell][3] */
  const double* eps_s; /* averaged solid volume fraction [ncell] */
} orc_fields;

/* Per-particle force breakdown of one evaluation; any pointer may be NULL. */
typedef struct {
  double* contact;  /* spring-dashpot + friction, particles and walls [n][3] */
  double* lub;      /* lubrication [n][3] */
  double* drag;     /* drag [n][3] */
  double* pressure; /* -V grad p [n][3] */
  double* added;    /* added mass [n][3] */
  double* total;    /* sum of the above + m g [n][3] */
  double* torque;   /* [n][3] */
  double* lift;     /* shear lift [n][3] */
} orc_forces_out;

/* ---- pair search (Section 2.5: neighbour lists + link-cell binning) ---- */
int orc_pairs_brute(const orc_params* p, int64_t n, const double* x, const double* d,
                    int64_t cap, int64_t* ij, int64_t* n_out);
int orc_pairs_cells(const orc_params* p, int64_t n, const double* x, const double* d,
                    int64_t cap, int64_t* ij, int64_t* n_out);

/* ---- one force evaluation (Eq. 1, Eqs. 4 and 10, Section 2.5) ----
 * v, w are the velocities the forces see; a_prev is the particle acceleration
 * stored at the previous step (added-mass lag).  hin holds the tangential
 * history before the evaluation; hout receives the history after it (contacts
 * with overlap > 0 only, in ascending (i, j) order with walls last for each i).
 * Returns 0, or -1 if cap_hout is too small, -2 on allocation failure. */
int orc_forces(const orc_params* p, int64_t n, const double* x, const double* v,
               const double* w, const double* d, const double* rho, const double* a_prev,
               const orc_fields* fl, const orc_contact* hin, int64_t nhin,
               orc_contact* hout, int64_t cap_hout, int64_t* nhout, orc_forces_out* out);

/* ---- time stepping: velocity Verlet with averaging every `average_every` steps ----
 * State arrays are updated in place: x, v, w, a (translational acceleration
 * a^n), alpha (angular acceleration), fdrag (drag of the last evaluation),
 * history (capacity cap_hist, count *nhist), eps_s [ncell] (last averaged
 * solid fraction, read by the drag), avg_out [4][ncell] (last smoothed fields,
 * may be NULL), step counter *step.  Returns 0, or a negative error. */
int orc_run(const orc_params* p, int64_t n, double* x, double* v, double* w, double* a,
            double* alpha, const double* d, const double* rho, double* fdrag,
            const double* U, const double* gradp, const double* dudt, double* eps_s,
            double* avg_out, orc_contact* hist, int64_t cap_hist, int64_t* nhist,
            int64_t* step, int nsteps, int average_every);

/* Initial evaluation: a = F/m + g, alpha = T/I at the given state with the
 * given a_prev (normally 0); history is read but not advanced. */
int orc_init_accel(const orc_params* p, int64_t n, const double* x, const double* v,
                   const double* w, double* a, double* alpha, const double* d,
                   const double* rho, double* fdrag, const double* U, const double* gradp,
                   const double* dudt, const double* eps_s, const orc_contact* hist,
                   int64_t nhist);

/* ---- averaging (Section 2.4, Eqs. 11-12) ---- */
/* raw [4][ncell]: channel 0 = sum V_p / V_c, channels 1..3 = sum f_drag / V_c */
int orc_deposit(const orc_params* p, int64_t n, const double* x, const double* d,
                const double* fdrag, double* raw);
/* flux [3][ncell]: sum V_p u_p / V_c, the solid volume flux eps_s U_s of the
 * continuity equation, deposited like the solid fraction (same cells, ID
 * order). */
int orc_deposit_flux(const orc_params* p, int64_t n, const double* x, const double* d,
                     const double* v, double* flux);
/* U_s [3][ncell] = flux / eps_s from the smoothed fields, where eps_s exceeds
 * ORC_US_EPS_MIN; 0 elsewhere (no solid there to carry a velocity). */
#define ORC_US_EPS_MIN 1e-9
void orc_solid_velocity(int64_t ncell, const double* eps_s, const double* flux, double* us);
#define ORC_SCHEME_EULER 0 /* backward Euler steps */
#define ORC_SCHEME_BDF2 1  /* second-order backward differences (first step Euler) */
/* Smooth nch channels [nch][ncell] by avg_ntau backward-Euler steps of the
 * diffusion equation up to pseudo-time b^2/4.  iters (may be NULL) receives the
 * total CG iteration count.  Returns 0, or -3 if CG failed to converge. */
int orc_diffuse(const orc_params* p, int nch, const double* in, double* out, int64_t* iters);
/* y = (I - dtau L_h) x for one channel (exposed for tests). */
void orc_apply_A(const orc_params* p, double dtau, const double* x, double* y);

#ifdef __cplusplus
}
#endif
#endif /* ORC_H */

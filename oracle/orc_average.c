/*
 * orc_average.c -- oracle particle-to-mesh averaging.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Section 2.4 (Diffusion-Based Averaging Method):
 *  - Eq. (11): the solid fraction of cell k at pseudo-time 0 is the total
 *    volume of the particles whose centre lies in k divided by the cell
 *    volume.  The drag is deposited the same way (per-particle forces summed
 *    per cell, Section 2.2's coupling scheme), as a force density; the sign
 *    stored is the force on the particles.  Sums run in particle-ID order.
 *    A centre on a cell face belongs to the upper cell; centres outside the
 *    mesh are clamped into the first/last cell.
 *  - The solid velocity U_s (Section 2.4 smooths it with the same procedure):
 *    the continuity equation carries the product eps_s U_s, so the particle
 *    volume flux sum V_p u_p / V_c is deposited like the solid fraction and
 *    smoothed like it, and U_s is the ratio of the two smoothed fields.  The
 *    weights are particle volumes (equal to mass weights for one particle
 *    density).  Where the smoothed eps_s is at rounding level the ratio
 *    means nothing and U_s is set to 0.
 *  - On a z mesh graded towards the bottom (orc_mesh.c) a particle's cell is
 *    found from the faces and each cell divides by its own volume; the
 *    diffusion is the finite-volume operator (face flux over the centre
 *    distance, per unit cell height), and CG solves it multiplied by the
 *    cell heights, which makes it symmetric positive definite.
 *  - Eq. (12): the deposited field then diffuses with unit diffusivity up to
 *    pseudo-time tau = b^2/4 (b = bandwidth; the paper states the equivalence
 *    to Gaussian averaging with bandwidth sqrt(4 tau)).  The application
 *    cases of Section 4 use a smaller bandwidth b_z across the bed than along
 *    it; the diffusivity along z is then (b_z/b)^2, so that each axis has
 *    its own Gaussian width sqrt(4 tau D_a) = b_a.  Space: the
 *    second-order central finite-volume Laplacian on the CFD mesh (Section
 *    2.5), periodic in x and y, zero flux through the walls at z = 0 and Lz
 *    (the no-flux wall condition of Section 2.4).  Time: avg_ntau implicit
 *    steps of dtau = tau/avg_ntau, each solved by plain conjugate gradients
 *    from its right-hand side to a relative residual of cg_rtol.  Backward
 *    Euler by default: (I - dtau L) phi^{m+1} = phi^m.  The paper names a
 *    second-order implicit scheme without giving it; avg_scheme = BDF2 takes
 *    the two-step backward difference formula
 *    (3 phi^{m+1} - 4 phi^m + phi^{m-1}) / (2 dtau) = L phi^{m+1},
 *    i.e. (I - (2/3) dtau L) phi^{m+1} = (4 phi^m - phi^{m-1}) / 3, started
 *    by one backward-Euler step.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Mesh cell of a position and the volumes of the cells, uniform or graded
 * along z (faces from orc_z_faces). */
typedef struct {
  double hx, hy, hz;
  double* zf; /* graded meshes only: faces [nz + 1] */
} orc_cells;

static int cells_open(const orc_params* p, orc_cells* m) {
  m->hx = p->Lx / p->nx, m->hy = p->Ly / p->ny, m->hz = p->Lz / p->nz;
  m->zf = NULL;
  if (orc_graded(p)) {
    m->zf = (double*)malloc(sizeof(double) * (size_t)(p->nz + 1));
    if (!m->zf) return -2;
    orc_z_faces(p, m->zf);
  }
  return 0;
}

static int64_t cell_of(const orc_params* p, const orc_cells* m, const double* xp) {
  int64_t a = (int64_t)floor(xp[0] / m->hx);
  int64_t b = (int64_t)floor(xp[1] / m->hy);
  int64_t c = m->zf ? (int64_t)orc_z_cell(m->zf, p->nz, xp[2]) : (int64_t)floor(xp[2] / m->hz);
  a = a < 0 ? 0 : (a >= p->nx ? p->nx - 1 : a);
  b = b < 0 ? 0 : (b >= p->ny ? p->ny - 1 : b);
  c = c < 0 ? 0 : (c >= p->nz ? p->nz - 1 : c);
  return (c * p->ny + b) * p->nx + a;
}

static double cell_volume(const orc_params* p, const orc_cells* m, int64_t k) {
  if (!m->zf) return m->hx * m->hy * m->hz;
  const int64_t c = k / ((int64_t)p->nx * p->ny);
  return m->hx * m->hy * (m->zf[c + 1] - m->zf[c]);
}

int orc_deposit(const orc_params* p, int64_t n, const double* x, const double* d,
                const double* fdrag, double* raw) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  orc_cells m;
  if (cells_open(p, &m)) return -2;
  memset(raw, 0, sizeof(double) * 4 * (size_t)ncell);
  for (int64_t i = 0; i < n; ++i) {
    int64_t k = cell_of(p, &m, x + 3 * i);
    double V = (M_PI / 6.0) * d[i] * d[i] * d[i];
    raw[k] += V;
    if (fdrag) {
      raw[ncell + k] += fdrag[3 * i];
      raw[2 * ncell + k] += fdrag[3 * i + 1];
      raw[3 * ncell + k] += fdrag[3 * i + 2];
    }
  }
  for (int64_t k = 0; k < ncell; ++k) {
    const double Vc = cell_volume(p, &m, k);
    for (int ch = 0; ch < 4; ++ch) raw[ch * ncell + k] /= Vc;
  }
  free(m.zf);
  return 0;
}

int orc_deposit_flux(const orc_params* p, int64_t n, const double* x, const double* d,
                     const double* v, double* flux) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  orc_cells m;
  if (cells_open(p, &m)) return -2;
  memset(flux, 0, sizeof(double) * 3 * (size_t)ncell);
  for (int64_t i = 0; i < n; ++i) {
    int64_t k = cell_of(p, &m, x + 3 * i);
    double V = (M_PI / 6.0) * d[i] * d[i] * d[i];
    for (int e = 0; e < 3; ++e) flux[e * ncell + k] += V * v[3 * i + e];
  }
  for (int64_t k = 0; k < ncell; ++k) {
    const double Vc = cell_volume(p, &m, k);
    for (int e = 0; e < 3; ++e) flux[e * ncell + k] /= Vc;
  }
  free(m.zf);
  return 0;
}

void orc_solid_velocity(int64_t ncell, const double* eps_s, const double* flux, double* us) {
  for (int64_t k = 0; k < ncell; ++k)
    for (int e = 0; e < 3; ++e)
      us[e * ncell + k] = eps_s[k] > ORC_US_EPS_MIN ? flux[e * ncell + k] / eps_s[k] : 0.0;
}

/* y = (I - dtau L_h) x.  L_h sums, over the six faces of a cell, the
 * difference to the neighbour divided by the squared spacing; wall faces
 * carry no flux. */
void orc_apply_A(const orc_params* p, double dtau, const double* x, double* y) {
  int nx = p->nx, ny = p->ny, nz = p->nz;
  double ix2 = 1.0 / ((p->Lx / nx) * (p->Lx / nx));
  double iy2 = 1.0 / ((p->Ly / ny) * (p->Ly / ny));
  double iz2 = 1.0 / ((p->Lz / nz) * (p->Lz / nz));
  double kz = 1.0; /* diffusivity along z */
  if (p->avg_bandwidth_z > 0.0 && p->avg_bandwidth > 0.0) {
    const double r = p->avg_bandwidth_z / p->avg_bandwidth;
    iz2 *= r * r;
    kz = r * r;
  }
  double* zf = NULL;
  if (orc_graded(p)) {
    zf = (double*)malloc(sizeof(double) * (size_t)(nz + 1));
    if (!zf) abort();
    orc_z_faces(p, zf);
  }
  for (int k = 0; k < nz; ++k) {
    for (int j = 0; j < ny; ++j) {
      for (int i = 0; i < nx; ++i) {
        int64_t c = ((int64_t)k * ny + j) * nx + i;
        double xc = x[c];
        int ip = (i + 1) % nx, im = (i + nx - 1) % nx;
        int jp = (j + 1) % ny, jm = (j + ny - 1) % ny;
        double lap = 0.0;
        lap += (x[((int64_t)k * ny + j) * nx + ip] - xc) * ix2;
        lap += (x[((int64_t)k * ny + j) * nx + im] - xc) * ix2;
        lap += (x[((int64_t)k * ny + jp) * nx + i] - xc) * iy2;
        lap += (x[((int64_t)k * ny + jm) * nx + i] - xc) * iy2;
        if (zf) {
          /* graded: flux through each face over the centre distance, per
           * unit cell height */
          const double hk = zf[k + 1] - zf[k], zc = 0.5 * (zf[k] + zf[k + 1]);
          if (k + 1 < nz)
            lap += (x[((int64_t)(k + 1) * ny + j) * nx + i] - xc) * kz /
                   (hk * (0.5 * (zf[k + 1] + zf[k + 2]) - zc));
          if (k > 0)
            lap += (x[((int64_t)(k - 1) * ny + j) * nx + i] - xc) * kz /
                   (hk * (zc - 0.5 * (zf[k - 1] + zf[k])));
        } else {
          if (k + 1 < nz) lap += (x[((int64_t)(k + 1) * ny + j) * nx + i] - xc) * iz2;
          if (k > 0) lap += (x[((int64_t)(k - 1) * ny + j) * nx + i] - xc) * iz2;
        }
        y[c] = xc - dtau * lap;
      }
    }
  }
  free(zf);
}

static double dotn(int64_t n, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) s += a[k] * b[k];
  return s;
}

/* y = H (I - dtau L_h) x with H the cell heights of a graded mesh: the
 * finite-volume operator scaled by the cell volumes, symmetric where
 * I - dtau L_h itself is not. */
static void apply_S(const orc_params* p, double dtau, const double* hcell, const double* x,
                    double* y) {
  const int64_t n = (int64_t)p->nx * p->ny * p->nz, plane = (int64_t)p->nx * p->ny;
  orc_apply_A(p, dtau, x, y);
  for (int64_t c = 0; c < n; ++c) y[c] *= hcell[c / plane];
}

static void apply_op(const orc_params* p, double dtau, const double* hcell, const double* x,
                     double* y) {
  if (hcell)
    apply_S(p, dtau, hcell, x, y);
  else
    orc_apply_A(p, dtau, x, y);
}

/* Solve (I - dtau L_h) x = b by conjugate gradients, starting from x = b; on
 * a graded mesh the system multiplied by the cell heights, which makes it
 * symmetric positive definite. */
static int cg_solve(const orc_params* p, double dtau, const double* b_in, double* x,
                    int64_t* iters, double* r, double* pv, double* Ap) {
  int64_t n = (int64_t)p->nx * p->ny * p->nz;
  memcpy(x, b_in, sizeof(double) * (size_t)n);
  double* hcell = NULL;
  double* bw = NULL;
  const double* b = b_in;
  if (orc_graded(p)) {
    const int64_t plane = (int64_t)p->nx * p->ny;
    hcell = (double*)malloc(sizeof(double) * (size_t)(p->nz + 1));
    bw = (double*)malloc(sizeof(double) * (size_t)n);
    if (!hcell || !bw) {
      free(hcell), free(bw);
      return -2;
    }
    orc_z_faces(p, hcell);
    for (int k = 0; k < p->nz; ++k) hcell[k] = hcell[k + 1] - hcell[k];
    for (int64_t c = 0; c < n; ++c) bw[c] = b_in[c] * hcell[c / plane];
    b = bw;
  }
  int rc = 0;
  double bn = sqrt(dotn(n, b, b));
  if (bn == 0.0) goto done;
  apply_op(p, dtau, hcell, x, Ap);
  for (int64_t k = 0; k < n; ++k) r[k] = b[k] - Ap[k];
  memcpy(pv, r, sizeof(double) * (size_t)n);
  double rr = dotn(n, r, r);
  int64_t it = 0;
  while (sqrt(rr) > p->cg_rtol * bn) {
    if (it > 10000) {
      rc = -3;
      goto done;
    }
    apply_op(p, dtau, hcell, pv, Ap);
    double alpha = rr / dotn(n, pv, Ap);
    for (int64_t k = 0; k < n; ++k) {
      x[k] += alpha * pv[k];
      r[k] -= alpha * Ap[k];
    }
    double rr2 = dotn(n, r, r);
    double beta = rr2 / rr;
    rr = rr2;
    for (int64_t k = 0; k < n; ++k) pv[k] = r[k] + beta * pv[k];
    ++it;
  }
  if (iters) *iters += it;
done:
  free(hcell), free(bw);
  return rc;
}

int orc_diffuse(const orc_params* p, int nch, const double* in, double* out, int64_t* iters) {
  int64_t n = (int64_t)p->nx * p->ny * p->nz;
  double tau = 0.25 * p->avg_bandwidth * p->avg_bandwidth;
  /* no pseudo-time steps: the deposited field itself (no smoothing) */
  int ntau = p->avg_ntau > 0 ? p->avg_ntau : 0;
  double dtau = ntau > 0 ? tau / ntau : 0.0;
  double* cur = (double*)malloc(sizeof(double) * (size_t)n);
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* pv = (double*)malloc(sizeof(double) * (size_t)n);
  double* Ap = (double*)malloc(sizeof(double) * (size_t)n);
  double* prev = (double*)malloc(sizeof(double) * (size_t)n);
  const int bdf2 = p->avg_scheme == ORC_SCHEME_BDF2;
  int rc = 0;
  if (iters) *iters = 0;
  if (!cur || !r || !pv || !Ap || !prev) {
    rc = -2;
    goto out;
  }
  for (int ch = 0; ch < nch; ++ch) {
    const double* src = in + (size_t)ch * n;
    double* dst = out + (size_t)ch * n;
    memcpy(cur, src, sizeof(double) * (size_t)n);
    for (int m = 0; m < ntau; ++m) {
      if (bdf2 && m > 0) {
        /* right-hand side (4 phi^m - phi^{m-1}) / 3 into prev, then solve */
        for (int64_t k = 0; k < n; ++k) prev[k] = (4.0 * cur[k] - prev[k]) / 3.0;
        rc = cg_solve(p, (2.0 / 3.0) * dtau, prev, dst, iters, r, pv, Ap);
      } else {
        rc = cg_solve(p, dtau, cur, dst, iters, r, pv, Ap);
      }
      if (rc) goto out;
      memcpy(prev, cur, sizeof(double) * (size_t)n);
      memcpy(cur, dst, sizeof(double) * (size_t)n);
    }
    if (ntau == 0) memcpy(dst, cur, sizeof(double) * (size_t)n);
  }
out:
  free(cur), free(r), free(pv), free(Ap), free(prev);
  return rc;
}

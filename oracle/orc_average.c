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

int orc_deposit(const orc_params* p, int64_t n, const double* x, const double* d,
                const double* fdrag, double* raw) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  double hx = p->Lx / p->nx, hy = p->Ly / p->ny, hz = p->Lz / p->nz;
  double Vc = hx * hy * hz;
  memset(raw, 0, sizeof(double) * 4 * (size_t)ncell);
  for (int64_t i = 0; i < n; ++i) {
    int64_t a = (int64_t)floor(x[3 * i] / hx);
    int64_t b = (int64_t)floor(x[3 * i + 1] / hy);
    int64_t c = (int64_t)floor(x[3 * i + 2] / hz);
    a = a < 0 ? 0 : (a >= p->nx ? p->nx - 1 : a);
    b = b < 0 ? 0 : (b >= p->ny ? p->ny - 1 : b);
    c = c < 0 ? 0 : (c >= p->nz ? p->nz - 1 : c);
    int64_t k = (c * p->ny + b) * p->nx + a;
    double V = (M_PI / 6.0) * d[i] * d[i] * d[i];
    raw[k] += V;
    if (fdrag) {
      raw[ncell + k] += fdrag[3 * i];
      raw[2 * ncell + k] += fdrag[3 * i + 1];
      raw[3 * ncell + k] += fdrag[3 * i + 2];
    }
  }
  for (int64_t k = 0; k < 4 * ncell; ++k) raw[k] /= Vc;
  return 0;
}

int orc_deposit_flux(const orc_params* p, int64_t n, const double* x, const double* d,
                     const double* v, double* flux) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  double hx = p->Lx / p->nx, hy = p->Ly / p->ny, hz = p->Lz / p->nz;
  double Vc = hx * hy * hz;
  memset(flux, 0, sizeof(double) * 3 * (size_t)ncell);
  for (int64_t i = 0; i < n; ++i) {
    int64_t a = (int64_t)floor(x[3 * i] / hx);
    int64_t b = (int64_t)floor(x[3 * i + 1] / hy);
    int64_t c = (int64_t)floor(x[3 * i + 2] / hz);
    a = a < 0 ? 0 : (a >= p->nx ? p->nx - 1 : a);
    b = b < 0 ? 0 : (b >= p->ny ? p->ny - 1 : b);
    c = c < 0 ? 0 : (c >= p->nz ? p->nz - 1 : c);
    int64_t k = (c * p->ny + b) * p->nx + a;
    double V = (M_PI / 6.0) * d[i] * d[i] * d[i];
    for (int e = 0; e < 3; ++e) flux[e * ncell + k] += V * v[3 * i + e];
  }
  for (int64_t k = 0; k < 3 * ncell; ++k) flux[k] /= Vc;
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
  if (p->avg_bandwidth_z > 0.0 && p->avg_bandwidth > 0.0) {
    const double r = p->avg_bandwidth_z / p->avg_bandwidth;
    iz2 *= r * r;  /* diffusivity along z */
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
        if (k + 1 < nz) lap += (x[((int64_t)(k + 1) * ny + j) * nx + i] - xc) * iz2;
        if (k > 0) lap += (x[((int64_t)(k - 1) * ny + j) * nx + i] - xc) * iz2;
        y[c] = xc - dtau * lap;
      }
    }
  }
}

static double dotn(int64_t n, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) s += a[k] * b[k];
  return s;
}

/* Solve (I - dtau L_h) x = b by conjugate gradients, starting from x = b. */
static int cg_solve(const orc_params* p, double dtau, const double* b, double* x,
                    int64_t* iters, double* r, double* pv, double* Ap) {
  int64_t n = (int64_t)p->nx * p->ny * p->nz;
  memcpy(x, b, sizeof(double) * (size_t)n);
  double bn = sqrt(dotn(n, b, b));
  if (bn == 0.0) return 0;
  orc_apply_A(p, dtau, x, Ap);
  for (int64_t k = 0; k < n; ++k) r[k] = b[k] - Ap[k];
  memcpy(pv, r, sizeof(double) * (size_t)n);
  double rr = dotn(n, r, r);
  int64_t it = 0;
  while (sqrt(rr) > p->cg_rtol * bn) {
    if (it > 10000) return -3;
    orc_apply_A(p, dtau, pv, Ap);
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
  return 0;
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

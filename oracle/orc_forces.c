/*
 * orc_forces.c -- oracle particle forces and time stepping.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * What is computed, and where it comes from:
 *  - Newton's equations for translation and rotation, Eq. (1a)-(1b): the
 *    particle force is contact + lubrication + fluid-particle + m g; the torque
 *    is contact + lubrication torque (Section 2.5 says particle rotation does
 *    not interact with the fluid, so there is no fluid torque).
 *  - Contact: linear spring-dashpot soft spheres (Section 2.1 and 2.5, after
 *    Cundall & Strack / Tsuji).  The paper gives only the model's name, the
 *    stiffness, the restitution and the friction coefficient (Table 1), so
 *    this oracle fixes the following reading:
 *      normal  F = -(k_n delta + gamma_n u_n) n      on i, n from i to j,
 *              delta = r_i + r_j - |x_j - x_i|, u_n = (v_i - v_j).n,
 *              gamma_n = 2 zeta sqrt(m_eff k_n),
 *              zeta = -ln e / sqrt(pi^2 + ln^2 e), m_eff = m_i m_j/(m_i+m_j),
 *              no clipping of tensile (damping-dominated) normal force;
 *      tangential: history spring xi (displacement of i relative to j),
 *              rotated into the current tangent plane keeping |xi|, then
 *              xi += v_t dt, F_t = -k_t xi - gamma_t v_t, capped at
 *              mu |F_n| with xi reset to -(F_t + gamma_t v_t)/k_t when capped;
 *              v_t is the tangential part of
 *              v_rel = v_i - v_j + (r_i w_i + r_j w_j) x n;
 *              torque on i: r_i n x F_t, on j: r_j n x F_t;
 *      a wall is a flat, fixed body of infinite mass (m_eff = m_i).
 *  - Lubrication: the normal force of the fluid squeezed out of the gap
 *    (Section 2.5: proportional to the relative velocity and inversely
 *    proportional to the gap), F = -6 pi mu a_eff^2 u_n / max(h, h_in) n on i with
 *    a_eff = r_i r_j/(r_i + r_j) (wall: r_i), active for gap h < h_out.
 *  - Drag: the Di Felice correlation (cited in Section 2.3), force on the
 *    particle f = 1/2 C_d rho_f (pi d^2/4) eps_f^(2-chi) |w| w with
 *    w = U_f - u_p, C_d = (0.63 + 4.8/sqrt(Re))^2, Re = rho_f d eps_f |w|/mu,
 *    chi = 3.7 - 0.65 exp(-(1.5 - log10 Re)^2/2); or Stokes f = 3 pi mu d w;
 *    or the Syamlal-O'Brien correlation of Eqs. (beta-i)-(drag-A):
 *    f = V_p beta w / (eps_f eps_s) with beta = (3/4) eps_s eps_f C_d rho_f |w|
 *    / (V_r^2 d), i.e. f = (3/4) V_p C_d rho_f |w| w / (V_r^2 d), where
 *    C_d = (0.63 + 4.8 sqrt(V_r/Re))^2, Re = rho_f d |w| / mu, and
 *    V_r = (A1 - 0.06 Re + sqrt((0.06 Re)^2 + 0.12 Re (2 A2 - A1) + A1^2)) / 2,
 *    A1 = eps_f^4.14, A2 = 0.8 eps_f^1.28 (eps_f <= 0.85) else eps_f^2.65.
 *    (The printed beta omits the eps_s eps_f that the force divides out, the
 *    C_d misses its square and prints 0.48, and Re misses 1/mu; they are read
 *    as in the correlation's source.)
 *    Eq. (4) prints the fluid-side orientation (u_p - U_f); on the particle the
 *    force points towards the fluid velocity.
 *  - Graded z meshes (orc_mesh.c): fields are interpolated linearly between
 *    the graded cell centres, and the curl's z differences divide by the
 *    centre distances.
 *  - Lift (Eq. particleLift, Saffman): f = C_l rho_f nu^(1/2) d^2 |omega|^(-1/2)
 *    (U_f - u_p) x omega with omega = curl U_f at the particle (0 when
 *    omega = 0).  The printed form lacks the |omega|^(-1/2) that makes it a
 *    force and orients the slip as u_p - U_f, which would push a particle
 *    lagging a shear flow towards the slower fluid; this is Saffman's form,
 *    whose coefficient 6.46/4 = 1.615 the paper rounds to C_l = 1.6.  The
 *    curl is taken at cell centres by central differences (periodic in x, y;
 *    one-sided at the first and last cell in z) and interpolated like U_f.
 *  - Pressure gradient: f = -V_p grad p (Eq. 2b's -grad p seen by a particle;
 *    it carries the buoyancy of the hydrostatic part).
 *  - Added mass, Eq. (10): f = C_add rho_f V_p (DU_f/Dt - a_prev), where
 *    a_prev is the particle acceleration of the previous step (Section 2.3
 *    says the particle term uses the previous time); the printed orientation
 *    is the fluid-side one.
 *  - Fluid values at the particle centre come from trilinear interpolation
 *    of cell-centred values (periodic x, y; clamped to the first and last
 *    cell centres in z).
 *  - Integration: velocity Verlet with forces evaluated at the half-step
 *    velocities.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------- small vector helpers ---------------- */
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double min_image(double dx, double L) {
  double h = 0.5 * L;
  if (dx > h) {
    dx -= L;
  } else if (dx < -h) {
    dx += L;
  }
  return dx;
}
static double wrap(double x, double L) {
  if (x >= L) x -= L;
  if (x < 0.0) x += L;
  if (x >= L) x = 0.0;
  return x;
}

/* ---------------- tangential history lookup (open addressing) ---------------- */
typedef struct {
  uint64_t* key;
  int64_t* val; /* index into the history array, -1 = empty */
  uint64_t mask;
  uint64_t stride;
} hmap;

static uint64_t hkey(const hmap* h, int64_t i, int64_t j) {
  return (uint64_t)i * h->stride + (uint64_t)(j + 2);
}
static uint64_t hslot(uint64_t k, uint64_t mask) {
  return (k * 0x9E3779B97F4A7C15ull >> 17) & mask;
}
static int hmap_build(hmap* h, int64_t n, const orc_contact* c, int64_t nc) {
  uint64_t cap = 16;
  while (cap < (uint64_t)(2 * nc + 2)) cap <<= 1;
  h->key = (uint64_t*)malloc(sizeof(uint64_t) * cap);
  h->val = (int64_t*)malloc(sizeof(int64_t) * cap);
  if (!h->key || !h->val) return -2;
  h->mask = cap - 1;
  h->stride = (uint64_t)n + 2;
  for (uint64_t s = 0; s < cap; ++s) h->val[s] = -1;
  for (int64_t q = 0; q < nc; ++q) {
    uint64_t k = hkey(h, c[q].i, c[q].j);
    uint64_t s = hslot(k, h->mask);
    while (h->val[s] >= 0 && h->key[s] != k) s = (s + 1) & h->mask;
    h->key[s] = k;
    h->val[s] = q;
  }
  return 0;
}
static int64_t hmap_find(const hmap* h, int64_t i, int64_t j) {
  uint64_t k = hkey(h, i, j);
  uint64_t s = hslot(k, h->mask);
  while (h->val[s] >= 0) {
    if (h->key[s] == k) return h->val[s];
    s = (s + 1) & h->mask;
  }
  return -1;
}
static void hmap_free(hmap* h) {
  free(h->key);
  free(h->val);
}

/* ---------------- interpolation ---------------- */
static void interp_weights(const orc_params* p, const double* xp, int64_t idx[8], double wt[8]) {
  double hx = p->Lx / p->nx, hy = p->Ly / p->ny, hz = p->Lz / p->nz;
  double sx = xp[0] / hx - 0.5, sy = xp[1] / hy - 0.5, sz = xp[2] / hz - 0.5;
  double fx0 = floor(sx), fy0 = floor(sy);
  double fx = sx - fx0, fy = sy - fy0;
  int64_t i0 = (((int64_t)fx0 % p->nx) + p->nx) % p->nx, i1 = (i0 + 1) % p->nx;
  int64_t j0 = (((int64_t)fy0 % p->ny) + p->ny) % p->ny, j1 = (j0 + 1) % p->ny;
  int64_t k0, k1;
  double fz;
  if (p->nz == 1) {
    k0 = k1 = 0;
    fz = 0.0;
  } else if (orc_graded(p)) {
    /* graded: linear between the two cell centres around z, clamped to the
     * first / last centre */
    double zf[p->nz + 1];
    orc_z_faces(p, zf);
    const double z = xp[2];
    const double zlo = 0.5 * (zf[0] + zf[1]), zhi = 0.5 * (zf[p->nz - 1] + zf[p->nz]);
    if (!(z > zlo)) {
      k0 = 0, fz = 0.0;
    } else if (z >= zhi) {
      k0 = p->nz - 2, fz = 1.0;
    } else {
      k0 = 0;
      while (k0 + 1 < p->nz - 1 && 0.5 * (zf[k0 + 1] + zf[k0 + 2]) <= z) ++k0;
      const double c0 = 0.5 * (zf[k0] + zf[k0 + 1]), c1 = 0.5 * (zf[k0 + 1] + zf[k0 + 2]);
      fz = (z - c0) / (c1 - c0);
    }
    k1 = k0 + 1;
  } else {
    if (sz < 0.0) sz = 0.0;
    if (sz > p->nz - 1) sz = p->nz - 1;
    k0 = (int64_t)floor(sz);
    if (k0 > p->nz - 2) k0 = p->nz - 2;
    k1 = k0 + 1;
    fz = sz - (double)k0;
  }
  int q = 0;
  for (int c = 0; c < 2; ++c) {
    for (int b = 0; b < 2; ++b) {
      for (int a = 0; a < 2; ++a) {
        int64_t ii = a ? i1 : i0, jj = b ? j1 : j0, kk = c ? k1 : k0;
        idx[q] = (kk * p->ny + jj) * p->nx + ii;
        wt[q] = (a ? fx : 1.0 - fx) * (b ? fy : 1.0 - fy) * (c ? fz : 1.0 - fz);
        ++q;
      }
    }
  }
}
static void interp_vec(const double* f, const int64_t idx[8], const double wt[8], double* out) {
  out[0] = out[1] = out[2] = 0.0;
  if (!f) return;
  for (int q = 0; q < 8; ++q)
    for (int c = 0; c < 3; ++c) out[c] += wt[q] * f[3 * idx[q] + c];
}
static double interp_scalar(const double* f, const int64_t idx[8], const double wt[8]) {
  double s = 0.0;
  if (!f) return 0.0;
  for (int q = 0; q < 8; ++q) s += wt[q] * f[idx[q]];
  return s;
}

/* ---------------- vorticity ---------------- */
/* omega = curl U at every cell centre [ncell][3]: central differences,
 * periodic in x and y; in z central inside, one-sided in the first and last
 * cell, zero when nz = 1. */
static void curl_cells(const orc_params* p, const double* U, double* om) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const double hx = p->Lx / nx, hy = p->Ly / ny, hz = p->Lz / nz;
  /* graded meshes: cell-centre heights for the z differences */
  double zcv[nz > 0 ? nz : 1];
  const double* zc = NULL;
  if (orc_graded(p)) {
    double zf[nz + 1];
    orc_z_faces(p, zf);
    for (int k = 0; k < nz; ++k) zcv[k] = 0.5 * (zf[k] + zf[k + 1]);
    zc = zcv;
  }
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int64_t c = ((int64_t)k * ny + j) * nx + i;
        const int64_t xp = ((int64_t)k * ny + j) * nx + (i + 1) % nx;
        const int64_t xm = ((int64_t)k * ny + j) * nx + (i + nx - 1) % nx;
        const int64_t yp = ((int64_t)k * ny + (j + 1) % ny) * nx + i;
        const int64_t ym = ((int64_t)k * ny + (j + ny - 1) % ny) * nx + i;
        double dUdx[3], dUdy[3], dUdz[3];
        for (int a = 0; a < 3; ++a) {
          dUdx[a] = (U[3 * xp + a] - U[3 * xm + a]) / (2.0 * hx);
          dUdy[a] = (U[3 * yp + a] - U[3 * ym + a]) / (2.0 * hy);
          if (nz == 1) {
            dUdz[a] = 0.0;
          } else {
            const int kp = k + 1 < nz ? k + 1 : k, km = k > 0 ? k - 1 : k;
            const int64_t zp = ((int64_t)kp * ny + j) * nx + i;
            const int64_t zm = ((int64_t)km * ny + j) * nx + i;
            dUdz[a] = (U[3 * zp + a] - U[3 * zm + a]) /
                      (zc ? zc[kp] - zc[km] : (double)(kp - km) * hz);
          }
        }
        om[3 * c + 0] = dUdy[2] - dUdz[1];
        om[3 * c + 1] = dUdz[0] - dUdx[2];
        om[3 * c + 2] = dUdx[1] - dUdy[0];
      }
}

/* ---------------- drag laws ---------------- */
static void drag_force(const orc_params* p, double d, double eps_f, const double* w, double* f) {
  double wm = sqrt(dot3(w, w));
  f[0] = f[1] = f[2] = 0.0;
  if (p->drag_law == ORC_DRAG_STOKES) {
    double c = 3.0 * M_PI * p->mu_f * d;
    for (int k = 0; k < 3; ++k) f[k] = c * w[k];
  } else if (p->drag_law == ORC_DRAG_DIFELICE) {
    double Re = p->rho_f * d * eps_f * wm / p->mu_f;
    if (Re < 1e-12) return;
    double cd = 0.63 + 4.8 / sqrt(Re);
    cd = cd * cd;
    double lg = 1.5 - log10(Re);
    double chi = 3.7 - 0.65 * exp(-0.5 * lg * lg);
    double area = 0.25 * M_PI * d * d;
    double c = 0.5 * cd * p->rho_f * area * pow(eps_f, 2.0 - chi) * wm;
    for (int k = 0; k < 3; ++k) f[k] = c * w[k];
  } else if (p->drag_law == ORC_DRAG_SYAMLAL) {
    double Re = p->rho_f * d * wm / p->mu_f;
    if (Re < 1e-12) return;
    double A1 = pow(eps_f, 4.14);
    double A2 = eps_f <= 0.85 ? 0.8 * pow(eps_f, 1.28) : pow(eps_f, 2.65);
    double Vr = 0.5 * (A1 - 0.06 * Re +
                       sqrt((0.06 * Re) * (0.06 * Re) + 0.12 * Re * (2.0 * A2 - A1) + A1 * A1));
    double cd = 0.63 + 4.8 * sqrt(Vr / Re);
    cd = cd * cd;
    double Vp = M_PI / 6.0 * d * d * d;
    double c = 0.75 * Vp * cd * p->rho_f * wm / (Vr * Vr * d);
    for (int k = 0; k < 3; ++k) f[k] = c * w[k];
  }
}

/* ---------------- contact helpers ---------------- */
static double damping_ratio(double e) {
  if (e >= 1.0) return 0.0;
  double le = log(e);
  return -le / sqrt(M_PI * M_PI + le * le);
}

/* Tangential spring update and Coulomb cap for one contact.
 * n: unit normal from i to its partner; vrel: velocity of i's contact point
 * relative to the partner's; xi: in = old history (already looked up, zero if
 * new), out = new history; Fn: magnitude of the normal contact force.
 * Returns the tangential force on i in ft. */
static void tangential(const orc_params* p, double kt, double gt, const double* n,
                       const double* vrel, double Fn, double* xi, double* ft) {
  double un = dot3(vrel, n);
  double vt[3] = {vrel[0] - un * n[0], vrel[1] - un * n[1], vrel[2] - un * n[2]};
  double old = sqrt(dot3(xi, xi));
  double xn = dot3(xi, n);
  double xp[3] = {xi[0] - xn * n[0], xi[1] - xn * n[1], xi[2] - xn * n[2]};
  double pm = sqrt(dot3(xp, xp));
  if (pm > 0.0) {
    double sc = old / pm;
    for (int k = 0; k < 3; ++k) xp[k] *= sc;
  } else {
    xp[0] = xp[1] = xp[2] = 0.0;
  }
  for (int k = 0; k < 3; ++k) xi[k] = xp[k] + vt[k] * p->dt;
  for (int k = 0; k < 3; ++k) ft[k] = -kt * xi[k] - gt * vt[k];
  double fm = sqrt(dot3(ft, ft));
  double cap = p->friction * Fn;
  if (fm > cap) {
    double sc = cap / fm;
    for (int k = 0; k < 3; ++k) ft[k] *= sc;
    if (kt > 0.0)
      for (int k = 0; k < 3; ++k) xi[k] = -(ft[k] + gt * vt[k]) / kt;
  }
}

static int cmp_contact(const void* a, const void* b) {
  const orc_contact* x = (const orc_contact*)a;
  const orc_contact* y = (const orc_contact*)b;
  if (x->i != y->i) return (x->i > y->i) - (x->i < y->i);
  return (x->j > y->j) - (x->j < y->j);
}

static void add3(double* a, int64_t i, const double* f, double s) {
  if (!a) return;
  a[3 * i] += s * f[0];
  a[3 * i + 1] += s * f[1];
  a[3 * i + 2] += s * f[2];
}

/* One wall interaction of particle i.  side = ORC_WALL_BOTTOM or ORC_WALL_TOP. */
static int wall_interaction(const orc_params* p, int64_t i, int side, const double* x,
                            const double* v, const double* w, double r, double m,
                            const hmap* hm, const orc_contact* hin, orc_contact* hout,
                            int64_t cap_hout, int64_t* nh, orc_forces_out* out) {
  double n[3] = {0.0, 0.0, side == ORC_WALL_BOTTOM ? -1.0 : 1.0};
  double dist = side == ORC_WALL_BOTTOM ? x[3 * i + 2] : p->Lz - x[3 * i + 2];
  double h = dist - r;
  double dfull = 2.0 * r;
  double h_out = p->lub_out_frac * dfull;
  if (!(h < h_out)) return 0;
  double rw[3] = {r * w[3 * i], r * w[3 * i + 1], r * w[3 * i + 2]};
  double rot[3];
  cross3(rw, n, rot);
  double vrel[3] = {v[3 * i] + rot[0], v[3 * i + 1] + rot[1], v[3 * i + 2] + rot[2]};
  double un = dot3(vrel, n);
  if (p->lubrication) {
    double h_in = p->lub_in_frac * dfull;
    double hh = h > h_in ? h : h_in;
    double Fl = 6.0 * M_PI * p->mu_f * r * r * un / hh;
    double f[3] = {-Fl * n[0], -Fl * n[1], -Fl * n[2]};
    add3(out->lub, i, f, 1.0);
  }
  double delta = r - dist;
  if (delta > 0.0) {
    double gn = 2.0 * damping_ratio(p->restitution) * sqrt(m * p->kn);
    double gt = p->gammat_over_gamman * gn;
    double kt = p->kt_over_kn * p->kn;
    double Frep = p->kn * delta + gn * un;
    double fnv[3] = {-Frep * n[0], -Frep * n[1], -Frep * n[2]};
    double xi[3] = {0.0, 0.0, 0.0};
    int64_t q = hmap_find(hm, i, side);
    if (q >= 0) memcpy(xi, hin[q].xi, sizeof(xi));
    double ft[3];
    tangential(p, kt, gt, n, vrel, fabs(Frep), xi, ft);
    add3(out->contact, i, fnv, 1.0);
    add3(out->contact, i, ft, 1.0);
    double tq[3];
    cross3(n, ft, tq);
    add3(out->torque, i, tq, r);
    if (*nh >= cap_hout) return -1;
    hout[*nh].i = i;
    hout[*nh].j = side;
    memcpy(hout[*nh].xi, xi, sizeof(xi));
    ++*nh;
  }
  return 0;
}

/* One pair's lubrication, contact force and torque (Sections 2.1, 2.5), on
 * i (j gets the opposite forces); kind 0: coincident centres (skipped),
 * 1: no contact, 2: contact (xi: its updated tangential history). */
typedef struct {
  double flub[3], fnv[3], ft[3], tq[3], xi[3];
  int kind;
} pair_val;

static void pair_eval(const orc_params* p, double zeta, double kt, int64_t i, int64_t j,
                      const double* x, const double* v, const double* w, const double* d,
                      const double* rho, const hmap* hm, const orc_contact* hin, pair_val* out) {
  out->kind = 0;
  double dx[3] = {min_image(x[3 * j] - x[3 * i], p->Lx), min_image(x[3 * j + 1] - x[3 * i + 1], p->Ly),
                  x[3 * j + 2] - x[3 * i + 2]};
  double s = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2];
  double dist = sqrt(s);
  if (!(dist > 0.0)) return; /* coincident centres: direction undefined */
  out->kind = 1;
  double nv[3] = {dx[0] / dist, dx[1] / dist, dx[2] / dist};
  double ri = 0.5 * d[i], rj = 0.5 * d[j];
  double rs = ri + rj;
  double rw[3] = {ri * w[3 * i] + rj * w[3 * j], ri * w[3 * i + 1] + rj * w[3 * j + 1],
                  ri * w[3 * i + 2] + rj * w[3 * j + 2]};
  double rot[3];
  cross3(rw, nv, rot);
  double vrel[3] = {v[3 * i] - v[3 * j] + rot[0], v[3 * i + 1] - v[3 * j + 1] + rot[1],
                    v[3 * i + 2] - v[3 * j + 2] + rot[2]};
  double un = dot3(vrel, nv);
  if (p->lubrication) {
    double h = dist - rs;
    double h_in = p->lub_in_frac * rs;
    double hh = h > h_in ? h : h_in;
    double aeff = ri * rj / rs;
    double Fl = 6.0 * M_PI * p->mu_f * aeff * aeff * un / hh;
    out->flub[0] = -Fl * nv[0];
    out->flub[1] = -Fl * nv[1];
    out->flub[2] = -Fl * nv[2];
  }
  double delta = rs - dist;
  if (delta > 0.0) {
    double mi = rho[i] * (M_PI / 6.0) * d[i] * d[i] * d[i];
    double mj = rho[j] * (M_PI / 6.0) * d[j] * d[j] * d[j];
    double meff = mi * mj / (mi + mj);
    double gn = 2.0 * zeta * sqrt(meff * p->kn);
    double gt = p->gammat_over_gamman * gn;
    double Frep = p->kn * delta + gn * un;
    out->fnv[0] = -Frep * nv[0];
    out->fnv[1] = -Frep * nv[1];
    out->fnv[2] = -Frep * nv[2];
    double xi[3] = {0.0, 0.0, 0.0};
    int64_t hq = hmap_find(hm, i, j);
    if (hq >= 0) memcpy(xi, hin[hq].xi, sizeof(xi));
    tangential(p, kt, gt, nv, vrel, fabs(Frep), xi, out->ft);
    cross3(nv, out->ft, out->tq);
    memcpy(out->xi, xi, sizeof(xi));
    out->kind = 2;
  }
}

int orc_forces(const orc_params* p, int64_t n, const double* x, const double* v,
               const double* w, const double* d, const double* rho, const double* a_prev,
               const orc_fields* fl, const orc_contact* hin, int64_t nhin,
               orc_contact* hout, int64_t cap_hout, int64_t* nhout, orc_forces_out* out) {
  double* arrs[8] = {out->contact, out->lub, out->drag, out->pressure,
                     out->added, out->total, out->torque, out->lift};
  for (int k = 0; k < 8; ++k)
    if (arrs[k]) memset(arrs[k], 0, sizeof(double) * 3 * (size_t)n);
  *nhout = 0;
  if (n == 0) return 0;

  /* scratch breakdown arrays if the caller did not ask for some */
  double* own[8] = {0};
  orc_forces_out o = *out;
  double** slots[8] = {&o.contact, &o.lub, &o.drag, &o.pressure, &o.added, &o.total, &o.torque,
                       &o.lift};
  for (int k = 0; k < 8; ++k) {
    if (!*slots[k]) {
      own[k] = (double*)calloc(3 * (size_t)n, sizeof(double));
      if (!own[k]) {
        for (int q = 0; q < k; ++q) free(own[q]);
        return -2;
      }
      *slots[k] = own[k];
    }
  }

  int rc = 0;
  hmap hm;
  int64_t* ij = NULL;
  double* omega = NULL; /* vorticity at cell centres, when the lift is on */
  if (p->c_lift > 0.0 && fl && fl->U) {
    omega = (double*)malloc(sizeof(double) * 3 * (size_t)p->nx * p->ny * p->nz);
    if (!omega) {
      for (int k = 0; k < 8; ++k) free(own[k]);
      return -2;
    }
    curl_cells(p, fl->U, omega);
  }
  if (hmap_build(&hm, n, hin, nhin) != 0) {
    rc = -2;
    goto done;
  }
  /* pair set (Section 2.5) */
  int64_t cap = 8 * n + 64, np = 0;
  for (;;) {
    ij = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)cap);
    if (!ij) {
      rc = -2;
      goto done_map;
    }
    int r = orc_pairs_cells(p, n, x, d, cap, ij, &np);
    if (r == 0) break;
    free(ij);
    ij = NULL;
    if (r == -2) {
      rc = -2;
      goto done_map;
    }
    cap = np + 64;
  }

  /* Each pair's forces depend on that pair alone: they are evaluated for a
   * chunk of pairs at a time (in parallel when OpenMP threads are on), then
   * added to the two particles in ascending pair order, so every sum is the
   * same whatever the number of threads. */
  double zeta = damping_ratio(p->restitution);
  double kt = p->kt_over_kn * p->kn;
  const int64_t chunk = (int64_t)1 << 20;
  pair_val* pv = (pair_val*)malloc(sizeof(pair_val) * (size_t)(np < chunk ? (np > 0 ? np : 1) : chunk));
  if (!pv) {
    rc = -2;
    goto done_pairs;
  }
  for (int64_t q0 = 0; q0 < np; q0 += chunk) {
    const int64_t q1 = np - q0 < chunk ? np : q0 + chunk;
#pragma omp parallel for schedule(static)
    for (int64_t q = q0; q < q1; ++q)
      pair_eval(p, zeta, kt, ij[2 * q], ij[2 * q + 1], x, v, w, d, rho, &hm, hin, &pv[q - q0]);
    for (int64_t q = q0; q < q1; ++q) {
      const pair_val* r = &pv[q - q0];
      if (r->kind == 0) continue;
      const int64_t i = ij[2 * q], j = ij[2 * q + 1];
      if (p->lubrication) {
        add3(o.lub, i, r->flub, 1.0);
        add3(o.lub, j, r->flub, -1.0);
      }
      if (r->kind == 2) {
        add3(o.contact, i, r->fnv, 1.0);
        add3(o.contact, j, r->fnv, -1.0);
        add3(o.contact, i, r->ft, 1.0);
        add3(o.contact, j, r->ft, -1.0);
        add3(o.torque, i, r->tq, 0.5 * d[i]);
        add3(o.torque, j, r->tq, 0.5 * d[j]);
        if (*nhout >= cap_hout) {
          rc = -1;
          free(pv);
          goto done_pairs;
        }
        hout[*nhout].i = i;
        hout[*nhout].j = j;
        memcpy(hout[*nhout].xi, r->xi, sizeof(r->xi));
        ++*nhout;
      }
    }
  }
  free(pv);

  /* walls, in particle order (their contacts join the history list) */
  for (int64_t i = 0; i < n; ++i) {
    double r = 0.5 * d[i];
    double V = (M_PI / 6.0) * d[i] * d[i] * d[i];
    double m = rho[i] * V;
    if (p->bottom_wall &&
        wall_interaction(p, i, ORC_WALL_BOTTOM, x, v, w, r, m, &hm, hin, hout, cap_hout, nhout, &o)) {
      rc = -1;
      goto done_pairs;
    }
    if (p->top_wall &&
        wall_interaction(p, i, ORC_WALL_TOP, x, v, w, r, m, &hm, hin, hout, cap_hout, nhout, &o)) {
      rc = -1;
      goto done_pairs;
    }
  }

  /* fluid-particle forces (Section 2.3) and the totals: each particle's own */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double V = (M_PI / 6.0) * d[i] * d[i] * d[i];
    double m = rho[i] * V;
    int64_t idx[8];
    double wt[8];
    interp_weights(p, x + 3 * i, idx, wt);
    double U[3], gp[3], du[3];
    interp_vec(fl ? fl->U : NULL, idx, wt, U);
    interp_vec(fl ? fl->gradp : NULL, idx, wt, gp);
    interp_vec(fl ? fl->dudt : NULL, idx, wt, du);
    double es = interp_scalar(fl ? fl->eps_s : NULL, idx, wt);
    if (es < 0.0) es = 0.0;
    if (es > p->eps_s_max) es = p->eps_s_max;
    double eps_f = 1.0 - es;
    double wrel[3] = {U[0] - v[3 * i], U[1] - v[3 * i + 1], U[2] - v[3 * i + 2]};
    double fd[3];
    drag_force(p, d[i], eps_f, wrel, fd);
    add3(o.drag, i, fd, 1.0);
    if (p->fluid_forces) {
      double fp[3] = {-V * gp[0], -V * gp[1], -V * gp[2]};
      add3(o.pressure, i, fp, 1.0);
      double ca = p->c_add * p->rho_f * V;
      const double* ap = a_prev ? a_prev + 3 * i : NULL;
      double fa[3] = {ca * (du[0] - (ap ? ap[0] : 0.0)), ca * (du[1] - (ap ? ap[1] : 0.0)),
                      ca * (du[2] - (ap ? ap[2] : 0.0))};
      add3(o.added, i, fa, 1.0);
    }
    if (omega) {
      double om[3];
      interp_vec(omega, idx, wt, om);
      double on = sqrt(dot3(om, om));
      if (on > 0.0) {
        double c = p->c_lift * p->rho_f * sqrt(p->mu_f / p->rho_f) * d[i] * d[i] / sqrt(on);
        double fl3[3] = {c * (wrel[1] * om[2] - wrel[2] * om[1]),
                         c * (wrel[2] * om[0] - wrel[0] * om[2]),
                         c * (wrel[0] * om[1] - wrel[1] * om[0])};
        add3(o.lift, i, fl3, 1.0);
      }
    }
    for (int c = 0; c < 3; ++c) {
      double g = c == 0 ? p->gx : (c == 1 ? p->gy : p->gz);
      o.total[3 * i + c] = o.contact[3 * i + c] + o.lub[3 * i + c] + o.drag[3 * i + c] +
                           o.pressure[3 * i + c] + o.added[3 * i + c] + o.lift[3 * i + c] +
                           m * g;
    }
  }
  qsort(hout, (size_t)*nhout, sizeof(orc_contact), cmp_contact);

done_pairs:
  free(ij);
done_map:
  hmap_free(&hm);
done:
  for (int k = 0; k < 8; ++k) free(own[k]);
  free(omega);
  return rc;
}

/* Accelerations from one evaluation (Eq. 1a-1b): a = F/m + g, alpha = T/I,
 * with F the non-gravity force sum and I = (2/5) m r^2. */
static int eval_accel(const orc_params* p, int64_t n, const double* x, const double* v,
                      const double* w, const double* d, const double* rho,
                      const double* a_prev, const orc_fields* fl, const orc_contact* hin,
                      int64_t nhin, orc_contact* hout, int64_t cap_hout, int64_t* nhout,
                      double* a, double* alpha, double* fdrag) {
  size_t sz = sizeof(double) * 3 * (size_t)n;
  double* buf = (double*)malloc(6 * sz + 1);
  if (!buf) return -2;
  orc_forces_out o;
  memset(&o, 0, sizeof(o));
  o.contact = buf;
  o.lub = buf + 3 * n;
  o.pressure = buf + 6 * n;
  o.added = buf + 9 * n;
  o.torque = buf + 12 * n;
  o.lift = buf + 15 * n;
  o.drag = fdrag;
  int rc = orc_forces(p, n, x, v, w, d, rho, a_prev, fl, hin, nhin, hout, cap_hout, nhout, &o);
  if (rc == 0) {
    double g[3] = {p->gx, p->gy, p->gz};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double V = (M_PI / 6.0) * d[i] * d[i] * d[i];
      double m = rho[i] * V;
      double r = 0.5 * d[i];
      double I = 0.4 * m * r * r;
      for (int c = 0; c < 3; ++c) {
        int64_t k = 3 * i + c;
        double F = o.contact[k] + o.lub[k] + o.drag[k] + o.pressure[k] + o.added[k] + o.lift[k];
        a[k] = F / m + g[c];
        alpha[k] = o.torque[k] / I;
      }
    }
  }
  free(buf);
  return rc;
}

int orc_init_accel(const orc_params* p, int64_t n, const double* x, const double* v,
                   const double* w, double* a, double* alpha, const double* d,
                   const double* rho, double* fdrag, const double* U, const double* gradp,
                   const double* dudt, const double* eps_s, const orc_contact* hist,
                   int64_t nhist) {
  orc_fields fl = {U, gradp, dudt, eps_s};
  int64_t cap = 16 * n + 64, nh = 0;
  orc_contact* tmp = (orc_contact*)malloc(sizeof(orc_contact) * (size_t)cap);
  double* ap = (double*)calloc(3 * (size_t)n + 1, sizeof(double));
  if (!tmp || !ap) {
    free(tmp), free(ap);
    return -2;
  }
  memcpy(ap, a, sizeof(double) * 3 * (size_t)n);
  int rc = eval_accel(p, n, x, v, w, d, rho, ap, &fl, hist, nhist, tmp, cap, &nh, a, alpha, fdrag);
  free(tmp), free(ap);
  return rc;
}

int orc_run(const orc_params* p, int64_t n, double* x, double* v, double* w, double* a,
            double* alpha, const double* d, const double* rho, double* fdrag,
            const double* U, const double* gradp, const double* dudt, double* eps_s,
            double* avg_out, orc_contact* hist, int64_t cap_hist, int64_t* nhist,
            int64_t* step, int nsteps, int average_every) {
  orc_fields fl = {U, gradp, dudt, eps_s};
  orc_contact* hnew = (orc_contact*)malloc(sizeof(orc_contact) * (size_t)(cap_hist + 1));
  double* aprev = (double*)malloc(sizeof(double) * (3 * (size_t)n + 1));
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  double* raw = (double*)malloc(sizeof(double) * 4 * (size_t)ncell);
  double* sm = (double*)malloc(sizeof(double) * 4 * (size_t)ncell);
  int rc = 0;
  if (!hnew || !aprev || !raw || !sm) {
    rc = -2;
    goto out;
  }
  double dt = p->dt;
  for (int s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < 3 * n; ++k) {
      v[k] += 0.5 * dt * a[k];
      w[k] += 0.5 * dt * alpha[k];
    }
    int escaped = 0;
#pragma omp parallel for schedule(static) reduction(| : escaped)
    for (int64_t i = 0; i < n; ++i) {
      x[3 * i] = wrap(x[3 * i] + dt * v[3 * i], p->Lx);
      x[3 * i + 1] = wrap(x[3 * i + 1] + dt * v[3 * i + 1], p->Ly);
      x[3 * i + 2] = x[3 * i + 2] + dt * v[3 * i + 2];
      escaped |= !(x[3 * i + 2] >= 0.0 && x[3 * i + 2] <= p->Lz);
    }
    if (escaped) {
      rc = -4; /* a particle left the domain through a wall */
      goto out;
    }
    memcpy(aprev, a, sizeof(double) * 3 * (size_t)n);
    int64_t nh = 0;
    rc = eval_accel(p, n, x, v, w, d, rho, aprev, &fl, hist, *nhist, hnew, cap_hist, &nh, a,
                    alpha, fdrag);
    if (rc) goto out;
    memcpy(hist, hnew, sizeof(orc_contact) * (size_t)nh);
    *nhist = nh;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < 3 * n; ++k) {
      v[k] += 0.5 * dt * a[k];
      w[k] += 0.5 * dt * alpha[k];
    }
    ++*step;
    if (average_every > 0 && (*step % average_every) == 0) {
      rc = orc_deposit(p, n, x, d, fdrag, raw);
      if (rc) goto out;
      rc = orc_diffuse(p, 4, raw, sm, NULL);
      if (rc) goto out;
      if (eps_s) memcpy(eps_s, sm, sizeof(double) * (size_t)ncell);
      if (avg_out) memcpy(avg_out, sm, sizeof(double) * 4 * (size_t)ncell);
    }
  }
out:
  free(hnew), free(aprev), free(raw), free(sm);
  return rc;
}

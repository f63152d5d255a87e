/*
 * bedgen.c -- seeded synthetic sediment beds (input generation only).
 *
 * Random sequential deposition in the style of Visscher & Bolsterli: spheres
 * are dropped one at a time at a uniformly random (x, y) of a periodic box,
 * fall vertically until they touch the floor or a resting sphere, then roll
 * over their supports (one sphere: down a great circle; two spheres: down the
 * groove circle; three: stop if gravity lies inside the cone of the contact
 * normals, otherwise lift off the support that would pull) until they rest on
 * the floor, on a stable pair, or on a stable triple.  Every move ends at an
 * exactly touching position, so the bed has no overlaps beyond rounding.
 *
 * This file holds no part of the particle method (no forces, no time
 * stepping, no averaging); it only places spheres.  Random numbers come from
 * splitmix64 (Steele, Lea & Flood 2014) seeded by the caller.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static uint64_t sm64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double urand(uint64_t* s) { return (double)(sm64(s) >> 11) * (1.0 / 9007199254740992.0); }

typedef struct {
  int* idx;
  int n, cap;
} column;

typedef struct {
  double Lx, Ly, hcx, hcy; /* column widths tile the periodic box exactly */
  int ncx, ncy;
  column* col;
  const double* x; /* [n][3] placed centres */
  const double* r;
  double rmax;
} grid;

static void col_insert(grid* g, int id) {
  double x = g->x[3 * id], y = g->x[3 * id + 1];
  int a = (int)floor(x / g->hcx) % g->ncx, b = (int)floor(y / g->hcy) % g->ncy;
  if (a < 0) a += g->ncx;
  if (b < 0) b += g->ncy;
  column* c = &g->col[b * g->ncx + a];
  if (c->n == c->cap) {
    c->cap = c->cap ? 2 * c->cap : 16;
    c->idx = (int*)realloc(c->idx, sizeof(int) * c->cap);
  }
  /* keep each column sorted by z (new spheres are usually the highest) */
  int pos = c->n++;
  double z = g->x[3 * id + 2];
  while (pos > 0 && g->x[3 * c->idx[pos - 1] + 2] > z) {
    c->idx[pos] = c->idx[pos - 1];
    --pos;
  }
  c->idx[pos] = id;
}

/* Collect spheres whose centre lies within horizontal distance `hr` of
 * (cx, cy) (periodic) and whose z lies in [zlo, zhi]; the candidate records
 * carry each sphere's image nearest to (cx, cy). */
typedef struct {
  int id;
  double c[3];
} cand;

static int gather(const grid* g, double cx, double cy, double hr, double zlo, double zhi,
                  cand** buf, int* cap) {
  int n = 0;
  int a0 = (int)floor((cx - hr) / g->hcx), a1 = (int)floor((cx + hr) / g->hcx);
  int b0 = (int)floor((cy - hr) / g->hcy), b1 = (int)floor((cy + hr) / g->hcy);
  if (a1 - a0 + 1 > g->ncx) a1 = a0 + g->ncx - 1;
  if (b1 - b0 + 1 > g->ncy) b1 = b0 + g->ncy - 1;
  for (int bb = b0; bb <= b1; ++bb) {
    int b = ((bb % g->ncy) + g->ncy) % g->ncy;
    for (int aa = a0; aa <= a1; ++aa) {
      int a = ((aa % g->ncx) + g->ncx) % g->ncx;
      const column* c = &g->col[b * g->ncx + a];
      /* binary search for the first sphere with z >= zlo */
      int lo = 0, hi = c->n;
      while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (g->x[3 * c->idx[mid] + 2] < zlo)
          lo = mid + 1;
        else
          hi = mid;
      }
      for (int q = lo; q < c->n; ++q) {
        int id = c->idx[q];
        double z = g->x[3 * id + 2];
        if (z > zhi) break;
        double dx = g->x[3 * id] - cx, dy = g->x[3 * id + 1] - cy;
        dx -= g->Lx * floor(dx / g->Lx + 0.5);
        dy -= g->Ly * floor(dy / g->Ly + 0.5);
        if (dx * dx + dy * dy > hr * hr) continue;
        if (n == *cap) {
          *cap = *cap ? 2 * *cap : 256;
          *buf = (cand*)realloc(*buf, sizeof(cand) * *cap);
        }
        (*buf)[n].id = id;
        (*buf)[n].c[0] = cx + dx;
        (*buf)[n].c[1] = cy + dy;
        (*buf)[n].c[2] = z;
        ++n;
      }
    }
  }
  return n;
}

static double dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void crs(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double nrm(double* a) {
  double m = sqrt(dot(a, a));
  if (m > 0) a[0] /= m, a[1] /= m, a[2] /= m;
  return m;
}

/* Smallest phi in (eps, phi_end] at which c0 + rho (cos phi e1 + sin phi e2)
 * is at distance R from q, entering (distance decreasing through R). */
static double arc_hit_sphere(const double* c0, double rho, const double* e1, const double* e2,
                             const double* q, double R, double phi_end) {
  double d[3] = {c0[0] - q[0], c0[1] - q[1], c0[2] - q[2]};
  double a = 2.0 * rho * dot(e1, d), b = 2.0 * rho * dot(e2, d);
  double c = R * R - dot(d, d) - rho * rho;
  double m = sqrt(a * a + b * b);
  if (m <= 0.0 || fabs(c) > m) return -1.0;
  double psi = atan2(b, a), ac = acos(c / m);
  double best = -1.0;
  for (int s = 0; s < 2; ++s) {
    double phi = s ? psi - ac : psi + ac;
    while (phi <= 1e-12) phi += 2.0 * M_PI;
    while (phi > 2.0 * M_PI + 1e-12) phi -= 2.0 * M_PI;
    if (phi > phi_end) continue;
    /* entering: derivative of squared distance negative at phi */
    double dd = -a * sin(phi) + b * cos(phi);
    if (dd > 0.0) continue;
    if (best < 0.0 || phi < best) best = phi;
  }
  return best;
}

static double arc_hit_floor(const double* c0, double rho, const double* e1, const double* e2,
                            double zf, double phi_end) {
  /* c0z + rho (cos phi e1z + sin phi e2z) = zf */
  double a = rho * e1[2], b = rho * e2[2], c = zf - c0[2];
  double m = sqrt(a * a + b * b);
  if (m <= 0.0 || fabs(c) > m) return -1.0;
  double psi = atan2(b, a), ac = acos(c / m);
  double best = -1.0;
  for (int s = 0; s < 2; ++s) {
    double phi = s ? psi - ac : psi + ac;
    while (phi <= 1e-12) phi += 2.0 * M_PI;
    while (phi > 2.0 * M_PI + 1e-12) phi -= 2.0 * M_PI;
    if (phi > phi_end) continue;
    double dz = -a * sin(phi) + b * cos(phi);
    if (dz > 0.0) continue;
    if (best < 0.0 || phi < best) best = phi;
  }
  return best;
}

/* Solve M lam = rhs for 3x3 M given by columns. Returns 0 if singular. */
static int solve3(const double* c0, const double* c1, const double* c2, const double* rhs,
                  double* lam) {
  double t[3];
  crs(c1, c2, t);
  double det = dot(c0, t);
  if (fabs(det) < 1e-14) return 0;
  double u[3];
  crs(rhs, c2, u);
  double v[3];
  crs(c1, rhs, v);
  lam[0] = dot(rhs, t) / det;
  lam[1] = dot(c0, u) / det;
  lam[2] = dot(c0, v) / det;
  return 1;
}

/* Place n spheres of radii r[] by random sequential deposition.  Returns the
 * number of spheres that hit the roll-iteration cap (left where they were). */
int bedgen_rsd(int n, const double* r, double Lx, double Ly, uint64_t seed, double* x) {
  double rmax = 0.0;
  for (int i = 0; i < n; ++i) rmax = r[i] > rmax ? r[i] : rmax;
  grid g;
  g.Lx = Lx;
  g.Ly = Ly;
  g.ncx = (int)floor(Lx / (2.0 * rmax));
  g.ncy = (int)floor(Ly / (2.0 * rmax));
  if (g.ncx < 1) g.ncx = 1;
  if (g.ncy < 1) g.ncy = 1;
  g.hcx = Lx / g.ncx;
  g.hcy = Ly / g.ncy;
  g.col = (column*)calloc((size_t)g.ncx * g.ncy, sizeof(column));
  g.x = x;
  g.r = r;
  g.rmax = rmax;
  cand* buf = NULL;
  int cap = 0;
  uint64_t s = seed;
  double zmax = 0.0;
  int capped = 0;
  for (int i = 0; i < n; ++i) {
    double ri = r[i];
    double P[3] = {urand(&s) * Lx, urand(&s) * Ly, zmax + 2.0 * rmax + ri};
    int sup[3], ns = 0; /* supports: sphere ids, -1 = floor */
    int done = 0, iter = 0;
    while (!done) {
      if (++iter > 64) {
        ++capped;
        break;
      }
      if (ns == 0) {
        /* vertical fall from P: the highest touching sphere below P, scanning
         * each sorted column from the top down */
        double hr = ri + rmax;
        double zb = ri;
        int who = -1;
        int a0 = (int)floor((P[0] - hr) / g.hcx), a1 = (int)floor((P[0] + hr) / g.hcx);
        int b0 = (int)floor((P[1] - hr) / g.hcy), b1 = (int)floor((P[1] + hr) / g.hcy);
        if (a1 - a0 + 1 > g.ncx) a1 = a0 + g.ncx - 1;
        if (b1 - b0 + 1 > g.ncy) b1 = b0 + g.ncy - 1;
        for (int bb = b0; bb <= b1; ++bb) {
          int b = ((bb % g.ncy) + g.ncy) % g.ncy;
          for (int aa = a0; aa <= a1; ++aa) {
            int a = ((aa % g.ncx) + g.ncx) % g.ncx;
            const column* c = &g.col[b * g.ncx + a];
            for (int q = c->n - 1; q >= 0; --q) {
              int id = c->idx[q];
              double zj = x[3 * id + 2];
              if (zj + hr < zb) break;
              double dx = x[3 * id] - P[0], dy = x[3 * id + 1] - P[1];
              dx -= Lx * floor(dx / Lx + 0.5);
              dy -= Ly * floor(dy / Ly + 0.5);
              double R = ri + r[id];
              double rr = dx * dx + dy * dy;
              if (rr >= R * R) continue;
              double zc = zj + sqrt(R * R - rr);
              if (zc <= P[2] + 1e-12 * R && zc > zb) {
                zb = zc;
                who = id;
              }
            }
          }
        }
        P[2] = zb;
        if (who < 0) {
          done = 1; /* resting on the floor */
        } else {
          sup[0] = who;
          ns = 1;
        }
        continue;
      }
      if (ns == 1) {
        /* roll down a great circle of the support */
        int A = sup[0];
        double cA[3] = {x[3 * A], x[3 * A + 1], x[3 * A + 2]};
        double dx = cA[0] - P[0], dy = cA[1] - P[1];
        dx -= Lx * floor(dx / Lx + 0.5);
        dy -= Ly * floor(dy / Ly + 0.5);
        cA[0] = P[0] + dx;
        cA[1] = P[1] + dy;
        double R = ri + r[A];
        double e1[3] = {(P[0] - cA[0]) / R, (P[1] - cA[1]) / R, (P[2] - cA[2]) / R};
        double u[3] = {e1[0], e1[1], 0.0};
        if (nrm(u) < 1e-9) {
          double t = 2.0 * M_PI * urand(&s);
          u[0] = cos(t), u[1] = sin(t), u[2] = 0.0;
        }
        double th0 = acos(e1[2] > 1.0 ? 1.0 : (e1[2] < -1.0 ? -1.0 : e1[2]));
        if (th0 >= 0.5 * M_PI - 1e-12) {
          /* at or below the equator: the sphere falls freely */
          ns = 0;
          P[0] += 1e-12 * R * u[0];
          P[1] += 1e-12 * R * u[1];
          continue;
        }
        e1[0] = sin(th0) * u[0], e1[1] = sin(th0) * u[1], e1[2] = cos(th0);
        double e2[3] = {cos(th0) * u[0], cos(th0) * u[1], -sin(th0)};
        double phi_end = 0.5 * M_PI - th0;
        int m = gather(&g, cA[0], cA[1], R + ri + rmax, cA[2] - R - ri - rmax,
                       cA[2] + R + ri + rmax, &buf, &cap);
        double best = phi_end;
        int who = -2;
        for (int q = 0; q < m; ++q) {
          if (buf[q].id == A) continue;
          double ph = arc_hit_sphere(cA, R, e1, e2, buf[q].c, ri + r[buf[q].id], best);
          if (ph > 0.0 && ph <= best) {
            best = ph;
            who = buf[q].id;
          }
        }
        double pf = arc_hit_floor(cA, R, e1, e2, ri, best);
        if (pf > 0.0 && pf <= best) {
          best = pf;
          who = -1;
        }
        for (int k = 0; k < 3; ++k) P[k] = cA[k] + R * (cos(best) * e1[k] + sin(best) * e2[k]);
        if (who == -1) {
          done = 1; /* touches the floor */
        } else if (who >= 0) {
          sup[1] = who;
          ns = 2;
        } else {
          ns = 0; /* reached the equator */
          P[0] += 1e-9 * R * u[0];
          P[1] += 1e-9 * R * u[1];
        }
        continue;
      }
      if (ns == 2) {
        int A = sup[0], B = sup[1];
        double cA[3], cB[3];
        for (int k = 0; k < 3; ++k) cA[k] = x[3 * A + k], cB[k] = x[3 * B + k];
        double d0 = cA[0] - P[0], d1 = cA[1] - P[1];
        d0 -= Lx * floor(d0 / Lx + 0.5), d1 -= Ly * floor(d1 / Ly + 0.5);
        cA[0] = P[0] + d0, cA[1] = P[1] + d1;
        d0 = cB[0] - P[0], d1 = cB[1] - P[1];
        d0 -= Lx * floor(d0 / Lx + 0.5), d1 -= Ly * floor(d1 / Ly + 0.5);
        cB[0] = P[0] + d0, cB[1] = P[1] + d1;
        double RA = ri + r[A], RB = ri + r[B];
        double w[3] = {cB[0] - cA[0], cB[1] - cA[1], cB[2] - cA[2]};
        double dAB = nrm(w);
        double t = (RA * RA - RB * RB + dAB * dAB) / (2.0 * dAB);
        double rho2 = RA * RA - t * t;
        double gp[3] = {w[2] * w[0], w[2] * w[1], w[2] * w[2] - 1.0}; /* -ez projected */
        if (rho2 <= 0.0 || nrm(gp) < 1e-9) {
          /* degenerate groove: keep the lower support only */
          sup[0] = cA[2] < cB[2] ? A : B;
          ns = 1;
          continue;
        }
        double rho = sqrt(rho2);
        double c0[3] = {cA[0] + t * w[0], cA[1] + t * w[1], cA[2] + t * w[2]};
        double e1[3] = {P[0] - c0[0], P[1] - c0[1], P[2] - c0[2]};
        /* remove the axial part (rounding) and normalise */
        double ax = dot(e1, w);
        for (int k = 0; k < 3; ++k) e1[k] -= ax * w[k];
        nrm(e1);
        double cs = dot(e1, gp);
        cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
        double phi_end = acos(cs);
        int who = -2;
        double best = phi_end;
        if (phi_end > 1e-12) {
          double e2[3] = {gp[0] - cs * e1[0], gp[1] - cs * e1[1], gp[2] - cs * e1[2]};
          nrm(e2);
          int m = gather(&g, c0[0], c0[1], rho + ri + rmax, c0[2] - rho - ri - rmax,
                         c0[2] + rho + ri + rmax, &buf, &cap);
          for (int q = 0; q < m; ++q) {
            if (buf[q].id == A || buf[q].id == B) continue;
            double ph = arc_hit_sphere(c0, rho, e1, e2, buf[q].c, ri + r[buf[q].id], best);
            if (ph > 0.0 && ph <= best) {
              best = ph;
              who = buf[q].id;
            }
          }
          double pf = arc_hit_floor(c0, rho, e1, e2, ri, best);
          if (pf > 0.0 && pf <= best) {
            best = pf;
            who = -1;
          }
          for (int k = 0; k < 3; ++k) P[k] = c0[k] + rho * (cos(best) * e1[k] + sin(best) * e2[k]);
        }
        if (who == -1) {
          done = 1;
          continue;
        }
        if (who >= 0) {
          sup[2] = who;
          ns = 3;
          continue;
        }
        /* lowest point of the groove: stable if both contacts push up */
        double nA[3] = {P[0] - cA[0], P[1] - cA[1], P[2] - cA[2]};
        double nB[3] = {P[0] - cB[0], P[1] - cB[1], P[2] - cB[2]};
        nrm(nA), nrm(nB);
        double ez[3] = {0, 0, 1}, cAB[3], t1[3], t2[3];
        crs(nA, nB, cAB);
        double den = dot(cAB, cAB);
        crs(ez, nB, t1);
        crs(nA, ez, t2);
        double lA = dot(t1, cAB) / den, lB = dot(t2, cAB) / den;
        if (lA > 0.0 && lB > 0.0) {
          done = 1;
        } else {
          sup[0] = lA <= lB ? B : A;
          ns = 1;
        }
        continue;
      }
      /* three supports */
      double nn[3][3];
      for (int q = 0; q < 3; ++q) {
        int id = sup[q];
        double c[3] = {x[3 * id], x[3 * id + 1], x[3 * id + 2]};
        double d0 = c[0] - P[0], d1 = c[1] - P[1];
        d0 -= Lx * floor(d0 / Lx + 0.5), d1 -= Ly * floor(d1 / Ly + 0.5);
        nn[q][0] = -d0, nn[q][1] = -d1, nn[q][2] = P[2] - c[2];
        nrm(nn[q]);
      }
      double ez[3] = {0, 0, 1}, lam[3];
      if (!solve3(nn[0], nn[1], nn[2], ez, lam)) {
        ns = 2; /* coplanar normals: drop the third */
        continue;
      }
      int worst = 0;
      for (int q = 1; q < 3; ++q)
        if (lam[q] < lam[worst]) worst = q;
      if (lam[worst] > 0.0) {
        done = 1;
      } else {
        int k = 0;
        for (int q = 0; q < 3; ++q)
          if (q != worst) sup[k++] = sup[q];
        ns = 2;
      }
    }
    P[0] -= Lx * floor(P[0] / Lx);
    P[1] -= Ly * floor(P[1] / Ly);
    if (P[0] >= Lx) P[0] = 0.0;
    if (P[1] >= Ly) P[1] = 0.0;
    x[3 * i] = P[0];
    x[3 * i + 1] = P[1];
    x[3 * i + 2] = P[2];
    if (P[2] > zmax) zmax = P[2];
    col_insert(&g, i);
  }
  for (int k = 0; k < g.ncx * g.ncy; ++k) free(g.col[k].idx);
  free(g.col);
  free(buf);
  return capped;
}

/* Random sequential insertion without overlap in [0,Lx)x[0,Ly)x[r, Lz-r]
 * (uniform trial positions, rejected on overlap with any placed sphere).
 * Returns 0, or -1 if some sphere found no place within max_trials. */
int bedgen_rsa(int n, const double* r, double Lx, double Ly, double Lz, uint64_t seed,
               int max_trials, double* x) {
  double rmax = 0.0;
  for (int i = 0; i < n; ++i) rmax = r[i] > rmax ? r[i] : rmax;
  uint64_t s = seed;
  /* uniform 3-D grid of cell size >= 2 rmax */
  int cx = (int)floor(Lx / (2 * rmax)), cy = (int)floor(Ly / (2 * rmax)),
      cz = (int)floor(Lz / (2 * rmax));
  if (cx < 1) cx = 1;
  if (cy < 1) cy = 1;
  if (cz < 1) cz = 1;
  int ncell = cx * cy * cz;
  int* head = (int*)malloc(sizeof(int) * ncell);
  int* next = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
  for (int k = 0; k < ncell; ++k) head[k] = -1;
  int rc = 0;
  for (int i = 0; i < n; ++i) {
    int ok = 0;
    for (int t = 0; t < max_trials && !ok; ++t) {
      double P[3] = {urand(&s) * Lx, urand(&s) * Ly, r[i] + urand(&s) * (Lz - 2 * r[i])};
      int a = (int)(P[0] / Lx * cx), b = (int)(P[1] / Ly * cy), c = (int)(P[2] / Lz * cz);
      a = a >= cx ? cx - 1 : a, b = b >= cy ? cy - 1 : b, c = c >= cz ? cz - 1 : c;
      ok = 1;
      for (int dc = -1; dc <= 1 && ok; ++dc) {
        int cc = c + dc;
        if (cc < 0 || cc >= cz) continue;
        for (int db = -1; db <= 1 && ok; ++db) {
          int bb = ((b + db) % cy + cy) % cy;
          for (int da = -1; da <= 1 && ok; ++da) {
            int aa = ((a + da) % cx + cx) % cx;
            for (int j = head[(cc * cy + bb) * cx + aa]; j >= 0; j = next[j]) {
              double dx = x[3 * j] - P[0], dy = x[3 * j + 1] - P[1], dz = x[3 * j + 2] - P[2];
              dx -= Lx * floor(dx / Lx + 0.5);
              dy -= Ly * floor(dy / Ly + 0.5);
              double R = r[i] + r[j];
              if (dx * dx + dy * dy + dz * dz < R * R) {
                ok = 0;
                break;
              }
            }
          }
        }
      }
      if (ok) {
        x[3 * i] = P[0], x[3 * i + 1] = P[1], x[3 * i + 2] = P[2];
        int k = (c * cy + b) * cx + a;
        next[i] = head[k];
        head[k] = i;
      }
    }
    if (!ok) {
      rc = -1;
      break;
    }
  }
  free(head);
  free(next);
  return rc;
}

/*
 * orc_pairs.c -- oracle pair search.  TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The pair set is the plain definition: all particle pairs whose centre
 * distance is below the contact distance plus the lubrication cut-off gap
 * (Section 2.5, neighbour lists and link-cell binning; the cut-off gap is a
 * fraction of the mean diameter).  orc_pairs_brute enumerates every i < j;
 * orc_pairs_cells reaches the same set through a link-cell grid, as the paper
 * says the DEM module does.  Both use the same predicate, evaluated in FP64
 * in this exact association with no fused multiply-add (the file is built
 * with -ffp-contract=off):
 *     dx = x_j - x_i, with the minimum-image shift on the periodic axes
 *     s  = (dx*dx + dy*dy) + dz*dz
 *     R  = (r_i + r_j) + f_out * (r_i + r_j)
 *     pair  <=>  s < R*R        (strict)
 * Output: pairs (i, j), i < j, in ascending lexicographic order, as
 * ij[2k] = i, ij[2k+1] = j.
 */
#include "orc.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

static double min_image(double dx, double L) {
  double h = 0.5 * L;
  if (dx > h) {
    dx -= L;
  } else if (dx < -h) {
    dx += L;
  }
  return dx;
}

static int in_range(const orc_params* p, const double* xi, const double* xj, double ri,
                    double rj) {
  double dx = min_image(xj[0] - xi[0], p->Lx);
  double dy = min_image(xj[1] - xi[1], p->Ly);
  double dz = xj[2] - xi[2];
  double s = (dx * dx + dy * dy) + dz * dz;
  double rs = ri + rj;
  double R = rs + p->lub_out_frac * rs;
  return s < R * R;
}

int orc_pairs_brute(const orc_params* p, int64_t n, const double* x, const double* d,
                    int64_t cap, int64_t* ij, int64_t* n_out) {
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = i + 1; j < n; ++j) {
      if (in_range(p, x + 3 * i, x + 3 * j, 0.5 * d[i], 0.5 * d[j])) {
        if (cnt < cap) {
          ij[2 * cnt] = i;
          ij[2 * cnt + 1] = j;
        }
        ++cnt;
      }
    }
  }
  *n_out = cnt;
  return cnt <= cap ? 0 : -1;
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/* The partners j > i of particle i in range, from the distinct cells around
 * i's cell, into *cand (grown as needed); returns -2 when out of memory. */
static int partners(const orc_params* p, const double* x, const double* d, int cx, int cy, int cz,
                    const int64_t* cell_of, const int64_t* start, const int64_t* members,
                    int64_t i, int64_t** cand, int64_t* cand_cap, int64_t* ncand) {
  int64_t ci = cell_of[i];
  int a0 = (int)(ci % cx), b0 = (int)((ci / cx) % cy), c0 = (int)(ci / ((int64_t)cx * cy));
  /* distinct neighbour cells (small grids would otherwise repeat a cell) */
  int64_t nb[27];
  int nnb = 0;
  for (int dc = -1; dc <= 1; ++dc) {
    int c = c0 + dc;
    if (c < 0 || c >= cz) continue;
    for (int db = -1; db <= 1; ++db) {
      int b = ((b0 + db) % cy + cy) % cy;
      for (int da = -1; da <= 1; ++da) {
        int a = ((a0 + da) % cx + cx) % cx;
        int64_t k = ((int64_t)c * cy + b) * cx + a;
        int seen = 0;
        for (int q = 0; q < nnb; ++q) seen |= (nb[q] == k);
        if (!seen) nb[nnb++] = k;
      }
    }
  }
  *ncand = 0;
  for (int q = 0; q < nnb; ++q) {
    for (int64_t m = start[nb[q]]; m < start[nb[q] + 1]; ++m) {
      int64_t j = members[m];
      if (j <= i) continue;
      if (!in_range(p, x + 3 * i, x + 3 * j, 0.5 * d[i], 0.5 * d[j])) continue;
      if (*ncand == *cand_cap) {
        int64_t nc = *cand_cap ? 2 * *cand_cap : 64;
        int64_t* t = (int64_t*)realloc(*cand, sizeof(int64_t) * nc);
        if (!t) return -2;
        *cand = t;
        *cand_cap = nc;
      }
      (*cand)[(*ncand)++] = j;
    }
  }
  return 0;
}

/* Link-cell search: a uniform grid whose cells are no smaller than the
 * largest possible pair range, so every partner of i lies in the 3x3x3 block
 * of cells around i's cell (wrapped on x, y; clipped on z). */
int orc_pairs_cells(const orc_params* p, int64_t n, const double* x, const double* d,
                    int64_t cap, int64_t* ij, int64_t* n_out) {
  *n_out = 0;
  if (n == 0) return 0;
  double dmax = 0.0;
  for (int64_t i = 0; i < n; ++i) dmax = d[i] > dmax ? d[i] : dmax;
  double range = dmax * (1.0 + p->lub_out_frac) * 1.000001;
  int cx, cy, cz;
  for (;;) { /* cells no smaller than the range; no more cells than ~4 per particle */
    cx = (int)floor(p->Lx / range), cy = (int)floor(p->Ly / range), cz = (int)floor(p->Lz / range);
    if (cx < 1) cx = 1;
    if (cy < 1) cy = 1;
    if (cz < 1) cz = 1;
    if ((double)cx * cy * cz <= 4.0 * (double)n + 64.0) break;
    range *= 1.25;
  }
  double hx = p->Lx / cx, hy = p->Ly / cy, hz = p->Lz / cz;
  int64_t ncell = (int64_t)cx * cy * cz;

  int64_t* cell_of = (int64_t*)malloc(sizeof(int64_t) * n);
  int64_t* start = (int64_t*)calloc(ncell + 1, sizeof(int64_t));
  int64_t* members = (int64_t*)malloc(sizeof(int64_t) * n);
  int64_t* fill = (int64_t*)calloc(ncell, sizeof(int64_t));
  if (!cell_of || !start || !members || !fill) {
    free(cell_of), free(start), free(members), free(fill);
    return -2;
  }
  for (int64_t i = 0; i < n; ++i) {
    int a = (int)floor(x[3 * i] / hx), b = (int)floor(x[3 * i + 1] / hy),
        c = (int)floor(x[3 * i + 2] / hz);
    a = a < 0 ? 0 : (a >= cx ? cx - 1 : a);
    b = b < 0 ? 0 : (b >= cy ? cy - 1 : b);
    c = c < 0 ? 0 : (c >= cz ? cz - 1 : c);
    cell_of[i] = ((int64_t)c * cy + b) * cx + a;
    start[cell_of[i] + 1]++;
  }
  for (int64_t k = 0; k < ncell; ++k) start[k + 1] += start[k];
  for (int64_t i = 0; i < n; ++i) members[start[cell_of[i]] + fill[cell_of[i]]++] = i;

  /* Each thread takes one contiguous block of particles (static schedule)
   * and lists its pairs, i ascending and each i's partners in ascending j,
   * in a buffer of its own; the buffers are then joined in thread order,
   * which is the order of a single pass over all particles. */
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  int64_t** buf = (int64_t**)calloc((size_t)nth, sizeof(int64_t*));
  int64_t* len = (int64_t*)calloc((size_t)nth, sizeof(int64_t));
  int oom = !buf || !len;
  if (!oom) {
#pragma omp parallel num_threads(nth) reduction(| : oom)
    {
      int t = 0;
#ifdef _OPENMP
      t = omp_get_thread_num();
#endif
      int64_t *cand = NULL, *out = NULL;
      int64_t cand_cap = 0, out_cap = 0, nout = 0;
#pragma omp for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        if (oom) continue;
        int64_t ncand = 0;
        if (partners(p, x, d, cx, cy, cz, cell_of, start, members, i, &cand, &cand_cap, &ncand)) {
          oom = 1;
          continue;
        }
        qsort(cand, (size_t)ncand, sizeof(int64_t), cmp_i64);
        if (nout + 2 * ncand > out_cap) {
          int64_t nc = out_cap ? 2 * out_cap : 1024;
          while (nc < nout + 2 * ncand) nc *= 2;
          int64_t* tmp = (int64_t*)realloc(out, sizeof(int64_t) * nc);
          if (!tmp) {
            oom = 1;
            continue;
          }
          out = tmp;
          out_cap = nc;
        }
        for (int64_t q = 0; q < ncand; ++q) {
          out[nout++] = i;
          out[nout++] = cand[q];
        }
      }
      free(cand);
      buf[t] = out;
      len[t] = nout / 2;
    }
  }
  int64_t cnt = 0;
  for (int t = 0; !oom && t < nth; ++t) {
    for (int64_t q = 0; q < len[t]; ++q, ++cnt)
      if (cnt < cap) {
        ij[2 * cnt] = buf[t][2 * q];
        ij[2 * cnt + 1] = buf[t][2 * q + 1];
      }
  }
  for (int t = 0; buf && t < nth; ++t) free(buf[t]);
  free(buf), free(len);
  if (oom) {
    free(cell_of), free(start), free(members), free(fill);
    return -2;
  }
  free(cell_of), free(start), free(members), free(fill);
  *n_out = cnt;
  return cnt <= cap ? 0 : -1;
}

void orc_set_threads(int nthreads) {
#ifdef _OPENMP
  omp_set_num_threads(nthreads > 0 ? nthreads : 1);
#else
  (void)nthreads;
#endif
}
int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

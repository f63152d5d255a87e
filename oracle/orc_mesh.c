/*
 * orc_mesh.c -- oracle mesh geometry along z.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Section 4's channel case refines the CFD mesh progressively towards the
 * bottom wall.  The grading is read as a geometric progression of cell
 * heights, h_k = h_0 q^k, with q^(nz-1) = z_grading, the ratio of the top
 * cell's height to the bottom cell's (the expansion-ratio convention of the
 * solver's mesh generator); z_grading <= 0 or = 1 is the uniform mesh, which
 * every routine handles on its own uniform path.
 */
#include "orc.h"

#include <math.h>

int orc_graded(const orc_params* p) {
  return p->nz > 1 && p->z_grading > 0.0 && p->z_grading != 1.0;
}

void orc_z_faces(const orc_params* p, double* zf) {
  const int nz = p->nz;
  zf[0] = 0.0;
  if (!orc_graded(p)) {
    for (int k = 1; k <= nz; ++k) zf[k] = p->Lz * k / nz;
    return;
  }
  /* relative heights q^k = z_grading^(k/(nz-1)), summed in order and scaled
   * to Lz (the closed form of the geometric sum, (q^nz - 1)/(q - 1), cancels
   * as the grading tends to 1) */
  double sum = 0.0;
  for (int k = 0; k < nz; ++k) sum += pow(p->z_grading, (double)k / (nz - 1));
  const double scale = p->Lz / sum;
  for (int k = 1; k <= nz; ++k)
    zf[k] = zf[k - 1] + pow(p->z_grading, (double)(k - 1) / (nz - 1)) * scale;
  zf[nz] = p->Lz;
}

int orc_z_cell(const double* zf, int nz, double z) {
  /* the cell whose [zf[k], zf[k+1]) holds z; a centre on a face belongs to
   * the upper cell; outside the mesh: the first / last cell */
  if (!(z >= zf[0])) return 0;
  if (z >= zf[nz]) return nz - 1;
  int lo = 0, hi = nz; /* zf[lo] <= z < zf[hi] */
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (zf[mid] <= z)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

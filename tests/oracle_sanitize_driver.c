/*
 * Exercises every oracle entry point on a small bed, for a build with the
 * host AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure,
 * see test_oracle_sanitizers.py).  Inputs are seeded and synthetic; the run
 * prints "ok" and exits 0 unless a sanitizer or an oracle return code
 * reports a problem.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "orc.h"

/* the network routines have no header of their own */
void orc_conv3d_fwd(int nx, int ny, int nz, int cin, int cout, int dil, const double* x,
                    const double* w, const double* b, double* y);
void orc_conv3d_bwd(int nx, int ny, int nz, int cin, int cout, int dil, const double* x,
                    const double* w, const double* dy, double* dx, double* dw, double* db);
int64_t orc_nn_param_count(int C);
double orc_nn_loss_grad(int nx, int ny, int nz, int C, double alpha, int bf16,
                        const double* params, const double* split, const double* lw,
                        const double* x, const double* target, double* grads);
void orc_adam(int64_t n, double* w, double* m, double* v, const double* g, double lr,
              double b1, double b2, double eps, int64_t t);

static uint64_t rng_state = 0x2545F4914F6CDD1Dull;
static double uniform(void) { /* xorshift64* */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (double)((rng_state * 0x2545F4914F6CDD1Dull) >> 11) * 0x1.0p-53;
}

static double* vec(size_t n) {
  double* p = (double*)calloc(n ? n : 1, sizeof(double));
  if (!p) {
    fprintf(stderr, "allocation failed\n");
    exit(2);
  }
  return p;
}

#define CHECK(call)                                          \
  do {                                                       \
    int rc_ = (call);                                        \
    if (rc_ != 0) {                                          \
      fprintf(stderr, "%s returned %d\n", #call, rc_);       \
      return 1;                                              \
    }                                                        \
  } while (0)

int main(void) {
  const int64_t n = 1500;
  const double D = 0.5e-3;
  orc_params p;
  memset(&p, 0, sizeof(p));
  p.Lx = 20 * D, p.Ly = 20 * D, p.Lz = 12 * D;
  p.nx = 8, p.ny = 8, p.nz = 6;
  p.kn = 1e3, p.restitution = 0.9, p.friction = 0.3, p.kt_over_kn = 2.0 / 7.0;
  p.lub_out_frac = 0.05, p.lub_in_frac = 0.001;
  p.rho_f = 1000.0, p.mu_f = 1e-3, p.c_add = 0.5, p.gz = -9.81, p.dt = 1e-6;
  p.drag_law = ORC_DRAG_SYAMLAL, p.lubrication = 1, p.fluid_forces = 1;
  p.bottom_wall = 1, p.top_wall = 1, p.eps_s_max = 0.7;
  p.avg_bandwidth = 3 * D, p.avg_ntau = 4, p.cg_rtol = 1e-12;
  p.avg_bandwidth_z = 2 * D, p.c_lift = 1.6, p.avg_scheme = ORC_SCHEME_BDF2;
  const int64_t ncell = (int64_t)p.nx * p.ny * p.nz;

  double *x = vec(3 * n), *v = vec(3 * n), *w = vec(3 * n), *a = vec(3 * n), *al = vec(3 * n);
  double *d = vec(n), *rho = vec(n), *fd = vec(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    d[i] = D * (0.7 + 0.6 * uniform());
    rho[i] = 2650.0;
    x[3 * i] = p.Lx * uniform();
    x[3 * i + 1] = p.Ly * uniform();
    x[3 * i + 2] = 0.5 * d[i] + (p.Lz - d[i]) * uniform();
    for (int k = 0; k < 3; ++k) {
      v[3 * i + k] = 0.01 * (uniform() - 0.5);
      w[3 * i + k] = 20.0 * (uniform() - 0.5);
    }
  }
  double *U = vec(3 * ncell), *gp = vec(3 * ncell), *du = vec(3 * ncell), *es = vec(ncell);
  for (int64_t c = 0; c < ncell; ++c) {
    for (int k = 0; k < 3; ++k) {
      U[3 * c + k] = 0.05 * (uniform() - 0.5);
      gp[3 * c + k] = k == 2 ? -9810.0 : 0.0;
      du[3 * c + k] = 0.1 * (uniform() - 0.5);
    }
    es[c] = 0.6 * uniform();
  }

  /* pair sets: brute force and cell list agree */
  const int64_t cap = 64 * n;
  int64_t *ij1 = (int64_t*)calloc(2 * cap, sizeof(int64_t)), *ij2 = (int64_t*)calloc(2 * cap, sizeof(int64_t));
  int64_t np1 = 0, np2 = 0;
  CHECK(orc_pairs_brute(&p, n, x, d, cap, ij1, &np1));
  CHECK(orc_pairs_cells(&p, n, x, d, cap, ij2, &np2));
  if (np1 != np2) {
    fprintf(stderr, "pair counts differ: %lld vs %lld\n", (long long)np1, (long long)np2);
    return 1;
  }

  /* one force evaluation with every component */
  orc_fields fl = {U, gp, du, es};
  double* comp[8];
  for (int k = 0; k < 8; ++k) comp[k] = vec(3 * n);
  orc_forces_out out = {comp[0], comp[1], comp[2], comp[3], comp[4], comp[5], comp[6], comp[7]};
  orc_contact* hist = (orc_contact*)calloc(16 * n + 64, sizeof(orc_contact));
  int64_t nh = 0;
  CHECK(orc_forces(&p, n, x, v, w, d, rho, NULL, &fl, NULL, 0, hist, 16 * n + 64, &nh, &out));

  /* a short run with averaging (BDF2, anisotropic bandwidth, lift) */
  double* avg = vec(4 * ncell);
  int64_t nhist = 0, step = 0;
  CHECK(orc_init_accel(&p, n, x, v, w, a, al, d, rho, fd, U, gp, du, es, NULL, 0));
  CHECK(orc_run(&p, n, x, v, w, a, al, d, rho, fd, U, gp, du, es, avg, hist, 16 * n + 64,
                &nhist, &step, 12, 4));

  /* deposition, flux, both schemes, solid velocity, the operator */
  double *raw = vec(7 * ncell), *sm = vec(7 * ncell), *us = vec(3 * ncell), *ax = vec(ncell);
  int64_t iters = 0;
  CHECK(orc_deposit(&p, n, x, d, fd, raw));
  CHECK(orc_deposit_flux(&p, n, x, d, v, raw + 4 * ncell));
  for (int scheme = 0; scheme < 2; ++scheme) {
    p.avg_scheme = scheme;
    CHECK(orc_diffuse(&p, 7, raw, sm, &iters));
  }
  orc_solid_velocity(ncell, sm, sm + 4 * ncell, us);
  orc_apply_A(&p, 1e-8, sm, ax);
  p.avg_ntau = 0;
  CHECK(orc_diffuse(&p, 1, raw, sm, &iters));

  /* the same on a z mesh graded towards the bottom */
  p.z_grading = 5.0, p.avg_ntau = 3, p.avg_scheme = ORC_SCHEME_EULER;
  CHECK(orc_deposit(&p, n, x, d, fd, raw));
  CHECK(orc_deposit_flux(&p, n, x, d, v, raw + 4 * ncell));
  CHECK(orc_diffuse(&p, 7, raw, sm, &iters));
  nh = 0;
  CHECK(orc_forces(&p, n, x, v, w, d, rho, NULL, &fl, NULL, 0, hist, 16 * n + 64, &nh, &out));

  /* network: one conv forward / backward, the loss gradient, an Adam step */
  const int mx = 5, my = 4, mz = 6, C = 4;
  const int64_t m = (int64_t)mx * my * mz;
  double *cx = vec(m * C), *cw = vec(27 * C * C), *cb = vec(C), *cy = vec(m * C);
  double *cdx = vec(m * C), *cdw = vec(27 * C * C), *cdb = vec(C);
  for (int64_t k = 0; k < m * C; ++k) cx[k] = uniform() - 0.5;
  for (int64_t k = 0; k < 27 * C * C; ++k) cw[k] = 0.1 * (uniform() - 0.5);
  orc_conv3d_fwd(mx, my, mz, C, C, 2, cx, cw, cb, cy);
  orc_conv3d_bwd(mx, my, mz, C, C, 2, cx, cw, cy, cdx, cdw, cdb);
  const int64_t np = orc_nn_param_count(8);
  double *prm = vec(np), *g = vec(np), *mm = vec(np), *vv = vec(np), *tgt = vec(m * 4);
  for (int64_t k = 0; k < np; ++k) prm[k] = 0.05 * (uniform() - 0.5);
  for (int64_t k = 0; k < m * 4; ++k) tgt[k] = uniform();
  const double split[4] = {0.06, 0.05, 2.25, 4.0};
  const double lw[4] = {1.0, 0.5, 2.0, 1.0};
  double loss = orc_nn_loss_grad(mx, my, mz, 8, 0.1, 1, prm, split, lw, cx, tgt, g);
  orc_adam(np, prm, mm, vv, g, 1e-3, 0.9, 0.999, 1e-8, 1);
  if (!isfinite(loss)) {
    fprintf(stderr, "non-finite loss\n");
    return 1;
  }

  free(x), free(v), free(w), free(a), free(al), free(d), free(rho), free(fd);
  free(U), free(gp), free(du), free(es), free(ij1), free(ij2), free(hist), free(avg);
  for (int k = 0; k < 8; ++k) free(comp[k]);
  free(raw), free(sm), free(us), free(ax);
  free(cx), free(cw), free(cb), free(cy), free(cdx), free(cdw), free(cdb);
  free(prm), free(g), free(mm), free(vv), free(tgt);
  printf("ok %lld pairs, %lld contacts, %lld steps\n", (long long)np1, (long long)nhist,
         (long long)step);
  return 0;
}

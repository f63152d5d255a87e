/*
 * orc_cnn.c -- oracle for the learned stand-in of the diffusion averaging:
 * a 6-layer 3-D convolutional network mapping the deposited fields (Eq. 11,
 * 4 channels) to the smoothed ones (Eq. 12).  TEST INFRASTRUCTURE ONLY (see
 * orc.h).  The network is not part of the paper; its definition here is the
 * reference the GPU kernels are checked against:
 *
 *   conv(x)[c][o] = b[o] + sum_t sum_i x[nb(c, t)][i] * w[t][i][o]
 *     taps t = (dz + 1)*9 + (dy + 1)*3 + (dx + 1), dz, dy, dx in {-1, 0, 1};
 *     nb(c, t) = cell (i + dx, j + dy, R(k + dil*dz)), periodic in x and y;
 *     in z the field is extended by reflection about the wall faces (mirror
 *     padding: plane -1 is plane 0, plane nz is plane nz-1, repeated with
 *     period 2 nz), the even extension that matches the zero-flux walls of
 *     the diffusion it stands in for;
 *   layer 1: h1 = phi(conv1(x - S x))                  (4 -> C channels)
 *   layers 2..5: h_l = h_{l-1} + phi(conv_l(h_{l-1}))  (C -> C)
 *   layer 6: y = S x + conv6(h5)                       (C -> 4)
 *   S, the global skip, is the diffusion of Eq. (12) split by axis: each of
 *   the N backward-Euler steps (I - dtau L)^-1 replaced by the product of the
 *   three one-dimensional implicit steps (I - c_x D_x)^-1 (I - c_y D_y)^-1
 *   (I - c_z D_z)^-1, c_a = dtau D_a / h_a^2, D_a the second difference
 *   (periodic in x, y; zero flux at the z walls), each solved exactly.  The
 *   one-dimensional operators commute, so S = S_x^N S_y^N S_z^N.  It
 *   differs from the exact steps only by the cross terms of the product
 *   (c_x c_z D_x D_z ...), so the network learns that small non-separable
 *   remainder, from the part of the field that S smooths away, x - S x;
 *   with no split given, S is the identity and the network reads x;
 *   phi = leaky ReLU with slope `alpha` for negative arguments;
 *   dilations along z: 1, 2, 4, 4, 2, 1.
 *   loss = mean over cells and channels of w_ch (y - target)^2 (channel
 *   weights w, 1 unless given).
 *
 * Arrays are channel-last, [cell][channel], cell = (k*ny + j)*nx + i.
 * Weights of all layers are packed in one vector: for each layer its
 * w[27][cin][cout] then b[cout].  With bf16 != 0 every stored activation
 * (h_l, and the pre-activations kept for the backward pass) and every
 * stored gradient tensor is rounded to the nearest bfloat16 (ties to even),
 * the storage precision of the GPU kernels; sums are always FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const int DIL[6] = {1, 2, 4, 4, 2, 1};

static double bf16_round(double v) {
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return v; /* inf / nan unchanged */
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

static int64_t nbr(int nx, int ny, int nz, int64_t c, int t, int dil) {
  int i = (int)(c % nx);
  int j = (int)((c / nx) % ny);
  int k = (int)(c / ((int64_t)nx * ny));
  int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  /* reflection into [0, nz): the even extension about both wall faces */
  int kk = (k + dil * dz) % (2 * nz);
  if (kk < 0) kk += 2 * nz;
  if (kk >= nz) kk = 2 * nz - 1 - kk;
  int ii = ((i + dx) % nx + nx) % nx;
  int jj = ((j + dy) % ny + ny) % ny;
  return ((int64_t)kk * ny + jj) * nx + ii;
}

/* y[c][o] = b[o] + sum_t sum_i x[nb(c,t)][i] w[t][i][o] */
void orc_conv3d_fwd(int nx, int ny, int nz, int cin, int cout, int dil, const double* x,
                    const double* w, const double* b, double* y) {
  int64_t n = (int64_t)nx * ny * nz;
  for (int64_t c = 0; c < n; ++c) {
    for (int o = 0; o < cout; ++o) y[c * cout + o] = b ? b[o] : 0.0;
    for (int t = 0; t < 27; ++t) {
      const int64_t q = nbr(nx, ny, nz, c, t, dil);
      for (int i = 0; i < cin; ++i) {
        double xv = x[q * cin + i];
        for (int o = 0; o < cout; ++o) y[c * cout + o] += xv * w[((int64_t)t * cin + i) * cout + o];
      }
    }
  }
}

/* Gradients of the convolution: dx (may be NULL), dw, db (accumulated into,
 * the caller zeroes them). */
void orc_conv3d_bwd(int nx, int ny, int nz, int cin, int cout, int dil, const double* x,
                    const double* w, const double* dy, double* dx, double* dw, double* db) {
  int64_t n = (int64_t)nx * ny * nz;
  if (dx) memset(dx, 0, sizeof(double) * (size_t)(n * cin));
  for (int64_t c = 0; c < n; ++c) {
    for (int o = 0; o < cout; ++o) db[o] += dy[c * cout + o];
    for (int t = 0; t < 27; ++t) {
      const int64_t q = nbr(nx, ny, nz, c, t, dil);
      for (int i = 0; i < cin; ++i) {
        double acc = 0.0;
        for (int o = 0; o < cout; ++o) {
          double g = dy[c * cout + o];
          dw[((int64_t)t * cin + i) * cout + o] += x[q * cin + i] * g;
          acc += w[((int64_t)t * cin + i) * cout + o] * g;
        }
        if (dx) dx[q * cin + i] += acc;
      }
    }
  }
}

/* One implicit step along a line of n values with stride st:
 * solves (1 + 2c) u_i - c u_{i-1} - c u_{i+1} = f_i in place, periodic
 * (cyclic tridiagonal, by the Sherman-Morrison correction of the tridiagonal
 * solve) or with zero-flux ends (u_{-1} = u_0, u_n = u_{n-1}). */
static void line_step(double* f, int n, int64_t st, double c, int periodic, double* w) {
  double* gam = w;      /* n: modified super-diagonal */
  double* u = w + n;    /* n */
  double* z = w + 2 * n; /* n */
  if (n == 1) return;   /* a single cell: no neighbour, nothing diffuses */
  if (!periodic) {
    /* Thomas algorithm; diagonal 1 + c at the ends */
    double b0 = 1.0 + c;
    double bet = b0;
    u[0] = f[0] / bet;
    for (int i = 1; i < n; ++i) {
      gam[i] = -c / bet;
      double bi = (i == n - 1) ? 1.0 + c : 1.0 + 2.0 * c;
      bet = bi - (-c) * gam[i];
      u[i] = (f[(int64_t)i * st] - (-c) * u[i - 1]) / bet;
    }
    for (int i = n - 2; i >= 0; --i) u[i] -= gam[i + 1] * u[i + 1];
    for (int i = 0; i < n; ++i) f[(int64_t)i * st] = u[i];
    return;
  }
  if (n == 2) {
    /* both neighbours of a cell are the other cell: [[1+2c, -2c], [-2c, 1+2c]] */
    double a = 1.0 + 2.0 * c, b = -2.0 * c, det = a * a - b * b;
    double f0 = f[0], f1 = f[st];
    f[0] = (a * f0 - b * f1) / det;
    f[st] = (a * f1 - b * f0) / det;
    return;
  }
  /* cyclic: A = T + w v^T with T tridiagonal (corners folded into the first
   * and last diagonal entries), w = (g, 0, .., 0, -c), v = (1, 0, .., 0, -c/g)
   * with g = -(1 + 2c) */
  const double diag = 1.0 + 2.0 * c, off = -c, g = -diag;
  /* solve T u = f and T z = w with the same factorisation */
  double bet = diag - g;
  u[0] = f[0] / bet;
  z[0] = g / bet;
  for (int i = 1; i < n; ++i) {
    gam[i] = off / bet;
    double bi = (i == n - 1) ? diag - off * off / g : diag;
    bet = bi - off * gam[i];
    double wi = (i == n - 1) ? off : 0.0;
    u[i] = (f[(int64_t)i * st] - off * u[i - 1]) / bet;
    z[i] = (wi - off * z[i - 1]) / bet;
  }
  for (int i = n - 2; i >= 0; --i) {
    u[i] -= gam[i + 1] * u[i + 1];
    z[i] -= gam[i + 1] * z[i + 1];
  }
  /* v = (1, 0, ..., 0, off / g) */
  const double vu = u[0] + off / g * u[n - 1], vz = z[0] + off / g * z[n - 1];
  const double fac = vu / (1.0 + vz);
  for (int i = 0; i < n; ++i) f[(int64_t)i * st] = u[i] - fac * z[i];
}

/* out = S in, channel-last [n][nchan]: N steps of the three exact
 * one-dimensional implicit steps (c[0..2] = c_x, c_y, c_z; c[3] = N). */
void orc_split_smooth(int nx, int ny, int nz, int nchan, const double* c, const double* in,
                      double* out) {
  const int64_t n = (int64_t)nx * ny * nz;
  memcpy(out, in, sizeof(double) * (size_t)(n * nchan));
  const int N = (int)c[3];
  int m = nx > ny ? nx : ny;
  m = m > nz ? m : nz;
  double* w = (double*)malloc(sizeof(double) * 3 * (size_t)m);
  for (int step = 0; step < N; ++step)
    for (int ch = 0; ch < nchan; ++ch) {
      for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
          line_step(out + (((int64_t)k * ny + j) * nx) * nchan + ch, nx, nchan, c[0], 1, w);
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i)
          line_step(out + (((int64_t)k * ny) * nx + i) * nchan + ch, ny, (int64_t)nx * nchan,
                    c[1], 1, w);
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
          line_step(out + ((int64_t)j * nx + i) * nchan + ch, nz, (int64_t)nx * ny * nchan, c[2],
                    0, w);
    }
  free(w);
}

int64_t orc_nn_param_count(int C) {
  int64_t p = 0;
  for (int l = 0; l < 6; ++l) {
    int cin = l == 0 ? 4 : C, cout = l == 5 ? 4 : C;
    p += 27LL * cin * cout + cout;
  }
  return p;
}

static void layer_shapes(int C, int l, int* cin, int* cout) {
  *cin = l == 0 ? 4 : C;
  *cout = l == 5 ? 4 : C;
}

static double* wptr(const double* params, int C, int l, double** bias) {
  int64_t off = 0;
  for (int q = 0; q < l; ++q) {
    int ci, co;
    layer_shapes(C, q, &ci, &co);
    off += 27LL * ci * co + co;
  }
  int ci, co;
  layer_shapes(C, l, &ci, &co);
  if (bias) *bias = (double*)params + off + 27LL * ci * co;
  return (double*)params + off;
}

/* Forward pass.  x [n][4] (normalised input), y [n][4] output.  If `keep`
 * is non-NULL it receives the tensors the backward pass needs, laid out as
 * z1..z5 (pre-activations, [n][C] each) then h1..h5 ([n][C] each).  split:
 * NULL (identity skip) or {c_x, c_y, c_z, N} of the skip S. */
void orc_nn_forward(int nx, int ny, int nz, int C, double alpha, int bf16, const double* params,
                    const double* split, const double* x, double* y, double* keep) {
  int64_t n = (int64_t)nx * ny * nz;
  double* z = (double*)malloc(sizeof(double) * (size_t)(n * C));
  double* h = (double*)malloc(sizeof(double) * (size_t)(n * C));
  double* xin = (double*)malloc(sizeof(double) * (size_t)(n * 4));
  double* sx = (double*)malloc(sizeof(double) * (size_t)(n * 4));
  if (split)
    orc_split_smooth(nx, ny, nz, 4, split, x, sx);
  else
    memset(sx, 0, sizeof(double) * (size_t)(n * 4));
  for (int64_t k = 0; k < n * 4; ++k) {
    const double v = split ? x[k] - sx[k] : x[k];
    xin[k] = bf16 ? bf16_round(v) : v;
  }
  for (int l = 0; l < 5; ++l) {
    double* b;
    double* w = wptr(params, C, l, &b);
    int ci, co;
    layer_shapes(C, l, &ci, &co);
    orc_conv3d_fwd(nx, ny, nz, ci, co, DIL[l], l == 0 ? xin : h, w, b, z);
    for (int64_t k = 0; k < n * C; ++k) {
      double zz = bf16 ? bf16_round(z[k]) : z[k];
      z[k] = zz;
      double a = zz > 0.0 ? zz : alpha * zz;
      double hv = l == 0 ? a : h[k] + a;
      h[k] = bf16 ? bf16_round(hv) : hv;
    }
    if (keep) {
      memcpy(keep + (size_t)l * n * C, z, sizeof(double) * (size_t)(n * C));
      memcpy(keep + (size_t)(5 + l) * n * C, h, sizeof(double) * (size_t)(n * C));
    }
  }
  double* b;
  double* w = wptr(params, C, 5, &b);
  orc_conv3d_fwd(nx, ny, nz, C, 4, DIL[5], h, w, b, y);
  for (int64_t k = 0; k < n * 4; ++k) y[k] += split ? sx[k] : x[k];
  free(z), free(h), free(xin), free(sx);
}

/* Loss and gradients with respect to all parameters (grads, same layout). */
double orc_nn_loss_grad(int nx, int ny, int nz, int C, double alpha, int bf16,
                        const double* params, const double* split, const double* lw,
                        const double* x, const double* target, double* grads) {
  int64_t n = (int64_t)nx * ny * nz;
  double* keep = (double*)malloc(sizeof(double) * (size_t)(10 * n * C));
  double* y = (double*)malloc(sizeof(double) * (size_t)(n * 4));
  orc_nn_forward(nx, ny, nz, C, alpha, bf16, params, split, x, y, keep);
  double loss = 0.0;
  double* dy = (double*)malloc(sizeof(double) * (size_t)(n * 4));
  for (int64_t k = 0; k < n * 4; ++k) {
    const double e = y[k] - target[k], wk = lw ? lw[k % 4] : 1.0;
    loss += wk * e * e;
    double g = 2.0 * wk * e / (double)(n * 4);
    dy[k] = bf16 ? bf16_round(g) : g;
  }
  loss /= (double)(n * 4);
  memset(grads, 0, sizeof(double) * (size_t)orc_nn_param_count(C));
  double* dh = (double*)malloc(sizeof(double) * (size_t)(n * C));
  double* dz = (double*)malloc(sizeof(double) * (size_t)(n * C));
  double* tmp = (double*)malloc(sizeof(double) * (size_t)(n * C));
  double* xin = (double*)malloc(sizeof(double) * (size_t)(n * 4));
  if (split) orc_split_smooth(nx, ny, nz, 4, split, x, xin);
  for (int64_t k = 0; k < n * 4; ++k) {
    const double v = split ? x[k] - xin[k] : x[k];
    xin[k] = bf16 ? bf16_round(v) : v;
  }
  /* layer 6 */
  {
    double *b, *gb;
    double* w = wptr(params, C, 5, &b);
    double* gw = wptr(grads, C, 5, &gb);
    orc_conv3d_bwd(nx, ny, nz, C, 4, DIL[5], keep + (size_t)9 * n * C, w, dy, dh, gw, gb);
    for (int64_t k = 0; k < n * C; ++k) dh[k] = bf16 ? bf16_round(dh[k]) : dh[k];
  }
  for (int l = 4; l >= 0; --l) {
    const double* z = keep + (size_t)l * n * C;
    for (int64_t k = 0; k < n * C; ++k) {
      double g = dh[k] * (z[k] > 0.0 ? 1.0 : alpha);
      dz[k] = bf16 ? bf16_round(g) : g;
    }
    double *b, *gb;
    double* w = wptr(params, C, l, &b);
    double* gw = wptr(grads, C, l, &gb);
    int ci, co;
    layer_shapes(C, l, &ci, &co);
    const double* hin = l == 0 ? xin : keep + (size_t)(5 + l - 1) * n * C;
    orc_conv3d_bwd(nx, ny, nz, ci, co, DIL[l], hin, w, dz, l == 0 ? NULL : tmp, gw, gb);
    if (l > 0) {
      /* residual path: dh_{l-1} = dh_l + conv^T(dz_l) */
      for (int64_t k = 0; k < n * C; ++k) {
        double g = dh[k] + tmp[k];
        dh[k] = bf16 ? bf16_round(g) : g;
      }
    }
  }
  free(keep), free(y), free(dy), free(dh), free(dz), free(tmp), free(xin);
  return loss;
}

/* One Adam step (Kingma & Ba) on n parameters; t is the 1-based step. */
void orc_adam(int64_t n, double* w, double* m, double* v, const double* g, double lr,
              double b1, double b2, double eps, int64_t t) {
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t k = 0; k < n; ++k) {
    m[k] = b1 * m[k] + (1.0 - b1) * g[k];
    v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
    double mh = m[k] / c1, vh = v[k] / c2;
    w[k] -= lr * mh / (sqrt(vh) + eps);
  }
}

// Drives the C ABI's host-side paths (parameter checks, workspace sizing,
// calls before a workspace, state-blob checks, error strings, null handling)
// in a build whose host code carries AddressSanitizer and UBSan; no call
// reaches a kernel.  Prints "ok" and exits 0 unless a sanitizer reports or a
// return code differs from the documented one.
#include <cstdio>
#include <cstring>

#include "sedimi.h"

static int failures = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      std::fprintf(stderr, "line %d: %s\n", __LINE__, #cond);     \
      ++failures;                                                 \
    }                                                             \
  } while (0)

static sedimi_params base() {
  sedimi_params p;
  std::memset(&p, 0, sizeof(p));
  p.Lx = 0.01, p.Ly = 0.01, p.Lz = 0.005, p.nx = 16, p.ny = 16, p.nz = 8;
  p.kn = 1e3, p.restitution = 0.9, p.friction = 0.3, p.kt_over_kn = 2.0 / 7.0;
  p.lub_out_frac = 0.05, p.lub_in_frac = 0.001;
  p.rho_f = 1000, p.mu_f = 1e-3, p.c_add = 0.5, p.gz = -9.81, p.dt = 1e-5;
  p.drag_law = SEDIMI_DRAG_DIFELICE, p.lubrication = 1, p.fluid_forces = 1;
  p.bottom_wall = 1, p.top_wall = 1, p.eps_s_max = 0.7;
  p.avg_bandwidth = 1.5e-3, p.avg_ntau = 4, p.avg_rtol = 1e-12;
  p.d_max = 0.5e-3, p.skin = 0.05e-3, p.max_neighbors = 24;
  return p;
}

int main() {
  sedimi_ctx* c = nullptr;
  sedimi_params p = base();
  EXPECT(sedimi_create(&p, 1000, &c) == SEDIMI_OK && c);
  const size_t ws = sedimi_workspace_bytes(c);
  EXPECT(ws > 0);
  // calls before a workspace
  EXPECT(sedimi_step(c, 1, 0) == SEDIMI_ENOMEM);
  EXPECT(std::strstr(sedimi_last_error(c), "workspace") != nullptr);
  EXPECT(sedimi_average(c) == SEDIMI_ENOMEM);
  EXPECT(sedimi_smooth(c, 4) == SEDIMI_ENOMEM);
  size_t sz = 0;
  EXPECT(sedimi_get_state(c, nullptr, 0, &sz) == SEDIMI_ENOMEM);
  EXPECT(sedimi_set_state(c, nullptr, 0) == SEDIMI_ENOMEM);
  sedimi_stats st;
  EXPECT(sedimi_get_stats(c, &st) == SEDIMI_ENOMEM);
  double buf[3] = {0, 0, 0};
  EXPECT(sedimi_get_field(c, SEDIMI_FIELD_US, buf) == SEDIMI_ENOMEM);
  EXPECT(sedimi_bind_workspace(c, reinterpret_cast<void*>(0x1001), 1 << 20) == SEDIMI_EINVAL);
  EXPECT(sedimi_bind_workspace(c, reinterpret_cast<void*>(0x100000), 16) == SEDIMI_ENOMEM);
  sedimi_destroy(c);
  // each rejected parameter set leaves no context behind
  struct Bad {
    const char* what;
    void (*set)(sedimi_params&);
  } bad[] = {
      {"nx", [](sedimi_params& q) { q.nx = 0; }},
      {"Lx", [](sedimi_params& q) { q.Lx = -1; }},
      {"restitution", [](sedimi_params& q) { q.restitution = 1.5; }},
      {"drag", [](sedimi_params& q) { q.drag_law = 99; }},
      {"lift", [](sedimi_params& q) { q.c_lift = -1; }},
      {"bandwidth_z", [](sedimi_params& q) { q.avg_bandwidth_z = -1; }},
      {"scheme", [](sedimi_params& q) { q.avg_scheme = 7; }},
      {"bdf2+nn", [](sedimi_params& q) { q.avg_scheme = SEDIMI_SCHEME_BDF2; q.nn_enable = 1; }},
      {"us+nn", [](sedimi_params& q) { q.avg_solid_velocity = 1; q.nn_enable = 1; }},
      {"slots", [](sedimi_params& q) { q.max_neighbors = 0; }},
      {"narrow", [](sedimi_params& q) { q.Lx = 2 * q.d_max; }},
      {"grading<0", [](sedimi_params& q) { q.z_grading = -1.0; }},
      {"graded+nn", [](sedimi_params& q) { q.z_grading = 4.0; q.nn_enable = 1; }},
  };
  for (const Bad& b : bad) {
    sedimi_params q = base();
    b.set(q);
    sedimi_ctx* d = nullptr;
    const int rc = sedimi_create(&q, 1000, &d);
    if (rc != SEDIMI_EINVAL || d) {
      std::fprintf(stderr, "%s: rc %d\n", b.what, rc);
      ++failures;
    }
    if (d) sedimi_destroy(d);
  }
  // every option on: creation and sizing only
  sedimi_params q = base();
  q.c_lift = 1.6, q.avg_solid_velocity = 1, q.avg_scheme = SEDIMI_SCHEME_BDF2;
  q.avg_solver = SEDIMI_SOLVE_ITERATIVE, q.drag_law = SEDIMI_DRAG_SYAMLAL;
  EXPECT(sedimi_create(&q, 5000, &c) == SEDIMI_OK);
  EXPECT(sedimi_workspace_bytes(c) > ws);
  sedimi_destroy(c);
  c = nullptr;
  // graded z meshes: the direct solve's eigen-decomposition runs at creation
  for (int nz : {2, 8, 64}) {
    sedimi_params g = base();
    g.z_grading = 5.0, g.nz = nz, g.avg_solver = SEDIMI_SOLVE_DIRECT;
    EXPECT(sedimi_create(&g, 1000, &c) == SEDIMI_OK && c);
    sedimi_destroy(c);
    c = nullptr;
  }
  EXPECT(sedimi_create(&p, -1, &c) == SEDIMI_EINVAL);
  if (c) sedimi_destroy(c);
  EXPECT(sedimi_step(nullptr, 1, 0) == SEDIMI_EINVAL);
  EXPECT(std::strcmp(sedimi_last_error(nullptr), "null context") == 0);
  sedimi_destroy(nullptr);
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}

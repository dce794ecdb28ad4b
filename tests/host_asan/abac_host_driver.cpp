// Exercises the host side of the C ABI (include/abac.h) end to end: plan creation with
// library- and caller-owned workspaces, the operators, synchronous and asynchronous
// MINRES, GMRES, a variable coefficient, tile overrides, kernel timing, groups (one launch
// per step and persistent), the request server with its group lane, the allocation-free
// P^{-1} entry point, and the argument checks of each.  Built with the host code of the library under
// AddressSanitizer (device code is not instrumented), it turns any out-of-bounds,
// use-after-free or double free in the host layer into a report and a non-zero exit.
// Prints HOST_DRIVER_OK when every call returned what it should.
#include <hip/hip_runtime.h>
#include <sanitizer/lsan_interface.h>
#include <unistd.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/abac.h"

static int g_fail = 0;

#define EXPECT(cond)                                                              \
  do {                                                                            \
    if (!(cond)) {                                                                \
      std::fprintf(stderr, "FAILED %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond,  \
                   abac_last_error());                                            \
      ++g_fail;                                                                   \
    }                                                                             \
  } while (0)

#define HIP_OK(call) EXPECT((call) == hipSuccess)

struct Dev {
  double* p = nullptr;
  explicit Dev(size_t n) { HIP_OK(hipMalloc(reinterpret_cast<void**>(&p), n * sizeof(double))); }
  ~Dev() { HIP_OK(hipFree(p)); }
};

// Right-hand side from a seeded N(0,1) source with zero initial data.
static void make_rhs(abac_plan* p, int nx, int ny, int nt, int batch, unsigned long long seed, double* f) {
  const size_t m = (size_t)nx * (ny ? ny : 1), N = m * nt;
  Dev src(batch * N), z(batch * m);
  EXPECT(abac_fill_normal(nullptr, src.p, batch * N, seed) == ABAC_OK);
  HIP_OK(hipMemset(z.p, 0, batch * m * sizeof(double)));
  EXPECT(abac_build_rhs(p, src.p, z.p, z.p, f) == ABAC_OK);
  HIP_OK(hipDeviceSynchronize());
}

static void argument_checks() {
  abac_plan* p = nullptr;
  EXPECT(abac_workspace_bytes(63, 0, 64, ABAC_PREC_FP64, 1) > 0);
  EXPECT(abac_workspace_bytes(10, 0, 64, ABAC_PREC_FP64, 1) == 0);    // nx + 1 not a power of two
  EXPECT(abac_workspace_bytes(63, 0, 64, ABAC_PREC_FP64, 0) == 0);    // batch 0
  EXPECT(abac_plan_create(10, 0, 64, 1.0, 1e-3, ABAC_PREC_FP64, 1, nullptr, nullptr, 0, &p) == ABAC_EINVAL);
  EXPECT(abac_plan_create(63, 0, 64, 1.0, 0.0, ABAC_PREC_FP64, 1, nullptr, nullptr, 0, &p) == ABAC_EINVAL);
  EXPECT(abac_plan_create(63, 0, 64, -1.0, 1e-3, ABAC_PREC_FP64, 1, nullptr, nullptr, 0, &p) == ABAC_EINVAL);
  EXPECT(abac_plan_create(63, 0, 64, 1.0, 1e-3, ABAC_PREC_FP64, 1, nullptr, nullptr, 0, nullptr) == ABAC_EINVAL);
  EXPECT(abac_plan_destroy(nullptr) == ABAC_OK);                       // like free(NULL)
  EXPECT(abac_status_string(ABAC_EBUDGET) != nullptr);
}

static void solve_1d() {
  const int nx = 255, nt = 64, B = 2;
  abac_plan* p = nullptr;
  EXPECT(abac_plan_create(nx, 0, nt, 1.0, 1e-3, ABAC_PREC_FP64, B, nullptr, nullptr, 0, &p) == ABAC_OK);
  if (!p) return;
  const size_t N = (size_t)nx * nt;
  Dev f(B * N), u(B * N), y(B * N);
  make_rhs(p, nx, 0, nt, B, 11, f.p);
  int iters[B], status[B];
  double relres[B];
  EXPECT(abac_minres_solve(p, f.p, u.p, 1e-8, 200, iters, relres, status) == ABAC_OK);
  for (int b = 0; b < B; ++b) EXPECT(status[b] == ABAC_OK && iters[b] > 0 && relres[b] < 1e-8);
  EXPECT(abac_apply_A(p, u.p, y.p) == ABAC_OK);
  EXPECT(abac_apply_T(p, u.p, y.p) == ABAC_OK);
  EXPECT(abac_apply_Pinv(p, f.p, y.p) == ABAC_OK);
  EXPECT(abac_apply_Cinv(p, f.p, y.p) == ABAC_OK);
  EXPECT(abac_apply_A(p, u.p, u.p) == ABAC_EINVAL);                    // y aliases x
  EXPECT(abac_gmres_solve(p, f.p, u.p, 1e-8, 200, 15, iters, relres, status) == ABAC_OK);
  EXPECT(abac_gmres_solve(p, f.p, u.p, 1e-8, 200, 16, iters, relres, status) == ABAC_EINVAL);
  // asynchronous form
  EXPECT(abac_minres_begin(p, f.p, u.p, 1e-8, 200) == ABAC_OK);
  int done = 0;
  for (int k = 0; k < 400 && !done; ++k) {
    EXPECT(abac_minres_advance(p, 1) == ABAC_OK);
    EXPECT(abac_minres_poll(p, &done) == ABAC_OK);
  }
  EXPECT(abac_minres_finish(p, iters, relres, status) == ABAC_OK);
  for (int b = 0; b < B; ++b) EXPECT(status[b] == ABAC_OK);
  // variable coefficient (host face arrays), then back to the constant one
  std::vector<double> ax(nx + 1);
  for (int i = 0; i <= nx; ++i) ax[i] = 1.0 + 0.5 * std::sin(0.01 * i);
  EXPECT(abac_plan_set_coefficient(p, ax.data(), nullptr, 1.0) == ABAC_OK);
  EXPECT(abac_minres_solve(p, f.p, u.p, 1e-8, 400, iters, relres, status) == ABAC_OK);
  ax[3] = -1.0;
  EXPECT(abac_plan_set_coefficient(p, ax.data(), nullptr, 1.0) == ABAC_EINVAL);
  EXPECT(abac_plan_set_coefficient(p, nullptr, nullptr, 0.0) == ABAC_OK);
  EXPECT(abac_plan_destroy(p) == ABAC_OK);
}

static void solve_2d_caller_workspace() {
  const int nx = 63, ny = 31, nt = 32, B = 1;
  const size_t ws = abac_workspace_bytes(nx, ny, nt, ABAC_PREC_FP32, B);
  EXPECT(ws > 0);
  void* w = nullptr;
  HIP_OK(hipMalloc(&w, ws));
  hipStream_t s;
  HIP_OK(hipStreamCreate(&s));
  abac_plan* p = nullptr;
  EXPECT(abac_plan_create(nx, ny, nt, 1.0, 1e-2, ABAC_PREC_FP32, B, s, w, ws - 8, &p) == ABAC_ENOMEM);
  EXPECT(abac_plan_create(nx, ny, nt, 1.0, 1e-2, ABAC_PREC_FP32, B, s, w, ws, &p) == ABAC_OK);
  if (p) {
    const size_t N = (size_t)nx * ny * nt;
    Dev f(N), u(N);
    make_rhs(p, nx, ny, nt, B, 12, f.p);
    int wg[6];
    EXPECT(abac_plan_tiles(p, wg) == ABAC_OK);
    EXPECT(abac_plan_set_tiles(p, 0, 0, 100, 0) == ABAC_EINVAL);
    EXPECT(abac_profile_enable(p, 1) == ABAC_OK);
    int iters, status;
    double relres, ms = 0;
    long long n = 0;
    EXPECT(abac_minres_solve(p, f.p, u.p, 1e-8, 200, &iters, &relres, &status) == ABAC_OK);
    EXPECT(abac_profile_read(p, ABAC_K_STENCIL, &ms, &n) == ABAC_OK && n > 0 && ms > 0);
    EXPECT(abac_profile_read(p, ABAC_K_COUNT, &ms, &n) == ABAC_EINVAL);
    EXPECT(abac_profile_reset(p) == ABAC_OK);
    EXPECT(abac_profile_enable(p, 0) == ABAC_OK);
    EXPECT(abac_plan_destroy(p) == ABAC_OK);
  }
  HIP_OK(hipStreamDestroy(s));
  HIP_OK(hipFree(w));
}

static void group_of_three() {
  const int shapes[3][3] = {{255, 0, 64}, {63, 63, 64}, {31, 15, 32}};
  abac_plan* p[3] = {nullptr, nullptr, nullptr};
  std::vector<Dev*> bufs;
  for (int i = 0; i < 3; ++i) {
    EXPECT(abac_plan_create(shapes[i][0], shapes[i][1], shapes[i][2], 1.0, 1e-3, ABAC_PREC_FP32, 1, nullptr, nullptr,
                            0, &p[i]) == ABAC_OK);
    if (!p[i]) return;
    const size_t N = (size_t)shapes[i][0] * (shapes[i][1] ? shapes[i][1] : 1) * shapes[i][2];
    bufs.push_back(new Dev(N));
    bufs.push_back(new Dev(N));
    make_rhs(p[i], shapes[i][0], shapes[i][1], shapes[i][2], 1, 20 + i, bufs[2 * i]->p);
    EXPECT(abac_minres_begin(p[i], bufs[2 * i]->p, bufs[2 * i + 1]->p, 1e-8, 200) == ABAC_OK);
  }
  abac_group* g = nullptr;
  EXPECT(abac_group_create(nullptr, &g) == ABAC_OK);
  if (g) {
    abac_plan* twice[2] = {p[0], p[0]};
    EXPECT(abac_group_set(g, twice, 2) == ABAC_EINVAL);
    EXPECT(abac_group_set(g, p, 3) == ABAC_OK);
    EXPECT(abac_group_run(g, 1, -1, 0.0) == ABAC_EINVAL);
    EXPECT(abac_group_run(g, 1, 0, -1.0) == ABAC_EINVAL);
    EXPECT(abac_group_check(g, nullptr) == ABAC_EINVAL);
    for (int k = 0; k < 200; ++k) {
      // one launch per step, then every step of two iterations in one persistent launch
      EXPECT((k < 2 ? abac_group_advance(g, 1) : abac_group_run(g, 2, 0, 0.0)) == ABAC_OK);
      int all = 1;
      for (int i = 0; i < 3; ++i) {
        int d = 0;
        EXPECT(abac_minres_poll(p[i], &d) == ABAC_OK);
        all &= d;
      }
      if (all) break;
    }
    int aborted = 1;
    EXPECT(abac_group_check(g, &aborted) == ABAC_OK);
    EXPECT(aborted == 0);
    EXPECT(abac_group_destroy(g) == ABAC_OK);
  }
  for (int i = 0; i < 3; ++i) {
    int iters, status;
    double relres;
    EXPECT(abac_minres_finish(p[i], &iters, &relres, &status) == ABAC_OK);
    EXPECT(status == ABAC_OK);
    EXPECT(abac_plan_destroy(p[i]) == ABAC_OK);
  }
  for (Dev* d : bufs) delete d;
}

static void server_with_lane() {
  abac_server* s = nullptr;
  EXPECT(abac_server_create(size_t(4) << 30, 4, &s) == ABAC_OK);
  if (!s) return;
  EXPECT(abac_server_group_lane(s, 100000) == ABAC_OK);
  const int shapes[5][3] = {{255, 0, 64}, {63, 63, 64}, {1023, 0, 64}, {127, 127, 128}, {31, 31, 32}};
  long long t[5];
  for (int i = 0; i < 5; ++i)
    EXPECT(abac_server_submit(s, shapes[i][0], shapes[i][1], shapes[i][2], 1.0, 1e-3, ABAC_PREC_FP32, 100 + i, 1e-8,
                              200, abac_server_clock(s), i % 2, &t[i]) == ABAC_OK);
  long long big;
  EXPECT(abac_server_submit(s, 4095, 0, 1024, 1.0, 1e-3, ABAC_PREC_FP64, 1, 1e-8, 200, abac_server_clock(s), 0,
                            &big) == ABAC_OK);
  int pending = 6;
  std::vector<double> uh((size_t)127 * 127 * 128);
  bool seen[6] = {false, false, false, false, false, false};
  for (int k = 0; k < 200000 && pending; ++k) {
    int active = 0, queued = 0;
    EXPECT(abac_server_step(s, &active, &queued) == ABAC_OK);
    for (int i = 0; i < 6; ++i) {
      if (seen[i]) continue;
      const long long tk = i < 5 ? t[i] : big;
      int iters, status;
      double relres, lat;
      const abac_status r = abac_server_result(s, tk, i % 2 ? uh.data() : nullptr, &iters, &relres, &status, &lat);
      if (r == ABAC_EAGAIN) continue;
      EXPECT(r == ABAC_OK && status == ABAC_OK);
      seen[i] = true;
      --pending;
    }
  }
  EXPECT(pending == 0);
  EXPECT(abac_server_result(s, t[0], nullptr, nullptr, nullptr, nullptr, nullptr) == ABAC_EINVAL);   // forgotten
  EXPECT(abac_server_destroy(s) == ABAC_OK);
}

static void noalloc_twice() {
  const int nx = 127, ny = 63, nt = 64;
  const size_t N = (size_t)nx * ny * nt;
  Dev r(N), z(N);
  EXPECT(abac_fill_normal(nullptr, r.p, N, 7) == ABAC_OK);
  EXPECT(abac_apply_Pinv_noalloc(nx, ny, nt, 1.0, 1e-3, ABAC_PREC_FP64, 1, r.p, z.p, nullptr) == ABAC_OK);
  EXPECT(abac_apply_Pinv_noalloc(31, 31, 32, 1.0, 1e-3, ABAC_PREC_FP32, 1, r.p, z.p, nullptr) == ABAC_OK);
  EXPECT(abac_apply_Pinv_noalloc(4095, 4095, 1024, 1.0, 1e-3, ABAC_PREC_FP64, 1, r.p, z.p, nullptr) == ABAC_EINVAL);
  HIP_OK(hipDeviceSynchronize());
}

int main() {
  argument_checks();
  solve_1d();
  solve_2d_caller_workspace();
  group_of_three();
  server_with_lane();
  noalloc_twice();
  int rc = 0;
  if (g_fail) {
    std::fprintf(stderr, "%d check(s) failed\n", g_fail);
    rc = 1;
  } else {
    std::printf("HOST_DRIVER_OK\n");
  }
  // Leak check now, then leave without running the static destructors: during the HIP
  // runtime's own teardown at exit the sanitizer's device-allocation hooks fail an
  // internal check (dev_runtime_unloaded_) as the HSA runtime releases memory, a
  // matter of the two runtimes, outside this library.  Leaks make the status non-zero.
  if (__lsan_do_recoverable_leak_check()) rc = 1;
  std::fflush(stdout);
  std::fflush(stderr);
  _exit(rc);
}

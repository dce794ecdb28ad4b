// Host side of the ABAC library: plan creation (FP64 spectral tables), workspace
// layout, the C ABI entry points and the MINRES launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <climits>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/abac.h"
#include "abac_internal.h"
#include "plan_internal.h"

using namespace abac;

namespace {

thread_local std::string g_last_error;

abac_status fail(abac_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

abac_status hip_fail(hipError_t e, const char* where) {
  return fail(ABAC_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                    \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
  } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

const int kTileCandidates[] = {64, 128, 256, 512, 1024};

// a tile fits when its dynamic LDS plus a margin for the kernels' static LDS
// (block reductions) fits the device's per-workgroup LDS
bool tile_fits(int kind, int L, int wg, int prec, int maxlds) {
  return transform_tile_valid(kind, L, wg, prec) && transform_lds_bytes(kind, L, wg, prec) + 8192 <= (size_t)maxlds;
}

int default_wg(int kind, int L, int prec, int maxlds) {
  for (int wg : {256, 512, 1024, 128, 64})
    if (tile_fits(kind, L, wg, prec, maxlds)) return wg;
  return 0;
}

struct Layout {
  // vectors: V x3, Z x kZSlots, W x2, R
  static constexpr int kVecs = 3 + kZSlots + 2 + 1;
  size_t twx, twy, twt, beta, abk, sc, sci, coef, scratch, vec[kVecs], kcoef, gst, gflags, gparts, st, partials,
      counters, total;
};

// Validate the problem and fill the size fields of a DevPlan.
abac_status describe(int nx, int ny, int nt, double T, double alpha, int prec, int batch, DevPlan& P) {
  if (prec != ABAC_PREC_FP64 && prec != ABAC_PREC_FP32 && prec != ABAC_PREC_NONE)
    return fail(ABAC_EINVAL, "prec must be 0 (FP64), 1 (FP32) or 2 (no preconditioner)");
  if (batch < 1) return fail(ABAC_EINVAL, "batch must be >= 1");
  if (!(T > 0) || !std::isfinite(T)) return fail(ABAC_EINVAL, "T must be positive and finite");
  if (!(alpha > 0) || !(alpha <= 1)) return fail(ABAC_EINVAL, "alpha must be in (0, 1]");
  if (!is_pow2(nt) || nt < 8 || nt > 1024) return fail(ABAC_EINVAL, "nt must be a power of two in [8, 1024]");
  if (ny < 0) return fail(ABAC_EINVAL, "ny must be >= 0");
  const int Mx = nx + 1;
  if (!is_pow2(Mx) || Mx < 8 || Mx > (ny ? 512 : 4096))
    return fail(ABAC_EINVAL, ny ? "nx+1 must be a power of two in [8, 512] in 2D" : "nx+1 must be a power of two in [8, 4096] in 1D");
  if (ny) {
    const int My = ny + 1;
    if (!is_pow2(My) || My < 8 || My > 512) return fail(ABAC_EINVAL, "ny+1 must be a power of two in [8, 512]");
  }
  std::memset(&P, 0, sizeof(P));
  P.nx = nx;
  P.ny = ny;
  P.nt = nt;
  P.B = batch;
  P.ny1 = ny ? ny : 1;
  P.Mx = Mx;
  P.My = ny ? ny + 1 : 1;
  P.m = nx * P.ny1;
  P.ms = Mx * P.ny1;
  P.N = (long long)nt * P.m;
  P.NS = (long long)nt * P.ms;
  const double hx = 1.0 / Mx;
  const double tau = T / nt;
  P.tau = tau;
  P.tau2 = tau * tau;
  P.cx = 0.5 * tau * tau / (hx * hx);
  P.cy = 0.0;
  P.c0 = 1.0 + 2.0 * P.cx;
  if (ny) {
    const double hy = 1.0 / (ny + 1);
    P.cy = 0.5 * tau * tau / (hy * hy);
    P.c0 += 2.0 * P.cy;
  }
  // matvec decomposition: two columns per thread and bands of 2 rows; blocks march
  // over st_chunk levels (and their mirrors).  Longer marches re-read fewer warm-up
  // levels, shorter ones give more blocks: the chunk is the longest of 64/32/16/8
  // levels whose blocks still fill the GPU once at the matvec's occupancy (2 waves on
  // each of the 1024 SIMDs).  The rule depends on the shape only (not on the batch), so
  // a batched solve sums its partials in the same order as a single one.
  P.st_cols = nx >= 2 ? 2 : 1;
  P.st_rows = ny && nx >= 2 ? 2 : 1;
  P.st_threads = std::min(kStencilThreads, ((nx + P.st_cols - 1) / P.st_cols + 63) / 64 * 64);
  P.st_chunk = 64;
  while (P.st_chunk > 8 && (long long)stencil_blocks(P) * (P.st_threads / 64) < kStencilWaves) P.st_chunk /= 2;
  P.maxparts = std::max(std::max(stencil_blocks(P), update_blocks(P)), std::max((P.nt * P.ny1 + 1) / 2, P.ms / 2));
  P.maxparts = (P.maxparts + 63) & ~63;
  P.prec = prec;
  return ABAC_OK;
}

Layout make_layout(const DevPlan& P, int prec) {
  Layout Lo{};
  const size_t real = prec == ABAC_PREC_FP32 ? sizeof(float) : sizeof(double);
  const size_t cplx = 2 * real;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  Lo.twx = take(cplx * 2 * P.Mx);
  Lo.twy = take(cplx * 2 * P.My);
  Lo.twt = take(cplx * P.nt);
  Lo.beta = take(real * P.ms);
  Lo.abk = take(cplx * 2 * P.nt);
  Lo.sc = take(real * P.nt);
  Lo.sci = take(real * P.nt);
  Lo.coef = take(sizeof(double) * ((size_t)P.ny1 * P.Mx + (P.ny ? (size_t)P.My * P.nx : 0)));
  Lo.scratch = take(prec == ABAC_PREC_NONE ? 0 : real * (size_t)P.NS * P.B);
  for (int i = 0; i < Layout::kVecs; ++i) Lo.vec[i] = take(sizeof(double) * (size_t)P.N * P.B);
  Lo.kcoef = take(sizeof(double) * 3 * kBasis * P.B);
  Lo.gst = take(sizeof(GmresState) * P.B);
  Lo.gflags = take(sizeof(GmresFlags) * P.B);
  Lo.gparts = take(sizeof(double) * (size_t)(kGmresMax + 1) * kVecMaxBlocks * P.B);
  Lo.st = take(sizeof(MinresState) * P.B);
  Lo.partials = take(sizeof(double) * (size_t)P.maxparts * P.B * PART_KINDS);
  Lo.counters = take(sizeof(unsigned) * P.B);
  Lo.total = o;
  return Lo;
}

}  // namespace


namespace {

template <typename F>
abac_status run_kernel(abac_plan* p, int kid, F&& launch, const char* what) {
  ProfPair pp{kid, nullptr, nullptr};
  if (p->prof) {
    for (hipEvent_t* e : {&pp.e0, &pp.e1}) {
      if (!p->event_pool.empty()) {
        *e = p->event_pool.back();
        p->event_pool.pop_back();
      } else {
        HIP_TRY(hipEventCreate(e));
      }
    }
    HIP_TRY(hipEventRecord(pp.e0, p->stream));
  }
  hipError_t e = launch();
  if (e != hipSuccess) return hip_fail(e, what);
  if (p->prof) {
    HIP_TRY(hipEventRecord(pp.e1, p->stream));
    p->pending.push_back(pp);
  }
  return ABAC_OK;
}

abac_status flush_prof(abac_plan* p) {
  if (p->pending.empty()) return ABAC_OK;
  HIP_TRY(hipStreamSynchronize(p->stream));
  for (auto& pp : p->pending) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, pp.e0, pp.e1));
    p->prof_ms[pp.kid] += ms;
    p->prof_n[pp.kid] += 1;
    p->event_pool.push_back(pp.e0);
    p->event_pool.push_back(pp.e1);
  }
  p->pending.clear();
  return ABAC_OK;
}

#define RUN(kid, expr)                                            \
  do {                                                            \
    abac_status s_ = run_kernel(p, kid, [&] { return (expr); }, #expr); \
    if (s_ != ABAC_OK) return s_;                                 \
  } while (0)

// z = P^{-1} r on the plan stream.  In MINRES mode (init != 0 or iter != 0) the
// first pass reads V_1 (init) or forms the Lanczos vector (iteration) and the last
// pass writes Z and finishes the scalar update.
abac_status enqueue_pinv(abac_plan* p, const double* r, double* z, int minres_mode) {
  const DevPlan& P = p->P;
  if (p->prec == ABAC_PREC_NONE) {
    const int mode = minres_mode == 0 ? INV_PLAIN : (minres_mode == 1 ? INV_GAMMA_INIT : INV_GAMMA_ITER);
    RUN(ABAC_K_DSTX_INV, launch_identity(P, mode, r, z, p->stream));
    if (minres_mode) RUN(ABAC_K_FIN, launch_fin(P, minres_mode == 1 ? FIN_GAMMA_INIT : FIN_GAMMA_ITER, 0.0, 0, p->stream));
    return ABAC_OK;
  }
  const int check = minres_mode != 0;
  const int fwd_mode = minres_mode == 2 ? FWD_LANCZOS : FWD_PLAIN;
  const double* in = minres_mode == 1 ? P.V[1] : r;
  // in MINRES mode the time pass forms <q, P^{-1} q> and the last pass writes z only
  const int inv_mode = minres_mode == 0 ? INV_PLAIN : (minres_mode == 1 ? INV_Z_INIT : INV_Z_ITER);
  if (P.wg_s) {
    RUN(ABAC_K_DSTX_FWD, launch_dst2_fwd(P, p->prec, fwd_mode, check, in, p->stream));
    RUN(ABAC_K_TIME, launch_time(P, p->prec, check, p->stream));
    RUN(ABAC_K_DSTX_INV, launch_dst2_inv(P, p->prec, inv_mode, z, p->stream));
  } else {
    RUN(ABAC_K_DSTX_FWD, launch_dstx_fwd(P, p->prec, fwd_mode, check, in, p->stream));
    if (P.ny) RUN(ABAC_K_DSTY, launch_dsty(P, p->prec, check, p->stream));
    RUN(ABAC_K_TIME, launch_time(P, p->prec, check, p->stream));
    if (P.ny) RUN(ABAC_K_DSTY, launch_dsty(P, p->prec, check, p->stream));
    RUN(ABAC_K_DSTX_INV, launch_dstx_inv(P, p->prec, inv_mode, z, p->stream));
  }
  if (minres_mode) RUN(ABAC_K_FIN, launch_fin(P, minres_mode == 1 ? FIN_GAMMA_INIT : FIN_GAMMA_ITER, 0.0, 0, p->stream));
  return ABAC_OK;
}

// z = C_alpha^{-1} r: the transform passes with the single time pass of weights
// mu^{-1} (identity for ABAC_PREC_NONE).  z may alias r.
abac_status enqueue_cinv(abac_plan* p, const double* r, double* z) {
  const DevPlan& P = p->P;
  if (p->prec == ABAC_PREC_NONE) {
    RUN(ABAC_K_DSTX_INV, launch_identity(P, INV_PLAIN, r, z, p->stream));
    return ABAC_OK;
  }
  if (P.wg_s) {
    RUN(ABAC_K_DSTX_FWD, launch_dst2_fwd(P, p->prec, FWD_PLAIN, 0, r, p->stream));
    RUN(ABAC_K_TIME, launch_time(P, p->prec, 0, p->stream, 1));
    RUN(ABAC_K_DSTX_INV, launch_dst2_inv(P, p->prec, INV_PLAIN, z, p->stream));
    return ABAC_OK;
  }
  RUN(ABAC_K_DSTX_FWD, launch_dstx_fwd(P, p->prec, FWD_PLAIN, 0, r, p->stream));
  if (P.ny) RUN(ABAC_K_DSTY, launch_dsty(P, p->prec, 0, p->stream));
  RUN(ABAC_K_TIME, launch_time(P, p->prec, 0, p->stream, 1));
  if (P.ny) RUN(ABAC_K_DSTY, launch_dsty(P, p->prec, 0, p->stream));
  RUN(ABAC_K_DSTX_INV, launch_dstx_inv(P, p->prec, INV_PLAIN, z, p->stream));
  return ABAC_OK;
}

abac_status enqueue_iteration(abac_plan* p) {
  const DevPlan& P = p->P;
  if (P.small) {
    RUN(ABAC_K_ITER, launch_iter_small(P, p->prec, p->f, p->u, p->stream));
    return ABAC_OK;
  }
  RUN(ABAC_K_STENCIL, launch_stencil(P, STENCIL_MINRES, nullptr, nullptr, nullptr, p->stream));
  RUN(ABAC_K_FIN, launch_fin(P, FIN_DELTA, 0.0, 0, p->stream));
  abac_status s = enqueue_pinv(p, nullptr, nullptr, 2);
  if (s != ABAC_OK) return s;
  RUN(ABAC_K_UPDATE, launch_update(P, p->u, p->stream));
  RUN(ABAC_K_FIN, launch_fin(P, FIN_RNORM, 0.0, 0, p->stream));
  RUN(ABAC_K_FORM, launch_form(P, p->u, p->stream));
  RUN(ABAC_K_RESIDUAL, launch_stencil(P, STENCIL_RESIDUAL, p->u, nullptr, p->f, p->stream));
  RUN(ABAC_K_FIN, launch_fin(P, FIN_RES, 0.0, 0, p->stream));
  return ABAC_OK;
}

// The set-up and every iteration end with a kernel that copies the per-RHS state
// into the host-mapped ring; this event marks when that copy is complete.
abac_status record_snapshot_event(abac_plan* p) {
  const int slot = (int)(p->ring_posted % kSnapRing);
  HIP_TRY(hipEventRecord(p->ring_ev[slot], p->stream));
  p->ring_posted++;
  return ABAC_OK;
}

abac_status launch_iteration(abac_plan* p) {
  if (p->prof || !p->use_graph) return enqueue_iteration(p);
  if (!p->iter_graph || p->graph_f != p->f || p->graph_u != p->u) {
    if (p->iter_graph) {
      HIP_TRY(hipGraphExecDestroy(p->iter_graph));
      p->iter_graph = nullptr;
    }
    hipStream_t user = p->stream;
    p->stream = p->cap_stream;
    HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed));
    abac_status s = enqueue_iteration(p);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    p->stream = user;
    if (s != ABAC_OK) return s;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->iter_graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    p->graph_f = p->f;
    p->graph_u = p->u;
  }
  HIP_TRY(hipGraphLaunch(p->iter_graph, p->stream));
  return ABAC_OK;
}

bool all_stopped(const MinresState* s, int B) {
  for (int b = 0; b < B; ++b)
    if (s[b].state == ST_RUNNING) return false;
  return true;
}

void fill_results(const MinresState* s, int B, int* iters, double* relres, int* status, abac_status* worst) {
  *worst = ABAC_OK;
  for (int b = 0; b < B; ++b) {
    if (iters) iters[b] = s[b].iter;
    if (relres) relres[b] = s[b].bnorm2 > 0 ? std::sqrt(s[b].res2 / s[b].bnorm2) : 0.0;
    int st = s[b].state == ST_DONE ? s[b].status : ABAC_ENOTCONV;
    if (status) status[b] = st;
    if (st != ABAC_OK && *worst == ABAC_OK) *worst = (abac_status)st;
  }
}


struct TuneKey {
  int prec, nx, ny, nt, batch;
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, nx, ny, nt, batch) < std::tie(o.prec, o.nx, o.ny, o.nt, o.batch);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::array<int, 4>> g_tune;
bool g_tune_loaded = false;

void tune_file_load() {
  const char* path = std::getenv("ABAC_TUNE_FILE");
  g_tune_loaded = true;
  if (!path) return;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return;
  TuneKey k;
  std::array<int, 4> v;
  while (std::fscanf(fp, "%d %d %d %d %d %d %d %d %d", &k.prec, &k.nx, &k.ny, &k.nt, &k.batch, &v[0], &v[1], &v[2],
                     &v[3]) == 9)
    g_tune[k] = v;
  std::fclose(fp);
}

void tune_file_save() {
  const char* path = std::getenv("ABAC_TUNE_FILE");
  if (!path) return;
  FILE* fp = std::fopen(path, "w");
  if (!fp) return;
  for (auto& kv : g_tune)
    std::fprintf(fp, "%d %d %d %d %d %d %d %d %d\n", kv.first.prec, kv.first.nx, kv.first.ny, kv.first.nt,
                 kv.first.batch, kv.second[0], kv.second[1], kv.second[2], kv.second[3]);
  std::fclose(fp);
}

// Time one launcher: one warm-up launch, then the mean of three.
template <typename F>
float time_launches(hipStream_t s, F&& launch) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 1e30f;
  if (hipEventCreate(&e1) != hipSuccess) return 1e30f;
  float ms = 1e30f;
  if (launch() == hipSuccess && hipEventRecord(e0, s) == hipSuccess) {
    bool ok = true;
    for (int i = 0; i < 3 && ok; ++i) ok = launch() == hipSuccess;
    if (ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess)
      (void)hipEventElapsedTime(&ms, e0, e1);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

// Autotuner of the transform tiles: for the first x pass, the y pass and the time
// pass, every legal workgroup size (64..1024 threads, LDS within the device limit) is
// timed on the plan's own scratch and buffers in the mode MINRES runs; the fastest is
// kept.  Results are cached per shape (and in
// ABAC_TUNE_FILE if set).  ABAC_TUNE=0 keeps the defaults.
abac_status autotune(DevPlan& P, int prec, hipStream_t s, int maxlds) {
  const char* env = std::getenv("ABAC_TUNE");
  if (env && env[0] == '0') return ABAC_OK;
  const TuneKey key{prec, P.nx, P.ny, P.nt, P.B};
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (!g_tune_loaded) tune_file_load();
    auto it = g_tune.find(key);
    // a cached choice is used only if every tile is still legal for these kernels
    // (an entry written by another build of the library may not be)
    if (it != g_tune.end() && tile_fits(TK_XFWD, 2 * P.Mx, it->second[0], prec, maxlds) &&
        tile_fits(TK_XINV, 2 * P.Mx, it->second[1], prec, maxlds) &&
        (!P.ny || tile_fits(TK_Y, 2 * P.My, it->second[2], prec, maxlds)) &&
        tile_fits(TK_TIME, P.nt, it->second[3], prec, maxlds)) {
      P.wg_x = it->second[0];
      P.wg_xi = it->second[1];
      P.wg_y = it->second[2];
      P.wg_t = it->second[3];
      return ABAC_OK;
    }
  }
  // run the fused MINRES variants on the workspace: a temporary running state with
  // unit scales (cleared again below) lets the Lanczos and <q, p> paths execute
  for (int i = 0; i < 3; ++i) HIP_TRY(hipMemsetAsync(P.V[i], 0, sizeof(double) * (size_t)P.N * P.B, s));
  {
    std::vector<MinresState> tmp(P.B);
    std::memset(tmp.data(), 0, sizeof(MinresState) * P.B);
    for (auto& t : tmp) {
      t.state = ST_RUNNING;
      t.sig = 1.0;
    }
    HIP_TRY(hipMemcpyAsync(P.st, tmp.data(), sizeof(MinresState) * P.B, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  auto pick = [&](int kind, int L, int* field, auto launch) {
    int best = *field;
    float best_ms = 1e30f;
    for (int wg : kTileCandidates) {
      if (!tile_fits(kind, L, wg, prec, maxlds)) continue;
      *field = wg;
      const float ms = time_launches(s, launch);
      if (ms < best_ms) {
        best_ms = ms;
        best = wg;
      }
    }
    *field = best;
  };
  // (the fused 2D passes have a fixed tile; the separate x and y passes are not used)
  if (!P.wg_s) {
    pick(TK_XFWD, 2 * P.Mx, &P.wg_x, [&] { return launch_dstx_fwd(P, prec, FWD_LANCZOS, 1, nullptr, s); });
    if (P.ny) pick(TK_Y, 2 * P.My, &P.wg_y, [&] { return launch_dsty(P, prec, 1, s); });
  }
  // the time pass carries the <q, P^{-1} q> partials, summed in an order that does not
  // depend on its tile, so it is timed like the others; so is the last pass, which in
  // MINRES mode only writes z
  pick(TK_TIME, P.nt, &P.wg_t, [&] { return launch_time(P, prec, 1, s); });
  if (!P.wg_s) pick(TK_XINV, 2 * P.Mx, &P.wg_xi, [&] { return launch_dstx_inv(P, prec, INV_Z_ITER, nullptr, s); });
  HIP_TRY(hipMemsetAsync(P.st, 0, sizeof(MinresState) * P.B, s));
  HIP_TRY(hipStreamSynchronize(s));
  (void)hipGetLastError();
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = {P.wg_x, P.wg_xi, P.wg_y, P.wg_t};
  tune_file_save();
  return ABAC_OK;
}

}  // namespace

namespace abac {

abac_status plan_peek_snapshot(abac_plan* p, long long seq, int* ready, const MinresState** states) {
  *ready = 0;
  if (seq < 0 || seq >= p->ring_posted || seq < p->ring_posted - kSnapRing) return ABAC_OK;
  const int slot = (int)(seq % kSnapRing);
  hipError_t e = hipEventQuery(p->ring_ev[slot]);
  if (e == hipErrorNotReady) return ABAC_OK;
  if (e != hipSuccess) return hip_fail(e, "hipEventQuery");
  *ready = 1;
  *states = p->h_ring + (size_t)slot * p->P.B;
  return ABAC_OK;
}

long long plan_snapshots_posted(const abac_plan* p) { return p->ring_posted; }

void set_last_error(const std::string& msg) { g_last_error = msg; }

}  // namespace abac

namespace {

// beta_q = (abar tau^2/2) * eigenvalue of -Laplace_h of scratch mode q in the sine basis,
// (4/h^2) sin^2(j pi h / 2) summed over the axes (pad column: 1, harmless); the time
// tables of mu_k(beta) = A_k + beta B_k with A_k = (1 - a w_k)^2, B_k = 1 + a^2 w_k^2,
// w_k = exp(-2 pi i k/nt), a = alpha^{1/nt}; 1 - a w_k is evaluated without
// cancellation as ((1-a) + 2 a sin^2(th/2)) + i a sin(th).  D_alpha scalings a^{+-t}.
void spectral_tables(const DevPlan& P, double alpha, double abar, std::vector<double>& beta,
                     std::vector<double>& abk, std::vector<double>& sc, std::vector<double>& sci) {
  const double pi = 3.14159265358979323846;
  const int nx = P.nx, ny = P.ny, nt = P.nt, Mx = P.Mx;
  const double hx = 1.0 / Mx, hy = ny ? 1.0 / P.My : 0.0;
  std::vector<double> kx(nx), ky(ny ? ny : 1, 0.0);
  for (int j = 0; j < nx; ++j) {
    const double sj = std::sin((j + 1) * pi * hx / 2.0);
    kx[j] = 4.0 / (hx * hx) * sj * sj;
  }
  for (int j = 0; j < ny; ++j) {
    const double sj = std::sin((j + 1) * pi * hy / 2.0);
    ky[j] = 4.0 / (hy * hy) * sj * sj;
  }
  beta.assign(P.ms, 1.0);
  for (int yy = 0; yy < P.ny1; ++yy)
    for (int xx = 0; xx < nx; ++xx)
      beta[(size_t)yy * Mx + xx] = 0.5 * abar * P.tau2 * (kx[xx] + (ny ? ky[yy] : 0.0));
  abk.assign(4 * nt, 0.0);
  sc.assign(nt, 0.0);
  sci.assign(nt, 0.0);
  const double la = std::log(alpha) / nt;
  const double a = std::exp(la);
  const double oma = -std::expm1(la);
  for (int k = 0; k < nt; ++k) {
    const double th = 2.0 * pi * k / nt;
    const double sh = std::sin(0.5 * th);
    const double re = oma + 2.0 * a * sh * sh, im = a * std::sin(th);
    abk[4 * k + 0] = re * re - im * im;
    abk[4 * k + 1] = 2.0 * re * im;
    abk[4 * k + 2] = 1.0 + a * a * std::cos(2.0 * th);
    abk[4 * k + 3] = -a * a * std::sin(2.0 * th);
    sc[k] = std::exp(la * k);
    sci[k] = std::exp(-la * k);
  }
}

// C_alpha can be (nearly) singular as alpha -> 1 (the remark on Strang's circulant,
// Section 2.1); true when the smallest |mu| is below 1e-12 of the largest.
bool spectrum_near_singular(const DevPlan& P, const std::vector<double>& beta, const std::vector<double>& abk) {
  double mu_min = 1e300, mu_max = 0.0;
  for (int k = 0; k < P.nt; ++k)
    for (size_t q = 0; q < (size_t)P.ms; ++q) {
      if (q % P.Mx == (size_t)(P.Mx - 1)) continue;
      const double mr = abk[4 * k] + beta[q] * abk[4 * k + 2], mi = abk[4 * k + 1] + beta[q] * abk[4 * k + 3];
      const double mag = std::hypot(mr, mi);
      mu_min = std::min(mu_min, mag);
      mu_max = std::max(mu_max, mag);
    }
  return mu_min <= 1e-12 * mu_max;
}

// Copy a table to the device in the transform precision, ordered on `stream` and
// complete on return (the host vector is temporary).
hipError_t upload_table(void* dst, const std::vector<double>& v, int prec, hipStream_t stream) {
  std::vector<float> f;
  const void* src = v.data();
  size_t bytes = v.size() * sizeof(double);
  if (prec == ABAC_PREC_FP32) {
    f.assign(v.begin(), v.end());
    src = f.data();
    bytes = f.size() * sizeof(float);
  }
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return e;
}

}  // namespace

// ---------------------------------------------------------------------------
// Plan-free, allocation-free P_alpha^{-1}: the spectral tables and the transform
// scratch live in one file-scope device array.  Each GPU holds its own copy at its own
// address; host code reaches it only through the address hipGetSymbolAddress returns
// on that device (the array's name on the host is a stand-in, not a device address).
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kNoallocBytes = (size_t)128 << 20;
__device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch`, looked up once per device with that
// device current.
abac_status noalloc_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ABAC_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_noalloc_ptr[dev] = ptr;
  }
  *out = g_noalloc_ptr[dev];
  return ABAC_OK;
}

struct NoallocLayout {
  size_t twx, twy, twt, beta, abk, sc, sci, scr, total;
};

NoallocLayout noalloc_layout(const DevPlan& P, int prec) {
  NoallocLayout Lo{};
  const size_t real = prec == ABAC_PREC_FP32 ? sizeof(float) : sizeof(double);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  Lo.twx = take(2 * real * 2 * P.Mx);
  Lo.twy = take(2 * real * 2 * P.My);
  Lo.twt = take(2 * real * P.nt);
  Lo.beta = take(real * P.ms);
  Lo.abk = take(2 * real * 2 * P.nt);
  Lo.sc = take(real * P.nt);
  Lo.sci = take(real * P.nt);
  Lo.scr = take(real * (size_t)P.NS * P.B);
  Lo.total = o;
  return Lo;
}

// The tables of plan creation, computed on the device in FP64 and stored in the
// transform precision: twiddles exp(-2 pi i e/L) of the x, y and time lengths; beta_q =
// (tau^2/2) (kx + ky) of each scratch mode (1 in the pad column); (A_k, B_k) with
// mu_k(beta) = A_k + beta B_k, A_k = (1 - a w_k)^2 evaluated without cancellation as
// ((1-a) + 2a sin^2(th/2)) + i a sin th, B_k = 1 + a^2 w_k^2; and a^{+-t}.
template <typename T>
__global__ void k_noalloc_tables(DevPlan P, double la, double a, double oma) {
  using C = cplx<T>;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < 2 * P.Mx) {
    double sn, cs;
    sincospi(2.0 * e / (2.0 * P.Mx), &sn, &cs);
    reinterpret_cast<C*>(const_cast<void*>(P.twx))[e] = C{(T)cs, (T)-sn};
  }
  if (e < 2 * P.My) {
    double sn, cs;
    sincospi(2.0 * e / (2.0 * P.My), &sn, &cs);
    reinterpret_cast<C*>(const_cast<void*>(P.twy))[e] = C{(T)cs, (T)-sn};
  }
  if (e < P.nt) {
    double sn, cs;
    sincospi(2.0 * e / P.nt, &sn, &cs);
    reinterpret_cast<C*>(const_cast<void*>(P.twt))[e] = C{(T)cs, (T)-sn};
    const double sh = sinpi((double)e / P.nt);
    const double re = oma + 2.0 * a * sh * sh, im = a * sinpi(2.0 * e / P.nt);
    double s2, c2;
    sincospi(4.0 * e / P.nt, &s2, &c2);
    C* abk = reinterpret_cast<C*>(const_cast<void*>(P.abk));
    abk[2 * e] = C{(T)(re * re - im * im), (T)(2.0 * re * im)};
    abk[2 * e + 1] = C{(T)(1.0 + a * a * c2), (T)(-a * a * s2)};
    reinterpret_cast<T*>(const_cast<void*>(P.sc))[e] = (T)exp(la * e);
    reinterpret_cast<T*>(const_cast<void*>(P.sci))[e] = (T)exp(-la * e);
  }
  if (e < P.ms) {
    const int yy = e / P.Mx, xx = e - yy * P.Mx;
    double b = 1.0;
    if (xx < P.nx) {
      const double hx = 1.0 / P.Mx;
      const double sx = sinpi((xx + 1) * hx * 0.5);
      double k = 4.0 / (hx * hx) * sx * sx;
      if (P.ny) {
        const double hy = 1.0 / P.My;
        const double sy = sinpi((yy + 1) * hy * 0.5);
        k += 4.0 / (hy * hy) * sy * sy;
      }
      b = 0.5 * P.tau2 * k;
    }
    reinterpret_cast<T*>(const_cast<void*>(P.beta))[e] = (T)b;
  }
}

}  // namespace

extern "C" {

size_t abac_workspace_bytes(int nx, int ny, int nt, int prec, int batch) {
  DevPlan P;
  if (describe(nx, ny, nt, 1.0, 0.5, prec, batch, P) != ABAC_OK) return 0;
  return make_layout(P, prec).total;
}

abac_status abac_plan_create(int nx, int ny, int nt, double T, double alpha, int prec, int batch, void* stream,
                             void* workspace, size_t workspace_bytes, abac_plan** out) {
  g_last_error.clear();
  if (!out) return fail(ABAC_EINVAL, "out is NULL");
  *out = nullptr;
  DevPlan P;
  abac_status s = describe(nx, ny, nt, T, alpha, prec, batch, P);
  if (s != ABAC_OK) return s;
  // default tiles: 256 threads where the length allows it, within the device LDS limit
  int dev = 0, maxlds = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  P.wg_x = default_wg(TK_XFWD, 2 * P.Mx, prec, maxlds);
  // the last pass: the smallest legal tile until the tuner has timed the others (it
  // keeps the LDS small and the occupancy high)
  P.wg_xi = 0;
  for (int wg : kTileCandidates)
    if (!P.wg_xi && tile_fits(TK_XINV, 2 * P.Mx, wg, prec, maxlds))
      P.wg_xi = wg;
  P.wg_y = ny ? default_wg(TK_Y, 2 * P.My, prec, maxlds) : 256;
  P.wg_t = default_wg(TK_TIME, nt, prec, maxlds);
  // square 2D grids whose level fits in LDS take the fused x-y passes (a rule of the
  // shape, since it fixes the order of the <q, p> sums); ABAC_SLAB=0 turns them off
  {
    const char* env = std::getenv("ABAC_SLAB");
    const bool off = env && env[0] == '0';
    P.wg_s = (prec == ABAC_PREC_NONE || off) ? 0 : slab_wg(nx, ny, prec, maxlds, 8192);
  }
  // small 1D problems run each iteration in one workgroup per right-hand side (a rule
  // of the shape; ABAC_SMALL=0 keeps the separate kernels)
  {
    const char* env = std::getenv("ABAC_SMALL");
    const bool off = env && env[0] == '0';
    P.small = !off && small_path_valid(nx, ny, nt, prec) ? 1 : 0;
  }
  if (prec != ABAC_PREC_NONE && (!P.wg_x || !P.wg_xi || !P.wg_y || !P.wg_t))
    return fail(ABAC_EINVAL, "transform does not fit the device LDS (" + std::to_string(maxlds) +
                                 " B); use the FP32 preconditioner for this size");
  const Layout Lo = make_layout(P, prec);
  void* ws = workspace;
  bool own = false;
  if (!ws) {
    hipError_t e = hipMalloc(&ws, Lo.total);
    if (e != hipSuccess) return fail(ABAC_ENOMEM, "hipMalloc of " + std::to_string(Lo.total) + " bytes failed");
    own = true;
  } else if (workspace_bytes < Lo.total) {
    return fail(ABAC_ENOMEM, "workspace too small: need " + std::to_string(Lo.total) + " bytes");
  } else if (((uintptr_t)ws & 255) != 0) {
    return fail(ABAC_EINVAL, "workspace must be 256-byte aligned");
  }
  char* base = static_cast<char*>(ws);
  P.twx = base + Lo.twx;
  P.twy = base + Lo.twy;
  P.twt = base + Lo.twt;
  P.beta = base + Lo.beta;
  P.abk = base + Lo.abk;
  P.sc = base + Lo.sc;
  P.sci = base + Lo.sci;
  P.scratch = base + Lo.scratch;
  for (int i = 0; i < 3; ++i) P.V[i] = reinterpret_cast<double*>(base + Lo.vec[i]);
  for (int i = 0; i < kZSlots; ++i) P.Z[i] = reinterpret_cast<double*>(base + Lo.vec[3 + i]);
  for (int i = 0; i < 2; ++i) P.W[i] = reinterpret_cast<double*>(base + Lo.vec[3 + kZSlots + i]);
  P.R = reinterpret_cast<double*>(base + Lo.vec[3 + kZSlots + 2]);
  P.kcoef = reinterpret_cast<double*>(base + Lo.kcoef);
  P.gst = reinterpret_cast<GmresState*>(base + Lo.gst);
  P.gflags = reinterpret_cast<GmresFlags*>(base + Lo.gflags);
  P.gparts = reinterpret_cast<double*>(base + Lo.gparts);
  P.st = reinterpret_cast<MinresState*>(base + Lo.st);
  P.partials = reinterpret_cast<double*>(base + Lo.partials);
  P.counters = reinterpret_cast<unsigned*>(base + Lo.counters);
  P.coef_x = nullptr;   // constant coefficient until abac_plan_set_coefficient
  P.coef_y = nullptr;

  // ---- spectral tables in FP64 --------------------------------------------
  const double pi = 3.14159265358979323846;
  const int Mx = P.Mx, My = P.My;
  std::vector<double> twx(4 * Mx), twy(4 * My), twt(2 * nt), beta(P.ms), abk(4 * nt), sc(nt), sci(nt);
  auto twiddles = [&](std::vector<double>& t, int L) {
    for (int e = 0; e < L; ++e) {
      // exp(-2 pi i e / L), symmetric evaluation to keep the table accurate
      const double ang = 2.0 * pi * (double)e / (double)L;
      t[2 * e] = std::cos(ang);
      t[2 * e + 1] = -std::sin(ang);
    }
  };
  twiddles(twx, 2 * Mx);
  twiddles(twy, 2 * My);
  twiddles(twt, nt);
  spectral_tables(P, alpha, 1.0, beta, abk, sc, sci);
  if (alpha > 0.5 && prec != ABAC_PREC_NONE && spectrum_near_singular(P, beta, abk)) {
    if (own) (void)hipFree(ws);
    return fail(ABAC_EINVAL, "C_alpha is numerically singular for this alpha and grid");
  }
  auto upload = [&](const void* dst, const std::vector<double>& v) -> hipError_t {
    if (prec != ABAC_PREC_FP32) return hipMemcpy(const_cast<void*>(dst), v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice);
    std::vector<float> f(v.begin(), v.end());
    return hipMemcpy(const_cast<void*>(dst), f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload(P.twx, twx);
  if (e == hipSuccess) e = upload(P.twy, twy);
  if (e == hipSuccess) e = upload(P.twt, twt);
  if (e == hipSuccess) e = upload(P.beta, beta);
  if (e == hipSuccess) e = upload(P.abk, abk);
  if (e == hipSuccess) e = upload(P.sc, sc);
  if (e == hipSuccess) e = upload(P.sci, sci);
  if (e == hipSuccess) e = hipMemset(P.counters, 0, sizeof(unsigned) * batch);
  if (e == hipSuccess) e = hipMemset(P.st, 0, sizeof(MinresState) * batch);
  if (e == hipSuccess && prec != ABAC_PREC_NONE)
    e = hipMemset(P.scratch, 0, (prec ? 4 : 8) * (size_t)P.NS * batch);
  if (e != hipSuccess) {
    if (own) (void)hipFree(ws);
    return hip_fail(e, "table upload");
  }
  // <q, P^{-1} q>: one partial per block of the identity kernel, or per mode pair of the
  // time pass
  P.gamma_nparts = prec == ABAC_PREC_NONE ? update_blocks(P) : P.ms / 2;
  if (prec != ABAC_PREC_NONE) {
    abac_status ts = autotune(P, prec, static_cast<hipStream_t>(stream), maxlds);
    if (ts != ABAC_OK) {
      if (own) (void)hipFree(ws);
      return ts;
    }
  }
  abac_plan* p = new abac_plan();
  p->P = P;
  p->prec = prec;
  p->T = T;
  p->alpha = alpha;
  p->stream = static_cast<hipStream_t>(stream);
  p->ws = ws;
  p->ws_bytes = Lo.total;
  p->own_ws = own;
  p->coef_ws = reinterpret_cast<double*>(base + Lo.coef);
  p->abar = 1.0;
  p->h_ring = nullptr;
  p->cap_stream = nullptr;
  p->iter_graph = nullptr;
  p->graph_f = nullptr;
  p->graph_u = nullptr;
  {
    const char* env = std::getenv("ABAC_GRAPH");
    p->use_graph = !(env && env[0] == '0');
  }
  e = hipHostMalloc(reinterpret_cast<void**>(&p->h_ring), sizeof(MinresState) * (size_t)kSnapRing * batch,
                    hipHostMallocMapped);
  if (e == hipSuccess) {
    std::memset(p->h_ring, 0, sizeof(MinresState) * (size_t)kSnapRing * batch);
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&p->P.host_ring), p->h_ring, 0);
  }
  for (int i = 0; e == hipSuccess && i < kSnapRing; ++i) e = hipEventCreateWithFlags(&p->ring_ev[i], hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    if (own) (void)hipFree(ws);
    delete p;
    return hip_fail(e, "host ring");
  }
  p->ring_posted = 0;
  p->f = nullptr;
  p->u = nullptr;
  p->active = false;
  p->prof = false;
  for (int k = 0; k < ABAC_K_COUNT; ++k) {
    p->prof_ms[k] = 0;
    p->prof_n[k] = 0;
  }
  *out = p;
  return ABAC_OK;
}

abac_status abac_plan_destroy(abac_plan* p) {
  if (!p) return ABAC_OK;
  (void)hipStreamSynchronize(p->stream);
  flush_prof(p);
  for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
  for (int i = 0; i < kSnapRing; ++i) (void)hipEventDestroy(p->ring_ev[i]);
  if (p->iter_graph) (void)hipGraphExecDestroy(p->iter_graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->h_ring) (void)hipHostFree(p->h_ring);
  if (p->own_ws) (void)hipFree(p->ws);
  delete p;
  return ABAC_OK;
}

abac_status abac_plan_set_coefficient(abac_plan* p, const double* a_xh, const double* a_yh, double abar) {
  g_last_error.clear();
  if (!p) return fail(ABAC_EINVAL, "plan is NULL");
  if (p->active) return fail(ABAC_EINVAL, "a solve is in progress on this plan");
  DevPlan& P = p->P;
  const size_t nfx = (size_t)P.ny1 * P.Mx, nfy = P.ny ? (size_t)P.My * P.nx : 0;
  std::vector<double> w(nfx + nfy);
  if (a_xh) {
    if (P.ny && !a_yh) return fail(ABAC_EINVAL, "a_yh is required in 2D");
    if (!(abar > 0) || !std::isfinite(abar)) return fail(ABAC_EINVAL, "abar must be positive and finite");
    for (size_t i = 0; i < nfx; ++i) {
      if (!(a_xh[i] > 0) || !std::isfinite(a_xh[i])) return fail(ABAC_EINVAL, "a_xh entries must be positive and finite");
      w[i] = P.cx * a_xh[i];
    }
    for (size_t i = 0; i < nfy; ++i) {
      if (!(a_yh[i] > 0) || !std::isfinite(a_yh[i])) return fail(ABAC_EINVAL, "a_yh entries must be positive and finite");
      w[nfx + i] = P.cy * a_yh[i];
    }
  } else {
    abar = 1.0;
  }
  std::vector<double> beta, abk, sc, sci;
  if (p->prec != ABAC_PREC_NONE) {
    spectral_tables(P, p->alpha, abar, beta, abk, sc, sci);
    if (p->alpha > 0.5 && spectrum_near_singular(P, beta, abk))
      return fail(ABAC_EINVAL, "the mean-coefficient C_alpha is numerically singular for this alpha");
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (a_xh) HIP_TRY(upload_table(p->coef_ws, w, ABAC_PREC_FP64, p->stream));
  if (p->prec != ABAC_PREC_NONE) HIP_TRY(upload_table(const_cast<void*>(P.beta), beta, p->prec, p->stream));
  P.coef_x = a_xh ? p->coef_ws : nullptr;
  P.coef_y = a_xh && P.ny ? p->coef_ws + nfx : nullptr;
  p->abar = abar;
  // kernels take the plan by value: a captured iteration holds the old coefficients
  if (p->iter_graph) {
    HIP_TRY(hipGraphExecDestroy(p->iter_graph));
    p->iter_graph = nullptr;
  }
  return ABAC_OK;
}

abac_status abac_build_rhs(abac_plan* p, const double* src, const double* psi0, const double* psi1, double* f) {
  if (!p || !src || !psi0 || !psi1 || !f) return fail(ABAC_EINVAL, "NULL argument");
  RUN(ABAC_K_RHS, launch_rhs(p->P, src, psi0, psi1, f, p->stream));
  return ABAC_OK;
}

abac_status abac_apply_A(abac_plan* p, const double* x, double* y) {
  if (!p || !x || !y) return fail(ABAC_EINVAL, "NULL argument");
  if (x == y) return fail(ABAC_EINVAL, "apply_A: y must not alias x");
  RUN(ABAC_K_STENCIL, launch_stencil(p->P, STENCIL_PLAIN, x, y, nullptr, p->stream));
  return ABAC_OK;
}

abac_status abac_apply_Pinv(abac_plan* p, const double* r, double* z) {
  if (!p || !r || !z) return fail(ABAC_EINVAL, "NULL argument");
  return enqueue_pinv(p, r, z, 0);
}

abac_status abac_apply_T(abac_plan* p, const double* x, double* y) {
  if (!p || !x || !y) return fail(ABAC_EINVAL, "NULL argument");
  if (x == y) return fail(ABAC_EINVAL, "y must not alias x");
  RUN(ABAC_K_STENCIL, launch_stencil(p->P, STENCIL_T, x, y, nullptr, p->stream));
  return ABAC_OK;
}

abac_status abac_apply_Cinv(abac_plan* p, const double* r, double* z) {
  if (!p || !r || !z) return fail(ABAC_EINVAL, "NULL argument");
  if (p->active) return fail(ABAC_EINVAL, "a solve is in progress on this plan");
  return enqueue_cinv(p, r, z);
}

abac_status abac_gmres_solve(abac_plan* p, const double* f, double* u, double tol, int maxit, int restart,
                             int* iters, double* relres, int* status) {
  g_last_error.clear();
  if (!p || !f || !u) return fail(ABAC_EINVAL, "NULL argument");
  if (p->active) return fail(ABAC_EINVAL, "a solve is in progress on this plan");
  if (!(tol > 0) || maxit < 1 || restart < 1 || restart > kGmresMax)
    return fail(ABAC_EINVAL, "need tol > 0, maxit >= 1 and 1 <= restart <= " + std::to_string(kGmresMax));
  if (f == u) return fail(ABAC_EINVAL, "u must not alias f");
  const DevPlan& P = p->P;
  const int B = P.B;
  double* z = P.V[0];
  double* t = P.V[2];
  std::vector<GmresFlags> fl(B);
  auto read_flags = [&]() -> abac_status {
    HIP_TRY(hipMemcpyAsync(fl.data(), P.gflags, sizeof(GmresFlags) * B, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return ABAC_OK;
  };
  auto any = [&](auto pred) {
    for (const auto& x : fl)
      if (pred(x)) return true;
    return false;
  };
  RUN(ABAC_K_INIT, launch_ginit(P, f, u, p->stream));
  RUN(ABAC_K_FIN, launch_gfin(P, G_INIT, tol, maxit, restart, p->stream));
  RUN(ABAC_K_GMRES, launch_gbase(P, gslot(P, 0), u, 0, p->stream));
  abac_status s = read_flags();
  if (s != ABAC_OK) return s;
  int j = 0;
  // every running right-hand side takes the same steps (restarts happen at the end of
  // a cycle, which all reach together), so one host-side column index serves all
  while (any([](const GmresFlags& x) { return x.state == ST_RUNNING; })) {
    s = enqueue_cinv(p, gslot(P, j), z);
    if (s != ABAC_OK) return s;
    double* w = gslot(P, j + 1);   // w is formed in the slot of v_{j+1}, which stays unnormalised
    RUN(ABAC_K_STENCIL, launch_stencil(P, STENCIL_T, z, w, nullptr, p->stream));
    RUN(ABAC_K_GMRES, launch_gdots(P, j, w, p->stream));
    RUN(ABAC_K_FIN, launch_gfin(P, G_DOTS1, 0.0, 0, 0, p->stream));
    RUN(ABAC_K_GMRES, launch_gaxpy(P, j, 1, w, p->stream));   // also the second pass's dots
    RUN(ABAC_K_FIN, launch_gfin(P, G_DOTS2, 0.0, 0, 0, p->stream));
    RUN(ABAC_K_GMRES, launch_gaxpy(P, j, 2, w, p->stream));
    RUN(ABAC_K_FIN, launch_gfin(P, G_NORM, 0.0, 0, 0, p->stream));
    if ((s = read_flags()) != ABAC_OK) return s;
    if (!any([](const GmresFlags& x) { return x.state == ST_RUNNING && x.need; })) {
      ++j;
      continue;
    }
    // form u = X0 + C^{-1}(V y) and check f - T u explicitly
    RUN(ABAC_K_GMRES, launch_gcomb(P, j, t, p->stream));
    s = enqueue_cinv(p, t, z);
    if (s != ABAC_OK) return s;
    RUN(ABAC_K_GMRES, launch_gaddx(P, u, z, p->stream));
    RUN(ABAC_K_RESIDUAL, launch_stencil(P, STENCIL_RESVEC, u, t, f, p->stream));
    RUN(ABAC_K_FIN, launch_gfin(P, G_CHECK, 0.0, 0, 0, p->stream));
    RUN(ABAC_K_GMRES, launch_gbase(P, t, u, 1, p->stream));
    if ((s = read_flags()) != ABAC_OK) return s;
    const bool restarted = any([](const GmresFlags& x) { return x.state == ST_RUNNING && x.k == 0; });
    j = restarted ? 0 : j + 1;
    if (j >= restart) return fail(ABAC_EDEVICE, "GMRES cycle bookkeeping out of step");
  }
  std::vector<GmresState> h(B);
  HIP_TRY(hipMemcpyAsync(h.data(), P.gst, sizeof(GmresState) * B, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  s = flush_prof(p);
  if (s != ABAC_OK) return s;
  abac_status worst = ABAC_OK;
  for (int b = 0; b < B; ++b) {
    if (iters) iters[b] = h[b].iter;
    if (relres) relres[b] = h[b].bnorm2 > 0 ? std::sqrt(h[b].res2 / h[b].bnorm2) : 0.0;
    if (status) status[b] = h[b].status;
    if (h[b].status != ABAC_OK && (worst == ABAC_OK || h[b].status == ABAC_EBREAKDOWN)) worst = (abac_status)h[b].status;
  }
  return worst;
}

abac_status abac_minres_begin(abac_plan* p, const double* f, double* u, double tol, int maxit) {
  if (!p || !f || !u) return fail(ABAC_EINVAL, "NULL argument");
  if (!(tol > 0) || maxit < 1) return fail(ABAC_EINVAL, "tol must be > 0 and maxit >= 1");
  if (f == u) return fail(ABAC_EINVAL, "u must not alias f");
  p->f = f;
  p->u = u;
  p->active = true;
  p->ring_posted = 0;
  if (p->P.small) {
    RUN(ABAC_K_INIT, launch_setup_small(p->P, p->prec, f, u, tol, maxit, p->stream));   // ends with the snapshot
    return record_snapshot_event(p);
  }
  RUN(ABAC_K_INIT, launch_init(p->P, f, u, tol, maxit, p->stream));
  abac_status s = enqueue_pinv(p, nullptr, nullptr, 1);   // ends with the set-up snapshot
  if (s != ABAC_OK) return s;
  return record_snapshot_event(p);
}

abac_status abac_minres_advance(abac_plan* p, int iterations) {
  if (!p || !p->active) return fail(ABAC_EINVAL, "no solve in progress");
  for (int i = 0; i < iterations; ++i) {
    abac_status s = launch_iteration(p);
    if (s != ABAC_OK) return s;
    s = record_snapshot_event(p);
    if (s != ABAC_OK) return s;
  }
  return ABAC_OK;
}

abac_status abac_minres_poll(abac_plan* p, int* done) {
  if (!p || !done) return fail(ABAC_EINVAL, "NULL argument");
  *done = 0;
  if (!p->active) {
    *done = 1;
    return ABAC_OK;
  }
  // newest completed snapshot of this solve
  for (long long k = p->ring_posted - 1; k >= 0 && k >= p->ring_posted - kSnapRing; --k) {
    const int slot = (int)(k % kSnapRing);
    hipError_t e = hipEventQuery(p->ring_ev[slot]);
    if (e == hipSuccess) {
      *done = all_stopped(p->h_ring + (size_t)slot * p->P.B, p->P.B) ? 1 : 0;
      return ABAC_OK;
    }
    if (e != hipErrorNotReady) return hip_fail(e, "hipEventQuery");
  }
  return ABAC_OK;
}

abac_status abac_minres_finish(abac_plan* p, int* iters, double* relres, int* status) {
  if (!p || !p->active) return fail(ABAC_EINVAL, "no solve in progress");
  std::vector<MinresState> h(p->P.B);
  HIP_TRY(hipMemcpyAsync(h.data(), p->P.st, sizeof(MinresState) * p->P.B, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  // The explicit residual of the final iterate is already known for right-hand sides
  // stopped by the convergence test or maxit; recompute it otherwise.
  bool report = false;
  for (int b = 0; b < p->P.B; ++b)
    if (h[b].state != ST_DONE || (h[b].status != ABAC_OK && h[b].status != ABAC_ENOTCONV) ||
        (h[b].status == ABAC_OK && h[b].iter > 0 && h[b].res2 > h[b].tol2 * h[b].bnorm2))
      report = true;
  if (report) {
    RUN(ABAC_K_FIN, launch_fin(p->P, FIN_FINAL, 0.0, 0, p->stream));
    RUN(ABAC_K_FORM, launch_form(p->P, p->u, p->stream));
    RUN(ABAC_K_RESIDUAL, launch_stencil(p->P, STENCIL_REPORT, p->u, nullptr, p->f, p->stream));
    RUN(ABAC_K_FIN, launch_fin(p->P, FIN_REPORT, 0.0, 0, p->stream));
    HIP_TRY(hipMemcpyAsync(h.data(), p->P.st, sizeof(MinresState) * p->P.B, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  p->active = false;
  abac_status worst;
  fill_results(h.data(), p->P.B, iters, relres, status, &worst);
  return worst;
}

abac_status abac_minres_solve(abac_plan* p, const double* f, double* u, double tol, int maxit, int* iters,
                              double* relres, int* status) {
  if (p && p->P.small && f && u && f != u && tol > 0 && maxit >= 1) {
    // small problems: the set-up and every iteration in one launch
    p->f = f;
    p->u = u;
    p->active = true;
    p->ring_posted = 0;
    RUN(ABAC_K_ITER, launch_solve_small(p->P, p->prec, f, u, tol, maxit, p->stream));
    return abac_minres_finish(p, iters, relres, status);
  }
  abac_status s = abac_minres_begin(p, f, u, tol, maxit);
  if (s != ABAC_OK) return s;
  // Keep up to kAhead iterations queued beyond the newest observed state while the
  // observed residual decay predicts that convergence is further away; near the
  // predicted stop, step one iteration at a time so no idle iterations are queued.
  const int kAhead = 2;
  const int B = p->P.B;
  long long enq = 0, obs = 0;
  long long est = LLONG_MAX;
  double rel_last = -1.0;
  while (true) {
    if (enq < maxit && enq - obs <= kAhead && enq < est) {
      s = abac_minres_advance(p, 1);
      if (s != ABAC_OK) return s;
      ++enq;
      continue;
    }
    if (obs >= enq) {
      if (enq >= maxit) break;
      est = enq + 1;   // prediction was early: take one more step
      continue;
    }
    const int slot = (int)((obs + 1) % kSnapRing);
    HIP_TRY(hipEventSynchronize(p->ring_ev[slot]));
    ++obs;
    const MinresState* snap = p->h_ring + (size_t)slot * B;
    if (all_stopped(snap, B)) break;
    double rel = 0.0;
    for (int b = 0; b < B; ++b)
      if (snap[b].state == ST_RUNNING && snap[b].bnorm2 > 0) rel = std::max(rel, std::sqrt(snap[b].rnorm2 / snap[b].bnorm2));
    if (rel_last > 0.0 && rel > 0.0 && rel < rel_last) {
      const double rem = std::ceil(std::log(tol / rel) / std::log(rel / rel_last));
      est = obs + (long long)std::max(1.0, std::min(rem, 1e6));
    } else {
      est = LLONG_MAX;
    }
    rel_last = rel;
  }
  return abac_minres_finish(p, iters, relres, status);
}

abac_status abac_profile_enable(abac_plan* p, int on) {
  if (!p) return fail(ABAC_EINVAL, "NULL plan");
  p->prof = on != 0;
  return ABAC_OK;
}

abac_status abac_profile_read(abac_plan* p, int kernel, double* total_ms, long long* launches) {
  if (!p || kernel < 0 || kernel >= ABAC_K_COUNT) return fail(ABAC_EINVAL, "bad argument");
  abac_status s = flush_prof(p);
  if (s != ABAC_OK) return s;
  if (total_ms) *total_ms = p->prof_ms[kernel];
  if (launches) *launches = p->prof_n[kernel];
  return ABAC_OK;
}

abac_status abac_profile_reset(abac_plan* p) {
  if (!p) return fail(ABAC_EINVAL, "NULL plan");
  abac_status s = flush_prof(p);
  if (s != ABAC_OK) return s;
  for (int k = 0; k < ABAC_K_COUNT; ++k) {
    p->prof_ms[k] = 0;
    p->prof_n[k] = 0;
  }
  return ABAC_OK;
}

abac_status abac_plan_set_tiles(abac_plan* p, int wg_x, int wg_y, int wg_t, int wg_xi) {
  g_last_error.clear();
  if (!p) return fail(ABAC_EINVAL, "plan is NULL");
  if (p->active) return fail(ABAC_EINVAL, "a solve is in progress on this plan");
  if (p->prec == ABAC_PREC_NONE) return fail(ABAC_EINVAL, "the plan has no transform passes");
  DevPlan& P = p->P;
  int dev = 0, maxlds = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if ((wg_x || wg_y || wg_xi) && P.wg_s) return fail(ABAC_EINVAL, "the plan uses the fused x-y passes");
  if (wg_y && !P.ny) return fail(ABAC_EINVAL, "a 1D plan has no y pass");
  if (wg_x && !tile_fits(TK_XFWD, 2 * P.Mx, wg_x, p->prec, maxlds))
    return fail(ABAC_EINVAL, "x-DST tile " + std::to_string(wg_x) + " is not legal for this plan");
  if (wg_y && !tile_fits(TK_Y, 2 * P.My, wg_y, p->prec, maxlds))
    return fail(ABAC_EINVAL, "y-DST tile " + std::to_string(wg_y) + " is not legal for this plan");
  if (wg_t && !tile_fits(TK_TIME, P.nt, wg_t, p->prec, maxlds))
    return fail(ABAC_EINVAL, "time tile " + std::to_string(wg_t) + " is not legal for this plan");
  if (wg_xi && !tile_fits(TK_XINV, 2 * P.Mx, wg_xi, p->prec, maxlds))
    return fail(ABAC_EINVAL, "last x-DST tile " + std::to_string(wg_xi) + " is not legal for this plan");
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (wg_xi) P.wg_xi = wg_xi;
  if (wg_x) P.wg_x = wg_x;
  if (wg_y) P.wg_y = wg_y;
  if (wg_t) P.wg_t = wg_t;
  // kernels take the plan by value: a captured iteration holds the old tiles
  if (p->iter_graph) {
    HIP_TRY(hipGraphExecDestroy(p->iter_graph));
    p->iter_graph = nullptr;
  }
  return ABAC_OK;
}

abac_status abac_plan_tiles(abac_plan* p, int* wg) {
  if (!p || !wg) return fail(ABAC_EINVAL, "NULL argument");
  wg[0] = p->P.wg_x;
  wg[1] = p->P.wg_y;
  wg[2] = p->P.wg_t;
  wg[3] = p->P.wg_xi;
  wg[4] = p->P.wg_s;
  wg[5] = p->P.small ? 512 : 0;
  return ABAC_OK;
}

abac_status abac_apply_Pinv_noalloc(int nx, int ny, int nt, double T, double alpha, int prec, int batch,
                                    const double* r, double* z, void* stream) {
  g_last_error.clear();
  if (!r || !z) return fail(ABAC_EINVAL, "NULL argument");
  if (prec != ABAC_PREC_FP64 && prec != ABAC_PREC_FP32)
    return fail(ABAC_EINVAL, "prec must be 0 (FP64) or 1 (FP32) transforms");
  if (!(alpha > 0) || !(alpha <= 0.5))
    return fail(ABAC_EINVAL, "alpha must be in (0, 0.5] (near 1 C_alpha may be singular: use a plan)");
  DevPlan P;
  abac_status s = describe(nx, ny, nt, T, alpha, prec, batch, P);
  if (s != ABAC_OK) return s;
  const NoallocLayout Lo = noalloc_layout(P, prec);
  if (Lo.total > kNoallocBytes)
    return fail(ABAC_EINVAL, "problem needs " + std::to_string(Lo.total) + " bytes of scratch; the allocation-free "
                             "entry point holds at most " + std::to_string(kNoallocBytes) +
                             " (use a plan with a workspace)");
  int dev = 0, maxlds = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  void* base_v = nullptr;
  s = noalloc_scratch(dev, &base_v);
  if (s != ABAC_OK) return s;
  // the fixed tile rules of plan creation, without timing (no tuner: it would write
  // trial launches into the shared scratch and synchronise the stream)
  P.wg_x = default_wg(TK_XFWD, 2 * P.Mx, prec, maxlds);
  P.wg_xi = 0;
  for (int wg : kTileCandidates)
    if (!P.wg_xi && tile_fits(TK_XINV, 2 * P.Mx, wg, prec, maxlds)) P.wg_xi = wg;
  P.wg_y = ny ? default_wg(TK_Y, 2 * P.My, prec, maxlds) : 256;
  P.wg_t = default_wg(TK_TIME, nt, prec, maxlds);
  P.wg_s = slab_wg(nx, ny, prec, maxlds, 8192);
  if (!P.wg_x || !P.wg_xi || !P.wg_y || !P.wg_t)
    return fail(ABAC_EINVAL, "transform does not fit the device LDS; use the FP32 transforms for this size");
  char* base = static_cast<char*>(base_v);
  P.twx = base + Lo.twx;
  P.twy = base + Lo.twy;
  P.twt = base + Lo.twt;
  P.beta = base + Lo.beta;
  P.abk = base + Lo.abk;
  P.sc = base + Lo.sc;
  P.sci = base + Lo.sci;
  P.scratch = base + Lo.scr;
  // every scratch value an apply reads is written earlier in the same apply (the first
  // pass writes whole rows, the zero pad column included), so nothing is cleared
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double la = std::log(alpha) / nt;
  const int n = std::max(std::max(2 * P.Mx, 2 * P.My), std::max(nt, P.ms));
  if (prec == ABAC_PREC_FP32)
    hipLaunchKernelGGL(k_noalloc_tables<float>, dim3((n + 255) / 256), dim3(256), 0, st, P, la, std::exp(la),
                       -std::expm1(la));
  else
    hipLaunchKernelGGL(k_noalloc_tables<double>, dim3((n + 255) / 256), dim3(256), 0, st, P, la, std::exp(la),
                       -std::expm1(la));
  HIP_TRY(hipGetLastError());
  hipError_t e;
  if (P.wg_s) {
    if ((e = launch_dst2_fwd(P, prec, FWD_PLAIN, 0, r, st)) != hipSuccess) return hip_fail(e, "launch_dst2_fwd");
    if ((e = launch_time(P, prec, 0, st)) != hipSuccess) return hip_fail(e, "launch_time");
    if ((e = launch_dst2_inv(P, prec, INV_PLAIN, z, st)) != hipSuccess) return hip_fail(e, "launch_dst2_inv");
  } else {
    if ((e = launch_dstx_fwd(P, prec, FWD_PLAIN, 0, r, st)) != hipSuccess) return hip_fail(e, "launch_dstx_fwd");
    if (P.ny && (e = launch_dsty(P, prec, 0, st)) != hipSuccess) return hip_fail(e, "launch_dsty");
    if ((e = launch_time(P, prec, 0, st)) != hipSuccess) return hip_fail(e, "launch_time");
    if (P.ny && (e = launch_dsty(P, prec, 0, st)) != hipSuccess) return hip_fail(e, "launch_dsty");
    if ((e = launch_dstx_inv(P, prec, INV_PLAIN, z, st)) != hipSuccess) return hip_fail(e, "launch_dstx_inv");
  }
  return ABAC_OK;
}

const char* abac_status_string(int s) {
  switch (s) {
    case ABAC_OK: return "ok";
    case ABAC_EINVAL: return "invalid argument";
    case ABAC_ENOMEM: return "out of memory";
    case ABAC_EDEVICE: return "device error";
    case ABAC_ENOTCONV: return "not converged";
    case ABAC_EBREAKDOWN: return "breakdown";
    case ABAC_EBUDGET: return "over budget";
    case ABAC_EAGAIN: return "not ready";
    default: return "unknown status";
  }
}

const char* abac_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

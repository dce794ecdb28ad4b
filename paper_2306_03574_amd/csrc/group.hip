// Solves of different grids advanced together: one launch per step of a MINRES
// iteration (Section 3's solver: matvec, Lanczos step with the three transform steps of
// Section 2.3 done twice, Givens QR, residual recurrence, stopping test) covers every
// member of a group, whatever its grid, instead of one launch per step per solve.
//
// A launch's blocks are the concatenation of the members' blocks of that step: block w
// finds its member r by a search over the step's prefix table, and runs the member's
// tile (the same per-tile device code as the member's own kernels) for its grid.  All
// list kernels use one workgroup size, kGroupWG threads (the scalar steps kFinThreads),
// so the tile of a transform pass is the one of that size; those passes are computed by
// the same arithmetic whatever the tile, the reductions are grouped as in the members'
// own kernels (one partial per logical matvec or vector block, one per mode pair of
// the time pass), and each member keeps its own state, partials and snapshots.  A
// member's results are therefore bitwise those of its solo solve.
//
// The persistent kernel runs the same step bodies for several iterations in one
// launch, with a grid-wide barrier between steps (abac_group_run).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/abac.h"
#include "abac_internal.h"
#include "minres_device.h"
#include "plan_internal.h"
#include "stencil_device.h"
#include "transform_device.h"

namespace abac {
namespace {

constexpr int kGroupWG = 256;
constexpr int kGroupFinThreads = 1024;   // as the members' scalar-step kernel
constexpr int kGroupMax = 64;
constexpr double kGroupTimeout = 2.0;    // seconds a persistent block waits at a barrier

enum GroupStep : int { GS_STENCIL = 0, GS_XFWD, GS_Y, GS_TIME, GS_XINV, GS_VEC, GS_FIN, GS_COUNT };

struct GroupMember {
  DevPlan P;
  const double* f;
  double* u;
};

// Device table of a group: the members and, per step, the first block of each member
// (off[step][n] = the launch's block count).
struct GroupTable {
  GroupMember m[kGroupMax];
  int off[GS_COUNT][kGroupMax + 1];
  int n;
};

// Member and block of block w of a step: r with off[r] <= w < off[r+1], then right-hand
// side b and the block lbk within it (per = blocks per right-hand side).
struct Where {
  int r, b, lbk, per;
};

__device__ __forceinline__ Where locate(const GroupTable* __restrict__ G, int step, int w) {
  const int* off = G->off[step];
  int lo = 0, hi = G->n;   // off[lo] <= w < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= w) lo = mid;
    else hi = mid;
  }
  Where at;
  at.r = lo;
  const int nb = G->m[lo].P.B;
  at.per = (off[lo + 1] - off[lo]) / nb;
  const int lw = w - off[lo];
  at.b = lw / at.per;
  at.lbk = lw - at.b * at.per;
  return at;
}

// ---- matvec: one logical block per workgroup, lanes beyond the member's column tile
// idle (they add 0 to the block's sum, so the partial is the member kernel's) ---------
template <int MODE>
__device__ __forceinline__ void group_stencil(const GroupTable* __restrict__ G, int w) {
  const Where at = locate(G, GS_STENCIL, w);
  const GroupMember& M = G->m[at.r];
  const DevPlan& P = M.P;
  const MinresState* st = P.st + at.b;
  if (st->state != ST_RUNNING) return;
  if (MODE == STENCIL_RESIDUAL && !st->need_check) return;
  const size_t off = (size_t)at.b * P.N;
  double acc = 0.0;
  const bool lane = (int)threadIdx.x < P.st_threads;
  if (MODE == STENCIL_MINRES) {
    const int j = st->iter + 1;
    const double* x = P.Z[zslot(j)] + off;
    double* y = P.V[(j + 1) % 3] + off;
    if (lane)
      acc = P.coef_x ? stencil_run<true, OUT_REV, true>(P, x, y, nullptr, at.lbk, at.per, threadIdx.x, true)
                     : stencil_run<false, OUT_REV, true>(P, x, y, nullptr, at.lbk, at.per, threadIdx.x, true);
  } else {
    const double* x = M.u + off;
    const double* f = M.f + off;
    if (lane)
      acc = P.coef_x ? stencil_run<true, OUT_RESNORM, false>(P, x, nullptr, f, at.lbk, at.per, threadIdx.x, true)
                     : stencil_run<false, OUT_RESNORM, false>(P, x, nullptr, f, at.lbk, at.per, threadIdx.x, true);
  }
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, MODE == STENCIL_MINRES ? PART_DELTA : PART_RES, at.b)[at.lbk] = bs;
}

// ---- scalar steps: one workgroup per right-hand side --------------------------------
// The fixed-order sum of n partials exactly as a block of V threads forms it (that of
// sum_parts with blockDim.x = V), computed by a block of blockDim.x threads, where
// blockDim.x divides V <= 1024: thread t stands in for threads t, t + blockDim.x, ...
// of the V-thread block, whose 64-lane waves it reduces one after the other, so every
// addition and its order are the V-thread block's.  Result valid in thread 0.
__device__ __forceinline__ double sum_parts_as(const double* __restrict__ part, int n, int V) {
  __shared__ double wsum[16];
  const double2* p2 = reinterpret_cast<const double2*>(part);
  const int n2 = n >> 1, lane = threadIdx.x & 63;
  for (int vt = threadIdx.x; vt < V; vt += blockDim.x) {
    double s = 0.0;
    for (int i = vt; i < n2; i += V) {
      const double2 v = p2[i];
      s += v.x + v.y;
    }
    if ((n & 1) && vt == 0) s += part[n - 1];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) wsum[vt >> 6] = s;
  }
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (V + 63) >> 6; ++i) tot += wsum[i];
  __syncthreads();
  return tot;
}

__device__ __forceinline__ void group_fin(const GroupTable* __restrict__ G, int w, int kind) {
  const Where at = locate(G, GS_FIN, w);
  const DevPlan& P = G->m[at.r].P;
  if (!fin_begin(P, at.b, kind)) return;
  int nparts;
  switch (kind) {
    case FIN_BNORM:
    case FIN_RNORM: nparts = G->off[GS_VEC][at.r + 1] - G->off[GS_VEC][at.r]; nparts /= P.B; break;
    case FIN_DELTA: nparts = stencil_blocks(P); break;
    case FIN_GAMMA_INIT:
    case FIN_GAMMA_ITER: nparts = P.gamma_nparts; break;
    default: nparts = stencil_blocks(P); break;
  }
  const double tot = sum_parts_as(part_slot(P, fin_part_kind(kind), at.b), nparts, kGroupFinThreads);
  if (threadIdx.x == 0) fin_scalar(P, at.b, kind, tot, 0.0, 0);
}

// ---- vector steps: residual recurrence, iterate from the basis ----------------------
__device__ __forceinline__ void group_update(const GroupTable* __restrict__ G, int w) {
  const Where at = locate(G, GS_VEC, w);
  const GroupMember& M = G->m[at.r];
  const DevPlan& P = M.P;
  if (P.st[at.b].state != ST_RUNNING) return;
  const double acc = update_part(P, at.b, M.u, at.lbk, at.per);
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_RNORM, at.b)[at.lbk] = bs;
}

__device__ __forceinline__ void group_form(const GroupTable* __restrict__ G, int w) {
  const Where at = locate(G, GS_VEC, w);
  const GroupMember& M = G->m[at.r];
  const DevPlan& P = M.P;
  const MinresState* st = P.st + at.b;
  if (!st->form_now) return;
  const int nb = st->nbasis;
  if (st->flush_now) form_dispatch<true>(P, at.b, nb, M.u, at.lbk, at.per);
  else form_dispatch<false>(P, at.b, nb, M.u, at.lbk, at.per);
}

// ---- transform passes: the member's tile of its own length, selected at run time ----
#define ABAC_GROUP_X_LENGTHS(CASE) CASE(16) CASE(32) CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096)
#define ABAC_GROUP_SLAB_LENGTHS(CASE) CASE(16) CASE(32) CASE(64) CASE(128) CASE(256)
#define ABAC_GROUP_T_LENGTHS(CASE) CASE(8) CASE(16) CASE(32) CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024)

// first pass: the Lanczos step and the x-DST, or the fused x-y pass
template <typename T>
__device__ __forceinline__ void group_xfwd(const GroupTable* __restrict__ G, int w) {
  const Where at = locate(G, GS_XFWD, w);
  const DevPlan& P = G->m[at.r].P;
  if (P.st[at.b].state != ST_RUNNING) return;
  constexpr int mode = FWD_LANCZOS;
  const double* in = nullptr;
  const int L = 2 * P.Mx;
  if (P.wg_s) {
#define CASE(LL) \
    case LL: if constexpr (slab_ok<T, LL, kGroupWG>()) dst2_fwd_tile<T, LL, kGroupWG>(P, mode, in, at.b, at.lbk); break;
    switch (L) { ABAC_GROUP_SLAB_LENGTHS(CASE) default: break; }
#undef CASE
  } else {
#define CASE(LL)                                                                                            \
    case LL:                                                                                                \
      if constexpr (tile_ok<T, LL, kGroupWG, TK_XFWD>())                                                    \
        dstx_fwd_tile<T, LL, kGroupWG>(P, mode, in, at.b, at.lbk, reinterpret_cast<const cplx<T>*>(P.twx)); \
      break;
    switch (L) { ABAC_GROUP_X_LENGTHS(CASE) default: break; }
#undef CASE
  }
}

template <typename T>
__device__ __forceinline__ void group_y(const GroupTable* __restrict__ G, int w) {
  const Where at = locate(G, GS_Y, w);
  const DevPlan& P = G->m[at.r].P;
  if (P.st[at.b].state != ST_RUNNING) return;
  const int lbk = xcd_remap(at.lbk, at.per);
#define CASE(LL) \
  case LL: if constexpr (tile_ok<T, LL, kGroupWG, TK_Y>()) dsty_tile<T, LL, kGroupWG>(P, at.b, lbk); break;
  switch (2 * P.My) { ABAC_GROUP_X_LENGTHS(CASE) default: break; }
#undef CASE
}

template <typename T>
__device__ __forceinline__ void group_time(const GroupTable* __restrict__ G, int w) {
  const Where at = locate(G, GS_TIME, w);
  const DevPlan& P = G->m[at.r].P;
  if (P.st[at.b].state != ST_RUNNING) return;
  const int lbk = xcd_remap(at.lbk, at.per);
#define CASE(LL) \
  case LL: if constexpr (tile_ok<T, LL, kGroupWG, TK_TIME>()) time_tile<T, LL, kGroupWG>(P, 0, at.b, lbk, 1); break;
  switch (P.nt) { ABAC_GROUP_T_LENGTHS(CASE) default: break; }
#undef CASE
}

// last pass: writes z_{j+1}; <q, P^{-1} q> came from the time pass
template <typename T>
__device__ __forceinline__ void group_xinv(const GroupTable* __restrict__ G, int w) {
  constexpr int mode = INV_Z_ITER;
  const Where at = locate(G, GS_XINV, w);
  const DevPlan& P = G->m[at.r].P;
  if (P.st[at.b].state != ST_RUNNING) return;
  const int L = 2 * P.Mx;
  if (P.wg_s) {
#define CASE(LL) \
    case LL: if constexpr (slab_ok<T, LL, kGroupWG>()) (void)dst2_inv_tile<T, LL, kGroupWG>(P, mode, nullptr, at.b, at.lbk); break;
    switch (L) { ABAC_GROUP_SLAB_LENGTHS(CASE) default: break; }
#undef CASE
  } else {
#define CASE(LL)                                                                                                     \
    case LL:                                                                                                         \
      if constexpr (tile_ok<T, LL, kGroupWG, TK_XINV>())                                                             \
        (void)dstx_inv_tile<T, LL, kGroupWG>(P, mode, nullptr, at.b, at.lbk, reinterpret_cast<const cplx<T>*>(P.twx)); \
      break;
    switch (L) { ABAC_GROUP_X_LENGTHS(CASE) default: break; }
#undef CASE
  }
}

#undef ABAC_GROUP_X_LENGTHS
#undef ABAC_GROUP_SLAB_LENGTHS
#undef ABAC_GROUP_T_LENGTHS

// ---- list kernels: one launch per step, one logical block per workgroup -------------
template <int MODE>
__global__ void __launch_bounds__(kGroupWG) k_group_stencil(const GroupTable* __restrict__ G) {
  group_stencil<MODE>(G, blockIdx.x);
}
__global__ void __launch_bounds__(kGroupFinThreads) k_group_fin(const GroupTable* __restrict__ G, int kind) {
  group_fin(G, blockIdx.x, kind);
}
__global__ void __launch_bounds__(kGroupWG) k_group_update(const GroupTable* __restrict__ G) {
  group_update(G, blockIdx.x);
}
__global__ void __launch_bounds__(kGroupWG) k_group_form(const GroupTable* __restrict__ G) {
  group_form(G, blockIdx.x);
}
template <typename T>
__global__ void __launch_bounds__(kGroupWG) k_group_xfwd(const GroupTable* __restrict__ G) {
  group_xfwd<T>(G, blockIdx.x);
}
template <typename T>
__global__ void __launch_bounds__(kGroupWG) k_group_y(const GroupTable* __restrict__ G) {
  group_y<T>(G, blockIdx.x);
}
template <typename T>
__global__ void __launch_bounds__(kGroupWG) k_group_time(const GroupTable* __restrict__ G) {
  group_time<T>(G, blockIdx.x);
}
template <typename T>
__global__ void __launch_bounds__(kGroupWG) k_group_xinv(const GroupTable* __restrict__ G) {
  group_xinv<T>(G, blockIdx.x);
}

// ---- persistent kernel: every step of `iterations` iterations in one launch ---------
// Barrier state in device memory.  count and gen are reset before each launch; aborted
// stays set until the host reads it (abac_group_check).
struct GridSync {
  unsigned count;   // blocks arrived at the current barrier
  unsigned gen;     // barriers completed in this launch
  int abort;        // a block stopped waiting: every block leaves the launch
  int aborted;      // sticky copy of abort
};

// Grid-wide barrier.  Inside one launch the L2s of the XCDs are not coherent with each
// other.  Every wave waits until its stores have reached its XCD's L2, then, after the
// workgroup barrier, thread 0 counts the block in with an agent-scope acquire-release
// atomic (which writes that L2 back first), the last block to arrive opens the next
// generation, and every wave acquires at agent scope after it.  A waiting
// block gives up once `deadline` ticks of the constant-rate clock have passed or
// another block gave up; false then tells every thread of the block to leave the
// kernel, so the launch always ends.
__device__ __forceinline__ bool grid_barrier(GridSync* gs, unsigned& gen, unsigned long long deadline) {
  __shared__ int pass;
  __builtin_amdgcn_s_waitcnt(0);   // this wave's stores have reached its XCD's L2
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned next = gen + 1;
    int ok = 1;
    if (__hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1) {
      __hip_atomic_store(&gs->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&gs->gen, next, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const unsigned long long t0 = wall_clock64();
      while (__hip_atomic_load(&gs->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != next) {
        if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
            wall_clock64() - t0 > deadline) {
          __hip_atomic_store(&gs->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&gs->aborted, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    gen = next;
    pass = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return pass;
}

// The step bodies, out of line so that each gets the registers of its own tile (inlined
// into one loop they would all share the largest tile's and spill).
template <int MODE>
__device__ __noinline__ void ps_stencil(const GroupTable* G, int w) { group_stencil<MODE>(G, w); }
__device__ __noinline__ void ps_fin(const GroupTable* G, int w, int kind) { group_fin(G, w, kind); }
__device__ __noinline__ void ps_update(const GroupTable* G, int w) { group_update(G, w); }
__device__ __noinline__ void ps_form(const GroupTable* G, int w) { group_form(G, w); }
template <typename T>
__device__ __noinline__ void ps_xfwd(const GroupTable* G, int w) { group_xfwd<T>(G, w); }
template <typename T>
__device__ __noinline__ void ps_y(const GroupTable* G, int w) { group_y<T>(G, w); }
template <typename T>
__device__ __noinline__ void ps_time(const GroupTable* G, int w) { group_time<T>(G, w); }
template <typename T>
__device__ __noinline__ void ps_xinv(const GroupTable* G, int w) { group_xinv<T>(G, w); }

// The grid is at most what the device holds at once; block k
// takes logical blocks k, k + gridDim.x, ... of each step, then the grid meets at a
// barrier, so a step starts only once the step before has finished for every member,
// as between the list kernels.  Each logical block runs the same body with the same
// workgroup size as in the list kernels (the scalar steps' sums keep the order of
// their 1024-thread blocks), so the results are bitwise those of abac_group_advance.
template <typename T>
__global__ void __launch_bounds__(kGroupWG)
k_group_persistent(const GroupTable* __restrict__ G, int iterations, GridSync* gs, unsigned long long deadline) {
  unsigned gen = 0;
  const int n = G->n;
  for (int it = 0; it < iterations; ++it) {
#define ABAC_STEP(STEP, CALL)                                             \
    if (G->off[STEP][n]) {                                                \
      for (int w = blockIdx.x; w < G->off[STEP][n]; w += gridDim.x) {     \
        CALL;                                                             \
        __syncthreads();                                                  \
      }                                                                   \
      if (!grid_barrier(gs, gen, deadline)) return;                       \
    }
    ABAC_STEP(GS_STENCIL, ps_stencil<STENCIL_MINRES>(G, w))
    ABAC_STEP(GS_FIN, ps_fin(G, w, FIN_DELTA))
    ABAC_STEP(GS_XFWD, ps_xfwd<T>(G, w))
    ABAC_STEP(GS_Y, ps_y<T>(G, w))
    ABAC_STEP(GS_TIME, ps_time<T>(G, w))
    ABAC_STEP(GS_Y, ps_y<T>(G, w))
    ABAC_STEP(GS_XINV, ps_xinv<T>(G, w))
    ABAC_STEP(GS_FIN, ps_fin(G, w, FIN_GAMMA_ITER))
    ABAC_STEP(GS_VEC, ps_update(G, w))
    ABAC_STEP(GS_FIN, ps_fin(G, w, FIN_RNORM))
    ABAC_STEP(GS_VEC, ps_form(G, w))
    ABAC_STEP(GS_STENCIL, ps_stencil<STENCIL_RESIDUAL>(G, w))
    ABAC_STEP(GS_FIN, ps_fin(G, w, FIN_RES))
#undef ABAC_STEP
  }
}

}  // namespace
}  // namespace abac

using namespace abac;

constexpr int kGroupStage = 4;   // pinned host copies of the table, used in turn

struct abac_group {
  hipStream_t stream;
  int prec;
  GroupTable* d_table;                 // the table the launches read
  GroupTable* h_stage[kGroupStage];    // pinned host copies, uploaded in stream order
  hipEvent_t stage_ev[kGroupStage];    // upload of each copy complete
  int stage_next;
  std::vector<abac_plan*> members;
  int blocks[GS_COUNT];
  size_t lds[GS_COUNT];
  hipEvent_t joined;             // members' set-up done (recorded on each member stream in turn)
  hipEvent_t done;               // the group's last enqueued work
  GridSync* d_sync;              // barrier state of the persistent kernel
  int device;                    // the device current at creation (the group's memory lives there)
};

namespace {

abac_status gfail(abac_status s, const std::string& msg) {
  set_last_error(msg);
  return s;
}

#define GHIP(expr)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return gfail(ABAC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Blocks per right-hand side of each step for a member's plan, and the dynamic LDS its
// tiles need at kGroupWG threads; false if a tile of that size is not legal for it.
bool member_shape(const DevPlan& P, int prec, int blocks[GS_COUNT], size_t lds[GS_COUNT]) {
  for (int k = 0; k < GS_COUNT; ++k) {
    blocks[k] = 0;
    lds[k] = 0;
  }
  const int Lx = 2 * P.Mx, Ly = 2 * P.My;
  blocks[GS_STENCIL] = stencil_blocks(P);
  blocks[GS_VEC] = update_blocks(P);
  blocks[GS_FIN] = 1;
  if (P.wg_s) {
    const size_t l = slab_lds_bytes(Lx, kGroupWG, prec);
    if (!l) return false;
    blocks[GS_XFWD] = blocks[GS_XINV] = P.nt;
    lds[GS_XFWD] = lds[GS_XINV] = l;
  } else {
    if (!transform_tile_valid(TK_XFWD, Lx, kGroupWG, prec) || !transform_tile_valid(TK_XINV, Lx, kGroupWG, prec))
      return false;
    const int S = kGroupWG / transform_tps(Lx, prec);
    blocks[GS_XFWD] = blocks[GS_XINV] = (P.nt * P.ny1 + 2 * S - 1) / (2 * S);
    lds[GS_XFWD] = transform_lds_bytes(TK_XFWD, Lx, kGroupWG, prec);
    lds[GS_XINV] = transform_lds_bytes(TK_XINV, Lx, kGroupWG, prec);
    if (P.ny) {
      if (!transform_tile_valid(TK_Y, Ly, kGroupWG, prec)) return false;
      const int Sy = kGroupWG / transform_tps(Ly, prec);
      blocks[GS_Y] = ((P.Mx / 2 + Sy - 1) / Sy) * P.nt;
      lds[GS_Y] = transform_lds_bytes(TK_Y, Ly, kGroupWG, prec);
    }
  }
  if (!transform_tile_valid(TK_TIME, P.nt, kGroupWG, prec)) return false;
  const int St = kGroupWG / transform_tps(P.nt, prec);
  blocks[GS_TIME] = (P.ms / 2 + St - 1) / St;
  lds[GS_TIME] = transform_lds_bytes(TK_TIME, P.nt, kGroupWG, prec);
  return true;
}

template <typename K, typename... A>
abac_status group_launch(abac_group* g, int step, int threads, K kernel, A... args) {
  if (!g->blocks[step]) return ABAC_OK;
  hipLaunchKernelGGL(kernel, dim3(g->blocks[step]), dim3(threads), g->lds[step], g->stream, g->d_table, args...);
  GHIP(hipGetLastError());
  return ABAC_OK;
}

#define GRUN(expr)                   \
  do {                               \
    abac_status s_ = (expr);         \
    if (s_ != ABAC_OK) return s_;    \
  } while (0)

template <typename T>
abac_status group_iteration(abac_group* g) {
  GRUN(group_launch(g, GS_STENCIL, kGroupWG, k_group_stencil<STENCIL_MINRES>));
  GRUN(group_launch(g, GS_FIN, kGroupFinThreads, k_group_fin, (int)FIN_DELTA));
  GRUN(group_launch(g, GS_XFWD, kGroupWG, k_group_xfwd<T>));
  GRUN(group_launch(g, GS_Y, kGroupWG, k_group_y<T>));
  GRUN(group_launch(g, GS_TIME, kGroupWG, k_group_time<T>));
  GRUN(group_launch(g, GS_Y, kGroupWG, k_group_y<T>));
  GRUN(group_launch(g, GS_XINV, kGroupWG, k_group_xinv<T>));
  GRUN(group_launch(g, GS_FIN, kGroupFinThreads, k_group_fin, (int)FIN_GAMMA_ITER));
  GRUN(group_launch(g, GS_VEC, kGroupWG, k_group_update));
  GRUN(group_launch(g, GS_FIN, kGroupFinThreads, k_group_fin, (int)FIN_RNORM));
  GRUN(group_launch(g, GS_VEC, kGroupWG, k_group_form));
  GRUN(group_launch(g, GS_STENCIL, kGroupWG, k_group_stencil<STENCIL_RESIDUAL>));
  GRUN(group_launch(g, GS_FIN, kGroupFinThreads, k_group_fin, (int)FIN_RES));
  return ABAC_OK;
}

// each member's snapshot of every enqueued iteration is complete behind this point
abac_status post_snapshots(abac_group* g, int iterations) {
  for (int it = 0; it < iterations; ++it)
    for (abac_plan* p : g->members) {
      const int slot = (int)(p->ring_posted % kSnapRing);
      GHIP(hipEventRecord(p->ring_ev[slot], g->stream));
      p->ring_posted++;
    }
  return ABAC_OK;
}

abac_status check_members(abac_group* g, int iterations) {
  if (iterations < 0) return gfail(ABAC_EINVAL, "iterations must be >= 0");
  for (abac_plan* p : g->members)
    if (!p->active) return gfail(ABAC_EINVAL, "a member's solve was finished; set the group again");
  return ABAC_OK;
}

// every member's stream waits for the group's work so far (later calls on a member,
// such as abac_minres_finish, are ordered after it)
abac_status group_release(abac_group* g) {
  GHIP(hipEventRecord(g->done, g->stream));
  for (abac_plan* p : g->members) GHIP(hipStreamWaitEvent(p->stream, g->done, 0));
  return ABAC_OK;
}

}  // namespace

namespace abac {
bool group_accepts(const abac_plan* p) {
  if (!p || p->prec == ABAC_PREC_NONE || p->P.small) return false;
  int blocks[GS_COUNT];
  size_t lds[GS_COUNT];
  return member_shape(p->P, p->prec, blocks, lds);
}
}  // namespace abac

extern "C" {

abac_status abac_group_create(void* stream, abac_group** out) {
  if (!out) return gfail(ABAC_EINVAL, "out is NULL");
  *out = nullptr;
  abac_group* g = new abac_group();
  g->stream = static_cast<hipStream_t>(stream);
  g->prec = -1;
  g->d_table = nullptr;
  g->stage_next = 0;
  for (int k = 0; k < kGroupStage; ++k) {
    g->h_stage[k] = nullptr;
    g->stage_ev[k] = nullptr;
  }
  g->joined = g->done = nullptr;
  g->d_sync = nullptr;
  g->device = 0;
  std::memset(g->blocks, 0, sizeof(g->blocks));
  std::memset(g->lds, 0, sizeof(g->lds));
  hipError_t e = hipGetDevice(&g->device);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&g->d_table), sizeof(GroupTable));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&g->d_sync), sizeof(GridSync));
  if (e == hipSuccess) e = hipMemsetAsync(g->d_sync, 0, sizeof(GridSync), g->stream);
  for (int k = 0; e == hipSuccess && k < kGroupStage; ++k) {
    e = hipHostMalloc(reinterpret_cast<void**>(&g->h_stage[k]), sizeof(GroupTable), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->stage_ev[k], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&g->joined, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&g->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    abac_group_destroy(g);
    return gfail(ABAC_ENOMEM, std::string("group set-up: ") + hipGetErrorString(e));
  }
  *out = g;
  return ABAC_OK;
}

abac_status abac_group_destroy(abac_group* g) {
  if (!g) return ABAC_OK;
  (void)hipStreamSynchronize(g->stream);
  for (int k = 0; k < kGroupStage; ++k) {
    if (g->stage_ev[k]) (void)hipEventDestroy(g->stage_ev[k]);
    if (g->h_stage[k]) (void)hipHostFree(g->h_stage[k]);
  }
  if (g->joined) (void)hipEventDestroy(g->joined);
  if (g->done) (void)hipEventDestroy(g->done);
  if (g->d_table) (void)hipFree(g->d_table);
  if (g->d_sync) (void)hipFree(g->d_sync);
  delete g;
  return ABAC_OK;
}

abac_status abac_group_set(abac_group* g, abac_plan* const* plans, int n) {
  set_last_error("");
  if (!g || (n && !plans)) return gfail(ABAC_EINVAL, "NULL argument");
  if (n < 0 || n > kGroupMax) return gfail(ABAC_EINVAL, "a group holds 0.." + std::to_string(kGroupMax) + " plans");
  // the next pinned copy, once its previous upload has completed
  const int k = g->stage_next;
  GHIP(hipEventSynchronize(g->stage_ev[k]));
  GroupTable& H = *g->h_stage[k];
  std::memset(&H, 0, sizeof(GroupTable));
  int prec = -1;
  int blocks[GS_COUNT], total[GS_COUNT] = {0};
  size_t lds[GS_COUNT], lmax[GS_COUNT] = {0};
  for (int r = 0; r < n; ++r) {
    abac_plan* p = plans[r];
    if (!p) return gfail(ABAC_EINVAL, "NULL plan in the group");
    for (int q = 0; q < r; ++q)
      if (plans[q] == p) return gfail(ABAC_EINVAL, "a plan appears twice in the group");
    if (!p->active) return gfail(ABAC_EINVAL, "every member needs a solve begun with abac_minres_begin");
    if (p->prec == ABAC_PREC_NONE) return gfail(ABAC_EINVAL, "members need a preconditioner (FP64 or FP32 transforms)");
    if (p->P.small) return gfail(ABAC_EINVAL, "small 1D plans already run an iteration in one launch");
    if (prec >= 0 && p->prec != prec) return gfail(ABAC_EINVAL, "members must share the transform precision");
    prec = p->prec;
    if (!member_shape(p->P, p->prec, blocks, lds))
      return gfail(ABAC_EINVAL, "a member's transform lengths have no " + std::to_string(kGroupWG) + "-thread tile");
    H.m[r].P = p->P;
    H.m[r].f = p->f;
    H.m[r].u = p->u;
    for (int k = 0; k < GS_COUNT; ++k) {
      H.off[k][r] = total[k];
      total[k] += blocks[k] * p->P.B;
      lmax[k] = std::max(lmax[k], lds[k]);
    }
  }
  for (int k = 0; k < GS_COUNT; ++k) {
    H.off[k][n] = total[k];
    g->blocks[k] = n ? total[k] : 0;
    g->lds[k] = lmax[k];
  }
  H.n = n;
  // the group's stream waits for each member's stream (its set-up), then takes the new
  // table in stream order: launches enqueued before read the old one
  for (int r = 0; r < n; ++r) {
    GHIP(hipEventRecord(g->joined, plans[r]->stream));
    GHIP(hipStreamWaitEvent(g->stream, g->joined, 0));
  }
  GHIP(hipMemcpyAsync(g->d_table, &H, sizeof(GroupTable), hipMemcpyHostToDevice, g->stream));
  GHIP(hipEventRecord(g->stage_ev[k], g->stream));
  g->stage_next = (k + 1) % kGroupStage;
  g->members.assign(plans, plans + n);
  g->prec = prec;
  return ABAC_OK;
}

abac_status abac_group_advance(abac_group* g, int iterations) {
  set_last_error("");
  if (!g) return gfail(ABAC_EINVAL, "NULL group");
  GRUN(check_members(g, iterations));
  for (int it = 0; it < iterations && !g->members.empty(); ++it) {
    GRUN(g->prec == ABAC_PREC_FP32 ? group_iteration<float>(g) : group_iteration<double>(g));
    GRUN(post_snapshots(g, 1));
  }
  return group_release(g);
}

abac_status abac_group_run(abac_group* g, int iterations, int blocks, double timeout_s) {
  set_last_error("");
  if (!g) return gfail(ABAC_EINVAL, "NULL group");
  GRUN(check_members(g, iterations));
  if (!(timeout_s >= 0) || timeout_s > 3600) return gfail(ABAC_EINVAL, "timeout_s must be in [0, 3600]");
  if (blocks < 0) return gfail(ABAC_EINVAL, "blocks must be >= 0");
  if (iterations == 0 || g->members.empty()) return group_release(g);
  const bool fp32 = g->prec == ABAC_PREC_FP32;
  const void* fn = fp32 ? reinterpret_cast<const void*>(&k_group_persistent<float>)
                        : reinterpret_cast<const void*>(&k_group_persistent<double>);
  size_t lds = 0;
  int most = 0;
  for (int k = 0; k < GS_COUNT; ++k) {
    if (k != GS_FIN) lds = std::max(lds, g->lds[k]);
    most = std::max(most, g->blocks[k]);
  }
  const int dev = g->device;
  int cur = 0, ncu = 0, per_cu = 0, khz = 0;
  GHIP(hipGetDevice(&cur));
  if (cur != dev) return gfail(ABAC_EINVAL, "the group's device must be current (the one at abac_group_create)");
  GHIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  GHIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  GHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kGroupWG, lds));
  if (per_cu < 1) return gfail(ABAC_EINVAL, "the members' tiles leave no room for a persistent block");
  // Every block must be resident at once: the grid is capped at what the device holds
  // (the occupancy of this kernel on every CU).  The launch is a plain one: a cooperative
  // launch would also promise residency, but on this runtime it failed in a child process
  // of a process that had made cooperative launches.  A block that other work keeps off the
  // device only delays the barriers until that work ends; past the time limit the
  // launch ends with the abort flag.  A barrier costs each block its own L2
  // write-back and invalidation, which the XCDs serve one block after another (about
  // 65 ns per block on MI355X), while fewer blocks take more logical blocks each (a few
  // microseconds per tile).  The default balances the two, sqrt(48 x the largest
  // step's logical blocks); a multiple of the 8 XCDs keeps the logical blocks of a step
  // on the XCDs the list kernels would give them.
  int grid = blocks ? blocks : (int)std::lround(std::sqrt(48.0 * most));
  grid = std::max(1, std::min(std::min(grid, per_cu * ncu), most));
  if (grid >= 8) grid -= grid % 8;
  unsigned long long deadline =
      (unsigned long long)((timeout_s > 0 ? timeout_s : kGroupTimeout) * (double)khz * 1000.0);
  // a fresh barrier (count, gen, abort); the sticky flag stays for abac_group_check
  GHIP(hipMemsetAsync(g->d_sync, 0, offsetof(GridSync, aborted), g->stream));
  if (fp32)
    hipLaunchKernelGGL((k_group_persistent<float>), dim3(grid), dim3(kGroupWG), lds, g->stream, g->d_table, iterations,
                       g->d_sync, deadline);
  else
    hipLaunchKernelGGL((k_group_persistent<double>), dim3(grid), dim3(kGroupWG), lds, g->stream, g->d_table,
                       iterations, g->d_sync, deadline);
  GHIP(hipGetLastError());
  GRUN(post_snapshots(g, iterations));
  return group_release(g);
}

abac_status abac_group_check(abac_group* g, int* aborted) {
  set_last_error("");
  if (!g || !aborted) return gfail(ABAC_EINVAL, "NULL argument");
  int flag = 0;
  GHIP(hipStreamSynchronize(g->stream));
  GHIP(hipMemcpy(&flag, &g->d_sync->aborted, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) GHIP(hipMemset(&g->d_sync->aborted, 0, sizeof(int)));
  *aborted = flag;
  return ABAC_OK;
}

}  // extern "C"

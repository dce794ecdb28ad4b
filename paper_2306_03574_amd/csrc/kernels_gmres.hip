// Restarted GMRES with right preconditioning by the block alpha-circulant matrix
// C_alpha (eqs. (1.5)-(1.7)) for the non-symmetric all-at-once system T u = f
// (eq. (1.2)); C_alpha^{-1} is applied by the transform passes with the single time
// pass of weights mu^{-1}.
//
// One Arnoldi step j (all right-hand sides in lockstep, grid.y = RHS):
//   z = C^{-1} v_j;  w = T z;
//   classical Gram-Schmidt: h1 = V^T w, w -= V h1; a second pass h2 = V^T w, w -= V h2
//   only when the first removed more than half of ||w||^2 (the Daniel-Gragg-Kaufman-
//   Stewart test with eta = 1/sqrt(2), ||w - V h1||^2 = ||w||^2 - ||h1||^2 in exact
//   arithmetic); the dots of the second pass ride along with the update of the first;
//   fixed-order sums;
//   H(:, j) = h1 + h2, H(j+1, j) = ||w||;  Givens rotations;  v_{j+1} = w / ||w||.
// Slot l holds v_l / sig_l: w is formed in the slot of v_{j+1} from the unnormalised
// v_j, so its coefficients carry the factor sig_j, and v_{j+1} = w / ||w|| is never
// written out (sig_{j+1} = 1 / ||w||).  Slot 0 is written normalised (sig_0 = 1).
// When the rotated residual meets tol, the cycle ends or maxit is reached, the iterate
// u = X0 + C^{-1}(V y) is formed (X0: the iterate at the start of the cycle) and the
// residual f - T u is checked explicitly; at the end of a cycle the next one starts
// from that residual.  Every reduction is a per-block partial summed in index order by
// a one-block-per-RHS kernel (deterministic, no atomics).
#include "abac_internal.h"

namespace abac {

namespace {

constexpr int kGFinThreads = 1024;

__device__ __forceinline__ void elem_range(const DevPlan& P, size_t* lo, size_t* hi) {
  const int nblk = gridDim.x;
  const size_t per = ((size_t)P.N + nblk - 1) / nblk;
  *lo = (size_t)blockIdx.x * per;
  *hi = *lo + per < (size_t)P.N ? *lo + per : (size_t)P.N;
}

__device__ __forceinline__ double* gpart(const DevPlan& P, int b, int l) {
  return P.gparts + ((size_t)b * (kGmresMax + 1) + l) * kVecMaxBlocks;
}

// v_0 = f (normalised later), X0 = 0, u = 0; ||f||^2 partials.
__global__ void __launch_bounds__(kVecThreads)
k_ginit(DevPlan P, const double* __restrict__ f, double* __restrict__ u) {
  const int b = blockIdx.y;
  const size_t off = (size_t)b * P.N;
  double* v0 = gslot(P, 0) + off;
  double* x0 = P.R + off;
  size_t lo, hi;
  elem_range(P, &lo, &hi);
  double acc = 0.0;
  for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    const double v = f[off + e];
    v0[e] = v;
    x0[e] = 0.0;
    u[off + e] = 0.0;
    acc += v * v;
  }
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_RNORM, b)[blockIdx.x] = bs;
}

// partial sums of <v_l, w>, l = 0..J, and of <w, w> (slot J+1), for the first
// Gram-Schmidt pass (the second pass's dots come from the first update sweep)
template <int J>
__device__ __forceinline__ void gdots_body(const DevPlan& P, int b, const double* __restrict__ w) {
  const size_t off = (size_t)b * P.N;
  const double* vs[J + 1];
#pragma unroll
  for (int l = 0; l <= J; ++l) vs[l] = gslot(P, l) + off;
  const double* ww = w + off;
  double acc[J + 2];
#pragma unroll
  for (int l = 0; l <= J + 1; ++l) acc[l] = 0.0;
  size_t lo, hi;
  elem_range(P, &lo, &hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    const double x = ww[e];
    double v[J + 1];
#pragma unroll
    for (int l = 0; l <= J; ++l) v[l] = vs[l][e];
#pragma unroll
    for (int l = 0; l <= J; ++l) acc[l] += v[l] * x;
    acc[J + 1] += x * x;
  }
#pragma unroll
  for (int l = 0; l <= J + 1; ++l) {
    const double bs = block_sum(acc[l]);
    if (threadIdx.x == 0) gpart(P, b, l)[blockIdx.x] = bs;
  }
}

// w -= sum_l h_l v_l (h = h1 on pass 1, h2 on pass 2) and ||w||^2 partials (pass 2,
// when it runs, replaces those of pass 1).  Pass 1 also forms the partial sums of
// <v_l, w> of the updated w for the second pass while v_l and w are in registers.
template <int J>
__device__ __forceinline__ void gaxpy_body(const DevPlan& P, int b, int pass, double* __restrict__ w) {
  const GmresState* st = P.gst + b;
  const size_t off = (size_t)b * P.N;
  const double* vs[J + 1];
  double h[J + 1];
#pragma unroll
  for (int l = 0; l <= J; ++l) {
    vs[l] = gslot(P, l) + off;
    h[l] = (pass == 1 ? st->h1[l] : st->h2[l]) * st->sig[l];
  }
  double* ww = w + off;
  size_t lo, hi;
  elem_range(P, &lo, &hi);
  double acc = 0.0;
  double dots[J + 1];
#pragma unroll
  for (int l = 0; l <= J; ++l) dots[l] = 0.0;
  for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    double v[J + 1];
#pragma unroll
    for (int l = 0; l <= J; ++l) v[l] = vs[l][e];
    double x = ww[e];
#pragma unroll
    for (int l = 0; l <= J; ++l) x -= h[l] * v[l];
    ww[e] = x;
    acc += x * x;
    if (pass == 1) {
#pragma unroll
      for (int l = 0; l <= J; ++l) dots[l] += v[l] * x;
    }
  }
  if (pass == 1 && st->reorth) {
#pragma unroll
    for (int l = 0; l <= J; ++l) {
      const double bd = block_sum(dots[l]);
      if (threadIdx.x == 0) gpart(P, b, l)[blockIdx.x] = bd;
    }
  }
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_RNORM, b)[blockIdx.x] = bs;
}

// t = sum_l y_l v_l, l = 0..J
template <int J>
__device__ __forceinline__ void gcomb_body(const DevPlan& P, int b, double* __restrict__ t) {
  const GmresState* st = P.gst + b;
  const size_t off = (size_t)b * P.N;
  const double* vs[J + 1];
  double y[J + 1];
#pragma unroll
  for (int l = 0; l <= J; ++l) {
    vs[l] = gslot(P, l) + off;
    y[l] = st->y[l] * st->sig[l];
  }
  double* tt = t + off;
  size_t lo, hi;
  elem_range(P, &lo, &hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    double v[J + 1];
#pragma unroll
    for (int l = 0; l <= J; ++l) v[l] = vs[l][e];
    double x = 0.0;
#pragma unroll
    for (int l = 0; l <= J; ++l) x += y[l] * v[l];
    tt[e] = x;
  }
}

#define ABAC_GCASES(CALL) \
  CALL(0) CALL(1) CALL(2) CALL(3) CALL(4) CALL(5) CALL(6) CALL(7) CALL(8) CALL(9) CALL(10) CALL(11) CALL(12) \
  CALL(13) CALL(14)
static_assert(kGmresMax == 15, "the dispatch lists one case per Arnoldi column j = 0 .. kGmresMax - 1");

__global__ void __launch_bounds__(kVecThreads)
k_gdots(DevPlan P, int j, const double* __restrict__ w) {
  const int b = blockIdx.y;
  if (P.gst[b].state != ST_RUNNING) return;
  switch (j) {
#define CASE(K) \
    case K: gdots_body<K>(P, b, w); break;
    ABAC_GCASES(CASE)
#undef CASE
    default: break;
  }
}

__global__ void __launch_bounds__(kVecThreads)
k_gaxpy(DevPlan P, int j, int pass, double* __restrict__ w) {
  const int b = blockIdx.y;
  if (P.gst[b].state != ST_RUNNING || (pass == 2 && !P.gst[b].reorth)) return;
  switch (j) {
#define CASE(K) \
    case K: gaxpy_body<K>(P, b, pass, w); break;
    ABAC_GCASES(CASE)
#undef CASE
    default: break;
  }
}

__global__ void __launch_bounds__(kVecThreads)
k_gcomb(DevPlan P, int j, double* __restrict__ t) {
  const int b = blockIdx.y;
  const GmresState* st = P.gst + b;
  if (st->state != ST_RUNNING || !st->need) return;
  switch (j) {
#define CASE(K) \
    case K: gcomb_body<K>(P, b, t); break;
    ABAC_GCASES(CASE)
#undef CASE
    default: break;
  }
}

// v_0 = src * scale: at set-up (src = v_0 itself) for running right-hand sides, or at a
// restart (src = the explicit residual) for those that restart, which also commit
// X0 = u.
__global__ void __launch_bounds__(kVecThreads)
k_gbase(DevPlan P, const double* __restrict__ src, const double* __restrict__ u, int restart_step) {
  const int b = blockIdx.y;
  const GmresState* st = P.gst + b;
  if (st->state != ST_RUNNING || (restart_step && !st->restart_now)) return;
  const size_t off = (size_t)b * P.N;
  double* v0 = gslot(P, 0) + off;
  double* x0 = P.R + off;
  const double sc = st->scale;
  size_t lo, hi;
  elem_range(P, &lo, &hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    v0[e] = src[off + e] * sc;
    if (restart_step) x0[e] = u[off + e];
  }
}

// u = X0 + z for right-hand sides that form their iterate
__global__ void __launch_bounds__(kVecThreads)
k_gaddx(DevPlan P, double* __restrict__ u, const double* __restrict__ z) {
  const int b = blockIdx.y;
  const GmresState* st = P.gst + b;
  if (st->state != ST_RUNNING || !st->need) return;
  const size_t off = (size_t)b * P.N;
  const double* x0 = P.R + off;
  size_t lo, hi;
  elem_range(P, &lo, &hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) u[off + e] = x0[e] + z[off + e];
}

__device__ void write_flags(const DevPlan& P, int b, const GmresState* st) {
  GmresFlags f;
  f.state = st->state;
  f.need = st->need;
  f.k = st->k;
  f.iter = st->iter;
  P.gflags[b] = f;
}

// The scalar steps, one block per right-hand side.
__global__ void __launch_bounds__(kGFinThreads)
k_gfin(DevPlan P, int kind, int nparts, double tol, int maxit, int restart) {
  const int b = blockIdx.x;
  GmresState* st = P.gst + b;
  if (kind != G_INIT && (st->state != ST_RUNNING || (kind == G_CHECK && !st->need))) {
    if (threadIdx.x == 0) write_flags(P, b, st);
    return;
  }
  if (kind == G_DOTS1 || kind == G_DOTS2) {
    const int j = st->k;
    if (kind == G_DOTS2 && !st->reorth) {   // no second pass: h2 = 0 (set by G_DOTS1)
      if (threadIdx.x == 0) write_flags(P, b, st);
      return;
    }
    double* h = kind == G_DOTS1 ? st->h1 : st->h2;
    double hh = 0.0;
    for (int l = 0; l <= j; ++l) {
      const double tot = sum_parts(gpart(P, b, l), nparts) * st->sig[l];
      if (threadIdx.x == 0) {
        h[l] = tot;
        hh += tot * tot;
      }
    }
    const double ww = kind == G_DOTS1 ? sum_parts(gpart(P, b, j + 1), nparts) : 0.0;
    if (threadIdx.x == 0) {
      if (kind == G_DOTS1) {
        // second pass unless the first kept more than half of ||w||^2
        const double left = ww - hh;
        st->reorth = !(left >= 0.5 * ww) || !(ww == ww) ? 1 : 0;
        if (!st->reorth)
          for (int l = 0; l <= j; ++l) st->h2[l] = 0.0;
      }
      st->restart_now = 0;   // the restart copy (if any) has run
      write_flags(P, b, st);
    }
    return;
  }
  const double tot = sum_parts(part_slot(P, kind == G_CHECK ? PART_RES : PART_RNORM, b), nparts);
  if (threadIdx.x != 0) return;
  switch (kind) {
    case G_INIT:
      st->bnorm2 = tot;
      st->tol2 = tol * tol;
      st->maxit = maxit;
      st->restart = restart;
      st->iter = 0;
      st->k = 0;
      st->explicit_mode = 0;
      st->need = 0;
      st->restart_now = 0;
      st->res2 = tot;
      st->status = 0;
      for (int l = 0; l <= kGmresMax; ++l) st->g[l] = 0.0;
      if (tot == 0.0) {
        st->state = ST_DONE;   // u = 0 is exact
      } else if (!(tot == tot) || tot > 1e300) {
        st->state = ST_DONE;
        st->status = -5;
      } else {
        st->state = ST_RUNNING;
        st->g[0] = sqrt(tot);
        st->scale = 1.0 / st->g[0];
        st->sig[0] = 1.0;
      }
      break;
    case G_NORM: {
      const int j = st->k;
      if (!(tot >= 0.0) || !(tot < 1e300)) {
        st->state = ST_DONE;
        st->status = -5;   // ABAC_EBREAKDOWN
        break;
      }
      const double hn = sqrt(tot);   // of w formed from the unnormalised v_j: times sig_j below
      double* col = st->H + (size_t)j * (kGmresMax + 1);
      const double sj = st->sig[j];
      for (int l = 0; l <= j; ++l) col[l] = sj * (st->h1[l] + st->h2[l]);
      col[j + 1] = sj * hn;
      st->sig[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
      for (int l = 0; l < j; ++l) {   // earlier rotations on the new column
        const double t = st->cs[l] * col[l] + st->sn[l] * col[l + 1];
        col[l + 1] = -st->sn[l] * col[l] + st->cs[l] * col[l + 1];
        col[l] = t;
      }
      const double rho = hypot(col[j], col[j + 1]);
      const double c = rho > 0.0 ? col[j] / rho : 1.0, s = rho > 0.0 ? col[j + 1] / rho : 0.0;
      st->cs[j] = c;
      st->sn[j] = s;
      col[j] = rho;
      col[j + 1] = 0.0;
      st->g[j + 1] = -s * st->g[j];
      st->g[j] = c * st->g[j];
      st->iter += 1;
      st->k = j + 1;
      st->resid2 = st->g[j + 1] * st->g[j + 1];
      st->need = st->resid2 <= st->tol2 * st->bnorm2 || st->explicit_mode || st->k == st->restart ||
                 st->iter >= st->maxit || hn == 0.0;
      if (st->need) {
        // back substitution with the rotated (upper triangular) H
        for (int r = j; r >= 0; --r) {
          double v = st->g[r];
          for (int c2 = r + 1; c2 <= j; ++c2) v -= st->H[(size_t)c2 * (kGmresMax + 1) + r] * st->y[c2];
          const double d = st->H[(size_t)r * (kGmresMax + 1) + r];
          st->y[r] = d != 0.0 ? v / d : 0.0;
        }
      }
      break;
    }
    case G_CHECK:
      st->res2 = tot;
      st->need = 0;
      if (tot <= st->tol2 * st->bnorm2) {
        st->state = ST_DONE;
        st->status = 0;
      } else if (!(tot == tot) || tot > 1e300) {
        st->state = ST_DONE;
        st->status = -5;
      } else if (st->iter >= st->maxit) {
        st->state = ST_DONE;
        st->status = -4;   // ABAC_ENOTCONV
      } else if (st->k >= st->restart) {
        // next cycle from the explicit residual
        st->restart_now = 1;
        st->k = 0;
        st->explicit_mode = 0;
        for (int l = 0; l <= kGmresMax; ++l) st->g[l] = 0.0;
        st->g[0] = sqrt(tot);
        st->scale = 1.0 / st->g[0];
        st->sig[0] = 1.0;
      } else {
        st->explicit_mode = 1;   // the rotated residual was optimistic: check every step
      }
      break;
    default:
      break;
  }
  write_flags(P, b, st);
}

}  // namespace

hipError_t launch_ginit(const DevPlan& P, const double* f, double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_ginit, dim3(update_blocks(P), P.B), dim3(kVecThreads), 0, s, P, f, u);
  return hipGetLastError();
}

hipError_t launch_gfin(const DevPlan& P, int kind, double tol, int maxit, int restart, hipStream_t s) {
  const int nparts = kind == G_CHECK ? stencil_grid(P, STENCIL_RESVEC) : update_blocks(P);
  hipLaunchKernelGGL(k_gfin, dim3(P.B), dim3(kGFinThreads), 0, s, P, kind, nparts, tol, maxit, restart);
  return hipGetLastError();
}

hipError_t launch_gdots(const DevPlan& P, int j, const double* w, hipStream_t s) {
  if (j < 0 || j >= kGmresMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gdots, dim3(update_blocks(P), P.B), dim3(kVecThreads), 0, s, P, j, w);
  return hipGetLastError();
}

hipError_t launch_gaxpy(const DevPlan& P, int j, int pass, double* w, hipStream_t s) {
  if (j < 0 || j >= kGmresMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gaxpy, dim3(update_blocks(P), P.B), dim3(kVecThreads), 0, s, P, j, pass, w);
  return hipGetLastError();
}

hipError_t launch_gbase(const DevPlan& P, const double* src, const double* u, int restart_step, hipStream_t s) {
  hipLaunchKernelGGL(k_gbase, dim3(update_blocks(P), P.B), dim3(kVecThreads), 0, s, P, src, u, restart_step);
  return hipGetLastError();
}

hipError_t launch_gcomb(const DevPlan& P, int j, double* t, hipStream_t s) {
  if (j < 0 || j >= kGmresMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gcomb, dim3(update_blocks(P), P.B), dim3(kVecThreads), 0, s, P, j, t);
  return hipGetLastError();
}

hipError_t launch_gaddx(const DevPlan& P, double* u, const double* z, hipStream_t s) {
  hipLaunchKernelGGL(k_gaddx, dim3(update_blocks(P), P.B), dim3(kVecThreads), 0, s, P, u, z);
  return hipGetLastError();
}

}  // namespace abac

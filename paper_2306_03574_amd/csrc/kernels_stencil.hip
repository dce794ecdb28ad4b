// Stencil and vector kernels of the ABAC MINRES path:
//   * Y T x matvec (eqs. (1.2), (1.4)) as an HBM sweep that marches over time levels
//     from both ends at once, so that <Y T z, z> pairs level k of T z with level
//     nt-1-k of z without a second read of z;
//   * the explicit residual ||f - T u|| used to confirm convergence;
//   * right-hand side assembly of eq. (1.2);
//   * solve set-up, the MINRES w / x / r update and the scalar steps (Givens QR of the
//     Lanczos tridiagonal matrix, stopping test) run by one block per right-hand side.
#include "abac_internal.h"
#include "minres_device.h"
#include "stencil_device.h"

namespace abac {

namespace {


// One kernel per mode and coefficient kind, so each gets the registers its own path
// needs.
template <int MODE, bool VAR>
__global__ void __launch_bounds__(kStencilThreads)
k_stencil(DevPlan P, const double* __restrict__ xin, double* __restrict__ yout, const double* __restrict__ fref) {
  const int b = blockIdx.y;
  MinresState* st = P.st + b;
  const double* x = xin;
  double* y = yout;
  if (MODE == STENCIL_MINRES) {
    if (st->state != ST_RUNNING) return;
    const int j = st->iter + 1;
    x = P.Z[zslot(j)];
    y = P.V[(j + 1) % 3];
  } else if (MODE == STENCIL_RESIDUAL) {
    // explicit residual only when the form kernel asked for a check
    if (st->state != ST_RUNNING || !st->need_check) return;
  }
  x += (size_t)b * P.N;
  if (y) y += (size_t)b * P.N;
  const double* f = fref ? fref + (size_t)b * P.N : nullptr;
  if (MODE == STENCIL_PLAIN) {
    stencil_run<VAR, OUT_REV, false>(P, x, y, f, blockIdx.x, gridDim.x, threadIdx.x, true);
    return;
  }
  if (MODE == STENCIL_T) {
    stencil_run<VAR, OUT_NAT, false>(P, x, y, f, blockIdx.x, gridDim.x, threadIdx.x, true);
    return;
  }
  double acc;
  if (MODE == STENCIL_MINRES)
    acc = stencil_run<VAR, OUT_REV, true>(P, x, y, f, blockIdx.x, gridDim.x, threadIdx.x, true);
  else if (MODE == STENCIL_RESVEC)
    acc = stencil_run<VAR, OUT_RESVEC, false>(P, x, y, f, blockIdx.x, gridDim.x, threadIdx.x, true);
  else
    acc = stencil_run<VAR, OUT_RESNORM, false>(P, x, y, f, blockIdx.x, gridDim.x, threadIdx.x, true);
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, MODE == STENCIL_MINRES ? PART_DELTA : PART_RES, b)[blockIdx.x] = bs;
}

// f_1 = tau^2 src_0 / 2 + tau psi1 + psi0; f_2 = tau^2 src_1 - L psi0; f_k = tau^2 src_{k-1}
__global__ void __launch_bounds__(kVecThreads)
k_rhs(DevPlan P, const double* __restrict__ src, const double* __restrict__ psi0,
      const double* __restrict__ psi1, double* __restrict__ f) {
  const size_t total = (size_t)P.B * P.N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t b = e / P.N;
    const size_t r = e - b * P.N;
    const int k = (int)(r / P.m);
    const int i = (int)(r - (size_t)k * P.m);
    const double s = src[e];
    double v = P.tau2 * s;
    if (k == 0) {
      v = 0.5 * P.tau2 * s + P.tau * psi1[b * P.m + i] + psi0[b * P.m + i];
    } else if (k == 1) {
      v -= apply_L(l_coef(P, i % P.nx, i / P.nx), psi0 + b * P.m, i);
    }
    f[e] = v;
  }
}

// Set-up of a solve: b = Y f into V_1, zero u; ||b||^2 partials.  (r_0 = b is read from
// V_1 by the first residual update, v_0 is never read, and the w vectors are written
// by the flush of the resident basis before they are first read.)
__global__ void __launch_bounds__(kVecThreads)
k_init(DevPlan P, const double* __restrict__ f, double* __restrict__ u) {
  const int b = blockIdx.y;
  const size_t off = (size_t)b * P.N;
  const int nblk = gridDim.x;
  const size_t per = ((size_t)P.N + nblk - 1) / nblk;
  const size_t lo = (size_t)blockIdx.x * per;
  const size_t hi = lo + per < (size_t)P.N ? lo + per : (size_t)P.N;
  double acc = 0.0;
  for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    const int k = (int)(e / P.m);
    const size_t i = e - (size_t)k * P.m;
    const double v = f[off + (size_t)(P.nt - 1 - k) * P.m + i];
    P.V[1][off + e] = v;   // v_1 = r_0 (the first update reads it as r_0)
    u[off + e] = 0.0;
    acc += v * v;
  }
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_RNORM, b)[blockIdx.x] = bs;
}

// Residual recurrence r = r1 r + r2 V_{j+1} and ||r||^2 partials; after the resident
// basis (j > kBasis) also w_j = wa Z_j - wb w_{j-1} - wc w_{j-2} and x += xc w_j.
__global__ void __launch_bounds__(kVecThreads)
k_update(DevPlan P, double* __restrict__ u) {
  const int b = blockIdx.y;
  if (P.st[b].state != ST_RUNNING) return;
  const double acc = update_part(P, b, u, blockIdx.x, gridDim.x);
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_RNORM, b)[blockIdx.x] = bs;
}

// Forms u (and at the flush w_j, w_{j-1}) from the resident basis for the right-hand
// sides whose scalar step (FIN_RNORM or FIN_FINAL) set form_now; the others return at
// once.  Writes no solve state.
__global__ void __launch_bounds__(kVecThreads)
k_form(DevPlan P, double* __restrict__ u) {
  const int b = blockIdx.y;
  const MinresState* st = P.st + b;
  if (!st->form_now) return;
  const int nb = st->nbasis;
  if (st->flush_now) form_dispatch<true>(P, b, nb, u, blockIdx.x, gridDim.x);
  else form_dispatch<false>(P, b, nb, u, blockIdx.x, gridDim.x);
}

// Identity preconditioner (MINRES-I): z = q, with the Lanczos step fused in.
__global__ void __launch_bounds__(kVecThreads)
k_identity(DevPlan P, int mode, const double* __restrict__ in, double* __restrict__ out) {
  const int b = blockIdx.y;
  const size_t off = (size_t)b * P.N;
  const int nblk = gridDim.x;
  const size_t per = ((size_t)P.N + nblk - 1) / nblk;
  const size_t lo = (size_t)blockIdx.x * per;
  const size_t hi = lo + per < (size_t)P.N ? lo + per : (size_t)P.N;
  if (mode == INV_PLAIN) {
    for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) out[off + e] = in[off + e];
    return;
  }
  const MinresState* st = P.st + b;
  if (st->state != ST_RUNNING) return;
  double acc = 0.0;
  if (mode == INV_GAMMA_INIT) {
    const double* __restrict__ q = P.V[1] + off;
    double* __restrict__ z = P.Z[zslot(1)] + off;
    for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
      const double v = q[e];
      z[e] = v;
      acc += v * v;
    }
  } else {
    const int j = st->iter + 1;
    double* __restrict__ q = P.V[(j + 1) % 3] + off;
    const double* __restrict__ vj = P.V[j % 3] + off;
    const double* __restrict__ vjm1 = P.V[j == 1 ? j % 3 : (j + 2) % 3] + off;   // v_0 has weight 0 at j = 1
    double* __restrict__ z = P.Z[zslot(j + 1)] + off;
    const double cA = st->sig, cB = st->delta * st->sig, cC = st->gamma * st->sig_prev;
    for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
      const double v = cA * q[e] - cB * vj[e] - cC * vjm1[e];
      q[e] = v;
      z[e] = v;
      acc += v * v;
    }
  }
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_GAMMA, b)[blockIdx.x] = bs;
}

constexpr int kFinThreads = 1024;

__global__ void __launch_bounds__(kFinThreads)
k_fin(DevPlan P, int kind, int nparts, double tol, int maxit) {
  const int b = blockIdx.x;
  if (!fin_begin(P, b, kind)) return;
  const double tot = sum_parts(part_slot(P, fin_part_kind(kind), b), nparts);
  if (threadIdx.x == 0) fin_scalar(P, b, kind, tot, tol, maxit);
}

}  // namespace

int stencil_grid(const DevPlan& P, int mode) {
  (void)mode;
  return stencil_blocks(P);
}

int update_blocks(const DevPlan& P) {
  long long want = (P.N + (long long)kVecThreads * kVecPerThread - 1) / ((long long)kVecThreads * kVecPerThread);
  if (want > kVecMaxBlocks) want = kVecMaxBlocks;
  if (want < 1) want = 1;
  return (int)want;
}

hipError_t launch_stencil(const DevPlan& P, int mode, const double* x, double* y, const double* f, hipStream_t s) {
  dim3 grid(stencil_grid(P, mode), P.B);
  const dim3 block(P.st_threads);
#define ABAC_STENCIL_CASE(M)                                                                           \
  case M:                                                                                              \
    if (P.coef_x)                                                                                      \
      hipLaunchKernelGGL((k_stencil<M, true>), grid, block, 0, s, P, x, y, f);                         \
    else                                                                                               \
      hipLaunchKernelGGL((k_stencil<M, false>), grid, block, 0, s, P, x, y, f);                        \
    break;
  switch (mode) {
    ABAC_STENCIL_CASE(STENCIL_PLAIN)
    ABAC_STENCIL_CASE(STENCIL_MINRES)
    ABAC_STENCIL_CASE(STENCIL_RESIDUAL)
    ABAC_STENCIL_CASE(STENCIL_REPORT)
    ABAC_STENCIL_CASE(STENCIL_T)
    ABAC_STENCIL_CASE(STENCIL_RESVEC)
    default: return hipErrorInvalidValue;
  }
#undef ABAC_STENCIL_CASE
  return hipGetLastError();
}

hipError_t launch_rhs(const DevPlan& P, const double* src, const double* psi0, const double* psi1, double* f,
                      hipStream_t s) {
  long long total = (long long)P.B * P.N;
  long long blocks = (total + kVecThreads - 1) / kVecThreads;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)blocks), dim3(kVecThreads), 0, s, P, src, psi0, psi1, f);
  return hipGetLastError();
}

hipError_t launch_init(const DevPlan& P, const double* f, double* u, double tol, int maxit, hipStream_t s) {
  dim3 grid(update_blocks(P), P.B);
  hipLaunchKernelGGL(k_init, grid, dim3(kVecThreads), 0, s, P, f, u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_fin(P, FIN_BNORM, tol, maxit, s);
}

hipError_t launch_update(const DevPlan& P, double* u, hipStream_t s) {
  dim3 grid(update_blocks(P), P.B);
  hipLaunchKernelGGL(k_update, grid, dim3(kVecThreads), 0, s, P, u);
  return hipGetLastError();
}

hipError_t launch_form(const DevPlan& P, double* u, hipStream_t s) {
  dim3 grid(update_blocks(P), P.B);
  hipLaunchKernelGGL(k_form, grid, dim3(kVecThreads), 0, s, P, u);
  return hipGetLastError();
}

hipError_t launch_identity(const DevPlan& P, int mode, const double* in, double* out, hipStream_t s) {
  dim3 grid(update_blocks(P), P.B);
  hipLaunchKernelGGL(k_identity, grid, dim3(kVecThreads), 0, s, P, mode, in, out);
  return hipGetLastError();
}

hipError_t launch_fin(const DevPlan& P, int kind, double tol, int maxit, hipStream_t s) {
  int nparts;
  switch (kind) {
    case FIN_BNORM:
    case FIN_RNORM: nparts = update_blocks(P); break;
    case FIN_DELTA: nparts = stencil_grid(P, STENCIL_MINRES); break;
    case FIN_GAMMA_INIT:
    case FIN_GAMMA_ITER: nparts = P.gamma_nparts; break;
    default: nparts = stencil_grid(P, STENCIL_RESIDUAL); break;
  }
  hipLaunchKernelGGL(k_fin, dim3(P.B), dim3(kFinThreads), 0, s, P, kind, nparts, tol, maxit);
  return hipGetLastError();
}

}  // namespace abac

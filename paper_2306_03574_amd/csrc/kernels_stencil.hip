// Stencil and vector kernels of the ABAC MINRES path:
//   * Y T x matvec (eqs. (1.2), (1.4)) as an HBM sweep that marches over time levels
//     from both ends at once, so that <Y T z, z> pairs level k of T z with level
//     nt-1-k of z without a second read of z;
//   * the explicit residual ||f - T u|| used to confirm convergence;
//   * right-hand side assembly of eq. (1.2);
//   * solve set-up, the MINRES w / x / r update and the scalar steps (Givens QR of the
//     Lanczos tridiagonal matrix, stopping test) run by one block per right-hand side.
#include "abac_internal.h"

namespace abac {

namespace {

constexpr int kVecThreads = 256;
constexpr int kVecPerThread = 16;
constexpr int kVecMaxBlocks = 1024;

// Weights and neighbour offsets of L at one spatial point:
//   (L s)_i = c s_i - w s_{i-1} - e s_{i+1} - so s_{i-nx} - no s_{i+nx}.
// Constant coefficient: L = I - (tau^2/2) Delta_h (eq. (1.2)).  Variable coefficient:
// L_a = I - (tau^2/2) Delta_{a,h} (eq. (3.2)) with the face weights of the plan.  A
// neighbour outside the grid is a zero Dirichlet value: its face weight stays in c,
// its own weight is 0 and its offset points back at the centre, so every load is
// unconditional and in bounds (no divergent branches around the loads, which would
// serialise them).
struct LCoef {
  double c, w, e, so, no;
  int ow, oe, os, on;   // offsets of the four neighbours (0 where outside the grid)
};

__device__ __forceinline__ LCoef l_coef(const DevPlan& P, int ix, int iy) {
  double w = P.cx, e = P.cx, so = P.cy, no = P.cy;
  if (P.coef_x) {
    const double* fx = P.coef_x + (size_t)iy * P.Mx + ix;
    w = fx[0];
    e = fx[1];
    so = no = 0.0;
    if (P.ny) {
      const double* fy = P.coef_y + (size_t)iy * P.nx + ix;
      so = fy[0];
      no = fy[P.nx];
    }
  }
  LCoef q;
  q.c = P.coef_x ? 1.0 + (w + e) + (so + no) : P.c0;
  const bool hw = ix > 0, he = ix < P.nx - 1;
  const bool hs = P.ny && iy > 0, hn = P.ny && iy < P.ny - 1;
  q.w = hw ? w : 0.0;
  q.e = he ? e : 0.0;
  q.so = hs ? so : 0.0;
  q.no = hn ? no : 0.0;
  q.ow = hw ? -1 : 0;
  q.oe = he ? 1 : 0;
  q.os = hs ? -P.nx : 0;
  q.on = hn ? P.nx : 0;
  return q;
}

// The five values of one level that (L s)_i reads, and L applied to them.
struct Lvl5 {
  double c, w, e, s, n;
};

__device__ __forceinline__ Lvl5 load5(const LCoef& q, const double* __restrict__ lvl, int i) {
  return {lvl[i], lvl[i + q.ow], lvl[i + q.oe], lvl[i + q.os], lvl[i + q.on]};
}

__device__ __forceinline__ double L_of(const LCoef& q, const Lvl5& v) {
  return q.c * v.c - (q.w * v.w + q.e * v.e) - (q.so * v.s + q.no * v.n);
}

// (L s)_i of one level.
__device__ __forceinline__ double apply_L(const LCoef& q, const double* __restrict__ lvl, int i) {
  return L_of(q, load5(q, lvl, i));
}

// One logical block of the matvec: spatial tile `tile`, forward levels [k0, k1) and
// their mirrors nt-1-k.  Returns this thread's contribution to the fused reduction
// (RES: sum of squared residuals against f; DOT: <Y T x, x>).  The march keeps L of
// the two previous levels in registers; every load is unconditional, so the loads of
// a step (and of the unrolled next step) are all in flight together.
template <bool RES, bool DOT>
__device__ __forceinline__ double stencil_tile(const DevPlan& P, const double* __restrict__ x,
                                               double* __restrict__ y, const double* __restrict__ f, int tile,
                                               int chunk) {
  const int n = P.nt, m = P.m;
  const int i = tile * kStencilThreads + threadIdx.x;
  if (i >= m) return 0.0;
  const LCoef q = l_coef(P, i % P.nx, i / P.nx);   // loaded once, reused on every level
  const int k0 = chunk * P.st_chunk;
  const int k1 = min(k0 + P.st_chunk, n / 2);
  double acc = 0.0;
  // forward march state: x_{k-1} and L of x_{k-1}, x_{k-2} (zero before level 0); the
  // loads come from a clamped level and are selected away, so they are unconditional
  const int a2 = max(k0 - 2, 0), a1 = max(k0 - 1, 0);
  const Lvl5 p2 = load5(q, x + (size_t)a2 * m, i), p1 = load5(q, x + (size_t)a1 * m, i);
  double Lf2 = k0 >= 2 ? L_of(q, p2) : 0.0;
  double zf1 = k0 >= 1 ? p1.c : 0.0, Lf1 = k0 >= 1 ? L_of(q, p1) : 0.0;
  // backward march state at kb = n-1-k0: x_kb, x_{kb-1} and L of them
  const int kb0 = n - 1 - k0;
  double zb0 = x[(size_t)kb0 * m + i], Lb0 = apply_L(q, x + (size_t)kb0 * m, i);
  double zb1 = x[(size_t)(kb0 - 1) * m + i], Lb1 = apply_L(q, x + (size_t)(kb0 - 1) * m, i);
  // two levels per trip (chunks are even): both steps' loads are issued together
#pragma unroll 2
  for (int k = k0; k < k1; ++k) {
    const Lvl5 cf = load5(q, x + (size_t)k * m, i);              // forward level k
    const Lvl5 cb = load5(q, x + (size_t)(n - 3 - k) * m, i);    // backward level kb - 2
    const double zk = cf.c, Lk = L_of(q, cf);
    const double out_f = Lk + Lf2 - 2.0 * zf1;          // (T x)_k
    const double zb2 = cb.c, Lb2 = L_of(q, cb);
    const double out_b = Lb0 + Lb2 - 2.0 * zb1;         // (T x)_kb, kb = n-1-k
    if (RES) {
      const double rf = f[(size_t)k * m + i] - out_f;
      const double rb = f[(size_t)(n - 1 - k) * m + i] - out_b;
      acc += rf * rf + rb * rb;
    } else {
      y[(size_t)(n - 1 - k) * m + i] = out_f;           // Y reverses time
      y[(size_t)k * m + i] = out_b;
      if (DOT) acc += out_f * zb0 + out_b * zk;
    }
    Lf2 = Lf1; zf1 = zk; Lf1 = Lk;
    zb0 = zb1; Lb0 = Lb1; zb1 = zb2; Lb1 = Lb2;
  }
  return acc;
}

// The blocks of one right-hand side (grid-stride, XCD-aware order).
template <bool RES, bool DOT>
__device__ __forceinline__ double stencil_run(const DevPlan& P, const double* __restrict__ x, double* __restrict__ y,
                                              const double* __restrict__ f) {
  const int tiles = (P.m + kStencilThreads - 1) / kStencilThreads;
  const int nblk = stencil_blocks(P);
  double acc = 0.0;
  for (int w = blockIdx.x; w < nblk; w += gridDim.x) {
    const int lb = xcd_remap(w, nblk);
    acc += stencil_tile<RES, DOT>(P, x, y, f, lb % tiles, lb / tiles);
  }
  return acc;
}

__global__ void __launch_bounds__(kStencilThreads)
k_stencil(DevPlan P, int mode, const double* __restrict__ xin, double* __restrict__ yout,
          const double* __restrict__ fref, int nparts_rnorm) {
  const int b = blockIdx.y;
  MinresState* st = P.st + b;
  const double* x = xin;
  double* y = yout;
  int part_kind = PART_RES;
  if (mode == STENCIL_MINRES) {
    if (st->state != ST_RUNNING) return;
    const int j = st->iter + 1;
    x = P.Z[j & 1];
    y = P.V[(j + 1) % 3];
    part_kind = PART_DELTA;
  } else if (mode == STENCIL_RESIDUAL) {
    // stopping test on the recurrence residual of the update kernel (same fixed-order
    // sum in every block); confirm explicitly when it passes
    if (st->state != ST_RUNNING) return;
    const double rn2 = sum_parts(part_slot(P, PART_RNORM, b), nparts_rnorm);
    __shared__ int need_sh;
    if (threadIdx.x == 0) {
      const int need = (rn2 <= st->tol2 * st->bnorm2) || st->explicit_mode || st->iter >= st->maxit || st->lucky ||
                       !(rn2 == rn2);
      need_sh = need;
      if (blockIdx.x == 0) {
        st->rnorm2 = rn2;
        st->need_check = need;
      }
    }
    __syncthreads();
    if (!need_sh) return;
  }
  x += (size_t)b * P.N;
  if (y) y += (size_t)b * P.N;
  const double* f = fref ? fref + (size_t)b * P.N : nullptr;
  double acc;
  if (mode == STENCIL_PLAIN) {
    stencil_run<false, false>(P, x, y, f);
    return;
  } else if (mode == STENCIL_MINRES) {
    acc = stencil_run<false, true>(P, x, y, f);
  } else {
    acc = stencil_run<true, false>(P, x, y, f);
  }
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, part_kind, b)[blockIdx.x] = bs;
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

// Set-up of a solve: b = Y f into R and V_1, zero V_0, W_0, W_1 and u; ||b||^2 partials.
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
    P.R[off + e] = v;
    P.V[1][off + e] = v;
    P.V[0][off + e] = 0.0;
    P.W[0][off + e] = 0.0;
    P.W[1][off + e] = 0.0;
    u[off + e] = 0.0;
    acc += v * v;
  }
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_RNORM, b)[blockIdx.x] = bs;
}

// w_j = wa Z_j - wb w_{j-1} - wc w_{j-2};  x += xc w_j;  r = r1 r + r2 V_{j+1};  ||r||^2
__global__ void __launch_bounds__(kVecThreads)
k_update(DevPlan P, double* __restrict__ u) {
  const int b = blockIdx.y;
  const MinresState* st = P.st + b;
  if (st->state != ST_RUNNING) return;
  const int j = st->iter;
  const double wa = st->wa, wb = st->wb, wc = st->wc, xc = st->xc, r1 = st->r1, r2 = st->r2;
  const size_t off = (size_t)b * P.N;
  const double* __restrict__ Zj = P.Z[j & 1] + off;
  const double* __restrict__ Wm1 = P.W[(j - 1) & 1] + off;
  double* __restrict__ Wm2 = P.W[j & 1] + off;
  const double* __restrict__ Vn = P.V[(j + 1) % 3] + off;
  double* __restrict__ R = P.R + off;
  double* __restrict__ X = u + off;
  const int nblk = gridDim.x;
  const size_t per = ((size_t)P.N + nblk - 1) / nblk;
  const size_t lo = (size_t)blockIdx.x * per;
  const size_t hi = lo + per < (size_t)P.N ? lo + per : (size_t)P.N;
  double acc = 0.0;
  for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    const double w = wa * Zj[e] - wb * Wm1[e] - wc * Wm2[e];
    Wm2[e] = w;
    X[e] += xc * w;
    const double r = r1 * R[e] + r2 * Vn[e];
    R[e] = r;
    acc += r * r;
  }
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_RNORM, b)[blockIdx.x] = bs;
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
    double* __restrict__ z = P.Z[1] + off;
    for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
      const double v = q[e];
      z[e] = v;
      acc += v * v;
    }
  } else {
    const int j = st->iter + 1;
    double* __restrict__ q = P.V[(j + 1) % 3] + off;
    const double* __restrict__ vj = P.V[j % 3] + off;
    const double* __restrict__ vjm1 = P.V[(j + 2) % 3] + off;
    double* __restrict__ z = P.Z[(j + 1) & 1] + off;
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

// Lanczos coefficient gamma_{j+1} and the Givens QR update of iteration j.
__device__ void step_gamma_iter(MinresState* st, double g2) {
  if (!(g2 >= 0.0) || !(g2 < 1e300)) {
    st->state = ST_DONE;
    st->status = -5;  // ABAC_EBREAKDOWN
    st->iter += 1;
    return;
  }
  const double gn = sqrt(g2);
  const double gam = st->gamma, del = st->delta;
  const double eps = st->s2 * gam;
  const double dbar = st->c2 * gam;
  const double dp = st->c1 * dbar + st->s1 * del;
  const double t2 = -st->s1 * dbar + st->c1 * del;
  const double rho = hypot(t2, gn);
  if (!(rho > 0.0) || !(rho < 1e300)) {
    st->state = ST_DONE;
    st->status = -5;
    st->iter += 1;
    return;
  }
  const double c = t2 / rho, s = gn / rho;
  st->wa = st->sig / rho;
  st->wb = dp / rho;
  st->wc = eps / rho;
  st->xc = c * st->eta;
  st->r1 = s * s;
  st->r2 = gn > 0.0 ? -s * c * st->eta / gn : 0.0;
  st->eta = -s * st->eta;
  st->c2 = st->c1; st->c1 = c;
  st->s2 = st->s1; st->s1 = s;
  st->sig_prev = st->sig;
  st->sig = gn > 0.0 ? 1.0 / gn : 0.0;
  st->gamma = gn;
  st->iter += 1;
  if (gn == 0.0) st->lucky = 1;
}

// Copy the state of right-hand side b into the next slot of the host-mapped ring
// (zero-copy: the host reads it after an event recorded behind this kernel).
__device__ __forceinline__ void post_snapshot(const DevPlan& P, int b) {
  MinresState* st = P.st + b;
  const int seq = st->snap;
  if (P.host_ring) P.host_ring[(size_t)(seq % kSnapRing) * P.B + b] = *st;
  st->snap = seq + 1;
}

constexpr int kFinThreads = 1024;

__global__ void __launch_bounds__(kFinThreads)
k_fin(DevPlan P, int kind, int nparts, double tol, int maxit) {
  const int b = blockIdx.x;
  MinresState* st = P.st + b;
  const bool posts = kind == FIN_GAMMA_INIT || kind == FIN_RES;   // end of set-up / of an iteration
  if ((kind != FIN_BNORM && kind != FIN_REPORT && st->state != ST_RUNNING) || (kind == FIN_RES && !st->need_check)) {
    if (posts && threadIdx.x == 0) post_snapshot(P, b);
    return;
  }
  int pk = PART_RES;
  switch (kind) {
    case FIN_BNORM: pk = PART_RNORM; break;
    case FIN_DELTA: pk = PART_DELTA; break;
    case FIN_GAMMA_INIT:
    case FIN_GAMMA_ITER: pk = PART_GAMMA; break;
    default: pk = PART_RES; break;
  }
  const double tot = sum_parts(part_slot(P, pk, b), nparts);
  if (threadIdx.x != 0) return;
  switch (kind) {
    case FIN_BNORM:
      st->bnorm2 = tot;
      st->tol2 = tol * tol;
      st->maxit = maxit;
      st->iter = 0;
      st->explicit_mode = 0;
      st->need_check = 0;
      st->lucky = 0;
      st->snap = 0;
      st->rnorm2 = tot;
      st->res2 = tot;
      st->status = 0;
      if (tot == 0.0) {
        st->state = ST_DONE;   // u = 0 is exact
      } else if (!(tot == tot) || tot > 1e300) {
        st->state = ST_DONE;
        st->status = -5;
      } else {
        st->state = ST_RUNNING;
      }
      break;
    case FIN_DELTA:
      st->delta = tot * st->sig * st->sig;
      break;
    case FIN_GAMMA_INIT:
      if (!(tot > 0.0) || !(tot < 1e300)) {
        st->state = ST_DONE;
        st->status = -5;
        break;
      }
      st->gamma = sqrt(tot);
      st->sig = 1.0 / st->gamma;
      st->sig_prev = 0.0;
      st->eta = st->gamma;
      st->c1 = 1.0; st->c2 = 1.0;
      st->s1 = 0.0; st->s2 = 0.0;
      st->iter = 0;
      break;
    case FIN_GAMMA_ITER:
      step_gamma_iter(st, tot);
      break;
    case FIN_RES:
      st->res2 = tot;
      if (tot <= st->tol2 * st->bnorm2) {
        st->state = ST_DONE;
        st->status = 0;
      } else if (!(tot == tot) || tot > 1e300) {
        st->state = ST_DONE;
        st->status = -5;
      } else if (st->iter >= st->maxit) {
        st->state = ST_DONE;
        st->status = -4;  // ABAC_ENOTCONV
      } else {
        st->explicit_mode = 1;
      }
      st->need_check = 0;
      break;
    case FIN_REPORT:
      st->res2 = tot;
      break;
  }
  if (posts) post_snapshot(P, b);
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
  hipLaunchKernelGGL(k_stencil, grid, dim3(kStencilThreads), 0, s, P, mode, x, y, f, update_blocks(P));
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

hipError_t launch_identity(const DevPlan& P, int mode, const double* in, double* out, hipStream_t s) {
  dim3 grid(update_blocks(P), P.B);
  hipLaunchKernelGGL(k_identity, grid, dim3(kVecThreads), 0, s, P, mode, in, out);
  return hipGetLastError();
}

hipError_t launch_fin(const DevPlan& P, int kind, double tol, int maxit, hipStream_t s) {
  int nparts;
  switch (kind) {
    case FIN_BNORM: nparts = update_blocks(P); break;
    case FIN_DELTA: nparts = stencil_grid(P, STENCIL_MINRES); break;
    case FIN_GAMMA_INIT:
    case FIN_GAMMA_ITER: nparts = P.gamma_nparts; break;
    default: nparts = stencil_grid(P, STENCIL_RESIDUAL); break;
  }
  hipLaunchKernelGGL(k_fin, dim3(P.B), dim3(kFinThreads), 0, s, P, kind, nparts, tol, maxit);
  return hipGetLastError();
}

}  // namespace abac

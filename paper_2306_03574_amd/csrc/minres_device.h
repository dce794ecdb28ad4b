// Device code of the MINRES steps (Section 3's solver; Paige-Saunders recurrences in
// the P^{-1} inner product): the residual / w / x update, forming the iterate from the
// resident Krylov basis, and the per-right-hand-side scalar steps (sums of partials,
// Givens QR, stopping test, snapshots).  Shared by the separate kernels and the fused
// small-problem iteration.
#pragma once
#include "abac_internal.h"

namespace abac {
namespace {

// Residual recurrence r = r1 r + r2 V_{j+1} and ||r||^2 partials; after the resident
// basis (j > kBasis) also w_j = wa Z_j - wb w_{j-1} - wc w_{j-2} and x += xc w_j.
// Elements [part N/nparts, (part+1) N/nparts) of right-hand side b; returns this
// thread's part of ||r||^2.  The caller skips stopped right-hand sides.
__device__ __forceinline__ double update_part(const DevPlan& P, int b, double* __restrict__ u, int part,
                                              int nparts) {
  const MinresState* st = P.st + b;
  const int j = st->iter;
  const double wa = st->wa, wb = st->wb, wc = st->wc, xc = st->xc, r1 = st->r1, r2 = st->r2;
  const size_t off = (size_t)b * P.N;
  const double* __restrict__ Vn = P.V[(j + 1) % 3] + off;
  double* __restrict__ R = P.R + off;
  const double* __restrict__ Rin = j == 1 ? P.V[1] + off : R;   // r_0 = v_1
  const size_t per = ((size_t)P.N + nparts - 1) / nparts;
  const size_t lo = (size_t)part * per;
  const size_t hi = lo + per < (size_t)P.N ? lo + per : (size_t)P.N;
  double acc = 0.0;
  if (j <= kBasis) {
    for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
      const double r = r1 * Rin[e] + r2 * Vn[e];
      R[e] = r;
      acc += r * r;
    }
  } else {
    const double* __restrict__ Zj = P.Z[zslot(j)] + off;
    const double* __restrict__ Wm1 = P.W[(j - 1) & 1] + off;
    double* __restrict__ Wm2 = P.W[j & 1] + off;
    double* __restrict__ X = u + off;
    for (size_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
      const double w = wa * Zj[e] - wb * Wm1[e] - wc * Wm2[e];
      Wm2[e] = w;
      X[e] += xc * w;
      const double r = r1 * R[e] + r2 * Vn[e];
      R[e] = r;
      acc += r * r;
    }
  }
  return acc;
}

// u = sum_l xm_l Z_l over the first NB basis slots; with FLUSH also
// W[kBasis & 1] = w_kBasis and W[(kBasis+1) & 1] = w_{kBasis-1} from their coefficients.
template <int NB, bool FLUSH>
__device__ __forceinline__ void form_from_basis(const DevPlan& P, int b, double* __restrict__ u, int part,
                                                int nparts) {
  const size_t off = (size_t)b * P.N;
  const double* kc = P.kcoef + (size_t)b * 3 * kBasis;
  double cx[NB], c1[NB], c2[NB];
  const double* zs[NB];
#pragma unroll
  for (int l = 0; l < NB; ++l) {
    cx[l] = kc[l];
    c1[l] = FLUSH ? kc[kBasis + l] : 0.0;
    c2[l] = FLUSH ? kc[2 * kBasis + l] : 0.0;
    zs[l] = P.Z[l] + off;
  }
  double* X = u + off;
  double* W1 = P.W[kBasis & 1] + off;
  double* W2 = P.W[(kBasis + 1) & 1] + off;
  const size_t per = ((size_t)P.N + nparts - 1) / nparts;
  const size_t lo = (size_t)part * per;
  const size_t hi = lo + per < (size_t)P.N ? lo + per : (size_t)P.N;
  // two elements per trip (the second clamped into range), so 2 NB loads are in flight
  for (size_t e0 = lo + threadIdx.x; e0 < hi; e0 += 2 * (size_t)blockDim.x) {
    const size_t e1 = e0 + blockDim.x;
    const size_t e1c = e1 < hi ? e1 : e0;
    double z0[NB], z1[NB];
#pragma unroll
    for (int l = 0; l < NB; ++l) {
      z0[l] = zs[l][e0];
      z1[l] = zs[l][e1c];
    }
    double ax0 = 0.0, a10 = 0.0, a20 = 0.0, ax1 = 0.0, a11 = 0.0, a21 = 0.0;
#pragma unroll
    for (int l = 0; l < NB; ++l) {
      ax0 += cx[l] * z0[l];
      ax1 += cx[l] * z1[l];
      if (FLUSH) {
        a10 += c1[l] * z0[l];
        a20 += c2[l] * z0[l];
        a11 += c1[l] * z1[l];
        a21 += c2[l] * z1[l];
      }
    }
    X[e0] = ax0;
    if (FLUSH) {
      W1[e0] = a10;
      W2[e0] = a20;
    }
    if (e1 < hi) {
      X[e1] = ax1;
      if (FLUSH) {
        W1[e1] = a11;
        W2[e1] = a21;
      }
    }
  }
}

template <bool FLUSH>
__device__ __forceinline__ void form_dispatch(const DevPlan& P, int b, int nb, double* u, int part, int nparts) {
  switch (nb) {
#define ABAC_FORM_CASE(K) \
    case K: form_from_basis<K, FLUSH>(P, b, u, part, nparts); break;
    ABAC_FORM_CASE(1) ABAC_FORM_CASE(2) ABAC_FORM_CASE(3) ABAC_FORM_CASE(4) ABAC_FORM_CASE(5) ABAC_FORM_CASE(6)
    ABAC_FORM_CASE(7) ABAC_FORM_CASE(8) ABAC_FORM_CASE(9) ABAC_FORM_CASE(10) ABAC_FORM_CASE(11) ABAC_FORM_CASE(12)
#undef ABAC_FORM_CASE
    default: break;
  }
}
static_assert(kBasis == 12, "form_dispatch lists one case per basis size");

// Lanczos coefficient gamma_{j+1} and the Givens QR update of iteration j.  In the
// basis phase the w and x recurrences run on coefficient vectors over the basis
// slots (kc: x, w_j, w_{j-1}), the same arithmetic the classic phase does on vectors.
__device__ void step_gamma_iter(MinresState* st, double* kc, double g2) {
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
  const int j = st->iter;
  if (j <= kBasis) {
    double* xm = kc;
    double* m1 = kc + kBasis;
    double* m2 = kc + 2 * kBasis;
    for (int l = 0; l < j; ++l) {
      const double w = (l == j - 1 ? st->wa : 0.0) - st->wb * m1[l] - st->wc * m2[l];
      m2[l] = m1[l];
      m1[l] = w;
      xm[l] += st->xc * w;
    }
    st->nbasis = j;
    st->basis_dirty = 1;
  }
}

// Copy the state of right-hand side b into the next slot of the host-mapped ring
// (zero-copy: the host reads it after an event recorded behind this kernel).
__device__ __forceinline__ void post_snapshot(const DevPlan& P, int b) {
  MinresState* st = P.st + b;
  const int seq = st->snap;
  if (P.host_ring) P.host_ring[(size_t)(seq % kSnapRing) * P.B + b] = *st;
  st->snap = seq + 1;
}

// First half of a scalar step of right-hand side b: the flag updates of the step kind
// (by thread 0 of the calling workgroup) and whether the step folds a sum into the
// state.  A skipped step that ends an iteration still posts the snapshot.  Every
// thread returns the same answer.
__device__ __forceinline__ bool fin_begin(const DevPlan& P, int b, int kind) {
  MinresState* st = P.st + b;
  const bool posts = kind == FIN_GAMMA_INIT || kind == FIN_RES;   // end of set-up / of an iteration
  if ((kind == FIN_RES || kind == FIN_REPORT) && threadIdx.x == 0 && st->form_now) {
    st->basis_dirty = 0;   // the form step wrote the iterate into u
    st->form_now = 0;
    st->flush_now = 0;
  }
  if (kind == FIN_FINAL || (kind == FIN_RNORM && st->state != ST_RUNNING)) {
    // a stopped solve (breakdown in this iteration, or the end of the solve) with a
    // stale u forms it from the basis
    if (threadIdx.x == 0) {
      st->form_now = st->basis_dirty;
      st->flush_now = 0;
    }
    return false;
  }
  if ((kind != FIN_BNORM && kind != FIN_REPORT && st->state != ST_RUNNING) || (kind == FIN_RES && !st->need_check)) {
    if (posts && threadIdx.x == 0) post_snapshot(P, b);
    return false;
  }
  return true;
}

// Which partial sums a scalar step folds in.
__device__ __forceinline__ int fin_part_kind(int kind) {
  switch (kind) {
    case FIN_BNORM: return PART_RNORM;
    case FIN_DELTA: return PART_DELTA;
    case FIN_GAMMA_INIT:
    case FIN_GAMMA_ITER: return PART_GAMMA;
    case FIN_RNORM: return PART_RNORM;
    default: return PART_RES;
  }
}

// Second half, thread 0 only: fold the sum `tot` into the state of right-hand side b
// (Givens QR, stopping test, ...) and post the snapshot at the end of an iteration.
__device__ void fin_scalar(const DevPlan& P, int b, int kind, double tot, double tol, int maxit) {
  MinresState* st = P.st + b;
  const bool posts = kind == FIN_GAMMA_INIT || kind == FIN_RES;
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
      st->nbasis = 0;
      st->basis_dirty = 0;   // u = 0 = x_0
      st->form_now = 0;
      st->flush_now = 0;
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
      for (int l = 0; l < 3 * kBasis; ++l) P.kcoef[(size_t)b * 3 * kBasis + l] = 0.0;
      break;
    case FIN_GAMMA_ITER:
      step_gamma_iter(st, P.kcoef + (size_t)b * 3 * kBasis, tot);
      break;
    case FIN_RNORM: {
      // stopping test on the recurrence residual; the explicit residual confirms it
      const int j = st->iter;
      const int need = (tot <= st->tol2 * st->bnorm2) || st->explicit_mode || j >= st->maxit || st->lucky ||
                       !(tot == tot);
      st->rnorm2 = tot;
      st->need_check = need;
      st->form_now = j <= kBasis && (need || j == kBasis);
      st->flush_now = j == kBasis;
      break;
    }
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
}  // namespace abac

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

// what a matvec block writes: Y T x (time-reversed, the symmetrised operator), T x,
// the residual vector f - T x, or only the squared residual norm
enum StencilOut : int { OUT_REV = 0, OUT_NAT = 1, OUT_RESVEC = 2, OUT_RESNORM = 3 };

// One logical block of the matvec: a band of RB grid rows times st_threads consecutive
// columns, forward levels [k0, k1) and their mirrors nt-1-k.  Each thread marches one
// column of the band.  Per level it loads the RB+2 rows of its column (the band and the
// two rows around it, clamped into the grid: a missing neighbour reads the centre with
// weight 0, as in l_coef), so the y-neighbours of every row come from registers, and the
// two x-neighbours of each row (L1 hits).  L of the two previous levels stays in
// registers.  Every load is unconditional, so a step's loads are all in flight together.
// VAR: variable coefficient, face weights per row; otherwise the x weights depend on the
// column only and the y weights on the (block-uniform) row only.
template <int RB, bool VAR>
struct Band {
  int rowoff[RB + 2];   // offsets of rows iy0-1 .. iy0+RB (clamped) at this column
  int ow, oe;           // x-neighbour offsets of this column
  double c[VAR ? RB : 1], w[VAR ? RB : 1], e[VAR ? RB : 1], so[VAR ? RB : 1], no[VAR ? RB : 1];
  double cw, ce;        // constant coefficient: x weights of this column
};

template <int RB, bool VAR>
__device__ __forceinline__ void band_level(const DevPlan& P, const Band<RB, VAR>& Bd, int iy0,
                                           const double* __restrict__ lvl, double* L, double* z) {
  double c[RB + 2], w[RB], e[RB];
#pragma unroll
  for (int r = 0; r < RB + 2; ++r) c[r] = lvl[Bd.rowoff[r]];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    w[r] = lvl[Bd.rowoff[r + 1] + Bd.ow];
    e[r] = lvl[Bd.rowoff[r + 1] + Bd.oe];
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if constexpr (VAR) {
      L[r] = Bd.c[r] * c[r + 1] - (Bd.w[r] * w[r] + Bd.e[r] * e[r]) - (Bd.so[r] * c[r] + Bd.no[r] * c[r + 2]);
    } else {
      const int iy = iy0 + r;
      const double so = P.ny && iy > 0 ? P.cy : 0.0;
      const double no = P.ny && iy < P.ny - 1 ? P.cy : 0.0;
      L[r] = P.c0 * c[r + 1] - (Bd.cw * w[r] + Bd.ce * e[r]) - (so * c[r] + no * c[r + 2]);
    }
    z[r] = c[r + 1];
  }
}

template <int RB, bool VAR, int OUT, bool DOT>
__device__ __forceinline__ double stencil_tile(const DevPlan& P, const double* __restrict__ x,
                                               double* __restrict__ y, const double* __restrict__ f, int band,
                                               int xt, int chunk) {
  const int n = P.nt, m = P.m, nx = P.nx, ny1 = P.ny1;
  const int ix_raw = xt * P.st_threads + threadIdx.x;
  const bool active = ix_raw < nx;
  const int ix = min(ix_raw, nx - 1);   // inactive lanes repeat the last column and store nothing
  const int iy0 = band * RB;
  Band<RB, VAR> Bd;
#pragma unroll
  for (int r = 0; r < RB + 2; ++r) Bd.rowoff[r] = min(max(iy0 - 1 + r, 0), ny1 - 1) * nx + ix;
  Bd.ow = ix > 0 ? -1 : 0;
  Bd.oe = ix < nx - 1 ? 1 : 0;
  if constexpr (VAR) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const LCoef q = l_coef(P, ix, min(iy0 + r, ny1 - 1));
      Bd.c[r] = q.c; Bd.w[r] = q.w; Bd.e[r] = q.e; Bd.so[r] = q.so; Bd.no[r] = q.no;
    }
  } else {
    Bd.cw = ix > 0 ? P.cx : 0.0;
    Bd.ce = ix < nx - 1 ? P.cx : 0.0;
  }
  const int k0 = chunk * P.st_chunk;
  const int k1 = min(k0 + P.st_chunk, n / 2);
  double acc = 0.0;
  double Lf2[RB], zf1[RB], Lf1[RB], zb0[RB], Lb0[RB], zb1[RB], Lb1[RB], tL[RB], tz[RB];
  {
    // forward state before level k0 (zero before level 0: the clamped level's values
    // are selected away); backward state at kb = n-1-k0 and kb-1
    const int a2 = max(k0 - 2, 0), a1 = max(k0 - 1, 0);
    band_level<RB, VAR>(P, Bd, iy0, x + (size_t)a2 * m, tL, tz);
#pragma unroll
    for (int r = 0; r < RB; ++r) Lf2[r] = k0 >= 2 ? tL[r] : 0.0;
    band_level<RB, VAR>(P, Bd, iy0, x + (size_t)a1 * m, tL, tz);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      Lf1[r] = k0 >= 1 ? tL[r] : 0.0;
      zf1[r] = k0 >= 1 ? tz[r] : 0.0;
    }
    const int kb0 = n - 1 - k0;
    band_level<RB, VAR>(P, Bd, iy0, x + (size_t)kb0 * m, Lb0, zb0);
    band_level<RB, VAR>(P, Bd, iy0, x + (size_t)(kb0 - 1) * m, Lb1, zb1);
  }
  for (int k = k0; k < k1; ++k) {
    double Lk[RB], zk[RB], Lb2[RB], zb2[RB];
    band_level<RB, VAR>(P, Bd, iy0, x + (size_t)k * m, Lk, zk);               // forward level k
    band_level<RB, VAR>(P, Bd, iy0, x + (size_t)(n - 3 - k) * m, Lb2, zb2);   // backward level kb - 2
    double* yf = y + (size_t)k * m;
    double* yb = y + (size_t)(n - 1 - k) * m;
    const double* ff = f + (size_t)k * m;
    const double* fb = f + (size_t)(n - 1 - k) * m;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const double out_f = Lk[r] + Lf2[r] - 2.0 * zf1[r];     // (T x)_k
      const double out_b = Lb0[r] + Lb2[r] - 2.0 * zb1[r];    // (T x)_kb, kb = n-1-k
      const int pos = Bd.rowoff[r + 1];
      if (active && iy0 + r < ny1) {
        if (OUT == OUT_RESNORM || OUT == OUT_RESVEC) {
          const double rf = ff[pos] - out_f;
          const double rb = fb[pos] - out_b;
          acc += rf * rf + rb * rb;
          if (OUT == OUT_RESVEC) {
            yf[pos] = rf;
            yb[pos] = rb;
          }
        } else if (OUT == OUT_NAT) {
          yf[pos] = out_f;
          yb[pos] = out_b;
        } else {
          yb[pos] = out_f;   // Y reverses time
          yf[pos] = out_b;
          if (DOT) acc += out_f * zb0[r] + out_b * zk[r];
        }
      }
      Lf2[r] = Lf1[r]; zf1[r] = zk[r]; Lf1[r] = Lk[r];
      zb0[r] = zb1[r]; Lb0[r] = Lb1[r]; zb1[r] = zb2[r]; Lb1[r] = Lb2[r];
    }
  }
  return acc;
}

// The blocks of one right-hand side (grid-stride, XCD-aware order: consecutive logical
// blocks are neighbouring column tiles and bands of the same levels).
template <int RB, bool VAR, int OUT, bool DOT>
__device__ __forceinline__ double stencil_run_rb(const DevPlan& P, const double* __restrict__ x,
                                                 double* __restrict__ y, const double* __restrict__ f) {
  const int xtiles = (P.nx + P.st_threads - 1) / P.st_threads;
  const int tiles = ((P.ny1 + RB - 1) / RB) * xtiles;
  const int nblk = stencil_blocks(P);
  double acc = 0.0;
  for (int w = blockIdx.x; w < nblk; w += gridDim.x) {
    const int lb = xcd_remap(w, nblk);
    const int tile = lb % tiles;
    acc += stencil_tile<RB, VAR, OUT, DOT>(P, x, y, f, tile / xtiles, tile % xtiles, lb / tiles);
  }
  return acc;
}

template <bool VAR, int OUT, bool DOT>
__device__ __forceinline__ double stencil_run(const DevPlan& P, const double* __restrict__ x, double* __restrict__ y,
                                              const double* __restrict__ f) {
  return P.ny ? stencil_run_rb<kStencilRows, VAR, OUT, DOT>(P, x, y, f) : stencil_run_rb<1, VAR, OUT, DOT>(P, x, y, f);
}

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
    stencil_run<VAR, OUT_REV, false>(P, x, y, f);
    return;
  }
  if (MODE == STENCIL_T) {
    stencil_run<VAR, OUT_NAT, false>(P, x, y, f);
    return;
  }
  double acc;
  if (MODE == STENCIL_MINRES)
    acc = stencil_run<VAR, OUT_REV, true>(P, x, y, f);
  else if (MODE == STENCIL_RESVEC)
    acc = stencil_run<VAR, OUT_RESVEC, false>(P, x, y, f);
  else
    acc = stencil_run<VAR, OUT_RESNORM, false>(P, x, y, f);
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
  const MinresState* st = P.st + b;
  if (st->state != ST_RUNNING) return;
  const int j = st->iter;
  const double wa = st->wa, wb = st->wb, wc = st->wc, xc = st->xc, r1 = st->r1, r2 = st->r2;
  const size_t off = (size_t)b * P.N;
  const double* __restrict__ Vn = P.V[(j + 1) % 3] + off;
  double* __restrict__ R = P.R + off;
  const double* __restrict__ Rin = j == 1 ? P.V[1] + off : R;   // r_0 = v_1
  const int nblk = gridDim.x;
  const size_t per = ((size_t)P.N + nblk - 1) / nblk;
  const size_t lo = (size_t)blockIdx.x * per;
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
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_RNORM, b)[blockIdx.x] = bs;
}

// u = sum_l xm_l Z_l over the first NB basis slots; with FLUSH also
// W[kBasis & 1] = w_kBasis and W[(kBasis+1) & 1] = w_{kBasis-1} from their coefficients.
template <int NB, bool FLUSH>
__device__ __forceinline__ void form_from_basis(const DevPlan& P, int b, double* __restrict__ u) {
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
  const int nblk = gridDim.x;
  const size_t per = ((size_t)P.N + nblk - 1) / nblk;
  const size_t lo = (size_t)blockIdx.x * per;
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
__device__ __forceinline__ void form_dispatch(const DevPlan& P, int b, int nb, double* u) {
  switch (nb) {
#define ABAC_FORM_CASE(K) \
    case K: form_from_basis<K, FLUSH>(P, b, u); break;
    ABAC_FORM_CASE(1) ABAC_FORM_CASE(2) ABAC_FORM_CASE(3) ABAC_FORM_CASE(4) ABAC_FORM_CASE(5) ABAC_FORM_CASE(6)
    ABAC_FORM_CASE(7) ABAC_FORM_CASE(8) ABAC_FORM_CASE(9) ABAC_FORM_CASE(10) ABAC_FORM_CASE(11) ABAC_FORM_CASE(12)
#undef ABAC_FORM_CASE
    default: break;
  }
}
static_assert(kBasis == 12, "form_dispatch lists one case per basis size");

// Forms u (and at the flush w_j, w_{j-1}) from the resident basis for the right-hand
// sides whose scalar step (FIN_RNORM or FIN_FINAL) set form_now; the others return at
// once.  Writes no solve state.
__global__ void __launch_bounds__(kVecThreads)
k_form(DevPlan P, double* __restrict__ u) {
  const int b = blockIdx.y;
  const MinresState* st = P.st + b;
  if (!st->form_now) return;
  const int nb = st->nbasis;
  if (st->flush_now) form_dispatch<true>(P, b, nb, u);
  else form_dispatch<false>(P, b, nb, u);
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

constexpr int kFinThreads = 1024;

__global__ void __launch_bounds__(kFinThreads)
k_fin(DevPlan P, int kind, int nparts, double tol, int maxit) {
  const int b = blockIdx.x;
  MinresState* st = P.st + b;
  const bool posts = kind == FIN_GAMMA_INIT || kind == FIN_RES;   // end of set-up / of an iteration
  if ((kind == FIN_RES || kind == FIN_REPORT) && threadIdx.x == 0 && st->form_now) {
    st->basis_dirty = 0;   // the form kernel wrote the iterate into u
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
    return;
  }
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
    case FIN_RNORM: pk = PART_RNORM; break;
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

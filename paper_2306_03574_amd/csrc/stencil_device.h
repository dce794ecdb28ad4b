// Device code of the Y T matvec (eqs. (1.2), (1.4)): the weights of L at a grid
// point (constant or variable coefficient) and the band-marching stencil tile.  Shared
// by the matvec kernels and the fused small-problem iteration.
#pragma once
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
                                               int xt, int chunk, int tx) {
  const int n = P.nt, m = P.m, nx = P.nx, ny1 = P.ny1;
  const int ix_raw = xt * P.st_threads + tx;
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

// Logical blocks first, first + stride, ... of one right-hand side, lane tx of each
// (the kernels: one logical block per workgroup, grid-stride, in XCD-aware order so that
// consecutive logical blocks, neighbouring column tiles and bands of the same levels,
// share an L2; the fused small-problem iteration: several logical blocks side by side
// in one workgroup, in natural order).
template <int RB, bool VAR, int OUT, bool DOT>
__device__ __forceinline__ double stencil_run_rb(const DevPlan& P, const double* __restrict__ x,
                                                 double* __restrict__ y, const double* __restrict__ f, int first,
                                                 int stride, int tx, bool remap) {
  const int xtiles = (P.nx + P.st_threads - 1) / P.st_threads;
  const int tiles = ((P.ny1 + RB - 1) / RB) * xtiles;
  const int nblk = stencil_blocks(P);
  double acc = 0.0;
  for (int w = first; w < nblk; w += stride) {
    const int lb = remap ? xcd_remap(w, nblk) : w;
    const int tile = lb % tiles;
    acc += stencil_tile<RB, VAR, OUT, DOT>(P, x, y, f, tile / xtiles, tile % xtiles, lb / tiles, tx);
  }
  return acc;
}

template <bool VAR, int OUT, bool DOT>
__device__ __forceinline__ double stencil_run(const DevPlan& P, const double* __restrict__ x, double* __restrict__ y,
                                              const double* __restrict__ f, int first, int stride, int tx,
                                              bool remap) {
  return P.ny ? stencil_run_rb<kStencilRows, VAR, OUT, DOT>(P, x, y, f, first, stride, tx, remap)
              : stencil_run_rb<1, VAR, OUT, DOT>(P, x, y, f, first, stride, tx, remap);
}

}  // namespace
}  // namespace abac

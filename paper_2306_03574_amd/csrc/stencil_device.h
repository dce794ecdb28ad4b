// Device code of the Y T matvec (eqs. (1.2), (1.4)): the weights of L at a grid
// point (constant or variable coefficient) and the band-marching stencil tiles (two
// columns per thread for the constant coefficient, one for the variable one).  Shared
// by the matvec kernels, the fused small-problem iteration and the group kernels.
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

// One column of a logical block of the matvec, one column per thread (the
// variable-coefficient tile, and grids one column wide): a band of RB grid rows, forward
// levels [k0, k1) and their mirrors nt-1-k.  Per level it loads the RB+2 rows of its
// column (the band and the two rows around it, clamped into the grid: a missing
// neighbour reads the centre with weight 0, as in l_coef), so the y-neighbours of every
// row come from registers, and the two x-neighbours of each row (L1 hits).  L of the two
// previous levels stays in registers.  Every load is unconditional, so a step's loads
// are all in flight together.
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
                                               int ix_raw, int chunk) {
  const int n = P.nt, m = P.m, nx = P.nx, ny1 = P.ny1;
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

// ---------------------------------------------------------------------------
// Two adjacent columns per thread (constant coefficient).  The band march of
// stencil_tile, with each thread owning columns c and c+1 (c even).  Per level and band
// row it issues two 16-byte loads, the pairs (c-1, c) and (c+1, c+2), which hold the
// row's two centre values and both x-neighbours; the RB+2 halo rows need only the pair
// (c, c+1).  That is RB*2 + 2 vector loads for 2*RB points, against 3*RB + 2 for RB
// points with one column per thread: the matvec issues about a third of the vector
// memory instructions per point.  Pair starts are clamped into [0, nx-2] so that every
// load stays inside its row; a clamped pair only ever stands in for a value whose weight
// is zero or for a column that is not written.  The per-point arithmetic is that of
// stencil_tile, term for term.
// centre values (columns c, c+1) of the RB+2 rows and the outer neighbours (c-1, c+2)
// of the RB band rows at one level
template <int RB>
struct Lvl2 {
  double c0[RB + 2], c1[RB + 2], w[RB], e[RB];
};

template <int RB>
__device__ __forceinline__ void pair_level(const int* rowoff, int sw, int se, int sc, bool c_from_wy, bool c1_from_ex,
                                           bool h_low, const double* __restrict__ lvl, Lvl2<RB>& v) {
  dpair W[RB], E[RB], H[2];
  H[0] = *reinterpret_cast<const dpair*>(lvl + rowoff[0] + sc);
  H[1] = *reinterpret_cast<const dpair*>(lvl + rowoff[RB + 1] + sc);
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    W[r] = *reinterpret_cast<const dpair*>(lvl + rowoff[r + 1] + sw);
    E[r] = *reinterpret_cast<const dpair*>(lvl + rowoff[r + 1] + se);
  }
  v.c0[0] = h_low ? H[0].x : H[0].y;
  v.c1[0] = H[0].y;
  v.c0[RB + 1] = h_low ? H[1].x : H[1].y;
  v.c1[RB + 1] = H[1].y;
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    v.w[r] = W[r].x;
    v.c0[r + 1] = c_from_wy ? W[r].y : W[r].x;
    v.c1[r + 1] = c1_from_ex ? E[r].x : E[r].y;
    v.e[r] = E[r].y;
  }
}

// L of the RB band rows at one level, columns c and c+1 (same expression as band_level)
template <int RB>
__device__ __forceinline__ void pair_L(const DevPlan& P, int iy0, double cw0, double ce0, double ce1, const Lvl2<RB>& v,
                                       double (*L)[2], double (*z)[2]) {
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int iy = iy0 + r;
    const double so = P.ny && iy > 0 ? P.cy : 0.0;
    const double no = P.ny && iy < P.ny - 1 ? P.cy : 0.0;
    L[r][0] = P.c0 * v.c0[r + 1] - (cw0 * v.w[r] + ce0 * v.c1[r + 1]) - (so * v.c0[r] + no * v.c0[r + 2]);
    L[r][1] = P.c0 * v.c1[r + 1] - (P.cx * v.c0[r + 1] + ce1 * v.e[r]) - (so * v.c1[r] + no * v.c1[r + 2]);
    z[r][0] = v.c0[r + 1];
    z[r][1] = v.c1[r + 1];
  }
}

template <int RB, int OUT, bool DOT>
__device__ __forceinline__ double stencil_tile2(const DevPlan& P, const double* __restrict__ x,
                                                double* __restrict__ y, const double* __restrict__ f, int band, int c,
                                                int chunk) {
  const int n = P.nt, m = P.m, nx = P.nx, ny1 = P.ny1;
  const bool act0 = c < nx, act1 = c + 1 < nx;
  const int iy0 = band * RB;
  int rowoff[RB + 2];
#pragma unroll
  for (int r = 0; r < RB + 2; ++r) rowoff[r] = min(max(iy0 - 1 + r, 0), ny1 - 1) * nx;
  // pair starts, clamped into [0, nx-2] (lanes past the row end use the last pair)
  const int sc = min(c, nx - 2);
  const int sw = min(max(c - 1, 0), nx - 2);
  const int se = min(c + 1, nx - 2);
  const bool c_from_wy = c == sw + 1;    // false only at c = 0 (no west neighbour)
  const bool c1_from_ex = c + 1 == se;   // false at the row end (c+1 = nx-1, or c+1 not a column)
  const bool h_low = c == sc;
  const double cw0 = c > 0 ? P.cx : 0.0;
  const double ce0 = c < nx - 1 ? P.cx : 0.0;
  const double ce1 = c + 1 < nx - 1 ? P.cx : 0.0;
  const int k0 = chunk * P.st_chunk;
  const int k1 = min(k0 + P.st_chunk, n / 2);
  double acc = 0.0;
  double Lf2[RB][2], zf1[RB][2], Lf1[RB][2], zb0[RB][2], Lb0[RB][2], zb1[RB][2], Lb1[RB][2], tL[RB][2], tz[RB][2];
  {
    Lvl2<RB> v;
    const int a2 = max(k0 - 2, 0), a1 = max(k0 - 1, 0);
    pair_level<RB>(rowoff, sw, se, sc, c_from_wy, c1_from_ex, h_low, x + (size_t)a2 * m, v);
    pair_L<RB>(P, iy0, cw0, ce0, ce1, v, tL, tz);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q) Lf2[r][q] = k0 >= 2 ? tL[r][q] : 0.0;
    pair_level<RB>(rowoff, sw, se, sc, c_from_wy, c1_from_ex, h_low, x + (size_t)a1 * m, v);
    pair_L<RB>(P, iy0, cw0, ce0, ce1, v, tL, tz);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        Lf1[r][q] = k0 >= 1 ? tL[r][q] : 0.0;
        zf1[r][q] = k0 >= 1 ? tz[r][q] : 0.0;
      }
    const int kb0 = n - 1 - k0;
    pair_level<RB>(rowoff, sw, se, sc, c_from_wy, c1_from_ex, h_low, x + (size_t)kb0 * m, v);
    pair_L<RB>(P, iy0, cw0, ce0, ce1, v, Lb0, zb0);
    pair_level<RB>(rowoff, sw, se, sc, c_from_wy, c1_from_ex, h_low, x + (size_t)(kb0 - 1) * m, v);
    pair_L<RB>(P, iy0, cw0, ce0, ce1, v, Lb1, zb1);
  }
  for (int k = k0; k < k1; ++k) {
    double Lk[RB][2], zk[RB][2], Lb2[RB][2], zb2[RB][2];
    {
      Lvl2<RB> vf, vb;
      pair_level<RB>(rowoff, sw, se, sc, c_from_wy, c1_from_ex, h_low, x + (size_t)k * m, vf);
      pair_level<RB>(rowoff, sw, se, sc, c_from_wy, c1_from_ex, h_low, x + (size_t)(n - 3 - k) * m, vb);
      pair_L<RB>(P, iy0, cw0, ce0, ce1, vf, Lk, zk);
      pair_L<RB>(P, iy0, cw0, ce0, ce1, vb, Lb2, zb2);
    }
    double* yf = y + (size_t)k * m;
    double* yb = y + (size_t)(n - 1 - k) * m;
    const double* ff = f + (size_t)k * m;
    const double* fb = f + (size_t)(n - 1 - k) * m;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      double out_f[2], out_b[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        out_f[q] = Lk[r][q] + Lf2[r][q] - 2.0 * zf1[r][q];     // (T x)_k
        out_b[q] = Lb0[r][q] + Lb2[r][q] - 2.0 * zb1[r][q];    // (T x)_kb, kb = n-1-k
      }
      const int row = rowoff[r + 1];
      if (act0 && iy0 + r < ny1) {
        if (OUT == OUT_RESNORM || OUT == OUT_RESVEC) {
          const dpair pf = *reinterpret_cast<const dpair*>(ff + row + sc);
          const dpair pb = *reinterpret_cast<const dpair*>(fb + row + sc);
          const double rf0 = (h_low ? pf.x : pf.y) - out_f[0];
          const double rb0 = (h_low ? pb.x : pb.y) - out_b[0];
          acc += rf0 * rf0 + rb0 * rb0;
          const double rf1 = pf.y - out_f[1];
          const double rb1 = pb.y - out_b[1];
          if (act1) acc += rf1 * rf1 + rb1 * rb1;
          if (OUT == OUT_RESVEC) {
            if (act1) {
              *reinterpret_cast<dpair*>(yf + row + c) = dpair{rf0, rf1};
              *reinterpret_cast<dpair*>(yb + row + c) = dpair{rb0, rb1};
            } else {
              yf[row + c] = rf0;
              yb[row + c] = rb0;
            }
          }
        } else {
          // Y reverses time: (T x)_k goes to level n-1-k and (T x)_kb to level k
          double* dk = OUT == OUT_NAT ? yf : yb;
          double* dkb = OUT == OUT_NAT ? yb : yf;
          if (act1) {
            *reinterpret_cast<dpair*>(dk + row + c) = dpair{out_f[0], out_f[1]};
            *reinterpret_cast<dpair*>(dkb + row + c) = dpair{out_b[0], out_b[1]};
          } else {
            dk[row + c] = out_f[0];
            dkb[row + c] = out_b[0];
          }
          if (DOT) {
            acc += out_f[0] * zb0[r][0] + out_b[0] * zk[r][0];
            if (act1) acc += out_f[1] * zb0[r][1] + out_b[1] * zk[r][1];
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        Lf2[r][q] = Lf1[r][q]; zf1[r][q] = zk[r][q]; Lf1[r][q] = Lk[r][q];
        zb0[r][q] = zb1[r][q]; Lb0[r][q] = Lb1[r][q]; zb1[r][q] = zb2[r][q]; Lb1[r][q] = Lb2[r][q];
      }
    }
  }
  return acc;
}

// Logical blocks first, first + stride, ... of one right-hand side, lane tx of each
// (the kernels: one logical block per workgroup, grid-stride, in XCD-aware order so that
// consecutive logical blocks, neighbouring column tiles and bands of the same levels,
// share an L2; the fused small-problem iteration: several logical blocks side by side
// in one workgroup, in natural order).  A block covers st_threads * st_cols columns:
// with two columns per thread the constant-coefficient tile takes columns
// (2 tx, 2 tx + 1) of its tile, the variable-coefficient tile marches columns tx and
// st_threads + tx one after the other.
template <int RB, bool VAR, int OUT, bool DOT>
__device__ __forceinline__ double stencil_run_rb(const DevPlan& P, const double* __restrict__ x,
                                                 double* __restrict__ y, const double* __restrict__ f, int first,
                                                 int stride, int tx, bool remap) {
  const int cols = P.st_threads * P.st_cols;
  const int xtiles = (P.nx + cols - 1) / cols;
  const int tiles = ((P.ny1 + RB - 1) / RB) * xtiles;
  const int nblk = stencil_blocks(P);
  double acc = 0.0;
  for (int w = first; w < nblk; w += stride) {
    const int lb = remap ? xcd_remap(w, nblk) : w;
    const int tile = lb % tiles;
    const int band = tile / xtiles, c0 = (tile % xtiles) * cols, chunk = lb / tiles;
    if constexpr (!VAR) {
      if (P.st_cols == 2) {
        acc += stencil_tile2<RB, OUT, DOT>(P, x, y, f, band, c0 + 2 * tx, chunk);
        continue;
      }
    }
    for (int q = 0; q < P.st_cols; ++q)
      acc += stencil_tile<RB, VAR, OUT, DOT>(P, x, y, f, band, c0 + q * P.st_threads + tx, chunk);
  }
  return acc;
}

template <bool VAR, int OUT, bool DOT>
__device__ __forceinline__ double stencil_run(const DevPlan& P, const double* __restrict__ x, double* __restrict__ y,
                                              const double* __restrict__ f, int first, int stride, int tx,
                                              bool remap) {
  return P.st_rows == 2 ? stencil_run_rb<2, VAR, OUT, DOT>(P, x, y, f, first, stride, tx, remap)
                        : stencil_run_rb<1, VAR, OUT, DOT>(P, x, y, f, first, stride, tx, remap);
}

}  // namespace
}  // namespace abac

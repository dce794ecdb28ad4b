// Device code of the transform passes of z = P_alpha^{-1} r (Section 2.3): per-tile
// bodies of the first x-DST pass (with the fused Lanczos step), the y-DST pass, the time
// pass K Y K Y (or the single K of C_alpha^{-1}) and the last x-DST pass (with the
// partial sums of <q, p>).  Each body is one workgroup's work on one tile; the kernels
// run one tile per workgroup, the fused small-problem iteration runs every tile of a
// right-hand side in one workgroup.
#pragma once
#include "abac_internal.h"

namespace abac {
namespace {

template <typename T, int L, int WG> constexpr int seqs_of() { return WG / fft_tps<T, L>(); }

// LDS bytes of the time pass's partials of <q, P^{-1} q>: one per thread, then one per
// group of G = min(8, TPS) threads of a sequence.
template <typename T, int L, int WG>
constexpr size_t time_red_bytes() {
  constexpr int TPS = fft_tps<T, L>(), G = TPS >= 8 ? 8 : TPS;
  return (size_t)(WG + WG / G) * sizeof(double);
}

// LDS bytes of one workgroup: the interleaved sequences; the inverse x pass reuses
// the region for its FP64 output staging; the y pass (length <= 1024) also holds its
// twiddle table, and the time pass its twiddles, spectral coefficients (A_k, B_k) and
// a^{+-t} scalings, each read once per block instead of once per butterfly or element.
template <typename T, int L, int WG, int KIND>
constexpr size_t lds_of() {
  constexpr size_t c = sizeof(cplx<T>);
  constexpr size_t data = (size_t)seqs_of<T, L, WG>() * L * c;
  if constexpr (KIND == TK_XINV) {
    constexpr size_t ostage = (size_t)2 * seqs_of<T, L, WG>() * (L / 2 + 1) * sizeof(double);
    return data > ostage ? data : ostage;
  } else if constexpr (KIND == TK_Y) {
    return data + (size_t)L * c;
  } else if constexpr (KIND == TK_TIME) {
    // + the partials of <q, P^{-1} q> where they do not fit the (A_k, B_k) table, which
    // they reuse once the weights are in registers
    constexpr size_t tables = (size_t)3 * L * c + (size_t)2 * L * sizeof(T);
    constexpr size_t red = time_red_bytes<T, L, WG>(), abk = (size_t)2 * L * c;
    return data + tables + (red > abk ? red : 0);
  } else {
    return data;
  }
}

template <typename T, int L, int WG, int KIND>
constexpr bool tile_ok() {
  return WG >= fft_tps<T, L>() && WG % fft_tps<T, L>() == 0 && WG % 64 == 0 && lds_of<T, L, WG, KIND>() <= kMaxTransformLds;
}

// Copy an n-entry table into LDS (the caller places the barrier).
template <typename V>
__device__ __forceinline__ void stage_table(V* dst, const V* __restrict__ src, int n) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
}

// Reciprocal square root, absolute value and sign transfer in the working precision
// (the FP32 path must not round-trip through the FP64 routines).  FP32 uses the
// hardware reciprocal square root directly: its arguments here (|mu|^2 and
// (|mu| + |Re mu|)/2 of the spectral weights, mu bounded away from 0 for every legal
// plan) are normal numbers, for which rsqrtf returns the same value; rsqrtf only adds
// the rescaling of subnormal arguments, five instructions around each of the pass's 36.
__device__ __forceinline__ float rsqrt_w(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double rsqrt_w(double v) { return rsqrt(v); }
__device__ __forceinline__ float fabs_w(float v) { return fabsf(v); }
__device__ __forceinline__ double fabs_w(double v) { return fabs(v); }
__device__ __forceinline__ float copysign_w(float a, float b) { return copysignf(a, b); }
__device__ __forceinline__ double copysign_w(double a, double b) { return copysign(a, b); }

template <typename T>
__device__ __forceinline__ cplx<T> inv_sqrt_principal(cplx<T> mu) {
  // 1/s(mu), s the principal square root.  With |mu| = sqrt(x^2 + y^2) and
  // w = sqrt((|mu| + |x|)/2):  s = (w, y/(2w)) for x >= 0 and (|y|/(2w), sign(y) w)
  // for x < 0, and 1/s = conj(s)/|mu|.  Two reciprocal square roots, no division.
  const T x = mu.x, y = mu.y;
  const T rr = x * x + y * y;
  const T g = rsqrt_w(rr);               // 1/|mu|
  const T w2 = (rr * g + fabs_w(x)) * (T)0.5;
  const T h = rsqrt_w(w2);               // 1/w
  const T w = w2 * h;
  T sr, si;
  if (x >= (T)0) {
    sr = w;
    si = (T)0.5 * y * h;
  } else {
    sr = (T)0.5 * fabs_w(y) * h;
    si = copysign_w(w, y);
  }
  return cplx<T>{sr * g, -si * g};
}

// Copy a [rows][width] tile held in LDS with row stride `ld` to `rows` consecutive
// global rows of length `width` (one contiguous range), coalesced.
template <typename TS, typename TD>
__device__ __forceinline__ void tile_out(TD* __restrict__ dst, const TS* src, int rows, int width, int ld) {
  const int total = rows * width;
  int e = threadIdx.x;
  int r = e / width, c = e - r * width;
  const int dr = blockDim.x / width, dc = blockDim.x - dr * width;
  for (; e < total; e += blockDim.x) {
    dst[e] = (TD)src[r * ld + c];
    r += dr;
    c += dc;
    if (c >= width) {
      c -= width;
      ++r;
    }
  }
}

// Copy cnt <= PER * WG contiguous values of src into LDS (converted to TD): every
// load of a thread is issued (from a clamped, in-bounds index) before any is used.
template <int PER, int WG, typename TS, typename TD>
__device__ __forceinline__ void stage_in(TD* dst, const TS* __restrict__ src, int cnt) {
  TS v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) v[u] = src[min((int)threadIdx.x + u * WG, cnt - 1)];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * WG;
    if (e < cnt) dst[e] = (TD)v[u];
  }
}

// ---------------------------------------------------------------------------
// first pass: DST-I along x of every row (FP64 in, transform precision out),
// optionally fused with the Lanczos step q = sig_j A Z_j - delta v_j - gamma_j v_{j-1}
// ---------------------------------------------------------------------------
// One tile (2 S rows) of right-hand side b; the caller skips stopped right-hand sides.
// tw: the length-L twiddle table (the plan's, or a copy the caller staged in LDS).
template <typename T, int L, int WG>
__device__ __forceinline__ void dstx_fwd_tile(const DevPlan& P, int mode, const double* __restrict__ in, int b,
                                              int tile, const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int R = FftShape<T, L>::R, TPS = L / R, S = seqs_of<T, L, WG>(), Mx = L / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  T* stage = reinterpret_cast<T*>(smem);
  const size_t off = (size_t)b * P.N;
  const double* src = in ? in + off : nullptr;
  double* qout = nullptr;
  const double* vj = nullptr;
  const double* vjm1 = nullptr;
  double cA = 1.0, cB = 0.0, cC = 0.0;
  if (mode == FWD_LANCZOS) {
    const MinresState* st = P.st + b;
    const int j = st->iter + 1;
    qout = P.V[(j + 1) % 3] + off;
    src = qout;
    vj = P.V[j % 3] + off;
    vjm1 = P.V[j == 1 ? j % 3 : (j + 2) % 3] + off;   // v_0 has weight 0 at j = 1
    cA = st->sig;
    cB = st->delta * st->sig;
    cC = st->gamma * st->sig_prev;
  }
  const int nx = P.nx;
  const int rows = P.nt * P.ny1;
  const int row0 = tile * 2 * S;
  const int nrows = min(2 * S, rows - row0);
  const size_t base = (size_t)row0 * nx;
  const int cnt = nrows * nx;
  // cnt <= 2 S nx < WG * R: each thread stages at most R values, in batches whose
  // loads (clamped to the tile, so unconditional) are all issued before they are used
  constexpr int BATCH = 4;
  if (mode == FWD_LANCZOS) {
#pragma unroll
    for (int u0 = 0; u0 < R; u0 += BATCH) {
      double a[BATCH], bv[BATCH], cv[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const size_t e = base + min((int)threadIdx.x + (u0 + u) * WG, cnt - 1);
        a[u] = src[e];
        bv[u] = vj[e];
        cv[u] = vjm1[e];
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int e = threadIdx.x + (u0 + u) * WG;
        if (e < cnt) {
          const double q = cA * a[u] - cB * bv[u] - cC * cv[u];
          qout[base + e] = q;
          stage[e] = (T)q;
        }
      }
    }
  } else {
    stage_in<R, WG>(stage, src + base, cnt);
  }
  __syncthreads();
  const int s = threadIdx.x % S, j = threadIdx.x / S;
  const int ra = 2 * s, rb = 2 * s + 1;
  const bool va = ra < nrows, vb = rb < nrows;
  C v[R];
  // odd extension of both rows, without branches (as in the inverse pass)
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int t = j + i * TPS;
    const int src = t < Mx ? max(t - 1, 0) : min(2 * Mx - t - 1, Mx - 2);
    const T a = stage[ra * nx + src], c = stage[rb * nx + src];
    const bool zero = t == 0 || t == Mx, neg = t > Mx;
    v[i] = C{zero || !va ? (T)0 : (neg ? -a : a), zero || !vb ? (T)0 : (neg ? -c : c)};
  }
  __syncthreads();
  fft_seq<T, L, false>(v, j, lds + s, S, tw);
  const T scl = (T)(1.0 / sqrt((double)L));
  // stage the transformed rows ([2S][Mx+1] padded) and write them out contiguously
  __syncthreads();
  constexpr int LDO = Mx + 1;
#pragma unroll
  for (int i = 0; i <= R / 2; ++i) {
    const int k = j + i * TPS;
    if (k == 0 || k > Mx) continue;
    if (k == Mx) {
      stage[ra * LDO + Mx - 1] = 0;
      stage[rb * LDO + Mx - 1] = 0;
    } else {
      stage[ra * LDO + k - 1] = -v[i].y * scl;
      stage[rb * LDO + k - 1] = v[i].x * scl;
    }
  }
  __syncthreads();
  T* out = reinterpret_cast<T*>(P.scratch) + (size_t)b * P.NS + (size_t)row0 * Mx;
  tile_out<T, T>(out, stage, nrows, Mx, LDO);
}

// ---------------------------------------------------------------------------
// y pass (2D): DST-I along y of every column, in place on the scratch; two adjacent
// columns form one complex sequence.
// ---------------------------------------------------------------------------
// One block of right-hand side b (logical block index lbk).
template <typename T, int L, int WG>
__device__ __forceinline__ void dsty_tile(const DevPlan& P, int b, int lbk) {
  using C = cplx<T>;
  constexpr int R = FftShape<T, L>::R, TPS = L / R, S = seqs_of<T, L, WG>(), My = L / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  C* tws = reinterpret_cast<C*>(smem);
  C* lds = tws + L;
  const int cpairs = P.Mx / 2;
  const int bpl = (cpairs + S - 1) / S;
  const int t = lbk / bpl, cb = lbk % bpl;
  const int s = threadIdx.x % S, j = threadIdx.x / S;
  const int cp = cb * S + s;
  const bool valid = cp < cpairs;
  const int ld = P.Mx / 2;
  C* col = reinterpret_cast<C*>(reinterpret_cast<T*>(P.scratch) + (size_t)b * P.NS + (size_t)t * P.ms) +
           min(cp, cpairs - 1);   // clamped: the loads below are unconditional
  C v[R];
  // each column value is loaded once (elements tt = j + i TPS < My, i < R/2) and placed
  // in LDS at tt and, negated, at its mirror 2 My - tt: the odd extension in natural
  // order, from which the FFT reads its input
#pragma unroll
  for (int i = 0; i < R / 2; ++i) {
    const int tt = j + i * TPS;
    v[i] = col[(size_t)max(tt - 1, 0) * ld];
  }
  C* my = lds + s;
#pragma unroll
  for (int i = 0; i < R / 2; ++i) {
    const int tt = j + i * TPS;
    const C x = !valid || tt == 0 ? C{0, 0} : v[i];
    my[tt * S] = x;
    if (tt > 0) my[(2 * My - tt) * S] = C{-x.x, -x.y};
  }
  if (j == 0) my[My * S] = C{0, 0};
  stage_table(tws, reinterpret_cast<const C*>(P.twy), L);
  __syncthreads();
  fft_seq<T, L, false, true>(v, j, my, S, tws);
  const T scl = (T)(1.0 / sqrt((double)L));
  if (!valid) return;
#pragma unroll
  for (int i = 0; i <= R / 2; ++i) {
    const int k = j + i * TPS;
    if (k == 0 || k >= My) continue;
    col[(size_t)(k - 1) * ld] = C{-v[i].y * scl, v[i].x * scl};
  }
}

// ---------------------------------------------------------------------------
// time pass: per spatial mode pair, out = K Y K Y g, in place on the scratch.
// ---------------------------------------------------------------------------

// Spectral weights of two real modes packed as one complex sequence z = g_a + i g_b:
// with Z = F z, the spectra of the two modes are (Z_k + conj Z_{-k})/2 and
// (Z_k - conj Z_{-k})/(2i); weighting them by Ma_k, Mb_k and repacking gives
//   Z'_k = ((Ma + Mb) Z_k + (Ma - Mb) conj Z_{-k}) / 2.
// mu is Hermitian in k (mu_{-k} = conj mu_k), so one thread handles the pair
// (k, nt-k) with a single evaluation of Ma_k, Mb_k.  Input and output in LDS, natural
// order; `scale` folds in the 1/nt of the inverse DFT.  The weights are mu^{-1/2}
// (ABAC factor) or, with inv1, mu^{-1} (the block alpha-circulant C_alpha^{-1}).
// 1/mu (the weights of C_alpha^{-1} itself)
template <typename T>
__device__ __forceinline__ cplx<T> inv_complex(cplx<T> mu) {
  const T g = (T)1 / (mu.x * mu.x + mu.y * mu.y);
  return cplx<T>{mu.x * g, -mu.y * g};
}

template <typename T, int NT>
struct SpectralWeights {
  static constexpr int NU = FftShape<T, NT>::R / 2 + 1;   // frequency slots of one thread
  cplx<T> sp[NU], sm[NU];
};

// The weights (Ma + Mb)/2 and (Ma - Mb)/2 (times `scale`) of the frequencies
// k = j + u TPS <= NT/2 this thread handles; they depend on the mode pair only, so both
// passes of K Y K Y use the same ones.
template <typename T, int NT>
__device__ __forceinline__ void spectral_weight_slot(SpectralWeights<T, NT>& W, int u, int k, const cplx<T>* abk, T ba,
                                                     T bb, T scale, int inv1) {
  using C = cplx<T>;
  const C A = abk[2 * k], Bk = abk[2 * k + 1];
  const C mua = C{A.x + ba * Bk.x, A.y + ba * Bk.y}, mub = C{A.x + bb * Bk.x, A.y + bb * Bk.y};
  const C Ma = inv1 ? inv_complex<T>(mua) : inv_sqrt_principal<T>(mua);
  const C Mb = inv1 ? inv_complex<T>(mub) : inv_sqrt_principal<T>(mub);
  W.sp[u] = cscale(cadd(Ma, Mb), scale);
  W.sm[u] = cscale(csub(Ma, Mb), scale);
}

template <typename T, int NT>
__device__ __forceinline__ void spectral_weights(SpectralWeights<T, NT>& W, int j, const cplx<T>* abk, T ba, T bb,
                                                 T scale, int inv1) {
  constexpr int R = FftShape<T, NT>::R, TPS = NT / R;
  // slots u < R/2 hold k = j + u TPS < nt/2; the last slot (k = nt/2) is applied only by
  // thread 0 (spectral_apply), so only thread 0 evaluates it
#pragma unroll
  for (int u = 0; u < R / 2; ++u) spectral_weight_slot<T, NT>(W, u, j + u * TPS, abk, ba, bb, scale, inv1);
  if (j == 0) spectral_weight_slot<T, NT>(W, R / 2, NT / 2, abk, ba, bb, scale, inv1);
}

// a b + c conj(d) for complex a, b, c, d, as explicit fused multiply-adds (three per
// component, one product rounded)
__device__ __forceinline__ float fma_w(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_w(double a, double b, double c) { return fma(a, b, c); }
template <typename C>
__device__ __forceinline__ C cmul_add_conj(C a, C b, C c, C d) {
  return C{fma_w(a.x, b.x, fma_w(-a.y, b.y, fma_w(c.x, d.x, c.y * d.y))),
           fma_w(a.x, b.y, fma_w(a.y, b.x, fma_w(c.y, d.x, -(c.x * d.y))))};
}

// Apply the weights to the packed spectrum held in registers (v[i] = Z[j + i TPS]):
// Z'_k = sp Z_k + sm conj Z_{-k} and Z'_{-k} = conj(sp) Z_{-k} + conj(sm) conj Z_k.
// Thread j >= 1 owns the pairs of its low slots u < R/2 (k = j + u TPS < nt/2) with
// the mirrored slots R-1-u of thread TPS-j, which travel through LDS at their natural
// positions (published, updated by the owner, read back); thread 0 pairs its own
// slots u and R-u.  The LDS region lds[e S] must be free on entry; on return other
// threads may still be reading it.
template <typename T, int NT>
__device__ __forceinline__ void spectral_apply(cplx<T>* v, int j, cplx<T>* my, int S,
                                               const SpectralWeights<T, NT>& W) {
  using C = cplx<T>;
  constexpr int R = FftShape<T, NT>::R, TPS = NT / R, H = R / 2;
  if (j != 0) {
#pragma unroll
    for (int i = H; i < R; ++i) my[(j + i * TPS) * S] = v[i];
  }
  __syncthreads();
  if (j != 0) {
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const int kp = NT - (j + u * TPS);
      const C zk = v[u], zp = my[kp * S];
      const C sp = W.sp[u], sm = W.sm[u];
      v[u] = cmul_add_conj(sp, zk, sm, zp);
      my[kp * S] = cmul_add_conj(cconj(sp), zp, cconj(sm), zk);
    }
  } else {
#pragma unroll
    for (int u = 0; u <= H; ++u) {
      const int up = (R - u) & (R - 1);
      const C zk = v[u], zp = v[up];
      const C sp = W.sp[u], sm = W.sm[u];
      const C a = cmul_add_conj(sp, zk, sm, zp);
      if (up != u) v[up] = cmul_add_conj(cconj(sp), zp, cconj(sm), zk);
      v[u] = a;
    }
  }
  __syncthreads();
  if (j != 0) {
#pragma unroll
    for (int i = H; i < R; ++i) v[i] = my[(j + i * TPS) * S];
  }
}

// inv1 = 0: out = K Y K Y g with mu^{-1/2} (the ABAC P^{-1}); inv1 = 1: out = K g with
// mu^{-1} and no time reversal (C_alpha^{-1} = S K S of eqs. (1.5)-(1.7)).
// One block (S mode pairs, logical block index lbk) of right-hand side b.
//
// gamma != 0 (ABAC only): also the MINRES inner product <q, P^{-1} q>.  With
// P^{-1} = C^{-1/2} (C^{-1/2})^T (eq. (1.9)) it equals ||(C^{-1/2})^T q||^2, and in the
// sine basis (C^{-1/2})^T = Y K Y per mode, so <q, P^{-1} q> = ||K Y g||^2 summed over
// the modes: the squared norm of the first factor's output, which this pass holds
// anyway.  Each mode pair writes its sum to part_slot(PART_GAMMA)[pair]; the sum over a
// pair runs in an order fixed by the sequence length (not by the tile), so the result
// does not depend on the workgroup size.  Its LDS steps ride on the barriers the second
// factor takes anyway.
template <typename T, int NT, int WG>
__device__ __forceinline__ void time_tile(const DevPlan& P, int inv1, int b, int lbk, int gamma = 0) {
  using C = cplx<T>;
  constexpr int R = FftShape<T, NT>::R, TPS = NT / R, S = seqs_of<T, NT, WG>();
  extern __shared__ __align__(16) unsigned char smem[];
  // LDS: twiddles [NT], (A_k, B_k) [2 NT], a^t [NT], a^-t [NT], then the sequences
  C* tws = reinterpret_cast<C*>(smem);
  C* abk = tws + NT;
  T* sc = reinterpret_cast<T*>(abk + 2 * NT);
  T* sci = sc + NT;
  C* lds = reinterpret_cast<C*>(sci + NT);
  // <q, P^{-1} q> partials: red[j S + s] per thread, red2[g S + s] per group of G threads;
  // they take the (A_k, B_k) table's place (free once the weights are in registers, i.e.
  // after the first FFT's first barrier) where it is large enough, else follow the
  // sequences
  constexpr int G = TPS >= 8 ? 8 : TPS;
  constexpr bool red_in_abk = time_red_bytes<T, NT, WG>() <= (size_t)2 * NT * sizeof(C);
  double* red = red_in_abk ? reinterpret_cast<double*>(abk) : reinterpret_cast<double*>(lds + S * NT);
  double* red2 = red + WG;
  const int s = threadIdx.x % S, j = threadIdx.x / S;
  const int npairs = P.ms / 2;
  const int pair = lbk * S + s;
  const bool valid = pair < npairs;
  const int pc = min(pair, npairs - 1);   // clamped: the loads below are unconditional
  const int ld = npairs;
  C* g = reinterpret_cast<C*>(reinterpret_cast<T*>(P.scratch) + (size_t)b * P.NS) + pair;
  const C* gin = reinterpret_cast<const C*>(reinterpret_cast<const T*>(P.scratch) + (size_t)b * P.NS) + pc;
  const T* __restrict__ beta = reinterpret_cast<const T*>(P.beta);
  const T ba = valid ? beta[2 * pc] : (T)1;
  const T bb = valid ? beta[2 * pc + 1] : (T)1;
  C* my = lds + s;
  C v[R];
  // Y (ABAC only): e_t = g_{nt-1-t}; the D scaling follows once the table is in LDS
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int t = j + i * TPS;
    v[i] = gin[(size_t)(inv1 ? t : NT - 1 - t) * ld];
  }
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = valid ? v[i] : C{0, 0};
  stage_table(tws, reinterpret_cast<const C*>(P.twt), NT);
  stage_table(abk, reinterpret_cast<const C*>(P.abk), 2 * NT);
  stage_table(sc, reinterpret_cast<const T*>(P.sc), NT);
  stage_table(sci, reinterpret_cast<const T*>(P.sci), NT);
  __syncthreads();
  const C* tw = tws;
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = cscale(v[i], sc[j + i * TPS]);
  SpectralWeights<T, NT> W;
  spectral_weights<T, NT>(W, j, abk, ba, bb, (T)(0.5 / NT), inv1);
  // first (or only) factor: FFT, weights, inverse FFT
  fft_seq<T, NT, false>(v, j, my, S, tw);
  __syncthreads();
  spectral_apply<T, NT>(v, j, my, S, W);
  __syncthreads();
  fft_seq<T, NT, true>(v, j, my, S, tw);
  double gsum = 0.0;   // with gamma: the pair's ||K Y g||^2, valid in thread j = 0
  if (gamma) {
    // this thread's part (K's output is a^{-t} v_t), published for the group sums below
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const double sv = (double)sci[j + i * TPS];
      a += sv * sv * ((double)v[i].x * v[i].x + (double)v[i].y * v[i].y);
    }
    red[j * S + s] = a;
  }
  if (!inv1) {
    // D^{-1}, Y, D between the factors, y_t = a^{2t-nt+1} c_{nt-1-t}, without moving data:
    // with g_s = y_{nt-1-s} (an elementwise scaling of c), the DFT of y at frequency k is
    // e^{2 pi i k/nt} G_k, G the inverse-direction DFT of g.  The weights act on G as on
    // the DFT of y (the phase at -k is the conjugate of the one at k), and the phase left
    // on the spectrum shifts the inverse DFT by one level: out_t = w_{t+1}.
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int t = j + i * TPS;
      v[i] = cscale(v[i], sc[NT - 1 - t] * sci[t]);
    }
    __syncthreads();
    if (gamma && j < TPS / G) {
      // groups of G consecutive threads of a sequence (red is visible after the barrier
      // above; red2 after the barriers inside the FFT below)
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < G; ++q) a += red[(j * G + q) * S + s];
      red2[j * S + s] = a;
    }
    fft_seq<T, NT, true>(v, j, my, S, tw);
    __syncthreads();
    if (gamma && j == 0) {
      for (int q = 0; q < TPS / G; ++q) gsum += red2[q * S + s];
    }
    spectral_apply<T, NT>(v, j, my, S, W);
    __syncthreads();
    fft_seq<T, NT, true>(v, j, my, S, tw);
  }
  const int shift = inv1 ? 0 : 1;
  if (valid) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int t = (j + i * TPS - shift) & (NT - 1);
      g[(size_t)t * ld] = cscale(v[i], sci[t]);
    }
  }
  if (gamma && j == 0 && valid) part_slot(P, PART_GAMMA, b)[pair] = gsum;
}

// ---------------------------------------------------------------------------
// last pass: inverse DST-I along x (transform precision in, FP64 out), optionally
// fused with the partial sums of <q, p>.
// ---------------------------------------------------------------------------
// One tile (2 S rows) of right-hand side b; returns this thread's part of <q, p> (0 in
// INV_PLAIN).  The caller skips stopped right-hand sides.  tw as for dstx_fwd_tile.
template <typename T, int L, int WG>
__device__ __forceinline__ double dstx_inv_tile(const DevPlan& P, int mode, double* __restrict__ outp, int b,
                                                int tile, const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int R = FftShape<T, L>::R, TPS = L / R, S = seqs_of<T, L, WG>(), Mx = L / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  T* stage = reinterpret_cast<T*>(smem);
  double* ostage = reinterpret_cast<double*>(smem);
  const size_t off = (size_t)b * P.N;
  double* out = outp ? outp + off : nullptr;
  const double* q = nullptr;
  const MinresState* st = P.st + b;
  if (mode != INV_PLAIN) {
    if (mode == INV_GAMMA_INIT || mode == INV_Z_INIT) {
      out = P.Z[zslot(1)] + off;
      if (mode == INV_GAMMA_INIT) q = P.V[1] + off;
    } else {
      const int jj = st->iter + 1;
      out = P.Z[zslot(jj + 1)] + off;
      if (mode == INV_GAMMA_ITER) q = P.V[(jj + 1) % 3] + off;
    }
  }
  const int nx = P.nx;
  const int rows = P.nt * P.ny1;
  const int row0 = tile * 2 * S;
  const int nrows = min(2 * S, rows - row0);
  const T* scr = reinterpret_cast<const T*>(P.scratch) + (size_t)b * P.NS + (size_t)row0 * Mx;
  const int cnt = nrows * Mx;   // <= 2 S Mx = WG * R
  stage_in<R, WG>(stage, scr, cnt);
  __syncthreads();
  const int s = threadIdx.x % S, j = threadIdx.x / S;
  const int ra = 2 * s, rb = 2 * s + 1;
  const bool va = ra < nrows, vb = rb < nrows;
  C v[R];
  // odd extension of both rows, without branches: element t is x[t-1] for 0 < t < Mx,
  // -x[2 Mx - t - 1] for t > Mx, 0 at t = 0 and t = Mx (rows past the tile read stale
  // LDS words of the staging area, selected away)
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int t = j + i * TPS;
    const int src = t < Mx ? max(t - 1, 0) : min(2 * Mx - t - 1, Mx - 2);
    const T a = stage[ra * Mx + src], c = stage[rb * Mx + src];
    const bool zero = t == 0 || t == Mx, neg = t > Mx;
    v[i] = C{zero || !va ? (T)0 : (neg ? -a : a), zero || !vb ? (T)0 : (neg ? -c : c)};
  }
  __syncthreads();
  fft_seq<T, L, false>(v, j, lds + s, S, tw);
  const double scl = 1.0 / sqrt((double)L);
  // stage the FP64 rows packed ([2S][nx]: the block's 2S output rows are one contiguous
  // run of memory, and the odd row length in 8-byte words spreads the sequences of a
  // wave over the banks) and write them out; with q, accumulate <q, p> in a fixed order
  // for a fixed tile
  __syncthreads();
  const int ldo = nx;
#pragma unroll
  for (int i = 0; i < R / 2; ++i) {   // k = j + i TPS < Mx; slot k-1 for k >= 1
    const int k = j + i * TPS;
    if (i > 0 || k > 0) {
      ostage[ra * ldo + k - 1] = -(double)v[i].y * scl;
      ostage[rb * ldo + k - 1] = (double)v[i].x * scl;
    }
  }
  __syncthreads();
  double* o = out + (size_t)row0 * nx;
  const int total = nrows * nx;   // < WG * R
  double acc = 0.0;
  if (!q) {
    // one contiguous run: 16-byte moves of pairs, and the odd last value
    const int npair = total / 2;
    for (int e = threadIdx.x; e < npair; e += WG)
      *reinterpret_cast<dpair*>(o + 2 * e) = *reinterpret_cast<const dpair*>(ostage + 2 * e);
    if ((total & 1) && threadIdx.x == 0) o[total - 1] = ostage[total - 1];
  } else {
    const double* qq = q ? q + (size_t)row0 * nx : nullptr;
    int r = (int)threadIdx.x / nx, c = (int)threadIdx.x - r * nx;
    const int dr = WG / nx, dc = WG - dr * nx;
    constexpr int BATCH = 8;
#pragma unroll
    for (int u0 = 0; u0 < R; u0 += BATCH) {
      double qv[BATCH];
      if (qq) {
#pragma unroll
        for (int u = 0; u < BATCH; ++u) qv[u] = qq[min((int)threadIdx.x + (u0 + u) * WG, total - 1)];
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int e = threadIdx.x + (u0 + u) * WG;
        if (e < total) {
          const double val = ostage[r * ldo + c];
          o[e] = val;
          if (qq) acc += val * qv[u];
        }
        r += dr;
        c += dc;
        if (c >= nx) {
          c -= nx;
          ++r;
        }
      }
    }
  }
  return acc;
}

// ---------------------------------------------------------------------------
// fused 2D passes, for square grids whose whole (y, x) level fits in LDS: one block
// per time level applies the DST-I along x and along y in LDS, so the y passes over
// HBM disappear (three transform passes per apply instead of five).  The level stays
// in LDS as [ny][Mx] in the transform precision (column Mx-1 the zero pad, as in the
// scratch layout, rows padded to Mx+1 entries so that the rows and the columns of
// neighbouring sequences fall in different LDS banks); its lines go through a separate
// exchange area, S sequences at a time.
// ---------------------------------------------------------------------------
template <typename T, int L>
constexpr size_t slab_bytes() {
  return ((size_t)(L / 2 - 1) * (L / 2 + 1) * sizeof(T) + 15) / 16 * 16;
}

template <typename T, int L, int WG>
constexpr size_t slab_lds_of() {
  return slab_bytes<T, L>() + (size_t)seqs_of<T, L, WG>() * L * sizeof(cplx<T>);
}

template <typename T, int L, int WG>
constexpr bool slab_ok() {
  return L >= 16 && L <= 256 && WG >= fft_tps<T, L>() && WG % fft_tps<T, L>() == 0 && WG % 64 == 0 &&
         slab_lds_of<T, L, WG>() <= kMaxTransformLds;
}

// Orthonormal DST-I, in place, of `nlines` lines of the level held in LDS (ROWS: the
// rows, element e of row l at slab[l (Mx+1) + e]; otherwise the columns, element e of
// column l at slab[e (Mx+1) + l]).  Lines of length M-1 = L/2-1 go two to a complex
// sequence of length L (odd extension); the transform of the first is minus the
// imaginary part, of the second the real part.  Rows write 0 to the pad column.
// All threads call it together; it ends with a barrier.
template <typename T, int L, int WG, bool ROWS>
__device__ __forceinline__ void slab_dst(T* slab, int nlines, cplx<T>* exch, const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int R = FftShape<T, L>::R, TPS = L / R, S = seqs_of<T, L, WG>(), M = L / 2, LD = M + 1;
  const int s = threadIdx.x % S, j = threadIdx.x / S;
  const int npairs = (nlines + 1) / 2;
  const T scl = (T)(1.0 / sqrt((double)L));
  for (int p0 = 0; p0 < npairs; p0 += S) {
    const int p = p0 + s;
    const bool va = 2 * p < nlines, vb = 2 * p + 1 < nlines;
    const int la = min(2 * p, nlines - 1), lb = min(2 * p + 1, nlines - 1);
    C v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int t = j + i * TPS;
      const int e = t < M ? max(t - 1, 0) : min(2 * M - t - 1, M - 2);
      const T a = slab[ROWS ? la * LD + e : e * LD + la];
      const T c = slab[ROWS ? lb * LD + e : e * LD + lb];
      const bool zero = t == 0 || t == M;
      const T sg = t < M ? (T)1 : (T)-1;
      v[i] = C{zero || !va ? (T)0 : sg * a, zero || !vb ? (T)0 : sg * c};
    }
    __syncthreads();   // the previous round's last reads of the exchange area are done
    fft_seq<T, L, false>(v, j, exch + s, S, tw);
#pragma unroll
    for (int i = 0; i <= R / 2; ++i) {
      const int k = j + i * TPS;
      if (k == 0 || k > M) continue;
      if (k == M) {
        if (ROWS) {
          if (va) slab[la * LD + M - 1] = 0;
          if (vb) slab[lb * LD + M - 1] = 0;
        }
        continue;
      }
      const int e = k - 1;
      if (va) slab[ROWS ? la * LD + e : e * LD + la] = -v[i].y * scl;
      if (vb) slab[ROWS ? lb * LD + e : e * LD + lb] = v[i].x * scl;
    }
  }
  __syncthreads();
}

// First pass, fused: (Lanczos step,) DST-I along x and y of level lvl of right-hand
// side b, written to the scratch.  The caller skips stopped right-hand sides.
template <typename T, int L, int WG>
__device__ __forceinline__ void dst2_fwd_tile(const DevPlan& P, int mode, const double* __restrict__ in, int b, int lvl) {
  using C = cplx<T>;
  constexpr int M = L / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  T* slab = reinterpret_cast<T*>(smem);
  C* exch = reinterpret_cast<C*>(smem + slab_bytes<T, L>());
  const size_t off = (size_t)b * P.N;
  const double* src = in ? in + off : nullptr;
  double* qout = nullptr;
  const double* vj = nullptr;
  const double* vjm1 = nullptr;
  double cA = 1.0, cB = 0.0, cC = 0.0;
  if (mode == FWD_LANCZOS) {
    const MinresState* st = P.st + b;
    const int j = st->iter + 1;
    qout = P.V[(j + 1) % 3] + off;
    src = qout;
    vj = P.V[j % 3] + off;
    vjm1 = P.V[j == 1 ? j % 3 : (j + 2) % 3] + off;   // v_0 has weight 0 at j = 1
    cA = st->sig;
    cB = st->delta * st->sig;
    cC = st->gamma * st->sig_prev;
  }
  const int nx = M - 1, cnt = nx * nx;
  const size_t base = (size_t)lvl * P.m;
  // stage the level; a thread's BATCH loads (clamped, so unconditional) are issued
  // before any is used
  constexpr int BATCH = 8;
  for (int e0 = 0; e0 < cnt; e0 += BATCH * WG) {
    double a[BATCH], bv[BATCH], cv[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const size_t e = base + min(e0 + (int)threadIdx.x + u * WG, cnt - 1);
      a[u] = src[e];
      if (mode == FWD_LANCZOS) {
        bv[u] = vj[e];
        cv[u] = vjm1[e];
      }
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int e = e0 + (int)threadIdx.x + u * WG;
      if (e < cnt) {
        double q = a[u];
        if (mode == FWD_LANCZOS) {
          q = cA * a[u] - cB * bv[u] - cC * cv[u];
          qout[base + e] = q;
        }
        const int r = e / nx;
        slab[r * (M + 1) + (e - r * nx)] = (T)q;
      }
    }
  }
  __syncthreads();
  slab_dst<T, L, WG, true>(slab, nx, exch, reinterpret_cast<const C*>(P.twx));
  slab_dst<T, L, WG, false>(slab, M, exch, reinterpret_cast<const C*>(P.twy));
  T* out = reinterpret_cast<T*>(P.scratch) + (size_t)b * P.NS + (size_t)lvl * P.ms;
  for (int e = threadIdx.x; e < nx * M; e += WG) {
    const int r = e / M;
    out[e] = slab[r * (M + 1) + (e - r * M)];
  }
}

// Last pass, fused: DST-I along y and x of level lvl of the scratch, FP64 rows out;
// returns this thread's part of <q, p> in the GAMMA modes (0 otherwise).  The caller
// skips stopped right-hand sides.
template <typename T, int L, int WG>
__device__ __forceinline__ double dst2_inv_tile(const DevPlan& P, int mode, double* __restrict__ outp, int b, int lvl) {
  using C = cplx<T>;
  constexpr int M = L / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  T* slab = reinterpret_cast<T*>(smem);
  C* exch = reinterpret_cast<C*>(smem + slab_bytes<T, L>());
  const size_t off = (size_t)b * P.N;
  double* out = outp ? outp + off : nullptr;
  const double* q = nullptr;
  const MinresState* st = P.st + b;
  if (mode != INV_PLAIN) {
    if (mode == INV_GAMMA_INIT || mode == INV_Z_INIT) {
      out = P.Z[zslot(1)] + off;
      if (mode == INV_GAMMA_INIT) q = P.V[1] + off;
    } else {
      const int jj = st->iter + 1;
      out = P.Z[zslot(jj + 1)] + off;
      if (mode == INV_GAMMA_ITER) q = P.V[(jj + 1) % 3] + off;
    }
  }
  const int nx = M - 1, cnt = nx * M;
  const T* scr = reinterpret_cast<const T*>(P.scratch) + (size_t)b * P.NS + (size_t)lvl * P.ms;
  constexpr int BATCH = 16;
  for (int e0 = 0; e0 < cnt; e0 += BATCH * WG) {
    T v[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) v[u] = scr[min(e0 + (int)threadIdx.x + u * WG, cnt - 1)];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int e = e0 + (int)threadIdx.x + u * WG;
      if (e < cnt) {
        const int r = e / M;
        slab[r * (M + 1) + (e - r * M)] = v[u];
      }
    }
  }
  __syncthreads();
  slab_dst<T, L, WG, false>(slab, M, exch, reinterpret_cast<const C*>(P.twy));
  slab_dst<T, L, WG, true>(slab, nx, exch, reinterpret_cast<const C*>(P.twx));
  const size_t base = (size_t)lvl * P.m;
  double* o = out + base;
  const double* qq = q ? q + base : nullptr;
  const int total = nx * nx;
  double acc = 0.0;
  for (int e0 = 0; e0 < total; e0 += BATCH * WG) {
    double qv[BATCH];
    if (qq) {
#pragma unroll
      for (int u = 0; u < BATCH; ++u) qv[u] = qq[min(e0 + (int)threadIdx.x + u * WG, total - 1)];
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int e = e0 + (int)threadIdx.x + u * WG;
      if (e < total) {
        const int r = e / nx;
        const double val = (double)slab[r * (M + 1) + (e - r * nx)];
        o[e] = val;
        if (qq) acc += val * qv[u];
      }
    }
  }
  return acc;
}


}  // namespace
}  // namespace abac

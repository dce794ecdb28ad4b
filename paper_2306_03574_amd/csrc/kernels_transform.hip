// Transform passes of z = P_alpha^{-1} r (Section 2.3), computed as
//     z = S [ K Y K Y ] S r,   K = D^{-1} F^{-1} diag(mu^{-1/2}) F D  (per spatial mode),
// where S is the orthonormal DST-I in space (S = S^T = S^{-1}, so the inner DST pair
// of the three-step recipe done twice cancels), F the DFT over the nt time levels,
// D = diag(a^t), a = alpha^{1/nt}, Y the time reversal, and mu the eigenvalues of
// C_alpha (eq. (1.7), Appendix A).  The transposed factor uses
// (C^{-1/2})^T = Y C^{-1/2} Y (Lemma on the realness and symmetry of C_alpha^{1/2},
// Section 2.1).
//
// DST-I of length M-1 is taken from a complex FFT of length 2M of the odd extension;
// two real rows ride in one complex sequence (real and imaginary part).  The time
// FFTs are real transforms of two spatial modes packed the same way; the per-mode
// spectral weights are applied to the packed spectrum in closed form.
//
// Scratch layout (private to the apply): [batch][nt][ny1][Mx] in the transform
// precision, Mx = nx+1; column Mx-1 is a zero pad so rows and mode pairs are aligned.
//
// Every transform kernel is instantiated for several workgroup sizes WG (tile =
// WG / TPS sequences per block); the plan's autotuner picks one per kernel.
#include <algorithm>

#include "abac_internal.h"

namespace abac {

namespace {

template <int L, int WG> constexpr int seqs_of() { return WG / fft_tps<L>(); }
template <typename T, int L, int WG>
constexpr bool tile_ok() {
  return WG >= fft_tps<L>() && WG % fft_tps<L>() == 0 && WG % 64 == 0 &&
         (size_t)seqs_of<L, WG>() * L * sizeof(cplx<T>) <= kMaxTransformLds;
}

template <typename T>
__device__ __forceinline__ cplx<T> inv_sqrt_principal(cplx<T> mu) {
  // 1/s(mu), s the principal square root.  With |mu| = sqrt(x^2 + y^2) and
  // w = sqrt((|mu| + |x|)/2):  s = (w, y/(2w)) for x >= 0 and (|y|/(2w), sign(y) w)
  // for x < 0, and 1/s = conj(s)/|mu|.  Two reciprocal square roots, no division.
  const T x = mu.x, y = mu.y;
  const T rr = x * x + y * y;
  const T g = rsqrt(rr);                 // 1/|mu|
  const T w2 = (rr * g + fabs(x)) * (T)0.5;
  const T h = rsqrt(w2);                 // 1/w
  const T w = w2 * h;
  T sr, si;
  if (x >= (T)0) {
    sr = w;
    si = (T)0.5 * y * h;
  } else {
    sr = (T)0.5 * fabs(y) * h;
    si = copysign(w, y);
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

// ---------------------------------------------------------------------------
// first pass: DST-I along x of every row (FP64 in, transform precision out),
// optionally fused with the Lanczos step q = sig_j A Z_j - delta v_j - gamma_j v_{j-1}
// ---------------------------------------------------------------------------
template <typename T, int L, int WG>
__global__ void __launch_bounds__(WG)
k_dstx_fwd(DevPlan P, int mode, int check, const double* __restrict__ in) {
  using C = cplx<T>;
  constexpr int R = FftShape<L>::R, TPS = L / R, S = seqs_of<L, WG>(), Mx = L / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  T* stage = reinterpret_cast<T*>(smem);
  const int b = blockIdx.y;
  const size_t off = (size_t)b * P.N;
  const double* src = in ? in + off : nullptr;
  double* qout = nullptr;
  const double* vj = nullptr;
  const double* vjm1 = nullptr;
  double cA = 1.0, cB = 0.0, cC = 0.0;
  if (check || mode == FWD_LANCZOS) {
    const MinresState* st = P.st + b;
    if (st->state != ST_RUNNING) return;
    if (mode == FWD_LANCZOS) {
      const int j = st->iter + 1;
      qout = P.V[(j + 1) % 3] + off;
      src = qout;
      vj = P.V[j % 3] + off;
      vjm1 = P.V[(j + 2) % 3] + off;
      cA = st->sig;
      cB = st->delta * st->sig;
      cC = st->gamma * st->sig_prev;
    }
  }
  const int nx = P.nx;
  const int rows = P.nt * P.ny1;
  const int row0 = blockIdx.x * 2 * S;
  const int nrows = min(2 * S, rows - row0);
  const size_t base = (size_t)row0 * nx;
  const int cnt = nrows * nx;
  if (mode == FWD_LANCZOS) {
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
      const double q = cA * src[base + e] - cB * vj[base + e] - cC * vjm1[base + e];
      qout[base + e] = q;
      stage[e] = (T)q;
    }
  } else {
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) stage[e] = (T)src[base + e];
  }
  __syncthreads();
  const int s = threadIdx.x % S, j = threadIdx.x / S;
  const int ra = 2 * s, rb = 2 * s + 1;
  const bool va = ra < nrows, vb = rb < nrows;
  C v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int t = j + i * TPS;
    T a = 0, c = 0;
    if (t > 0 && t < Mx) {
      if (va) a = stage[ra * nx + t - 1];
      if (vb) c = stage[rb * nx + t - 1];
    } else if (t > Mx) {
      const int idx = 2 * Mx - t - 1;
      if (va) a = -stage[ra * nx + idx];
      if (vb) c = -stage[rb * nx + idx];
    }
    v[i] = C{a, c};
  }
  __syncthreads();
  fft_seq<T, L, false>(v, j, lds + s, S, reinterpret_cast<const C*>(P.twx));
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
template <typename T, int L, int WG>
__global__ void __launch_bounds__(WG)
k_dsty(DevPlan P, int check) {
  using C = cplx<T>;
  constexpr int R = FftShape<L>::R, TPS = L / R, S = seqs_of<L, WG>(), My = L / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int b = blockIdx.y;
  if (check && P.st[b].state != ST_RUNNING) return;
  const int cpairs = P.Mx / 2;
  const int bpl = (cpairs + S - 1) / S;
  const int t = blockIdx.x / bpl, cb = blockIdx.x % bpl;
  const int s = threadIdx.x % S, j = threadIdx.x / S;
  const int cp = cb * S + s;
  const bool valid = cp < cpairs;
  const int ld = P.Mx / 2;
  C* col = reinterpret_cast<C*>(reinterpret_cast<T*>(P.scratch) + (size_t)b * P.NS + (size_t)t * P.ms) + cp;
  C v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int tt = j + i * TPS;
    C z{0, 0};
    if (valid) {
      if (tt > 0 && tt < My) {
        z = col[(size_t)(tt - 1) * ld];
      } else if (tt > My) {
        const C w = col[(size_t)(2 * My - tt - 1) * ld];
        z = C{-w.x, -w.y};
      }
    }
    v[i] = z;
  }
  fft_seq<T, L, false>(v, j, lds + s, S, reinterpret_cast<const C*>(P.twy));
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
// order; `scale` folds in the 1/nt of the inverse DFT.
template <typename T, int NT>
__device__ __forceinline__ void spectral_pairs(cplx<T>* my, int S, int j, const cplx<T>* __restrict__ abk, T ba, T bb,
                                               T scale) {
  using C = cplx<T>;
  constexpr int R = FftShape<NT>::R, TPS = NT / R;
  constexpr int NU = R / 2 + 1;
#pragma unroll 2
  for (int u = 0; u < NU; ++u) {
    const int k = j + u * TPS;
    if (k > NT / 2 || (u == R / 2 && j != 0)) continue;
    const int kp = (NT - k) & (NT - 1);
    const C zk = my[k * S], zp = my[kp * S];
    const C A = abk[2 * k], Bk = abk[2 * k + 1];
    const C Ma = inv_sqrt_principal<T>(C{A.x + ba * Bk.x, A.y + ba * Bk.y});
    const C Mb = inv_sqrt_principal<T>(C{A.x + bb * Bk.x, A.y + bb * Bk.y});
    const C sp = cscale(cadd(Ma, Mb), scale), sm = cscale(csub(Ma, Mb), scale);
    my[k * S] = cadd(cmul(sp, zk), cmul(sm, cconj(zp)));
    if (kp != k) my[kp * S] = cadd(cmul(cconj(sp), zp), cmul(cconj(sm), cconj(zk)));
  }
}

template <typename T, int NT, int WG>
__global__ void __launch_bounds__(WG)
k_time(DevPlan P, int check) {
  using C = cplx<T>;
  constexpr int R = FftShape<NT>::R, TPS = NT / R, S = seqs_of<NT, WG>();
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int b = blockIdx.y;
  if (check && P.st[b].state != ST_RUNNING) return;
  const int s = threadIdx.x % S, j = threadIdx.x / S;
  const int npairs = P.ms / 2;
  const int pair = blockIdx.x * S + s;
  const bool valid = pair < npairs;
  const int ld = npairs;
  C* g = reinterpret_cast<C*>(reinterpret_cast<T*>(P.scratch) + (size_t)b * P.NS) + pair;
  const T* __restrict__ sc = reinterpret_cast<const T*>(P.sc);
  const T* __restrict__ sci = reinterpret_cast<const T*>(P.sci);
  const C* __restrict__ abk = reinterpret_cast<const C*>(P.abk);
  const C* __restrict__ tw = reinterpret_cast<const C*>(P.twt);
  const T* __restrict__ beta = reinterpret_cast<const T*>(P.beta);
  const T ba = valid ? beta[2 * pair] : (T)1;
  const T bb = valid ? beta[2 * pair + 1] : (T)1;
  C* my = lds + s;
  C v[R];
  // Y then D: e_t = a^t g_{nt-1-t}
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int t = j + i * TPS;
    const C z = valid ? g[(size_t)(NT - 1 - t) * ld] : C{0, 0};
    v[i] = cscale(z, sc[t]);
  }
  const T half_inv_n = (T)(0.5 / NT);
#pragma unroll 1
  for (int rep = 0; rep < 2; ++rep) {
    fft_seq<T, NT, false>(v, j, my, S, tw);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) my[(j + i * TPS) * S] = v[i];
    __syncthreads();
    spectral_pairs<T, NT>(my, S, j, abk, ba, bb, half_inv_n);
    __syncthreads();
    fft_seq<T, NT, true, true>(v, j, my, S, tw);
    if (rep == 0) {
      // D^{-1}, then Y, then D:  h_t = a^{2t-nt+1} c_{nt-1-t}
      __syncthreads();
#pragma unroll
      for (int i = 0; i < R; ++i) my[(j + i * TPS) * S] = v[i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int t = j + i * TPS;
        v[i] = cscale(my[(NT - 1 - t) * S], sc[t] * sci[NT - 1 - t]);
      }
      __syncthreads();
    }
  }
  if (!valid) return;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int t = j + i * TPS;
    g[(size_t)t * ld] = cscale(v[i], sci[t]);
  }
}

// ---------------------------------------------------------------------------
// last pass: inverse DST-I along x (transform precision in, FP64 out), optionally
// fused with the partial sums of <q, p>.
// ---------------------------------------------------------------------------
template <typename T, int L, int WG>
__global__ void __launch_bounds__(WG)
k_dstx_inv(DevPlan P, int mode, double* __restrict__ outp) {
  using C = cplx<T>;
  constexpr int R = FftShape<L>::R, TPS = L / R, S = seqs_of<L, WG>(), Mx = L / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  T* stage = reinterpret_cast<T*>(smem);
  double* ostage = reinterpret_cast<double*>(smem);
  const int b = blockIdx.y;
  const size_t off = (size_t)b * P.N;
  double* out = outp ? outp + off : nullptr;
  const double* q = nullptr;
  const MinresState* st = P.st + b;
  if (mode != INV_PLAIN) {
    if (st->state != ST_RUNNING) return;
    if (mode == INV_GAMMA_INIT) {
      out = P.Z[1] + off;
      q = P.V[1] + off;
    } else {
      const int jj = st->iter + 1;
      out = P.Z[(jj + 1) & 1] + off;
      q = P.V[(jj + 1) % 3] + off;
    }
  }
  const int nx = P.nx;
  const int rows = P.nt * P.ny1;
  const int row0 = blockIdx.x * 2 * S;
  const int nrows = min(2 * S, rows - row0);
  const T* scr = reinterpret_cast<const T*>(P.scratch) + (size_t)b * P.NS + (size_t)row0 * Mx;
  const int cnt = nrows * Mx;
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) stage[e] = scr[e];
  __syncthreads();
  const int s = threadIdx.x % S, j = threadIdx.x / S;
  const int ra = 2 * s, rb = 2 * s + 1;
  const bool va = ra < nrows, vb = rb < nrows;
  C v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int t = j + i * TPS;
    T a = 0, c = 0;
    if (t > 0 && t < Mx) {
      if (va) a = stage[ra * Mx + t - 1];
      if (vb) c = stage[rb * Mx + t - 1];
    } else if (t > Mx) {
      const int idx = 2 * Mx - t - 1;
      if (va) a = -stage[ra * Mx + idx];
      if (vb) c = -stage[rb * Mx + idx];
    }
    v[i] = C{a, c};
  }
  __syncthreads();
  fft_seq<T, L, false>(v, j, lds + s, S, reinterpret_cast<const C*>(P.twx));
  const double scl = 1.0 / sqrt((double)L);
  // stage the FP64 rows ([2S][nx+2] padded: odd stride in 8-byte words) and write
  // them out contiguously; with q, accumulate <q, p> in a fixed order for a fixed tile
  __syncthreads();
  const int ldo = nx + 2;
#pragma unroll
  for (int i = 0; i <= R / 2; ++i) {
    const int k = j + i * TPS;
    if (k == 0 || k >= Mx) continue;
    ostage[ra * ldo + k - 1] = -(double)v[i].y * scl;
    ostage[rb * ldo + k - 1] = (double)v[i].x * scl;
  }
  __syncthreads();
  double* o = out + (size_t)row0 * nx;
  const int total = nrows * nx;
  double acc = 0.0;
  {
    const double* qq = q ? q + (size_t)row0 * nx : nullptr;
    int e = threadIdx.x;
    int r = e / nx, c = e - r * nx;
    const int dr = blockDim.x / nx, dc = blockDim.x - dr * nx;
    for (; e < total; e += blockDim.x) {
      const double val = ostage[r * ldo + c];
      o[e] = val;
      if (qq) acc += val * qq[e];
      r += dr;
      c += dc;
      if (c >= nx) {
        c -= nx;
        ++r;
      }
    }
  }
  if (mode == INV_PLAIN) return;
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_GAMMA, b)[blockIdx.x] = bs;
}

// ---------------------------------------------------------------------------
// launchers: one instantiation per (precision, length, workgroup size)
// ---------------------------------------------------------------------------
template <typename T, int L, int WG>
hipError_t launch_x_fwd_t(const DevPlan& P, int mode, int check, const double* in, hipStream_t s) {
  if constexpr (!tile_ok<T, L, WG>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int S = seqs_of<L, WG>();
    const int rows = P.nt * P.ny1;
    dim3 grid((rows + 2 * S - 1) / (2 * S), P.B);
    const size_t lds = (size_t)S * L * sizeof(cplx<T>);
    hipLaunchKernelGGL((k_dstx_fwd<T, L, WG>), grid, dim3(WG), lds, s, P, mode, check, in);
    return hipGetLastError();
  }
}

template <typename T, int L, int WG>
hipError_t launch_x_inv_t(const DevPlan& P, int mode, double* out, hipStream_t s) {
  if constexpr (!tile_ok<T, L, WG>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int S = seqs_of<L, WG>();
    const int rows = P.nt * P.ny1;
    dim3 grid((rows + 2 * S - 1) / (2 * S), P.B);
    const size_t lds = std::max((size_t)S * L * sizeof(cplx<T>), (size_t)2 * S * (L / 2 + 1) * sizeof(double));
    hipLaunchKernelGGL((k_dstx_inv<T, L, WG>), grid, dim3(WG), lds, s, P, mode, out);
    return hipGetLastError();
  }
}

template <typename T, int L, int WG>
hipError_t launch_y_t(const DevPlan& P, int check, hipStream_t s) {
  if constexpr (!tile_ok<T, L, WG>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int S = seqs_of<L, WG>();
    const int cpairs = P.Mx / 2;
    const int bpl = (cpairs + S - 1) / S;
    dim3 grid(bpl * P.nt, P.B);
    const size_t lds = (size_t)S * L * sizeof(cplx<T>);
    hipLaunchKernelGGL((k_dsty<T, L, WG>), grid, dim3(WG), lds, s, P, check);
    return hipGetLastError();
  }
}

template <typename T, int NT, int WG>
hipError_t launch_time_t(const DevPlan& P, int check, hipStream_t s) {
  if constexpr (!tile_ok<T, NT, WG>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int S = seqs_of<NT, WG>();
    const int npairs = P.ms / 2;
    dim3 grid((npairs + S - 1) / S, P.B);
    const size_t lds = (size_t)S * NT * sizeof(cplx<T>);
    hipLaunchKernelGGL((k_time<T, NT, WG>), grid, dim3(WG), lds, s, P, check);
    return hipGetLastError();
  }
}

#define ABAC_SWITCH_WG(WGVAR, CALL, LL)      \
  switch (WGVAR) {                           \
    case 64: return CALL(LL, 64);            \
    case 128: return CALL(LL, 128);          \
    case 256: return CALL(LL, 256);          \
    case 512: return CALL(LL, 512);          \
    case 1024: return CALL(LL, 1024);        \
    default: return hipErrorInvalidValue;    \
  }

#define ABAC_SWITCH_L(LVAR, WGVAR, CALL)                                           \
  switch (LVAR) {                                                                  \
    case 8: ABAC_SWITCH_WG(WGVAR, CALL, 8)                                         \
    case 16: ABAC_SWITCH_WG(WGVAR, CALL, 16)                                       \
    case 32: ABAC_SWITCH_WG(WGVAR, CALL, 32)                                       \
    case 64: ABAC_SWITCH_WG(WGVAR, CALL, 64)                                       \
    case 128: ABAC_SWITCH_WG(WGVAR, CALL, 128)                                     \
    case 256: ABAC_SWITCH_WG(WGVAR, CALL, 256)                                     \
    case 512: ABAC_SWITCH_WG(WGVAR, CALL, 512)                                     \
    case 1024: ABAC_SWITCH_WG(WGVAR, CALL, 1024)                                   \
    case 2048: ABAC_SWITCH_WG(WGVAR, CALL, 2048)                                   \
    case 4096: ABAC_SWITCH_WG(WGVAR, CALL, 4096)                                   \
    case 8192: ABAC_SWITCH_WG(WGVAR, CALL, 8192)                                   \
    default: return hipErrorInvalidValue;                                          \
  }

template <typename T>
hipError_t x_fwd_dispatch(const DevPlan& P, int mode, int check, const double* in, hipStream_t s) {
#define CALL(LL, WW) launch_x_fwd_t<T, LL, WW>(P, mode, check, in, s)
  ABAC_SWITCH_L(2 * P.Mx, P.wg_x, CALL)
#undef CALL
}

template <typename T>
hipError_t x_inv_dispatch(const DevPlan& P, int mode, double* out, hipStream_t s) {
#define CALL(LL, WW) launch_x_inv_t<T, LL, WW>(P, mode, out, s)
  ABAC_SWITCH_L(2 * P.Mx, P.wg_xi, CALL)
#undef CALL
}

template <typename T>
hipError_t y_dispatch(const DevPlan& P, int check, hipStream_t s) {
#define CALL(LL, WW) launch_y_t<T, LL, WW>(P, check, s)
  ABAC_SWITCH_L(2 * P.My, P.wg_y, CALL)
#undef CALL
}

template <typename T>
hipError_t time_dispatch(const DevPlan& P, int check, hipStream_t s) {
#define CALL(LL, WW) launch_time_t<T, LL, WW>(P, check, s)
  ABAC_SWITCH_L(P.nt, P.wg_t, CALL)
#undef CALL
}

template <typename T> hipError_t tile_check_t(int L, int wg) {
#define CALL(LL, WW) (tile_ok<T, LL, WW>() ? hipSuccess : hipErrorInvalidValue)
  ABAC_SWITCH_L(L, wg, CALL)
#undef CALL
}

}  // namespace

hipError_t launch_dstx_fwd(const DevPlan& P, int prec, int mode, int check, const double* in, hipStream_t s) {
  return prec ? x_fwd_dispatch<float>(P, mode, check, in, s) : x_fwd_dispatch<double>(P, mode, check, in, s);
}

hipError_t launch_dsty(const DevPlan& P, int prec, int check, hipStream_t s) {
  return prec ? y_dispatch<float>(P, check, s) : y_dispatch<double>(P, check, s);
}

hipError_t launch_time(const DevPlan& P, int prec, int check, hipStream_t s) {
  return prec ? time_dispatch<float>(P, check, s) : time_dispatch<double>(P, check, s);
}

hipError_t launch_dstx_inv(const DevPlan& P, int prec, int mode, double* out, hipStream_t s) {
  return prec ? x_inv_dispatch<float>(P, mode, out, s) : x_inv_dispatch<double>(P, mode, out, s);
}

bool transform_tile_valid(int L, int wg, int prec) {
  return (prec ? tile_check_t<float>(L, wg) : tile_check_t<double>(L, wg)) == hipSuccess;
}

int transform_tps(int L) {
  switch (L) {
    case 8: return fft_tps<8>();
    case 16: return fft_tps<16>();
    case 32: return fft_tps<32>();
    case 64: return fft_tps<64>();
    case 128: return fft_tps<128>();
    case 256: return fft_tps<256>();
    case 512: return fft_tps<512>();
    case 1024: return fft_tps<1024>();
    case 2048: return fft_tps<2048>();
    case 4096: return fft_tps<4096>();
    case 8192: return fft_tps<8192>();
    default: return 0;
  }
}

int dstx_blocks(const DevPlan& P, int wg) {
  const int S = wg / transform_tps(2 * P.Mx);
  const int rows = P.nt * P.ny1;
  return (rows + 2 * S - 1) / (2 * S);
}

size_t transform_lds_bytes(int L, int wg, int prec) {
  const size_t c = prec ? sizeof(float2) : sizeof(double2);
  return (size_t)(wg / transform_tps(L)) * L * c;
}

}  // namespace abac

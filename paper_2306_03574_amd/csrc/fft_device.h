// Device FFT building blocks for gfx950 (CDNA4): register-resident radix-2/4/8/16
// butterflies and a Stockham autosort driver whose intermediate exchanges go through
// LDS.  Power-of-two lengths 4..8192.  Complex values are HIP vector types
// (double2 / float2).
//
// Register layout contract (same on input and output): a sequence of length L is
// held by TPS = L/R threads; thread j holds elements j + i*TPS, i = 0..R-1, where R
// is the outer radix of the length.  Many sequences share one workgroup; their LDS
// storage is interleaved (element e of sequence s at lds[e*S + s]) so that threads
// with consecutive s touch consecutive LDS addresses.
#pragma once
#include <hip/hip_runtime.h>

namespace abac {

template <typename T> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };
template <typename T> using cplx = typename cplx_of<T>::type;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return C{a.x, -a.y}; }
template <typename C, typename T> __device__ __forceinline__ C cscale(C a, T s) { return C{a.x * s, a.y * s}; }

// multiply by exp(-i pi/2) = -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C rot90(C a) {
  return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}

// multiply by exp(-+ 2 pi i e / 16) for a compile-time e (forward sign -, inverse +)
template <bool INV, int E, typename C> __device__ __forceinline__ C tw16(C a) {
  using T = decltype(a.x);
  constexpr int e = E & 15;
  if constexpr (e == 0) return a;
  else if constexpr (e == 4) return rot90<INV>(a);
  else if constexpr (e == 8) return C{-a.x, -a.y};
  else if constexpr (e == 12) return rot90<!INV>(a);
  else {
    // cos/sin of 2 pi e/16 for e in 1..15, exact to double rounding
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
    constexpr double c2 = 0.70710678118654752440;
    constexpr double cs[16] = {1, c1, c2, s1, 0, -s1, -c2, -c1, -1, -c1, -c2, -s1, 0, s1, c2, c1};
    constexpr double sn[16] = {0, s1, c2, c1, 1, c1, c2, s1, 0, -s1, -c2, -c1, -1, -c1, -c2, -s1};
    const T c = (T)cs[e];
    const T s = INV ? (T)sn[e] : (T)(-sn[e]);
    return C{a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

// In-register DFTs, natural order in and out: u[k] <- sum_n u[n] W^{nk}.
template <bool INV, typename C> __device__ __forceinline__ void dft2(C* u) {
  C t = u[0];
  u[0] = cadd(t, u[1]);
  u[1] = csub(t, u[1]);
}

template <bool INV, typename C> __device__ __forceinline__ void dft4s(C& u0, C& u1, C& u2, C& u3) {
  C t0 = cadd(u0, u2), t1 = csub(u0, u2), t2 = cadd(u1, u3), t3 = rot90<INV>(csub(u1, u3));
  u0 = cadd(t0, t2);
  u2 = csub(t0, t2);
  u1 = cadd(t1, t3);
  u3 = csub(t1, t3);
}

template <bool INV, typename C> __device__ __forceinline__ void dft4(C* u) { dft4s<INV>(u[0], u[1], u[2], u[3]); }

template <bool INV, typename C> __device__ __forceinline__ void dft8(C* u) {
  // decimation in time: even / odd halves
  C e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6];
  C o0 = u[1], o1 = u[3], o2 = u[5], o3 = u[7];
  dft4s<INV>(e0, e1, e2, e3);
  dft4s<INV>(o0, o1, o2, o3);
  o1 = tw16<INV, 2>(o1);
  o2 = tw16<INV, 4>(o2);
  o3 = tw16<INV, 6>(o3);
  u[0] = cadd(e0, o0); u[4] = csub(e0, o0);
  u[1] = cadd(e1, o1); u[5] = csub(e1, o1);
  u[2] = cadd(e2, o2); u[6] = csub(e2, o2);
  u[3] = cadd(e3, o3); u[7] = csub(e3, o3);
}

template <bool INV, typename C> __device__ __forceinline__ void dft16(C* u) {
  // 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
  C a[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    C x0 = u[n2], x1 = u[n2 + 4], x2 = u[n2 + 8], x3 = u[n2 + 12];
    dft4s<INV>(x0, x1, x2, x3);   // x_k1 for this n2
    a[4 * n2 + 0] = x0;
    a[4 * n2 + 1] = x1;
    a[4 * n2 + 2] = x2;
    a[4 * n2 + 3] = x3;
  }
  // twiddles W16^{n2 k1}
  a[5] = tw16<INV, 1>(a[5]);  a[6] = tw16<INV, 2>(a[6]);  a[7] = tw16<INV, 3>(a[7]);
  a[9] = tw16<INV, 2>(a[9]);  a[10] = tw16<INV, 4>(a[10]); a[11] = tw16<INV, 6>(a[11]);
  a[13] = tw16<INV, 3>(a[13]); a[14] = tw16<INV, 6>(a[14]); a[15] = tw16<INV, 9>(a[15]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C y0 = a[k1], y1 = a[4 + k1], y2 = a[8 + k1], y3 = a[12 + k1];
    dft4s<INV>(y0, y1, y2, y3);   // over n2 -> k2
    u[k1 + 0] = y0;
    u[k1 + 4] = y1;
    u[k1 + 8] = y2;
    u[k1 + 12] = y3;
  }
}

template <int R, bool INV, typename C> __device__ __forceinline__ void dftR(C* u) {
  if constexpr (R == 2) dft2<INV>(u);
  else if constexpr (R == 4) dft4<INV>(u);
  else if constexpr (R == 8) dft8<INV>(u);
  else if constexpr (R == 16) dft16<INV>(u);
  else static_assert(R == 2, "unsupported radix");
}

// Factorisation of each supported length: outer radix R (first and last pass) and
// up to two middle radices (0 = absent).  Middle radices divide R.
template <int L> struct FftShapeDefault;
#define ABAC_FFT_SHAPE(LL, RR, M1, M2) \
  template <> struct FftShapeDefault<LL> { static constexpr int R = RR, m1 = M1, m2 = M2; \
    static constexpr int passes = (LL == RR) ? 1 : 2 + (M1 ? 1 : 0) + (M2 ? 1 : 0); };
ABAC_FFT_SHAPE(4, 4, 0, 0)
ABAC_FFT_SHAPE(8, 8, 0, 0)
ABAC_FFT_SHAPE(16, 4, 0, 0)
ABAC_FFT_SHAPE(32, 4, 2, 0)
ABAC_FFT_SHAPE(64, 8, 0, 0)
ABAC_FFT_SHAPE(128, 8, 2, 0)
ABAC_FFT_SHAPE(256, 16, 0, 0)
ABAC_FFT_SHAPE(512, 8, 8, 0)
ABAC_FFT_SHAPE(1024, 16, 4, 0)
ABAC_FFT_SHAPE(2048, 16, 8, 0)
ABAC_FFT_SHAPE(4096, 16, 16, 0)
ABAC_FFT_SHAPE(8192, 16, 2, 16)
#undef ABAC_FFT_SHAPE

// The factorisation per precision.  FP64 values take twice the registers of FP32 ones,
// so FP64 passes favour radix 8 (more threads per sequence, higher occupancy) and FP32
// passes radix 16 (fewer exchanges through LDS): 512 = 16 x 2 x 16 in FP32, and
// 256 = 8 x 4 x 8 and 1024 = 8 x 4 x 4 x 8 in FP64, differ from the shared table.
template <typename T, int L> struct FftShape : FftShapeDefault<L> {};
template <> struct FftShape<float, 512> {
  static constexpr int R = 16, m1 = 2, m2 = 0, passes = 3;
};
template <> struct FftShape<double, 256> {
  static constexpr int R = 8, m1 = 4, m2 = 0, passes = 3;
};
template <> struct FftShape<double, 1024> {
  static constexpr int R = 8, m1 = 4, m2 = 4, passes = 4;
};

template <typename T, int L> constexpr int fft_tps() { return L / FftShape<T, L>::R; }

// One Stockham (decimation in time, autosort) pass of radix r over a length-L
// sequence, for the butterflies owned by this thread.  Butterfly b reads elements
// b + i*(L/r), multiplies element i by W_{Ns r}^{i (b mod Ns)}, applies a radix-r
// DFT and writes element i to position (b/Ns)*Ns*r + (b mod Ns) + i*Ns.
// The twiddle table holds tw[e] = exp(-2 pi i e / L), e = 0..L-1.
template <typename C, int L, int r, bool INV>
__device__ __forceinline__ void stockham_twiddle(C* u, int b, int Ns, const C* __restrict__ tw) {
  if (Ns == 1) return;
  const int k = b % Ns;
  const int step = (L / (Ns * r)) * k;
#pragma unroll
  for (int i = 1; i < r; ++i) {
    C w = tw[i * step];
    if (INV) w.y = -w.y;
    u[i] = cmul(u[i], w);
  }
}

template <typename C, int L, int r>
__device__ __forceinline__ int stockham_dst(int b, int Ns, int i) {
  return (b / Ns) * Ns * r + (b % Ns) + i * Ns;
}

// Full FFT of one sequence held in registers (v[i] = x[j + i*TPS]); on return
// v[i] = X[j + i*TPS].  All threads of the workgroup must call it together.  The
// LDS region lds[e*S] (e < L) must be free on entry (the caller puts a barrier
// between its last LDS reads and this call); on return other threads may still be
// reading it, so the caller must barrier before writing it again.  With FROM_LDS the
// input is read from lds[e*S] in natural order instead (the caller barriers after
// writing it).
template <typename T, int L, bool INV, bool FROM_LDS = false>
__device__ __forceinline__ void fft_seq(cplx<T>* v, int j, cplx<T>* lds, int S, const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using Sh = FftShape<T, L>;
  constexpr int R = Sh::R;
  constexpr int TPS = L / R;
  if constexpr (FROM_LDS) {
    // input in natural order in LDS (written and fenced by the caller)
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = lds[(j + i * TPS) * S];
    __syncthreads();
  }
  // pass 0: radix R, Ns = 1
  dftR<R, INV>(v);
  if constexpr (Sh::passes == 1) {
    return;
  } else {
    int Ns = 1;
#pragma unroll
    for (int i = 0; i < R; ++i) lds[stockham_dst<C, L, R>(j, Ns, i) * S] = v[i];
    Ns *= R;
    __syncthreads();
    // middle passes
    if constexpr (Sh::m1 != 0) {
      constexpr int r = Sh::m1;
      constexpr int NB = R / r;   // butterflies per thread
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = u * TPS + j;
#pragma unroll
        for (int i = 0; i < r; ++i) v[u * r + i] = lds[(b + i * (L / r)) * S];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = u * TPS + j;
        stockham_twiddle<C, L, r, INV>(v + u * r, b, Ns, tw);
        dftR<r, INV>(v + u * r);
#pragma unroll
        for (int i = 0; i < r; ++i) lds[stockham_dst<C, L, r>(b, Ns, i) * S] = v[u * r + i];
      }
      Ns *= r;
      __syncthreads();
    }
    if constexpr (Sh::m2 != 0) {
      constexpr int r = Sh::m2;
      constexpr int NB = R / r;
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = u * TPS + j;
#pragma unroll
        for (int i = 0; i < r; ++i) v[u * r + i] = lds[(b + i * (L / r)) * S];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = u * TPS + j;
        stockham_twiddle<C, L, r, INV>(v + u * r, b, Ns, tw);
        dftR<r, INV>(v + u * r);
#pragma unroll
        for (int i = 0; i < r; ++i) lds[stockham_dst<C, L, r>(b, Ns, i) * S] = v[u * r + i];
      }
      Ns *= r;
      __syncthreads();
    }
    // last pass: radix R, butterfly b = j, output lands at j + i*Ns with Ns = TPS
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = lds[(j + i * TPS) * S];
    stockham_twiddle<C, L, R, INV>(v, j, Ns, tw);
    dftR<R, INV>(v);
  }
}

}  // namespace abac

// Seeded synthetic sources generated on the device: i.i.d. N(0,1) values from the
// counter-based Philox4x32-10 generator (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC 2011) followed by the Box-Muller transform.
// Element e uses counter (e/4, 0, 0, 0) and key (seed_lo, seed_hi); the four 32-bit
// words u_i map to uniforms (u_i + 0.5) 2^-32 and pairs (0,1), (2,3) to normals
// sqrt(-2 ln U0) (cos 2 pi U1, sin 2 pi U1).  Input generation only: no solver arithmetic.
#include "abac_internal.h"

namespace abac {

namespace {

struct U4 {
  unsigned x, y, z, w;
};

__device__ __forceinline__ void mulhilo(unsigned a, unsigned b, unsigned& hi, unsigned& lo) {
  const unsigned long long p = (unsigned long long)a * b;
  hi = (unsigned)(p >> 32);
  lo = (unsigned)p;
}

__device__ __forceinline__ U4 philox4x32_10(U4 c, unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    unsigned hi0, lo0, hi1, lo1;
    mulhilo(0xD2511F53u, c.x, hi0, lo0);
    mulhilo(0xCD9E8D57u, c.z, hi1, lo1);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

__global__ void k_fill_normal(double* __restrict__ out, unsigned long long n, unsigned long long seed) {
  const unsigned k0 = (unsigned)seed, k1 = (unsigned)(seed >> 32);
  const unsigned long long nblk = (n + 3) / 4;
  for (unsigned long long q = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; q < nblk;
       q += (unsigned long long)gridDim.x * blockDim.x) {
    const U4 r = philox4x32_10(U4{(unsigned)q, (unsigned)(q >> 32), 0u, 0u}, k0, k1);
    const double s = 2.3283064365386963e-10;  // 2^-32
    const double u0 = ((double)r.x + 0.5) * s, u1 = ((double)r.y + 0.5) * s;
    const double u2 = ((double)r.z + 0.5) * s, u3 = ((double)r.w + 0.5) * s;
    const double a = sqrt(-2.0 * log(u0)), c = sqrt(-2.0 * log(u2));
    const double two_pi = 6.283185307179586477;
    double v[4] = {a * cos(two_pi * u1), a * sin(two_pi * u1), c * cos(two_pi * u3), c * sin(two_pi * u3)};
    const unsigned long long e0 = q * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (e0 + i < n) out[e0 + i] = v[i];
  }
}

__global__ void k_fill_zero(double* __restrict__ out, unsigned long long n) {
  for (unsigned long long e = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (unsigned long long)gridDim.x * blockDim.x)
    out[e] = 0.0;
}

}  // namespace

hipError_t launch_fill_normal(double* out, unsigned long long n, unsigned long long seed, hipStream_t s) {
  unsigned long long blocks = ((n + 3) / 4 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_normal, dim3((unsigned)blocks), dim3(256), 0, s, out, n, seed);
  return hipGetLastError();
}

hipError_t launch_fill_zero(double* out, unsigned long long n, hipStream_t s) {
  unsigned long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, out, n);
  return hipGetLastError();
}

}  // namespace abac

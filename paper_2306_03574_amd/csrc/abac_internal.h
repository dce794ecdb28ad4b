// Internal definitions shared by the HIP translation units of the ABAC library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_device.h"

namespace abac {

// Solve state of one right-hand side, resident in device memory.  Every scalar of
// the MINRES recurrence lives here; kernels read what they need at entry and the
// last block of a reduction writes the new values.
enum : int { ST_IDLE = 0, ST_RUNNING = 1, ST_DONE = 2 };

struct MinresState {
  double gamma;     // gamma_j, current Lanczos off-diagonal
  double sig;       // 1/gamma_j: scale of the stored (unnormalised) v_j and z_j
  double sig_prev;  // 1/gamma_{j-1}: scale of the stored v_{j-1} (0 at j = 1)
  double delta;     // delta_j = <A z_j, z_j>
  double c1, c2;    // Givens cosines c_{j-1}, c_{j-2}
  double s1, s2;    // Givens sines s_{j-1}, s_{j-2}
  double eta;       // running right-hand side of the rotated least-squares problem
  double wa, wb, wc;  // w_j = wa * Zslot_j - wb * w_{j-1} - wc * w_{j-2}
  double xc;        // x_j = x_{j-1} + xc * w_j
  double r1, r2;    // r_j = r1 * r_{j-1} + r2 * Vslot_{j+1}
  double rnorm2;    // ||r_j||^2 from the recurrence
  double bnorm2;    // ||b||^2
  double tol2;      // tol^2
  double res2;      // last explicit ||b - A x||^2
  int iter;         // completed iterations
  int maxit;
  int state;        // ST_*
  int status;       // abac_status of this right-hand side
  int explicit_mode;
  int need_check;
  int pad0, pad1;
};

// Everything a kernel needs about a plan, passed by value.
struct DevPlan {
  int nx, ny, nt, B;   // ny = 0 in 1D
  int ny1;             // max(ny, 1): rows per level
  int Mx, My;          // nx+1, ny+1 (My = 1 in 1D)
  int m;               // nx * ny1: unknowns per level
  int ms;              // Mx * ny1: scratch modes per level (one zero pad column)
  int pad_;
  long long N;         // nt * m: unknowns per right-hand side
  long long NS;        // nt * ms: scratch values per right-hand side
  double c0, cx, cy;   // (L s)_i = c0 s_i - cx (s_{i-1} + s_{i+1}) - cy (s_{i-nx} + s_{i+nx})
  double tau, tau2;
  // spectral tables, stored in the transform precision
  const void* twx;     // 2*Mx complex twiddles exp(-2 pi i e/(2 Mx))
  const void* twy;     // 2*My complex twiddles (2D)
  const void* twt;     // nt complex twiddles exp(-2 pi i e/nt)
  const void* beta;    // ms real: (tau^2/2) * eigenvalue of -Laplace_h of each scratch mode
  const void* abk;     // 2*nt complex: (A_k, B_k), mu_k(beta) = A_k + beta * B_k
  const void* sc;      // nt real: a^t,  a = alpha^{1/nt}
  const void* sci;     // nt real: a^{-t}
  void* scratch;       // B * NS transform values
  // MINRES vectors, each B * N doubles
  double* V[3];
  double* Z[2];
  double* W[2];
  double* R;
  MinresState* st;     // B entries
  double* partials;    // B * maxparts
  unsigned* counters;  // B entries
  int maxparts;
  int pad2_;
};

// ---------------------------------------------------------------------------
// deterministic reductions: fixed-order block sums, partials per block, and a
// last-block-done finalisation that sums the partials in index order.
// ---------------------------------------------------------------------------

// Sum of v over the block; the result is valid in thread 0.  Ends with a barrier so
// the shared buffer can be reused.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red_ws[16];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red_ws[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red_ws[i];
  }
  __syncthreads();
  return s;
}

// Publish this block's partial for right-hand side b and report whether the block
// is the last of the nblocks contributing ones.  Uniform result across the block.
__device__ __forceinline__ bool arrive_last(const DevPlan& P, int b, int blk, int nblocks, double partial) {
  __shared__ int amlast;
  if (threadIdx.x == 0) {
    P.partials[(size_t)b * P.maxparts + blk] = partial;
    __threadfence();
    const unsigned t = atomicAdd(P.counters + b, 1u);
    amlast = (t == (unsigned)(nblocks - 1));
  }
  __syncthreads();
  const bool last = amlast != 0;
  if (last) __threadfence();
  return last;
}

// In the last block: fixed-order sum of the nblocks partials (result in thread 0),
// and the counter reset for the next reduction.
__device__ __forceinline__ double finish_sum(const DevPlan& P, int b, int nblocks) {
  const volatile double* part = P.partials + (size_t)b * P.maxparts;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) s += part[i];
  s = block_sum(s);
  if (threadIdx.x == 0) {
    atomicExch(P.counters + b, 0u);
  }
  return s;
}

// Workgroups are dispatched round-robin over the 8 XCDs; remap the hardware block
// index so each XCD receives a contiguous range of logical blocks (shared halo
// rows then hit the same L2).
__device__ __forceinline__ int xcd_remap(int w, int n) {
  const int q = n >> 3, rem = n & 7;
  const int x = w & 7, slot = w >> 3;
  return x * q + (x < rem ? x : rem) + slot;
}

// ---------------------------------------------------------------------------
// host-side launchers (defined in the kernel translation units)
// ---------------------------------------------------------------------------
enum StencilMode : int { STENCIL_PLAIN = 0, STENCIL_MINRES = 1, STENCIL_RESIDUAL = 2, STENCIL_REPORT = 3 };
enum FwdMode : int { FWD_PLAIN = 0, FWD_LANCZOS = 1 };
enum InvMode : int { INV_PLAIN = 0, INV_GAMMA_INIT = 1, INV_GAMMA_ITER = 2 };

int stencil_blocks(const DevPlan& P);
int update_blocks(const DevPlan& P);
int dstx_blocks(const DevPlan& P, int prec);

hipError_t launch_stencil(const DevPlan& P, int mode, const double* x, double* y, const double* f, hipStream_t s);
hipError_t launch_rhs(const DevPlan& P, const double* src, const double* psi0, const double* psi1, double* f,
                      hipStream_t s);
hipError_t launch_init(const DevPlan& P, const double* f, double* u, double tol, int maxit, hipStream_t s);
hipError_t launch_update(const DevPlan& P, double* u, hipStream_t s);

// check != 0: skip right-hand sides whose solve is not running
hipError_t launch_dstx_fwd(const DevPlan& P, int prec, int mode, int check, const double* in, hipStream_t s);
hipError_t launch_dsty(const DevPlan& P, int prec, int check, hipStream_t s);
hipError_t launch_time(const DevPlan& P, int prec, int check, hipStream_t s);
hipError_t launch_dstx_inv(const DevPlan& P, int prec, int mode, double* out, hipStream_t s);
size_t transform_lds_bytes(int L, int prec);

}  // namespace abac

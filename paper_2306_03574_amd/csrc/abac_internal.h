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
constexpr int kSnapRing = 16;   // host snapshot slots per right-hand side
constexpr size_t kMaxTransformLds = 152 * 1024;   // dynamic LDS per transform block (gfx950: 160 KB per workgroup, 8 KB kept for static LDS)

// Resident Krylov basis: z_1 .. z_kBasis each keep a slot of their own, and the
// iterate is formed from them (x_j = sum_l y_l z_l) only when a residual check, a
// breakdown or the end of the solve needs it, so an iteration updates just the
// residual vector.  From z_{kBasis+1} on, z alternates between two more slots and
// w and x follow the classic three-term recurrences (after one flush that forms x,
// w_kBasis and w_{kBasis-1} from the basis).
constexpr int kBasis = 12;
constexpr int kZSlots = kBasis + 2;
__host__ __device__ inline int zslot(int j) { return j <= kBasis ? j - 1 : kBasis + (j & 1); }

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
  int need_check;   // set by the form kernel: confirm convergence explicitly
  int lucky;        // gamma_{j+1} == 0: the Krylov space is invariant
  int snap;         // sequence number of the next host snapshot
  int nbasis;       // basis slots with coefficients (basis phase)
  int basis_dirty;  // u does not yet hold the iterate of the basis coefficients
  int form_now;     // this iteration forms u from the basis (flush: also w_j, w_{j-1})
  int flush_now;
};

// vector kernels: 256 threads, about 16 elements per thread, at most 1024 blocks per
// right-hand side (update_blocks)
constexpr int kVecThreads = 256;
constexpr int kVecPerThread = 16;
constexpr int kVecMaxBlocks = 1024;

// Restarted GMRES (right preconditioning with C_alpha^{-1}) on T u = f: per right-hand
// side state.  The Arnoldi basis v_0 .. v_restart lives in the plan's Krylov vector
// slots (so restart <= kGmresMax), H is the rotated Hessenberg matrix, column-major.
constexpr int kGmresMax = 15;
struct GmresState {
  double H[(kGmresMax + 1) * kGmresMax];   // H[c * (kGmresMax + 1) + l]: row l, column c
  double cs[kGmresMax], sn[kGmresMax];     // Givens rotations
  double g[kGmresMax + 1];                 // rotated beta e_1
  double y[kGmresMax];                     // least-squares solution (when forming u)
  double h1[kGmresMax + 1], h2[kGmresMax + 1];   // the two Gram-Schmidt passes of a column
  double sig[kGmresMax + 1];                 // v_l = sig_l * (slot l): slots hold unnormalised vectors
  double bnorm2, tol2, scale, res2, resid2;
  int iter, k, maxit, restart, state, status, need, explicit_mode, restart_now;
  int reorth;   // the current column needs the second Gram-Schmidt pass
};
// what the host reads after every step
struct GmresFlags {
  int state, need, k, iter;
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
  // variable coefficient a(x) of div(a grad u) (eq. (3.2)); both NULL for a = 1.
  // coef_x: ny1 rows of Mx face weights (tau^2/2) a(x_{i+1/2}, y_j) / hx^2, i = 0..nx;
  // coef_y (2D): My rows of nx face weights (tau^2/2) a(x_i, y_{j+1/2}) / hy^2, j = 0..ny.
  const double* coef_x;
  const double* coef_y;
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
  double* Z[kZSlots];  // slot zslot(j) holds the stored z_j
  double* W[2];
  double* kcoef;       // per right-hand side, 3 x kBasis: coefficients of x_j, w_j, w_{j-1} on the basis
  GmresState* gst;     // B entries (GMRES solves)
  GmresFlags* gflags;  // B entries
  double* gparts;      // B x (kGmresMax + 1) x kVecMaxBlocks partial dot products
  double* R;
  MinresState* st;     // B entries
  double* partials;    // PART_KINDS * B * maxparts
  unsigned* counters;  // B entries
  MinresState* host_ring;  // device view of the host-mapped snapshot ring (kSnapRing * B)
  int maxparts;
  // workgroup sizes of the transform kernels (chosen by the plan's autotuner)
  int wg_x, wg_xi, wg_y, wg_t;
  int wg_s;            // fused 2D passes (0: separate x and y passes)
  int small;           // 1: one workgroup per right-hand side runs a whole iteration
  int st_chunk;        // forward time levels per matvec block
  int st_threads;      // threads per matvec block
  int st_cols;         // columns per matvec thread (2, or 1 for a one-column grid)
  int st_rows;         // grid rows per matvec block (1 in 1D)
  int gamma_nparts;    // partial sums of <q, P^{-1} q> per right-hand side
  int prec;            // 0 FP64 transforms, 1 FP32 transforms, 2 no preconditioner
};

// ---------------------------------------------------------------------------
// deterministic reductions: every block of a reducing kernel writes one partial
// (fixed-order block sum) into its own slot; a later kernel sums the slots in index
// order.  Kernel boundaries provide the visibility, so no fences or atomics are used.
// ---------------------------------------------------------------------------
enum PartKind : int { PART_DELTA = 0, PART_GAMMA = 1, PART_RNORM = 2, PART_RES = 3, PART_KINDS = 4 };

__device__ __forceinline__ double* part_slot(const DevPlan& P, int kind, int b) {
  return P.partials + ((size_t)kind * P.B + b) * P.maxparts;
}

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

// Fixed-order sum of n partials by the whole block (pairs per thread, then the block
// tree); result valid in thread 0.  `part` is 16-byte aligned.
__device__ __forceinline__ double sum_parts(const double* __restrict__ part, int n) {
  double s = 0.0;
  const double2* p2 = reinterpret_cast<const double2*>(part);
  const int n2 = n >> 1;
  for (int i = threadIdx.x; i < n2; i += blockDim.x) {
    const double2 v = p2[i];
    s += v.x + v.y;
  }
  if ((n & 1) && threadIdx.x == 0) s += part[n - 1];
  return block_sum(s);
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
// PLAIN: y = Y T x; MINRES: the Lanczos matvec with <Y T z, z>; RESIDUAL: ||f - T u||^2
// when the solve asked for a check; REPORT: ||f - T u||^2 always; T: y = T x (natural
// time order); RESVEC: y = f - T x and its squared norm (partials in PART_RES)
enum StencilMode : int {
  STENCIL_PLAIN = 0, STENCIL_MINRES = 1, STENCIL_RESIDUAL = 2, STENCIL_REPORT = 3, STENCIL_T = 4, STENCIL_RESVEC = 5
};
enum FwdMode : int { FWD_PLAIN = 0, FWD_LANCZOS = 1 };
// last pass: INV_PLAIN writes out; the MINRES set-up (INIT) and iteration (ITER) modes
// write z_1 / z_{j+1} into its basis slot, with (GAMMA) or without (Z: the time pass
// forms <q, P^{-1} q>) the partial sums of <q, p>
enum InvMode : int { INV_PLAIN = 0, INV_GAMMA_INIT = 1, INV_GAMMA_ITER = 2, INV_Z_INIT = 3, INV_Z_ITER = 4 };
enum FinKind : int {
  FIN_BNORM = 0, FIN_DELTA = 1, FIN_GAMMA_INIT = 2, FIN_GAMMA_ITER = 3, FIN_RES = 4, FIN_REPORT = 5,
  FIN_RNORM = 6,   // stopping test on the recurrence residual; decides forming u
  FIN_FINAL = 7    // end of a solve: form u if it is stale
};

// matvec decomposition: a block covers a band of st_rows grid rows times
// st_threads * st_cols columns, and st_chunk forward time levels (plus their mirrors)
// two doubles moved by one 16-byte access; 8-byte alignment suffices on gfx950 (rows of
// odd length start at odd 8-byte offsets)
typedef double dpair __attribute__((ext_vector_type(2), aligned(8)));

constexpr int kStencilThreads = 256;
constexpr int kStencilWaves = 2048;   // 2 waves per SIMD on 256 CUs x 4 SIMDs
__host__ __device__ inline int stencil_blocks(const DevPlan& P) {
  const int cols = P.st_threads * P.st_cols;
  const int tiles = ((P.ny1 + P.st_rows - 1) / P.st_rows) * ((P.nx + cols - 1) / cols);
  const int nchunks = (P.nt / 2 + P.st_chunk - 1) / P.st_chunk;
  return tiles * nchunks;
}
int stencil_grid(const DevPlan& P, int mode);
int update_blocks(const DevPlan& P);
int dstx_blocks(const DevPlan& P, int wg);

hipError_t launch_stencil(const DevPlan& P, int mode, const double* x, double* y, const double* f, hipStream_t s);
hipError_t launch_rhs(const DevPlan& P, const double* src, const double* psi0, const double* psi1, double* f,
                      hipStream_t s);
hipError_t launch_init(const DevPlan& P, const double* f, double* u, double tol, int maxit, hipStream_t s);
hipError_t launch_update(const DevPlan& P, double* u, hipStream_t s);
// identity preconditioner: z = r (mode 0), or the MINRES set-up / Lanczos step with
// z = q and the partials of <q, q> (modes INV_GAMMA_INIT / INV_GAMMA_ITER)
hipError_t launch_identity(const DevPlan& P, int mode, const double* in, double* out, hipStream_t s);

// GMRES steps (kernels_gmres.hip); gslot(l) is the vector slot of Arnoldi vector v_l
enum GmresFin : int { G_INIT = 0, G_DOTS1 = 1, G_DOTS2 = 2, G_NORM = 3, G_CHECK = 4 };
hipError_t launch_ginit(const DevPlan& P, const double* f, double* u, hipStream_t s);
hipError_t launch_gfin(const DevPlan& P, int kind, double tol, int maxit, int restart, hipStream_t s);
hipError_t launch_gdots(const DevPlan& P, int j, const double* w, hipStream_t s);
hipError_t launch_gaxpy(const DevPlan& P, int j, int pass, double* w, hipStream_t s);
hipError_t launch_gbase(const DevPlan& P, const double* src, const double* u, int restart_step, hipStream_t s);
hipError_t launch_gcomb(const DevPlan& P, int j, double* t, hipStream_t s);
hipError_t launch_gaddx(const DevPlan& P, double* u, const double* z, hipStream_t s);
__host__ __device__ inline double* gslot(const DevPlan& P, int l) { return l < kZSlots ? P.Z[l] : P.W[l - kZSlots]; }
static_assert(kGmresMax + 1 <= kZSlots + 2, "the Arnoldi basis must fit the Z and W slots");
// u (and at the flush w_j, w_{j-1}) from the resident basis, for right-hand sides whose
// scalar step set form_now
hipError_t launch_form(const DevPlan& P, double* u, hipStream_t s);
// one block per right-hand side: fixed-order sum of the partials of a reduction and
// the scalar step that consumes it
hipError_t launch_fin(const DevPlan& P, int kind, double tol, int maxit, hipStream_t s);

// check != 0: skip right-hand sides whose solve is not running
hipError_t launch_dstx_fwd(const DevPlan& P, int prec, int mode, int check, const double* in, hipStream_t s);
hipError_t launch_dsty(const DevPlan& P, int prec, int check, hipStream_t s);
// inv1 = 1: the single time pass of C_alpha^{-1} (mu^{-1}, no time reversal); with check
// (and inv1 = 0) the pass also writes the partials of <q, P^{-1} q> (PART_GAMMA, one
// per mode pair)
hipError_t launch_time(const DevPlan& P, int prec, int check, hipStream_t s, int inv1 = 0);
hipError_t launch_dstx_inv(const DevPlan& P, int prec, int mode, double* out, hipStream_t s);
// fused 2D first / last pass (square grids whose level fits in LDS; P.wg_s != 0)
hipError_t launch_dst2_fwd(const DevPlan& P, int prec, int mode, int check, const double* in, hipStream_t s);
hipError_t launch_dst2_inv(const DevPlan& P, int prec, int mode, double* out, hipStream_t s);
int slab_wg(int nx, int ny, int prec, int maxlds, size_t margin);
// dynamic LDS bytes of the fused 2D passes with workgroup wg (0 if not legal)
size_t slab_lds_bytes(int L, int wg, int prec);
// fused small-problem iteration (1D, nt * nx <= 4096; P.small != 0)
hipError_t launch_iter_small(const DevPlan& P, int prec, const double* f, double* u, hipStream_t s);
hipError_t launch_setup_small(const DevPlan& P, int prec, const double* f, double* u, double tol, int maxit,
                              hipStream_t s);
hipError_t launch_solve_small(const DevPlan& P, int prec, const double* f, double* u, double tol, int maxit,
                              hipStream_t s);
bool small_path_valid(int nx, int ny, int nt, int prec);
// transform kernel kinds (tile validity and LDS size differ per kind)
enum TransformKind : int { TK_XFWD = 0, TK_XINV = 1, TK_Y = 2, TK_TIME = 3 };
// dynamic LDS bytes of one workgroup (0 if the tile is not legal)
size_t transform_lds_bytes(int kind, int L, int wg, int prec);
bool transform_tile_valid(int kind, int L, int wg, int prec);
int transform_tps(int L, int prec);   // threads per sequence of length L (prec 1: FP32)

}  // namespace abac

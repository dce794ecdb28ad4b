// Fused MINRES set-up, iteration and whole solve for small 1D problems (N = nt * nx <= 4096
// unknowns).
//
// At these sizes an iteration of the separate kernels (matvec, scalar step, three
// transform passes, scalar step, update, scalar step, iterate, residual, scalar step)
// is bound by the launch latency of its eleven kernels, not by memory.  Here one
// workgroup per right-hand side runs the whole iteration, tile after tile, with
// workgroup barriers between the steps, so an iteration is one launch.  The steps use
// the same per-tile device code as the separate kernels, in the same order and under
// the same per-right-hand-side conditions (Section 3's MINRES: Lanczos in the P^{-1}
// inner product, Givens QR, residual recurrence, explicit check); only the order of
// the partial sums differs (one workgroup sums its own tiles, in a fixed order, so the
// result does not depend on the batch).
#include "../../include/abac.h"
#include "abac_internal.h"
#include "minres_device.h"
#include "stencil_device.h"
#include "transform_device.h"

namespace abac {

namespace {

constexpr int kSmallWG = 512;

// u = sum_l xm_l z_l over the first nb basis slots (with flush also the two w vectors
// from their coefficients), the whole right-hand side by one workgroup.
__device__ void form_small(const DevPlan& P, int b, double* __restrict__ u, int nb, bool flush) {
  const size_t off = (size_t)b * P.N;
  const double* kc = P.kcoef + (size_t)b * 3 * kBasis;
  double* X = u + off;
  double* W1 = P.W[kBasis & 1] + off;
  double* W2 = P.W[(kBasis + 1) & 1] + off;
  for (int e = threadIdx.x; e < P.N; e += blockDim.x) {
    double ax = 0.0, a1 = 0.0, a2 = 0.0;
    for (int l = 0; l < nb; ++l) {
      const double z = P.Z[l][off + e];
      ax += kc[l] * z;
      a1 += kc[kBasis + l] * z;
      a2 += kc[2 * kBasis + l] * z;
    }
    X[e] = ax;
    if (flush) {
      W1[e] = a1;
      W2[e] = a2;
    }
  }
}

// Stencil over every logical block of right-hand side b: the workgroup holds
// kSmallWG / st_threads logical blocks side by side.
template <int OUT, bool DOT>
__device__ __forceinline__ double stencil_small(const DevPlan& P, const double* x, double* y, const double* f) {
  const int grp = kSmallWG / P.st_threads;
  const int first = threadIdx.x / P.st_threads, tx = threadIdx.x % P.st_threads;
  return P.coef_x ? stencil_run<true, OUT, DOT>(P, x, y, f, first, grp, tx, false)
                  : stencil_run<false, OUT, DOT>(P, x, y, f, first, grp, tx, false);
}

// LDS: the largest tile region of the steps, then the x twiddle table, staged once per
// launch (the tiles of one workgroup run one after another, so twiddles read from
// global memory would expose their latency in every FFT pass).
template <typename T, int L, int NT>
constexpr size_t small_tile_lds() {
  constexpr size_t a = lds_of<T, L, kSmallWG, TK_XFWD>();
  constexpr size_t b = lds_of<T, L, kSmallWG, TK_XINV>();
  constexpr size_t c = lds_of<T, NT, kSmallWG, TK_TIME>();
  return ((a > b ? (a > c ? a : c) : (b > c ? b : c)) + 15) / 16 * 16;
}

template <typename T, int L, int NT>
constexpr size_t small_lds() {
  return small_tile_lds<T, L, NT>() + (size_t)L * sizeof(cplx<T>);
}

template <typename T, int L, int NT>
__device__ __forceinline__ const cplx<T>* stage_twiddles_small(const DevPlan& P) {
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem + small_tile_lds<T, L, NT>());
  stage_table(tw, reinterpret_cast<const cplx<T>*>(P.twx), L);
  __syncthreads();
  return tw;
}

template <typename T, int L, int NT>
constexpr bool small_ok() {
  return tile_ok<T, L, kSmallWG, TK_XFWD>() && tile_ok<T, L, kSmallWG, TK_XINV>() &&
         tile_ok<T, NT, kSmallWG, TK_TIME>() && small_lds<T, L, NT>() <= kMaxTransformLds &&
         (L / 2 - 1) * NT <= 4096 && (sizeof(T) == 4 || NT <= 128);   // FP64 nt = 256 would spill
}

// One MINRES iteration of right-hand side blockIdx.x (1D, x-DST length L, nt = NT); every
// thread of the workgroup calls it, and every branch below is uniform (state read after a
// barrier).
template <typename T, int L, int NT>
__device__ __noinline__ void iter_small(const DevPlan& P, const double* __restrict__ f, double* __restrict__ u,
                                        const cplx<T>* twx) {
  constexpr int WG = kSmallWG;
  const int b = blockIdx.x;
  const size_t off = (size_t)b * P.N;
  MinresState* st = P.st + b;
  const int tid = threadIdx.x;
  // matvec q = Y T z_j with <Y T z_j, z_j>, then delta_j
  if (st->state == ST_RUNNING) {
    const int j = st->iter + 1;
    const double acc = stencil_small<OUT_REV, true>(P, P.Z[zslot(j)] + off, P.V[(j + 1) % 3] + off, nullptr);
    const double tot = block_sum(acc);
    if (fin_begin(P, b, FIN_DELTA) && tid == 0) fin_scalar(P, b, FIN_DELTA, tot, 0.0, 0);
    __syncthreads();
  }
  // Lanczos vector and z_{j+1} = P^{-1} q: x-DST (Lanczos fused), time pass with the
  // partials of <q, P^{-1} q>, inverse x-DST, then gamma_{j+1} and the Givens step
  if (st->state == ST_RUNNING) {
    constexpr int SX = seqs_of<T, L, WG>(), ST = seqs_of<T, NT, WG>();
    const int xtiles = (P.nt + 2 * SX - 1) / (2 * SX);
    const int ttiles = (P.ms / 2 + ST - 1) / ST;
    for (int t = 0; t < xtiles; ++t) {
      dstx_fwd_tile<T, L, WG>(P, FWD_LANCZOS, nullptr, b, t, twx);
      __syncthreads();
    }
    for (int t = 0; t < ttiles; ++t) {
      time_tile<T, NT, WG>(P, 0, b, t, 1);
      __syncthreads();
    }
    const double tot = sum_parts(part_slot(P, PART_GAMMA, b), P.ms / 2);
    for (int t = 0; t < xtiles; ++t) {
      dstx_inv_tile<T, L, WG>(P, INV_Z_ITER, nullptr, b, t, twx);
      __syncthreads();
    }
    if (fin_begin(P, b, FIN_GAMMA_ITER) && tid == 0) fin_scalar(P, b, FIN_GAMMA_ITER, tot, 0.0, 0);
    __syncthreads();
  }
  // residual recurrence and the stopping test (a stopped solve marks a stale u)
  {
    double tot = 0.0;
    if (st->state == ST_RUNNING) tot = block_sum(update_part(P, b, u, 0, 1));
    if (fin_begin(P, b, FIN_RNORM) && tid == 0) fin_scalar(P, b, FIN_RNORM, tot, 0.0, 0);
    __syncthreads();
  }
  // the iterate from the resident basis when a check, a stop or the flush needs it
  if (st->form_now) {
    form_small(P, b, u, st->nbasis, st->flush_now != 0);
    __syncthreads();
  }
  // explicit residual check, end of the iteration (snapshot)
  {
    double tot = 0.0;
    if (st->state == ST_RUNNING && st->need_check)
      tot = block_sum(stencil_small<OUT_RESNORM, false>(P, u + off, nullptr, f + off));
    if (fin_begin(P, b, FIN_RES) && tid == 0) fin_scalar(P, b, FIN_RES, tot, 0.0, 0);
  }
}

template <typename T, int L, int NT>
__global__ void __launch_bounds__(kSmallWG)
k_iter_small(DevPlan P, const double* __restrict__ f, double* __restrict__ u) {
  iter_small<T, L, NT>(P, f, u, stage_twiddles_small<T, L, NT>(P));
}


// Set-up of a solve of right-hand side blockIdx.x in one workgroup: b = Y f into v_1,
// u = 0, ||b||^2, then z_1 = P^{-1} b and gamma_1 (the separate kernels' set-up and
// first preconditioner apply, in the same order and under the same conditions).
template <typename T, int L, int NT>
__device__ __noinline__ void setup_small(const DevPlan& P, const double* __restrict__ f, double* __restrict__ u,
                                         double tol, int maxit, const cplx<T>* twx) {
  constexpr int WG = kSmallWG;
  const int b = blockIdx.x;
  const size_t off = (size_t)b * P.N;
  MinresState* st = P.st + b;
  const int tid = threadIdx.x;
  {
    double acc = 0.0;
    for (int e = tid; e < P.N; e += WG) {
      const int k = e / P.m;
      const double v = f[off + (size_t)(P.nt - 1 - k) * P.m + (e - k * P.m)];
      P.V[1][off + e] = v;
      u[off + e] = 0.0;
      acc += v * v;
    }
    const double tot = block_sum(acc);
    if (fin_begin(P, b, FIN_BNORM) && tid == 0) fin_scalar(P, b, FIN_BNORM, tot, tol, maxit);
    __syncthreads();
  }
  double tot = 0.0;
  if (st->state == ST_RUNNING) {
    constexpr int SX = seqs_of<T, L, WG>(), ST = seqs_of<T, NT, WG>();
    const int xtiles = (P.nt + 2 * SX - 1) / (2 * SX);
    const int ttiles = (P.ms / 2 + ST - 1) / ST;
    for (int t = 0; t < xtiles; ++t) {
      dstx_fwd_tile<T, L, WG>(P, FWD_PLAIN, P.V[1], b, t, twx);
      __syncthreads();
    }
    for (int t = 0; t < ttiles; ++t) {
      time_tile<T, NT, WG>(P, 0, b, t, 1);
      __syncthreads();
    }
    tot = sum_parts(part_slot(P, PART_GAMMA, b), P.ms / 2);
    for (int t = 0; t < xtiles; ++t) {
      dstx_inv_tile<T, L, WG>(P, INV_Z_INIT, nullptr, b, t, twx);
      __syncthreads();
    }
  }
  if (fin_begin(P, b, FIN_GAMMA_INIT) && tid == 0) fin_scalar(P, b, FIN_GAMMA_INIT, tot, 0.0, 0);
}

template <typename T, int L, int NT>
__global__ void __launch_bounds__(kSmallWG)
k_setup_small(DevPlan P, const double* __restrict__ f, double* __restrict__ u, double tol, int maxit) {
  setup_small<T, L, NT>(P, f, u, tol, maxit, stage_twiddles_small<T, L, NT>(P));
}

// A whole solve in one launch: the set-up, then iterations until the right-hand side
// stops (at most maxit + 1, a safety net: the state machine stops it by maxit).
template <typename T, int L, int NT>
__global__ void __launch_bounds__(kSmallWG)
k_solve_small(DevPlan P, const double* __restrict__ f, double* __restrict__ u, double tol, int maxit) {
  // The right-hand side's scalar state stays in LDS for the whole solve (the scalar steps
  // and every thread's state tests read it many times per iteration) and goes back to
  // memory at the end.  Q addresses it as Q.st + blockIdx.x, like the kernels' state.
  __shared__ MinresState st_lds;
  const int b = blockIdx.x;
  if (threadIdx.x == 0) st_lds = P.st[b];
  DevPlan Q = P;
  Q.st = reinterpret_cast<MinresState*>(reinterpret_cast<uintptr_t>(&st_lds) - (uintptr_t)b * sizeof(MinresState));
  const cplx<T>* twx = stage_twiddles_small<T, L, NT>(Q);   // its barrier also publishes st_lds
  setup_small<T, L, NT>(Q, f, u, tol, maxit, twx);
  for (int it = 0; it <= maxit; ++it) {
    __syncthreads();   // the previous step's state is visible to every thread
    if (st_lds.state != ST_RUNNING) break;
    iter_small<T, L, NT>(Q, f, u, twx);
  }
  __syncthreads();
  if (threadIdx.x == 0) P.st[b] = st_lds;
}

// what: 0 one iteration, 1 the set-up, 2 a whole solve (set-up and iterations)
template <typename T, int L, int NT>
hipError_t launch_small_t(const DevPlan& P, const double* f, double* u, hipStream_t s, int what, double tol,
                          int maxit) {
  if constexpr (!small_ok<T, L, NT>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr size_t lds = small_lds<T, L, NT>();
    if (what == 1)
      hipLaunchKernelGGL((k_setup_small<T, L, NT>), dim3(P.B), dim3(kSmallWG), lds, s, P, f, u, tol, maxit);
    else if (what == 2)
      hipLaunchKernelGGL((k_solve_small<T, L, NT>), dim3(P.B), dim3(kSmallWG), lds, s, P, f, u, tol, maxit);
    else
      hipLaunchKernelGGL((k_iter_small<T, L, NT>), dim3(P.B), dim3(kSmallWG), lds, s, P, f, u);
    return hipGetLastError();
  }
}

#define ABAC_SMALL_NT(LL, CALL)               \
  switch (P.nt) {                             \
    case 8: return CALL(LL, 8);               \
    case 16: return CALL(LL, 16);             \
    case 32: return CALL(LL, 32);             \
    case 64: return CALL(LL, 64);             \
    case 128: return CALL(LL, 128);           \
    case 256: return CALL(LL, 256);           \
    default: return hipErrorInvalidValue;     \
  }

template <typename T>
hipError_t small_dispatch(const DevPlan& P, const double* f, double* u, hipStream_t s, int what, double tol,
                          int maxit) {
#define CALL(LL, NN) launch_small_t<T, LL, NN>(P, f, u, s, what, tol, maxit)
  switch (2 * P.Mx) {
    case 16: ABAC_SMALL_NT(16, CALL)
    case 32: ABAC_SMALL_NT(32, CALL)
    case 64: ABAC_SMALL_NT(64, CALL)
    case 128: ABAC_SMALL_NT(128, CALL)
    default: return hipErrorInvalidValue;
  }
#undef CALL
}

template <typename T>
bool small_valid_t(int L, int nt) {
#define CALL(LL, NN) small_ok<T, LL, NN>()
  switch (L) {
#define ABAC_SMALL_NT_OK(LL)                                                                            \
  case LL:                                                                                             \
    switch (nt) {                                                                                      \
      case 8: return CALL(LL, 8);                                                                      \
      case 16: return CALL(LL, 16);                                                                    \
      case 32: return CALL(LL, 32);                                                                    \
      case 64: return CALL(LL, 64);                                                                    \
      case 128: return CALL(LL, 128);                                                                  \
      case 256: return CALL(LL, 256);                                                                  \
      default: return false;                                                                           \
    }
    ABAC_SMALL_NT_OK(16) ABAC_SMALL_NT_OK(32) ABAC_SMALL_NT_OK(64) ABAC_SMALL_NT_OK(128)
#undef ABAC_SMALL_NT_OK
    default: return false;
  }
#undef CALL
}

}  // namespace

hipError_t launch_iter_small(const DevPlan& P, int prec, const double* f, double* u, hipStream_t s) {
  return prec ? small_dispatch<float>(P, f, u, s, 0, 0.0, 0) : small_dispatch<double>(P, f, u, s, 0, 0.0, 0);
}

hipError_t launch_setup_small(const DevPlan& P, int prec, const double* f, double* u, double tol, int maxit,
                              hipStream_t s) {
  return prec ? small_dispatch<float>(P, f, u, s, 1, tol, maxit) : small_dispatch<double>(P, f, u, s, 1, tol, maxit);
}

hipError_t launch_solve_small(const DevPlan& P, int prec, const double* f, double* u, double tol, int maxit,
                              hipStream_t s) {
  return prec ? small_dispatch<float>(P, f, u, s, 2, tol, maxit) : small_dispatch<double>(P, f, u, s, 2, tol, maxit);
}

bool small_path_valid(int nx, int ny, int nt, int prec) {
  if (ny || prec == ABAC_PREC_NONE) return false;
  const int L = 2 * (nx + 1);
  return prec ? small_valid_t<float>(L, nt) : small_valid_t<double>(L, nt);
}

}  // namespace abac

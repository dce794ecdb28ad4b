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
#include "transform_device.h"

namespace abac {

namespace {

template <typename T, int L, int WG>
__global__ void __launch_bounds__(WG)
k_dstx_fwd(DevPlan P, int mode, int check, const double* __restrict__ in) {
  if ((check || mode == FWD_LANCZOS) && P.st[blockIdx.y].state != ST_RUNNING) return;
  dstx_fwd_tile<T, L, WG>(P, mode, in, blockIdx.y, blockIdx.x, reinterpret_cast<const cplx<T>*>(P.twx));
}

template <typename T, int L, int WG>
__global__ void __launch_bounds__(WG)
k_dsty(DevPlan P, int check) {
  if (check && P.st[blockIdx.y].state != ST_RUNNING) return;
  // XCD-aware order: the blocks one XCD runs together read neighbouring column pairs of
  // a level, so partial cache lines are shared in its L2
  dsty_tile<T, L, WG>(P, blockIdx.y, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int NT, int WG>
__global__ void __launch_bounds__(WG)
k_time(DevPlan P, int check, int inv1) {
  if (check && P.st[blockIdx.y].state != ST_RUNNING) return;
  // XCD-aware order: the blocks one XCD runs together read neighbouring column ranges of
  // each time level, so partial cache lines are shared in its L2.  In MINRES mode
  // (check) the pass also forms the partials of <q, P^{-1} q>.
  time_tile<T, NT, WG>(P, inv1, blockIdx.y, xcd_remap(blockIdx.x, gridDim.x), check && !inv1);
}

template <typename T, int L, int WG>
__global__ void __launch_bounds__(WG)
k_dstx_inv(DevPlan P, int mode, double* __restrict__ outp) {
  const int b = blockIdx.y;
  if (mode != INV_PLAIN && P.st[b].state != ST_RUNNING) return;
  const double acc = dstx_inv_tile<T, L, WG>(P, mode, outp, b, blockIdx.x, reinterpret_cast<const cplx<T>*>(P.twx));
  if (mode != INV_GAMMA_INIT && mode != INV_GAMMA_ITER) return;
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_GAMMA, b)[blockIdx.x] = bs;
}

// fused 2D passes (square grids whose level fits in LDS; tile bodies in
// transform_device.h): one block per time level
// first pass, fused: (Lanczos step,) DST-I along x and y of one level, level written
// to the scratch.  Modes and checks as in k_dstx_fwd.
template <typename T, int L, int WG>
__global__ void __launch_bounds__(WG)
k_dst2_fwd(DevPlan P, int mode, int check, const double* __restrict__ in) {
  if ((check || mode == FWD_LANCZOS) && P.st[blockIdx.y].state != ST_RUNNING) return;
  dst2_fwd_tile<T, L, WG>(P, mode, in, blockIdx.y, blockIdx.x);
}

// last pass, fused: DST-I along y and x of one level of the scratch, FP64 rows out,
// with the block's partial of <q, p> in the GAMMA modes (one partial per level).  Modes
// as in k_dstx_inv.
template <typename T, int L, int WG>
__global__ void __launch_bounds__(WG)
k_dst2_inv(DevPlan P, int mode, double* __restrict__ outp) {
  const int b = blockIdx.y;
  if (mode != INV_PLAIN && P.st[b].state != ST_RUNNING) return;
  const double acc = dst2_inv_tile<T, L, WG>(P, mode, outp, b, blockIdx.x);
  if (mode != INV_GAMMA_INIT && mode != INV_GAMMA_ITER) return;
  const double bs = block_sum(acc);
  if (threadIdx.x == 0) part_slot(P, PART_GAMMA, b)[blockIdx.x] = bs;
}

// ---------------------------------------------------------------------------
// launchers: one instantiation per (precision, length, workgroup size)
// ---------------------------------------------------------------------------
template <typename T, int L, int WG>
hipError_t launch_x_fwd_t(const DevPlan& P, int mode, int check, const double* in, hipStream_t s) {
  if constexpr (!tile_ok<T, L, WG, TK_XFWD>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int S = seqs_of<T, L, WG>();
    const int rows = P.nt * P.ny1;
    dim3 grid((rows + 2 * S - 1) / (2 * S), P.B);
    const size_t lds = lds_of<T, L, WG, TK_XFWD>();
    hipLaunchKernelGGL((k_dstx_fwd<T, L, WG>), grid, dim3(WG), lds, s, P, mode, check, in);
    return hipGetLastError();
  }
}

template <typename T, int L, int WG>
hipError_t launch_x_inv_t(const DevPlan& P, int mode, double* out, hipStream_t s) {
  if constexpr (!tile_ok<T, L, WG, TK_XINV>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int S = seqs_of<T, L, WG>();
    const int rows = P.nt * P.ny1;
    dim3 grid((rows + 2 * S - 1) / (2 * S), P.B);
    const size_t lds = lds_of<T, L, WG, TK_XINV>();
    hipLaunchKernelGGL((k_dstx_inv<T, L, WG>), grid, dim3(WG), lds, s, P, mode, out);
    return hipGetLastError();
  }
}

template <typename T, int L, int WG>
hipError_t launch_y_t(const DevPlan& P, int check, hipStream_t s) {
  if constexpr (!tile_ok<T, L, WG, TK_Y>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int S = seqs_of<T, L, WG>();
    const int cpairs = P.Mx / 2;
    const int bpl = (cpairs + S - 1) / S;
    dim3 grid(bpl * P.nt, P.B);
    const size_t lds = lds_of<T, L, WG, TK_Y>();
    hipLaunchKernelGGL((k_dsty<T, L, WG>), grid, dim3(WG), lds, s, P, check);
    return hipGetLastError();
  }
}

template <typename T, int NT, int WG>
hipError_t launch_time_t(const DevPlan& P, int check, int inv1, hipStream_t s) {
  if constexpr (!tile_ok<T, NT, WG, TK_TIME>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int S = seqs_of<T, NT, WG>();
    const int npairs = P.ms / 2;
    dim3 grid((npairs + S - 1) / S, P.B);
    const size_t lds = lds_of<T, NT, WG, TK_TIME>();
    hipLaunchKernelGGL((k_time<T, NT, WG>), grid, dim3(WG), lds, s, P, check, inv1);
    return hipGetLastError();
  }
}

template <typename T, int L, int WG>
hipError_t launch_slab_t(const DevPlan& P, bool fwd, int mode, int check, const double* in, double* out,
                         hipStream_t s) {
  if constexpr (!slab_ok<T, L, WG>()) {
    return hipErrorInvalidValue;
  } else {
    dim3 grid(P.nt, P.B);
    const size_t lds = slab_lds_of<T, L, WG>();
    if (fwd)
      hipLaunchKernelGGL((k_dst2_fwd<T, L, WG>), grid, dim3(WG), lds, s, P, mode, check, in);
    else
      hipLaunchKernelGGL((k_dst2_inv<T, L, WG>), grid, dim3(WG), lds, s, P, mode, out);
    return hipGetLastError();
  }
}

#define ABAC_SWITCH_SLAB(LVAR, WGVAR, CALL)                                               \
  switch (LVAR) {                                                                         \
    case 16: switch (WGVAR) { case 64: return CALL(16, 64); default: break; } break;      \
    case 32: switch (WGVAR) { case 64: return CALL(32, 64); case 128: return CALL(32, 128); default: break; } break; \
    case 64: switch (WGVAR) { case 128: return CALL(64, 128); case 256: return CALL(64, 256); default: break; } break; \
    case 128: switch (WGVAR) { case 256: return CALL(128, 256); case 512: return CALL(128, 512); default: break; } break; \
    case 256: switch (WGVAR) { case 256: return CALL(256, 256); case 512: return CALL(256, 512); default: break; } break; \
    default: break;                                                                       \
  }

template <typename T>
hipError_t slab_dispatch(const DevPlan& P, bool fwd, int mode, int check, const double* in, double* out,
                         hipStream_t s) {
#define CALL(LL, WW) launch_slab_t<T, LL, WW>(P, fwd, mode, check, in, out, s)
  ABAC_SWITCH_SLAB(2 * P.Mx, P.wg_s, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

template <typename T> size_t slab_lds_t(int L, int wg) {
#define CALL(LL, WW) (slab_ok<T, LL, WW>() ? slab_lds_of<T, LL, WW>() : (size_t)0)
  ABAC_SWITCH_SLAB(L, wg, CALL)
#undef CALL
  return 0;
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
hipError_t time_dispatch(const DevPlan& P, int check, int inv1, hipStream_t s) {
#define CALL(LL, WW) launch_time_t<T, LL, WW>(P, check, inv1, s)
  ABAC_SWITCH_L(P.nt, P.wg_t, CALL)
#undef CALL
}

template <typename T, int KIND> hipError_t tile_check_t(int L, int wg) {
#define CALL(LL, WW) (tile_ok<T, LL, WW, KIND>() ? hipSuccess : hipErrorInvalidValue)
  ABAC_SWITCH_L(L, wg, CALL)
#undef CALL
}

template <typename T, int KIND> size_t lds_bytes_t(int L, int wg) {
#define CALL(LL, WW) lds_of<T, LL, WW, KIND>()
  ABAC_SWITCH_L(L, wg, CALL)
#undef CALL
}

template <typename T> hipError_t tile_check_k(int kind, int L, int wg) {
  switch (kind) {
    case TK_XFWD: return tile_check_t<T, TK_XFWD>(L, wg);
    case TK_XINV: return tile_check_t<T, TK_XINV>(L, wg);
    case TK_Y: return tile_check_t<T, TK_Y>(L, wg);
    case TK_TIME: return tile_check_t<T, TK_TIME>(L, wg);
    default: return hipErrorInvalidValue;
  }
}

template <typename T> size_t lds_bytes_k(int kind, int L, int wg) {
  switch (kind) {
    case TK_XFWD: return lds_bytes_t<T, TK_XFWD>(L, wg);
    case TK_XINV: return lds_bytes_t<T, TK_XINV>(L, wg);
    case TK_Y: return lds_bytes_t<T, TK_Y>(L, wg);
    case TK_TIME: return lds_bytes_t<T, TK_TIME>(L, wg);
    default: return 0;
  }
}

}  // namespace

hipError_t launch_dstx_fwd(const DevPlan& P, int prec, int mode, int check, const double* in, hipStream_t s) {
  return prec ? x_fwd_dispatch<float>(P, mode, check, in, s) : x_fwd_dispatch<double>(P, mode, check, in, s);
}

hipError_t launch_dsty(const DevPlan& P, int prec, int check, hipStream_t s) {
  return prec ? y_dispatch<float>(P, check, s) : y_dispatch<double>(P, check, s);
}

hipError_t launch_time(const DevPlan& P, int prec, int check, hipStream_t s, int inv1) {
  return prec ? time_dispatch<float>(P, check, inv1, s) : time_dispatch<double>(P, check, inv1, s);
}

hipError_t launch_dstx_inv(const DevPlan& P, int prec, int mode, double* out, hipStream_t s) {
  return prec ? x_inv_dispatch<float>(P, mode, out, s) : x_inv_dispatch<double>(P, mode, out, s);
}

hipError_t launch_dst2_fwd(const DevPlan& P, int prec, int mode, int check, const double* in, hipStream_t s) {
  return prec ? slab_dispatch<float>(P, true, mode, check, in, nullptr, s)
              : slab_dispatch<double>(P, true, mode, check, in, nullptr, s);
}

hipError_t launch_dst2_inv(const DevPlan& P, int prec, int mode, double* out, hipStream_t s) {
  return prec ? slab_dispatch<float>(P, false, mode, 0, nullptr, out, s)
              : slab_dispatch<double>(P, false, mode, 0, nullptr, out, s);
}

// Workgroup of the fused 2D passes for this shape, or 0 where they do not apply (1D,
// non-square grids, levels too large for LDS).  A fixed rule of the shape: the
// largest instantiated workgroup whose sequences per round do not exceed the line
// pairs of a level and whose LDS (plus `margin` for static LDS) fits `maxlds`.
int slab_wg(int nx, int ny, int prec, int maxlds, size_t margin) {
  if (!ny || nx != ny) return 0;
  const int L = 2 * (nx + 1);
  const int tps = transform_tps(L, prec);
  if (!tps) return 0;
  for (int wg : {512, 256, 128, 64}) {
    if (wg / tps > std::max((nx + 1) / 2, 64 / tps)) continue;
    const size_t lds = prec ? slab_lds_t<float>(L, wg) : slab_lds_t<double>(L, wg);
    if (lds && lds + margin <= (size_t)maxlds) return wg;
  }
  return 0;
}

size_t slab_lds_bytes(int L, int wg, int prec) {
  return prec == 1 ? slab_lds_t<float>(L, wg) : slab_lds_t<double>(L, wg);
}

bool transform_tile_valid(int kind, int L, int wg, int prec) {
  return (prec ? tile_check_k<float>(kind, L, wg) : tile_check_k<double>(kind, L, wg)) == hipSuccess;
}

template <typename T> int transform_tps_t(int L) {
  switch (L) {
    case 8: return fft_tps<T, 8>();
    case 16: return fft_tps<T, 16>();
    case 32: return fft_tps<T, 32>();
    case 64: return fft_tps<T, 64>();
    case 128: return fft_tps<T, 128>();
    case 256: return fft_tps<T, 256>();
    case 512: return fft_tps<T, 512>();
    case 1024: return fft_tps<T, 1024>();
    case 2048: return fft_tps<T, 2048>();
    case 4096: return fft_tps<T, 4096>();
    case 8192: return fft_tps<T, 8192>();
    default: return 0;
  }
}

int transform_tps(int L, int prec) { return prec == 1 ? transform_tps_t<float>(L) : transform_tps_t<double>(L); }

int dstx_blocks(const DevPlan& P, int wg) {
  const int S = wg / transform_tps(2 * P.Mx, P.prec);
  const int rows = P.nt * P.ny1;
  return (rows + 2 * S - 1) / (2 * S);
}

size_t transform_lds_bytes(int kind, int L, int wg, int prec) {
  if (!transform_tile_valid(kind, L, wg, prec)) return 0;
  return prec ? lds_bytes_k<float>(kind, L, wg) : lds_bytes_k<double>(kind, L, wg);
}

}  // namespace abac

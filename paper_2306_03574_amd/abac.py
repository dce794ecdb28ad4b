"""Thin Python binding of ``libabac.so`` (the C ABI declared in ``include/abac.h``).

Argument marshalling only: every step of the solver runs in the HIP library.  PyTorch
supplies device memory (the plan workspace and all vectors are torch tensors on the
GPU) and the HIP stream.  There is no fallback: if the library is not built or no
GPU is present, construction raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libabac.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, EBREAKDOWN, EBUDGET, EAGAIN = 0, -1, -2, -3, -4, -5, -6, -7
PREC = {"fp64": 0, "fp32": 1, "none": 2}
KERNELS = {"stencil": 0, "dstx_fwd": 1, "dsty": 2, "time": 3, "dstx_inv": 4, "update": 5,
           "residual": 6, "init": 7, "rhs": 8, "fin": 9, "form": 10, "gmres": 11, "iter": 12}

EXPORTED = [
    "abac_workspace_bytes", "abac_plan_create", "abac_plan_destroy", "abac_build_rhs", "abac_apply_A",
    "abac_apply_Pinv", "abac_minres_solve", "abac_minres_begin", "abac_minres_advance", "abac_minres_poll",
    "abac_minres_finish", "abac_profile_enable", "abac_profile_read", "abac_profile_reset",
    "abac_status_string", "abac_last_error", "abac_fill_normal", "abac_server_create", "abac_server_destroy",
    "abac_server_submit", "abac_server_step", "abac_server_result", "abac_server_clock",
    "abac_server_bytes_in_use", "abac_plan_tiles", "abac_plan_set_coefficient", "abac_apply_T", "abac_apply_Cinv",
    "abac_gmres_solve", "abac_plan_set_tiles", "abac_apply_Pinv_noalloc", "abac_group_create",
    "abac_group_destroy", "abac_group_set", "abac_group_advance", "abac_group_run", "abac_group_check",
    "abac_server_group_lane",
]

_lib = None


class AbacError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libabac.so and declare the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2306_03574_amd.build.build() first")
    lib = ctypes.CDLL(path)
    P, I, D, SZ, VP = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
    lib.abac_workspace_bytes.argtypes = [I, I, I, I, I]
    lib.abac_workspace_bytes.restype = SZ
    lib.abac_plan_create.argtypes = [I, I, I, D, D, I, I, VP, VP, SZ, ctypes.POINTER(P)]
    lib.abac_plan_create.restype = I
    lib.abac_plan_destroy.argtypes = [P]
    lib.abac_plan_destroy.restype = I
    lib.abac_build_rhs.argtypes = [P, VP, VP, VP, VP]
    lib.abac_build_rhs.restype = I
    lib.abac_apply_A.argtypes = [P, VP, VP]
    lib.abac_apply_A.restype = I
    lib.abac_apply_Pinv.argtypes = [P, VP, VP]
    lib.abac_apply_Pinv.restype = I
    lib.abac_minres_solve.argtypes = [P, VP, VP, D, I, VP, VP, VP]
    lib.abac_minres_solve.restype = I
    lib.abac_minres_begin.argtypes = [P, VP, VP, D, I]
    lib.abac_minres_begin.restype = I
    lib.abac_minres_advance.argtypes = [P, I]
    lib.abac_minres_advance.restype = I
    lib.abac_minres_poll.argtypes = [P, ctypes.POINTER(I)]
    lib.abac_minres_poll.restype = I
    lib.abac_minres_finish.argtypes = [P, VP, VP, VP]
    lib.abac_minres_finish.restype = I
    lib.abac_profile_enable.argtypes = [P, I]
    lib.abac_profile_enable.restype = I
    lib.abac_profile_read.argtypes = [P, I, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong)]
    lib.abac_profile_read.restype = I
    lib.abac_profile_reset.argtypes = [P]
    lib.abac_profile_reset.restype = I
    lib.abac_status_string.argtypes = [I]
    lib.abac_status_string.restype = ctypes.c_char_p
    lib.abac_last_error.argtypes = []
    lib.abac_last_error.restype = ctypes.c_char_p
    LL, ULL = ctypes.c_longlong, ctypes.c_ulonglong
    lib.abac_fill_normal.argtypes = [VP, VP, SZ, ULL]
    lib.abac_fill_normal.restype = I
    lib.abac_server_create.argtypes = [SZ, I, ctypes.POINTER(P)]
    lib.abac_server_create.restype = I
    lib.abac_server_destroy.argtypes = [P]
    lib.abac_server_destroy.restype = I
    lib.abac_server_submit.argtypes = [P, I, I, I, D, D, I, ULL, D, I, D, I, ctypes.POINTER(LL)]
    lib.abac_server_submit.restype = I
    lib.abac_server_step.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.abac_server_step.restype = I
    lib.abac_server_result.argtypes = [P, LL, VP, ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(I),
                                       ctypes.POINTER(D)]
    lib.abac_server_result.restype = I
    lib.abac_server_clock.argtypes = [P]
    lib.abac_server_clock.restype = D
    lib.abac_plan_tiles.argtypes = [P, ctypes.POINTER(I)]
    lib.abac_plan_tiles.restype = I
    lib.abac_apply_T.argtypes = [P, VP, VP]
    lib.abac_apply_T.restype = I
    lib.abac_apply_Cinv.argtypes = [P, VP, VP]
    lib.abac_apply_Cinv.restype = I
    lib.abac_gmres_solve.argtypes = [P, VP, VP, D, I, I, VP, VP, VP]
    lib.abac_gmres_solve.restype = I
    lib.abac_plan_set_coefficient.argtypes = [P, VP, VP, D]
    lib.abac_plan_set_coefficient.restype = I
    lib.abac_apply_Pinv_noalloc.argtypes = [I, I, I, D, D, I, I, VP, VP, VP]
    lib.abac_apply_Pinv_noalloc.restype = I
    lib.abac_server_group_lane.argtypes = [P, SZ]
    lib.abac_server_group_lane.restype = I
    lib.abac_group_create.argtypes = [VP, ctypes.POINTER(P)]
    lib.abac_group_create.restype = I
    lib.abac_group_destroy.argtypes = [P]
    lib.abac_group_destroy.restype = I
    lib.abac_group_set.argtypes = [P, ctypes.POINTER(P), I]
    lib.abac_group_set.restype = I
    lib.abac_group_advance.argtypes = [P, I]
    lib.abac_group_advance.restype = I
    lib.abac_group_run.argtypes = [P, I, I, D]
    lib.abac_group_run.restype = I
    lib.abac_group_check.argtypes = [P, ctypes.POINTER(I)]
    lib.abac_group_check.restype = I
    lib.abac_plan_set_tiles.argtypes = [P, I, I, I, I]
    lib.abac_plan_set_tiles.restype = I
    lib.abac_server_bytes_in_use.argtypes = [P]
    lib.abac_server_bytes_in_use.restype = SZ
    _lib = lib
    return lib


def _check(status: int, what: str, ok=(OK,)):
    if status not in ok:
        lib = load_library()
        raise AbacError(status, f"{what}: {lib.abac_status_string(status).decode()} "
                                f"({lib.abac_last_error().decode()})")
    return status


def fill_normal(out: torch.Tensor, seed: int, stream=None):
    """Fill a float64 device tensor with the library's seeded Philox N(0,1) values."""
    if out.device.type != "cuda" or out.dtype != torch.float64 or not out.is_contiguous():
        raise TypeError("out must be a contiguous float64 GPU tensor")
    s = stream if stream is not None else torch.cuda.current_stream(out.device)
    _check(load_library().abac_fill_normal(ctypes.c_void_p(s.cuda_stream), ctypes.c_void_p(out.data_ptr()),
                                           out.numel(), seed), "abac_fill_normal")
    return out


def apply_Pinv_noalloc(r: torch.Tensor, nx: int, ny: int, nt: int, T: float = 1.0, alpha: float = 1e-3,
                       prec: str = "fp64", z: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """z = P_alpha^{-1} r without a plan and without any device allocation by the
    library (abac_apply_Pinv_noalloc).  r: contiguous float64 GPU tensor [batch][nt][...]."""
    per = nt * nx * (ny if ny else 1)
    if r.device.type != "cuda" or r.dtype != torch.float64 or not r.is_contiguous() or r.numel() % per:
        raise TypeError(f"r must be a contiguous float64 GPU tensor of batch x {per} values")
    z = torch.empty_like(r) if z is None else z
    if z.device != r.device or z.dtype != torch.float64 or not z.is_contiguous() or z.numel() != r.numel():
        raise TypeError("z must be a contiguous float64 GPU tensor like r")
    s = stream if stream is not None else torch.cuda.current_stream(r.device)
    with torch.cuda.device(r.device):
        _check(load_library().abac_apply_Pinv_noalloc(nx, ny, nt, float(T), float(alpha), PREC[prec],
                                                      r.numel() // per, ctypes.c_void_p(r.data_ptr()),
                                                      ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(s.cuda_stream)),
               "abac_apply_Pinv_noalloc")
    return z


def workspace_bytes(nx: int, ny: int, nt: int, prec: str = "fp64", batch: int = 1) -> int:
    return int(load_library().abac_workspace_bytes(nx, ny, nt, PREC[prec], batch))


class Plan:
    """A solver plan for one grid (nx, ny, nt), final time T and alpha, with a fixed
    batch of right-hand sides, bound to a torch CUDA (HIP) stream."""

    def __init__(self, nx: int, ny: int, nt: int, T: float = 1.0, alpha: float = 1e-3, prec: str = "fp64",
                 batch: int = 1, device="cuda:0", stream: torch.cuda.Stream | None = None):
        lib = load_library()
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("the ABAC library needs a GPU (torch.cuda is not available)")
        self.nx, self.ny, self.nt, self.T, self.alpha, self.prec, self.batch = nx, ny, nt, T, alpha, prec, batch
        self.level_shape = (ny, nx) if ny else (nx,)
        self.shape = (batch, nt) + self.level_shape
        self.N = nt * nx * (ny if ny else 1)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = lib.abac_workspace_bytes(nx, ny, nt, PREC[prec], batch)
        if nbytes == 0:
            raise AbacError(EINVAL, f"unsupported problem nx={nx} ny={ny} nt={nt} prec={prec} batch={batch}")
        self.workspace = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.abac_plan_create(nx, ny, nt, float(T), float(alpha), PREC[prec], batch,
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.c_void_p(aligned),
                                        ctypes.c_size_t(nbytes), ctypes.byref(handle)), "abac_plan_create")
        self._h = handle
        self._lib = lib
        self._f = None
        self._u = None

    # -- helpers ---------------------------------------------------------------
    def _vec(self, t: torch.Tensor, name: str) -> ctypes.c_void_p:
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != torch.float64:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if not t.is_contiguous() or t.numel() != self.batch * self.N:
            raise ValueError(f"{name} must be contiguous with {self.batch * self.N} elements")
        return ctypes.c_void_p(t.data_ptr())

    def _level(self, t: torch.Tensor, name: str) -> ctypes.c_void_p:
        m = self.N // self.nt
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != torch.float64:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if not t.is_contiguous() or t.numel() != self.batch * m:
            raise ValueError(f"{name} must be contiguous with {self.batch * m} elements")
        return ctypes.c_void_p(t.data_ptr())

    def empty(self) -> torch.Tensor:
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    # -- operators -------------------------------------------------------------
    def build_rhs(self, src, psi0, psi1, f=None):
        f = self.empty() if f is None else f
        _check(self._lib.abac_build_rhs(self._h, self._vec(src, "src"), self._level(psi0, "psi0"),
                                        self._level(psi1, "psi1"), self._vec(f, "f")), "abac_build_rhs")
        return f

    def apply_A(self, x, y=None):
        y = self.empty() if y is None else y
        _check(self._lib.abac_apply_A(self._h, self._vec(x, "x"), self._vec(y, "y")), "abac_apply_A")
        return y

    def apply_Pinv(self, r, z=None):
        z = self.empty() if z is None else z
        _check(self._lib.abac_apply_Pinv(self._h, self._vec(r, "r"), self._vec(z, "z")), "abac_apply_Pinv")
        return z

    def apply_T(self, x, y=None):
        """y = T x (natural time order)."""
        y = self.empty() if y is None else y
        _check(self._lib.abac_apply_T(self._h, self._vec(x, "x"), self._vec(y, "y")), "abac_apply_T")
        return y

    def apply_Cinv(self, r, z=None):
        """z = C_alpha^{-1} r (the block alpha-circulant preconditioner)."""
        z = self.empty() if z is None else z
        _check(self._lib.abac_apply_Cinv(self._h, self._vec(r, "r"), self._vec(z, "z")), "abac_apply_Cinv")
        return z

    def gmres(self, f, u=None, tol: float = 1e-8, maxit: int = 500, restart: int = 15):
        """Right-preconditioned GMRES(restart) on T u = f.  Returns (u, iters, relres, status)."""
        u = self.empty() if u is None else u
        iters = (ctypes.c_int * self.batch)()
        relres = (ctypes.c_double * self.batch)()
        status = (ctypes.c_int * self.batch)()
        _check(self._lib.abac_gmres_solve(self._h, self._vec(f, "f"), self._vec(u, "u"), float(tol), int(maxit),
                                          int(restart), iters, relres, status), "abac_gmres_solve",
               ok=(OK, ENOTCONV, EBREAKDOWN))
        return u, list(iters), list(relres), list(status)

    def solve(self, f, u=None, tol: float = 1e-8, maxit: int = 500):
        """MINRES on Y T u = Y f.  Returns (u, iters[list], relres[list], status[list])."""
        u = self.empty() if u is None else u
        iters = (ctypes.c_int * self.batch)()
        relres = (ctypes.c_double * self.batch)()
        status = (ctypes.c_int * self.batch)()
        _check(self._lib.abac_minres_solve(self._h, self._vec(f, "f"), self._vec(u, "u"), float(tol), int(maxit),
                                           iters, relres, status), "abac_minres_solve",
               ok=(OK, ENOTCONV, EBREAKDOWN))
        return u, list(iters), list(relres), list(status)

    # -- asynchronous solve ----------------------------------------------------
    def begin(self, f, u, tol: float = 1e-8, maxit: int = 500):
        self._f, self._u = f, u
        _check(self._lib.abac_minres_begin(self._h, self._vec(f, "f"), self._vec(u, "u"), float(tol), int(maxit)),
               "abac_minres_begin")

    def advance(self, iterations: int = 1):
        _check(self._lib.abac_minres_advance(self._h, int(iterations)), "abac_minres_advance")

    def poll(self) -> bool:
        d = ctypes.c_int(0)
        _check(self._lib.abac_minres_poll(self._h, ctypes.byref(d)), "abac_minres_poll")
        return bool(d.value)

    def finish(self):
        iters = (ctypes.c_int * self.batch)()
        relres = (ctypes.c_double * self.batch)()
        status = (ctypes.c_int * self.batch)()
        _check(self._lib.abac_minres_finish(self._h, iters, relres, status), "abac_minres_finish",
               ok=(OK, ENOTCONV, EBREAKDOWN))
        self._f = None
        return list(iters), list(relres), list(status)

    def set_coefficient(self, a_xh=None, a_yh=None, abar: float | None = None):
        """Variable coefficient a(x) of u_tt = div(a grad u) + f (eq. (3.1)): face values
        a_xh [ny1][nx+1] at (x_{i+1/2}, y_j) and, in 2D, a_yh [ny+1][nx] at (x_i, y_{j+1/2}),
        host arrays; abar is the preconditioner's constant coefficient (eq. (3.3)).
        a_xh=None restores a = 1."""
        import numpy as np
        if a_xh is None:
            _check(self._lib.abac_plan_set_coefficient(self._h, None, None, 1.0), "abac_plan_set_coefficient")
            return
        ny1 = self.ny if self.ny else 1
        ax = np.ascontiguousarray(a_xh, dtype=np.float64)
        if ax.size != ny1 * (self.nx + 1):
            raise ValueError(f"a_xh must hold {ny1} x {self.nx + 1} values")
        ay = None
        if self.ny:
            if a_yh is None:
                raise ValueError("a_yh is required in 2D")
            ay = np.ascontiguousarray(a_yh, dtype=np.float64)
            if ay.size != (self.ny + 1) * self.nx:
                raise ValueError(f"a_yh must hold {self.ny + 1} x {self.nx} values")
        if abar is None:
            raise ValueError("abar (the preconditioner's constant coefficient) is required")
        _check(self._lib.abac_plan_set_coefficient(
            self._h, ctypes.c_void_p(ax.ctypes.data), ctypes.c_void_p(ay.ctypes.data) if ay is not None else None,
            float(abar)), "abac_plan_set_coefficient")

    def tiles(self):
        """Workgroup sizes: dict(dstx_fwd, dsty, time, dstx_inv, slab, small); slab is the
        fused x-y passes' workgroup, 0 when the plan uses separate x and y passes; small is
        the workgroup that runs a whole iteration per right-hand side, 0 when the plan
        launches the separate kernels."""
        wg = (ctypes.c_int * 6)()
        _check(self._lib.abac_plan_tiles(self._h, wg), "abac_plan_tiles")
        return {"dstx_fwd": wg[0], "dsty": wg[1], "time": wg[2], "dstx_inv": wg[3], "slab": wg[4],
                "small": wg[5]}

    def set_tiles(self, dstx_fwd: int = 0, dsty: int = 0, time: int = 0, dstx_inv: int = 0):
        """Override the tuned tiles of the first x pass, the y pass, the time pass and the
        last x pass (threads per workgroup; 0 keeps the current one).  Raises
        AbacError(EINVAL) for a tile that is not legal for its kernel."""
        _check(self._lib.abac_plan_set_tiles(self._h, int(dstx_fwd), int(dsty), int(time), int(dstx_inv)),
               "abac_plan_set_tiles")

    # -- kernel timing -----------------------------------------------------------
    def profile(self, on: bool = True):
        _check(self._lib.abac_profile_enable(self._h, 1 if on else 0), "abac_profile_enable")

    def profile_read(self, kernel: str):
        ms = ctypes.c_double(0)
        n = ctypes.c_longlong(0)
        _check(self._lib.abac_profile_read(self._h, KERNELS[kernel], ctypes.byref(ms), ctypes.byref(n)),
               "abac_profile_read")
        return ms.value, n.value

    def profile_reset(self):
        _check(self._lib.abac_profile_reset(self._h), "abac_profile_reset")

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._lib.abac_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Solves of different grids advanced together, one launch per MINRES step for all
    members (abac_group_*).  Members are Plan objects with a solve begun (Plan.begin)."""

    def __init__(self, device="cuda:0", stream: torch.cuda.Stream | None = None):
        self._lib = load_library()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self._lib.abac_group_create(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                   "abac_group_create")
        self._h = h
        self._members = []

    def set(self, plans):
        arr = (ctypes.c_void_p * max(len(plans), 1))(*[p._h.value for p in plans])
        _check(self._lib.abac_group_set(self._h, arr, len(plans)), "abac_group_set")
        self._members = list(plans)

    def advance(self, iterations: int = 1):
        _check(self._lib.abac_group_advance(self._h, int(iterations)), "abac_group_advance")

    def run(self, iterations: int = 1, blocks: int = 0, timeout_s: float = 0.0):
        """The same iterations as advance(), in one persistent launch of `blocks`
        workgroups (0: the library's default) (abac_group_run)."""
        with torch.cuda.device(self.device):
            _check(self._lib.abac_group_run(self._h, int(iterations), int(blocks), float(timeout_s)),
                   "abac_group_run")

    def check(self) -> bool:
        """Whether a persistent launch gave up at a barrier since the last check."""
        flag = ctypes.c_int(0)
        _check(self._lib.abac_group_check(self._h, ctypes.byref(flag)), "abac_group_check")
        return bool(flag.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.abac_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


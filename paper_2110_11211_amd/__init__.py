"""MI355X-native SFC two-level overlapping Schwarz solver.

Thin ctypes binding of the C ABI in include/sfcdd.h (libsfcdd.so, built for
gfx950 by `build_lib.build()`).  The binding only marshals arguments: every
step of setup, preconditioner application and solve runs in the library's HIP
kernels.  PyTorch provides device memory (the workspace and the vectors) and
the stream.  There is no CPU fallback: if the library cannot be loaded the
import of `lib()` raises.

Method: Griebel, Schweitzer, Troska, "A dimension-oblivious domain
decomposition method based on space-filling curves" (Sec. 3.3, Alg. 1-3).
"""
from __future__ import annotations

import ctypes
import os
from fractions import Fraction
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfcdd.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, EOVERFLOW, ENOTSPD, ESTAGNATED = 0, -1, -2, -3, -4, -5, -6, -7
_STATUS = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENOTCONV: "ENOTCONV",
           EOVERFLOW: "EOVERFLOW", ENOTSPD: "ENOTSPD", ESTAGNATED: "ESTAGNATED"}
WEIGHTING = {"none": 0, "omega": 1, "D": 2}
VARIANT = {"additive": 0, "balanced": 1, "deflated": 2}
FACTOR_DTYPE = {"fp64": 0, "fp32": 1}
LOCAL_SOLVER = {"cholesky": 0, "inverse": 1}
METHOD = {"pcg": 0, "fcg": 1, "richardson": 2}
SOLVE_PLAIN_START = 256
SOLVE_RECURSIVE = 512
SOLVE_ENERGY = 1024
CURVE = {"zorder": 0, "hilbert": 1}
NOALLOC_WORKSPACE_BYTES = 256 << 20  # SFCDD_NOALLOC_WORKSPACE_BYTES
LAYOUT = {"natural": 0, "sfc": 1}
COARSE_PRECISION = {"auto": 0, "fp64": 1}
COARSE_SOLVER = {"dense": 0, "iterative": 1}
LOCAL_ORDER = {"diagonal": 0, "curve": 1, "dense": 2}
COARSE_SPLIT = {"auto": 0, "off": 1}

EXPORTS = ["sfcdd_workspace_size", "sfcdd_workspace_size_batch", "sfcdd_setup", "sfcdd_setup_batch",
           "sfcdd_setup_noalloc",
           "sfcdd_apply_precond", "sfcdd_matvec", "sfcdd_solve", "sfcdd_grad_coeff",
           "sfcdd_get_partition", "sfcdd_get_batch_stats", "sfcdd_partition_host", "sfcdd_autotune",
           "sfcdd_get_info", "sfcdd_set_profiling", "sfcdd_get_kernel_time", "sfcdd_read_probe",
           "sfcdd_ct_combine", "sfcdd_ct_layout", "sfcdd_tune", "sfcdd_destroy", "sfcdd_last_error"]
KERNELS = {"local_solve": 0, "scatter": 1, "spmv": 2, "coarse": 3, "spmv_b": 4}


class SfcddError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("level", ctypes.POINTER(ctypes.c_int32)),
                ("npts", ctypes.POINTER(ctypes.c_int32)), ("coeff", ctypes.POINTER(ctypes.c_double)),
                ("P", ctypes.c_int32), ("gamma_num", ctypes.c_int64), ("gamma_den", ctypes.c_int64),
                ("q", ctypes.c_int32), ("weighting", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("factor_dtype", ctypes.c_int32), ("local_solver", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("curve", ctypes.c_int32),
                ("coarse_precision", ctypes.c_int32), ("coarse_solver", ctypes.c_int32),
                ("coarse_tol", ctypes.c_double), ("local_order", ctypes.c_int32),
                ("coarse_split", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("xi", ctypes.c_double),
                ("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("coarse_steps", ctypes.c_int32), ("coarse_unconverged", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("P", ctypes.c_int32), ("q", ctypes.c_int32),
                ("N0", ctypes.c_int32), ("max_Ni", ctypes.c_int32), ("min_Ni", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("sum_Ni", ctypes.c_int64), ("factor_bytes", ctypes.c_int64),
                ("factor_algo_bytes", ctypes.c_int64), ("coarse_bytes", ctypes.c_int64),
                ("setup_ms", ctypes.c_double * 6), ("ngrids", ctypes.c_int32),
                ("trsv_waves", ctypes.c_int32), ("coarse_fp32", ctypes.c_int32),
                ("coarse_inv_fp32", ctypes.c_int32), ("coarse_iterative", ctypes.c_int32),
                ("N0d", ctypes.c_int32), ("ell_width", ctypes.c_int32), ("coarse_steps", ctypes.c_int32),
                ("factor_rows", ctypes.c_int32), ("factor_pair", ctypes.c_int32),
                ("spmv_points", ctypes.c_int32), ("spmv_window", ctypes.c_int32),
                ("local_order", ctypes.c_int32), ("factor_flops", ctypes.c_double),
                ("coarse_split", ctypes.c_int32 * 3)]


class Tuning(ctypes.Structure):
    _fields_ = [("trsv_waves", ctypes.c_int32), ("spmv_points", ctypes.c_int32),
                ("spmv_window", ctypes.c_int32), ("factor_rows", ctypes.c_int32),
                ("factor_pair", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("trsv_ms", ctypes.c_double), ("trsv_default_ms", ctypes.c_double),
                ("spmv_ms", ctypes.c_double), ("spmv_default_ms", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("setup_default_ms", ctypes.c_double),
                ("trsv_stream", ctypes.c_int32)]


TUNE = {"trsv": 1, "spmv": 2, "setup": 4, "all": 7}


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded C-ABI library; builds it first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from .build_lib import build
        build()
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.sfcdd_workspace_size.argtypes = [P(Params), P(ctypes.c_size_t)]
    L.sfcdd_workspace_size_batch.argtypes = [i32, P(Params), P(ctypes.c_size_t)]
    L.sfcdd_setup.argtypes = [P(Params), vp, ctypes.c_size_t, vp, P(vp)]
    L.sfcdd_setup_batch.argtypes = [i32, P(Params), vp, ctypes.c_size_t, vp, P(vp)]
    L.sfcdd_setup_noalloc.argtypes = [P(Params), vp, P(vp)]
    L.sfcdd_get_batch_stats.argtypes = [vp, P(i32), P(dbl)]
    L.sfcdd_autotune.argtypes = [vp, i32, P(dbl)]
    L.sfcdd_tune.argtypes = [vp, i32, i32, P(Tuning)]
    L.sfcdd_apply_precond.argtypes = [vp, vp, vp]
    L.sfcdd_matvec.argtypes = [vp, vp, vp]
    L.sfcdd_solve.argtypes = [vp, vp, vp, dbl, i32, i32, dbl, P(SolveInfo)]
    L.sfcdd_grad_coeff.argtypes = [vp, vp, vp, P(dbl)]
    L.sfcdd_get_partition.argtypes = [vp, i32, P(i32), P(i64), P(i64), P(dbl), P(i32)]
    L.sfcdd_partition_host.argtypes = [P(Params), P(i64), P(i64), P(dbl), P(i32)]
    L.sfcdd_get_info.argtypes = [vp, P(Info)]
    L.sfcdd_set_profiling.argtypes = [vp, i32]
    L.sfcdd_get_kernel_time.argtypes = [vp, i32, P(dbl), P(i64)]
    L.sfcdd_ct_layout.argtypes = [i32, i32, i32, i32, P(i32), P(i32), P(i32), P(dbl), P(i32)]
    L.sfcdd_destroy.argtypes = [vp]
    L.sfcdd_last_error.argtypes = [vp]
    L.sfcdd_last_error.restype = ctypes.c_char_p
    for name in EXPORTS[:-1]:
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st: int, ctx=None):
    if st != OK:
        msg = lib().sfcdd_last_error(ctx)
        raise SfcddError(st, msg.decode() if msg else "")


def make_params(levels=None, npts=None, coeff=None, P=1, gamma=Fraction(1, 2), q=0,
                weighting="omega", variant="balanced", factor_dtype="fp64",
                local_solver="cholesky", layout="natural", curve="zorder", coarse_precision="auto",
                coarse_solver="dense", coarse_tol=0.0, local_order="diagonal", coarse_split="auto"):
    """Builds the sfcdd_params struct; returns (struct, keepalive)."""
    g = Fraction(gamma)
    d = len(levels) if levels is not None else len(npts)
    keep = []
    prm = Params()
    prm.d = d
    if levels is not None:
        arr = (ctypes.c_int32 * d)(*[int(v) for v in levels])
        keep.append(arr)
        prm.level = arr
    if npts is not None:
        arr = (ctypes.c_int32 * d)(*[int(v) for v in npts])
        keep.append(arr)
        prm.npts = arr
    if coeff is not None:
        arr = (ctypes.c_double * d)(*[float(v) for v in coeff])
        keep.append(arr)
        prm.coeff = arr
    prm.P = int(P)
    prm.gamma_num = g.numerator
    prm.gamma_den = g.denominator
    prm.q = int(q)
    prm.weighting = WEIGHTING[weighting]
    prm.variant = VARIANT[variant]
    prm.factor_dtype = FACTOR_DTYPE[factor_dtype]
    prm.local_solver = LOCAL_SOLVER[local_solver]
    prm.layout = LAYOUT[layout]
    prm.curve = CURVE[curve]
    prm.coarse_precision = COARSE_PRECISION[coarse_precision]
    prm.coarse_solver = COARSE_SOLVER[coarse_solver]
    prm.coarse_tol = float(coarse_tol)
    prm.local_order = LOCAL_ORDER[local_order]
    prm.coarse_split = COARSE_SPLIT[coarse_split]
    return prm, keep


def workspace_size(**kw) -> int:
    prm, keep = make_params(**kw)
    n = ctypes.c_size_t()
    _check(lib().sfcdd_workspace_size(ctypes.byref(prm), ctypes.byref(n)))
    return int(n.value)


def read_probe(buf, repeats: int = 5) -> float:
    """Best time (ms) of a streaming read of the device tensor `buf` (whole
    bytes, 16-byte aligned); bytes / time is the device's streaming-read rate."""
    import torch
    nbytes = buf.numel() * buf.element_size()
    ms = ctypes.c_double()
    stream = torch.cuda.current_stream(buf.device)
    _check(lib().sfcdd_read_probe(ctypes.c_void_p(buf.data_ptr()), ctypes.c_size_t(nbytes),
                                  ctypes.c_void_p(stream.cuda_stream), int(repeats), ctypes.byref(ms)))
    return float(ms.value)


def partition_host(**kw):
    """(ta, Ni, omega, q) of the decomposition, computed on the host only."""
    import numpy as np
    prm, keep = make_params(**kw)
    Pn = prm.P
    ta = (ctypes.c_int64 * Pn)()
    Ni = (ctypes.c_int64 * Pn)()
    om = (ctypes.c_double * Pn)()
    q = ctypes.c_int32()
    _check(lib().sfcdd_partition_host(ctypes.byref(prm), ta, Ni, om, ctypes.byref(q)))
    return np.array(ta[:], dtype=np.int64), np.array(Ni[:], dtype=np.int64), np.array(om[:]), int(q.value)


class SFCSchwarz:
    """One set-up solver context: grid, partition, factors, coarse operator.

    All vectors are float64 torch tensors of length N on the context's device,
    in natural order (first coordinate fastest) unless layout="sfc".  Work is
    enqueued on the torch stream current at construction.  workspace="static"
    selects the allocation-free setup (sfcdd_setup_noalloc): the library's
    static per-device workspace, which a later such setup on the device takes
    over.
    """

    def __init__(self, levels: Optional[Sequence[int]] = None, npts: Optional[Sequence[int]] = None,
                 coeff: Optional[Sequence[float]] = None, P: int = 1, gamma=Fraction(1, 2), q: int = 0,
                 weighting: str = "omega", variant: str = "balanced", factor_dtype: str = "fp64",
                 local_solver: str = "cholesky", layout: str = "natural", device="cuda:0",
                 workspace=None, curve: str = "zorder", coarse_precision: str = "auto",
                 coarse_solver: str = "dense", coarse_tol: float = 0.0, local_order: str = "diagonal",
                 coarse_split: str = "auto"):
        import torch
        self._torch = torch
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("SFCSchwarz needs a ROCm GPU device")
        self.kw = dict(levels=levels, npts=npts, coeff=coeff, P=P, gamma=gamma, q=q, weighting=weighting,
                       variant=variant, factor_dtype=factor_dtype, local_solver=local_solver,
                       layout=layout, curve=curve, coarse_precision=coarse_precision,
                       coarse_solver=coarse_solver, coarse_tol=coarse_tol, local_order=local_order,
                       coarse_split=coarse_split)
        prm, self._keep = make_params(**self.kw)
        self._prm = prm
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            ctx = ctypes.c_void_p()
            if isinstance(workspace, str):
                if workspace != "static":
                    raise ValueError('workspace must be a uint8 tensor, None or "static"')
                self.ws = None
                _check(lib().sfcdd_setup_noalloc(ctypes.byref(prm), ctypes.c_void_p(self.stream.cuda_stream),
                                                 ctypes.byref(ctx)), None if not ctx.value else ctx)
            else:
                self.ws = self._workspace(workspace)
                _check(lib().sfcdd_setup(ctypes.byref(prm), ctypes.c_void_p(self.ws.data_ptr()),
                                         self.ws.numel(), ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(ctx)), None if not ctx.value else ctx)
        self.ctx = ctx
        inf = Info()
        _check(lib().sfcdd_get_info(self.ctx, ctypes.byref(inf)), self.ctx)
        self.N = int(inf.N)
        self.d = prm.d
        self._info = inf

    # -- helpers -----------------------------------------------------------
    def _query_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().sfcdd_workspace_size(ctypes.byref(self._prm), ctypes.byref(n)))
        return int(n.value)

    @property
    def workspace_bytes(self) -> int:
        """Workspace bytes the library plans for this problem."""
        if getattr(self, "_ws_bytes", None) is None:
            self._ws_bytes = self._query_bytes()
        return self._ws_bytes

    def _workspace(self, workspace):
        """The caller's uint8 workspace tensor (its size is checked by the
        library's setup, which fails with ENOMEM when it is short), else a new
        one of the planned size."""
        torch = self._torch
        if workspace is not None:
            if not isinstance(workspace, torch.Tensor) or workspace.device != self.device \
                    or workspace.dtype != torch.uint8 or not workspace.is_contiguous():
                raise ValueError(f"workspace must be a contiguous uint8 tensor on {self.device}")
            return workspace
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)

    def _vec(self, t, name):
        torch = self._torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device \
                or t.numel() != self.N or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor of {self.N} entries on {self.device}")
        return ctypes.c_void_p(t.data_ptr())

    def info(self) -> dict:
        i = self._info
        return {k: (list(getattr(i, k)) if k in ("setup_ms", "coarse_split") else getattr(i, k))
                for k, _ in Info._fields_}

    # -- operators ---------------------------------------------------------
    def apply(self, g, out=None):
        """h = C^{-1} g (Alg. 2 / eq. balSW)."""
        torch = self._torch
        h = torch.empty_like(g) if out is None else out
        _check(lib().sfcdd_apply_precond(self.ctx, self._vec(g, "g"), self._vec(h, "h")), self.ctx)
        return h

    def matvec(self, x, out=None):
        torch = self._torch
        y = torch.empty_like(x) if out is None else out
        _check(lib().sfcdd_matvec(self.ctx, self._vec(x, "x"), self._vec(y, "y")), self.ctx)
        return y

    def solve(self, b, x0=None, rtol=1e-9, max_iter=1000, method="pcg", xi=0.0, check=True,
              plain_start=False, recursive=False, energy=False):
        """x with A x = b to relative residual rtol; returns (x, info dict).
        plain_start: balanced variant only, start from x0 as given and apply
        the full balanced operator every iteration (otherwise the start is
        coarse-corrected and each iteration needs one coarse solve).
        recursive: stop on the recursive residual of the iteration alone
        (otherwise it is confirmed on the true residual).
        energy: b must be zero; stop when the energy norm of the iterate (the
        error) falls below rtol (the Sec. 4.1 protocol)."""
        torch = self._torch
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        inf = SolveInfo()
        code = METHOD[method] | (SOLVE_PLAIN_START if plain_start else 0) | (SOLVE_RECURSIVE if recursive else 0) \
            | (SOLVE_ENERGY if energy else 0)
        st = lib().sfcdd_solve(self.ctx, self._vec(b, "b"), self._vec(x, "x"), float(rtol), int(max_iter),
                               code, float(xi), ctypes.byref(inf))
        if check:
            _check(st, self.ctx)
        info = {k: getattr(inf, k) for k, _ in SolveInfo._fields_}
        info["status"] = st
        return x, info

    def grad_coeff(self, lam, u):
        """dJ/da_j = -lam^T (dA/da_j) u (host list of d floats)."""
        out = (ctypes.c_double * self.d)()
        _check(lib().sfcdd_grad_coeff(self.ctx, self._vec(lam, "lam"), self._vec(u, "u"), out), self.ctx)
        return [float(v) for v in out]

    def set_profiling(self, on: bool = True):
        _check(lib().sfcdd_set_profiling(self.ctx, 1 if on else 0), self.ctx)

    def kernel_time(self, kind: str):
        """(total ms, launches) of a timed kernel class since profiling was enabled."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().sfcdd_get_kernel_time(self.ctx, KERNELS[kind], ctypes.byref(ms), ctypes.byref(n)),
               self.ctx)
        return float(ms.value), int(n.value)

    def partition(self) -> dict:
        import numpy as np
        Pn = self.kw["P"]
        sfc = (ctypes.c_int32 * self.N)()
        ta = (ctypes.c_int64 * Pn)()
        Ni = (ctypes.c_int64 * Pn)()
        om = (ctypes.c_double * Pn)()
        q = ctypes.c_int32()
        _check(lib().sfcdd_get_partition(self.ctx, 0, sfc, ta, Ni, om, ctypes.byref(q)), self.ctx)
        return {"sfc_index": np.ctypeslib.as_array(sfc).astype(np.int64), "ta": np.array(ta[:]),
                "Ni": np.array(Ni[:]), "omega": np.array(om[:]), "q": int(q.value)}

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().sfcdd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SFCSchwarzBatch(SFCSchwarz):
    """Many independent grids in one context (e.g. one layer of the
    combination technique): every setup phase and solver operator runs as one
    launch over all grids.  `grids` is a list of dicts with the per-grid keys
    levels / npts, coeff, P, gamma, q, curve; the other options are shared.  Vectors
    concatenate the grids in order (see `offsets`)."""

    def __init__(self, grids, weighting: str = "omega", variant: str = "balanced",
                 factor_dtype: str = "fp64", local_solver: str = "cholesky", layout: str = "natural",
                 device="cuda:0", workspace=None, local_order: str = "diagonal"):
        import torch
        self._torch = torch
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("SFCSchwarzBatch needs a ROCm GPU device")
        G = len(grids)
        arr = (Params * G)()
        self._keep = []
        for k, gk in enumerate(grids):
            prm, keep = make_params(levels=gk.get("levels"), npts=gk.get("npts"), coeff=gk.get("coeff"),
                                    P=gk["P"], gamma=gk.get("gamma", Fraction(1, 2)), q=gk.get("q", 0),
                                    weighting=weighting, variant=variant, factor_dtype=factor_dtype,
                                    local_solver=local_solver, layout=layout,
                                    curve=gk.get("curve", "zorder"), local_order=local_order)
            arr[k] = prm
            self._keep.append(keep)
        self._arr = arr
        self.G = G
        self.kw = dict(P=sum(g["P"] for g in grids), weighting=weighting, variant=variant,
                       factor_dtype=factor_dtype, local_solver=local_solver, layout=layout,
                       local_order=local_order)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.ws = self._workspace(workspace)
            ctx = ctypes.c_void_p()
            st = lib().sfcdd_setup_batch(G, arr, ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
            _check(st, None if not ctx.value else ctx)
        self.ctx = ctx
        inf = Info()
        _check(lib().sfcdd_get_info(self.ctx, ctypes.byref(inf)), self.ctx)
        self.N = int(inf.N)
        self.G = G
        self.d = None
        self._info = inf
        sizes = []
        for gk in grids:
            nn = [(1 << l) - 1 for l in gk["levels"]] if gk.get("levels") is not None else list(gk["npts"])
            sizes.append(int(__import__("numpy").prod(nn)))
        self.sizes = sizes
        self.offsets = [0]
        for v in sizes:
            self.offsets.append(self.offsets[-1] + v)

    def _query_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().sfcdd_workspace_size_batch(self.G, self._arr, ctypes.byref(n)))
        return int(n.value)

    def split(self, v):
        """Per-grid views of a concatenated vector."""
        return [v[self.offsets[k]:self.offsets[k + 1]] for k in range(self.G)]

    def batch_stats(self):
        """(iterations, relative residuals) per grid of the last solve."""
        its = (ctypes.c_int32 * self.G)()
        res = (ctypes.c_double * self.G)()
        _check(lib().sfcdd_get_batch_stats(self.ctx, its, res), self.ctx)
        return list(its), list(res)

    def partition(self, grid: int = 0) -> dict:
        import numpy as np
        Pn = self._arr[grid].P
        Ng = self.sizes[grid]
        sfc = (ctypes.c_int32 * Ng)()
        ta = (ctypes.c_int64 * Pn)()
        Ni = (ctypes.c_int64 * Pn)()
        om = (ctypes.c_double * Pn)()
        q = ctypes.c_int32()
        _check(lib().sfcdd_get_partition(self.ctx, grid, sfc, ta, Ni, om, ctypes.byref(q)), self.ctx)
        return {"sfc_index": np.ctypeslib.as_array(sfc).astype(np.int64), "ta": np.array(ta[:]),
                "Ni": np.array(Ni[:]), "omega": np.array(om[:]), "q": int(q.value)}


def _autotune(self, repeats: int = 5):
    """Picks the fastest subdomain-solve launch shape on this context's own
    factors; returns the time per application (ms)."""
    ms = ctypes.c_double()
    _check(lib().sfcdd_autotune(self.ctx, int(repeats), ctypes.byref(ms)), self.ctx)
    inf = Info()
    _check(lib().sfcdd_get_info(self.ctx, ctypes.byref(inf)), self.ctx)
    self._info = inf
    return float(ms.value)


SFCSchwarz.autotune = _autotune


def _tune(self, what="all", repeats: int = 3) -> dict:
    """Autotunes the launch shapes (sfcdd_tune; what: "trsv", "spmv", "setup",
    "all" or a list of them) on this context; returns the chosen shapes and
    their times against the defaults (ms)."""
    bits = TUNE[what] if isinstance(what, str) else sum(TUNE[w] for w in what)
    rep = Tuning()
    _check(lib().sfcdd_tune(self.ctx, int(repeats), int(bits), ctypes.byref(rep)), self.ctx)
    inf = Info()
    _check(lib().sfcdd_get_info(self.ctx, ctypes.byref(inf)), self.ctx)
    self._info = inf
    return {k: getattr(rep, k) for k, _ in Tuning._fields_}


SFCSchwarz.tune = _tune

from .autograd import PoissonSolve, solve_poisson  # noqa: E402,F401
from .ct import CombinationTechnique  # noqa: E402,F401

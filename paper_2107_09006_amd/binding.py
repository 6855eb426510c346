"""ctypes binding of the lsq2l C ABI (``include/lsq2l.h``).

Argument marshalling only: every step of setup, solve and backward runs in
the HIP library.  Device memory comes from PyTorch tensors (float64/int32 on
a ROCm device); the current PyTorch stream is handed to the library.  There
is no fallback: a missing library or a non-GPU tensor raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsq2l.so")

OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, CHOL_BREAKDOWN, PCG_BREAKDOWN = 0, 1, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
ADDITIVE, ONE_LEVEL, BALANCED, RAS, DEFLATED = 0, 1, 2, 3, 4
PCG, LSQR, GMRES = 0, 1, 2
ORDER_AUTO, ORDER_SPLIT, ORDER_GLOBAL = 0, 1, 2
FACTOR_CHOLESKY, FACTOR_QR = 0, 1

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP",
                -4: "CHOL_BREAKDOWN", -5: "PCG_BREAKDOWN"}

# every function the header declares
EXPORTS = ["lsq2l_default_options", "lsq2l_setup", "lsq2l_setup_batched", "lsq2l_solve",
           "lsq2l_solve_batched", "lsq2l_backward", "lsq2l_spmv", "lsq2l_apply_preconditioner",
           "lsq2l_get_info", "lsq2l_get_subdomain", "lsq2l_get_coarse_basis",
           "lsq2l_time_kernel", "lsq2l_autotune", "lsq2l_transpose", "lsq2l_transpose_noalloc",
           "lsq2l_destroy",
           "lsq2l_release_cache", "lsq2l_last_error"]


class Options(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_it", C.c_int32), ("precision", C.c_int32),
                ("flexible", C.c_int32), ("variant", C.c_int32), ("nev_max", C.c_int32),
                ("check_every", C.c_int32), ("use_graph", C.c_int32), ("krylov", C.c_int32),
                ("restart", C.c_int32), ("diag_shift_rel", C.c_double),
                ("adjoint_tol", C.c_double), ("autotune", C.c_int32), ("solve_order", C.c_int32),
                ("local_factor", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("relres", C.c_double),
                ("relres_rec", C.c_double), ("solve_ms", C.c_double),
                ("backward_err", C.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SetupInfo(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64), ("nparts", C.c_int32),
                ("ninstances", C.c_int32), ("n0", C.c_int64), ("max_ni", C.c_int32),
                ("max_p", C.c_int32), ("factor_bytes", C.c_int64),
                ("factor_dense_bytes", C.c_int64), ("factor_tiles", C.c_int64),
                ("factor_nnz_min", C.c_int64), ("shift", C.c_double),
                ("t_plan_ms", C.c_double), ("t_assemble_ms", C.c_double),
                ("t_factor_ms", C.c_double), ("t_eigen_ms", C.c_double),
                ("t_coarse_ms", C.c_double), ("t_total_ms", C.c_double),
                ("spmv_lanes_A", C.c_int32), ("spmv_lanes_AT", C.c_int32),
                ("t_prepare_ms", C.c_double), ("split_tiles", C.c_int64),
                ("solve_permuted", C.c_int32), ("mixed_fallback", C.c_int32)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Problem(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("colind", C.c_void_p), ("vals", C.c_void_p),
                ("part", C.c_void_p), ("nparts", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblsq2l.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2107_09006_amd.build.build()")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.lsq2l_default_options.argtypes = [C.POINTER(Options)]
    lib.lsq2l_default_options.restype = None
    lib.lsq2l_setup.argtypes = [i64, i64, i64, vp, vp, vp, vp, i32, i32, dbl, C.POINTER(Options),
                                vp, C.POINTER(vp)]
    lib.lsq2l_setup_batched.argtypes = [i32, C.POINTER(Problem), dbl, C.POINTER(Options), vp,
                                        C.POINTER(vp)]
    lib.lsq2l_solve.argtypes = [vp, vp, vp, C.POINTER(SolveInfo)]
    lib.lsq2l_solve_batched.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(SolveInfo)]
    lib.lsq2l_autotune.argtypes = [vp, i32, vp]
    lib.lsq2l_transpose.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.lsq2l_transpose_noalloc.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.lsq2l_backward.argtypes = [vp, vp, vp, vp, C.POINTER(SolveInfo)]
    lib.lsq2l_spmv.argtypes = [vp, i32, vp, vp]
    lib.lsq2l_apply_preconditioner.argtypes = [vp, vp, vp]
    lib.lsq2l_get_info.argtypes = [vp, C.POINTER(SetupInfo)]
    lib.lsq2l_get_subdomain.argtypes = [vp, i32, vp, vp, vp, vp]
    lib.lsq2l_get_coarse_basis.argtypes = [vp, i32, vp]
    lib.lsq2l_time_kernel.argtypes = [vp, i32, i32, C.POINTER(dbl), C.POINTER(dbl)]
    lib.lsq2l_destroy.argtypes = [vp]
    lib.lsq2l_destroy.restype = None
    lib.lsq2l_release_cache.argtypes = []
    lib.lsq2l_release_cache.restype = None
    lib.lsq2l_last_error.restype = C.c_char_p
    for name in ["lsq2l_setup", "lsq2l_setup_batched", "lsq2l_solve", "lsq2l_solve_batched",
                 "lsq2l_backward", "lsq2l_spmv", "lsq2l_apply_preconditioner", "lsq2l_get_info",
                 "lsq2l_get_subdomain", "lsq2l_get_coarse_basis", "lsq2l_time_kernel",
                 "lsq2l_autotune", "lsq2l_transpose", "lsq2l_transpose_noalloc"]:
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


class Lsq2lError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lsq2l {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status: int, allow=(OK,)):
    if status not in allow:
        raise Lsq2lError(status, _lib.lsq2l_last_error().decode())
    return status


def default_options(**kw) -> Options:
    lib = load_library()
    o = Options()
    lib.lsq2l_default_options(C.byref(o))
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, v)
    return o


def _dev(t, dtype):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("expected a tensor on a ROCm device")
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise TypeError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _to_device(a, dtype, device):
    """A contiguous device tensor of the given dtype (no copy if it already is one)."""
    import torch
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    npdt = {torch.int32: np.int32, torch.int64: np.int64, torch.float64: np.float64}[dtype]
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=npdt))).to(device)


def _part_arg(part, device):
    """The partition as the ABI takes it: a device tensor is passed as is
    (int32, contiguous), anything else as a host int32 array."""
    import torch
    if isinstance(part, torch.Tensor) and part.is_cuda:
        t = part.to(dtype=torch.int32).contiguous()
        return C.c_void_p(t.data_ptr()), t
    a = np.ascontiguousarray(np.asarray(part.cpu() if isinstance(part, torch.Tensor) else part,
                                        dtype=np.int32))
    return a.ctypes.data_as(C.c_void_p), a


def _stream(device):
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Solver:
    """A preconditioner handle: setup on construction, then solve/backward."""

    def __init__(self, rowptr, colind, vals, part, nparts: int, m: int, n: int, tau: float,
                 overlap: int = 1, device="cuda:0", **options):
        import torch
        lib = load_library()
        self.device = torch.device(device)
        self.m, self.n = int(m), int(n)
        self.rowptr = _to_device(rowptr, torch.int64, self.device)
        self.colind = _to_device(colind, torch.int32, self.device)
        self.vals = _to_device(vals, torch.float64, self.device)
        self.nnz = int(self.colind.numel())
        part_ptr, self._part = _part_arg(part, self.device)
        self.opts = default_options(**options)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.lsq2l_setup(self.m, self.n, self.nnz, _dev(self.rowptr, torch.int64),
                                 _dev(self.colind, torch.int32), _dev(self.vals, torch.float64),
                                 part_ptr, int(nparts), int(overlap),
                                 float(tau), C.byref(self.opts), _stream(self.device), C.byref(h))
        _check(st)
        self.handle = h
        self.nparts = int(nparts)
        self.ninstances = 1

    @classmethod
    def batched(cls, problems, tau: float, device="cuda:0", **options):
        """problems: list of (rowptr, colind, vals, part, nparts, m, n)."""
        import torch
        lib = load_library()
        self = cls.__new__(cls)
        self.device = torch.device(device)
        self._keep = []
        arr = (Problem * len(problems))()
        M = N = NNZ = 0
        for k, (rp, ci, va, pt, npart, m, n) in enumerate(problems):
            rp_t = _to_device(rp, torch.int64, self.device)
            ci_t = _to_device(ci, torch.int32, self.device)
            va_t = _to_device(va, torch.float64, self.device)
            pt_ptr, pt_keep = _part_arg(pt, self.device)
            self._keep += [rp_t, ci_t, va_t, pt_keep]
            arr[k] = Problem(int(m), int(n), int(ci_t.numel()), rp_t.data_ptr(), ci_t.data_ptr(),
                             va_t.data_ptr(), pt_ptr.value, int(npart), 0)
            M += int(m); N += int(n); NNZ += int(ci_t.numel())
        self.opts = default_options(**options)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.lsq2l_setup_batched(len(problems), arr, float(tau), C.byref(self.opts),
                                         _stream(self.device), C.byref(h))
        _check(st)
        self.handle = h
        self.m, self.n, self.nnz = M, N, NNZ
        self.ninstances = len(problems)
        self.nparts = sum(int(p[4]) for p in problems)
        self.sizes = [(int(p[5]), int(p[6])) for p in problems]
        return self

    # -- calls --------------------------------------------------------------
    def solve(self, b, x=None, allow_not_converged=False):
        import torch
        lib = load_library()
        if x is None:
            x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        infos = (SolveInfo * self.ninstances)()
        with torch.cuda.device(self.device):
            st = lib.lsq2l_solve(self.handle, _dev(b, torch.float64), _dev(x, torch.float64), infos)
        _check(st, (OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        return x, [i.asdict() for i in infos], st

    def solve_batched(self, bs, xs=None, allow_not_converged=False):
        """One right-hand side and one solution tensor per instance of a
        batched handle (lsq2l_solve_batched)."""
        import torch
        lib = load_library()
        if xs is None:
            xs = [torch.empty(n, dtype=torch.float64, device=self.device) for _, n in self.sizes]
        bp = (C.c_void_p * self.ninstances)(*[_dev(b, torch.float64).value for b in bs])
        xp = (C.c_void_p * self.ninstances)(*[_dev(x, torch.float64).value for x in xs])
        infos = (SolveInfo * self.ninstances)()
        with torch.cuda.device(self.device):
            st = lib.lsq2l_solve_batched(self.handle, bp, xp, infos)
        _check(st, (OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        return xs, [i.asdict() for i in infos], st

    def backward(self, g, want_b=True, want_vals=True, allow_not_converged=False):
        """dL/db and dL/dvals for g = dL/dx.  The adjoint solve stops on its
        normwise backward error (see lsq2l_backward); a solve that misses it
        raises unless allow_not_converged."""
        import torch
        lib = load_library()
        dLdb = torch.empty(self.m, dtype=torch.float64, device=self.device) if want_b else None
        dLdv = torch.empty(self.nnz, dtype=torch.float64, device=self.device) if want_vals else None
        infos = (SolveInfo * self.ninstances)()
        with torch.cuda.device(self.device):
            st = lib.lsq2l_backward(self.handle, _dev(g, torch.float64),
                                    _dev(dLdb, torch.float64) if want_b else None,
                                    _dev(dLdv, torch.float64) if want_vals else None, infos)
        _check(st, (OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        return dLdb, dLdv, [i.asdict() for i in infos]

    def spmv(self, x, trans=False):
        import torch
        lib = load_library()
        y = torch.empty(self.n if trans else self.m, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib.lsq2l_spmv(self.handle, 1 if trans else 0, _dev(x, torch.float64),
                                  _dev(y, torch.float64)))
        return y

    def apply_preconditioner(self, r, out=None):
        """z = M r; ``out`` (n doubles on the device, may be ``r``) receives z."""
        import torch
        lib = load_library()
        z = torch.empty(self.n, dtype=torch.float64, device=self.device) if out is None else out
        with torch.cuda.device(self.device):
            _check(lib.lsq2l_apply_preconditioner(self.handle, _dev(r, torch.float64),
                                                  _dev(z, torch.float64)))
        return z

    def info(self) -> dict:
        inf = SetupInfo()
        _check(load_library().lsq2l_get_info(self.handle, C.byref(inf)))
        return inf.asdict()

    def subdomain(self, i: int) -> dict:
        lib = load_library()
        sizes = np.zeros(4, dtype=np.int32)
        _check(lib.lsq2l_get_subdomain(self.handle, int(i), sizes.ctypes.data, None, None, None))
        I = np.zeros(max(1, sizes[0]), dtype=np.int32)
        X = np.zeros(max(1, sizes[1]), dtype=np.int32)
        G = np.zeros(max(1, sizes[2]), dtype=np.int32)
        _check(lib.lsq2l_get_subdomain(self.handle, int(i), None, I.ctypes.data, X.ctypes.data,
                                       G.ctypes.data))
        return {"I": I[:sizes[0]], "Xi": X[:sizes[1]], "G": G[:sizes[2]], "p": int(sizes[3])}

    def coarse_basis(self, i: int) -> np.ndarray:
        d = self.subdomain(i)
        X = np.zeros((max(1, d["p"]), max(1, d["I"].size)), dtype=np.float64)
        _check(load_library().lsq2l_get_coarse_basis(self.handle, int(i), X.ctypes.data))
        return X[:d["p"], :d["I"].size].T.copy()

    def autotune(self, reps: int = 10, shapes=None):
        """Measured SpMV shapes for A and A^T (lsq2l_autotune); with reps=0,
        sets them from `shapes` (0 = LDS row blocks, else lanes per row)."""
        import torch
        lanes = np.zeros(2, dtype=np.int32)
        if shapes is not None:
            lanes[:] = shapes
        with torch.cuda.device(self.device):
            _check(load_library().lsq2l_autotune(self.handle, int(reps), lanes.ctypes.data))
        return int(lanes[0]), int(lanes[1])

    def time_kernel(self, kernel: int, reps: int = 20):
        """(mean ms per launch, algorithmic bytes per launch) of a hot-path kernel."""
        import torch
        ms, by = C.c_double(), C.c_double()
        with torch.cuda.device(self.device):
            _check(load_library().lsq2l_time_kernel(self.handle, int(kernel), int(reps),
                                                    C.byref(ms), C.byref(by)))
        return ms.value, by.value

    def close(self):
        if getattr(self, "handle", None):
            load_library().lsq2l_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def transpose(m, n, rowptr, colind, vals=None, device="cuda:0", noalloc=False, out=None):
    """A^T of a CSR matrix on the device (lsq2l_transpose, or
    lsq2l_transpose_noalloc with ``noalloc``): returns (trowptr, trow, tvals
    or None, tperm) as device tensors.  ``out`` may hold those four output
    tensors, preallocated (the no-allocation caller's case)."""
    import torch
    lib = load_library()
    fn = lib.lsq2l_transpose_noalloc if noalloc else lib.lsq2l_transpose
    dev = torch.device(device)
    rp = _to_device(rowptr, torch.int32, dev)
    ci = _to_device(colind, torch.int32, dev)
    nnz = int(ci.numel())
    va = _to_device(vals, torch.float64, dev) if vals is not None else None
    if out is None:
        trp = torch.empty(int(n) + 1, dtype=torch.int32, device=dev)
        tr = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        tp = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        tv = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev) if va is not None else None
    else:
        trp, tr, tv, tp = out
    with torch.cuda.device(dev):
        _check(fn(int(m), int(n), nnz, _dev(rp, torch.int32),
                                   _dev(ci, torch.int32) if nnz else None,
                                   _dev(va, torch.float64) if va is not None else None,
                                   _dev(trp, torch.int32), _dev(tr, torch.int32),
                                   _dev(tv, torch.float64) if tv is not None else None,
                                   _dev(tp, torch.int32), _stream(dev)))
    return trp, tr[:nnz], (tv[:nnz] if tv is not None else None), tp[:nnz]


def release_cache() -> None:
    """Free the device memory that destroyed handles left in the library's
    process-wide cache (handles still alive keep theirs)."""
    load_library().lsq2l_release_cache()


def solver_from_problem(prob, device="cuda:0", **options) -> Solver:
    """Convenience: build a Solver from a ``workloads.Problem``."""
    return Solver(prob.indptr, prob.indices, prob.data, prob.part, prob.nparts, prob.m, prob.n,
                  prob.tau, device=device, **options)

"""ctypes binding of libfemh (include/femh.h).

Argument marshalling only: every step of the solver runs in the HIP library.
The raw C entry points are exposed under their C names (``femh_solve`` ...);
``Context`` / ``Problem`` / ``Server`` wrap them for Python callers, taking
problems and waves in the layout of the ``workloads`` package and torch
tensors for device buffers.  PyTorch provides device memory (through an
allocator callback bound to its caching allocator) and the stream.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfemh.so")

FEMH_OK = 0
FEMH_E_INVALID = -1
FEMH_E_NONFINITE = -2
FEMH_E_OOM = -3
FEMH_E_DEVICE = -4
FEMH_E_NOT_CONVERGED = -5
FEMH_E_BREAKDOWN = -6
FEMH_E_CANCELLED = -7
FEMH_E_PENDING = -8
FEMH_E_NOT_FOUND = -9
STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "NONFINITE", -3: "OOM", -4: "DEVICE", -5: "NOT_CONVERGED",
                -6: "BREAKDOWN", -7: "CANCELLED", -8: "PENDING", -9: "NOT_FOUND"}

FEMH_FACE_ABC = 0
FEMH_FACE_NATURAL = 1
FEMH_FACE_SYM = 2
FEMH_FACE_ANTISYM = 3
FEMH_FP64 = 0
FEMH_MIXED = 1
FEMH_MIXED_MATRIX = 2
FEMH_PRECOND_JACOBI = 0
FEMH_PRECOND_NONE = 1
FEMH_PRECOND_BIC0 = 2


class FemhError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"femh status {status} ({STATUS_NAMES.get(status, '?')}): {msg}")
        self.status = status


class femh_c128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class femh_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class femh_problem_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("h", C.c_double * 3), ("origin", C.c_double * 3),
                ("eps_r", C.c_void_p), ("mu_r", C.c_void_p), ("pec", C.c_void_p),
                ("outer_face", C.c_int32 * 6), ("k0", C.c_double), ("penalty_s", C.c_double),
                ("arrays_on_device", C.c_int32), ("penalty_surface", C.c_int32)]


class femh_plane_wave(C.Structure):
    _fields_ = [("d", C.c_double * 3), ("p", femh_c128 * 3)]


class femh_solve_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("precond", C.c_int32), ("rtol", C.c_double),
                ("max_iter", C.c_int32), ("precond_block", C.c_int32), ("inner_rtol", C.c_double),
                ("max_outer", C.c_int32),
                ("check_every", C.c_int32)]


class femh_solve_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("outer_iters", C.c_int32),
                ("reserved", C.c_int32), ("rel_residual", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {"status": self.status, "iters": self.iters, "outer_iters": self.outer_iters,
                "rel_residual": self.rel_residual, "seconds": self.seconds}


class femh_problem_info(C.Structure):
    _fields_ = [("grid_nodes", C.c_int64), ("n_nodes", C.c_int64), ("n_unknowns", C.c_int64),
                ("nnzb", C.c_int64), ("device_bytes", C.c_int64)]


class femh_server_opts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_slots", C.c_int32), ("chunk_iters", C.c_int32),
                ("batch_rhs", C.c_int32), ("reserved", C.c_int32)]


class femh_server_report(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("cancelled", C.c_int64), ("rejected", C.c_int64), ("rhs_completed", C.c_int64),
                ("p50_seconds", C.c_double), ("p99_seconds", C.c_double),
                ("requests_per_second", C.c_double), ("rhs_per_second", C.c_double),
                ("peak_resident_bytes", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
PI64 = C.POINTER(C.c_int64)
PD = C.POINTER(C.c_double)

# name -> (restype, argtypes); the full C API of include/femh.h
SIGNATURES = {
    "femh_ctx_create": (C.c_int, [C.c_int, C.POINTER(femh_allocator), P, C.POINTER(P)]),
    "femh_ctx_destroy": (None, [P]),
    "femh_last_error": (C.c_char_p, []),
    "femh_version": (C.c_int, []),
    "femh_validate_desc": (C.c_int, [C.POINTER(femh_problem_desc), C.c_char_p, C.c_size_t]),
    "femh_estimate_bytes": (C.c_int, [C.POINTER(femh_problem_desc), I32, I32, PI64]),
    "femh_validate_waves": (C.c_int, [I32, C.POINTER(femh_plane_wave), C.c_char_p, C.c_size_t]),
    "femh_problem_create": (C.c_int, [P, C.POINTER(femh_problem_desc), C.POINTER(P)]),
    "femh_problem_get_info": (C.c_int, [P, C.POINTER(femh_problem_info)]),
    "femh_problem_destroy": (None, [P]),
    "femh_import_bsr": (C.c_int, [P, I64, I64, P, P, P, C.POINTER(P)]),
    "femh_solve_rhs_dev": (C.c_int, [P, I32, P, C.POINTER(femh_solve_opts), P, C.POINTER(femh_solve_stats)]),
    "femh_spmv": (C.c_int, [P, I32, P, P, I32, PD]),
    "femh_solve": (C.c_int, [P, I32, C.POINTER(femh_plane_wave), C.POINTER(femh_solve_opts), P,
                             C.POINTER(femh_solve_stats)]),
    "femh_solve_dev": (C.c_int, [P, I32, C.POINTER(femh_plane_wave), C.POINTER(femh_solve_opts), P,
                                 C.POINTER(femh_solve_stats)]),
    "femh_solve_batched_dev": (C.c_int, [P, I32, C.POINTER(femh_plane_wave), C.POINTER(femh_solve_opts), P,
                                         C.POINTER(femh_solve_stats)]),
    "femh_export_bsr": (C.c_int, [P, P, P, P]),
    "femh_export_bsr_c64": (C.c_int, [P, P]),
    "femh_export_rhs": (C.c_int, [P, I32, C.POINTER(femh_plane_wave), P]),
    "femh_export_jacobi": (C.c_int, [P, P]),
    "femh_export_bic0": (C.c_int, [P, I32, C.POINTER(I64), P, P, P]),
    "femh_bic0_apply_dev": (C.c_int, [P, I32, P, P, I32, PD]),
    "femh_spmv_dev": (C.c_int, [P, I32, P, P, I32, PD]),
    "femh_spmm_dev": (C.c_int, [P, I32, I32, P, P, I32, PD]),
    "femh_spmm_tile": (C.c_int, [P, C.POINTER(I32), C.POINTER(I32)]),
    "femh_spmm_noalloc_dev": (C.c_int, [P, I32, I32, P, P]),
    "femh_spmv_half_dev": (C.c_int, [P, P, P, I32, PD]),
    "femh_spmm_set_tile": (C.c_int, [P, I32, I32]),
    "femh_bw_probe": (C.c_int, [P, I64, I32, PD]),
    "femh_profile_enable": (C.c_int, [P, I32]),
    "femh_profile_read": (C.c_int, [P, C.c_double * 4, C.c_int64 * 4, I32]),
    "femh_server_create": (C.c_int, [P, C.POINTER(femh_server_opts), C.POINTER(P)]),
    "femh_server_submit": (C.c_int, [P, C.POINTER(femh_problem_desc), I32, C.POINTER(femh_plane_wave),
                                     C.POINTER(femh_solve_opts), C.POINTER(C.c_uint64)]),
    "femh_server_poll": (C.c_int, [P, C.c_uint64, I32, P, C.POINTER(femh_solve_stats)]),
    "femh_server_cancel": (C.c_int, [P, C.c_uint64]),
    "femh_server_report_get": (C.c_int, [P, C.POINTER(femh_server_report)]),
    "femh_server_destroy": (None, [P]),
}

_lib = None

# Live handles, closed children-first at interpreter exit (before torch, whose
# allocator serves the library's device memory, is torn down).
_live_children = weakref.WeakSet()
_live_contexts = weakref.WeakSet()


def _close_all():
    for obj in list(_live_children):
        try:
            obj.close()
        except Exception:
            pass
    for obj in list(_live_contexts):
        try:
            obj.close()
        except Exception:
            pass


_atexit_registered = False


def _register_exit_cleanup():
    # registered after torch is imported, so it runs before torch's own
    # exit handlers (atexit runs in reverse order of registration)
    global _atexit_registered
    if not _atexit_registered:
        atexit.register(_close_all)
        _atexit_registered = True


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libfemh.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libfemh.so not found at {path}: build it with "
                          f"`python -m paper_0704_2344_amd.build` (there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def __getattr__(name):
    # femh.femh_solve etc. resolve to the C entry points
    if name.startswith("femh_") and name in SIGNATURES:
        return getattr(load(), name)
    raise AttributeError(name)


def last_error() -> str:
    return load().femh_last_error().decode()


def check(status: int, ok=(FEMH_OK,)):
    if status not in ok:
        raise FemhError(status, last_error())
    return status


# --------------------------------------------------------------- marshalling
def _c128_array(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


class _Keep:
    """Holds host arrays alive while a descriptor that points at them is used."""

    def __init__(self):
        self.items = []

    def add(self, x):
        self.items.append(x)
        return x


def make_desc(prob, device_arrays: Optional[dict] = None, keep: Optional[_Keep] = None,
              penalty_surface: int = 0) -> femh_problem_desc:
    """femh_problem_desc from a workloads.Problem.  With device_arrays
    ({"eps_r": tensor, "mu_r": tensor, "pec": tensor}) the descriptor points
    at device memory instead of the problem's host arrays; penalty_surface = 1
    asks for the printed penalty surface term averaged with its transpose."""
    d = femh_problem_desc()
    d.penalty_surface = penalty_surface
    d.nx, d.ny, d.nz = prob.nx, prob.ny, prob.nz
    for a in range(3):
        d.h[a] = prob.h[a]
        d.origin[a] = prob.origin[a]
    for f in range(6):
        d.outer_face[f] = int(prob.faces[f])
    d.k0 = prob.k0
    d.penalty_s = prob.penalty_s
    if device_arrays is not None:
        d.arrays_on_device = 1
        d.eps_r = device_arrays["eps_r"].data_ptr() if device_arrays.get("eps_r") is not None else None
        d.mu_r = device_arrays["mu_r"].data_ptr() if device_arrays.get("mu_r") is not None else None
        d.pec = device_arrays["pec"].data_ptr() if device_arrays.get("pec") is not None else None
        return d
    keep = keep if keep is not None else _Keep()
    eps = keep.add(_c128_array(prob.eps_r).reshape(-1))
    mu = keep.add(_c128_array(prob.mu_r).reshape(-1))
    pec = keep.add(np.ascontiguousarray(np.asarray(prob.pec, dtype=np.uint8).reshape(-1)))
    d.eps_r = eps.ctypes.data
    d.mu_r = mu.ctypes.data
    d.pec = pec.ctypes.data
    d._keep = keep  # noqa: SLF001  (keeps the arrays alive with the struct)
    return d


def make_waves(waves: Sequence) -> "C.Array":
    arr = (femh_plane_wave * len(waves))()
    for i, w in enumerate(waves):
        dvec = np.asarray(w.d, dtype=np.float64)
        pvec = np.asarray(w.p, dtype=np.complex128)
        for c in range(3):
            arr[i].d[c] = float(dvec[c])
            arr[i].p[c].re = float(pvec[c].real)
            arr[i].p[c].im = float(pvec[c].imag)
    return arr


def make_opts(precision=FEMH_FP64, rtol=1e-6, max_iter=0, inner_rtol=0.0, max_outer=0,
              check_every=0, precond=FEMH_PRECOND_JACOBI, precond_block=0) -> femh_solve_opts:
    o = femh_solve_opts()
    o.precision = precision
    o.precond = precond
    o.precond_block = precond_block
    o.rtol = rtol
    o.max_iter = max_iter
    o.inner_rtol = inner_rtol
    o.max_outer = max_outer
    o.check_every = check_every
    return o


def check_device_tensor(t, dtype, min_numel: int, device: int, what: str):
    """Refuse a tensor the C ABI cannot take safely: the entry points receive
    bare device pointers and no lengths, so a host tensor, a wrong element
    type, a strided view or a short buffer would turn into out-of-bounds
    device accesses.  Raises FemhError(FEMH_E_INVALID)."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise FemhError(FEMH_E_INVALID, f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.device.type != "cuda" or (t.device.index if t.device.index is not None else 0) != device:
        raise FemhError(FEMH_E_INVALID, f"{what}: tensor on {t.device}, the context is on cuda:{device}")
    if t.dtype != dtype:
        raise FemhError(FEMH_E_INVALID, f"{what}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise FemhError(FEMH_E_INVALID, f"{what}: tensor is not contiguous")
    if t.numel() < min_numel:
        raise FemhError(FEMH_E_INVALID, f"{what}: {t.numel()} elements, at least {min_numel} needed")


def _vector_dtype(precision):
    import torch

    if precision == FEMH_MIXED:
        return torch.complex64
    if precision in (FEMH_FP64, FEMH_MIXED_MATRIX):
        return torch.complex128
    raise FemhError(FEMH_E_INVALID, f"unknown precision {precision}")


# ----------------------------------------------------------- torch bridge
class TorchAllocator:
    """femh_allocator backed by torch's caching allocator on one device and
    stream."""

    def __init__(self, device: int = 0):
        import torch

        self.torch = torch
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)
        self.struct = femh_allocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, user):
        try:
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except Exception:  # out of memory -> NULL; the library reports FEMH_E_OOM
            return None

    def _do_free(self, ptr, user):
        self.torch.cuda.caching_allocator_delete(ptr)


class Context:
    """A femh context on a torch device, launching on torch's current stream."""

    def __init__(self, device: int = 0, use_torch: bool = True):
        self.lib = load()
        self.device = device
        h = C.c_void_p()
        self.handle = None
        if use_torch:
            import torch

            torch.cuda.set_device(device)
            self.allocator = TorchAllocator(device)
            stream = C.c_void_p(torch.cuda.current_stream(device).cuda_stream)
            check(self.lib.femh_ctx_create(device, C.byref(self.allocator.struct), stream, C.byref(h)))
        else:
            self.allocator = None
            check(self.lib.femh_ctx_create(device, None, None, C.byref(h)))
        self.handle = h
        self.children = weakref.WeakSet()
        _live_contexts.add(self)
        _register_exit_cleanup()

    def close(self):
        if self.handle:
            for ch in list(self.children):
                ch.close()
            self.lib.femh_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bw_probe(self, nbytes: int = 1 << 30, reps: int = 10) -> float:
        g = C.c_double()
        check(self.lib.femh_bw_probe(self.handle, nbytes, reps, C.byref(g)))
        return g.value

    def profile(self, on: bool):
        check(self.lib.femh_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self, reset=True):
        sec = (C.c_double * 4)()
        cnt = (C.c_int64 * 4)()
        check(self.lib.femh_profile_read(self.handle, sec, cnt, 1 if reset else 0))
        return list(sec), list(cnt)


class Problem:
    """An assembled problem resident on the device."""

    def __init__(self, ctx: Context, prob, device_arrays: Optional[dict] = None, penalty_surface: int = 0):
        self.ctx = ctx
        self.lib = ctx.lib
        self.spec = prob
        keep = _Keep()
        desc = make_desc(prob, device_arrays, keep, penalty_surface)
        h = C.c_void_p()
        check(self.lib.femh_problem_create(ctx.handle, C.byref(desc), C.byref(h)))
        self.handle = h
        ctx.children.add(self)
        _live_children.add(self)
        info = femh_problem_info()
        check(self.lib.femh_problem_get_info(h, C.byref(info)))
        self.info = info
        self.n_nodes = info.n_nodes
        self.n_unknowns = info.n_unknowns
        self.nnzb = info.nnzb
        self.grid_nodes = info.grid_nodes

    @classmethod
    def from_bsr(cls, ctx: Context, row_ptr, col_idx, vals):
        """A problem made from an assembled block matrix (femh_import_bsr):
        row_ptr [nb + 1], col_idx [nnzb], vals [nnzb, 3, 3] complex128, host
        arrays.  It has no mesh: solve it with solve_rhs_dev."""
        rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int32))
        ci = np.ascontiguousarray(np.asarray(col_idx, dtype=np.int32))
        v = np.ascontiguousarray(np.asarray(vals, dtype=np.complex128))
        if v.shape != (len(ci), 3, 3) or len(rp) < 2:
            raise FemhError(FEMH_E_INVALID, f"vals must be [nnzb, 3, 3] with nnzb = len(col_idx) (got {v.shape})")
        self = cls.__new__(cls)
        self.ctx = ctx
        self.lib = ctx.lib
        self.spec = None
        h = C.c_void_p()
        check(self.lib.femh_import_bsr(ctx.handle, len(rp) - 1, len(ci), rp.ctypes.data, ci.ctypes.data,
                                       v.ctypes.data, C.byref(h)))
        self.handle = h
        ctx.children.add(self)
        _live_children.add(self)
        info = femh_problem_info()
        check(self.lib.femh_problem_get_info(h, C.byref(info)))
        self.info = info
        self.n_nodes = info.n_nodes
        self.n_unknowns = info.n_unknowns
        self.nnzb = info.nnzb
        self.grid_nodes = info.grid_nodes
        return self

    def solve_rhs_dev(self, b, x, **opt_kw):
        """Solve A x = b for given right-hand sides: b and x complex128 device
        tensors [nrhs, n_unknowns] (or [n_unknowns]); x is overwritten."""
        import torch

        nrhs = 1 if b.dim() == 1 else b.shape[0]
        n = nrhs * self.n_unknowns
        check_device_tensor(b, torch.complex128, n, self.ctx.device, "solve_rhs_dev b")
        check_device_tensor(x, torch.complex128, n, self.ctx.device, "solve_rhs_dev x")
        o = make_opts(**opt_kw)
        stats = (femh_solve_stats * nrhs)()
        st = self.lib.femh_solve_rhs_dev(self.handle, nrhs, b.data_ptr(), C.byref(o), x.data_ptr(), stats)
        check(st, ok=(FEMH_OK, FEMH_E_NOT_CONVERGED, FEMH_E_BREAKDOWN))
        return [s.as_dict() for s in stats], st

    def spmv(self, x, precision=FEMH_FP64, reps=1):
        """Host-vector product (femh_spmv): returns (y, mean device seconds)."""
        xv = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
        if xv.shape != (self.n_unknowns,):
            raise FemhError(FEMH_E_INVALID, f"x must have {self.n_unknowns} entries")
        y = np.zeros_like(xv)
        t = C.c_double()
        check(self.lib.femh_spmv(self.handle, precision, xv.ctypes.data, y.ctypes.data, reps, C.byref(t)))
        return y, t.value

    def close(self):
        if self.handle:
            self.lib.femh_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def grid_shape(self, nrhs):
        s = self.spec
        return (nrhs, s.nz + 1, s.ny + 1, s.nx + 1, 3)

    def solve(self, waves, **opt_kw):
        """Host-output solve: returns (H[nrhs, nz+1, ny+1, nx+1, 3], stats list, status)."""
        w = make_waves(waves)
        o = make_opts(**opt_kw)
        out = np.zeros(self.grid_shape(len(waves)), dtype=np.complex128)
        stats = (femh_solve_stats * len(waves))()
        st = self.lib.femh_solve(self.handle, len(waves), w, C.byref(o), out.ctypes.data, stats)
        check(st, ok=(FEMH_OK, FEMH_E_NOT_CONVERGED, FEMH_E_BREAKDOWN))
        return out, [s.as_dict() for s in stats], st

    def solve_dev(self, waves, out_tensor, batched: bool = False, **opt_kw):
        """Device-output solve into a complex128 torch tensor of grid shape."""
        import torch

        check_device_tensor(out_tensor, torch.complex128, len(waves) * 3 * self.grid_nodes, self.ctx.device,
                            "solve_dev output")
        w = make_waves(waves)
        o = make_opts(**opt_kw)
        stats = (femh_solve_stats * len(waves))()
        fn = self.lib.femh_solve_batched_dev if batched else self.lib.femh_solve_dev
        st = fn(self.handle, len(waves), w, C.byref(o), out_tensor.data_ptr(), stats)
        check(st, ok=(FEMH_OK, FEMH_E_NOT_CONVERGED, FEMH_E_BREAKDOWN))
        return [s.as_dict() for s in stats], st

    def export_bsr(self):
        row_ptr = np.zeros(self.n_nodes + 1, dtype=np.int32)
        col = np.zeros(self.nnzb, dtype=np.int32)
        vals = np.zeros((self.nnzb, 3, 3), dtype=np.complex128)
        check(self.lib.femh_export_bsr(self.handle, row_ptr.ctypes.data, col.ctypes.data, vals.ctypes.data))
        return row_ptr, col, vals

    def export_bsr_c64(self):
        vals = np.zeros((self.nnzb, 3, 3), dtype=np.complex64)
        check(self.lib.femh_export_bsr_c64(self.handle, vals.ctypes.data))
        return vals

    def export_rhs(self, waves):
        w = make_waves(waves)
        b = np.zeros((len(waves), self.n_unknowns), dtype=np.complex128)
        check(self.lib.femh_export_rhs(self.handle, len(waves), w, b.ctypes.data))
        return b

    def export_jacobi(self):
        d = np.zeros(self.n_unknowns, dtype=np.complex128)
        check(self.lib.femh_export_jacobi(self.handle, d.ctypes.data))
        return d

    def export_bic0(self, nodes_per_block=4):
        """The block incomplete Cholesky factor L (scalar CSR: row_ptr, col,
        vals; columns ascending, diagonal last) for blocks of nodes_per_block
        nodes, built on the device if needed."""
        nnz = I64(0)
        check(self.lib.femh_export_bic0(self.handle, nodes_per_block, C.byref(nnz), None, None, None))
        row_ptr = np.zeros(self.n_unknowns + 1, dtype=np.int32)
        col = np.zeros(nnz.value, dtype=np.int32)
        vals = np.zeros(nnz.value, dtype=np.complex128)
        check(self.lib.femh_export_bic0(self.handle, nodes_per_block, C.byref(nnz), row_ptr.ctypes.data,
                                        col.ctypes.data, vals.ctypes.data))
        return row_ptr, col, vals

    def bic0_apply_dev(self, r, z, nodes_per_block=4, reps=1):
        """z = (L L^T)^-1 r with the block incomplete Cholesky factor (device
        complex128 tensors [n_unknowns]); returns the mean kernel seconds."""
        import torch

        check_device_tensor(r, torch.complex128, self.n_unknowns, self.ctx.device, "bic0_apply_dev r")
        check_device_tensor(z, torch.complex128, self.n_unknowns, self.ctx.device, "bic0_apply_dev z")
        t = C.c_double()
        check(self.lib.femh_bic0_apply_dev(self.handle, nodes_per_block, r.data_ptr(), z.data_ptr(), reps,
                                           C.byref(t)))
        return t.value

    def spmv_dev(self, x, y, precision=FEMH_FP64, reps=1):
        dt = _vector_dtype(precision)
        check_device_tensor(x, dt, self.n_unknowns, self.ctx.device, "spmv_dev x")
        check_device_tensor(y, dt, self.n_unknowns, self.ctx.device, "spmv_dev y")
        t = C.c_double()
        check(self.lib.femh_spmv_dev(self.handle, precision, x.data_ptr(), y.data_ptr(), reps, C.byref(t)))
        return t.value

    def spmv_half_dev(self, x, y, reps=1):
        import torch

        check_device_tensor(x, torch.complex128, self.n_unknowns, self.ctx.device, "spmv_half_dev x")
        check_device_tensor(y, torch.complex128, self.n_unknowns, self.ctx.device, "spmv_half_dev y")
        t = C.c_double()
        check(self.lib.femh_spmv_half_dev(self.handle, x.data_ptr(), y.data_ptr(), reps, C.byref(t)))
        return t.value

    def spmm_tile(self):
        kind, blocks = I32(), I32()
        check(self.lib.femh_spmm_tile(self.handle, C.byref(kind), C.byref(blocks)))
        return kind.value, blocks.value

    def spmm_set_tile(self, kind, blocks):
        check(self.lib.femh_spmm_set_tile(self.handle, kind, blocks))

    def spmm_dev(self, X, Y, reps=1, precision=FEMH_MIXED_MATRIX):
        import torch

        if X.dim() != 2 or Y.shape != X.shape or X.shape[0] != self.n_unknowns or not 1 <= X.shape[1] <= 64:
            raise FemhError(FEMH_E_INVALID, f"spmm_dev: X and Y must both be [{self.n_unknowns}, ncols] with "
                                            f"1 <= ncols <= 64 (got {tuple(X.shape)} and {tuple(Y.shape)})")
        check_device_tensor(X, torch.complex128, X.numel(), self.ctx.device, "spmm_dev X")
        check_device_tensor(Y, torch.complex128, X.numel(), self.ctx.device, "spmm_dev Y")
        t = C.c_double()
        check(self.lib.femh_spmm_dev(self.handle, precision, X.shape[1], X.data_ptr(), Y.data_ptr(), reps,
                                     C.byref(t)))
        return t.value


class Server:
    """Continuous-batching request loop (femh_server_*)."""

    def __init__(self, ctx: Context, hbm_budget_bytes=0, max_slots=0, chunk_iters=0, batch_rhs=False):
        self.ctx = ctx
        self.lib = ctx.lib
        o = femh_server_opts(hbm_budget_bytes, max_slots, chunk_iters, int(bool(batch_rhs)), 0)
        h = C.c_void_p()
        check(self.lib.femh_server_create(ctx.handle, C.byref(o), C.byref(h)))
        self.handle = h
        ctx.children.add(self)
        _live_children.add(self)

    def submit(self, prob, waves, penalty_surface: int = 0, **opt_kw) -> int:
        keep = _Keep()
        desc = make_desc(prob, None, keep, penalty_surface)
        w = make_waves(waves)
        o = make_opts(**opt_kw)
        t = C.c_uint64()
        check(self.lib.femh_server_submit(self.handle, C.byref(desc), len(waves), w, C.byref(o), C.byref(t)))
        return t.value

    def poll(self, ticket, nrhs, grid_shape=None, timeout_ms=-1, want_field=True):
        out = np.zeros(grid_shape, dtype=np.complex128) if (want_field and grid_shape) else None
        stats = (femh_solve_stats * nrhs)()
        st = self.lib.femh_server_poll(self.handle, ticket, timeout_ms,
                                       out.ctypes.data if out is not None else None, stats)
        return st, out, [s.as_dict() for s in stats]

    def cancel(self, ticket):
        return self.lib.femh_server_cancel(self.handle, ticket)

    def report(self):
        r = femh_server_report()
        check(self.lib.femh_server_report_get(self.handle, C.byref(r)))
        return r.as_dict()

    def close(self):
        if self.handle:
            self.lib.femh_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

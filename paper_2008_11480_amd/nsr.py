"""Thin Python binding of libnsr (include/nsr.h), argument marshalling only.

Every step of the solve runs in the HIP library; this module converts torch
tensors to device pointers and streams, and C structs to Python objects.
Importing it does not load the library; the first call does, and raises if
``libnsr.so`` has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnsr.so")
_lib = None

# ns_status
NS_OK, NS_EINVAL, NS_ENOTSPD, NS_EDIVERGED, NS_ENOCONV = 0, -1, -2, -3, -4
NS_ENOMEM, NS_EHIP, NS_EBUSY, NS_EPRECISION, NS_ESTATE = -5, -6, -7, -8, -9
# ns_precision
PREC_FP64, PREC_FP32, PREC_MIXED_BF16, PREC_MIXED_SPLIT = 0, 1, 2, 3
# ns_scale
SCALE_FROBENIUS, SCALE_INF_HALF, SCALE_DIAG = 0, 1, 2
# ns_factorization
FACT = {"horner": 0, "squaring": 1, "table": 2, "unified": 3, "unified_plus1": 4,
        "composite_double": 5, "sri": 6, "composite_general": 7}
# ns_stop_reason
STOP_NAMES = {0: "none", 1: "f_tol", 2: "floor", 3: "k_max", 4: "diverged", 5: "resid_tol",
              6: "refine_max", 7: "refine_stall", 8: "precision"}

HIST_F = 65
HIST_R = 200

# Every exported symbol of include/nsr.h, for the load check.
EXPORTS = (
    "ns_workspace_bytes", "ns_create", "ns_destroy", "ns_bind", "ns_init_scale", "ns_step",
    "ns_get_G", "ns_get_F", "ns_richardson_step", "richardson_ns_solve", "ns_set_symmetric",
    "ns_timing_enable", "ns_set_composite_rates",
    "ns_timing_read", "ns_timing_reset", "ns_gemm_f64", "ns_gemm_f64_partials",
    "ns_gemm_f64_scratch_bytes", "ns_gemm_f64_ws",
    "ns_gemm_f32", "ns_gemm_bf16_nt", "ns_gemm_lp_partials", "ns_gemm_f32_split",
    "ns_gemm_f32_split_scratch_bytes", "ns_gemm_bf16_nt_ws", "ns_gemm_bf16_scratch_bytes",
    "ns_gemm_f32_split_noalloc", "ns_tile_set", "ns_tile_get",
    "ns_batch_workspace_bytes", "ns_batch_create", "ns_batch_set_launch", "ns_batch_set_lockstep",
    "ns_batch_submit",
    "ns_batch_poll", "ns_batch_autotune", "ns_batch_timeline", "ns_batch_destroy",
    "ns_batch_set_ledger", "ns_ledger_create", "ns_ledger_admit", "ns_ledger_release",
    "ns_ledger_query", "ns_ledger_destroy", "ns_solve_footprint",
    "ns_status_string", "ns_last_error", "ns_version",
)


class NSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"nsr error {status}: {msg}")
        self.status = status


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int), ("factorization", ctypes.c_int), ("p", ctypes.c_int),
        ("w", ctypes.c_int), ("k_max", ctypes.c_int), ("refine_max", ctypes.c_int),
        ("floor_detect", ctypes.c_int), ("scale", ctypes.c_int), ("eps", ctypes.c_double),
        ("f_tol", ctypes.c_double), ("resid_tol", ctypes.c_double), ("theta0_mode", ctypes.c_int),
        ("accel_q", ctypes.c_int), ("init_order", ctypes.c_int), ("init_p", ctypes.c_int),
        ("init_w", ctypes.c_int), ("graph", ctypes.c_int),
    ]


class SolveReportC(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("ns_stop", ctypes.c_int), ("refine_stop", ctypes.c_int),
        ("ns_steps", ctypes.c_int), ("refine_steps", ctypes.c_int), ("precision", ctypes.c_int),
        ("alpha", ctypes.c_double), ("rel_resid", ctypes.c_double), ("mmm", ctypes.c_int64),
        ("gemm_flop", ctypes.c_double), ("n_fnorm", ctypes.c_int),
        ("fnorm_hist", ctypes.c_double * HIST_F), ("n_resid", ctypes.c_int),
        ("resid_hist", ctypes.c_double * HIST_R),
    ]


@dataclasses.dataclass
class SolveReport:
    status: int
    ns_stop: str
    refine_stop: str
    ns_steps: int
    refine_steps: int
    precision: int
    alpha: float
    rel_resid: float
    mmm: int
    gemm_flop: float
    fnorm_hist: list
    resid_hist: list


def lib() -> ctypes.CDLL:
    """Load libnsr.so (once).  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run paper_2008_11480_amd.build.build()")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    pd = ctypes.POINTER(ctypes.c_double)
    sig = {
        "ns_workspace_bytes": (ctypes.c_size_t, [i64, ci, ci]),
        "ns_create": (ci, [ci, vp, i64, ci, vp, ctypes.c_size_t, ctypes.POINTER(vp)]),
        "ns_destroy": (ci, [vp]),
        "ns_bind": (ci, [vp, vp, i64]),
        "ns_init_scale": (ci, [vp, ci, dbl, pd, pd]),
        "ns_step": (ci, [vp, ci, ci, ci, ci, pd]),
        "ns_get_G": (ci, [vp, vp, i64]),
        "ns_get_F": (ci, [vp, vp, i64]),
        "ns_richardson_step": (ci, [vp, vp, vp, pd]),
        "richardson_ns_solve": (ci, [vp, vp, vp, ctypes.POINTER(SolveOpts),
                                     ctypes.POINTER(SolveReportC)]),
        "ns_set_symmetric": (ci, [vp, ci]),
        "ns_set_composite_rates": (ci, [vp, ci, vp]),
        "ns_timing_enable": (ci, [vp, ci]),
        "ns_timing_read": (ci, [vp, ci, ctypes.POINTER(i64), pd, pd]),
        "ns_timing_reset": (ci, [vp]),
        "ns_gemm_f64": (ci, [vp, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64,
                             dbl, dbl, ci, vp]),
        "ns_gemm_f64_partials": (i64, [i64, i64, ci]),
        "ns_gemm_f64_scratch_bytes": (ctypes.c_size_t, [i64, i64, i64, ci]),
        "ns_gemm_f64_ws": (ci, [vp, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64,
                                dbl, dbl, ci, vp, ctypes.c_size_t, vp]),
        "ns_gemm_f32": (ci, [vp, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp,
                             i64, ctypes.c_float, ctypes.c_float, vp]),
        "ns_gemm_bf16_nt": (ci, [vp, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64,
                                 vp, i64, ctypes.c_float, ctypes.c_float, vp]),
        "ns_gemm_lp_partials": (i64, [i64, i64]),
        "ns_gemm_f32_split": (ci, [vp, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp,
                                   i64, vp, i64, ctypes.c_float, ctypes.c_float, vp, vp,
                                   ctypes.c_size_t]),
        "ns_gemm_f32_split_scratch_bytes": (ctypes.c_size_t, [i64, i64, i64]),
        "ns_tile_set": (ci, [ci, ci, ci]),
        "ns_tile_get": (ci, [ci, ci]),
        "ns_gemm_f32_split_noalloc": (ci, [vp, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp,
                                           i64, vp, i64, vp, i64, ctypes.c_float,
                                           ctypes.c_float, vp]),
        "ns_gemm_bf16_nt_ws": (ci, [vp, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp,
                                    i64, vp, i64, ctypes.c_float, ctypes.c_float, ci, vp, vp,
                                    ctypes.c_size_t]),
        "ns_gemm_bf16_scratch_bytes": (ctypes.c_size_t, [i64, i64, i64, ci]),
        "ns_batch_workspace_bytes": (ctypes.c_size_t, [i64, ci, ci]),
        "ns_batch_create": (ci, [ci, vp, i64, ci, ci, ci, vp, ctypes.c_size_t,
                                 ctypes.POINTER(vp)]),
        "ns_batch_set_launch": (ci, [vp, ci, ci]),
        "ns_batch_set_lockstep": (ci, [vp, ci]),
        "ns_batch_submit": (ci, [vp, ci, vp, vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                                 ctypes.POINTER(ctypes.c_uint64)]),
        "ns_batch_poll": (ci, [vp, ctypes.c_uint64, ci, vp]),
        "ns_batch_autotune": (ci, [vp, ci, vp, vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                                   ctypes.POINTER(ci), ctypes.POINTER(ci), pd]),
        "ns_batch_timeline": (ci, [vp, ctypes.c_uint64, vp, vp]),
        "ns_batch_destroy": (ci, [vp]),
        "ns_batch_set_ledger": (ci, [vp, vp]),
        "ns_ledger_create": (ci, [ctypes.c_size_t, ctypes.POINTER(vp)]),
        "ns_ledger_admit": (ci, [vp, ctypes.c_size_t]),
        "ns_ledger_release": (ci, [vp, ctypes.c_size_t]),
        "ns_ledger_query": (ci, [vp, ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_uint64),
                                 ctypes.POINTER(ctypes.c_uint64)]),
        "ns_ledger_destroy": (ci, [vp]),
        "ns_solve_footprint": (ctypes.c_size_t, [i64, ci, ci]),
        "ns_status_string": (ctypes.c_char_p, [ci]),
        "ns_last_error": (ctypes.c_char_p, []),
        "ns_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int) -> int:
    if status != NS_OK:
        msg = lib().ns_last_error().decode(errors="replace")
        raise NSError(status, msg)
    return status


def _ptr(t) -> int | None:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream_handle(stream) -> int | None:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) or None


def _require_cuda_f64(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")


def workspace_bytes(n: int, precision: int = PREC_FP64, composite: int = 0) -> int:
    """Workspace of a solver; ``composite``: 0 (classical / table forms),
    1 or True (also double Newton-Schulz, [sri], one-loop general composite),
    2 or 3 (general composite with that many loops)."""
    return int(lib().ns_workspace_bytes(int(n), int(precision), int(composite)))


class Solver:
    """One ``ns_solver`` handle with its workspace (allocated by torch)."""

    def __init__(self, n: int, precision: int = PREC_FP64, composite: int = 1,
                 device: int | None = None, stream=None):
        import torch
        L = lib()
        self.n = int(n)
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = workspace_bytes(n, precision, composite)
        if nbytes == 0:
            raise NSError(NS_EINVAL, "unsupported size/precision")
        self.precision = int(precision)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8,
                                     device=f"cuda:{self.device}")
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        h = ctypes.c_void_p()
        check(L.ns_create(self.device, _stream_handle(self.stream), self.n, int(precision),
                          aligned, nbytes, ctypes.byref(h)))
        self._h = h
        self._A = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ns_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_symmetric(self, enable: bool):
        check(lib().ns_set_symmetric(self._h, 1 if enable else 0))

    def set_composite_rates(self, rates):
        """Loop orders m_i of the general composite form (``form="composite_general"``)."""
        arr = (ctypes.c_int * len(rates))(*[int(m) for m in rates])
        check(lib().ns_set_composite_rates(self._h, len(rates), arr))

    def bind(self, A):
        _require_cuda_f64(A, "A")
        if A.dim() != 2 or A.shape[0] != self.n or A.shape[1] != self.n or A.stride(1) != 1:
            raise ValueError("A must be n x n with unit column stride")
        self._A = A
        check(lib().ns_bind(self._h, _ptr(A), A.stride(0)))

    def init_scale(self, scale: int = SCALE_FROBENIUS, eps: float = 0.0):
        a, f = ctypes.c_double(), ctypes.c_double()
        check(lib().ns_init_scale(self._h, int(scale), float(eps), ctypes.byref(a),
                                  ctypes.byref(f)))
        return a.value, f.value

    def step(self, order: int, form: str = "squaring", p: int = 0, w: int = 0) -> float:
        f = ctypes.c_double()
        check(lib().ns_step(self._h, int(order), FACT[form], int(p), int(w), ctypes.byref(f)))
        return f.value

    def get_G(self, out=None):
        import torch
        if out is None:
            out = torch.empty(self.n, self.n, dtype=torch.float64, device=f"cuda:{self.device}")
        check(lib().ns_get_G(self._h, _ptr(out), out.stride(0)))
        return out

    def get_F(self, out=None):
        import torch
        if out is None:
            out = torch.empty(self.n, self.n, dtype=torch.float64, device=f"cuda:{self.device}")
        check(lib().ns_get_F(self._h, _ptr(out), out.stride(0)))
        return out

    def richardson_step(self, b, theta) -> float:
        _require_cuda_f64(b, "b")
        _require_cuda_f64(theta, "theta")
        r = ctypes.c_double()
        check(lib().ns_richardson_step(self._h, _ptr(b), _ptr(theta), ctypes.byref(r)))
        return r.value

    def solve(self, b, theta, order: int | str = 8, form: str = "squaring", p: int = 0,
              w: int = 0, k_max: int = 64, refine_max: int = 64, floor_detect: bool = True,
              scale: int = SCALE_FROBENIUS, eps: float = 0.0, f_tol: float = 0.0,
              resid_tol: float = 1e-12, theta0_mode: int = 0, accel_q: int = 0,
              init_order: int = 0, init_p: int = 0, init_w: int = 0, graph: bool = False,
              raise_on_error: bool = True, kappa: float | None = None, table=None):
        """``richardson_ns_solve``.  ``order="auto"``: the program (order, form,
        p, w) comes from ``table`` (default: ``autotune.default_table()``),
        tuned for this solver's N and precision and for ``kappa`` (None: the
        table's hint); ``form`` is then ignored."""
        _require_cuda_f64(b, "b")
        _require_cuda_f64(theta, "theta")
        if order == "auto":
            from . import autotune
            prog = (table or autotune.default_table()).lookup(self.n, kappa, self.precision)
            order, form, p, w = prog.order, prog.form, prog.p, prog.w
        o = SolveOpts(order=order, factorization=FACT[form], p=p, w=w, k_max=k_max,
                      refine_max=refine_max, floor_detect=1 if floor_detect else 0, scale=scale,
                      eps=eps, f_tol=f_tol, resid_tol=resid_tol, theta0_mode=theta0_mode,
                      accel_q=accel_q, init_order=init_order, init_p=init_p, init_w=init_w,
                      graph=1 if graph else 0)
        rep = SolveReportC()
        st = lib().richardson_ns_solve(self._h, _ptr(b), _ptr(theta), ctypes.byref(o),
                                       ctypes.byref(rep))
        if st not in (NS_OK, NS_ENOCONV, NS_EDIVERGED):
            check(st)                       # argument / state / HIP errors always raise
        if st == NS_EDIVERGED and raise_on_error:
            check(st)
        return SolveReport(
            status=rep.status, ns_stop=STOP_NAMES.get(rep.ns_stop, "?"),
            refine_stop=STOP_NAMES.get(rep.refine_stop, "?"), ns_steps=rep.ns_steps,
            refine_steps=rep.refine_steps, precision=rep.precision, alpha=rep.alpha,
            rel_resid=rep.rel_resid, mmm=rep.mmm, gemm_flop=rep.gemm_flop,
            fnorm_hist=list(rep.fnorm_hist[:rep.n_fnorm]),
            resid_hist=list(rep.resid_hist[:rep.n_resid]))

    # timing -------------------------------------------------------------
    def timing(self, enable: bool):
        check(lib().ns_timing_enable(self._h, 1 if enable else 0))

    def timing_reset(self):
        check(lib().ns_timing_reset(self._h))

    def timing_read(self, kind: int = 0):
        n = ctypes.c_int64()
        ms, fl = ctypes.c_double(), ctypes.c_double()
        check(lib().ns_timing_read(self._h, int(kind), ctypes.byref(n), ctypes.byref(ms),
                                   ctypes.byref(fl)))
        return n.value, ms.value, fl.value


GEMM_SYMMETRIC = 1


def gemm_f64_scratch_bytes(m: int, n: int, k: int, symmetric: bool = False) -> int:
    """Scratch that lets :func:`gemm_f64` split the K range of its last,
    partial round of tiles (0: no split for this shape)."""
    return int(lib().ns_gemm_f64_scratch_bytes(m, n, k, GEMM_SYMMETRIC if symmetric else 0))


def gemm_f64(X, Y, D=None, E1=None, E2=None, diag: float = 0.0, scale: float = 1.0,
             want_sumsq: bool = False, symmetric: bool = False, stream=None, scratch=None):
    """``D = diag I + scale X Y + E1 + E2`` through the library's MFMA GEMM
    (``symmetric``: upper tiles computed, lower triangle mirrored; ``scratch``:
    a device tensor for the split-K tail, see :func:`gemm_f64_scratch_bytes`)."""
    import torch
    for t, nm in ((X, "X"), (Y, "Y")):
        _require_cuda_f64(t, nm)
    m, k = X.shape
    k2, n = Y.shape
    if k2 != k:
        raise ValueError("inner dimensions differ")
    if D is None:
        D = torch.empty(m, n, dtype=torch.float64, device=X.device)
    flags = GEMM_SYMMETRIC if symmetric else 0
    ss = None
    if want_sumsq:
        ss = torch.zeros(1 + int(lib().ns_gemm_f64_partials(m, n, flags)), dtype=torch.float64,
                         device=X.device)
    sbytes = 0 if scratch is None else scratch.numel() * scratch.element_size()
    check(lib().ns_gemm_f64_ws(_stream_handle(stream), m, n, k, _ptr(X), X.stride(0), _ptr(Y),
                               Y.stride(0), _ptr(D), D.stride(0), _ptr(E1),
                               E1.stride(0) if E1 is not None else 0, _ptr(E2),
                               E2.stride(0) if E2 is not None else 0, float(diag), float(scale),
                               flags, _ptr(scratch), sbytes, _ptr(ss)))
    return (D, ss[0]) if want_sumsq else D


def _report_from_c(rep) -> SolveReport:
    return SolveReport(
        status=rep.status, ns_stop=STOP_NAMES.get(rep.ns_stop, "?"),
        refine_stop=STOP_NAMES.get(rep.refine_stop, "?"), ns_steps=rep.ns_steps,
        refine_steps=rep.refine_steps, precision=rep.precision, alpha=rep.alpha,
        rel_resid=rep.rel_resid, mmm=rep.mmm, gemm_flop=rep.gemm_flop,
        fnorm_hist=list(rep.fnorm_hist[:rep.n_fnorm]),
        resid_hist=list(rep.resid_hist[:rep.n_resid]))


class PackedSystems:
    """A batch's systems stored back to back in three flat float64 device
    tensors: ``A`` holds each ``A_i`` row-major (``n_i x n_i``, leading
    dimension ``n_i``), ``b`` and ``theta`` the vectors.  A submission of a
    packed batch computes its pointer arrays with numpy from the three base
    addresses instead of one call per tensor (`Batch.submit_packed`)."""

    def __init__(self, ns, device=None):
        import torch
        self.n = np.ascontiguousarray(np.asarray(ns, dtype=np.int64))
        if self.n.ndim != 1 or (self.n < 1).any():
            raise ValueError("sizes must be a 1-d list of positive integers")
        sq = self.n * self.n
        self.a_off = np.concatenate(([0], np.cumsum(sq)[:-1])).astype(np.int64)
        self.v_off = np.concatenate(([0], np.cumsum(self.n)[:-1])).astype(np.int64)
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.A = torch.empty(int(sq.sum()), dtype=torch.float64, device=dev)
        self.b = torch.empty(int(self.n.sum()), dtype=torch.float64, device=dev)
        self.theta = torch.zeros(int(self.n.sum()), dtype=torch.float64, device=dev)

    def __len__(self) -> int:
        return int(self.n.size)

    def A_of(self, i: int):
        k, o = int(self.n[i]), int(self.a_off[i])
        return self.A[o:o + k * k].view(k, k)

    def b_of(self, i: int):
        return self.b[int(self.v_off[i]):int(self.v_off[i] + self.n[i])]

    def theta_of(self, i: int):
        return self.theta[int(self.v_off[i]):int(self.v_off[i] + self.n[i])]

    @classmethod
    def from_host(cls, As, bs, device=None):
        """Pack host (numpy) systems; theta starts at zero."""
        import torch
        P = cls([a.shape[0] for a in As], device)
        P.A.copy_(torch.from_numpy(np.concatenate([np.ascontiguousarray(a, dtype=np.float64)
                                                   .ravel() for a in As])))
        P.b.copy_(torch.from_numpy(np.concatenate([np.asarray(b, dtype=np.float64)
                                                   for b in bs])))
        return P

    def pointers(self):
        """(n, A pointers, b pointers, theta pointers) as numpy arrays."""
        pa = (self.A.data_ptr() + 8 * self.a_off).astype(np.uint64)
        pb = (self.b.data_ptr() + 8 * self.v_off).astype(np.uint64)
        pt = (self.theta.data_ptr() + 8 * self.v_off).astype(np.uint64)
        return self.n, pa, pb, pt


_REPORT_COLUMNS = ("status", "precision", "ns_steps", "refine_steps", "ns_stop", "refine_stop",
                   "alpha", "rel_resid", "mmm", "gemm_flop")


def _report_dtype():
    """numpy view of SolveReportC's scalar fields (offsets from ctypes)."""
    kinds = {ctypes.c_int: np.int32, ctypes.c_int64: np.int64, ctypes.c_double: np.float64}
    types = dict(SolveReportC._fields_)
    return np.dtype({"names": list(_REPORT_COLUMNS),
                     "formats": [kinds[types[f]] for f in _REPORT_COLUMNS],
                     "offsets": [getattr(SolveReportC, f).offset for f in _REPORT_COLUMNS],
                     "itemsize": ctypes.sizeof(SolveReportC)})


def _report_arrays(reps, count: int) -> dict:
    """Columns of a ctypes SolveReportC array as numpy arrays (no per-report
    Python objects)."""
    arr = np.frombuffer(reps, dtype=_report_dtype(), count=count)
    return {f: arr[f].copy() for f in _REPORT_COLUMNS}


class Ledger:
    """``ns_ledger``: HBM-footprint admission (host memory only, thread-safe)."""

    def __init__(self, budget_bytes: int):
        h = ctypes.c_void_p()
        check(lib().ns_ledger_create(int(budget_bytes), ctypes.byref(h)))
        self._h = h

    def admit(self, nbytes: int) -> bool:
        """True if admitted; False if over the budget now (NS_ENOMEM).  Raises
        NSError(NS_EINVAL) for a footprint above the whole budget."""
        st = lib().ns_ledger_admit(self._h, int(nbytes))
        if st == NS_ENOMEM:
            return False
        check(st)
        return True

    def release(self, nbytes: int):
        check(lib().ns_ledger_release(self._h, int(nbytes)))

    def query(self) -> dict:
        v = [ctypes.c_size_t() for _ in range(3)] + [ctypes.c_uint64() for _ in range(2)]
        check(lib().ns_ledger_query(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("in_use", "peak", "budget", "admitted", "refused"),
                        (x.value for x in v)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ns_ledger_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_footprint(n: int, precision: int = PREC_FP64, composite: int = 0) -> int:
    """``ns_solve_footprint``: workspace plus A, b, theta of one solve."""
    return int(lib().ns_solve_footprint(int(n), int(precision), int(composite)))


class Batch:
    """``ns_batch`` handle: many independent systems per persistent launch."""

    def __init__(self, max_n: int, max_count: int, slots: int | None = None,
                 precision: int = PREC_FP32, device: int | None = None, stream=None):
        import torch
        L = lib()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if slots is None:
            cus = torch.cuda.get_device_properties(self.device).multi_processor_count
            slots = min(max_count, 4 * cus)
        self.max_n, self.max_count, self.slots = int(max_n), int(max_count), int(slots)
        nbytes = int(L.ns_batch_workspace_bytes(self.max_n, self.max_count, self.slots))
        if nbytes == 0:
            raise NSError(NS_EINVAL, "bad batch sizes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8,
                                     device=f"cuda:{self.device}")
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        h = ctypes.c_void_p()
        check(L.ns_batch_create(self.device, _stream_handle(self.stream), self.max_n,
                                self.max_count, self.slots, int(precision), aligned, nbytes,
                                ctypes.byref(h)))
        self._h = h
        self._keep = None
        self._count = 0

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ns_batch_destroy(self._h)
            self._h = None

    def set_ledger(self, ledger: "Ledger | None"):
        """Admit each submission's A, b, theta bytes through ``ledger``
        (``submit`` then raises NSError(NS_ENOMEM) when over the budget)."""
        check(lib().ns_batch_set_ledger(self._h, ledger._h if ledger is not None else None))
        self._ledger = ledger

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _arrays(As, bs, thetas):
        count = len(As)
        if not (len(bs) == count and len(thetas) == count):
            raise ValueError("A, b, theta lists differ in length")
        n = (ctypes.c_int64 * count)()
        lda = (ctypes.c_int64 * count)()
        pa = (ctypes.c_void_p * count)()
        pb = (ctypes.c_void_p * count)()
        pt = (ctypes.c_void_p * count)()
        for i, (A, b, t) in enumerate(zip(As, bs, thetas)):
            _require_cuda_f64(A, "A")
            _require_cuda_f64(b, "b")
            _require_cuda_f64(t, "theta")
            if A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1:
                raise ValueError("each A must be square with unit column stride")
            if b.numel() != A.shape[0] or t.numel() != A.shape[0]:
                raise ValueError("b / theta length must match A")
            n[i], lda[i] = A.shape[0], A.stride(0)
            pa[i], pb[i], pt[i] = A.data_ptr(), b.data_ptr(), t.data_ptr()
        return count, n, pa, lda, pb, pt

    @staticmethod
    def _opts(order=4, k_max=64, refine_max=64, floor_detect=True, f_tol=0.0, resid_tol=1e-10,
              scale=SCALE_FROBENIUS, eps=0.0, graph=False):
        return SolveOpts(order=order, factorization=FACT["squaring"], p=0, w=0, k_max=k_max,
                         refine_max=refine_max, floor_detect=1 if floor_detect else 0,
                         scale=scale, eps=eps, f_tol=f_tol, resid_tol=resid_tol,
                         theta0_mode=0, graph=1 if graph else 0)

    def set_launch(self, waves: int, groups: int = 0):
        check(lib().ns_batch_set_launch(self._h, int(waves), int(groups)))

    def set_lockstep(self, min_count: int):
        """``ns_batch_set_lockstep``: lockstep float64 re-solves in
        submissions of at least ``min_count`` systems (0: off)."""
        check(lib().ns_batch_set_lockstep(self._h, int(min_count)))

    def submit(self, As, bs, thetas, **opts) -> int:
        count, n, pa, lda, pb, pt = self._arrays(As, bs, thetas)
        o = self._opts(**opts)
        t = ctypes.c_uint64()
        check(lib().ns_batch_submit(self._h, count, n, pa, lda, pb, pt, ctypes.byref(o),
                                    ctypes.byref(t)))
        self._keep = (As, bs, thetas)
        self._count = count
        return t.value

    def submit_packed(self, systems: "PackedSystems", **opts) -> int:
        """Submit a packed batch (see `PackedSystems`); same options as
        `submit`."""
        n, pa, pb, pt = systems.pointers()
        o = self._opts(**opts)
        t = ctypes.c_uint64()
        check(lib().ns_batch_submit(self._h, len(systems), n.ctypes.data, pa.ctypes.data,
                                    n.ctypes.data, pb.ctypes.data, pt.ctypes.data,
                                    ctypes.byref(o), ctypes.byref(t)))
        self._keep = systems
        self._count = len(systems)
        return t.value

    def poll_arrays(self, ticket: int, wait: bool = True):
        """Like `poll`, but the reports come back as numpy columns (status,
        precision, ns_steps, refine_steps, ns_stop, refine_stop, alpha,
        rel_resid, mmm, gemm_flop) without the NS histories; None if still
        running (wait=False)."""
        reps = (SolveReportC * max(self._count, 1))()
        st = lib().ns_batch_poll(self._h, int(ticket), 1 if wait else 0, reps)
        if st == NS_EBUSY:
            return None
        if st not in (NS_OK, NS_ENOCONV):
            check(st)
        self._keep = None
        return _report_arrays(reps, self._count)

    def poll(self, ticket: int, wait: bool = True):
        """List of SolveReport on completion, None if still running (wait=False)."""
        reps = (SolveReportC * max(self._count, 1))()
        st = lib().ns_batch_poll(self._h, int(ticket), 1 if wait else 0, reps)
        if st == NS_EBUSY:
            return None
        if st not in (NS_OK, NS_ENOCONV):
            check(st)
        self._keep = None
        return [_report_from_c(reps[i]) for i in range(self._count)]

    def timeline(self, ticket: int):
        """(times_us [count, 4], workgroup [count, 2]) of the last polled ticket:
        begin / end of the float32 and float64 attempts (NaN: not run)."""
        times = np.zeros((self._count, 4), dtype=np.float64)
        wg = np.zeros((self._count, 2), dtype=np.int32)
        check(lib().ns_batch_timeline(self._h, int(ticket), times.ctypes.data, wg.ctypes.data))
        return times, wg

    def autotune(self, As, bs, thetas, **opts):
        count, n, pa, lda, pb, pt = self._arrays(As, bs, thetas)
        o = self._opts(**opts)
        w, g, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        check(lib().ns_batch_autotune(self._h, count, n, pa, lda, pb, pt, ctypes.byref(o),
                                      ctypes.byref(w), ctypes.byref(g), ctypes.byref(ms)))
        return w.value, g.value, ms.value


def gemm_lp(X, Y, nt: bool, D=None, want_bf16: bool = False, E1=None, E2=None,
            diag: float = 0.0, scale: float = 1.0, want_sumsq: bool = False, stream=None):
    """float32 NN (``nt=False``: D = X Y) or bf16 NT (``nt=True``: D = X Y^T)
    MFMA GEMM with the fused epilogue.  Returns (D, Db or None, sumsq or None)."""
    import torch
    want_dtype = torch.bfloat16 if nt else torch.float32
    for t, nm in ((X, "X"), (Y, "Y")):
        if not t.is_cuda or t.dtype != want_dtype or t.stride(-1) != 1:
            raise TypeError(f"{nm} must be a row-major {want_dtype} CUDA tensor")
    m, k = X.shape
    n = Y.shape[0] if nt else Y.shape[1]
    if (Y.shape[1] if nt else Y.shape[0]) != k:
        raise ValueError("inner dimensions differ")
    for t in (E1, E2):
        if t is not None and (t.dtype != torch.float32 or not t.is_cuda):
            raise TypeError("addends must be float32 CUDA tensors")
    if D is None:
        D = torch.empty(m, n, dtype=torch.float32, device=X.device)
    Db = torch.empty(m, n, dtype=torch.bfloat16, device=X.device) if want_bf16 else None
    ss = None
    if want_sumsq:
        ss = torch.zeros(1 + int(lib().ns_gemm_lp_partials(m, n)), dtype=torch.float64,
                         device=X.device)
    fn = lib().ns_gemm_bf16_nt if nt else lib().ns_gemm_f32
    check(fn(_stream_handle(stream), m, n, k, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0),
             _ptr(D), D.stride(0), _ptr(Db), Db.stride(0) if Db is not None else 0,
             _ptr(E1), E1.stride(0) if E1 is not None else 0, _ptr(E2),
             E2.stride(0) if E2 is not None else 0, float(diag), float(scale), _ptr(ss)))
    return D, Db, (ss[0] if ss is not None else None)


def gemm_bf16_sym(X, Y, D=None, want_bf16: bool = False, E1=None, E2=None,
                  diag: float = 0.0, scale: float = 1.0, want_sumsq: bool = False,
                  symmetric: bool = True, scratch=None, stream=None):
    """bf16 NT product D = diag I + scale X Y^T + E1 + E2 through
    ``ns_gemm_bf16_nt_ws``; with ``symmetric`` only the upper tiles are
    computed and mirrored (see nsr.h).  Returns (D, Db or None, sumsq or None)."""
    import torch
    for t, nm in ((X, "X"), (Y, "Y")):
        if not t.is_cuda or t.dtype != torch.bfloat16 or t.stride(-1) != 1:
            raise TypeError(f"{nm} must be a row-major bfloat16 CUDA tensor")
    m, k = X.shape
    n = Y.shape[0]
    if Y.shape[1] != k:
        raise ValueError("inner dimensions differ")
    if D is None:
        D = torch.empty(m, n, dtype=torch.float32, device=X.device)
    Db = torch.empty(m, n, dtype=torch.bfloat16, device=X.device) if want_bf16 else None
    ss = None
    if want_sumsq:
        ss = torch.zeros(1 + int(lib().ns_gemm_lp_partials(m, n)), dtype=torch.float64,
                         device=X.device)
    flags = GEMM_SYMMETRIC if symmetric else 0
    nbytes = int(lib().ns_gemm_bf16_scratch_bytes(m, n, k, flags))
    if scratch is None and nbytes > 0:
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
    check(lib().ns_gemm_bf16_nt_ws(
        _stream_handle(stream), m, n, k, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0),
        _ptr(D), D.stride(0), _ptr(Db), Db.stride(0) if Db is not None else 0,
        _ptr(E1), E1.stride(0) if E1 is not None else 0, _ptr(E2),
        E2.stride(0) if E2 is not None else 0, float(diag), float(scale), flags, _ptr(ss),
        _ptr(scratch), scratch.numel() * scratch.element_size() if scratch is not None else 0))
    return D, Db, (ss[0] if ss is not None else None)


def gemm_f32_split(X, Y, D=None, want_bf16: bool = False, E1=None, E2=None,
                   diag: float = 0.0, scale: float = 1.0, want_sumsq: bool = False,
                   scratch=None, stream=None):
    """float32-class D = diag I + scale X Y + E1 + E2 from split half-precision
    operands (see ``ns_gemm_f32_split``).  Returns (D, Db or None, sumsq or
    None); scratch (uint8 device tensor) is allocated when not given."""
    import torch
    for t, nm in ((X, "X"), (Y, "Y")):
        if not t.is_cuda or t.dtype != torch.float32 or t.stride(-1) != 1:
            raise TypeError(f"{nm} must be a row-major float32 CUDA tensor")
    m, k = X.shape
    n = Y.shape[1]
    if Y.shape[0] != k:
        raise ValueError("inner dimensions differ")
    for t in (E1, E2):
        if t is not None and (t.dtype != torch.float32 or not t.is_cuda):
            raise TypeError("addends must be float32 CUDA tensors")
    if D is None:
        D = torch.empty(m, n, dtype=torch.float32, device=X.device)
    Db = torch.empty(m, n, dtype=torch.bfloat16, device=X.device) if want_bf16 else None
    ss = None
    if want_sumsq:
        ss = torch.zeros(1 + int(lib().ns_gemm_lp_partials(m, n)), dtype=torch.float64,
                         device=X.device)
    nbytes = int(lib().ns_gemm_f32_split_scratch_bytes(m, n, k))
    if scratch is None:
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
    check(lib().ns_gemm_f32_split(
        _stream_handle(stream), m, n, k, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0),
        _ptr(D), D.stride(0), _ptr(Db), Db.stride(0) if Db is not None else 0,
        _ptr(E1), E1.stride(0) if E1 is not None else 0, _ptr(E2),
        E2.stride(0) if E2 is not None else 0, float(diag), float(scale), _ptr(ss),
        _ptr(scratch), scratch.numel() * scratch.element_size()))
    return D, Db, (ss[0] if ss is not None else None)


# GEMM families of the tile table (NS_TILE_* in include/nsr.h) and their tiles.
TILE_F64, TILE_F32, TILE_BF16, TILE_F16S = 0, 1, 2, 3
TILE_OPTIONS = {TILE_F64: (64, 128, 256), TILE_F32: (64, 128, 256), TILE_BF16: (64, 128, 256),
                TILE_F16S: (64, 128, 256)}


def tile_set(family: int, log2_dim: int, tile: int):
    """``ns_tile_set``: the tile of a family's products with max(m, n) in
    (2^(log2_dim - 1), 2^log2_dim]; 0 restores the library's rule."""
    check(lib().ns_tile_set(int(family), int(log2_dim), int(tile)))


def tile_get(family: int, log2_dim: int) -> int:
    return int(lib().ns_tile_get(int(family), int(log2_dim)))


# Size of the library's built-in scratch of ns_gemm_f32_split_noalloc (include/nsr.h).
SPLIT_NOALLOC_MAX_BYTES = 64 << 20


def gemm_f32_split_noalloc(X, Y, D=None, want_bf16: bool = False, E1=None, E2=None,
                           diag: float = 0.0, scale: float = 1.0, sumsq=None, stream=None):
    """``ns_gemm_f32_split_noalloc``: the split product of ``gemm_f32_split``
    with the library's built-in scratch (no scratch argument).  ``sumsq``, when
    given, is a one-element float64 CUDA tensor that receives sum(D^2).
    Returns (D, Db or None)."""
    import torch
    for t, nm in ((X, "X"), (Y, "Y")):
        if not t.is_cuda or t.dtype != torch.float32 or t.stride(-1) != 1:
            raise TypeError(f"{nm} must be a row-major float32 CUDA tensor")
    m, k = X.shape
    n = Y.shape[1]
    if Y.shape[0] != k:
        raise ValueError("inner dimensions differ")
    for t in (E1, E2):
        if t is not None and (t.dtype != torch.float32 or not t.is_cuda):
            raise TypeError("addends must be float32 CUDA tensors")
    if sumsq is not None and (sumsq.dtype != torch.float64 or not sumsq.is_cuda
                              or sumsq.numel() < 1):
        raise TypeError("sumsq must be a float64 CUDA tensor with at least one element")
    if D is None:
        D = torch.empty(m, n, dtype=torch.float32, device=X.device)
    Db = torch.empty(m, n, dtype=torch.bfloat16, device=X.device) if want_bf16 else None
    check(lib().ns_gemm_f32_split_noalloc(
        _stream_handle(stream), m, n, k, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0),
        _ptr(D), D.stride(0), _ptr(Db), Db.stride(0) if Db is not None else 0,
        _ptr(E1), E1.stride(0) if E1 is not None else 0, _ptr(E2),
        E2.stride(0) if E2 is not None else 0, float(diag), float(scale), _ptr(sumsq)))
    return D, Db


def exported_symbols() -> list[str]:
    """Names of EXPORTS that the loaded library actually exports."""
    L = lib()
    out = []
    for name in EXPORTS:
        try:
            getattr(L, name)
            out.append(name)
        except AttributeError:
            pass
    return out


def solve_np(A: np.ndarray, b: np.ndarray, **kw):
    """Convenience: copy host arrays to the GPU, solve, copy theta back."""
    import torch
    dev = torch.device("cuda")
    At = torch.from_numpy(np.ascontiguousarray(A)).to(dev)
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    th = torch.zeros_like(bt)
    s = Solver(A.shape[0], composite=kw.get("form") == "composite_double")
    s.bind(At)
    rep = s.solve(bt, th, **kw)
    torch.cuda.synchronize()
    return th.cpu().numpy(), rep

"""Python binding of the TLR library (include/tlr.h, include/tlr_kernels.h).

Argument marshalling only: every computation runs in libtlr.so.  PyTorch
provides device memory (through the allocator callbacks of the C ABI) and the
current HIP stream.  Loading fails loudly when the library has not been
built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtlr.so")

TLR_OK = 0
TLR_ERR_ARG = -1
TLR_ERR_OOM = -2
TLR_ERR_DEVICE = -3
TLR_ERR_STATE = -4
TLR_ERR_NOT_SPD = 1
TLR_ERR_ZERO_PIVOT = 2
EPS_ABS, EPS_REL = 0, 1
FP64, MIXED_FP32, MIXED_BF16, MIXED_AUTO = 0, 1, 2, 3
FLAG_KERNEL_TIMING, FLAG_PHASE_TIMING, FLAG_SERIAL_SAMPLING, FLAG_MODIFIED_CHOL = 1, 2, 4, 8
FLAG_DIAG_GRAPH, FLAG_SCHUR_COMP = 16, 32
PHASES = ("gblocks", "sample", "orth", "batch", "project", "trsm", "append", "diag")
KERNEL_EXP, KERNEL_MATERN15 = 0, 1
INPUT, FACTOR = 0, 1

_STATUS = {0: "TLR_OK", -1: "TLR_ERR_ARG", -2: "TLR_ERR_OOM", -3: "TLR_ERR_DEVICE",
           -4: "TLR_ERR_STATE", 1: "TLR_ERR_NOT_SPD", 2: "TLR_ERR_ZERO_PIVOT"}


class TLRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("bs", ctypes.c_int), ("eps_mode", ctypes.c_int), ("precision", ctypes.c_int),
                ("shift", ctypes.c_double), ("max_active", ctypes.c_int), ("r_min", ctypes.c_int),
                ("seed", ctypes.c_ulonglong), ("flags", ctypes.c_int), ("bs_tail", ctypes.c_int),
                ("tail_active", ctypes.c_int), ("auto_shift", ctypes.c_int),
                ("sample_strip", ctypes.c_int), ("conv_factor", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("info", ctypes.c_int), ("tau", ctypes.c_double), ("norm_a", ctypes.c_double),
                ("flops", ctypes.c_double), ("flops_paper", ctypes.c_double),
                ("bytes_alg", ctypes.c_double), ("ara_iters", ctypes.c_longlong),
                ("tile_iters", ctypes.c_longlong), ("full_rank_tiles", ctypes.c_longlong),
                ("max_rank", ctypes.c_int), ("mean_rank", ctypes.c_double),
                ("factor_bytes", ctypes.c_double), ("sample_launches", ctypes.c_longlong),
                ("sample_ms", ctypes.c_double), ("sample_bytes", ctypes.c_double),
                ("sample_flops", ctypes.c_double), ("fp32_tile_iters", ctypes.c_longlong),
                ("shift", ctypes.c_double), ("shift_retries", ctypes.c_int),
                ("t_total", ctypes.c_double), ("t_phase", ctypes.c_double * 8),
                ("bf16_tile_iters", ctypes.c_longlong), ("t_host_issue", ctypes.c_double),
                ("t_host_wait", ctypes.c_double), ("modified_pivots", ctypes.c_longlong)]

    def as_dict(self) -> Dict[str, float]:
        out = {f: getattr(self, f) for f, _ in self._fields_}
        out["t_phase"] = list(self.t_phase)
        return out


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


class GemmProblem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("N", ctypes.c_int), ("K", ctypes.c_int),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double)]


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_LL = ctypes.c_longlong
_D = ctypes.c_double
_U = ctypes.c_uint
_ULL = ctypes.c_ulonglong
_IP = ctypes.POINTER(ctypes.c_int)
_LLP = ctypes.POINTER(ctypes.c_longlong)
_DP = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "tlr_opts_default": (None, [ctypes.POINTER(Opts)]),
    "tlr_create": (_I, [_LL, _I, _IP, ctypes.POINTER(Allocator), _P, ctypes.POINTER(_P)]),
    "tlr_set_diag": (_I, [_P, _I, _P, _I, _I]),
    "tlr_set_tile": (_I, [_P, _I, _I, _P, _P, _I, _I]),
    "tlr_compress": (_I, [_P, _LL, _LL, _I, _D, ctypes.POINTER(Opts), ctypes.POINTER(Allocator), _P,
                          ctypes.POINTER(_P)]),
    "tlr_compress_kernel": (_I, [_P, _I, _LL, _I, _D, _D, _I, _D, ctypes.POINTER(Opts),
                                 ctypes.POINTER(Allocator), _P, ctypes.POINTER(_P)]),
    "tlr_potrf": (_I, [_P, _D, ctypes.POINTER(Opts), ctypes.POINTER(Stats), _P]),
    "tlr_ldlt": (_I, [_P, _D, ctypes.POINTER(Opts), _P, ctypes.POINTER(Stats), _P]),
    "tlr_potrf_pivoted": (_I, [_P, _D, ctypes.POINTER(Opts), _IP, ctypes.POINTER(Stats), _P]),
    "tlr_get_perm": (_I, [_P, _IP]),
    "tlr_tune_tile": (_I, [_P, _I, _LL, _I, _D, _D, _D, ctypes.POINTER(Opts), _IP, _I,
                           ctypes.POINTER(Allocator), _P, _IP, _DP, _IP]),
    "tlr_tune_reset": (None, []),
    "tlr_factor_batched": (_I, [_I, ctypes.POINTER(_P), _I, _D, ctypes.POINTER(Opts),
                                ctypes.POINTER(_P), ctypes.POINTER(Stats), _P]),
    "tlr_potrf_batched": (_I, [_I, ctypes.POINTER(_P), _DP, ctypes.POINTER(Opts),
                               ctypes.POINTER(Stats), _P]),
    "tlr_ldlt_batched": (_I, [_I, ctypes.POINTER(_P), _DP, ctypes.POINTER(Opts),
                              ctypes.POINTER(_P), ctypes.POINTER(Stats), _P]),
    "tlr_solve": (_I, [_P, _I, _P, _LL, _P]),
    "tlr_solve_noalloc": (_I, [_P, _I, _P, _LL, _P]),
    "tlr_solve_noalloc_max_bytes": (ctypes.c_size_t, []),
    "tlr_matvec": (_I, [_P, _I, _P, _LL, _P, _LL, _P]),
    "tlr_recompress": (_I, [_P, _I, _D, _P]),
    "tlr_pcg": (_I, [_P, _P, _P, _P, _D, _I, _IP, _DP, _P]),
    "tlr_get_info": (_I, [_P, _LLP, _IP, _IP, _IP]),
    "tlr_get_ranks": (_I, [_P, _I, _IP]),
    "tlr_get_offsets": (_I, [_P, _I, _LLP]),
    "tlr_get_tile": (_I, [_P, _I, _I, _I, _DP, _DP, _I]),
    "tlr_get_diag": (_I, [_P, _I, _I, _DP, _I]),
    "tlr_get_pivots": (_I, [_P, _DP]),
    "tlr_get_sort_order": (_I, [_P, _I, _IP]),
    "tlr_destroy": (_I, [_P]),
    "tlr_last_error": (ctypes.c_char_p, []),
    "tlrk_gemm_batched": (_I, [_I, _I, _I, ctypes.POINTER(GemmProblem), _P]),
    "tlrk_potrf": (_I, [_I, _P, _I, _IP, _P]),
    "tlrk_ldlt": (_I, [_I, _P, _I, _P, _IP, _P]),
    "tlrk_trsm": (_I, [_I, _I, _P, _I, _P, _I, _I, _I, _P]),
    "tlrk_philox": (_I, [_I, _ULL, _U, _U, _U, _P, _P]),
    "tlrk_randn": (_I, [_I, _I, _ULL, _U, _U, _U, _P, _P]),
    "tlrk_randn_iters": (_I, [_I, _I, _I, _ULL, _U, _U, _I, _U, _P, _P]),
    "tlrk_ara": (_I, [_I, _I, _P, _D, _I, _I, _ULL, _P, _P, _IP, _IP, _P]),
    "tlrk_sort_ranks": (_I, [_I, _IP, _IP, _IP]),
    "tlrk_compact": (_I, [_I, _IP, _IP, _IP, _IP, _I, _IP, _I]),
}


_hip = None


def hip_runtime():
    """Make the process's HIP runtime visible to libtlr.so, which links none.

    PyTorch's ROCm wheel carries its own libamdhip64; loading a second
    runtime (the system's) beside it would give the process two HIP runtimes
    whose devices and streams do not mix.  So torch's runtime is promoted to
    global symbol scope (dlopen of an already loaded library returns it) and
    libtlr.so binds to it; without torch the system runtime is used."""
    global _hip
    if _hip is None:
        cands = []
        try:
            import torch
            cands.append(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
        except ImportError:  # pragma: no cover
            pass
        rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
        cands += [os.path.join(rocm, "lib", "libamdhip64.so"), "libamdhip64.so"]
        err = None
        for c in cands:
            if os.path.sep in c and not os.path.exists(c):
                continue
            try:
                _hip = ctypes.CDLL(c, mode=ctypes.RTLD_GLOBAL)
                break
            except OSError as e:  # pragma: no cover
                err = e
        if _hip is None:
            raise RuntimeError("no HIP runtime library found: %s" % err)
    return _hip


def lib():
    """The loaded libtlr.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtlr.so not built: run `python -m paper_2108_11932_amd.build`")
        hip_runtime()
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def _check(status: int):
    if status != TLR_OK:
        msg = lib().tlr_last_error()
        raise TLRError(status, msg.decode() if msg else "")


def opts(**kw) -> Opts:
    """tlr_opts with the library defaults, overridden by keyword arguments."""
    o = Opts()
    lib().tlr_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


# ---------------------------------------------------------------- torch glue

def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class TorchAllocator:
    """Backs the library's device allocations with torch's caching allocator."""

    def __init__(self):
        self._live = {}
        self.calls = 0   # allocations requested by the library so far
        self._alloc_cb = _ALLOC_FN(self._alloc)
        self._free_cb = _FREE_FN(self._free)
        self.struct = Allocator(None, self._alloc_cb, self._free_cb)

    def _alloc(self, ctx, nbytes, stream):
        torch = _torch()
        self.calls += 1
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        except RuntimeError:
            return None
        self._live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ctx, p, stream):
        self._live.pop(p, None)

    @property
    def live_bytes(self) -> int:
        return sum(t.numel() for t in self._live.values())


class TLRMatrix:
    """Owner of a tlr_matrix_t handle and of the allocator behind it."""

    def __init__(self, handle: ctypes.c_void_p, allocator: Optional[TorchAllocator]):
        self.h = handle
        self.allocator = allocator
        n = ctypes.c_longlong()
        m = ctypes.c_int()
        nb = ctypes.c_int()
        f = ctypes.c_int()
        _check(lib().tlr_get_info(self.h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(nb),
                                  ctypes.byref(f)))
        self.n, self.m, self.nb = n.value, m.value, nb.value

    # -- construction
    @staticmethod
    def create(n: int, m: int, ranks: Optional[np.ndarray] = None,
               use_torch_allocator: bool = True) -> "TLRMatrix":
        alloc = TorchAllocator() if use_torch_allocator else None
        h = ctypes.c_void_p()
        rp = None
        if ranks is not None:
            r = np.ascontiguousarray(ranks, dtype=np.int32)
            rp = r.ctypes.data_as(_IP)
        _check(lib().tlr_create(n, m, rp, ctypes.byref(alloc.struct) if alloc else None, _stream(),
                                ctypes.byref(h)))
        return TLRMatrix(h, alloc)

    @staticmethod
    def from_tlr(n: int, m: int, diag, u: dict, v: dict) -> "TLRMatrix":
        """Upload host tiles: diag[k] (m x m), u[i, j] / v[i, j] (m x r)."""
        nb = -(-n // m)
        ranks = np.zeros((nb, nb), dtype=np.int32)
        for (i, j), uu in u.items():
            ranks[i, j] = uu.shape[1]
        t = TLRMatrix.create(n, m, ranks)
        for k in range(nb):
            d = np.asfortranarray(diag[k], dtype=np.float64)
            _check(lib().tlr_set_diag(t.h, k, d.ctypes.data_as(_P), d.shape[0], 0))
        for (i, j), uu in u.items():
            if uu.shape[1] == 0:
                continue
            U = np.asfortranarray(uu, dtype=np.float64)
            V = np.asfortranarray(v[i, j], dtype=np.float64)
            _check(lib().tlr_set_tile(t.h, i, j, U.ctypes.data_as(_P), V.ctypes.data_as(_P), m, 0))
        return t

    @staticmethod
    def compress(a, m: int, eps: float, o: Optional[Opts] = None) -> "TLRMatrix":
        """tlr_compress of a dense symmetric torch cuda float64 matrix."""
        torch = _torch()
        # the row-major storage of a^T is the column-major storage of a
        at = a.to(dtype=torch.float64).t().contiguous()
        n = a.shape[0]
        alloc = TorchAllocator()
        h = ctypes.c_void_p()
        _check(lib().tlr_compress(_ptr(at), n, n, m, eps, ctypes.byref(o or opts()),
                                  ctypes.byref(alloc.struct), _stream(), ctypes.byref(h)))
        return TLRMatrix(h, alloc)

    @staticmethod
    def compress_kernel(points, kernel: int, ell: float, diag_add: float, m: int, eps: float,
                        o: Optional[Opts] = None) -> "TLRMatrix":
        """tlr_compress_kernel of N points (numpy or torch, N x dim)."""
        torch = _torch()
        p = torch.as_tensor(np.ascontiguousarray(points, dtype=np.float64)).cuda().contiguous()
        n, dim = p.shape
        alloc = TorchAllocator()
        h = ctypes.c_void_p()
        _check(lib().tlr_compress_kernel(_ptr(p), dim, n, kernel, ell, diag_add, m, eps,
                                         ctypes.byref(o or opts()), ctypes.byref(alloc.struct),
                                         _stream(), ctypes.byref(h)))
        torch.cuda.current_stream().synchronize()
        return TLRMatrix(h, alloc)

    # -- factorizations
    def potrf(self, eps: float, o: Optional[Opts] = None) -> Dict[str, float]:
        st = Stats()
        _check(lib().tlr_potrf(self.h, eps, ctypes.byref(o or opts()), ctypes.byref(st), _stream()))
        return st.as_dict()

    def potrf_status(self, eps: float, o: Optional[Opts] = None) -> Tuple[int, Dict[str, float]]:
        st = Stats()
        s = lib().tlr_potrf(self.h, eps, ctypes.byref(o or opts()), ctypes.byref(st), _stream())
        return s, st.as_dict()

    def potrf_pivoted(self, eps: float, o: Optional[Opts] = None):
        """Pivoted Cholesky; returns (stats, perm) with position t of the
        factor holding original block perm[t]."""
        st = Stats()
        perm = np.zeros(self.nb, dtype=np.int32)
        _check(lib().tlr_potrf_pivoted(self.h, eps, ctypes.byref(o or opts()),
                                       perm.ctypes.data_as(_IP), ctypes.byref(st), _stream()))
        return st.as_dict(), perm

    def perm(self):
        p = np.zeros(self.nb, dtype=np.int32)
        _check(lib().tlr_get_perm(self.h, p.ctypes.data_as(_IP)))
        return p

    def ldlt(self, eps: float, o: Optional[Opts] = None):
        torch = _torch()
        d = torch.empty(self.n, dtype=torch.float64, device="cuda")
        st = Stats()
        _check(lib().tlr_ldlt(self.h, eps, ctypes.byref(o or opts()), _ptr(d), ctypes.byref(st),
                              _stream()))
        return st.as_dict(), d

    def ldlt_status(self, eps: float, o: Optional[Opts] = None):
        st = Stats()
        s = lib().tlr_ldlt(self.h, eps, ctypes.byref(o or opts()), None, ctypes.byref(st), _stream())
        return s, st.as_dict()

    # -- products and solves (torch cuda float64, N x nrhs, column-major data)
    def solve(self, b):
        """Returns (A)^{-1} b for b of shape (N,) or (N, nrhs)."""
        torch = _torch()
        x = _to_colmajor(b)
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        _check(lib().tlr_solve(self.h, nrhs, _ptr(x), self.n, _stream()))
        return _from_colmajor(x, b.shape)

    def solve_noalloc(self, b):
        """As solve(), through tlr_solve_noalloc (workspace in the library's
        fixed per-GPU scratch array, no allocation inside the call)."""
        x = _to_colmajor(b)
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        _check(lib().tlr_solve_noalloc(self.h, nrhs, _ptr(x), self.n, _stream()))
        return _from_colmajor(x, b.shape)

    def pcg(self, b, precond: Optional["TLRMatrix"] = None, rtol: float = 1e-10,
            maxit: int = 1000, x0=None):
        """tlr_pcg with this handle's input matrix as the operator and the
        factor of `precond` as the preconditioner: (x, iterations, relres)."""
        torch = _torch()
        bd = b.to(dtype=torch.float64).contiguous()
        x = torch.zeros_like(bd) if x0 is None else x0.to(dtype=torch.float64).clone().contiguous()
        it = ctypes.c_int()
        rr = ctypes.c_double()
        _check(lib().tlr_pcg(self.h, precond.h if precond is not None else None, _ptr(bd), _ptr(x),
                             rtol, maxit, ctypes.byref(it), ctypes.byref(rr), _stream()))
        return x, it.value, rr.value

    def matvec(self, x):
        torch = _torch()
        xc = _to_colmajor(x)
        nrhs = 1 if x.dim() == 1 else x.shape[1]
        y = torch.empty_like(xc)
        _check(lib().tlr_matvec(self.h, nrhs, _ptr(xc), self.n, _ptr(y), self.n, _stream()))
        return _from_colmajor(y, x.shape)

    def recompress(self, tau: float, which: int = FACTOR):
        """SVD post-recompression of every low rank tile of the factor (or
        input) at the absolute threshold tau (tlr_recompress)."""
        _check(lib().tlr_recompress(self.h, which, float(tau), _stream()))

    # -- inspection
    def ranks(self, which: int = INPUT) -> np.ndarray:
        r = np.zeros((self.nb, self.nb), dtype=np.int32)
        _check(lib().tlr_get_ranks(self.h, which, r.ctypes.data_as(_IP)))
        return r

    def offsets(self, which: int = INPUT) -> np.ndarray:
        o = np.zeros((self.nb, self.nb), dtype=np.int64)
        _check(lib().tlr_get_offsets(self.h, which, o.ctypes.data_as(_LLP)))
        return o

    def tile(self, which: int, i: int, j: int) -> Tuple[np.ndarray, np.ndarray]:
        r = int(self.ranks(which)[i, j])
        U = np.zeros((self.m, r), order="F")
        V = np.zeros((self.m, r), order="F")
        if r:
            _check(lib().tlr_get_tile(self.h, which, i, j, U.ctypes.data_as(_DP),
                                      V.ctypes.data_as(_DP), self.m))
        return U, V

    def diag(self, which: int, k: int) -> np.ndarray:
        D = np.zeros((self.m, self.m), order="F")
        _check(lib().tlr_get_diag(self.h, which, k, D.ctypes.data_as(_DP), self.m))
        return D

    def pivots(self) -> np.ndarray:
        d = np.zeros(self.nb * self.m)
        _check(lib().tlr_get_pivots(self.h, d.ctypes.data_as(_DP)))
        return d

    def sort_order(self, k: int) -> list:
        """Block rows of column k in the sortRanks order of the last factorization."""
        n = self.nb - k - 1
        r = np.zeros(max(n, 1), dtype=np.int32)
        _check(lib().tlr_get_sort_order(self.h, k, r.ctypes.data_as(_IP)))
        return r[:n].tolist()

    def to_host(self, which: int = FACTOR):
        """(diag list, U dict, V dict) of the input or the factor, host numpy."""
        ranks = self.ranks(which)
        diag = [self.diag(which, k) for k in range(self.nb)]
        u, v = {}, {}
        for i in range(self.nb):
            for j in range(i):
                u[i, j], v[i, j] = self.tile(which, i, j)
        return diag, u, v, ranks

    def close(self):
        if self.h:
            lib().tlr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def factor_batched(mats, eps: float, o: Optional[Opts] = None, ldl: bool = False):
    """tlr_factor_batched over a list of TLRMatrix: returns (status, list of
    stats dicts, list of pivot tensors (LDL^T) or None)."""
    torch = _torch()
    n = len(mats)
    hs = (_P * n)(*[mt.h for mt in mats])
    sts = (Stats * n)()
    dl = None
    darr = None
    if ldl:
        dl = [torch.empty(mt.n, dtype=torch.float64, device="cuda") for mt in mats]
        darr = (_P * n)(*[ctypes.c_void_p(d.data_ptr()) for d in dl])
    s = lib().tlr_factor_batched(n, hs, int(ldl), eps, ctypes.byref(o or opts()), darr, sts,
                                 _stream())
    return s, [st.as_dict() for st in sts], dl


def factor_batched_eps(mats, eps, o: Optional[Opts] = None, ldl: bool = False):
    """tlr_potrf_batched / tlr_ldlt_batched with one threshold per matrix:
    returns (status, list of stats dicts, list of pivot tensors or None)."""
    torch = _torch()
    n = len(mats)
    hs = (_P * n)(*[mt.h for mt in mats])
    ev = np.ascontiguousarray(eps, dtype=np.float64)
    sts = (Stats * n)()
    if ldl:
        dl = [torch.empty(mt.n, dtype=torch.float64, device="cuda") for mt in mats]
        darr = (_P * n)(*[ctypes.c_void_p(d.data_ptr()) for d in dl])
        s = lib().tlr_ldlt_batched(n, hs, ev.ctypes.data_as(_DP), ctypes.byref(o or opts()), darr,
                                   sts, _stream())
        return s, [st.as_dict() for st in sts], dl
    s = lib().tlr_potrf_batched(n, hs, ev.ctypes.data_as(_DP), ctypes.byref(o or opts()), sts,
                                _stream())
    return s, [st.as_dict() for st in sts], None


def _to_colmajor(b):
    """A column-major (Fortran) copy of a 1-D or 2-D tensor as flat storage."""
    if b.dim() == 1:
        return b.contiguous().clone()
    return b.t().contiguous().clone()


def _from_colmajor(x, shape):
    if len(shape) == 1:
        return x
    return x.view(shape[1], shape[0]).t()


# ---------------------------------------------------------------- kernels

def gemm_batched(trans_a: bool, trans_b: bool, problems):
    """problems: list of dicts with M, N, K, A, lda, B, ldb, C, ldc, alpha,
    beta (A/B/C torch cuda float64 tensors holding column-major data)."""
    arr = (GemmProblem * max(1, len(problems)))()
    for i, p in enumerate(problems):
        arr[i] = GemmProblem(p["M"], p["N"], p["K"], p["A"].data_ptr(), p["lda"], p["B"].data_ptr(),
                             p["ldb"], p["C"].data_ptr(), p["ldc"], p["alpha"], p["beta"])
    _check(lib().tlrk_gemm_batched(int(trans_a), int(trans_b), len(problems), arr, _stream()))


def potrf_tile(a) -> int:
    """In-place dense Cholesky of a column-major m x m torch tensor (flat
    storage of a^T); returns info."""
    m = int(round(a.numel() ** 0.5))
    info = ctypes.c_int()
    _check(lib().tlrk_potrf(m, _ptr(a), m, ctypes.byref(info), _stream()))
    return info.value


def tune_tile(points, kernel: int, ell: float, diag_add: float, eps: float,
              candidates=(256, 512, 1024), o: Optional[Opts] = None):
    """tlr_tune_tile: (best tile size, {candidate: ms} or None when cached)."""
    torch = _torch()
    p = torch.as_tensor(np.ascontiguousarray(points, dtype=np.float64)).cuda().contiguous()
    n, dim = p.shape
    cand = np.ascontiguousarray(candidates, dtype=np.int32)
    ms = np.zeros(len(cand), dtype=np.float64)
    best = ctypes.c_int()
    cached = ctypes.c_int()
    alloc = TorchAllocator()
    _check(lib().tlr_tune_tile(_ptr(p), dim, n, kernel, ell, diag_add, eps, ctypes.byref(o or opts()),
                               cand.ctypes.data_as(_IP), len(cand), ctypes.byref(alloc.struct),
                               _stream(), ctypes.byref(best), ms.ctypes.data_as(_DP),
                               ctypes.byref(cached)))
    return best.value, (None if cached.value else dict(zip(cand.tolist(), ms.tolist())))


def ldlt_tile(a, d) -> int:
    m = int(round(a.numel() ** 0.5))
    info = ctypes.c_int()
    _check(lib().tlrk_ldlt(m, _ptr(a), m, _ptr(d), ctypes.byref(info), _stream()))
    return info.value


def trsm(m: int, n: int, l, b, unit: bool = False, trans: bool = False):
    _check(lib().tlrk_trsm(m, n, _ptr(l), m, _ptr(b), m, int(unit), int(trans), _stream()))


def philox(n: int, seed: int, c1: int, c2: int, c3: int):
    torch = _torch()
    out = torch.empty(4 * n, dtype=torch.int32, device="cuda")
    _check(lib().tlrk_philox(n, seed, c1, c2, c3, _ptr(out), _stream()))
    return out.cpu().numpy().view(np.uint32)


def randn(rows: int, cols: int, seed: int, k: int, t: int, s: int):
    torch = _torch()
    out = torch.empty(rows * cols, dtype=torch.float64, device="cuda")
    _check(lib().tlrk_randn(rows, cols, seed, k, t, s, _ptr(out), _stream()))
    return out.cpu().numpy().reshape(cols, rows).T


def randn_iters(rows: int, cols0: int, cols1: int, seed: int, k: int, t0: int, nt: int, s: int):
    """Test matrices of nt consecutive iterations: list of rows x cols numpy arrays."""
    torch = _torch()
    cm = max(cols0, cols1)
    out = torch.empty(max(1, nt * rows * cm), dtype=torch.float64, device="cuda")
    _check(lib().tlrk_randn_iters(rows, cols0, cols1, seed, k, t0, nt, s, _ptr(out), _stream()))
    h = out.cpu().numpy()
    res = []
    for i in range(nt):
        c = cols0 if t0 + i == 0 else cols1
        res.append(h[i * rows * cm:i * rows * cm + rows * c].reshape(c, rows).T)
    return res


def ara(tiles, tau: float, bs: int = 16, r_min: int = 1, seed: int = 1):
    """Batched ARA of explicit tiles (torch cuda float64, count x m x m holding
    column-major tiles).  Returns (Q, B, ranks, iters) with Q/B torch tensors
    in the same layout."""
    torch = _torch()
    count, m = tiles.shape[0], tiles.shape[1]
    Q = torch.zeros_like(tiles)
    B = torch.zeros_like(tiles)
    ranks = np.zeros(count, dtype=np.int32)
    iters = np.zeros(count, dtype=np.int32)
    _check(lib().tlrk_ara(m, count, _ptr(tiles), tau, bs, r_min, seed, _ptr(Q), _ptr(B),
                          ranks.ctypes.data_as(_IP), iters.ctypes.data_as(_IP), _stream()))
    return Q, B, ranks, iters


def sort_ranks(ranks, rows):
    r = np.ascontiguousarray(ranks, dtype=np.int32)
    w = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros(len(r), dtype=np.int32)
    _check(lib().tlrk_sort_ranks(len(r), r.ctypes.data_as(_IP), w.ctypes.data_as(_IP),
                                 out.ctypes.data_as(_IP)))
    return out


def compact(nslots: int, act, flags, waiting, cursor: int, s_max: int):
    a = np.zeros(max(nslots, s_max, 1), dtype=np.int32)
    a[:len(act)] = act
    cnt = ctypes.c_int(len(act))
    cur = ctypes.c_int(cursor)
    f = np.ascontiguousarray(flags, dtype=np.int32)
    w = np.ascontiguousarray(waiting, dtype=np.int32) if len(waiting) else np.zeros(1, np.int32)
    _check(lib().tlrk_compact(nslots, a.ctypes.data_as(_IP), ctypes.byref(cnt),
                              f.ctypes.data_as(_IP), w.ctypes.data_as(_IP), len(waiting),
                              ctypes.byref(cur), s_max))
    return a[:cnt.value].tolist(), cur.value

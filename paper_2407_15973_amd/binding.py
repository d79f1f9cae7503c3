"""ctypes binding of libmpbjac (argument marshalling only).

Every numerical step runs in the HIP library; this module only converts
arrays to device tensors, allocates the workspaces the library asks for with
PyTorch, and passes pointers and the current stream. If the library is not
built, ``load()`` raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpbjac.so")

FP64, FP32, BF16, FP16 = 0, 1, 2, 3
UNIFORM, FIXED, RULE, LEARNED, EXPLICIT = 0, 1, 2, 3, 4
TEMPORAL_NONE, TEMPORAL_HL, TEMPORAL_LH = 0, 1, 2
STORE_FULL, STORE_BAND, STORE_SYM = 0, 1, 2
PCG_TEXTBOOK, PCG_SINGLE_REDUCTION = 0, 1
HINTS_AUTO, HINTS_PLAIN, HINTS_STREAM = 0, 1, 2   # bjac_cache_hints
OK, NOT_CONVERGED, EINVAL, ENOTSPD, EBREAKDOWN, EHIP, ENOMEM = 0, 1, -1, -2, -3, -4, -5
MLP_NPARAM = 5443
MLP_NBLOB = MLP_NPARAM + 32
NFEAT = 16

# exported symbols declared in include/mpbjac.h
SYMBOLS = (
    "bjac_abi_version", "bjac_strerror", "bjac_setup_query", "bjac_setup", "bjac_destroy",
    "bjac_get_info", "bjac_get_tags", "bjac_get_features", "bjac_get_block", "bjac_get_band", "bjac_apply",
    "bjac_spmv", "bjac_round", "pcg_workspace_query", "pcg_workspace_query_csr", "pcg_solve", "bjac_mlp_forward",
    "bjac_mlp_workspace_query", "bjac_mlp_backward", "bjac_mlp_adam",
    "pcg_batched_workspace_query", "pcg_solve_batched", "pcg_batched_tune", "bjac_apply_multi",
    "bjac_poly_setup_query", "bjac_poly_setup", "pcg_solve_noalloc", "bjac_stream_probe",
)


class bjac_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p)]


class bjac_policy(C.Structure):
    _fields_ = [("mode", C.c_int32), ("low", C.c_int32), ("temporal", C.c_int32), ("storage", C.c_int32),
                ("adp_tol", C.c_double), ("theta", C.c_double), ("d16", C.c_double),
                ("mlp_blob", C.c_void_p), ("explicit_tags", C.c_void_p), ("band_rtol", C.c_double)]


class bjac_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("nb", C.c_int32), ("max_block", C.c_int32),
                ("blocks_per_prec", C.c_int32 * 4), ("low_bytes", C.c_int64), ("high_bytes", C.c_int64),
                ("temporal", C.c_int32), ("mode", C.c_int32), ("ntiles", C.c_int32), ("reserved", C.c_int32)]


class bjac_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("chunk", C.c_int32),
                ("relres_hist", C.c_void_p), ("high_hist", C.c_void_p), ("profile", C.c_int32),
                ("verify", C.c_int32), ("variant", C.c_int32), ("cache_hints", C.c_int32)]


class bjac_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("relres", C.c_double), ("rnorm0", C.c_double),
                ("high_applications", C.c_int32), ("graph_launches", C.c_int32), ("solve_ms", C.c_double),
                ("spmv_ms", C.c_double), ("apply_ms", C.c_double), ("update_ms", C.c_double),
                ("n_spmv", C.c_int32), ("n_apply", C.c_int32), ("n_update", C.c_int32), ("restarts", C.c_int32),
                ("true_relres", C.c_double)]


class bjac_poly_params(C.Structure):
    _fields_ = [("k", C.c_int32), ("t", C.c_int32), ("low", C.c_int32), ("temporal", C.c_int32),
                ("adp_tol", C.c_double)]


class bjac_batch_cfg(C.Structure):
    _fields_ = [("spmv_grab", C.c_int32), ("wg_per_cu", C.c_int32), ("spmv_wg_per_cu", C.c_int32),
                ("apply_rows", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libmpbjac.so and declare its signatures. Raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2407_15973_amd.build.build()")
    L = C.CDLL(path)
    vp, i32, i64, dbl, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    P = C.POINTER
    sig = {
        "bjac_abi_version": (C.c_int, []),
        "bjac_strerror": (C.c_char_p, [C.c_int]),
        "bjac_setup_query": (C.c_int, [P(bjac_csr), vp, i32, P(bjac_policy), P(sz)]),
        "bjac_setup": (C.c_int, [P(bjac_csr), vp, i32, P(bjac_policy), vp, sz, vp, P(vp)]),
        "bjac_destroy": (None, [vp]),
        "bjac_get_info": (C.c_int, [vp, P(bjac_info)]),
        "bjac_get_tags": (C.c_int, [vp, vp]),
        "bjac_get_features": (C.c_int, [vp, vp]),
        "bjac_get_block": (C.c_int, [vp, i32, i32, vp, P(dbl)]),
        "bjac_get_band": (C.c_int, [vp, i32, vp]),
        "bjac_apply": (C.c_int, [vp, i32, vp, vp, vp]),
        "bjac_spmv": (C.c_int, [P(bjac_csr), vp, vp, vp]),
        "bjac_round": (C.c_int, [vp, vp, i64, i32, dbl, vp]),
        "pcg_workspace_query": (C.c_int, [i64, P(sz)]),
        "pcg_workspace_query_csr": (C.c_int, [P(bjac_csr), P(sz)]),
        "pcg_solve": (C.c_int, [P(bjac_csr), vp, vp, vp, P(bjac_solve_opts), vp, sz, P(bjac_stats), vp]),
        "pcg_solve_noalloc": (C.c_int, [P(bjac_csr), vp, vp, vp, P(bjac_solve_opts), P(bjac_stats), vp]),
        "bjac_stream_probe": (C.c_int, [vp, i32, vp, i32, C.c_int64, i32, i32, vp, vp]),
        "bjac_mlp_forward": (C.c_int, [vp, vp, i32, vp, vp, vp]),
        "bjac_mlp_workspace_query": (C.c_int, [i32, P(sz)]),
        "bjac_mlp_backward": (C.c_int, [vp, vp, vp, i32, vp, vp, vp, sz, vp]),
        "bjac_mlp_adam": (C.c_int, [vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float, C.c_float, vp]),
        "bjac_apply_multi": (C.c_int, [vp, vp, vp, i32, vp]),
        "bjac_poly_setup_query": (C.c_int, [P(bjac_csr), vp, i32, P(bjac_poly_params), P(sz)]),
        "bjac_poly_setup": (C.c_int, [P(bjac_csr), vp, i32, P(bjac_poly_params), vp, sz, vp, P(vp)]),
        "pcg_batched_workspace_query": (C.c_int, [P(bjac_csr), vp, i32, vp, vp, P(bjac_batch_cfg), P(sz)]),
        "pcg_solve_batched": (C.c_int, [P(bjac_csr), vp, i32, vp, vp, vp, vp, P(bjac_solve_opts),
                                        P(bjac_batch_cfg), vp, sz, vp, vp, vp, P(bjac_stats), vp]),
        "pcg_batched_tune": (C.c_int, [P(bjac_csr), vp, i32, vp, vp, vp, vp, P(bjac_batch_cfg), i32, i32, vp, sz,
                                       vp, P(i32), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class MpbjacError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        msg = load().bjac_strerror(code).decode()
        super().__init__(f"{what}: {msg} (code {code})")


def _check(code, what):
    if code < 0:
        raise MpbjacError(code, what)
    return code


def _torch():
    import torch
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


# ------------------------------------------------------------------ matrices
class DeviceCSR:
    """A CSR matrix resident in device memory (int32 indices, FP64 values)."""

    def __init__(self, A, device="cuda"):
        torch = _torch()
        self.n = int(A.n)
        self.nnz = int(A.nnz)
        self.row_ptr = torch.as_tensor(np.ascontiguousarray(A.row_ptr, dtype=np.int32), device=device)
        self.col_idx = torch.as_tensor(np.ascontiguousarray(A.col_idx, dtype=np.int32), device=device)
        self.val = torch.as_tensor(np.ascontiguousarray(A.val, dtype=np.float64), device=device)
        self.c = bjac_csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                          self.val.data_ptr())


def spmv(A: DeviceCSR, p):
    torch = _torch()
    q = torch.empty_like(p)
    _check(load().bjac_spmv(C.byref(A.c), _ptr(p), _ptr(q), _stream()), "bjac_spmv")
    return q


def round_bits(x, prec: int, scale: float = 1.0):
    """Correctly rounded RNE(x / scale) in FP32 / BF16 / FP16; returns the raw bits
    as an int32 (FP32) or int16 (16-bit) tensor."""
    torch = _torch()
    out = torch.empty(x.numel(), dtype=torch.int32 if prec == FP32 else torch.int16, device=x.device)
    _check(load().bjac_round(_ptr(x), _ptr(out), x.numel(), prec, float(scale), _stream()), "bjac_round")
    return out


# ------------------------------------------------------------ preconditioner
@dataclass
class Policy:
    mode: int = UNIFORM
    low: int = FP32
    temporal: int = TEMPORAL_NONE
    adp_tol: float = math.inf
    theta: float = 1e-2
    d16: float = 1.0
    mlp_blob: object = None          # device float tensor [MLP_NBLOB]
    explicit_tags: object = None     # numpy uint8 [nb]
    storage: int = STORE_FULL        # STORE_BAND: band-truncated inverses; STORE_SYM: upper quarters of blocks of 32-64
    band_rtol: float = 0.0           # <= 0: each block's unit roundoff

    def c(self):
        tags = None if self.explicit_tags is None else np.ascontiguousarray(self.explicit_tags, dtype=np.uint8)
        self._tags_keep = tags
        return bjac_policy(self.mode, self.low, self.temporal, self.storage, self.adp_tol, self.theta, self.d16,
                           self.mlp_blob.data_ptr() if self.mlp_blob is not None else None,
                           tags.ctypes.data if tags is not None else None, self.band_rtol)


class BlockJacobi:
    """Handle of a block-Jacobi setup: the stored precision maps live in a
    PyTorch-allocated workspace owned by this object."""

    def __init__(self, A: DeviceCSR, block_ptr, policy: Policy | None = None):
        torch = _torch()
        L = load()
        self.A = A
        self.policy = policy or Policy()
        self.block_ptr = np.ascontiguousarray(block_ptr, dtype=np.int32)
        self.nb = len(self.block_ptr) - 1
        pol = self.policy.c()
        nbytes = C.c_size_t()
        _check(L.bjac_setup_query(C.byref(A.c), self.block_ptr.ctypes.data, self.nb, C.byref(pol),
                                  C.byref(nbytes)), "bjac_setup_query")
        self.ws = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=A.val.device)
        h = C.c_void_p()
        _check(L.bjac_setup(C.byref(A.c), self.block_ptr.ctypes.data, self.nb, C.byref(pol), _ptr(self.ws),
                            nbytes.value, _stream(), C.byref(h)), "bjac_setup")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.bjac_destroy(h)
            self.h = None

    def info(self) -> dict:
        inf = bjac_info()
        _check(load().bjac_get_info(self.h, C.byref(inf)), "bjac_get_info")
        return {"n": inf.n, "nb": inf.nb, "max_block": inf.max_block,
                "blocks_per_prec": list(inf.blocks_per_prec), "low_bytes": inf.low_bytes,
                "high_bytes": inf.high_bytes, "temporal": inf.temporal, "mode": inf.mode, "ntiles": inf.ntiles}

    def tags(self) -> np.ndarray:
        out = np.empty(self.nb, dtype=np.uint8)
        _check(load().bjac_get_tags(self.h, out.ctypes.data), "bjac_get_tags")
        return out

    def features(self) -> np.ndarray:
        out = np.empty((self.nb, NFEAT), dtype=np.float32)
        _check(load().bjac_get_features(self.h, out.ctypes.data), "bjac_get_features")
        return out

    def block(self, k: int, which: int = 0):
        b = int(self.block_ptr[k + 1] - self.block_ptr[k])
        out = np.empty((b, b), dtype=np.float64)
        sc = C.c_double()
        _check(load().bjac_get_block(self.h, which, k, out.ctypes.data, C.byref(sc)), "bjac_get_block")
        return out, sc.value

    def band_widths(self, which: int = 0) -> np.ndarray:
        """Half-bandwidth of every stored block (band storage only)."""
        out = np.empty(self.nb, dtype=np.uint8)
        _check(load().bjac_get_band(self.h, which, out.ctypes.data), "bjac_get_band")
        return out

    def apply(self, r, which: int = 0):
        z = _torch().empty_like(r)
        _check(load().bjac_apply(self.h, which, _ptr(r), _ptr(z), _stream()), "bjac_apply")
        return z

    def apply_multi(self, R):
        """Z = M^-1 R for a contiguous (n, m) FP64 device tensor, m <= 8."""
        assert R.dim() == 2 and R.is_contiguous()
        Z = _torch().empty_like(R)
        _check(load().bjac_apply_multi(self.h, _ptr(R), _ptr(Z), R.shape[1], _stream()), "bjac_apply_multi")
        return Z


class PaperBJAC(BlockJacobi):
    """Handle of the paper-mode BJAC(k, t): k outer steps, t Jacobi sweeps per
    block solve, FP32 (low) or FP64 application; any block sizes. The device
    CSR must outlive the handle."""

    def __init__(self, A: DeviceCSR, block_ptr, k=2, t=2, low=True, temporal=TEMPORAL_NONE, adp_tol=math.inf):
        torch = _torch()
        L = load()
        self.A = A
        self.block_ptr = np.ascontiguousarray(block_ptr, dtype=np.int32)
        self.nb = len(self.block_ptr) - 1
        self.params = bjac_poly_params(int(k), int(t), 1 if low else 0, int(temporal), float(adp_tol))
        nbytes = C.c_size_t()
        _check(L.bjac_poly_setup_query(C.byref(A.c), self.block_ptr.ctypes.data, self.nb, C.byref(self.params),
                                       C.byref(nbytes)), "bjac_poly_setup_query")
        self.ws = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=A.val.device)
        h = C.c_void_p()
        _check(L.bjac_poly_setup(C.byref(A.c), self.block_ptr.ctypes.data, self.nb, C.byref(self.params),
                                 _ptr(self.ws), nbytes.value, _stream(), C.byref(h)), "bjac_poly_setup")
        self.h = h


@dataclass
class SolveResult:
    x: object
    iters: int
    status: int
    relres: float
    rnorm0: float
    high_applications: int
    graph_launches: int
    solve_ms: float
    relres_hist: object = None
    high_hist: object = None
    kernel_ms: dict = None        # profile mode: {"spmv": (total_ms, launches), ...}
    restarts: int = 0             # verify: residual replacements
    true_relres: float = -1.0     # verify: FP64 ||b - A x|| / ||b|| computed on the device


class Solver:
    """Reusable PCG workspace for one matrix size. ``compact_index`` (default)
    grows it to hold the compact copy of the matrix the SpMV reads
    (pcg_workspace_query_csr: 8-bit column and value codes, or 16-bit column
    offsets)."""

    def __init__(self, n: int, device="cuda", compact_index=True):
        torch = _torch()
        nbytes = C.c_size_t()
        _check(load().pcg_workspace_query(n, C.byref(nbytes)), "pcg_workspace_query")
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        self.n = n
        self.compact_index = compact_index

    def solve(self, A: DeviceCSR, M: BlockJacobi, b, tol=1e-10, maxit=5000, chunk=16, history=False, x=None,
              raise_on_error=True, profile=False, verify=0, variant=PCG_TEXTBOOK,
              cache_hints=HINTS_AUTO) -> SolveResult:
        torch = _torch()
        if self.compact_index:
            nbytes = C.c_size_t()
            _check(load().pcg_workspace_query_csr(C.byref(A.c), C.byref(nbytes)), "pcg_workspace_query_csr")
            if self.ws.numel() < nbytes.value:
                self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.ws.device)
        x = torch.empty_like(b) if x is None else x
        rh = torch.empty(maxit, dtype=torch.float64, device=b.device) if history else None
        hh = torch.zeros(maxit + 1, dtype=torch.uint8, device=b.device) if history else None
        opts = bjac_solve_opts(tol, maxit, chunk, rh.data_ptr() if rh is not None else None,
                               hh.data_ptr() if hh is not None else None, 1 if profile else 0, int(verify),
                               int(variant), int(cache_hints))
        st = bjac_stats()
        rc = load().pcg_solve(C.byref(A.c), M.h, _ptr(b), _ptr(x), C.byref(opts), _ptr(self.ws),
                              self.ws.numel(), C.byref(st), _stream())
        if rc < 0 and (raise_on_error or rc != EBREAKDOWN):
            raise MpbjacError(rc, "pcg_solve")
        res = SolveResult(x, st.iters, rc, st.relres, st.rnorm0, st.high_applications, st.graph_launches,
                          st.solve_ms, restarts=st.restarts, true_relres=st.true_relres)
        if profile:
            res.kernel_ms = {"spmv": (st.spmv_ms, st.n_spmv), "apply": (st.apply_ms, st.n_apply),
                             "update": (st.update_ms, st.n_update)}
        if history:
            res.relres_hist = rh[:st.iters].cpu().numpy()
            napp = st.iters if rc == OK else st.iters + 1   # no application after the converged update
            res.high_hist = hh[:napp].cpu().numpy()
        return res


def solve_noalloc(A: DeviceCSR, M: BlockJacobi, b, x, tol=1e-10, maxit=5000, chunk=16, variant=PCG_TEXTBOOK,
                  verify=0, cache_hints=HINTS_AUTO) -> SolveResult:
    """pcg_solve_noalloc: the solve with the library's static device
    workspace (no allocation inside the call; b and x are the caller's)."""
    opts = bjac_solve_opts(tol, maxit, chunk, None, None, 0, int(verify), int(variant), int(cache_hints))
    st = bjac_stats()
    rc = load().pcg_solve_noalloc(C.byref(A.c), M.h, _ptr(b), _ptr(x), C.byref(opts), C.byref(st), _stream())
    if rc < 0:
        raise MpbjacError(rc, "pcg_solve_noalloc")
    return SolveResult(x, st.iters, rc, st.relres, st.rnorm0, st.high_applications, st.graph_launches,
                       st.solve_ms, restarts=st.restarts, true_relres=st.true_relres)


def stream_probe(ins, outs, grid=0, unroll=1, sink=None):
    """bjac_stream_probe on lists of equal-length device FP64 tensors (one
    launch on the current stream)."""
    n = (ins[0] if ins else outs[0]).numel()
    pin = (C.c_void_p * max(1, len(ins)))(*[t.data_ptr() for t in ins])
    pout = (C.c_void_p * max(1, len(outs)))(*[t.data_ptr() for t in outs])
    _check(load().bjac_stream_probe(pin, len(ins), pout, len(outs), n, grid, unroll, _ptr(sink), _stream()),
           "bjac_stream_probe")


# ------------------------------------------------------------------- MLP
def mlp_forward(blob, feat, want_logits=True, want_tags=False):
    torch = _torch()
    n = feat.shape[0]
    logits = torch.empty((n, 3), dtype=torch.float32, device=feat.device) if want_logits else None
    tags = torch.empty(n, dtype=torch.uint8, device=feat.device) if want_tags else None
    _check(load().bjac_mlp_forward(_ptr(blob), _ptr(feat), n, _ptr(logits), _ptr(tags), _stream()),
           "bjac_mlp_forward")
    return logits, tags


class MlpTrainer:
    """Gradient and Adam steps of the selector network through the library."""

    def __init__(self, n: int, device="cuda"):
        torch = _torch()
        nbytes = C.c_size_t()
        _check(load().bjac_mlp_workspace_query(n, C.byref(nbytes)), "bjac_mlp_workspace_query")
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        self.n = n
        self.grad = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.m = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=device)
        self.v = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=device)
        self.t = 0

    def backward(self, blob, feat, labels):
        n = feat.shape[0]
        assert n <= self.n
        _check(load().bjac_mlp_backward(_ptr(blob), _ptr(feat), _ptr(labels), n, _ptr(self.grad),
                                        _ptr(self.loss), _ptr(self.ws), self.ws.numel(), _stream()),
               "bjac_mlp_backward")
        return self.grad, self.loss

    def adam(self, blob, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        _check(load().bjac_mlp_adam(_ptr(blob), _ptr(self.grad), _ptr(self.m), _ptr(self.v), self.t, lr, b1, b2,
                                    eps, _stream()), "bjac_mlp_adam")


# ------------------------------------------------------------ batched PCG
@dataclass
class BatchResult:
    x: object                 # device [sum rows_s * m_s], system-major, row-major per system
    col_iters: np.ndarray
    col_status: np.ndarray
    col_relres: np.ndarray
    status: int
    iters: int
    graph_launches: int
    solve_ms: float
    kernel_ms: dict = None        # profile mode: {"spmv": (total_ms, launches), ...}


class BatchSolver:
    """Batched multi-right-hand-side PCG over a stacked block-diagonal system.

    ``sys_row`` (nsys + 1 row offsets) and ``sys_m`` (columns per system) are
    host arrays; the workspace is sized for the largest of the configurations
    this object is asked to run."""

    def __init__(self, A: DeviceCSR, M: BlockJacobi, sys_row, sys_m):
        self.A, self.M = A, M
        self.sys_row = np.ascontiguousarray(sys_row, dtype=np.int32)
        self.sys_m = np.ascontiguousarray(sys_m, dtype=np.int32)
        self.nsys = len(self.sys_m)
        self.ncols = int(self.sys_m.sum())
        self.veclen = int(np.sum(np.diff(self.sys_row).astype(np.int64) * self.sys_m))
        self.ws = None

    def _query(self, cfg: bjac_batch_cfg) -> int:
        nbytes = C.c_size_t()
        _check(load().pcg_batched_workspace_query(C.byref(self.A.c), self.M.h, self.nsys,
                                                  self.sys_row.ctypes.data, self.sys_m.ctypes.data,
                                                  C.byref(cfg), C.byref(nbytes)), "pcg_batched_workspace_query")
        return nbytes.value

    def _ensure(self, nbytes: int):
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = _torch().empty(max(1, nbytes), dtype=_torch().uint8, device=self.A.val.device)

    def solve(self, b, tol=1e-10, maxit=5000, chunk=16, cfg=(0, 0, 0, 0), x=None, profile=False) -> BatchResult:
        torch = _torch()
        c = bjac_batch_cfg(*cfg)
        self._ensure(self._query(c))
        x = torch.empty_like(b) if x is None else x
        its = np.zeros(self.ncols, dtype=np.int32)
        sts = np.zeros(self.ncols, dtype=np.int32)
        rel = np.zeros(self.ncols, dtype=np.float64)
        opts = bjac_solve_opts(tol, maxit, chunk, None, None, 1 if profile else 0, 0)
        st = bjac_stats()
        rc = load().pcg_solve_batched(C.byref(self.A.c), self.M.h, self.nsys, self.sys_row.ctypes.data,
                                      self.sys_m.ctypes.data, _ptr(b), _ptr(x), C.byref(opts), C.byref(c),
                                      _ptr(self.ws), self.ws.numel(), its.ctypes.data, sts.ctypes.data,
                                      rel.ctypes.data, C.byref(st), _stream())
        if rc < 0 and rc != EBREAKDOWN:
            raise MpbjacError(rc, "pcg_solve_batched")
        res = BatchResult(x, its, sts, rel, rc, st.iters, st.graph_launches, st.solve_ms)
        if profile:
            res.kernel_ms = {"spmv": (st.spmv_ms, st.n_spmv), "apply": (st.apply_ms, st.n_apply),
                             "reduce": (st.update_ms, st.n_update)}
        return res

    def tune(self, b, cands, iters=8):
        """Times ``iters`` iterations under each (spmv_grab, wg_per_cu[, spmv_wg_per_cu[, apply_rows]]);
        returns (best index, ms per iteration of every candidate)."""
        torch = _torch()
        arr = (bjac_batch_cfg * len(cands))(*[bjac_batch_cfg(*c) for c in cands])
        self._ensure(max(self._query(c) for c in arr))
        x = torch.empty_like(b)
        ms = np.zeros(len(cands), dtype=np.float32)
        best = C.c_int32(-1)
        _check(load().pcg_batched_tune(C.byref(self.A.c), self.M.h, self.nsys, self.sys_row.ctypes.data,
                                       self.sys_m.ctypes.data, _ptr(b), _ptr(x), arr, len(cands), iters,
                                       _ptr(self.ws), self.ws.numel(), ms.ctypes.data, C.byref(best), _stream()),
               "pcg_batched_tune")
        return int(best.value), ms

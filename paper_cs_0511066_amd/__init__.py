"""Exact integer determinant on one MI355X: Python binding of libdet.so.

Argument marshalling only: every step of the computation runs in the HIP
library built from paper_cs_0511066_amd/csrc (kernels for gfx950 plus the
host reconstruction code).  The names follow the C ABI in include/det.h and
include/det_host.h.  Importing this package fails loudly when libdet.so has
not been built; there is no fallback.

Matrices may be numpy int64 arrays (host memory) or torch int64 CUDA tensors
(device memory, used in place).
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdet.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_cs_0511066_amd/_build.py` "
        "(or __graft_entry__.build())")

# One HIP runtime per process: torch ships its own libamdhip64 (same soname
# as the system one).  Loading torch first makes the dynamic linker bind
# libdet.so to that copy, so torch's device pointers and streams are valid
# handles for the library.  Without torch the system runtime is used.
try:
    import torch  # noqa: F401
except ImportError:   # pragma: no cover
    torch = None

_lib = ctypes.CDLL(LIB_PATH)

c_i64, c_u32, c_u64, c_int, c_double = ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
P = ctypes.POINTER

DET_OK = 0
STATUS = {0: "DET_OK", 1: "DET_E_INVALID", 2: "DET_E_NOT_PRIME", 3: "DET_E_PRIME_RANGE",
          4: "DET_E_SINGULAR_MOD_P", 5: "DET_E_OVERFLOW", 6: "DET_E_NOMEM",
          7: "DET_E_BUFFER_TOO_SMALL", 8: "DET_E_DEVICE"}
PATHS = {"auto": 0, "fp64": 1, "int8": 2}


class DetError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


class det_opts(ctypes.Structure):
    _fields_ = [("log2_inv_eps", c_double), ("certify", c_int), ("seed", c_u64),
                ("n_rhs", c_int), ("prime_bits", c_int), ("path", c_int), ("adaptive", c_int),
                ("lift_primes", c_int)]


class det_report(ctypes.Structure):
    _fields_ = [("primes_used", c_i64), ("lifting_steps", c_i64), ("sn_bits", c_i64),
                ("et_rounds", c_i64), ("hadamard_bits", c_i64), ("early_terminated", c_int),
                ("bonus_factors", c_int), ("t_lif_ms", c_double), ("t_cra_ms", c_double),
                ("t_host_ms", c_double), ("solvings", c_i64), ("timing_switch", c_int),
                ("t_solve_ms", c_double), ("t_lu_ms", c_double), ("lift_primes", c_i64)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("det_ctx_create", c_int, [c_int, ctypes.c_size_t, P(ctypes.c_void_p)])
_sig("det_ctx_destroy", None, [ctypes.c_void_p])
_sig("det_ctx_set_stream", c_int, [ctypes.c_void_p, ctypes.c_void_p])
_sig("det_status_str", ctypes.c_char_p, [c_int])
_sig("det_last_error", ctypes.c_char_p, [ctypes.c_void_p])
_sig("det_opts_default", None, [P(det_opts)])
_sig("det_mod_primes", c_int, [ctypes.c_void_p, ctypes.c_void_p, c_i64, c_i64, P(c_u32), c_i64,
                               P(c_u32), c_int])
_sig("dixon_lift", c_int, [ctypes.c_void_p, ctypes.c_void_p, c_i64, c_i64, P(c_i64), c_u32, c_i64,
                           P(c_u32)])
_sig("dixon_lift_multi", c_int, [ctypes.c_void_p, ctypes.c_void_p, c_i64, c_i64, P(c_i64), c_i64,
                                 c_u32, c_i64, P(c_u32)])
_sig("dixon_lift_primes", c_int, [ctypes.c_void_p, ctypes.c_void_p, c_i64, c_i64, P(c_i64), P(c_u32),
                                  c_i64, c_i64, P(c_u32)])
_sig("det_introspective", c_int, [ctypes.c_void_p, ctypes.c_void_p, c_i64, c_i64, P(det_opts),
                                  P(c_int), P(c_u32), c_i64, P(c_i64), P(det_report)])
_sig("det_batch", c_int, [ctypes.c_void_p, c_i64, P(ctypes.c_void_p), P(c_i64), P(c_i64),
                          P(det_opts), P(c_int), P(c_u32), c_i64, P(c_i64), P(c_int),
                          P(c_double)])
_sig("det_autotune", c_int, [ctypes.c_void_p, ctypes.c_char_p])
_sig("det_autotune_read", c_int, [ctypes.c_void_p, c_i64, P(ctypes.c_int32), P(ctypes.c_int32),
                                  P(ctypes.c_int32), P(c_double), P(c_i64)])
_sig("det_mod_primes_noalloc", c_int, [c_int, ctypes.c_void_p, ctypes.c_void_p, c_i64, c_i64,
                                       P(c_u32), c_i64, P(c_u32)])
class det_server_report(ctypes.Structure):
    _fields_ = [("submitted", c_i64), ("completed", c_i64), ("waiting", c_i64), ("admitted", c_i64),
                ("max_admitted", c_i64), ("rounds", c_i64), ("queue_items", c_i64),
                ("hbm_budget", c_i64), ("hbm_in_use", c_i64), ("hbm_peak", c_i64)]


_sig("det_server_create", c_int, [ctypes.c_void_p, ctypes.c_size_t, P(det_opts), P(ctypes.c_void_p)])
_sig("det_server_submit", c_int, [ctypes.c_void_p, ctypes.c_void_p, c_i64, c_i64, P(c_i64)])
_sig("det_server_poll", c_int, [ctypes.c_void_p, c_i64, c_int, P(c_int), P(c_int), P(c_u32), c_i64,
                                P(c_i64), P(c_double)])
_sig("det_server_stats", c_int, [ctypes.c_void_p, P(det_server_report)])
_sig("det_server_destroy", None, [ctypes.c_void_p])
_sig("det_profile_select", c_int, [ctypes.c_void_p, c_int])
_sig("det_profile_read", c_int, [ctypes.c_void_p, P(c_i64), P(c_double), P(c_double), P(c_double)])
_sig("det_host_is_prime", c_int, [c_u32])
_sig("det_host_sample_primes", c_int, [c_u64, c_int, c_i64, P(c_u32)])
_sig("det_host_hadamard_log2", c_double, [P(c_i64), c_i64, c_i64])
_sig("det_host_et_run_length", c_i64, [c_double, c_int, c_double])
_sig("det_host_crt", c_int, [P(c_u32), P(c_u32), c_i64, P(c_int), P(c_u32), c_i64, P(c_i64), P(c_i64)])
_sig("det_host_ratrecon", c_int, [P(c_u32), c_i64, P(c_u32), c_i64, c_i64, c_i64, c_u64, P(c_int),
                                  P(c_u32), c_i64, P(c_i64), P(c_u32), c_i64, P(c_i64)])
_sig("det_host_bigint", c_int, [c_int, c_int, P(c_u32), c_i64, c_int, P(c_u32), c_i64, P(c_int),
                                P(c_u32), c_i64, P(c_i64)])
_sig("det_host_extended_bonus", c_int, [P(c_u64), c_i64, c_i64, P(c_u32), c_i64, c_i64, c_i64,
                                        P(c_u32), c_i64, P(c_i64), P(c_u32), c_i64, P(c_i64),
                                        P(c_i64)])

EXPORTED = ["det_ctx_create", "det_ctx_destroy", "det_ctx_set_stream", "det_status_str",
            "det_last_error", "det_opts_default", "det_mod_primes", "dixon_lift", "dixon_lift_multi",
            "dixon_lift_primes",
            "det_introspective", "det_batch", "det_autotune", "det_autotune_read",
            "det_mod_primes_noalloc", "det_server_create", "det_server_submit", "det_server_poll",
            "det_server_stats", "det_server_destroy", "det_profile_select", "det_profile_read", "det_host_is_prime", "det_host_sample_primes",
            "det_host_hadamard_log2", "det_host_et_run_length", "det_host_crt",
            "det_host_ratrecon", "det_host_bigint", "det_host_extended_bonus"]


# ------------------------------------------------------------------ helpers
def _u32p(a: np.ndarray):
    return a.ctypes.data_as(P(c_u32))


def _i64p(a: np.ndarray):
    return a.ctypes.data_as(P(c_i64))


def _to_limbs(v: int) -> np.ndarray:
    v = abs(int(v))
    out = []
    while v:
        out.append(v & 0xFFFFFFFF)
        v >>= 32
    return np.asarray(out, dtype=np.uint32)


def _from_limbs(sign: int, limbs) -> int:
    v = 0
    for x in reversed(list(limbs)):
        v = (v << 32) | int(x)
    return sign * v


def _matrix_arg(A):
    """(pointer, n, lda, keepalive) for a numpy int64 matrix or a torch int64
    CUDA tensor (row-major, unit column stride)."""
    try:
        import torch  # noqa: F401
        is_tensor = hasattr(A, "data_ptr") and hasattr(A, "is_cuda")
    except ImportError:
        is_tensor = False
    if is_tensor:
        import torch
        if A.dtype != torch.int64 or A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1:
            raise ValueError("expected a square row-major int64 tensor")
        return ctypes.c_void_p(A.data_ptr()), int(A.shape[0]), int(A.stride(0)), A
    M = np.ascontiguousarray(np.asarray(A, dtype=np.int64))
    if M.ndim != 2 or M.shape[0] != M.shape[1]:
        raise ValueError("expected a square matrix")
    n = M.shape[0]
    return ctypes.c_void_p(M.ctypes.data if n else 0), n, max(n, 1), M


# Contexts still open when the interpreter exits are closed by an atexit
# handler, which runs before any module or runtime teardown; a context found
# by the garbage collector during finalisation is left alone (its memory goes
# with the process), so no HIP call is made after the runtime has started to
# shut down.
_live: "weakref.WeakSet[Context]" = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    for c in list(_live):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """A det_ctx: device workspace and stream of the library."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        st = _lib.det_ctx_create(device, hbm_budget_bytes, ctypes.byref(h))
        if st != DET_OK:
            raise DetError(st, "det_ctx_create failed (no usable HIP device?)")
        self._h = h
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _lib.det_ctx_destroy(h)

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st: int):
        if st != DET_OK:
            raise DetError(st, _lib.det_last_error(self._h).decode())

    KERNELS = {"none": 0, "lift_x": 1, "lift_r": 2, "gemm_f64": 3, "gemm_i8": 4, "panel": 5,
               "trsm": 6, "tri_inv": 7, "residues": 8, "lift": 9}

    def profile_select(self, kernel: str):
        """Time every launch of one kernel class with HIP events (det_profile_select)."""
        self._check(_lib.det_profile_select(self._h, self.KERNELS[kernel]))

    def profile_read(self) -> dict:
        """Launch count, summed ms, algorithmic bytes and ops since the last read."""
        n, ms, b, o = c_i64(0), c_double(0), c_double(0), c_double(0)
        self._check(_lib.det_profile_read(self._h, ctypes.byref(n), ctypes.byref(ms),
                                          ctypes.byref(b), ctypes.byref(o)))
        return {"launches": int(n.value), "ms": float(ms.value), "bytes": float(b.value),
                "ops": float(o.value)}

    def set_stream(self, hip_stream: int | None):
        self._check(_lib.det_ctx_set_stream(self._h, ctypes.c_void_p(hip_stream or 0)))

    # ---- entry points (names of include/det.h)
    def det_mod_primes(self, A, primes, path: str = "auto") -> np.ndarray:
        ptr, n, lda, keep = _matrix_arg(A)
        ps = np.ascontiguousarray(np.asarray(primes, dtype=np.uint32))
        out = np.zeros(len(ps), dtype=np.uint32)
        self._check(_lib.det_mod_primes(self._h, ptr, n, lda, _u32p(ps), len(ps), _u32p(out),
                                        PATHS[path]))
        del keep
        return out

    def dixon_lift(self, A, b, p: int, k: int) -> np.ndarray:
        ptr, n, lda, keep = _matrix_arg(A)
        bb = np.ascontiguousarray(np.asarray(b, dtype=np.int64))
        if bb.shape != (n,):
            raise ValueError("b must have n entries")
        out = np.zeros((k, n), dtype=np.uint32)
        self._check(_lib.dixon_lift(self._h, ptr, n, lda, _i64p(bb), p, k, _u32p(out)))
        del keep
        return out

    def dixon_lift_multi(self, A, B, p: int, k: int) -> np.ndarray:
        """Digits of A^{-1} b_h mod p^k for every column b_h of the n x m
        matrix B (dixon_lift_multi): an m x k x n array."""
        ptr, n, lda, keep = _matrix_arg(A)
        BB = np.ascontiguousarray(np.asarray(B, dtype=np.int64))
        if BB.ndim != 2 or BB.shape[0] != n:
            raise ValueError("B must be n x m")
        m = BB.shape[1]
        out = np.zeros((m, k, n), dtype=np.uint32)
        self._check(_lib.dixon_lift_multi(self._h, ptr, n, lda, _i64p(BB), m, p, k, _u32p(out)))
        del keep
        return out

    def dixon_lift_primes(self, A, b, primes, k: int) -> np.ndarray:
        """Digits of A^{-1} b mod p_z^k for several primes lifted side by side
        (dixon_lift_primes): an np x k x n array."""
        ptr, n, lda, keep = _matrix_arg(A)
        bb = np.ascontiguousarray(np.asarray(b, dtype=np.int64))
        if bb.shape != (n,):
            raise ValueError("b must have n entries")
        ps = np.ascontiguousarray(np.asarray(primes, dtype=np.uint32))
        out = np.zeros((len(ps), k, n), dtype=np.uint32)
        self._check(_lib.dixon_lift_primes(self._h, ptr, n, lda, _i64p(bb), _u32p(ps), len(ps), k,
                                           _u32p(out)))
        del keep
        return out

    def det_introspective(self, A, certify: bool = False, seed: int | None = None,
                          log2_inv_eps: float | None = None, n_rhs: int | None = None,
                          prime_bits: int | None = None, path: str | None = None,
                          adaptive: bool | None = None, report: bool = False,
                          lift_primes: int | None = None):
        ptr, n, lda, keep = _matrix_arg(A)
        o = det_opts()
        _lib.det_opts_default(ctypes.byref(o))
        o.certify = int(bool(certify))
        if lift_primes is not None:
            o.lift_primes = lift_primes
        if seed is not None:
            o.seed = seed
        if log2_inv_eps is not None:
            o.log2_inv_eps = log2_inv_eps
        if n_rhs is not None:
            o.n_rhs = n_rhs
        if prime_bits is not None:
            o.prime_bits = prime_bits
        if path is not None:
            o.path = PATHS[path]
        if adaptive is not None:
            o.adaptive = int(bool(adaptive))
        cap = max(8, 2 * n + 8)
        rep = det_report()
        while True:
            mag = np.zeros(cap, dtype=np.uint32)
            sign = c_int(0)
            cnt = c_i64(0)
            st = _lib.det_introspective(self._h, ptr, n, lda, ctypes.byref(o), ctypes.byref(sign),
                                        _u32p(mag), cap, ctypes.byref(cnt), ctypes.byref(rep))
            if st == 7:
                cap = int(cnt.value)
                continue
            self._check(st)
            break
        del keep
        det = _from_limbs(sign.value, mag[:cnt.value])
        if report:
            return det, {f: getattr(rep, f) for f, _ in det_report._fields_}
        return det


    def det_batch(self, matrices, certify: bool = False, seed: int | None = None,
                  log2_inv_eps: float | None = None, prime_bits: int | None = None,
                  timings: bool = False):
        """Exact determinants of a list of square int64 matrices (numpy or
        torch CUDA tensors of any sizes) in one det_batch call.  Returns the
        list of determinants, and with timings=True also the time at which
        each result was ready, in ms since the call started."""
        args = [_matrix_arg(A) for A in matrices]
        m = len(args)
        o = det_opts()
        _lib.det_opts_default(ctypes.byref(o))
        o.certify = int(bool(certify))
        if seed is not None:
            o.seed = seed
        if log2_inv_eps is not None:
            o.log2_inv_eps = log2_inv_eps
        if prime_bits is not None:
            o.prime_bits = prime_bits
        ptrs = (ctypes.c_void_p * max(m, 1))(*[a[0] for a in args])
        ns = np.asarray([a[1] for a in args] or [0], dtype=np.int64)
        ldas = np.asarray([a[2] for a in args] or [0], dtype=np.int64)
        stride = max(8, 2 * int(ns.max()) + 8) if m else 8
        while True:
            sign = np.zeros(max(m, 1), dtype=np.int32)
            mag = np.zeros(max(m, 1) * stride, dtype=np.uint32)
            cnt = np.zeros(max(m, 1), dtype=np.int64)
            stat = np.zeros(max(m, 1), dtype=np.int32)
            tdone = np.zeros(max(m, 1), dtype=np.float64)
            st = _lib.det_batch(self._h, m, ptrs, _i64p(ns), _i64p(ldas), ctypes.byref(o),
                                sign.ctypes.data_as(P(c_int)), _u32p(mag), stride, _i64p(cnt),
                                stat.ctypes.data_as(P(c_int)), tdone.ctypes.data_as(P(c_double)))
            if st == 7 and np.any(stat[:m] == 7):
                stride = int(cnt[:m].max())
                continue
            self._check(st)
            break
        del args
        dets = [_from_limbs(int(sign[i]), mag[i * stride:i * stride + int(cnt[i])]) for i in range(m)]
        if timings:
            return dets, tdone[:m].tolist()
        return dets

    def autotune(self, cache_path: str | None = None) -> list[dict]:
        """Run (or load from cache_path) the launch-shape autotuner of the
        persistent LU kernel (det_autotune); returns the table."""
        self._check(_lib.det_autotune(self._h, cache_path.encode() if cache_path else None))
        return self.autotune_table()

    def autotune_table(self) -> list[dict]:
        cap = 16
        nm = np.zeros(cap, dtype=np.int32)
        va = np.zeros(cap, dtype=np.int32)
        bp = np.zeros(cap, dtype=np.int32)
        ip = np.zeros(cap, dtype=np.float64)
        cnt = c_i64(0)
        i32 = P(ctypes.c_int32)
        self._check(_lib.det_autotune_read(self._h, cap, nm.ctypes.data_as(i32), va.ctypes.data_as(i32),
                                           bp.ctypes.data_as(i32), ip.ctypes.data_as(P(c_double)),
                                           ctypes.byref(cnt)))
        return [{"nmax": int(nm[i]), "variant": int(va[i]), "blocks_per_cu": int(bp[i]),
                 "items_per_ms": float(ip[i])} for i in range(min(cap, cnt.value))]


def det_mod_primes_noalloc(A, primes, device: int = 0, hip_stream: int | None = None) -> np.ndarray:
    """det(A) mod p for each prime with no device allocation by the library
    (det_mod_primes_noalloc): A must be a torch int64 CUDA tensor."""
    ptr, n, lda, keep = _matrix_arg(A)
    ps = np.ascontiguousarray(np.asarray(primes, dtype=np.uint32))
    out = np.zeros(len(ps), dtype=np.uint32)
    st = _lib.det_mod_primes_noalloc(device, ctypes.c_void_p(hip_stream or 0), ptr, n, lda,
                                     _u32p(ps), len(ps), _u32p(out))
    del keep
    if st != DET_OK:
        raise DetError(st, "det_mod_primes_noalloc")
    return out


class Server:
    """A det_server on a context (det_server_*): submit matrices, poll for
    their determinants.  The context must not be used while the server runs."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, seed: int | None = None,
                 certify: bool = False, log2_inv_eps: float | None = None,
                 prime_bits: int | None = None, lift_primes: int | None = None):
        o = det_opts()
        _lib.det_opts_default(ctypes.byref(o))
        o.certify = int(bool(certify))
        if lift_primes is not None:
            o.lift_primes = lift_primes
        if seed is not None:
            o.seed = seed
        if log2_inv_eps is not None:
            o.log2_inv_eps = log2_inv_eps
        if prime_bits is not None:
            o.prime_bits = prime_bits
        h = ctypes.c_void_p()
        ctx._check(_lib.det_server_create(ctx._h, hbm_budget_bytes, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._ctx = ctx
        self._keep = {}

    def submit(self, A) -> int:
        ptr, n, lda, keep = _matrix_arg(A)
        rid = c_i64(0)
        st = _lib.det_server_submit(self._h, ptr, n, lda, ctypes.byref(rid))
        if st != DET_OK:
            raise DetError(st, "det_server_submit")
        self._keep[rid.value] = n
        return int(rid.value)

    def poll(self, request_id: int, timeout_ms: int = -1):
        """(done, det or None, latency_ms or None)."""
        n = self._keep.get(request_id, 0)
        cap = max(8, 2 * n + 8)
        while True:
            done, sign, cnt, lat = c_int(0), c_int(0), c_i64(0), c_double(0)
            mag = np.zeros(cap, dtype=np.uint32)
            st = _lib.det_server_poll(self._h, request_id, timeout_ms, ctypes.byref(done),
                                      ctypes.byref(sign), _u32p(mag), cap, ctypes.byref(cnt),
                                      ctypes.byref(lat))
            if st == 7:
                cap = int(cnt.value)
                continue
            if st != DET_OK:
                raise DetError(st, "det_server_poll")
            if not done.value:
                return False, None, None
            return True, _from_limbs(sign.value, mag[:cnt.value]), float(lat.value)

    def stats(self) -> dict:
        r = det_server_report()
        st = _lib.det_server_stats(self._h, ctypes.byref(r))
        if st != DET_OK:
            raise DetError(st, "det_server_stats")
        return {f: int(getattr(r, f)) for f, _ in det_server_report._fields_}

    def close(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _lib.det_server_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


_default_ctx: Context | None = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(0)
    return _default_ctx


def det_mod_primes(A, primes, path: str = "auto") -> np.ndarray:
    """residues[j] = det(A) mod primes[j] (see include/det.h)."""
    return default_context().det_mod_primes(A, primes, path)


def dixon_lift(A, b, p: int, k: int) -> np.ndarray:
    """k x n base-p digits of A^{-1} b (see include/det.h)."""
    return default_context().dixon_lift(A, b, p, k)


def det_introspective(A, **kw):
    """Exact det(A) as a Python int (see include/det.h)."""
    return default_context().det_introspective(A, **kw)


# ------------------------------------------------------------------ host-side steps
def det_host_is_prime(q: int) -> bool:
    return bool(_lib.det_host_is_prime(q))


def det_host_sample_primes(seed: int, bits: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint32)
    st = _lib.det_host_sample_primes(seed, bits, count, _u32p(out))
    if st != DET_OK:
        raise DetError(st)
    return out


def det_host_hadamard_log2(A) -> float:
    M = np.ascontiguousarray(np.asarray(A, dtype=np.int64))
    n = M.shape[0]
    return float(_lib.det_host_hadamard_log2(_i64p(M), n, max(n, 1)))


def det_host_et_run_length(log2_inv_eps: float, bits: int, logl_H: float) -> int:
    return int(_lib.det_host_et_run_length(log2_inv_eps, bits, logl_H))


def det_host_crt(residues, primes):
    """(r, same_run): symmetric-range CRT value and the trailing unchanged run."""
    rs = np.ascontiguousarray(np.asarray(residues, dtype=np.uint32))
    ps = np.ascontiguousarray(np.asarray(primes, dtype=np.uint32))
    cap = 2 * len(ps) + 4
    mag = np.zeros(cap, dtype=np.uint32)
    sign, ln, same = c_int(0), c_i64(0), c_i64(0)
    st = _lib.det_host_crt(_u32p(rs), _u32p(ps), len(ps), ctypes.byref(sign), _u32p(mag), cap,
                           ctypes.byref(ln), ctypes.byref(same))
    if st != DET_OK:
        raise DetError(st)
    return _from_limbs(sign.value, mag[:ln.value]), int(same.value)


def det_host_ratrecon(u: int, m: int, Nbits: int, Dbits: int, prime_base: int = 0):
    """(a, d) with a = u d mod m, |a| <= 2^Nbits, 0 < d <= 2^Dbits, or None
    (prime_base: q when m is a power of the prime q, else 0)."""
    ul, ml = _to_limbs(u % m), _to_limbs(m)
    cap = len(ml) + 4
    am, dm = np.zeros(cap, dtype=np.uint32), np.zeros(cap, dtype=np.uint32)
    asg, al, dl = c_int(0), c_i64(0), c_i64(0)
    st = _lib.det_host_ratrecon(_u32p(ul), len(ul), _u32p(ml), len(ml), Nbits, Dbits, prime_base,
                                ctypes.byref(asg), _u32p(am), cap, ctypes.byref(al), _u32p(dm), cap,
                                ctypes.byref(dl))
    if st == 1:
        return None
    if st != DET_OK:
        raise DetError(st)
    return _from_limbs(asg.value, am[:al.value]), _from_limbs(1, dm[:dl.value])


def det_host_bigint(op: str, a: int, b: int) -> int:
    code = {"add": 0, "sub": 1, "mul": 2, "floordiv": 3, "mod": 4, "gcd": 5}[op]
    al, bl = _to_limbs(a), _to_limbs(b)
    sa = (a > 0) - (a < 0)
    sb = (b > 0) - (b < 0)
    cap = len(al) + len(bl) + 4
    out = np.zeros(cap, dtype=np.uint32)
    so, ln = c_int(0), c_i64(0)
    st = _lib.det_host_bigint(code, sa, _u32p(al), len(al), sb, _u32p(bl), len(bl),
                              ctypes.byref(so), _u32p(out), cap, ctypes.byref(ln))
    if st != DET_OK:
        raise DetError(st)
    return _from_limbs(so.value, out[:ln.value])


def det_host_extended_bonus(comb, p, Nbits: int, Dbits: int):
    """(s~, pi~, failed) of the extended bonus from the combination digits:
    comb[h, a, i] = R_a . (digit i of x_h) for one prime p (an m x m x k
    array), or comb[h, a, z, i] = R_a . (digit i of x_h mod p_z) for a list
    of primes p (m x m x np x k), the liftings combined by Chinese
    remaindering."""
    cb = np.asarray(comb, dtype=np.uint64)
    primes = [int(p)] if np.isscalar(p) else [int(q) for q in p]
    if cb.ndim == 3:
        cb = cb[:, :, None, :]
    if cb.ndim != 4 or cb.shape[0] != cb.shape[1] or cb.shape[2] != len(primes):
        raise ValueError("comb must be m x m x k (one prime) or m x m x np x k")
    cb = np.ascontiguousarray(cb)
    m, _, npr, k = cb.shape
    ps = np.ascontiguousarray(np.asarray(primes, dtype=np.uint32))
    cap = int((Nbits + Dbits) * m // 32 + 8)
    sm, pm = np.zeros(cap, dtype=np.uint32), np.zeros(cap, dtype=np.uint32)
    sl, pl, failed = c_i64(0), c_i64(0), c_i64(0)
    st = _lib.det_host_extended_bonus(cb.ctypes.data_as(P(c_u64)), m, k, _u32p(ps), npr, Nbits,
                                      Dbits, _u32p(sm), cap, ctypes.byref(sl), _u32p(pm), cap,
                                      ctypes.byref(pl), ctypes.byref(failed))
    if st != DET_OK:
        raise DetError(st)
    return _from_limbs(1, sm[:sl.value]), _from_limbs(1, pm[:pl.value]), int(failed.value)

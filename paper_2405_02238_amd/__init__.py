"""Python binding of the MI355X HE matrix-multiplication library (libhegmm.so).

Argument marshalling only: every step of the method runs in the HIP library.
The binding loads the in-tree `libhegmm.so` (built by `build.py`) and raises
if it is missing; there is no fallback.  torch is used only to name the HIP
stream work is enqueued on.

Names follow include/hegmm.h: keygen / encrypt / hegmm / decrypt are the
client-encrypt, cloud-multiply, client-decrypt split of the paper's
Algorithm 2 (HEGMM-Enhanced) for C = A x B of arbitrary shape.
"""
from __future__ import annotations

import ctypes
import os
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhegmm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "hegmm.h")

HG_OK, HG_EINVAL, HG_ENOFIT, HG_ENOKEY, HG_ENOMEM, HG_EDEVICE, HG_ESTATE = 0, -1, -2, -3, -4, -5, -6
_NAMES = {-1: "EINVAL", -2: "ENOFIT", -3: "ENOKEY", -4: "ENOMEM", -5: "EDEVICE", -6: "ESTATE"}


class HGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class _ServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("lanes", ctypes.c_int32), ("hbm_budget", ctypes.c_uint64)]


class _Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("t", ctypes.c_uint64), ("L", ctypes.c_uint32),
                ("alpha", ctypes.c_uint32), ("method", ctypes.c_uint32), ("min_blocks", ctypes.c_uint32),
                ("relin", ctypes.c_uint32), ("ks_order", ctypes.c_uint32), ("prime_bits", ctypes.c_uint32),
                ("sigma", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_SIGS = {
    "hg_ctx_create": [ctypes.POINTER(_Params), ctypes.c_int, _PP],
    "hg_set_allocator": [_P, _ALLOC_FN, _RELEASE_FN, _P],
    "hg_keygen": [_P, ctypes.c_uint64, _i32p, ctypes.c_size_t],
    "hg_keygen_rotations": [_P, _i32p, ctypes.c_size_t],
    "hg_drop_secret": [_P],
    "hg_encrypt": [_P, ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _PP],
    "hg_hegmm": [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _PP, _P],
    "hg_hegmm_batch": [_P, ctypes.c_size_t, _PP, _PP, _i32p, _PP, _P],
    "hg_hegmm_noalloc": [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P],
    "hg_decrypt": [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _u64p],
    "hg_ct_export": [_P, _P, _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
    "hg_ct_import": [_P, _u64p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, _PP],
    "hg_encrypt_slots": [_P, _i64p, ctypes.c_uint64, _PP],
    "hg_decrypt_slots": [_P, _P, _u64p],
    "hg_rotate": [_P, _P, ctypes.c_int, _PP, _P],
    "hg_mul": [_P, _P, _P, _PP, _P],
    "hg_add": [_P, _P, _P, _PP, _P],
    "hg_cmul": [_P, _P, _i64p, _PP, _P],
    "hg_mod_switch": [_P, _P, ctypes.c_int, _PP, _P],
    "hg_plan_info": [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64p],
    "hg_primes": [_P, _u64p],
    "hg_set_timing": [_P, ctypes.c_int],
    "hg_tune": [_P, ctypes.c_char_p, ctypes.c_int64],
    "hg_last_timing": [_P, _f64p],
    "hg_launch_timing": [_P, _f64p],
    "hg_request_footprint": [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)],
    "hg_server_create": [_P, _P, _PP],
    "hg_server_submit": [_P, _u64p, ctypes.c_size_t, _u64p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                         ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)],
    "hg_server_wait": [_P, ctypes.c_uint64, _P, ctypes.c_size_t, _P],
    "hg_server_stats": [_P, _f64p],
    "hg_server_pause": [_P, ctypes.c_int],
    "hg_set_partition": [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int, _i32p, ctypes.c_int],
    "hg_get_partition": [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, ctypes.c_size_t,
                         ctypes.POINTER(ctypes.c_size_t)],
    "hg_bench_modmul": [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64)],
    "hg_bench_stream": [ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)],
    "hg_graph_create": [_P, ctypes.c_size_t, _PP, _PP, _i32p, _PP, _PP],
    "hg_graph_launch": [_P, _P],
    "hg_ct_load": [_P, _P, _u64p, ctypes.c_size_t, _P],
}


def declared_symbols() -> List[str]:
    """Every entry point declared in include/hegmm.h."""
    import re
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hg_[a-z_0-9]+)\s*\(", text)))


def load(path: str = LIB_PATH):
    """Load libhegmm.so; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2405_02238_amd.build`")
    lib = ctypes.CDLL(path)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    lib.hg_ctx_destroy.argtypes = [_P]
    lib.hg_ctx_destroy.restype = None
    lib.hg_ct_free.argtypes = [_P]
    lib.hg_ct_free.restype = None
    lib.hg_server_destroy.argtypes = [_P]
    lib.hg_server_destroy.restype = None
    lib.hg_graph_destroy.argtypes = [_P]
    lib.hg_graph_destroy.restype = None
    lib.hg_last_error.argtypes = []
    lib.hg_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(code: int):
    if code != HG_OK:
        raise HGError(code, _lib.hg_last_error().decode())


def bench_modmul(form: int, q: int, blocks: int = 4096, iters: int = 256, reps: int = 5, device: int = 0) -> float:
    """hg_bench_modmul: modular products per second (form 0 FP64, 1 Shoup, 2 Barrett)."""
    load()
    out = ctypes.c_double(0.0)
    chk = ctypes.c_uint64(0)
    _check(_lib.hg_bench_modmul(device, form, q, blocks, iters, reps, ctypes.byref(out), ctypes.byref(chk)))
    return out.value


def bench_stream(nbytes: int, mode: int, reps: int = 5, device: int = 0) -> float:
    """hg_bench_stream: bytes per second read (mode 0) or read + written (mode 1)."""
    load()
    out = ctypes.c_double(0.0)
    _check(_lib.hg_bench_stream(device, nbytes, mode, reps, ctypes.byref(out)))
    return out.value


def current_stream() -> Optional[int]:
    """The HIP stream torch currently uses on its device (None: null stream)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


class Ciphertext:
    """Handle of a device ciphertext (packed operand, result or raw slot ct)."""

    def __init__(self, ctx: "Context", ptr: int):
        self.ctx = ctx
        self.ptr = ptr

    def free(self):
        if self.ptr:
            _lib.hg_ct_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def export(self) -> np.ndarray:
        """Canonical serialisation (coefficient form, residues in [0, q_i))."""
        need = ctypes.c_size_t(0)
        _check(_lib.hg_ct_export(self.ctx.ptr, self.ptr, None, 0, ctypes.byref(need)))
        buf = np.empty(need.value, dtype=np.uint64)
        _check(_lib.hg_ct_export(self.ctx.ptr, self.ptr, buf.ctypes.data, need.value, ctypes.byref(need)))
        return buf


class Context:
    """hg_ctx: one BGV parameter set on one GPU."""

    def __init__(self, N: int, t: int, L: int, alpha: int, device: int = 0, method: int = 2, min_blocks: int = 1,
                 relin: int = 0, ks_order: int = 0, prime_bits: int = 50, sigma: float = 3.2):
        """method 2: HEGMM-En (Algorithm 2); method 1: Algorithm 1, for comparison
        (method 3: Algorithm 1 with sigma / tau evaluated on the ciphertexts).
        min_blocks > 1 forces that many inner blocks per product; relin 1
        relinearises every loop product on its own (eager); ks_order 1 composes
        every linear transform in the paper's HE-Rot, HE-CMult, HE-Add order
        (one division by P per rotation); prime_bits bounds the primes; sigma
        is the error width (hg_params)."""
        load()
        p = _Params(N, t, L, alpha, method, min_blocks, relin, ks_order, prime_bits, sigma)
        out = ctypes.c_void_p()
        _check(_lib.hg_ctx_create(ctypes.byref(p), device, ctypes.byref(out)))
        self.ptr = out.value
        self.N, self.t, self.L, self.alpha, self.method, self.min_blocks = N, t, L, alpha, method, min_blocks
        self.relin = relin
        self.ks_order, self.prime_bits = ks_order, prime_bits
        self.device = device
        self.S = N // 2

    def close(self):
        if getattr(self, "ptr", None):
            _lib.hg_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ct(self, out: ctypes.c_void_p) -> Ciphertext:
        return Ciphertext(self, out.value)

    def set_allocator(self, alloc: Optional[Callable[[int, Optional[int]], int]],
                      release: Optional[Callable[[int], None]]):
        """hg_set_allocator: alloc(nbytes, stream) -> device pointer (0 on
        failure), release(ptr); both None restores hipMalloc / hipFree."""
        if alloc is None and release is None:
            _check(_lib.hg_set_allocator(self.ptr, _ALLOC_FN(), _RELEASE_FN(), None))
            self._alloc_cbs = None
            return
        a = _ALLOC_FN(lambda nbytes, stream, user: alloc(nbytes, stream) or None)
        r = _RELEASE_FN(lambda ptr, user: release(ptr))
        _check(_lib.hg_set_allocator(self.ptr, a, r, None))
        # every callback object stays alive as long as the context: handles made
        # while it was in force still return their memory through it
        self._alloc_cbs_all = getattr(self, "_alloc_cbs_all", []) + [(a, r)]
        self._alloc_cbs = (a, r)

    def use_torch_allocator(self):
        """Route ciphertext handles through torch's caching allocator (stream
        ordered; freeing a handle then does not wait for the device)."""
        import torch
        dev = self.device

        def alloc(nbytes, stream):
            return torch.cuda.caching_allocator_alloc(nbytes, device=dev, stream=stream or 0)

        self.set_allocator(alloc, torch.cuda.caching_allocator_delete)

    def keygen(self, seed: int, shapes: Sequence[Tuple[int, int, int]] = ()):
        arr = np.ascontiguousarray(np.array(list(shapes), dtype=np.int32).reshape(-1))
        _check(_lib.hg_keygen(self.ptr, seed, arr, len(shapes)))

    def keygen_rotations(self, zs: Sequence[int]):
        arr = np.ascontiguousarray(np.array(list(zs), dtype=np.int32))
        _check(_lib.hg_keygen_rotations(self.ptr, arr, len(arr)))

    def drop_secret(self):
        _check(_lib.hg_drop_secret(self.ptr))

    def encrypt(self, role: int, X: np.ndarray, m: int, l: int, n: int, nonce: int = 0) -> Ciphertext:
        X = np.ascontiguousarray(np.asarray(X, dtype=np.int64).reshape(-1))
        out = ctypes.c_void_p()
        _check(_lib.hg_encrypt(self.ptr, role, X, m, l, n, nonce, ctypes.byref(out)))
        return self._ct(out)

    def hegmm(self, A: Ciphertext, B: Ciphertext, m: int, l: int, n: int, stream: Optional[int] = None) -> Ciphertext:
        out = ctypes.c_void_p()
        s = current_stream() if stream is None else stream
        _check(_lib.hg_hegmm(self.ptr, A.ptr, B.ptr, m, l, n, ctypes.byref(out), s))
        return self._ct(out)

    def set_partition(self, m: int, l: int, n: int, rows: Sequence[int], cols: Sequence[int]):
        """hg_set_partition: the output blocks of a product (Section IV-D)."""
        r = np.ascontiguousarray(rows, dtype=np.int32)
        c = np.ascontiguousarray(cols, dtype=np.int32)
        _check(_lib.hg_set_partition(self.ptr, m, l, n, r, r.size, c, c.size))

    def partition(self, m: int, l: int, n: int) -> Tuple[List[int], List[int]]:
        """hg_get_partition: (row block sizes, column block sizes)."""
        cnt = ctypes.c_size_t(0)
        _check(_lib.hg_get_partition(self.ptr, m, l, n, None, 0, ctypes.byref(cnt)))
        out = np.zeros(cnt.value, dtype=np.int32)
        _check(_lib.hg_get_partition(self.ptr, m, l, n, out.ctypes.data, out.size, ctypes.byref(cnt)))
        nr, nc = int(out[0]), int(out[1])
        return [int(x) for x in out[2:2 + nr]], [int(x) for x in out[2 + nr:2 + nr + nc]]

    def hegmm_noalloc(self, A: Ciphertext, B: Ciphertext, m: int, l: int, n: int, out: Ciphertext,
                      stream: Optional[int] = None) -> Ciphertext:
        """hg_hegmm_noalloc: the product written into the existing handle `out`
        with no device allocation (fixed per-GPU workspace); returns `out`."""
        s = current_stream() if stream is None else stream
        _check(_lib.hg_hegmm_noalloc(self.ptr, A.ptr, B.ptr, m, l, n, out.ptr, s))
        return out

    def hegmm_batch(self, As: Sequence[Ciphertext], Bs: Sequence[Ciphertext], shapes, stream=None) -> List[Ciphertext]:
        cnt = len(As)
        pa = (ctypes.c_void_p * cnt)(*[a.ptr for a in As])
        pb = (ctypes.c_void_p * cnt)(*[b.ptr for b in Bs])
        pc = (ctypes.c_void_p * cnt)()
        mln = np.ascontiguousarray(np.array(list(shapes), dtype=np.int32).reshape(-1))
        s = current_stream() if stream is None else stream
        _check(_lib.hg_hegmm_batch(self.ptr, cnt, ctypes.cast(pa, _PP), ctypes.cast(pb, _PP), mln,
                                   ctypes.cast(pc, _PP), s))
        return [Ciphertext(self, pc[i]) for i in range(cnt)]

    def decrypt(self, C: Ciphertext, m: int, l: int, n: int) -> np.ndarray:
        out = np.empty(m * n, dtype=np.uint64)
        _check(_lib.hg_decrypt(self.ptr, C.ptr, m, l, n, out))
        return out.reshape(m, n).astype(np.int64)

    def import_ct(self, words: np.ndarray, ncts: int, comps: int = 2) -> Ciphertext:
        w = np.ascontiguousarray(words, dtype=np.uint64)
        out = ctypes.c_void_p()
        _check(_lib.hg_ct_import(self.ptr, w, w.size, ncts, comps, ctypes.byref(out)))
        return self._ct(out)

    def encrypt_slots(self, slots: Sequence[int], nonce: int = 0) -> Ciphertext:
        v = np.zeros(self.S, dtype=np.int64)
        v[: len(slots)] = np.asarray(slots, dtype=np.int64)
        out = ctypes.c_void_p()
        _check(_lib.hg_encrypt_slots(self.ptr, v, nonce, ctypes.byref(out)))
        return self._ct(out)

    def decrypt_slots(self, ct: Ciphertext) -> np.ndarray:
        out = np.empty(self.S, dtype=np.uint64)
        _check(_lib.hg_decrypt_slots(self.ptr, ct.ptr, out))
        return out.astype(np.int64)

    def rotate(self, ct: Ciphertext, z: int, stream=None) -> Ciphertext:
        out = ctypes.c_void_p()
        _check(_lib.hg_rotate(self.ptr, ct.ptr, z, ctypes.byref(out), current_stream() if stream is None else stream))
        return self._ct(out)

    def mul(self, a: Ciphertext, b: Ciphertext, stream=None) -> Ciphertext:
        out = ctypes.c_void_p()
        _check(_lib.hg_mul(self.ptr, a.ptr, b.ptr, ctypes.byref(out), current_stream() if stream is None else stream))
        return self._ct(out)

    def add(self, a: Ciphertext, b: Ciphertext, stream=None) -> Ciphertext:
        out = ctypes.c_void_p()
        _check(_lib.hg_add(self.ptr, a.ptr, b.ptr, ctypes.byref(out), current_stream() if stream is None else stream))
        return self._ct(out)

    def cmul(self, a: Ciphertext, slots: Sequence[int], stream=None) -> Ciphertext:
        v = np.zeros(self.S, dtype=np.int64)
        v[: len(slots)] = np.asarray(slots, dtype=np.int64)
        out = ctypes.c_void_p()
        _check(_lib.hg_cmul(self.ptr, a.ptr, v, ctypes.byref(out), current_stream() if stream is None else stream))
        return self._ct(out)

    def mod_switch(self, a: Ciphertext, drop: int = 1, stream=None) -> Ciphertext:
        """hg_mod_switch: the same plaintext at `drop` ciphertext primes fewer."""
        out = ctypes.c_void_p()
        _check(_lib.hg_mod_switch(self.ptr, a.ptr, drop, ctypes.byref(out),
                                  current_stream() if stream is None else stream))
        return self._ct(out)

    def plan_info(self, m: int, l: int, n: int) -> dict:
        out = np.zeros(10, dtype=np.int64)
        _check(_lib.hg_plan_info(self.ptr, m, l, n, out))
        keys = ["transposed", "nb", "lb", "d", "M", "K", "W", "rotations", "masks", "ks_terms"]
        return dict(zip(keys, (int(x) for x in out)))

    def primes(self) -> List[int]:
        out = np.zeros(self.L + self.alpha, dtype=np.uint64)
        _check(_lib.hg_primes(self.ptr, out))
        return [int(x) for x in out]

    def tune(self, name: str, value: int):
        """Set an execution knob (results are bit-identical for every value)."""
        _check(_lib.hg_tune(self.ptr, name.encode(), int(value)))

    def set_timing(self, on: bool):
        _check(_lib.hg_set_timing(self.ptr, 1 if on else 0))

    def set_launch_timing(self, on: bool):
        """hg_set_timing mode 2: time the transform-pass inner-product launches
        of the following calls, read with launch_timing()."""
        _check(_lib.hg_set_timing(self.ptr, 2 if on else 0))

    def launch_timing(self) -> dict:
        out = np.zeros(4, dtype=np.float64)
        _check(_lib.hg_launch_timing(self.ptr, out))
        return {"ip_kernel": float(out[0]), "ip_launches": int(out[1]),
                "md_fwd_kernel": float(out[2]), "md_fwd_launches": int(out[3])}

    def last_timing(self) -> dict:
        out = np.zeros(9, dtype=np.float64)
        _check(_lib.hg_last_timing(self.ptr, out))
        keys = ["hoist", "inner_product", "div_by_p", "tensor", "relin", "fold", "total", "ip_kernel",
                "ip_launches"]
        return dict(zip(keys, (float(x) for x in out)))

    def load_ct(self, ct: "Ciphertext", words: np.ndarray, stream=None):
        """Overwrite ct's contents with canonical words (export layout)."""
        w = np.ascontiguousarray(words, dtype=np.uint64)
        _check(_lib.hg_ct_load(self.ptr, ct.ptr, w, w.size, current_stream() if stream is None else stream))

    def record_batch(self, As, Bs, shapes) -> "Graph":
        """Record the batch as a replayable graph (see hg_graph_create)."""
        return Graph(self, As, Bs, shapes)

    def request_footprint(self, m: int, l: int, n: int) -> int:
        out = ctypes.c_uint64(0)
        _check(_lib.hg_request_footprint(self.ptr, m, l, n, ctypes.byref(out)))
        return int(out.value)


class Server:
    """hg_server: continuous-batching request loop over a keyed context.

    While it exists its thread owns the context; use only submit / wait /
    stats until close()."""

    def __init__(self, ctx: Context, max_batch: int = 64, lanes: int = 2, hbm_budget: int = 0):
        cfg = _ServerConfig(max_batch, lanes, hbm_budget)
        out = ctypes.c_void_p()
        _check(_lib.hg_server_create(ctx.ptr, ctypes.byref(cfg), ctypes.byref(out)))
        self.ptr = out.value
        self.ctx = ctx
        self.words = 2 * ctx.L * ctx.N

    def submit(self, a_words: np.ndarray, b_words: np.ndarray, m: int, l: int, n: int) -> int:
        a = np.ascontiguousarray(a_words, dtype=np.uint64)
        b = np.ascontiguousarray(b_words, dtype=np.uint64)
        t = ctypes.c_uint64(0)
        _check(_lib.hg_server_submit(self.ptr, a, a.size, b, b.size, m, l, n, ctypes.byref(t)))
        return int(t.value)

    def wait(self, ticket: int):
        """(result words, (submit, start, done) seconds on the server clock)."""
        out = np.empty(self.words, dtype=np.uint64)
        times = np.zeros(3, dtype=np.float64)
        _check(_lib.hg_server_wait(self.ptr, ticket, out.ctypes.data, out.size, times.ctypes.data))
        return out, tuple(float(x) for x in times)

    def pause(self, paused: bool = True):
        """Hold (or resume) admission: submitted requests queue up meanwhile."""
        _check(_lib.hg_server_pause(self.ptr, 1 if paused else 0))

    def stats(self) -> dict:
        out = np.zeros(8, dtype=np.float64)
        _check(_lib.hg_server_stats(self.ptr, out))
        keys = ["done", "groups", "mean_group", "peak_footprint", "peak_lanes_busy", "queued", "footprint",
                "clock"]
        return dict(zip(keys, (float(x) for x in out)))

    def close(self):
        if getattr(self, "ptr", None):
            _lib.hg_server_destroy(self.ptr)
            self.ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """hg_graph: a recorded batch.  Keeps its operand and result handles alive."""

    def __init__(self, ctx: Context, As, Bs, shapes):
        cnt = len(As)
        pa = (ctypes.c_void_p * cnt)(*[a.ptr for a in As])
        pb = (ctypes.c_void_p * cnt)(*[b.ptr for b in Bs])
        pc = (ctypes.c_void_p * cnt)()
        mln = np.ascontiguousarray(np.array(list(shapes), dtype=np.int32).reshape(-1))
        out = ctypes.c_void_p()
        _check(_lib.hg_graph_create(ctx.ptr, cnt, ctypes.cast(pa, _PP), ctypes.cast(pb, _PP), mln,
                                    ctypes.cast(pc, _PP), ctypes.byref(out)))
        self.ptr = out.value
        self.ctx = ctx
        self.inputs = (list(As), list(Bs))
        self.outputs = [Ciphertext(ctx, pc[i]) for i in range(cnt)]

    def launch(self, stream=None):
        _check(_lib.hg_graph_launch(self.ptr, current_stream() if stream is None else stream))

    def close(self):
        if getattr(self, "ptr", None):
            _lib.hg_graph_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

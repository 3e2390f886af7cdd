"""MI355X (gfx950) library for the key-switching path of 32-bit RNS-CKKS
(HMult, HRot, rescale, KeySwitch, NTT, BConv), after Cheddar (arXiv 2407.13055).

This module is a thin ctypes binding of ``libckks_hip.so`` (C ABI declared in
``include/ckks_hip.h``): it marshals torch device tensors and the current
HIP stream into the C calls and turns error codes into exceptions.  Every
arithmetic step runs in the library's HIP kernels; there is no fallback.

Residue tensors are torch.int32 (bit pattern of the uint32 residues) on the
GPU, limb-major [limbs][N]; ciphertexts are [2][level][N] (b then a), keys
[dnum][2][n_q+n_p][N], as the header states.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libckks_hip.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ckks_hip.h")

OP_BCONV, OP_KEYSWITCH, OP_HMULT, OP_HROT, OP_RESCALE, OP_HROT_HOISTED, OP_HROT_SUM = 1, 2, 3, 4, 5, 6, 7
OP_RESCALE_RATIONAL = 8

_lib = None


class CkksError(RuntimeError):
    pass


class Tuning(ctypes.Structure):
    """ckks_tuning: launch-shape knobs of a context (results do not depend on them)."""
    _fields_ = [("bconv_tpw_up", ctypes.c_int32), ("bconv_tpw_down", ctypes.c_int32),
                ("xcd_pair", ctypes.c_int32), ("rows_per_thread", ctypes.c_int32), ("col_threads", ctypes.c_int32),
                ("rows_per_thread_single", ctypes.c_int32), ("keymult_rows", ctypes.c_int32),
                ("keymult_rows_single", ctypes.c_int32), ("cols_per_thread", ctypes.c_int32),
                ("cols_per_thread_single", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"bconv_tpw_up": self.bconv_tpw_up, "bconv_tpw_down": self.bconv_tpw_down, "xcd_pair": self.xcd_pair,
                "rows_per_thread": self.rows_per_thread, "col_threads": self.col_threads,
                "rows_per_thread_single": self.rows_per_thread_single, "keymult_rows": self.keymult_rows,
                "keymult_rows_single": self.keymult_rows_single, "cols_per_thread": self.cols_per_thread,
                "cols_per_thread_single": self.cols_per_thread_single}


class _Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32), ("n_p", ctypes.c_uint32),
                ("q", ctypes.POINTER(ctypes.c_uint64)), ("p", ctypes.POINTER(ctypes.c_uint64))]


class _Ct(ctypes.Structure):
    """ckks_ct: ciphertext buffer with its level and scale."""
    _fields_ = [("data", ctypes.c_void_p), ("level", ctypes.c_int32), ("scale", ctypes.c_double)]


class Ciphertext:
    """A ciphertext tensor [2][level][N] (int32 residues, evaluation domain)
    with the scale of the message it holds (Sec. 2.1); the level is the
    tensor's second dimension."""

    def __init__(self, data, scale: float):
        self.data, self.scale = data, float(scale)

    @property
    def level(self) -> int:
        return int(self.data.shape[1])


def lib() -> ctypes.CDLL:
    """Load the built library; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CkksError("libckks_hip.so is not built; run __graft_entry__.build() or "
                            "python paper_2407_13055_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        i32p = ctypes.POINTER(ctypes.c_int32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        sig = {
            "ckks_last_error": ([], ctypes.c_char_p),
            "ckks_prime_chain": ([i, i, i, u64p], i),
            "ckks_ctx_create": ([ctypes.POINTER(_Params), ctypes.POINTER(vp)], i),
            "ckks_ctx_create_windowed": ([ctypes.POINTER(_Params), i32p, i32p, i, ctypes.POINTER(vp)], i),
            "ckks_ctx_destroy": ([vp], None),
            "ckks_ctx_tune": ([vp, ctypes.POINTER(Tuning)], i),
            "ckks_ctx_tuning": ([vp, ctypes.POINTER(Tuning)], i),
            "ckks_workspace_size": ([vp, i, i, i, i, ctypes.POINTER(sz)], i),
            "ckks_ntt": ([vp, vp, i32p, i, vp], i),
            "ckks_intt": ([vp, vp, i32p, i, vp], i),
            "ckks_bconv": ([vp, vp, i32p, i, vp, i32p, i, vp, sz, vp], i),
            "ckks_keyswitch": ([vp, vp, i, vp, vp, vp, vp, sz, vp], i),
            "ckks_hmult": ([vp, vp, i, vp, i, vp, i, vp, vp, sz, vp], i),
            "ckks_hmult_rescale": ([vp, vp, i, vp, i, vp, i, vp, vp, sz, vp], i),
            "ckks_hmult_rescale_noalloc": ([vp, vp, i, vp, i, vp, i, vp, vp], i),
            "ckks_hrot": ([vp, vp, i, i, i, vp, vp, vp, sz, vp], i),
            "ckks_hmult_rescale_batch": ([vp, i, vp, vp, i, i, vp, i, vp, vp, vp, sz, vp], i),
            "ckks_hmult_batch": ([vp, i, vp, vp, i, i, vp, i, vp, vp, vp, sz, vp], i),
            "ckks_hadd": ([vp, vp, i, vp, i, i, vp, vp], i),
            "ckks_padd": ([vp, vp, i, vp, i, i, vp, vp], i),
            "ckks_pmult": ([vp, vp, i, vp, i, i, vp, vp], i),
            "ckks_hconj": ([vp, vp, i, i, vp, vp, vp, sz, vp], i),
            "ckks_hrot_sum_hoisted": ([vp, vp, i, i, i, vp, vp, i, vp, vp, vp, sz, vp], i),
            "ckks_rescale_rational": ([vp, vp, i, i32p, i, i32p, vp, vp, sz, vp], i),
            "ckks_hrot_batch": ([vp, i, vp, i, i, vp, i, vp, i, vp, vp, sz, vp], i),
            "ckks_hrot_hoisted": ([vp, vp, i, i, i, vp, vp, i, vp, vp, sz, vp], i),
            "ckks_rescale": ([vp, vp, i, vp, vp, sz, vp], i),
            "ckks_ct_hmult": ([vp, ctypes.POINTER(_Ct), ctypes.POINTER(_Ct), vp, i, ctypes.POINTER(_Ct), vp, sz, vp], i),
            "ckks_ct_hmult_rescale": ([vp, ctypes.POINTER(_Ct), ctypes.POINTER(_Ct), vp, i, ctypes.POINTER(_Ct), vp,
                                       sz, vp], i),
            "ckks_ct_rescale": ([vp, ctypes.POINTER(_Ct), ctypes.POINTER(_Ct), vp, sz, vp], i),
            "ckks_ct_hrot": ([vp, ctypes.POINTER(_Ct), i, i, vp, ctypes.POINTER(_Ct), vp, sz, vp], i),
            "ckks_profile_start": ([vp, i], i),
            "ckks_profile_stop": ([vp], i),
            "ckks_profile_kernels": ([vp, ctypes.POINTER(i)], i),
            "ckks_profile_kernel": ([vp, i, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(i),
                                     ctypes.POINTER(ctypes.c_double)], i),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != 0:
        raise CkksError("ckks error %d: %s" % (rc, lib().ckks_last_error().decode()))


def prime_chain(bits: int, log_n: int, count: int) -> list[int]:
    """The `count` largest primes below 2^bits that are 1 mod 2N, descending."""
    out = (ctypes.c_uint64 * max(count, 1))()
    _check(lib().ckks_prime_chain(bits, log_n, count, out))
    return [int(out[i]) for i in range(count)]


def _ids(ids) -> ctypes.Array:
    return (ctypes.c_int32 * len(ids))(*[int(x) for x in ids])


def _ptr(t) -> int:
    """Device address of a tensor; the library reads dense row-major buffers,
    so strided views are refused."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise CkksError("tensor arguments must be contiguous (got strides %s)" % (tuple(t.stride()),))
    return t.data_ptr()


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def to_device(a, device="cuda"):
    """numpy uint32 residues -> torch.int32 device tensor (same bits)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(device)


def to_host(t) -> np.ndarray:
    """torch.int32 residue tensor -> numpy uint32."""
    return t.detach().cpu().numpy().view(np.uint32)


class Context:
    """Parameter set (ring degree, q's, p's) with its device tables.

    windows: optional list of (start, length) over q, one per level, for the
    25-30 prime system in the inverted-terminal layout (Sec. 3.2, 3.3); a
    level is then named by its window's length, and every level uses one key
    over P * Q_max (ckks_ctx_create_windowed)."""

    def __init__(self, log_n: int, q, p, windows=None):
        self.log_n, self.q, self.p = int(log_n), [int(x) for x in q], [int(x) for x in p]
        self.windows = None if windows is None else [(int(a), int(b)) for a, b in windows]
        qa = (ctypes.c_uint64 * len(self.q))(*self.q)
        pa = (ctypes.c_uint64 * len(self.p))(*self.p)
        prm = _Params(self.log_n, len(self.q), len(self.p), qa, pa)
        h = ctypes.c_void_p()
        if self.windows is None:
            _check(lib().ckks_ctx_create(ctypes.byref(prm), ctypes.byref(h)))
        else:
            st = (ctypes.c_int32 * len(self.windows))(*[a for a, _ in self.windows])
            ln = (ctypes.c_int32 * len(self.windows))(*[b for _, b in self.windows])
            _check(lib().ckks_ctx_create_windowed(ctypes.byref(prm), st, ln, len(self.windows), ctypes.byref(h)))
        self.h = h
        import torch
        self.device = torch.cuda.current_device() if torch.cuda.is_available() else 0
        self._ws = {}        # per stream handle: cached workspace allocated on that stream
        self._ws_sizes = {}

    def close(self):
        if getattr(self, "h", None):
            lib().ckks_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def n_q(self) -> int:
        return len(self.q)

    @property
    def alpha(self) -> int:
        return len(self.p)

    @property
    def dnum(self) -> int:
        return -(-self.n_q // self.alpha)

    def tune(self, bconv_tpw_up: int = 2, bconv_tpw_down: int = 2, xcd_pair: int = 1,
             rows_per_thread: int = 16, col_threads: int = 256, rows_per_thread_single: int = 4,
             keymult_rows: int = 4, keymult_rows_single: int = 4, cols_per_thread: int = 4,
             cols_per_thread_single: int = 4) -> None:
        """Set the launch-shape knobs (rebuilds the launch plans; synchronizes the device).
        rows_per_thread_single / keymult_rows_single / cols_per_thread_single: the row-pass /
        KeyMult / column-pass width of single-operation launches (0: the batched knob).  The
        defaults are the context's own: the setting the tuner picks on MI355X at N = 2^16."""
        _check(lib().ckks_ctx_tune(self.h, ctypes.byref(Tuning(bconv_tpw_up, bconv_tpw_down, xcd_pair,
                                                                rows_per_thread, col_threads,
                                                                rows_per_thread_single, keymult_rows,
                                                                keymult_rows_single, cols_per_thread,
                                                                cols_per_thread_single))))

    @property
    def tuning(self) -> dict:
        t = Tuning()
        _check(lib().ckks_ctx_tuning(self.h, ctypes.byref(t)))
        return t.as_dict()

    def workspace_size(self, op: int, level: int = 0, n_in: int = 0, n_out: int = 0) -> int:
        b = ctypes.c_size_t()
        _check(lib().ckks_workspace_size(self.h, op, level, n_in, n_out, ctypes.byref(b)))
        return b.value

    def workspace(self, nbytes: int, stream=None):
        """A cached device workspace of at least nbytes (uint8 tensor), one per
        stream: it is allocated while that stream is current, so torch's
        caching allocator reuses its block only for later work on the same
        stream (a grown workspace never hands its old block to another stream
        while this one may still use it)."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        key = s.cuda_stream
        w = self._ws.get(key)
        if w is None or w.numel() < nbytes:
            self._ws.pop(key, None)
            with torch.cuda.stream(s):
                w = torch.empty(max(nbytes, 16), dtype=torch.uint8, device="cuda:%d" % self.device)
            self._ws[key] = w
        return w

    def _ws_for(self, op, level=0, n_in=0, n_out=0, ws=None, stream=None):
        """(address, bytes) of the workspace of one call: the caller's, checked,
        or the cached one of the call's stream."""
        if ws is not None:
            return self._buf(ws, "ws", dtype="uint8"), ws.numel()
        key = (op, level, n_in, n_out)
        need = self._ws_sizes.get(key)
        if need is None:
            need = self._ws_sizes[key] = self.workspace_size(op, level, n_in, n_out)
        w = self.workspace(need, stream)
        return w.data_ptr(), w.numel()

    # -- argument checks (before anything reaches the C ABI) ------------------
    def _buf(self, t, name: str, numel: int = 0, dtype: str = "int32"):
        """Address of a dense device tensor on this context's GPU holding at
        least `numel` elements of `dtype` (int32 residues or uint8 bytes)."""
        import torch
        if not isinstance(t, torch.Tensor):
            raise CkksError("%s: expected a torch tensor, got %s" % (name, type(t).__name__))
        if not t.is_cuda or t.device.index != self.device:
            raise CkksError("%s: must be on cuda:%d (got %s)" % (name, self.device, t.device))
        want = torch.int32 if dtype == "int32" else torch.uint8
        if t.dtype != want:
            raise CkksError("%s: dtype must be %s (got %s)" % (name, want, t.dtype))
        if not t.is_contiguous():
            raise CkksError("%s: must be contiguous (got strides %s)" % (name, tuple(t.stride())))
        if t.numel() < numel:
            raise CkksError("%s: holds %d elements, the call needs %d" % (name, t.numel(), numel))
        return t.data_ptr()

    def _ct(self, t, name: str, level: int):
        """(address, its level) of a ciphertext [2][l][N], l >= level."""
        if getattr(t, "dim", lambda: 0)() != 3 or t.shape[0] != 2 or t.shape[2] != self.n:
            raise CkksError("%s: expected shape [2][level][%d] (got %s)" % (name, self.n, tuple(getattr(t, "shape", ()))))
        if t.shape[1] < level:
            raise CkksError("%s: level %d is below the operation level %d" % (name, t.shape[1], level))
        return self._buf(t, name), int(t.shape[1])

    def _cts(self, t, name: str, level: int):
        """(address, slots, level) of ciphertext slots [n][2][l][N], l >= level."""
        if getattr(t, "dim", lambda: 0)() != 4 or t.shape[1] != 2 or t.shape[3] != self.n:
            raise CkksError("%s: expected shape [n][2][level][%d] (got %s)" % (name, self.n, tuple(getattr(t, "shape", ()))))
        if t.shape[2] < level:
            raise CkksError("%s: level %d is below the operation level %d" % (name, t.shape[2], level))
        return self._buf(t, name), int(t.shape[0]), int(t.shape[2])

    @property
    def key_residues(self) -> int:
        """Residues of one evaluation key [dnum][2][n_q+n_p][N]."""
        return self.dnum * 2 * (self.n_q + self.alpha) * self.n

    def rescaled_level(self, level: int) -> int:
        """Limbs after HMult + rescale at `level`: level - 1, or on a windowed
        context the limb count of the window below (0 if none)."""
        if self.windows is None:
            return level - 1
        below = [ln for _, ln in self.windows if ln < level]
        return max(below) if below else 0

    # -- ring operations --------------------------------------------------
    def ntt(self, data, prime_ids, stream=None):
        d = self._buf(data, "data", len(prime_ids) * self.n)
        _check(lib().ckks_ntt(self.h, d, _ids(prime_ids), len(prime_ids), _stream(stream)))

    def intt(self, data, prime_ids, stream=None):
        d = self._buf(data, "data", len(prime_ids) * self.n)
        _check(lib().ckks_intt(self.h, d, _ids(prime_ids), len(prime_ids), _stream(stream)))

    def bconv(self, x, in_ids, out, out_ids, ws=None, stream=None):
        px = self._buf(x, "x", len(in_ids) * self.n)
        po = self._buf(out, "out", len(out_ids) * self.n)
        w, nb = self._ws_for(OP_BCONV, 0, len(in_ids), len(out_ids), ws, stream)
        _check(lib().ckks_bconv(self.h, px, _ids(in_ids), len(in_ids), po, _ids(out_ids),
                                len(out_ids), w, nb, _stream(stream)))

    # -- mechanisms ---------------------------------------------------------
    def keyswitch(self, d, level, evk, out0, out1, ws=None, stream=None):
        L = level * self.n
        pd, pk = self._buf(d, "d", L), self._buf(evk, "evk", self.key_residues)
        p0, p1 = self._buf(out0, "out0", L), self._buf(out1, "out1", L)
        w, nb = self._ws_for(OP_KEYSWITCH, level, ws=ws, stream=stream)
        _check(lib().ckks_keyswitch(self.h, pd, level, pk, p0, p1, w, nb, _stream(stream)))

    def _hmult_args(self, ct_a, ct_b, rlk, level, out, out_level):
        pa, la = self._ct(ct_a, "ct_a", level)
        pb, lb = self._ct(ct_b, "ct_b", level)
        return pa, la, pb, lb, self._buf(rlk, "rlk", self.key_residues), self._buf(out, "out",
                                                                                  2 * out_level * self.n)

    def hmult(self, ct_a, ct_b, rlk, level, out, ws=None, stream=None):
        pa, la, pb, lb, pk, po = self._hmult_args(ct_a, ct_b, rlk, level, out, level)
        w, nb = self._ws_for(OP_HMULT, level, ws=ws, stream=stream)
        _check(lib().ckks_hmult(self.h, pa, la, pb, lb, pk, level, po, w, nb, _stream(stream)))

    def hmult_rescale(self, ct_a, ct_b, rlk, level, out, ws=None, stream=None):
        pa, la, pb, lb, pk, po = self._hmult_args(ct_a, ct_b, rlk, level, out, self.rescaled_level(level))
        w, nb = self._ws_for(OP_HMULT, level, ws=ws, stream=stream)
        _check(lib().ckks_hmult_rescale(self.h, pa, la, pb, lb, pk, level, po, w, nb, _stream(stream)))

    def hmult_rescale_noalloc(self, ct_a, ct_b, rlk, level, out, stream=None):
        """As hmult_rescale, with the library's own per-GPU scratch array as
        the workspace (ckks_hmult_rescale_noalloc: nothing is allocated; calls
        that overlap on one GPU race on that array)."""
        pa, la, pb, lb, pk, po = self._hmult_args(ct_a, ct_b, rlk, level, out, self.rescaled_level(level))
        _check(lib().ckks_hmult_rescale_noalloc(self.h, pa, la, pb, lb, pk, level, po, _stream(stream)))

    # -- batched forms ---------------------------------------------------------
    @staticmethod
    def batch_items(levels, keys=None, rots=None, srcs=None, device="cuda"):
        """Device array of ckks_batch_item {level, key, rot, src} (int32 [n][4]);
        src defaults to the item's own slot i."""
        import torch
        n = len(levels)
        a = np.zeros((n, 4), dtype=np.int32)
        a[:, 0] = np.asarray(levels, dtype=np.int32)
        if keys is not None:
            a[:, 1] = np.asarray(keys, dtype=np.int32)
        if rots is not None:
            a[:, 2] = np.asarray(rots, dtype=np.int32)
        a[:, 3] = np.arange(n, dtype=np.int32) if srcs is None else np.asarray(srcs, dtype=np.int32)
        return torch.from_numpy(a).to(device)

    def hmult_rescale_batch(self, a, b, items, max_level, rlk, out, ws=None, stream=None):
        """a, b: [n_src][2][level_in][N]; items: batch_items(levels[, srcs]); out: [n][2][max_level-1][N]
        ([n][2][L'][N] on a windowed context, L' the limb count of the window below max_level)."""
        self._hmult_batch(lib().ckks_hmult_rescale_batch, a, b, items, max_level, rlk, out, ws, stream,
                          self.rescaled_level(max_level))

    def hmult_batch(self, a, b, items, max_level, rlk, out, ws=None, stream=None):
        """HMult+relin without rescale: out: [n][2][max_level][N]."""
        self._hmult_batch(lib().ckks_hmult_batch, a, b, items, max_level, rlk, out, ws, stream, max_level)

    def _items(self, items, n):
        """Address of a device item array [n][4] int32 (ckks_batch_item)."""
        return self._buf(items, "items", 4 * n)

    def _batch_ws(self, ws, nbytes, stream):
        if ws is None:
            ws = self.workspace(nbytes, stream)
        return self._buf(ws, "ws", nbytes, dtype="uint8"), ws.numel()

    def _hmult_batch(self, fn, a, b, items, max_level, rlk, out, ws, stream, out_level):
        pa, n_src, la = self._cts(a, "a", max_level)
        pb, n_src_b, lb = self._cts(b, "b", max_level)
        if (n_src_b, lb) != (n_src, la):
            raise CkksError("a and b must have the same slots and level (%s vs %s)" % (tuple(a.shape), tuple(b.shape)))
        n = out.shape[0]
        po = self._buf(out, "out", n * 2 * out_level * self.n)
        w, nb = self._batch_ws(ws, n * self.workspace_size(OP_HMULT, max_level), stream)
        _check(fn(self.h, n, pa, pb, n_src, la, self._items(items, n), max_level,
                  self._buf(rlk, "rlk", self.key_residues), po, w, nb, _stream(stream)))

    def hrot_batch(self, ct, items, max_level, keys, out, ws=None, stream=None):
        """ct: [n][2][level_in][N]; items: batch_items(levels, keys, rots); keys:
        [n_keys][dnum][2][n_q+n_p][N]; out: [n][2][max_level][N]."""
        pc, n_src, lc = self._cts(ct, "ct", max_level)
        n = out.shape[0]
        po = self._buf(out, "out", n * 2 * max_level * self.n)
        n_keys = keys.shape[0]
        pk = self._buf(keys, "keys", n_keys * self.key_residues)
        w, nb = self._batch_ws(ws, n * self.workspace_size(OP_HROT, max_level), stream)
        _check(lib().ckks_hrot_batch(self.h, n, pc, n_src, lc, self._items(items, n), max_level, pk, n_keys, po, w,
                                     nb, _stream(stream)))

    def hrot_hoisted(self, ct, level, items, keys, outs, ws=None, stream=None):
        """ct: [2][level_in][N]; items: batch_items([level]*n_rot, keys, rots); keys:
        [n_keys][dnum][2][n_q+n_p][N]; outs: [n_rot][2][level][N]."""
        pc, lc = self._ct(ct, "ct", level)
        n_rot = outs.shape[0]
        po = self._buf(outs, "outs", n_rot * 2 * level * self.n)
        n_keys = keys.shape[0]
        pk = self._buf(keys, "keys", n_keys * self.key_residues)
        w, nb = self._batch_ws(ws, self.workspace_size(OP_HROT_HOISTED, level, n_rot), stream)
        _check(lib().ckks_hrot_hoisted(self.h, pc, lc, level, n_rot, self._items(items, n_rot), pk, n_keys, po, w, nb,
                                       _stream(stream)))

    def hrot_sum_hoisted(self, ct, level, items, keys, pts, out, ws=None, stream=None):
        """out = sum_i pts[i] * HRot(ct, rot_i) with one ModUp and one ModDown.
        items: batch_items([level]*n, keys, rots); pts: [n][n_q+n_p][N]."""
        pc, lc = self._ct(ct, "ct", level)
        n_rot = pts.shape[0]
        pp = self._buf(pts, "pts", n_rot * (self.n_q + self.alpha) * self.n)
        po = self._buf(out, "out", 2 * level * self.n)
        n_keys = keys.shape[0]
        pk = self._buf(keys, "keys", n_keys * self.key_residues)
        w, nb = self._batch_ws(ws, self.workspace_size(OP_HROT_SUM, level), stream)
        _check(lib().ckks_hrot_sum_hoisted(self.h, pc, lc, level, n_rot, self._items(items, n_rot), pk, n_keys, pp,
                                           po, w, nb, _stream(stream)))

    def hrot(self, ct, level, k, rk, out, ws=None, stream=None):
        pc, lc = self._ct(ct, "ct", level)
        pk, po = self._buf(rk, "rk", self.key_residues), self._buf(out, "out", 2 * level * self.n)
        w, nb = self._ws_for(OP_HROT, level, ws=ws, stream=stream)
        _check(lib().ckks_hrot(self.h, pc, lc, level, k, pk, po, w, nb, _stream(stream)))

    # -- element-wise mechanisms and conjugation -----------------------------
    def _pt(self, pt, level):
        if getattr(pt, "dim", lambda: 0)() != 2 or pt.shape[1] != self.n or pt.shape[0] < level:
            raise CkksError("pt: expected shape [>= %d][%d] (got %s)" % (level, self.n, tuple(getattr(pt, "shape", ()))))
        return self._buf(pt, "pt"), int(pt.shape[0])

    def hadd(self, ct_a, ct_b, level, out, stream=None):
        """out = ct_a + ct_b; ct_*: [2][level_*][N]; out: [2][level][N] (may be ct_a or ct_b)."""
        pa, la = self._ct(ct_a, "ct_a", level)
        pb, lb = self._ct(ct_b, "ct_b", level)
        _check(lib().ckks_hadd(self.h, pa, la, pb, lb, level, self._buf(out, "out", 2 * level * self.n),
                               _stream(stream)))

    def padd(self, ct, pt, level, out, stream=None):
        """out = (b + pt, a); pt: [>= level][N] evaluation-domain plaintext."""
        pc, lc = self._ct(ct, "ct", level)
        pp, lp = self._pt(pt, level)
        _check(lib().ckks_padd(self.h, pc, lc, pp, lp, level, self._buf(out, "out", 2 * level * self.n),
                               _stream(stream)))

    def pmult(self, ct, pt, level, out, stream=None):
        """out = (b * pt, a * pt) slot-wise."""
        pc, lc = self._ct(ct, "ct", level)
        pp, lp = self._pt(pt, level)
        _check(lib().ckks_pmult(self.h, pc, lc, pp, lp, level, self._buf(out, "out", 2 * level * self.n),
                                _stream(stream)))

    def hconj(self, ct, level, ck, out, ws=None, stream=None):
        """Slot-wise complex conjugation with the conjugation key ck."""
        pc, lc = self._ct(ct, "ct", level)
        pk, po = self._buf(ck, "ck", self.key_residues), self._buf(out, "out", 2 * level * self.n)
        w, nb = self._ws_for(OP_HROT, level, ws=ws, stream=stream)
        _check(lib().ckks_hconj(self.h, pc, lc, level, pk, po, w, nb, _stream(stream)))

    def rescale_rational(self, ct, in_ids, out_ids, out, ws=None, stream=None):
        """Rational rescaling from the primes in_ids to out_ids (prime ids of
        this context); ct: [2][len(in_ids)][N], out: [2][len(out_ids)][N]."""
        pc = self._buf(ct, "ct", 2 * len(in_ids) * self.n)
        po = self._buf(out, "out", 2 * len(out_ids) * self.n)
        w, nb = self._batch_ws(ws, self.workspace_size(OP_RESCALE_RATIONAL, 0, len(in_ids), len(out_ids)), stream)
        _check(lib().ckks_rescale_rational(self.h, pc, len(in_ids), _ids(in_ids), len(out_ids), _ids(out_ids),
                                           po, w, nb, _stream(stream)))

    # -- ciphertexts with their scale (ckks_ct) ------------------------------
    def _ct_struct(self, ct: Ciphertext, name: str, level: int = 1) -> _Ct:
        p, lv = self._ct(ct.data, name, level)
        return _Ct(p, lv, ct.scale)

    def _ct_out(self, out: Ciphertext, name: str, limbs: int) -> _Ct:
        if getattr(out.data, "dim", lambda: 0)() != 3 or out.data.shape[0] != 2 or out.data.shape[2] != self.n \
                or out.data.shape[1] != limbs:
            raise CkksError("%s: expected shape [2][%d][%d] (got %s)" % (name, limbs, self.n, tuple(out.data.shape)))
        return _Ct(self._buf(out.data, name), limbs, out.scale)

    def ct_hmult(self, a: Ciphertext, b: Ciphertext, rlk, level: int, out: Ciphertext, ws=None, stream=None):
        """HMult + relinearisation; sets out.scale = a.scale * b.scale."""
        ca, cb, co = self._ct_struct(a, "a", level), self._ct_struct(b, "b", level), self._ct_out(out, "out", level)
        w, nb = self._ws_for(OP_HMULT, level, ws=ws, stream=stream)
        _check(lib().ckks_ct_hmult(self.h, ctypes.byref(ca), ctypes.byref(cb), self._buf(rlk, "rlk", self.key_residues),
                                   level, ctypes.byref(co), w, nb, _stream(stream)))
        out.scale = co.scale
        return out

    def ct_hmult_rescale(self, a: Ciphertext, b: Ciphertext, rlk, level: int, out: Ciphertext, ws=None,
                         stream=None):
        """HMult + relinearisation + rescale; out.scale = a.scale * b.scale
        divided by the dropped modulus (times the added one on a windowed context)."""
        ca, cb = self._ct_struct(a, "a", level), self._ct_struct(b, "b", level)
        co = self._ct_out(out, "out", self.rescaled_level(level))
        w, nb = self._ws_for(OP_HMULT, level, ws=ws, stream=stream)
        _check(lib().ckks_ct_hmult_rescale(self.h, ctypes.byref(ca), ctypes.byref(cb),
                                           self._buf(rlk, "rlk", self.key_residues), level, ctypes.byref(co), w, nb,
                                           _stream(stream)))
        out.scale = co.scale
        return out

    def ct_rescale(self, ct: Ciphertext, out: Ciphertext, ws=None, stream=None):
        """Rescale by the last prime; out.scale = ct.scale / q_{level-1}."""
        ci = self._ct_struct(ct, "ct")
        co = self._ct_out(out, "out", ci.level - 1)
        w, nb = self._ws_for(OP_RESCALE, ws=ws, stream=stream)
        _check(lib().ckks_ct_rescale(self.h, ctypes.byref(ci), ctypes.byref(co), w, nb, _stream(stream)))
        out.scale = co.scale
        return out

    def ct_hrot(self, ct: Ciphertext, level: int, k: int, rk, out: Ciphertext, ws=None, stream=None):
        """HRot by k; out.scale = ct.scale."""
        ci, co = self._ct_struct(ct, "ct", level), self._ct_out(out, "out", level)
        w, nb = self._ws_for(OP_HROT, level, ws=ws, stream=stream)
        _check(lib().ckks_ct_hrot(self.h, ctypes.byref(ci), level, k, self._buf(rk, "rk", self.key_residues),
                                  ctypes.byref(co), w, nb, _stream(stream)))
        out.scale = co.scale
        return out

    # -- kernel timing ------------------------------------------------------
    def profile_start(self, max_launches: int = 4096):
        _check(lib().ckks_profile_start(self.h, max_launches))

    def profile_stop(self):
        _check(lib().ckks_profile_stop(self.h))

    def profile_report(self) -> dict:
        """{kernel name: (launches, total ms)} of the recorded launches."""
        n = ctypes.c_int()
        _check(lib().ckks_profile_kernels(self.h, ctypes.byref(n)))
        out = {}
        for i in range(n.value):
            name, cnt, ms = ctypes.c_char_p(), ctypes.c_int(), ctypes.c_double()
            _check(lib().ckks_profile_kernel(self.h, i, ctypes.byref(name), ctypes.byref(cnt), ctypes.byref(ms)))
            out[name.value.decode()] = (cnt.value, ms.value)
        return out

    def rescale(self, ct, out, ws=None, stream=None):
        pc, lc = self._ct(ct, "ct", 1)
        po = self._buf(out, "out", 2 * max(lc - 1, 0) * self.n)
        w, nb = self._ws_for(OP_RESCALE, ws=ws, stream=stream)
        _check(lib().ckks_rescale(self.h, pc, lc, po, w, nb, _stream(stream)))

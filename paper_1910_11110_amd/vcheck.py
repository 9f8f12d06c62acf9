"""ctypes binding of libvcheck (include/vcheck.h).

Argument marshalling only: every step of the check runs in the library's HIP
kernels.  Inputs may be numpy arrays (host memory, copied by the library) or torch
CUDA tensors (device memory, borrowed by the library until the next sync).  The
binding refuses to run when the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvcheck.so")

VC_OK, VC_EINVAL, VC_ENOMEM, VC_EDEVICE, VC_ESTATE, VC_ETRUNC, VC_EBUDGET, VC_EAGAIN = 0, -1, -2, -3, -4, -5, -6, -7
VC_DEVICE_INPUT, VC_DEVICE_INIT, VC_TRANSLATE_CHECK, VC_LIFETIME_EVENTS, VC_DECLARED_EXTEND = 1, 2, 4, 8, 16
NO_MOTHER = 0xFFFFFFFF

_lib = None


class VCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libvcheck error {code}: {msg}")
        self.code = code


class vc_completion(C.Structure):
    _fields_ = [("stream", C.c_uint64), ("chunk", C.c_uint64), ("first_event", C.c_uint64),
                ("n_events", C.c_uint64), ("n_violations", C.c_uint64), ("first_violation", C.c_uint64),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double), ("status", C.c_int)]


def lib():
    """The loaded library; raises if it is missing (build it with build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libvcheck.so is not built ({LIB_PATH}); run paper_1910_11110_amd/build.py")
        # One HIP runtime per process: when PyTorch provides device memory and streams,
        # load its runtime first so that the library binds to the same instance.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, u64, u32, i32 = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int
        pu64, pu32, pP = C.POINTER(C.c_uint64), C.POINTER(C.c_uint32), C.POINTER(C.c_void_p)
        sig = {
            "vc_ctx_create": ([i32, P, pP], i32),
            "vc_ctx_destroy": ([P], i32),
            "vc_last_error": ([], C.c_char_p),
            "vc_sync": ([P], i32),
            "vc_trace_load": ([P, P, u64, u32, P, u32, pP], i32),
            "vc_trace_set_arrays": ([P, P, P, u32], i32),
            "vc_trace_set_dynamic_arrays": ([P, P, P, P, u32], i32),
            "vc_trace_load_spaces": ([P, P, u64, u32, u32, P, u32, pP], i32),
            "vc_read_event_status16": ([P, P, u64], i32),
            "vc_check_declared": ([P, P, u64, P, u32, P, P, P, P, P, u32, pP], i32),
            "vc_run_programs": ([P, P, u64, P, u32, P, P, u64, pP], i32),
            "vc_programs_run": ([P], i32),
            "vc_programs_read": ([P, P, P, P, P, P, P], i32),
            "vc_programs_free": ([P], i32),
            "vc_batch_info": ([P, P, P, P, P], i32),
            "vc_read_overlap_sets": ([P, P, P, u64, pu64], i32),
            "vc_translate": ([P, P, u64, P, u32, P, P, u32, pP], i32),
            "vc_check": ([P], i32),
            "vc_trace_info": ([P, pu64, pu32], i32),
            "vc_read_events": ([P, P, u64, pu64], i32),
            "vc_read_event_status": ([P, P, u64], i32),
            "vc_read_violations": ([P, P, u64, pu64, pu64], i32),
            "vc_read_final_status": ([P, P, u32], i32),
            "vc_read_induced_stuck": ([P, pu64], i32),
            "vc_trace_device_results": ([P, pP, pP, pP], i32),
            "vc_trace_free": ([P], i32),
            "vc_batch_check": ([P, P, u32], i32),
            "vc_server_create": ([P, u64, u32, pP], i32),
            "vc_server_destroy": ([P], i32),
            "vc_stream_open": ([P, u32, P, P, P, pu64], i32),
            "vc_stream_submit": ([P, u64, P, u32, P, pu64], i32),
            "vc_poll": ([P, C.POINTER(vc_completion), u32, pu32], i32),
            "vc_stream_close": ([P, u64, P], i32),
            "vc_server_now": ([P], C.c_double),
            "vc_translate_run": ([P], i32),
            "vc_profile_enable": ([P, i32], i32),
            "vc_profile_reset": ([P], i32),
            "vc_profile_read": ([P, C.c_char_p, u32, P, P, u32, pu32], i32),
            "vc_check_small_noalloc": ([P, P, u64, u32, P, P, P, P, P], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int):
    if rc != VC_OK:
        raise VCError(rc, lib().vc_last_error().decode())


def _is_torch_cuda(a) -> bool:
    return hasattr(a, "is_cuda") and hasattr(a, "data_ptr") and a.is_cuda


def _buf(a, dtype):
    """(pointer, keep-alive object, is_device) for a numpy array or a torch CUDA tensor."""
    if a is None:
        return None, None, False
    if _is_torch_cuda(a):
        assert a.is_contiguous(), "device buffers must be contiguous"
        return C.c_void_p(a.data_ptr()), a, True
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data_as(C.c_void_p), arr, False


class Context:
    def __init__(self, device: int = 0, stream=None):
        """stream: None for a library-owned stream, or a torch.cuda.Stream / raw handle."""
        h = C.c_void_p()
        raw = None
        if stream is not None:
            raw = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        _check(lib().vc_ctx_create(device, raw, C.byref(h)))
        self.h = h
        self.device = device

    def sync(self):
        _check(lib().vc_sync(self.h))

    def profile(self, on: bool = True):
        _check(lib().vc_profile_enable(self.h, 1 if on else 0))

    def profile_reset(self):
        _check(lib().vc_profile_reset(self.h))

    def profile_read(self) -> dict:
        """{kernel name: (total ms, launches)} since the last reset."""
        n = C.c_uint32()
        _check(lib().vc_profile_read(self.h, None, 0, None, None, 0, C.byref(n)))
        k = n.value
        names = C.create_string_buffer(64 * (k + 1) + 1)
        ms = np.zeros(max(k, 1), np.float64)
        cnt = np.zeros(max(k, 1), np.uint64)
        _check(lib().vc_profile_read(self.h, names, len(names), ms.ctypes.data_as(C.c_void_p),
                                     cnt.ctypes.data_as(C.c_void_p), k, C.byref(n)))
        keys = names.value.decode().split("\n")[:k]
        return {keys[i]: (float(ms[i]), int(cnt[i])) for i in range(k)}

    def close(self):
        if self.h:
            lib().vc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Violations:
    indices: np.ndarray
    total: int
    first: int


class Trace:
    """A loaded trace (plain events or the result of a translation)."""

    def __init__(self, ctx: Context, handle, keep=()):
        self.ctx = ctx
        self.h = handle
        self._keep = list(keep)

    @classmethod
    def load(cls, ctx: Context, events, n_ids: int, init=None, lifetimes: bool = False) -> "Trace":
        p, keep, dev = _buf(events, np.uint32)
        n = int(keep.numel() if dev else keep.size)
        ip, ikeep, idev = _buf(init, np.uint8)
        flags = (VC_DEVICE_INPUT if dev else 0) | (VC_DEVICE_INIT if idev else 0) | \
            (VC_LIFETIME_EVENTS if lifetimes else 0)
        h = C.c_void_p()
        _check(lib().vc_trace_load(ctx.h, p, n, n_ids, ip, flags, C.byref(h)))
        return cls(ctx, h, (keep, ikeep) if (dev or idev) else ())

    @classmethod
    def load_spaces(cls, ctx: Context, events, n_ids: int, k: int, init=None) -> "Trace":
        """A trace over k memory spaces (k-space event words)."""
        p, keep, dev = _buf(events, np.uint32)
        n = int(keep.numel() if dev else keep.size)
        ip, ikeep, idev = _buf(init, np.uint8)
        flags = (VC_DEVICE_INPUT if dev else 0) | (VC_DEVICE_INIT if idev else 0)
        h = C.c_void_p()
        _check(lib().vc_trace_load_spaces(ctx.h, p, n, n_ids, k, ip, flags, C.byref(h)))
        return cls(ctx, h, (keep, ikeep) if (dev or idev) else ())

    def status16(self) -> np.ndarray:
        n, _ = self.info()
        out = np.empty(max(n, 1), np.uint16)
        _check(lib().vc_read_event_status16(self.h, out.ctypes.data_as(C.c_void_p), n))
        return out[:n]

    def set_arrays(self, lo, hi):
        lp, lk, ld = _buf(lo, np.uint32)
        hp, hk, hd = _buf(hi, np.uint32)
        assert ld == hd
        _check(lib().vc_trace_set_arrays(self.h, lp, hp, VC_DEVICE_INPUT if ld else 0))
        if ld:
            self._keep += [lk, hk]

    def set_dynamic_arrays(self, lo, hi, mother):
        """Arrays created (op 6) and destroyed (op 7) during the trace; mother[x] is the
        vector a partial vector lies in, NO_MOTHER for a vector (host arrays)."""
        lo = np.ascontiguousarray(lo, dtype=np.uint32)
        hi = np.ascontiguousarray(hi, dtype=np.uint32)
        mo = np.ascontiguousarray(mother, dtype=np.uint32)
        _check(lib().vc_trace_set_dynamic_arrays(self.h, lo.ctypes.data_as(C.c_void_p), hi.ctypes.data_as(C.c_void_p),
                                                 mo.ctypes.data_as(C.c_void_p), 0))

    def check(self):
        _check(lib().vc_check(self.h))

    def rerun(self):
        """Re-runs the translation (and its check) of a translated trace."""
        _check(lib().vc_translate_run(self.h))

    def info(self):
        n, k = C.c_uint64(), C.c_uint32()
        _check(lib().vc_trace_info(self.h, C.byref(n), C.byref(k)))
        return n.value, k.value

    def events(self) -> np.ndarray:
        n = C.c_uint64()
        _check(lib().vc_read_events(self.h, None, 0, C.byref(n)))
        out = np.empty(max(n.value, 1), np.uint32)
        _check(lib().vc_read_events(self.h, out.ctypes.data_as(C.c_void_p), out.size, C.byref(n)))
        return out[:n.value]

    def status(self) -> np.ndarray:
        n, _ = self.info()
        out = np.empty(max(n, 1), np.uint8)
        _check(lib().vc_read_event_status(self.h, out.ctypes.data_as(C.c_void_p), n))
        return out[:n]

    def violations(self) -> Violations:
        tot, first = C.c_uint64(), C.c_uint64()
        _check(lib().vc_read_violations(self.h, None, 0, C.byref(tot), C.byref(first)))
        out = np.empty(max(tot.value, 1), np.uint32)
        _check(lib().vc_read_violations(self.h, out.ctypes.data_as(C.c_void_p), tot.value, C.byref(tot),
                                        C.byref(first)))
        return Violations(out[:tot.value], tot.value, first.value)

    def final(self) -> np.ndarray:
        _, k = self.info()
        out = np.empty(max(k, 1), np.uint8)
        _check(lib().vc_read_final_status(self.h, out.ctypes.data_as(C.c_void_p), k))
        return out[:k]

    def induced_stuck(self) -> int:
        n = C.c_uint64()
        _check(lib().vc_read_induced_stuck(self.h, C.byref(n)))
        return n.value

    def overlap_sets(self):
        _, k = self.info()
        off = np.empty(k + 1, np.uint64)
        nn = C.c_uint64()
        _check(lib().vc_read_overlap_sets(self.h, off.ctypes.data_as(C.c_void_p), None, 0, C.byref(nn)))
        nbr = np.empty(max(nn.value, 1), np.uint32)
        _check(lib().vc_read_overlap_sets(self.h, off.ctypes.data_as(C.c_void_p), nbr.ctypes.data_as(C.c_void_p),
                                          nbr.size, C.byref(nn)))
        return off, nbr[:nn.value]

    def device_results(self):
        s, f, v = C.c_void_p(), C.c_void_p(), C.c_void_p()
        _check(lib().vc_trace_device_results(self.h, C.byref(s), C.byref(f), C.byref(v)))
        return s.value, f.value, v.value

    def free(self):
        if self.h:
            lib().vc_trace_free(self.h)
            self.h = None
            self._keep = []

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def translate(ctx: Context, comp_off, decls, n_vars: int, body_off=None, body=None, check: bool = False) -> Trace:
    cp, ck, cd = _buf(comp_off, np.uint64)
    dp, dk, dd = _buf(decls, np.uint32)
    bp, bk, bd = _buf(body_off, np.uint64)
    yp, yk, yd = _buf(body, np.uint32)
    n_comp = int((ck.numel() if cd else ck.size)) - 1
    dev = cd or dd
    flags = (VC_DEVICE_INPUT if dev else 0) | (VC_TRANSLATE_CHECK if check else 0)
    h = C.c_void_p()
    _check(lib().vc_translate(ctx.h, cp, n_comp, dp, n_vars, bp, yp, flags, C.byref(h)))
    return Trace(ctx, h, (ck, dk, bk, yk) if dev else ())


def check_small_noalloc(ctx: Context, events, n_ids: int, init, status, final, violations, counts):
    """vc_check_small_noalloc on torch CUDA tensors (events uint32/int32, 16-byte aligned;
    init uint8 or None; status uint8[n]; final uint8[n_ids]; violations int32[n];
    counts int64[3]).  Enqueued on the context's stream; nothing is allocated."""
    for a in (events, status, final, violations, counts) + ((init,) if init is not None else ()):
        assert _is_torch_cuda(a) and a.is_contiguous(), "device tensors expected"
    ip = None if init is None else C.c_void_p(init.data_ptr())
    _check(lib().vc_check_small_noalloc(ctx.h, C.c_void_p(events.data_ptr()), events.numel(), n_ids, ip,
                                        C.c_void_p(status.data_ptr()), C.c_void_p(final.data_ptr()),
                                        C.c_void_p(violations.data_ptr()), C.c_void_p(counts.data_ptr())))


def check_declared(ctx: Context, comp_off, decls, n_vars: int, body_off, body, idx=None, lo=None, hi=None,
                   extend: bool = False) -> Trace:
    """Well-declaredness of a component program with explicit bodies: the returned
    trace's status() is the verdict byte of every component, violations() the
    components that are not well-declared."""
    cp, ck, cd = _buf(comp_off, np.uint64)
    dp, dk, dd = _buf(decls, np.uint32)
    bp, bk, bdv = _buf(body_off, np.uint64)
    yp, yk, yd = _buf(body, np.uint32)
    ip, ik, idv = _buf(idx, np.uint32)
    dev = cd or dd or bdv or yd or idv
    n_comp = int(ck.numel() if cd else ck.size) - 1
    lp = hp = None
    if lo is not None:
        lo = np.ascontiguousarray(lo, dtype=np.uint32)
        hi = np.ascontiguousarray(hi, dtype=np.uint32)
        lp, hp = lo.ctypes.data_as(C.c_void_p), hi.ctypes.data_as(C.c_void_p)
    flags = (VC_DEVICE_INPUT if dev else 0) | (VC_DECLARED_EXTEND if extend else 0)
    h = C.c_void_p()
    _check(lib().vc_check_declared(ctx.h, cp, n_comp, dp, n_vars, bp, yp, ip, lp, hp, flags, C.byref(h)))
    return Trace(ctx, h, (ck, dk, bk, yk, ik) if dev else ())


class Programs:
    """Structured programs run on the GPU (one lane per program)."""

    def __init__(self, ctx: Context, prog_off, words, n_vars: int, choice=None, init=None, fuel: int = 1 << 12):
        po = np.ascontiguousarray(prog_off, dtype=np.uint64)
        w = np.ascontiguousarray(words, dtype=np.uint32)
        ch = None if choice is None else np.ascontiguousarray(choice, dtype=np.uint64)
        ini = None if init is None else np.ascontiguousarray(init, dtype=np.uint8)
        self.n, self.n_vars, self.ctx = po.size - 1, n_vars, ctx
        h = C.c_void_p()
        _check(lib().vc_run_programs(ctx.h, po.ctypes.data_as(C.c_void_p), self.n, w.ctypes.data_as(C.c_void_p),
                                     n_vars, None if ch is None else ch.ctypes.data_as(C.c_void_p),
                                     None if ini is None else ini.ctypes.data_as(C.c_void_p), fuel, C.byref(h)))
        self.h = h

    def run(self):
        _check(lib().vc_programs_run(self.h))

    def read(self):
        """(steps, effects, stuck, first, done, final[n, n_vars])"""
        n = max(self.n, 1)
        outs = [np.empty(n, np.uint64) for _ in range(4)]
        done = np.empty(n, np.uint8)
        fin = np.empty(n * self.n_vars, np.uint8)
        _check(lib().vc_programs_read(self.h, *[o.ctypes.data_as(C.c_void_p) for o in outs],
                                      done.ctypes.data_as(C.c_void_p), fin.ctypes.data_as(C.c_void_p)))
        return tuple(o[:self.n] for o in outs) + (done[:self.n], fin[:self.n * self.n_vars].reshape(self.n, self.n_vars))

    def free(self):
        if self.h:
            lib().vc_programs_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def batch_check(ctx: Context, traces):
    arr = (C.c_void_p * len(traces))(*[t.h for t in traces])
    _check(lib().vc_batch_check(ctx.h, arr, len(traces)))


class Server:
    def __init__(self, ctx: Context, hbm_budget: int, max_batch_events: int = 1 << 22):
        h = C.c_void_p()
        _check(lib().vc_server_create(ctx.h, hbm_budget, max_batch_events, C.byref(h)))
        self.h = h
        self.ctx = ctx

    def open(self, n_ids: int, lo=None, hi=None, init=None) -> int:
        lp, lk, _ = _buf(lo, np.uint32)
        hp, hk, _ = _buf(hi, np.uint32)
        ip, ik, _ = _buf(init, np.uint8)
        s = C.c_uint64()
        _check(lib().vc_stream_open(self.h, n_ids, lp, hp, ip, C.byref(s)))
        return s.value

    def submit(self, stream: int, events: np.ndarray, status_out: np.ndarray | None = None) -> int:
        ev = np.ascontiguousarray(events, dtype=np.uint32)
        sp = None if status_out is None else status_out.ctypes.data_as(C.c_void_p)
        ch = C.c_uint64()
        rc = lib().vc_stream_submit(self.h, stream, ev.ctypes.data_as(C.c_void_p), ev.size, sp, C.byref(ch))
        _check(rc)
        return ch.value

    def poll(self, cap: int = 4096):
        out = (vc_completion * cap)()
        n = C.c_uint32()
        _check(lib().vc_poll(self.h, out, cap, C.byref(n)))
        return [out[i] for i in range(n.value)]

    def close_stream(self, stream: int, n_ids: int) -> np.ndarray:
        fin = np.empty(max(n_ids, 1), np.uint8)
        _check(lib().vc_stream_close(self.h, stream, fin.ctypes.data_as(C.c_void_p)))
        return fin[:n_ids]

    def now(self) -> float:
        return lib().vc_server_now(self.h)

    def close(self):
        if self.h:
            lib().vc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""ctypes binding of libldpcfd.so (see include/ldpc_fd.h for the contract).

Argument marshalling only: every step of decoding runs in the library's HIP
kernels.  PyTorch supplies device buffers and the current HIP stream.  Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libldpcfd.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "ldpc_fd.h")

OK, E_INVALID, E_UNSUPPORTED, E_NOMEM, E_HIP = 0, -1, -2, -3, -4
PREC = {"fp32": 0, "fp16": 1, "bf16": 2, "log8": 3}
MODE = {"plain": 0, "fused": 1, "logsp": 2, "fsp": 3}
STATUS_CONVERGED, STATUS_MISMATCH = 1, 2
K_FUSED, K_CHECK, K_VAR = 0, 1, 2
TUNE = {"lane_entries": 0, "grid_blocks": 1, "chunk": 2, "graphs": 3, "tail_entries": 4, "tail_frames": 5, "precise": 6, "decision_mfma": 7, "tail_split": 8,
        "quant_bits": 9, "quant_step": 10, "tail_chunk": 11, "batch_retire": 12, "first_chunk": 13}

_lib = None
_c_void_p, _i32, _i64, _u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32

_SIGS = {
    "ldpc_fd_create_code": (_i32, [_i32, _i32, _i32, _c_void_p, _c_void_p, _c_void_p, _u32, ctypes.POINTER(_c_void_p)]),
    "ldpc_fd_destroy_code": (_i32, [_c_void_p]),
    "ldpc_fd_code_info": (_i32, [_c_void_p] + [ctypes.POINTER(_i32)] * 5),
    "ldpc_fd_workspace_bytes": (_i32, [_c_void_p, _i32, _i32, _i32, ctypes.POINTER(_i64)]),
    "ldpc_fd_decode": (_i32, [_c_void_p, _i32, _c_void_p, _i32, _i32, _i32, _c_void_p, _c_void_p, _c_void_p,
                              _c_void_p, _c_void_p, _i64, _c_void_p]),
    "ldpc_fd_round": (_i32, [_c_void_p, _i32, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                             _c_void_p, _i32, _i32, _c_void_p]),
    "ldpc_fd_round_noalloc": (_i32, [_c_void_p, _i32, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                     _c_void_p, _c_void_p, _i32, _i32, _c_void_p]),
    "ldpc_fd_posterior": (_i32, [_c_void_p, _i32, _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "ldpc_fd_decode_posterior": (_i32, [_c_void_p, _i32, _c_void_p, _i32, _c_void_p, _c_void_p, _i64, _c_void_p,
                                        _c_void_p]),
    "ldpc_fd_decode_symbols": (_i32, [_c_void_p, _i32, _c_void_p, _i32, _c_void_p, _c_void_p, _i64, _c_void_p,
                                      _c_void_p, _c_void_p]),
    "ldpc_fd_decode_prior": (_i32, [_c_void_p, _i32, _c_void_p, _i32, _i32, _c_void_p, _c_void_p, _c_void_p,
                                    _c_void_p, _c_void_p, _i64, _c_void_p]),
    "ldpc_fd_set_tuning": (_i32, [_c_void_p, _i32, _i32]),
    "ldpc_fd_get_tuning": (_i32, [_c_void_p, _i32, ctypes.POINTER(_i32)]),
    "ldpc_fd_profile_enable": (_i32, [_i32]),
    "ldpc_fd_profile_read": (_i32, [_i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]),
    "ldpc_fd_last_error": (ctypes.c_char_p, []),
    "ldpc_fd_pool_slot_bytes": (_i32, [_c_void_p, _i32, ctypes.POINTER(_i64)]),
    "ldpc_fd_pool_create": (_i32, [ctypes.POINTER(_c_void_p), _i32, ctypes.POINTER(_i32), _i32, _c_void_p,
                                   ctypes.POINTER(_c_void_p)]),
    "ldpc_fd_pool_destroy": (_i32, [_c_void_p]),
    "ldpc_fd_pool_free_slots": (_i32, [_c_void_p, _i32, ctypes.POINTER(_i32)]),
    "ldpc_fd_pool_submit": (_i32, [_c_void_p, _i32, _c_void_p, _i32, _c_void_p, _i32, ctypes.POINTER(_i32)]),
    "ldpc_fd_pool_step": (_i32, [_c_void_p, _i32]),
    "ldpc_fd_pool_harvest": (_i32, [_c_void_p, _i32, _i32, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                    ctypes.POINTER(_i32)]),
    "ldpc_fd_pool_active": (_i32, [_c_void_p, _i32, ctypes.POINTER(_i32)]),
    "ldpc_fd_pool_create_budget": (_i32, [ctypes.POINTER(_c_void_p), _i32, _i64, _i32, _c_void_p,
                                          ctypes.POINTER(_c_void_p)]),
    "ldpc_fd_pool_budget_slots": (_i32, [ctypes.POINTER(_c_void_p), _i32, _i64, _i32, ctypes.POINTER(_i32)]),
    "ldpc_fd_decode_ex": (_i32, [_c_void_p, _c_void_p, _c_void_p]),
    "ldpc_fd_pool_set_schedule": (_i32, [_c_void_p, _i32, _i32]),
    "ldpc_fd_run_rounds": (_i32, [_c_void_p, _i32, _c_void_p, _i32, _i32, _c_void_p, _c_void_p, _c_void_p,
                                  _c_void_p, _i32, _i32, _c_void_p]),
}

FLAG_NO_EARLY_STOP, FLAG_VALIDATION, FLAG_ASYNC = 1, 2, 4


class DecodeArgs(ctypes.Structure):
    """ldpc_fd_decode_args (include/ldpc_fd.h)."""
    _fields_ = [("frames", _i32), ("max_iter", _i32), ("prec", _i32), ("mode", _i32), ("flags", _u32),
                ("llr", _c_void_p), ("hard", _c_void_p), ("synd", _c_void_p), ("iters", _c_void_p),
                ("status", _c_void_p), ("posterior", _c_void_p), ("workspace", _c_void_p),
                ("workspace_bytes", _i64)]


class LdpcFdError(RuntimeError):
    def __init__(self, rc, msg):
        super().__init__(f"libldpcfd error {rc}: {msg}")
        self.rc = rc


def lib():
    """Load libldpcfd.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                               "python -m paper_1008_4370_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Names of the functions declared in include/ldpc_fd.h."""
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ldpc_fd_\w+)\s*\(", text, re.M)))


def _check(rc):
    if rc != OK:
        raise LdpcFdError(rc, lib().ldpc_fd_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Code:
    """A code object on the current HIP device (Sec. 2: {x : Hx = 0})."""

    def __init__(self, M, N, m, row_ptr, col, val, poly: int = 0):
        self.M, self.N, self.m = int(M), int(N), int(m)
        self._rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self._col = np.ascontiguousarray(col, dtype=np.int32)
        self._val = np.ascontiguousarray(val, dtype=np.uint16)
        h = ctypes.c_void_p()
        _check(lib().ldpc_fd_create_code(self.M, self.N, self.m, self._rp.ctypes.data, self._col.ctypes.data,
                                         self._val.ctypes.data, int(poly), ctypes.byref(h)))
        self.handle = h
        vals = [_i32() for _ in range(5)]
        _check(lib().ldpc_fd_code_info(self.handle, *[ctypes.byref(v) for v in vals]))
        self.E, self.kmax = vals[3].value, vals[4].value
        self.q = 1 << self.m

    def set_tuning(self, **kw):
        for k, v in kw.items():
            _check(lib().ldpc_fd_set_tuning(self.handle, TUNE[k], int(v)))

    def get_tuning(self) -> dict:
        out = {}
        for k, key in TUNE.items():
            v = _i32()
            _check(lib().ldpc_fd_get_tuning(self.handle, key, ctypes.byref(v)))
            out[k] = v.value
        return out

    @classmethod
    def from_synth(cls, code):
        return cls(code.M, code.N, code.m, code.row_ptr, code.col, code.val, code.poly)

    def close(self):
        if getattr(self, "handle", None):
            lib().ldpc_fd_destroy_code(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(code: Code, frames: int, prec: str = "fp32", mode: str = "fused") -> int:
    out = _i64()
    _check(lib().ldpc_fd_workspace_bytes(code.handle, int(frames), PREC[prec], MODE[mode], ctypes.byref(out)))
    return out.value


class Decoder:
    """Reusable decode context: output tensors and workspace for up to `frames`."""

    def __init__(self, code: Code, frames: int, prec: str = "fp32", mode: str = "fused", device="cuda"):
        import torch
        self.code, self.frames, self.prec, self.mode = code, int(frames), prec, mode
        F = self.frames
        self.ws_bytes = workspace_bytes(code, F, prec, mode)
        self.workspace = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        self.hard = torch.empty((F, code.N), dtype=torch.uint8, device=device)
        self.synd = torch.empty((F, code.M), dtype=torch.uint8, device=device)
        self.iters = torch.empty((F,), dtype=torch.int32, device=device)
        self.status = torch.empty((F,), dtype=torch.int32, device=device)

    def __call__(self, llr, max_iter: int):
        """llr: device float32 [F, N, m] (F <= frames).  Returns views of the outputs."""
        F = llr.shape[0]
        assert F <= self.frames and llr.is_contiguous() and llr.dtype.itemsize == 4
        assert tuple(llr.shape[1:]) == (self.code.N, self.code.m)
        _check(lib().ldpc_fd_decode(self.code.handle, F, _ptr(llr), int(max_iter), PREC[self.prec],
                                    MODE[self.mode], _ptr(self.hard), _ptr(self.synd), _ptr(self.iters),
                                    _ptr(self.status), _ptr(self.workspace), self.ws_bytes, _stream()))
        self._last = (llr, F)
        return dict(hard=self.hard[:F], synd=self.synd[:F], iters=self.iters[:F], status=self.status[:F])

    def decode_ex(self, llr, max_iter: int, flags: int = 0):
        """ldpc_fd_decode_ex with `flags` (FLAG_*); with FLAG_VALIDATION the
        result also holds the FP64 posteriors [F, N, q]."""
        import torch
        F = llr.shape[0]
        assert F <= self.frames and llr.is_contiguous() and llr.dtype == torch.float32
        assert tuple(llr.shape[1:]) == (self.code.N, self.code.m)
        post = None
        if flags & FLAG_VALIDATION:
            post = torch.empty((F, self.code.N, self.code.q), dtype=torch.float64, device=llr.device)
        a = DecodeArgs(F, int(max_iter), PREC[self.prec], MODE[self.mode], int(flags), llr.data_ptr(),
                       self.hard.data_ptr(), self.synd.data_ptr(), self.iters.data_ptr(), self.status.data_ptr(),
                       None if post is None else post.data_ptr(), self.workspace.data_ptr(), self.ws_bytes)
        _check(lib().ldpc_fd_decode_ex(self.code.handle, ctypes.byref(a), _stream()))
        self._last = (llr, F)
        out = dict(hard=self.hard[:F], synd=self.synd[:F], iters=self.iters[:F], status=self.status[:F])
        if post is not None:
            out["posterior"] = post
        return out

    def decode_prior(self, prior, max_iter: int):
        """prior: device float32 [F, N, q] symbol priors (ldpc_fd_decode_prior;
        FUSED mode).  Returns views of the outputs."""
        F = prior.shape[0]
        assert self.mode == "fused" and F <= self.frames and prior.is_contiguous() and prior.dtype.itemsize == 4
        assert tuple(prior.shape[1:]) == (self.code.N, self.code.q)
        _check(lib().ldpc_fd_decode_prior(self.code.handle, F, _ptr(prior), int(max_iter), PREC[self.prec],
                                          _ptr(self.hard), _ptr(self.synd), _ptr(self.iters), _ptr(self.status),
                                          _ptr(self.workspace), self.ws_bytes, _stream()))
        self._last = None
        return dict(hard=self.hard[:F], synd=self.synd[:F], iters=self.iters[:F], status=self.status[:F])

    def posterior(self):
        """Validation mode: FP64 posteriors [F, N, q] of the last decode's frames
        at their stopping rounds (FUSED mode; ldpc_fd_decode_posterior)."""
        import torch
        if self.mode != "fused":
            raise ValueError("posteriors of a decode need the fused mode's message buffers")
        if not self._last:
            raise ValueError("posteriors follow a decode from BPSK LLRs")
        llr, F = self._last
        out = torch.empty((F, self.code.N, self.code.q), dtype=torch.float64, device=llr.device)
        _check(lib().ldpc_fd_decode_posterior(self.code.handle, F, _ptr(llr), PREC[self.prec], _ptr(self.iters),
                                              _ptr(self.workspace), self.ws_bytes, _ptr(out), _stream()))
        return out

    def symbols(self, soft: bool = False):
        """Symbol-MAP decisions [F, N] (uint8) of the last decode's frames at their
        stopping rounds, and with soft=True also their FP32 posteriors [F, N, q]
        (FUSED mode; ldpc_fd_decode_symbols)."""
        import torch
        if self.mode != "fused":
            raise ValueError("symbol decisions of a decode need the fused mode's message buffers")
        if not self._last:
            raise ValueError("symbol decisions follow a decode from BPSK LLRs")
        llr, F = self._last
        sym = torch.empty((F, self.code.N), dtype=torch.uint8, device=llr.device)
        post = torch.empty((F, self.code.N, self.code.q), dtype=torch.float32, device=llr.device) if soft else None
        _check(lib().ldpc_fd_decode_symbols(self.code.handle, F, _ptr(llr), PREC[self.prec], _ptr(self.iters),
                                            _ptr(self.workspace), self.ws_bytes, _ptr(sym), _ptr(post), _stream()))
        return (sym, post) if soft else sym


def decode(code: Code, llr, max_iter: int, prec: str = "fp32", mode: str = "fused"):
    """One-shot decode of device LLRs [F, N, m] (allocates its own buffers)."""
    return Decoder(code, llr.shape[0], prec, mode, device=llr.device)(llr, max_iter)


def round_step(code: Code, llr, c2v_in=None, mode: str = "plain", prec: str = "fp32"):
    """One flooding round from an imported FP32 state (ldpc_fd_round)."""
    import torch
    F = llr.shape[0]
    dev = llr.device
    c2v_out = torch.empty((F, code.E, code.q), dtype=torch.float32, device=dev)
    v2c_out = torch.empty_like(c2v_out) if mode != "fused" else None
    hard = torch.zeros((F, code.N), dtype=torch.uint8, device=dev)
    fsynd = torch.zeros((F, code.M), dtype=torch.uint8, device=dev)
    synd = torch.zeros((F, code.M), dtype=torch.uint8, device=dev)
    _check(lib().ldpc_fd_round(code.handle, F, _ptr(llr), _ptr(c2v_in), _ptr(v2c_out), _ptr(c2v_out),
                               _ptr(hard), _ptr(fsynd), _ptr(synd), MODE[mode], PREC[prec], _stream()))
    return dict(c2v=c2v_out, v2c=v2c_out, hard=hard, fsynd=fsynd, synd=synd)


def run_rounds(code: Code, llr, rounds: int, c2v=None, mode: str = "fused", prec: str = "fp32"):
    """ldpc_fd_run_rounds: `rounds` rounds from the FP32 state c2v [F, E, q]
    (None: from the channel).  Returns the new state and the last decision."""
    import torch
    F = llr.shape[0]
    dev = llr.device
    state = (torch.empty((F, code.E, code.q), dtype=torch.float32, device=dev) if c2v is None
             else c2v.clone().contiguous())
    hard = torch.zeros((F, code.N), dtype=torch.uint8, device=dev)
    fsynd = torch.zeros((F, code.M), dtype=torch.uint8, device=dev)
    synd = torch.zeros((F, code.M), dtype=torch.uint8, device=dev)
    _check(lib().ldpc_fd_run_rounds(code.handle, F, _ptr(llr), int(rounds), 1 if c2v is None else 0, _ptr(state),
                                    _ptr(hard), _ptr(fsynd), _ptr(synd), MODE[mode], PREC[prec], _stream()))
    return dict(c2v=state, hard=hard, fsynd=fsynd, synd=synd)


def round_step_noalloc(code: Code, llr, c2v_in=None, mode: str = "plain", prec: str = "fp32"):
    """ldpc_fd_round_noalloc: the same round with the library's static scratch
    (no device allocation inside the call, no synchronisation)."""
    import torch
    F = llr.shape[0]
    dev = llr.device
    c2v_out = torch.empty((F, code.E, code.q), dtype=torch.float32, device=dev)
    v2c_out = torch.empty_like(c2v_out) if mode != "fused" else None
    hard = torch.zeros((F, code.N), dtype=torch.uint8, device=dev)
    fsynd = torch.zeros((F, code.M), dtype=torch.uint8, device=dev)
    synd = torch.zeros((F, code.M), dtype=torch.uint8, device=dev)
    _check(lib().ldpc_fd_round_noalloc(code.handle, F, _ptr(llr), _ptr(c2v_in), _ptr(v2c_out), _ptr(c2v_out),
                                       _ptr(hard), _ptr(fsynd), _ptr(synd), MODE[mode], PREC[prec], _stream()))
    return dict(c2v=c2v_out, v2c=v2c_out, hard=hard, fsynd=fsynd, synd=synd)


def posterior(code: Code, llr, c2v):
    """Validation mode: FP64 posteriors [F, N, q] from an FP32 check-to-variable
    state [F, E, q] (ldpc_fd_posterior)."""
    import torch
    F = llr.shape[0]
    assert c2v.dtype == torch.float32 and c2v.is_contiguous() and tuple(c2v.shape) == (F, code.E, code.q)
    out = torch.empty((F, code.N, code.q), dtype=torch.float64, device=llr.device)
    _check(lib().ldpc_fd_posterior(code.handle, F, _ptr(llr), _ptr(c2v), _ptr(out), _stream()))
    return out


def profile_enable(on: bool = True):
    _check(lib().ldpc_fd_profile_enable(1 if on else 0))


def profile_read(kernel: int):
    """(total milliseconds, launches) of a per-round kernel since the last read."""
    ms, n = ctypes.c_double(), _i64()
    _check(lib().ldpc_fd_profile_read(int(kernel), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def pool_slot_bytes(code: Code, prec: str = "fp32") -> int:
    out = _i64()
    _check(lib().ldpc_fd_pool_slot_bytes(code.handle, PREC[prec], ctypes.byref(out)))
    return out.value


def pool_budget_slots(codes, hbm_budget: int, prec: str = "fp32") -> list[int]:
    """Slot counts a pool created from an HBM budget of `hbm_budget` bytes gets
    (ldpc_fd_pool_budget_slots)."""
    arr = (ctypes.c_void_p * len(codes))(*[c.handle for c in codes])
    out = (_i32 * len(codes))()
    _check(lib().ldpc_fd_pool_budget_slots(arr, len(codes), int(hbm_budget), PREC[prec], out))
    return [int(x) for x in out]


class Pool:
    """Continuous-batching decode pool over several codes (ldpc_fd_pool_*)."""

    def __init__(self, codes, slots=None, prec: str = "fp32", hbm_budget: int | None = None):
        """slots: frame slots per code, or None with hbm_budget (bytes) to let
        the library size them (ldpc_fd_pool_create_budget)."""
        self.codes = list(codes)
        arr = (ctypes.c_void_p * len(self.codes))(*[c.handle for c in self.codes])
        h = ctypes.c_void_p()
        if slots is None:
            if hbm_budget is None:
                raise ValueError("give slots or hbm_budget")
            _check(lib().ldpc_fd_pool_create_budget(arr, len(self.codes), int(hbm_budget), PREC[prec], _stream(),
                                                    ctypes.byref(h)))
        else:
            sl = (_i32 * len(slots))(*[int(s) for s in slots])
            _check(lib().ldpc_fd_pool_create(arr, len(self.codes), sl, PREC[prec], _stream(), ctypes.byref(h)))
        self.handle = h
        if slots is None:
            slots = []
            for k in range(len(self.codes)):
                n = _i32()
                _check(lib().ldpc_fd_pool_free_slots(self.handle, k, ctypes.byref(n)))
                slots.append(n.value)
        self.slots = [int(s) for s in slots]
        self.prec = prec
        self._bufs = [None] * len(self.codes)

    def free_slots(self, k: int) -> int:
        n = _i32()
        _check(lib().ldpc_fd_pool_free_slots(self.handle, k, ctypes.byref(n)))
        return n.value

    def submit(self, k: int, llr, tags, max_iter: int) -> int:
        """Admit frames llr [n, N, m] (device float32, contiguous) of code k;
        returns the number taken.  The library reads n * N * m floats from
        llr's pointer, so the shape, type, device and layout are checked here
        (ValueError) before the call."""
        import torch
        if not 0 <= k < len(self.codes):
            raise ValueError(f"code index {k} outside 0..{len(self.codes) - 1}")
        code = self.codes[k]
        if not isinstance(llr, torch.Tensor):
            raise ValueError("llr must be a torch tensor")
        if llr.dtype != torch.float32:
            raise ValueError(f"llr must be float32, not {llr.dtype}")
        if llr.dim() != 3 or tuple(llr.shape[1:]) != (code.N, code.m):
            raise ValueError(f"llr must have shape [n, {code.N}, {code.m}], not {tuple(llr.shape)}")
        if not llr.is_contiguous():
            raise ValueError("llr must be contiguous")
        if not llr.is_cuda:
            raise ValueError("llr must be in device memory")
        n = int(llr.shape[0])
        t = np.ascontiguousarray(np.asarray(tags, dtype=np.uint64)) if tags is not None else None
        if t is not None and (t.ndim != 1 or t.shape[0] < n):
            raise ValueError(f"tags must hold at least {n} entries")
        got = _i32()
        _check(lib().ldpc_fd_pool_submit(self.handle, k, _ptr(llr), n,
                                         None if t is None else t.ctypes.data, int(max_iter), ctypes.byref(got)))
        return got.value

    def set_schedule(self, schedule: int, lead: int = 0):
        """0: every code's passes concurrently; 1: the heaviest code starts after
        the others' first `lead` passes (ldpc_fd_pool_set_schedule)."""
        _check(lib().ldpc_fd_pool_set_schedule(self.handle, int(schedule), int(lead)))

    def step(self, passes: int = 1):
        _check(lib().ldpc_fd_pool_step(self.handle, int(passes)))

    def harvest(self, k: int, cap: int):
        N = self.codes[k].N
        if self._bufs[k] is None or self._bufs[k][0].shape[0] < cap:
            self._bufs[k] = (np.zeros(cap, np.uint64), np.zeros(cap, np.int32), np.zeros(cap, np.uint32),
                             np.zeros((cap, N), np.uint8))
        tg, it, st, hd = self._bufs[k]
        n = _i32()
        _check(lib().ldpc_fd_pool_harvest(self.handle, k, cap, tg.ctypes.data, it.ctypes.data, st.ctypes.data,
                                          hd.ctypes.data, ctypes.byref(n)))
        m = n.value
        return tg[:m].copy(), it[:m].copy(), st[:m].copy(), hd[:m].copy()

    def active(self, k: int) -> int:
        n = _i32()
        _check(lib().ldpc_fd_pool_active(self.handle, k, ctypes.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "handle", None):
            lib().ldpc_fd_pool_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

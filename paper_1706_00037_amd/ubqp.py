"""ctypes binding of libubqp.so (include/ubqp.h).

Argument marshalling only: every step runs in the HIP library.  Device buffers
are torch CUDA tensors (bit-packed solutions are int64 tensors holding the
uint64 words); the library launches on torch's current stream of the device.
The binding checks on the host that every tensor is on the right device,
contiguous, of the right dtype and large enough, because the library cannot
see the size of a device buffer.  It raises if libubqp.so is not built.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libubqp.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ubqp.h")

UBQP_OK, UBQP_EINVAL, UBQP_ERANGE, UBQP_EASYM, UBQP_ENOMEM, UBQP_EDEVICE = 0, -1, -2, -3, -4, -5
UBQP_DERIV_START, UBQP_TIMING = 1, 2
PHASES = ("diversify", "eval", "screen", "ascent", "select")
MAX_N, MAX_M, MAX_H = 8192, 1 << 22, 256
INT64_MIN = -(1 << 63)

_lib = None


class UbqpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ubqp error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("H", ctypes.c_int32), ("lam_num", ctypes.c_int32),
                ("lam_den", ctypes.c_int32), ("G", ctypes.c_int32), ("max_flips", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("run_seed", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("best_f", ctypes.c_int64), ("have_best", ctypes.c_int32), ("generations", ctypes.c_int32),
                ("best_x_host", ctypes.c_void_p), ("stats_host", ctypes.c_void_p),
                ("gen_ms_host", ctypes.c_void_p), ("phase_ms_host", ctypes.c_void_p)]


def declared_functions() -> list[str]:
    """Names of the functions declared in include/ubqp.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*UBQP_API\s+(?:const\s+)?\w+\s*\*?\s*(ubqp_\w+)\s*\(", text, flags=re.M)


def load():
    """Load libubqp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "ubqp_create": [ctypes.POINTER(P), ctypes.c_int, P],
        "ubqp_set_stream": [P, P],
        "ubqp_destroy": [P],
        "ubqp_sync": [P],
        "ubqp_problem_create": [P, i32, P, ctypes.POINTER(P)],
        "ubqp_problem_destroy": [P],
        "ubqp_problem_info": [P, P, P, P],
        "ubqp_diversify": [P, i32, P, i64, i32, P, i64],
        "ubqp_eval": [P, P, P, i64, P],
        "ubqp_screen": [P, P, i64, i32, i32, P, P, P],
        "ubqp_ascent": [P, P, P, i64, P, P, i64, P, i32, P],
        "ubqp_multistart": [P, P, ctypes.POINTER(Params), P, ctypes.POINTER(Result)],
        "ubqp_run_create": [P, P, ctypes.POINTER(Params), P, ctypes.POINTER(P)],
        "ubqp_run_step": [P, i32],
        "ubqp_run_result": [P, ctypes.POINTER(Result)],
        "ubqp_run_destroy": [P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.ubqp_run_footprint.argtypes = [P, ctypes.POINTER(Params)]
    L.ubqp_run_footprint.restype = ctypes.c_int64
    L.ubqp_last_error.argtypes = [P]
    L.ubqp_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _words(n: int) -> int:
    return (n + 63) // 64


class Problem:
    """Q resident on the device (ubqp_problem_create)."""

    def __init__(self, ctx: "Context", Q):
        Q = np.ascontiguousarray(Q, dtype=np.int32)
        if Q.ndim != 2 or Q.shape[0] != Q.shape[1]:
            raise ValueError("Q must be square")
        self.ctx = ctx
        self.n = int(Q.shape[0])
        self.W = _words(self.n)
        h = ctypes.c_void_p()
        ctx._call("ubqp_problem_create", ctx.h, self.n, Q.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
        self.h = h
        n_, npad, planes = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ctx._call("ubqp_problem_info", h, ctypes.byref(n_), ctypes.byref(npad), ctypes.byref(planes))
        self.n_pad, self.planes = npad.value, planes.value

    def close(self):
        if self.h is not None:
            load().ubqp_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _result_buffers(W, G):
    out = dict(best_x=np.zeros(W, np.uint64), stats=np.zeros((G, 5), np.int64), gen_ms=np.zeros(G, np.float64),
               phase_ms=np.zeros((G, len(PHASES)), np.float64))
    res = Result(0, 0, 0, out["best_x"].ctypes.data, out["stats"].ctypes.data, out["gen_ms"].ctypes.data,
                 out["phase_ms"].ctypes.data)
    return out, res


def _result_dict(out, res):
    g = int(res.generations)
    return dict(best_f=int(res.best_f), have_best=bool(res.have_best), generations=g, best_x=out["best_x"],
                stats=out["stats"][:g], gen_ms=out["gen_ms"][:g], phase_ms=out["phase_ms"][:g])


class Run:
    """A multi-start run advanced generation by generation (ubqp_run_*)."""

    def __init__(self, ctx: "Context", prob: Problem, pr: Params, f_dump=None):
        self.ctx, self.prob, self.pr = ctx, prob, pr
        self.h = None
        dump = ctx._t(f_dump, ctx.torch.int64, pr.G * pr.M, "f_dump") if f_dump is not None else None
        h = ctypes.c_void_p()
        ctx._call("ubqp_run_create", ctx.h, prob.h, ctypes.byref(pr), dump, ctypes.byref(h))
        self.h = h

    def step(self, generations: int = 1):
        self.ctx._call("ubqp_run_step", self.h, generations)

    def result(self) -> dict:
        out, res = _result_buffers(self.prob.W, self.pr.G)
        self.ctx._call("ubqp_run_result", self.h, ctypes.byref(res))
        return _result_dict(out, res)

    def close(self):
        if self.h is not None:
            load().ubqp_run_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A ubqp_ctx on one device, launching on torch's current stream."""

    def __init__(self, device: int = 0):
        import torch

        self.torch = torch
        self.L = load()
        self.device = device
        h = ctypes.c_void_p()
        rc = self.L.ubqp_create(ctypes.byref(h), device, ctypes.c_void_p(self._stream()))
        if rc != UBQP_OK:
            raise UbqpError(rc, "ubqp_create failed")
        self.h = h

    def _stream(self) -> int:
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _call(self, name, *args):
        if name not in ("ubqp_problem_create", "ubqp_problem_info"):
            self.L.ubqp_set_stream(self.h, ctypes.c_void_p(self._stream()))
        rc = getattr(self.L, name)(*args)
        if rc != UBQP_OK:
            raise UbqpError(rc, self.L.ubqp_last_error(self.h).decode())
        return rc

    # ---- tensor checks -------------------------------------------------
    def _t(self, t, dtype, min_numel, name):
        torch = self.torch
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.device.index != self.device:
            raise ValueError(f"{name} must be a CUDA tensor on device {self.device}")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() < min_numel:
            raise ValueError(f"{name} holds {t.numel()} elements, needs {min_numel}")
        return ctypes.c_void_p(t.data_ptr())

    # ---- entry points ----------------------------------------------------
    def problem(self, Q) -> Problem:
        return Problem(self, Q)

    def diversify(self, n, seeds, H, X, M=None):
        torch = self.torch
        W = _words(n)
        S = seeds.numel() // W
        M = X.numel() // W if M is None else M
        self._call("ubqp_diversify", self.h, n, self._t(seeds, torch.int64, S * W, "seeds"), S, H,
                   self._t(X, torch.int64, M * W, "X"), M)

    def eval(self, prob: Problem, X, f, M=None):
        torch = self.torch
        M = X.numel() // prob.W if M is None else M
        self._call("ubqp_eval", self.h, prob.h, self._t(X, torch.int64, M * prob.W, "X"), M,
                   self._t(f, torch.int64, M, "f"))

    def screen(self, f, lam_num, lam_den, idx, npass, sum_max, M=None):
        torch = self.torch
        M = f.numel() if M is None else M
        self._call("ubqp_screen", self.h, self._t(f, torch.int64, M, "f"), M, lam_num, lam_den,
                   self._t(idx, torch.int32, M, "idx"), self._t(npass, torch.int64, 1, "npass"),
                   self._t(sum_max, torch.int64, 2, "sum_max"))

    def ascent(self, prob: Problem, X, idx, nidx, f, flips, max_idx=None, max_flips=0):
        torch = self.torch
        max_idx = idx.numel() if max_idx is None else max_idx
        M = X.numel() // prob.W
        self._call("ubqp_ascent", self.h, prob.h, self._t(X, torch.int64, M * prob.W, "X"), M,
                   self._t(idx, torch.int32, max_idx, "idx"), self._t(nidx, torch.int64, 1, "nidx"),
                   max_idx, self._t(f, torch.int64, M, "f"), max_flips, self._t(flips, torch.int32, M, "flips"))

    def multistart(self, prob: Problem, M, H, lam_num, lam_den, G, max_flips=0, run_seed=0, flags=0,
                   f_dump=None):
        """The whole loop in one call.  Returns dict(best_f, have_best, best_x (numpy
        uint64 [W]), stats (numpy int64 [G, 5]), gen_ms (numpy float64 [G]))."""
        torch = self.torch
        pr = Params(M, H, lam_num, lam_den, G, max_flips, flags, run_seed)
        out, res = _result_buffers(prob.W, G)
        dump = self._t(f_dump, torch.int64, G * M, "f_dump") if f_dump is not None else None
        self._call("ubqp_multistart", self.h, prob.h, ctypes.byref(pr), dump, ctypes.byref(res))
        return _result_dict(out, res)

    def run(self, prob: Problem, M, H, lam_num, lam_den, G, max_flips=0, run_seed=0, flags=0,
            f_dump=None) -> "Run":
        return Run(self, prob, Params(M, H, lam_num, lam_den, G, max_flips, flags, run_seed), f_dump)

    def footprint(self, prob: Problem, M, H, G) -> int:
        pr = Params(M, H, 1, 2, G, 0, 0, 0)
        return int(self.L.ubqp_run_footprint(prob.h, ctypes.byref(pr)))

    def sync(self):
        self._call("ubqp_sync", self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            self.L.ubqp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

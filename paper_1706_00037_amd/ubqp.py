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

UBQP_OK, UBQP_EINVAL, UBQP_ERANGE, UBQP_EASYM, UBQP_ENOMEM, UBQP_EDEVICE, UBQP_EBUSY = 0, -1, -2, -3, -4, -5, -6
UBQP_ELIMIT = -7
UBQP_DERIV_START, UBQP_TIMING, UBQP_NO_GRAPH, UBQP_AUTOTUNE, UBQP_BLEND = 1, 2, 4, 8, 16
UBQP_EVAL_VARIANTS = 6
UBQP_FMT_ORLIB, UBQP_FMT_TRIPLETS = 1, 2
PHASES = ("diversify", "eval", "screen", "ascent", "select", "ascent_kernel")  # the last is a part of "ascent"
MAX_N, MAX_M, MAX_H = 8192, 1 << 22, 256
UBQP_SCREEN_NOALLOC_MAX_M = 1 << 22
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


class SeqParams(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("samples", ctypes.c_int32), ("H", ctypes.c_int32),
                ("lam_num", ctypes.c_int32), ("lam_den", ctypes.c_int32), ("max_flips", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("flags", ctypes.c_uint32), ("pad_", ctypes.c_int32),
                ("run_seed", ctypes.c_uint64), ("time_budget_ms", ctypes.c_double)]


class SeqResult(ctypes.Structure):
    _fields_ = [("best_x_host", ctypes.c_void_p), ("history_host", ctypes.c_void_p),
                ("history_ms_host", ctypes.c_void_p), ("history_cap", ctypes.c_int64), ("f_dump_d", ctypes.c_void_p),
                ("best_f", ctypes.c_int64), ("have_best", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("iterations_done", ctypes.c_int64), ("sample_sum", ctypes.c_int64), ("start_f", ctypes.c_int64),
                ("passers", ctypes.c_int64), ("flips", ctypes.c_int64), ("improvements", ctypes.c_int64),
                ("windows", ctypes.c_int64), ("evaluated", ctypes.c_int64), ("ms", ctypes.c_double),
                ("ms_device", ctypes.c_double)]


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
        "ubqp_problem_create_typed": [P, i32, P, i32, ctypes.POINTER(P)],
        "ubqp_problem_destroy": [P],
        "ubqp_problem_info": [P, P, P, P],
        "ubqp_problem_set_flip_limit": [P, i32],
        "ubqp_diversify": [P, i32, P, i64, i32, P, i64],
        "ubqp_blend": [P, i32, P, i64, i64, i64, u64, P],
        "ubqp_sequential": [P, P, P, P],
        "ubqp_mfma_peak": [P, P],
        "ubqp_read_peak": [P, i64, i64, i64, P],
        "ubqp_eval_ops": [P, i64, P, P],
        "ubqp_relink": [P, P, P, i64, P, i64, i32, P, P, P, P],
        "ubqp_eval": [P, P, P, i64, P],
        "ubqp_eval_variant": [P, P, P, i64, P, i32],
        "ubqp_tune_eval": [P, P, i64, ctypes.POINTER(i32), P],
        "ubqp_screen": [P, P, i64, i32, i32, P, P, P],
        "ubqp_screen_noalloc": [P, P, i64, i32, i32, P, P, P],
        "ubqp_ascent": [P, P, P, i64, P, P, i64, P, i32, P],
        "ubqp_multistart": [P, P, ctypes.POINTER(Params), P, ctypes.POINTER(Result)],
        "ubqp_run_create": [P, P, ctypes.POINTER(Params), P, ctypes.POINTER(P)],
        "ubqp_run_step": [P, i32],
        "ubqp_run_result": [P, ctypes.POINTER(Result)],
        "ubqp_run_destroy": [P],
        "ubqp_batch_create": [P, i32, P, ctypes.POINTER(Params), ctypes.POINTER(P)],
        "ubqp_batch_step": [P, i32],
        "ubqp_batch_result": [P, i32, ctypes.POINTER(Result)],
        "ubqp_batch_destroy": [P],
        "ubqp_server_create": [P, i64, i32, ctypes.POINTER(P)],
        "ubqp_server_submit": [P, i32, P, i32, ctypes.POINTER(Params), P, P, ctypes.POINTER(i64)],
        "ubqp_server_wait": [P, i64, P, i32, ctypes.POINTER(i32)],
        "ubqp_server_set_queue_limit": [P, i64],
        "ubqp_server_stats": [P, P],
        "ubqp_server_destroy": [P],
        "ubqp_read_instance": [ctypes.c_char_p, i32, i32, P, P, P, i64, P, i32],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.ubqp_run_footprint.argtypes = [P, ctypes.POINTER(Params)]
    L.ubqp_run_footprint.restype = ctypes.c_int64
    L.ubqp_batch_footprint.argtypes = [i32, P, ctypes.POINTER(Params)]
    L.ubqp_batch_footprint.restype = ctypes.c_int64
    L.ubqp_request_footprint.argtypes = [i32, i32, ctypes.POINTER(Params)]
    L.ubqp_request_footprint.restype = ctypes.c_int64
    L.ubqp_last_error.argtypes = [P]
    L.ubqp_last_error.restype = ctypes.c_char_p
    L.ubqp_server_error.argtypes = [P]
    L.ubqp_server_error.restype = ctypes.c_char_p
    _lib = L
    return L


def read_instance(path: str, fmt: int = UBQP_FMT_ORLIB, index: int = 0):
    """Problem `index` of a benchmark file (ubqp_read_instance): returns
    (dense symmetric int32 numpy matrix, number of problems in the file)."""
    L = load()
    err = ctypes.create_string_buffer(512)
    count, n = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = L.ubqp_read_instance(os.fsencode(path), fmt, index, ctypes.byref(count), ctypes.byref(n), None, 0,
                              err, len(err))
    if rc != UBQP_OK:
        raise UbqpError(rc, err.value.decode())
    Q = np.zeros((n.value, n.value), dtype=np.int32)
    rc = L.ubqp_read_instance(os.fsencode(path), fmt, index, ctypes.byref(count), ctypes.byref(n),
                              Q.ctypes.data_as(ctypes.c_void_p), Q.size, err, len(err))
    if rc != UBQP_OK:
        raise UbqpError(rc, err.value.decode())
    return Q, count.value


def time_to_target(result: dict, target: int):
    """First generation whose incumbent reaches `target` in a run's result (its
    stats and gen_ms): (generation, ms from the start of the run to the end of
    that generation), or None when no generation reaches it."""
    stats, gen_ms = result["stats"], result["gen_ms"]
    for g in range(int(result["generations"])):
        if int(stats[g][4]) >= target:
            return g, float(gen_ms[g])
    return None


def _words(n: int) -> int:
    return (n + 63) // 64


_ELEM = {np.dtype(np.int8): 1, np.dtype(np.int16): 2, np.dtype(np.int32): 4}


def _coefficients(Q):
    """Q as a contiguous int8 / int16 / int32 square array (other integer types become int32)."""
    Q = np.asarray(Q)
    if Q.dtype not in _ELEM:
        Q = Q.astype(np.int32)
    Q = np.ascontiguousarray(Q)
    if Q.ndim != 2 or Q.shape[0] != Q.shape[1]:
        raise ValueError("Q must be square")
    return Q


class Problem:
    """Q resident on the device (ubqp_problem_create_typed: int8, int16 or int32
    coefficients, checked and converted on the device)."""

    def __init__(self, ctx: "Context", Q):
        Q = _coefficients(Q)
        self.ctx = ctx
        self.n = int(Q.shape[0])
        self.W = _words(self.n)
        h = ctypes.c_void_p()
        ctx._call("ubqp_problem_create_typed", ctx.h, self.n, Q.ctypes.data_as(ctypes.c_void_p), _ELEM[Q.dtype],
                  ctypes.byref(h))
        self.h = h
        n_, npad, planes = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ctx._call("ubqp_problem_info", h, ctypes.byref(n_), ctypes.byref(npad), ctypes.byref(planes))
        self.n_pad, self.planes = npad.value, planes.value

    def set_flip_limit(self, limit: int):
        """Flips an ascent to a local optimum may make on this problem before it stops
        and reports UBQP_ELIMIT (0: the default 64 n_pad + 4096)."""
        self.ctx._call("ubqp_problem_set_flip_limit", self.h, int(limit))

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


class Batch:
    """Several multi-start runs advanced together (ubqp_batch_*): one launch per
    step covers every instance."""

    def __init__(self, ctx: "Context", probs, params):
        self.ctx, self.probs = ctx, list(probs)
        self.params = (Params * len(params))(*params)
        self.h = None
        handles = (ctypes.c_void_p * len(self.probs))(*[p.h.value for p in self.probs])
        self._handles = handles
        h = ctypes.c_void_p()
        ctx._call("ubqp_batch_create", ctx.h, len(self.probs), ctypes.cast(handles, ctypes.c_void_p), self.params,
                  ctypes.byref(h))
        self.h = h

    def step(self, generations: int = 1):
        self.ctx._call("ubqp_batch_step", self.h, generations)

    def result(self, i: int) -> dict:
        out, res = _result_buffers(self.probs[i].W, self.params[i].G)
        self.ctx._call("ubqp_batch_result", self.h, i, ctypes.byref(res))
        return _result_dict(out, res)

    def close(self):
        if self.h is not None:
            load().ubqp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RequestInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("generations", ctypes.c_int32),
                ("best_f", ctypes.c_int64), ("have_best", ctypes.c_int32), ("planes", ctypes.c_int32),
                ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


SERVER_STATS = ("submitted", "finished", "failed", "generations", "max_running", "pool_high", "waiting", "admitted")


def _params(M, H, lam_num, lam_den, G, max_flips=0, run_seed=0, flags=0):
    return Params(M, H, lam_num, lam_den, G, max_flips, flags, run_seed)


def request_footprint(n: int, elem_bytes: int, params: dict) -> int:
    """Pool bytes a request of n variables occupies while admitted (ubqp_request_footprint)."""
    pr = _params(**params)
    return int(load().ubqp_request_footprint(n, elem_bytes, ctypes.byref(pr)))


class Server:
    """The request server (ubqp_server_*): solves submitted problems several at a
    time on one device, each result equal to the solve run alone.

    Q arrays (int8 / int16 / int32) are kept referenced until their request is
    reported by wait(); page-locked arrays make the upload asynchronous."""

    def __init__(self, ctx: "Context", pool_bytes: int, max_active: int):
        self.ctx = ctx
        self.L = ctx.L
        self.h = None
        h = ctypes.c_void_p()
        ctx._call("ubqp_server_create", ctx.h, int(pool_bytes), int(max_active), ctypes.byref(h))
        self.h = h
        self._live = {}

    def _err(self, rc):
        raise UbqpError(rc, self.L.ubqp_server_error(self.h).decode())

    def submit(self, Q, M, H, lam_num, lam_den, G, max_flips=0, run_seed=0, flags=0) -> int:
        if isinstance(Q, np.ndarray):
            Q = _coefficients(Q)
            n, elem, ptr = int(Q.shape[0]), _ELEM[Q.dtype], Q.ctypes.data
        else:                                   # a page-locked torch tensor [n, n]
            if Q.dim() != 2 or Q.shape[0] != Q.shape[1] or not Q.is_contiguous() or Q.device.type != "cpu":
                raise ValueError("Q must be a contiguous square host tensor")
            n, elem, ptr = int(Q.shape[0]), Q.element_size(), Q.data_ptr()
        pr = _params(M, H, lam_num, lam_den, G, max_flips, run_seed, flags)
        bx = np.zeros(_words(n), np.uint64)
        st = np.zeros((G, 5), np.int64)
        rid = ctypes.c_int64()
        rc = self.L.ubqp_server_submit(self.h, n, ctypes.c_void_p(ptr), elem, ctypes.byref(pr),
                                       bx.ctypes.data_as(ctypes.c_void_p), st.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.byref(rid))
        if rc != UBQP_OK:
            self._err(rc)
        self._live[rid.value] = (Q, bx, st)
        return rid.value

    def set_queue_limit(self, max_waiting: int):
        """At most max_waiting requests wait for admission (0: no limit); a submit
        beyond it raises UbqpError with code UBQP_EBUSY."""
        rc = self.L.ubqp_server_set_queue_limit(self.h, int(max_waiting))
        if rc != UBQP_OK:
            self._err(rc)

    def wait(self, timeout_s=None, max_items: int = 256) -> list:
        """Finished requests (at least one unless the timeout passes), as dicts."""
        buf = (RequestInfo * max_items)()
        cnt = ctypes.c_int32()
        tus = -1 if timeout_s is None else int(timeout_s * 1e6)
        rc = self.L.ubqp_server_wait(self.h, tus, ctypes.cast(buf, ctypes.c_void_p), max_items, ctypes.byref(cnt))
        if rc != UBQP_OK:
            self._err(rc)
        out = []
        for k in range(cnt.value):
            r = buf[k]
            Q, bx, st = self._live.pop(r.id)
            out.append(dict(id=r.id, status=r.status, generations=r.generations, best_f=int(r.best_f),
                            have_best=bool(r.have_best), planes=r.planes, best_x=bx, stats=st[:r.generations],
                            t_submit_ns=r.t_submit_ns, t_admit_ns=r.t_admit_ns, t_start_ns=r.t_start_ns,
                            t_done_ns=r.t_done_ns))
        return out

    def stats(self) -> dict:
        a = np.zeros(8, np.int64)
        self.L.ubqp_server_stats(self.h, a.ctypes.data_as(ctypes.c_void_p))
        return dict(zip(SERVER_STATS, (int(v) for v in a)))

    def close(self):
        if self.h is not None:
            self.L.ubqp_server_destroy(self.h)
            self.h = None
            self._live.clear()

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
        if name not in ("ubqp_problem_info",):
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

    def blend(self, n, seeds, X, g, run_seed, M=None):
        torch = self.torch
        W = _words(n)
        S = seeds.numel() // W
        M = X.numel() // W if M is None else M
        self._call("ubqp_blend", self.h, n, self._t(seeds, torch.int64, S * W, "seeds"), S, M, g, run_seed,
                   self._t(X, torch.int64, M * W, "X"))

    def eval(self, prob: Problem, X, f, M=None):
        torch = self.torch
        M = X.numel() // prob.W if M is None else M
        self._call("ubqp_eval", self.h, prob.h, self._t(X, torch.int64, M * prob.W, "X"), M,
                   self._t(f, torch.int64, M, "f"))

    def eval_variant(self, prob: Problem, X, f, variant: int, M=None):
        torch = self.torch
        M = X.numel() // prob.W if M is None else M
        self._call("ubqp_eval_variant", self.h, prob.h, self._t(X, torch.int64, M * prob.W, "X"), M,
                   self._t(f, torch.int64, M, "f"), variant)

    def tune_eval(self, prob: Problem, M: int):
        """(chosen variant, milliseconds of each variant) for prob at M candidates."""
        v = ctypes.c_int32()
        ms = np.zeros(UBQP_EVAL_VARIANTS, np.float64)
        self._call("ubqp_tune_eval", self.h, prob.h, M, ctypes.byref(v), ms.ctypes.data_as(ctypes.c_void_p))
        return int(v.value), [float(t) for t in ms]

    def screen(self, f, lam_num, lam_den, idx, npass, sum_max, M=None):
        torch = self.torch
        M = f.numel() if M is None else M
        self._call("ubqp_screen", self.h, self._t(f, torch.int64, M, "f"), M, lam_num, lam_den,
                   self._t(idx, torch.int32, M, "idx"), self._t(npass, torch.int64, 1, "npass"),
                   self._t(sum_max, torch.int64, 2, "sum_max"))

    def screen_noalloc(self, f, lam_num, lam_den, idx, npass, sum_max, M=None):
        """ubqp_screen_noalloc: the screen with its partials in the library's static
        device scratch (no allocation; calls overlapping on one GPU race)."""
        torch = self.torch
        M = f.numel() if M is None else M
        self._call("ubqp_screen_noalloc", self.h, self._t(f, torch.int64, M, "f"), M, lam_num, lam_den,
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

    def batch(self, probs, params) -> Batch:
        """params: list of dicts with keys M, H, lam_num, lam_den, G and optional
        max_flips, run_seed, flags."""
        ps = [Params(d["M"], d["H"], d["lam_num"], d["lam_den"], d["G"], d.get("max_flips", 0), d.get("flags", 0),
                     d.get("run_seed", 0)) for d in params]
        return Batch(self, probs, ps)

    def multistart_batched(self, probs, params) -> list:
        b = self.batch(probs, params)
        try:
            b.step(params[0]["G"])
            return [b.result(i) for i in range(len(probs))]
        finally:
            b.close()

    def sequential(self, prob: Problem, iterations, samples, H, lam_num, lam_den, max_flips=0, batch=0, run_seed=0,
                   flags=0, time_budget_ms=0.0, f_dump=None, history_cap=1 << 16) -> dict:
        """The main loop of Fig. 2 one candidate per iteration (ubqp_sequential)."""
        sp = SeqParams(iterations, samples, H, lam_num, lam_den, max_flips, batch, flags, 0, run_seed,
                       float(time_budget_ms))
        bx = np.zeros(prob.W, np.uint64)
        hist = np.zeros((history_cap, 2), np.int64)
        hms = np.zeros(history_cap, np.float64)
        dump = self._t(f_dump, self.torch.int64, iterations, "f_dump") if f_dump is not None else None
        r = SeqResult(bx.ctypes.data, hist.ctypes.data, hms.ctypes.data, history_cap, dump)
        self._call("ubqp_sequential", self.h, prob.h, ctypes.byref(sp), ctypes.byref(r))
        k = min(int(r.improvements), history_cap)
        return dict(best_f=int(r.best_f), have_best=bool(r.have_best), best_x=bx, iterations_done=int(r.iterations_done),
                    sample_sum=int(r.sample_sum), start_f=int(r.start_f), passers=int(r.passers), flips=int(r.flips),
                    improvements=int(r.improvements), windows=int(r.windows), evaluated=int(r.evaluated),
                    ms=float(r.ms), ms_device=float(r.ms_device), history=hist[:k].copy(),
                    history_ms=hms[:k].copy())

    def relink(self, prob: Problem, elite, pairs, X_out, f_mid, f_out, steps, max_flips=0):
        """Greedy path relinking of pairs (P x 2 int32 device tensor of elite row
        indices) then ascent (ubqp_relink); device tensors in and out."""
        torch = self.torch
        W = prob.W
        E = elite.numel() // W
        P = pairs.numel() // 2
        self._call("ubqp_relink", self.h, prob.h, self._t(elite, torch.int64, E * W, "elite"), E,
                   self._t(pairs, torch.int32, 2 * P, "pairs"), P, max_flips, self._t(X_out, torch.int64, P * W, "X_out"),
                   self._t(f_mid, torch.int64, P, "f_mid"), self._t(f_out, torch.int64, P, "f_out"),
                   self._t(steps, torch.int32, P, "steps"))

    def relink_elite(self, prob: Problem, elite, max_flips=0) -> dict:
        """Every ordered pair of distinct rows of `elite` (numpy uint64 E x W), in
        row-major order: dict(pairs, X, f_mid, f_out, steps) on the host."""
        torch = self.torch
        elite = np.ascontiguousarray(elite, np.uint64)
        E = elite.shape[0]
        pairs = np.array([(a, b) for a in range(E) for b in range(E) if a != b], np.int32).reshape(-1, 2)
        P = pairs.shape[0]
        ed = torch.from_numpy(elite.view(np.int64)).cuda()
        pd = torch.from_numpy(pairs).cuda()
        X = torch.empty((P, prob.W), dtype=torch.int64, device="cuda")
        fm = torch.empty(P, dtype=torch.int64, device="cuda")
        fo = torch.empty(P, dtype=torch.int64, device="cuda")
        st = torch.empty(P, dtype=torch.int32, device="cuda")
        self.relink(prob, ed, pd, X, fm, fo, st, max_flips)
        self.sync()
        return dict(pairs=pairs, X=X.cpu().numpy().view(np.uint64), f_mid=fm.cpu().numpy(), f_out=fo.cpu().numpy(),
                    steps=st.cpu().numpy())

    def eval_ops(self, prob: Problem, M: int):
        """(executed, dense) int8 matrix-core operations of one evaluation of M
        candidates on prob (ubqp_eval_ops)."""
        ex, de = ctypes.c_double(), ctypes.c_double()
        rc = self.L.ubqp_eval_ops(prob.h, int(M), ctypes.byref(ex), ctypes.byref(de))
        if rc != UBQP_OK:
            raise UbqpError(rc, "ubqp_eval_ops")
        return float(ex.value), float(de.value)

    def read_peak(self, nbytes: int, window: int, per_block: int) -> float:
        """Read bandwidth in GB/s of a streaming kernel over a buffer of nbytes, each
        block cycling through a window (ubqp_read_peak)."""
        v = ctypes.c_double()
        self._call("ubqp_read_peak", self.h, int(nbytes), int(window), int(per_block), ctypes.byref(v))
        return float(v.value)

    def mfma_peak(self) -> float:
        """Sustained int8 matrix-core rate of the device in TOP/s (ubqp_mfma_peak)."""
        v = ctypes.c_double()
        self._call("ubqp_mfma_peak", self.h, ctypes.byref(v))
        return float(v.value)

    def server(self, pool_bytes: int, max_active: int) -> Server:
        return Server(self, pool_bytes, max_active)

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

"""Python binding of libflowmi (MI355X TV-L1 optical flow by preconditioned dual optimisation).

Argument marshalling only: every step of the method runs in the HIP kernels of libflowmi.so,
reached through its C ABI (include/flow.h).  PyTorch supplies device memory and the stream.
The library must be built first (python -m paper_2011_10979_amd.build); without it every entry
point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field, fields

import torch  # noqa: F401  (loads the HIP runtime that libflowmi then shares)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflowmi.so")

FLOW_OK, FLOW_E_INVAL, FLOW_E_NOMEM, FLOW_E_HIP, FLOW_E_NONFINITE, FLOW_E_BUSY, FLOW_E_NOTFOUND = 0, -1, -2, -3, -4, -5, -6
SCHEMES = {"padmm": 0, "rpadmm2": 1, "pdr": 2, "alg1": 3}
STORAGE = {"f32": 0, "f16": 1}
MAX_LEVELS = 16


class FlowError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"flow status {status}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("scheme", ctypes.c_int32), ("lam", ctypes.c_double),
                ("beta", ctypes.c_double), ("c", ctypes.c_double), ("relax", ctypes.c_double),
                ("sigma", ctypes.c_double), ("tau", ctypes.c_double), ("gs_sweeps", ctypes.c_int32),
                ("intensity_scale", ctypes.c_double), ("levels", ctypes.c_int32), ("warps", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("storage", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("tol", ctypes.c_double), ("check_every", ctypes.c_int32), ("alg1_tau", ctypes.c_double),
                ("alg1_sigma", ctypes.c_double)]


class _Result(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("energy", "dual", "gap", "residual", "tv", "data")]


class _Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("H", ctypes.c_int32 * MAX_LEVELS), ("W", ctypes.c_int32 * MAX_LEVELS),
                ("iterations", ctypes.c_int64 * MAX_LEVELS), ("iter_ms", ctypes.c_double * MAX_LEVELS),
                ("total_ms", ctypes.c_double), ("px_iter", ctypes.c_int64), ("graph_replayed", ctypes.c_int32),
                ("level_px", ctypes.c_int64 * MAX_LEVELS), ("launches", ctypes.c_int64 * MAX_LEVELS)]


class _AdmmState(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("w", "u", "v", "px", "py", "q1x", "q1y", "q2x", "q2y", "s", "u0", "v0")]


class _PdrState(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("w", "u", "v", "wb", "ub", "vb", "pbx", "pby", "qb1x", "qb1y",
                                                "qb2x", "qb2y")]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("epochs", ctypes.c_int64), ("active", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("peak_active", ctypes.c_int32), ("arena_bytes", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64),
                ("peak_bytes_in_use", ctypes.c_uint64), ("graphs_captured", ctypes.c_int64)]


class _Pair(ctypes.Structure):
    _fields_ = [("I0", ctypes.c_void_p), ("I1", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("ld", ctypes.c_int64), ("u", ctypes.c_void_p), ("v", ctypes.c_void_p), ("ld_uv", ctypes.c_int64),
                ("res", ctypes.c_void_p), ("levels", ctypes.c_int32)]


_lib = None

EXPORTS = ["flow_params_default", "flow_create", "flow_destroy", "flow_solve", "flow_solve_batched",
           "flow_set_stats", "flow_get_stats", "flow_memory_in_use", "flow_last_error", "flow_op_downsample",
           "flow_op_derivatives", "flow_op_linearize", "flow_op_upsample", "flow_op_admm_iter", "flow_op_pdr_iter",
           "flow_op_energy", "flow_tune_set", "flow_op_admm_tb", "flow_autotune", "flow_get_tuning",
           "flow_tune_choice", "flow_autotune_batched", "flow_server_create", "flow_server_destroy",
           "flow_server_submit", "flow_server_step", "flow_server_poll", "flow_server_drain",
           "flow_server_get_stats", "flow_working_set_bytes", "flow_op_pdr_tb", "flow_op_alg1_tb",
           "flow_solve_static", "flow_static_bytes", "flow_tune_batched_stage"]


def lib():
    """Load libflowmi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2011_10979_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "flow_params_default": [ctypes.POINTER(_Params)],
            "flow_create": [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_size_t],
            "flow_destroy": [vp],
            "flow_solve": [vp, vp, vp, i32, i32, i64, ctypes.POINTER(_Params), vp, vp, i64, ctypes.POINTER(_Result), vp],
            "flow_solve_batched": [vp, i32, ctypes.POINTER(_Pair), ctypes.POINTER(_Params), vp],
            "flow_solve_static": [vp, vp, i32, i32, i64, ctypes.POINTER(_Params), vp, vp, i64, ctypes.POINTER(_Result),
                                  vp],
            "flow_static_bytes": [i32, i32, ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(ctypes.c_uint64)],
            "flow_autotune_batched": [vp, i32, ctypes.POINTER(_Pair), ctypes.POINTER(_Params), vp],
            "flow_tune_batched_stage": [vp, i32, ctypes.POINTER(_Pair), ctypes.POINTER(_Params), i32, i32, i32, i32],
            "flow_server_create": [vp, ctypes.POINTER(_Params), ctypes.c_size_t, i32, vp, ctypes.POINTER(vp)],
            "flow_server_destroy": [vp],
            "flow_working_set_bytes": [i32, i32, ctypes.POINTER(_Params), i32, ctypes.POINTER(ctypes.c_uint64)],
            "flow_server_submit": [vp, ctypes.POINTER(_Pair), ctypes.POINTER(ctypes.c_uint64)],
            "flow_server_step": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)],
            "flow_server_poll": [vp, ctypes.c_uint64, ctypes.POINTER(i32)],
            "flow_server_drain": [vp],
            "flow_server_get_stats": [vp, ctypes.POINTER(_ServerStats)],
            "flow_set_stats": [vp, i32],
            "flow_autotune": [vp, i32, i32, ctypes.POINTER(_Params), vp],
            "flow_get_tuning": [vp, ctypes.c_char_p, ctypes.c_size_t],
            "flow_tune_choice": [vp, i32, i32, i32, i32, i32, i32, i32, i32],
            "flow_get_stats": [vp, ctypes.POINTER(_Stats)],
            "flow_memory_in_use": [vp, ctypes.POINTER(ctypes.c_size_t)],
            "flow_op_downsample": [vp, i32, i32, i64, vp, i64, vp],
            "flow_op_derivatives": [vp, i32, i32, i64, vp, vp, vp],
            "flow_op_linearize": [vp, vp, vp, vp, vp, vp, i32, i32, i64, dbl, dbl, vp, vp, vp, vp, vp],
            "flow_op_upsample": [vp, i64, vp, i32, i32, i64, dbl, vp],
            "flow_op_admm_iter": [ctypes.POINTER(_AdmmState), ctypes.POINTER(_AdmmState), vp, vp, vp, vp, i32, i32,
                                  i64, ctypes.POINTER(_Params), vp],
            "flow_op_admm_tb": [ctypes.POINTER(_AdmmState), ctypes.POINTER(_AdmmState), vp, vp, vp, vp, i32, i32, i64,
                                ctypes.POINTER(_Params), i32, i32, i32, i32, i32, vp],
            "flow_op_pdr_iter": [ctypes.POINTER(_PdrState), vp, vp, vp, vp, vp, vp, vp, i32, i32, i64,
                                 ctypes.POINTER(_Params), vp],
            "flow_op_pdr_tb": [ctypes.POINTER(_PdrState), ctypes.POINTER(_PdrState), vp, vp, vp, vp, vp, vp, i32, i32,
                               i64, ctypes.POINTER(_Params), i32, i32, i32, vp],
            "flow_op_alg1_tb": [ctypes.POINTER(_PdrState), ctypes.POINTER(_PdrState), vp, vp, vp, vp, vp, vp, i32, i32,
                                i64, ctypes.POINTER(_Params), i32, i32, i32, vp],
            "flow_op_energy": [ctypes.POINTER(_AdmmState), vp, vp, vp, i32, i32, i64, dbl, dbl, ctypes.POINTER(_Result),
                               vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.flow_tune_set.argtypes = [ctypes.c_char_p, ctypes.c_int64]
        L.flow_tune_set.restype = ctypes.c_int
        L.flow_last_error.argtypes = []
        L.flow_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def set_tuning(key: str, value: int):
    """Process-wide kernel tuning knob (see flow_tune_set)."""
    _check(lib().flow_tune_set(key.encode(), int(value)))


def _check(status):
    if status != FLOW_OK:
        raise FlowError(status, lib().flow_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _plane(t, name="tensor"):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.dim() == 2):
        raise TypeError(f"{name} must be a 2-D float32 CUDA tensor")
    if t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} must be row-major with a row pitch >= its width")
    return t


def _like(t):
    """Uninitialised plane with the same shape AND row pitch as t (the kernels address every plane
    of one call with a single pitch, so outputs must share it)."""
    H, W = t.shape
    ld = t.stride(0)
    return torch.empty((H, ld), device=t.device, dtype=torch.float32)[:, :W]


def _same_layout(ref, planes, what):
    for k, t in planes:
        if t is None:
            continue
        _plane(t, k)
        if t.shape != ref.shape or t.stride() != ref.stride():
            raise ValueError(f"{what}: plane {k} must have shape {tuple(ref.shape)} and strides {ref.stride()}")


@dataclass
class Params:
    """Mirror of flow_params (defaults as in flow_params_default)."""
    scheme: str = "padmm"
    lam: float = 0.05
    beta: float = 0.0
    c: float = 0.05
    relax: float = 1.0
    sigma: float = 2.0
    tau: float = 0.4
    gs_sweeps: int = 1
    intensity_scale: float = 255.0
    levels: int = 5
    warps: int = 5
    iters: int = 50
    storage: str = "f32"
    use_graph: int = 1
    tol: float = 0.0
    check_every: int = 10
    alg1_tau: float = 0.1
    alg1_sigma: float = 1.25

    def c_struct(self) -> _Params:
        p = _Params()
        _check(lib().flow_params_default(ctypes.byref(p)))
        for f in fields(self):
            val = getattr(self, f.name)
            if f.name == "scheme":
                val = SCHEMES[val]
            elif f.name == "storage":
                val = STORAGE[val]
            setattr(p, f.name, val)
        return p


def _result_dict(r: _Result):
    return {k: getattr(r, k) for k, _ in _Result._fields_}


class Context:
    """A flow_ctx: device arena, graphs and scratch of one GPU."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().flow_create(ctypes.byref(self._h), device, hbm_budget_bytes))

    def close(self):
        if self._h:
            lib().flow_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stats(self, enable: bool):
        _check(lib().flow_set_stats(self._h, 1 if enable else 0))

    def stats(self):
        s = _Stats()
        _check(lib().flow_get_stats(self._h, ctypes.byref(s)))
        n = s.levels
        return dict(levels=n, H=list(s.H[:n]), W=list(s.W[:n]), iterations=list(s.iterations[:n]),
                    iter_ms=list(s.iter_ms[:n]), total_ms=s.total_ms, px_iter=s.px_iter,
                    graph_replayed=bool(s.graph_replayed), level_px=list(s.level_px[:n]),
                    launches=list(s.launches[:n]))

    def autotune(self, H, W, params: Params | None = None, **kw):
        """Time every iteration-kernel choice on the level shapes of an H x W pair; later solves of
        this context use the fastest per level.  Returns the JSON report as a dict."""
        import json
        params = params or Params(**kw)
        _check(lib().flow_autotune(self._h, H, W, ctypes.byref(params.c_struct()), _stream()))
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().flow_get_tuning(self._h, buf, len(buf)))
        return json.loads(buf.value.decode() or "{}")

    def set_batched_stage(self, pairs, level, order, K, ew, params: Params | None = None, **kw):
        """Pin the stage choice of `level` for batches with these pairs' stage shapes (see
        flow_tune_batched_stage; `order` 0 table, 1 work queue, or a wave-row code 2049 / 3073 / 4097)."""
        _set_batched_stage(self, pairs, level, order, K, ew, params or Params(**kw))

    def set_choice(self, key: str, mode: int, K: int = 0, rows: int = 0):
        """Apply one level-shape choice of an autotune report (key "<H>x<W>[w]i<iters>[p<sweeps>]") by hand."""
        import re
        m = re.fullmatch(r"(\d+)x(\d+)(w?)i(\d+)(?:p(\d+)|(a))?", key)
        if not m:
            raise ValueError(f"bad tuning key {key!r}")
        H, W, hw, it = int(m.group(1)), int(m.group(2)), m.group(3) == "w", int(m.group(4))
        sweeps = int(m.group(5)) if m.group(5) else (-1 if m.group(6) else 0)
        _check(lib().flow_tune_choice(self._h, H, W, int(hw), it, sweeps, int(mode), int(K), int(rows)))

    def memory_in_use(self):
        b = ctypes.c_size_t()
        _check(lib().flow_memory_in_use(self._h, ctypes.byref(b)))
        return b.value

    def solve(self, I0, I1, params: Params | None = None, u=None, v=None, **kw):
        """Flow (u, v) from I0 to I1 (2-D float32 CUDA tensors in [0, 1]); returns (u, v, result)."""
        params = params or Params(**kw)
        _plane(I0, "I0")
        _plane(I1, "I1")
        if I0.shape != I1.shape or I0.stride() != I1.stride():
            raise ValueError("I0 and I1 must have the same shape and strides")
        H, W = I0.shape
        if u is None:
            u = torch.empty((H, W), device=I0.device, dtype=torch.float32)
        if v is None:
            v = torch.empty((H, W), device=I0.device, dtype=torch.float32)
        _plane(u, "u")
        _plane(v, "v")
        if u.stride() != v.stride():
            raise ValueError("u and v must share strides")
        res = _Result()
        _check(lib().flow_solve(self._h, _ptr(I0), _ptr(I1), H, W, I0.stride(0), ctypes.byref(params.c_struct()),
                                _ptr(u), _ptr(v), u.stride(0), ctypes.byref(res), _stream()))
        return u, v, _result_dict(res)

    def _pairs(self, pairs):
        n = len(pairs)
        arr = (_Pair * n)()
        results = [_Result() for _ in range(n)]
        outs = []
        for k, pr in enumerate(pairs):
            I0, I1 = pr[0], pr[1]
            levels = int(pr[2]) if len(pr) > 2 else 0
            _plane(I0, "I0")
            _plane(I1, "I1")
            if I0.shape != I1.shape or I0.stride() != I1.stride():
                raise ValueError(f"pair {k}: I0 and I1 must have the same shape and layout")
            H, W = I0.shape
            u = torch.empty((H, W), device=I0.device, dtype=torch.float32)
            v = torch.empty((H, W), device=I0.device, dtype=torch.float32)
            arr[k] = _Pair(I0.data_ptr(), I1.data_ptr(), H, W, I0.stride(0), u.data_ptr(), v.data_ptr(), W,
                           ctypes.cast(ctypes.byref(results[k]), ctypes.c_void_p), levels)
            outs.append((u, v))
        return arr, results, outs

    def solve_batched(self, pairs, params: Params | None = None, **kw):
        """pairs: list of (I0, I1) or (I0, I1, levels); all pairs advance together (one launch per
        step over all pairs).  Returns a list of (u, v, result)."""
        params = params or Params(**kw)
        arr, results, outs = self._pairs(pairs)
        _check(lib().flow_solve_batched(self._h, len(pairs), arr, ctypes.byref(params.c_struct()), _stream()))
        return [(u, v, _result_dict(r)) for (u, v), r in zip(outs, results)]

    def autotune_batched(self, pairs, params: Params | None = None, **kw):
        """Time the batched tile-launch choices per stage of this batch; later solve_batched calls
        on batches with the same stage shapes use the fastest.  Returns the report (the choice of
        each stage) as a dict."""
        import json
        params = params or Params(**kw)
        arr, _, _ = self._pairs(pairs)
        _check(lib().flow_autotune_batched(self._h, len(pairs), arr, ctypes.byref(params.c_struct()), _stream()))
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().flow_get_tuning(self._h, buf, len(buf)))
        return json.loads(buf.value.decode() or "{}")


def _set_batched_stage(ctx, pairs, level, order, K, ew, params):
    arr, _, _ = ctx._pairs(pairs)
    _check(lib().flow_tune_batched_stage(ctx._h, len(pairs), arr, ctypes.byref(params.c_struct()), int(level),
                                         int(order), int(K), int(ew)))


def working_set_bytes(H, W, params: Params | None = None, levels: int = 0, **kw):
    """Device bytes of one pair's working set (see flow_working_set_bytes)."""
    params = params or Params(**kw)
    b = ctypes.c_uint64()
    _check(lib().flow_working_set_bytes(int(H), int(W), ctypes.byref(params.c_struct()), int(levels), ctypes.byref(b)))
    return b.value


def solve_static(I0, I1, params: Params | None = None, u=None, v=None, **kw):
    """flow_solve_static: the plain solve on the current device's static workspace (no context, no
    device allocation by the library; built-in kernel plan).  Returns (u, v, result)."""
    params = params or Params(**kw)
    _plane(I0, "I0")
    _plane(I1, "I1")
    if I0.shape != I1.shape or I0.stride() != I1.stride():
        raise ValueError("I0 and I1 must have the same shape and strides")
    H, W = I0.shape
    if u is None:
        u = torch.empty((H, W), device=I0.device, dtype=torch.float32)
    if v is None:
        v = torch.empty((H, W), device=I0.device, dtype=torch.float32)
    _plane(u, "u")
    _plane(v, "v")
    if u.stride() != v.stride():
        raise ValueError("u and v must share strides")
    res = _Result()
    _check(lib().flow_solve_static(_ptr(I0), _ptr(I1), H, W, I0.stride(0), ctypes.byref(params.c_struct()), _ptr(u),
                                   _ptr(v), u.stride(0), ctypes.byref(res), _stream()))
    return u, v, _result_dict(res)


def static_bytes(H, W, params: Params | None = None, **kw):
    """(bytes flow_solve_static needs for an H x W pair, the static workspace size)."""
    params = params or Params(**kw)
    need, limit = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().flow_static_bytes(int(H), int(W), ctypes.byref(params.c_struct()), ctypes.byref(need),
                                   ctypes.byref(limit)))
    return need.value, limit.value


class Server:
    """Continuous-batching serving engine (flow_server_*): submit pairs as they arrive, call step()
    to run one epoch (every admitted pair advances one warp; queued pairs are admitted as slots and
    budget free up), poll tickets for completion."""

    def __init__(self, ctx: Context, params: Params | None = None, budget_bytes: int = 0, max_active: int = 64,
                 **kw):
        self.params = params or Params(**kw)
        self._stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib().flow_server_create(ctx._h, ctypes.byref(self.params.c_struct()), int(budget_bytes),
                                        int(max_active), ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._ctx = ctx
        self._live = {}

    def submit(self, I0, I1, levels: int = 0):
        _plane(I0, "I0")
        _plane(I1, "I1")
        if I0.shape != I1.shape or I0.stride() != I1.stride():
            raise ValueError("I0 and I1 must have the same shape and layout")
        H, W = I0.shape
        u = torch.empty((H, W), device=I0.device, dtype=torch.float32)
        v = torch.empty((H, W), device=I0.device, dtype=torch.float32)
        res = _Result()
        pr = _Pair(I0.data_ptr(), I1.data_ptr(), H, W, I0.stride(0), u.data_ptr(), v.data_ptr(), W,
                   ctypes.cast(ctypes.byref(res), ctypes.c_void_p), int(levels))
        t = ctypes.c_uint64()
        _check(lib().flow_server_submit(self._h, ctypes.byref(pr), ctypes.byref(t)))
        self._live[t.value] = (I0, I1, u, v, res)       # keeps the buffers alive until done
        return t.value

    def step(self):
        a, q = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().flow_server_step(self._h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def poll(self, ticket):
        """None while running; (u, v, result) once done.  A pair that finished with a non-finite
        energy or gap raises FlowError (FLOW_E_NONFINITE) once, with its outputs in .result; the
        ticket is collected either way."""
        d = ctypes.c_int32()
        st = lib().flow_server_poll(self._h, ticket, ctypes.byref(d))
        if st == FLOW_E_NONFINITE:
            err = FlowError(st, lib().flow_last_error().decode())
            _, _, u, v, res = self._live.pop(ticket)
            err.result = (u, v, _result_dict(res))
            raise err
        _check(st)
        if not d.value:
            return None
        _, _, u, v, res = self._live.pop(ticket)
        return u, v, _result_dict(res)

    def drain(self):
        _check(lib().flow_server_drain(self._h))

    def stats(self):
        s = _ServerStats()
        _check(lib().flow_server_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in _ServerStats._fields_}

    def close(self):
        if self._h:
            lib().flow_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------ operator-level calls -----------------------------------
def downsample(src):
    _plane(src, "src")
    H, W = src.shape
    dst = torch.empty(((H + 1) // 2, (W + 1) // 2), device=src.device, dtype=torch.float32)
    _check(lib().flow_op_downsample(_ptr(src), H, W, src.stride(0), _ptr(dst), dst.stride(0), _stream()))
    return dst


def derivatives(I):
    _plane(I, "I")
    Dx = _like(I)
    Dy = _like(I)
    _same_layout(I, [("Dx", Dx), ("Dy", Dy)], "derivatives")
    _check(lib().flow_op_derivatives(_ptr(I), I.shape[0], I.shape[1], I.stride(0), _ptr(Dx), _ptr(Dy), _stream()))
    return Dx, Dy


def linearize(I0, I1, Dx, Dy, u0, v0, kappa=255.0, beta=0.0):
    _plane(I0, "I0")
    Ix, Iy, It = (_like(I0) for _ in range(3))
    _same_layout(I0, [("I1", I1), ("Dx", Dx), ("Dy", Dy), ("u0", u0), ("v0", v0), ("Ix", Ix), ("Iy", Iy),
                      ("It", It)], "linearize")
    at = torch.zeros(1, device=I0.device, dtype=torch.float32)
    H, W = I0.shape
    _check(lib().flow_op_linearize(_ptr(I0), _ptr(I1), _ptr(Dx), _ptr(Dy), _ptr(u0), _ptr(v0), H, W, I0.stride(0),
                                   kappa, beta, _ptr(Ix), _ptr(Iy), _ptr(It), _ptr(at), _stream()))
    return Ix, Iy, It, at


def upsample(coarse, shape, scale):
    _plane(coarse, "coarse")
    Hf, Wf = shape
    if coarse.shape != ((Hf + 1) // 2, (Wf + 1) // 2):
        raise ValueError("coarse plane must be ceil(H/2) x ceil(W/2)")
    fine = torch.empty((Hf, Wf), device=coarse.device, dtype=torch.float32)
    _check(lib().flow_op_upsample(_ptr(coarse), coarse.stride(0), _ptr(fine), Hf, Wf, fine.stride(0), scale,
                                  _stream()))
    return fine


ADMM_KEYS = ("w", "u", "v", "px", "py", "q1x", "q1y", "q2x", "q2y", "s", "u0", "v0")
PDR_KEYS = ("w", "u", "v", "wb", "ub", "vb", "pbx", "pby", "qb1x", "qb1y", "qb2x", "qb2y")


def _admm_struct(st):
    return _AdmmState(*[st[k].data_ptr() if st.get(k) is not None else None for k in ADMM_KEYS])


def admm_iter(state, Ix, Iy, It, at, params: Params):
    """One ADMM-family iteration; state: dict of planes (ADMM_KEYS); returns the new state dict.
    With "u0", "v0" in the state the increment form is used (u, v are u - u0, It is relative)."""
    ref = _plane(state["u"], "u")
    out = {k: (_like(t) if t is not None else None) for k, t in state.items() if k not in ("u0", "v0")}
    _same_layout(ref, list(state.items()) + [(k + "_out", t) for k, t in out.items()]
                 + [("Ix", Ix), ("Iy", Iy), ("It", It)], "admm_iter")
    H, W = ref.shape
    _check(lib().flow_op_admm_iter(ctypes.byref(_admm_struct(state)), ctypes.byref(_admm_struct(out)), _ptr(Ix),
                                   _ptr(Iy), _ptr(It), _ptr(at), H, W, state["u"].stride(0),
                                   ctypes.byref(params.c_struct()), _stream()))
    return out


def admm_tb(state, Ix, Iy, It, at, params: Params, iters, threads=256, tile_h=16, tile_w=32, order=0):
    """`iters` iterations in one launch of the K-iteration tile kernel (increment form: the state
    must hold "u0", "v0"); returns the new state dict."""
    ref = _plane(state["u"], "u")
    out = {k: (_like(t) if t is not None else None) for k, t in state.items() if k not in ("u0", "v0")}
    _same_layout(ref, list(state.items()) + [(k + "_out", t) for k, t in out.items()]
                 + [("Ix", Ix), ("Iy", Iy), ("It", It)], "admm_tb")
    H, W = ref.shape
    _check(lib().flow_op_admm_tb(ctypes.byref(_admm_struct(state)), ctypes.byref(_admm_struct(out)), _ptr(Ix),
                                 _ptr(Iy), _ptr(It), _ptr(at), H, W, ref.stride(0), ctypes.byref(params.c_struct()),
                                 iters, threads, tile_h, tile_w, int(order), _stream()))
    return out


def pdr_iter(state, Ix, Iy, It, params: Params, s_out=None):
    """One pDR iteration in place on the dict of planes (PDR_KEYS)."""
    ref = _plane(state["u"], "u")
    H, W = ref.shape
    work = [_like(ref) for _ in range(3)]
    _same_layout(ref, list(state.items()) + [("work%d" % i, t) for i, t in enumerate(work)]
                 + [("Ix", Ix), ("Iy", Iy), ("It", It), ("s_out", s_out)], "pdr_iter")
    st = _PdrState(*[state[k].data_ptr() if state.get(k) is not None else None for k in PDR_KEYS])
    _check(lib().flow_op_pdr_iter(ctypes.byref(st), _ptr(work[0]), _ptr(work[1]), _ptr(work[2]), _ptr(s_out),
                                  _ptr(Ix), _ptr(Iy), _ptr(It), H, W, state["u"].stride(0),
                                  ctypes.byref(params.c_struct()), _stream()))
    return state


def alg1_tb(state, Ix, Iy, It, u0, v0, params: Params, iters, tile_h=16, tile_w=32):
    """`iters` ALG1 iterations in one launch of its tile kernel (state planes as for pDR; y in the
    y bar slots); returns (new state dict, s_out).  I_t is relative to (u0, v0)."""
    return pdr_tb(state, Ix, Iy, It, u0, v0, params, iters, tile_h, tile_w, _entry="flow_op_alg1_tb")


def pdr_tb(state, Ix, Iy, It, u0, v0, params: Params, iters, tile_h=16, tile_w=32, _entry="flow_op_pdr_tb"):
    """`iters` pDR iterations in one launch of the tile kernel; returns (new state dict, s_out).
    I_t is relative to (u0, v0)."""
    ref = _plane(state["u"], "u")
    H, W = ref.shape
    out = {k: (_like(ref) if state.get(k) is not None else None) for k in PDR_KEYS}
    s_out = _like(ref)
    _same_layout(ref, [(k, v) for k, v in state.items() if v is not None] +
                 [(k, v) for k, v in out.items() if v is not None] +
                 [("Ix", Ix), ("Iy", Iy), ("It", It), ("u0", u0), ("v0", v0), ("s_out", s_out)], "pdr_tb")
    st_in = _PdrState(*[state[k].data_ptr() if state.get(k) is not None else None for k in PDR_KEYS])
    st_out = _PdrState(*[out[k].data_ptr() if out.get(k) is not None else None for k in PDR_KEYS])
    _check(getattr(lib(), _entry)(ctypes.byref(st_in), ctypes.byref(st_out), _ptr(s_out), _ptr(Ix), _ptr(Iy), _ptr(It),
                                _ptr(u0), _ptr(v0), H, W, ref.stride(0), ctypes.byref(params.c_struct()), int(iters),
                                int(tile_h), int(tile_w), _stream()))
    return out, s_out


def energy(state, Ix, Iy, It, lam=0.05, beta=0.0):
    ref = _plane(state["u"], "u")
    _same_layout(ref, list(state.items()) + [("Ix", Ix), ("Iy", Iy), ("It", It)], "energy")
    H, W = ref.shape
    r = _Result()
    _check(lib().flow_op_energy(ctypes.byref(_admm_struct(state)), _ptr(Ix), _ptr(Iy), _ptr(It), H, W,
                                state["u"].stride(0), lam, beta, ctypes.byref(r), _stream()))
    return _result_dict(r)

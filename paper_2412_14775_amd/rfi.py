"""Thin ctypes binding of librfi (include/rfi.h), with the same names as the C ABI.

Argument marshalling only: every step of the screen runs in the HIP kernels of
librfi.so.  PyTorch supplies device memory and streams.  Because the C ABI sees
raw pointers, this layer checks each tensor's device, dtype, contiguity and
size against the plan before passing its pointer on, so that no kernel is ever
given a buffer shorter than the plan implies.

The binding fails loudly (RfiError) when librfi.so is missing: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librfi.so")

RFI_OK = 0
RFI_ERR_INVALID_ARGUMENT = -1
RFI_ERR_OUT_OF_MEMORY = -2
RFI_ERR_DEVICE = -3
RFI_ERR_UNSUPPORTED = -4

RFI_VIS_CF32 = 0
RFI_VIS_CF16 = 1

RFI_OPT_NO_SK = 1
RFI_OPT_NO_DS = 2
RFI_OPT_ADAPTIVE = 4
RFI_OPT_PAPER_MIXED = 8

RFI_FLAG_SK_LOW = 1
RFI_FLAG_SK_HIGH = 2
RFI_FLAG_DS_RE = 4
RFI_FLAG_DS_IM = 8

STATE_RECORD_BYTES = 64

# Every symbol include/rfi.h declares (checked by the CPU test suite).
EXPORTS = (
    "rfi_params_default", "rfi_plan_create", "rfi_screen", "rfi_destroy", "rfi_last_error",
    "rfi_plan_footprint", "rfi_state_bytes", "rfi_state_get", "rfi_state_set",
    "rfi_state_reset", "rfi_probe_sink_floats", "rfi_probe_read", "rfi_probe_copy", "rfi_probe_half_sums",
    "rfi_server_create", "rfi_server_now", "rfi_server_submit", "rfi_server_poll",
    "rfi_server_drain", "rfi_server_get_stats", "rfi_server_destroy",
    "rfi_sk_null_moments", "rfi_thresholds_from_pfa", "rfi_calibrate_from_stats",
)


class RfiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"librfi error {code}: {msg}")
        self.code = code


class rfi_params(ctypes.Structure):
    _fields_ = [
        ("n_stations", ctypes.c_int32),
        ("n_baselines", ctypes.c_int32),
        ("n_channels", ctypes.c_int32),
        ("n_samples", ctypes.c_int32),
        ("block_m", ctypes.c_int32),
        ("vis_format", ctypes.c_int32),
        ("sk_d", ctypes.c_float),
        ("sk_low", ctypes.c_float),
        ("sk_high", ctypes.c_float),
        ("ds_gamma", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("options", ctypes.c_uint32),
        ("kappa_sk", ctypes.c_float),
        ("kappa_ds", ctypes.c_float),
        ("n_warm", ctypes.c_int32),
        ("block_f", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rfi_server_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("n_slots", ctypes.c_int32),
                ("hbm_budget", ctypes.c_uint64), ("use_graphs", ctypes.c_int32),
                ("max_graphs", ctypes.c_int32)]


class rfi_request(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("vis", ctypes.c_void_p), ("avg", ctypes.c_void_p),
                ("weight", ctypes.c_void_p), ("flags", ctypes.c_void_p), ("stats", ctypes.c_void_p),
                ("arrival", ctypes.c_double), ("tag", ctypes.c_uint64)]


class rfi_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("arrival", ctypes.c_double), ("admitted", ctypes.c_double), ("done", ctypes.c_double)]


class rfi_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("peak_inflight_bytes", ctypes.c_uint64),
                ("peak_inflight", ctypes.c_int32), ("graphs", ctypes.c_int32),
                ("graphs_cached", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librfi.so (built by ``__graft_entry__.build()``); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RfiError(RFI_ERR_UNSUPPORTED,
                       f"{path} is missing: build it with __graft_entry__.build()")
    # PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Loading torch
    # first makes librfi's dependency on that soname bind to the same runtime, so
    # device pointers and stream handles from torch are valid inside librfi.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    runtimes = hip_runtimes_loaded()
    if len(runtimes) > 1:
        raise RfiError(RFI_ERR_DEVICE, "two HIP runtimes are loaded in this process "
                       f"({', '.join(sorted(runtimes))}); import torch before loading librfi")
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    sig = {
        "rfi_params_default": (None, [P(rfi_params)]),
        "rfi_plan_create": (ctypes.c_int, [P(rfi_params), ctypes.c_int, P(vp)]),
        "rfi_screen": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "rfi_destroy": (ctypes.c_int, [vp]),
        "rfi_last_error": (ctypes.c_char_p, []),
        "rfi_plan_footprint": (ctypes.c_int, [vp, P(ctypes.c_size_t)]),
        "rfi_state_bytes": (ctypes.c_size_t, [vp]),
        "rfi_state_get": (ctypes.c_int, [vp, vp, ctypes.c_size_t]),
        "rfi_state_set": (ctypes.c_int, [vp, vp, ctypes.c_size_t]),
        "rfi_state_reset": (ctypes.c_int, [vp, vp]),
        "rfi_probe_sink_floats": (ctypes.c_size_t, [ctypes.c_size_t]),
        "rfi_probe_read": (ctypes.c_int, [vp, ctypes.c_size_t, vp, vp]),
        "rfi_probe_copy": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
        "rfi_probe_half_sums": (ctypes.c_int, [vp, vp]),
        "rfi_server_create": (ctypes.c_int, [P(rfi_server_config), P(vp)]),
        "rfi_server_now": (ctypes.c_double, [vp]),
        "rfi_server_submit": (ctypes.c_int, [vp, P(rfi_request)]),
        "rfi_server_poll": (ctypes.c_int, [vp, P(rfi_completion), ctypes.c_int32,
                                           P(ctypes.c_int32), ctypes.c_double]),
        "rfi_server_drain": (ctypes.c_int, [vp, ctypes.c_double]),
        "rfi_server_get_stats": (ctypes.c_int, [vp, P(rfi_server_stats)]),
        "rfi_server_destroy": (ctypes.c_int, [vp]),
        "rfi_sk_null_moments": (ctypes.c_int, [ctypes.c_int32, ctypes.c_float, P(ctypes.c_double),
                                               P(ctypes.c_double), P(ctypes.c_double)]),
        "rfi_thresholds_from_pfa": (ctypes.c_int, [ctypes.c_int32, ctypes.c_float, ctypes.c_double,
                                                   ctypes.c_double, P(ctypes.c_float), P(ctypes.c_float),
                                                   P(ctypes.c_float)]),
        "rfi_calibrate_from_stats": (ctypes.c_int, [vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_float,
                                                    ctypes.c_double, ctypes.c_double, P(ctypes.c_float),
                                                    P(ctypes.c_float), P(ctypes.c_float), P(ctypes.c_float)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def hip_runtimes_loaded():
    """Distinct libamdhip64 files mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def _check(rc: int):
    if rc != RFI_OK:
        raise RfiError(rc, rfi_last_error())


def rfi_last_error() -> str:
    return load_library().rfi_last_error().decode()


def rfi_params_default(**overrides) -> rfi_params:
    p = rfi_params()
    load_library().rfi_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def rfi_plan_create(params: rfi_params, device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load_library().rfi_plan_create(ctypes.byref(params), device, ctypes.byref(h)))
    return h.value


def rfi_destroy(plan: Optional[int]) -> None:
    _check(load_library().rfi_destroy(plan))


def rfi_plan_footprint(plan: int) -> int:
    n = ctypes.c_size_t()
    _check(load_library().rfi_plan_footprint(plan, ctypes.byref(n)))
    return n.value


def rfi_state_bytes(plan: int) -> int:
    return load_library().rfi_state_bytes(plan)


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def rfi_screen(plan: int, vis, avg, weight, flags=None, stats=None, stream=None) -> None:
    """Raw entry point: pointers (ints) or tensors, no size checks.  Prefer ``Plan.screen``."""
    _check(load_library().rfi_screen(plan, _ptr(vis), _ptr(avg), _ptr(weight), _ptr(flags),
                                     _ptr(stats), _stream_handle(stream)))


def rfi_state_get(plan: int, host_buffer) -> None:
    """Copy the adaptive state into a writable host buffer (numpy array or bytearray)."""
    import numpy as np
    a = np.asarray(host_buffer)
    _check(load_library().rfi_state_get(plan, a.ctypes.data, a.nbytes))


def rfi_state_set(plan: int, host_buffer) -> None:
    import numpy as np
    a = np.ascontiguousarray(host_buffer)
    _check(load_library().rfi_state_set(plan, a.ctypes.data, a.nbytes))


def rfi_state_reset(plan: int, stream=None) -> None:
    _check(load_library().rfi_state_reset(plan, _stream_handle(stream)))


def rfi_probe_sink_floats(nbytes: int) -> int:
    return load_library().rfi_probe_sink_floats(nbytes)


def rfi_probe_read(src, nbytes: int, sink, stream=None) -> None:
    _check(load_library().rfi_probe_read(_ptr(src), nbytes, _ptr(sink), _stream_handle(stream)))


def rfi_probe_copy(dst, src, nbytes: int, stream=None) -> None:
    _check(load_library().rfi_probe_copy(_ptr(dst), _ptr(src), nbytes, _stream_handle(stream)))


HALF_SUMS_VALUES = 65536


def rfi_probe_half_sums(mismatches, stream=None) -> None:
    """Device check of the complex-half sums (include/rfi.h); `mismatches` is a device tensor
    of HALF_SUMS_VALUES 32-bit counters, written by the call."""
    if hasattr(mismatches, "numel") and mismatches.numel() * mismatches.element_size() < 4 * HALF_SUMS_VALUES:
        raise ValueError(f"mismatches must hold {HALF_SUMS_VALUES} 32-bit counters")
    _check(load_library().rfi_probe_half_sums(_ptr(mismatches), _stream_handle(stream)))


# --------------------------------------------------------------------------- checked plan wrapper

class Plan:
    """A plan with tensor-level checks; outputs allocated with torch on the plan's device."""

    def __init__(self, params: rfi_params, device: int = 0):
        import torch
        self.params = params
        self.device = torch.device("cuda", device)
        self.handle = rfi_plan_create(params, device)
        p = params
        self.B, self.C, self.T, self.M = p.n_baselines, p.n_channels, p.n_samples, p.block_m
        self.F = p.block_f
        self.G = self.C // self.F           # channel groups (windows span F channels)
        self.nW = self.T // self.M
        self.cf16 = p.vis_format == RFI_VIS_CF16

    def close(self):
        if self.handle is not None:
            rfi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def vis_shape(self):
        return (self.B, self.C, self.T, 4, 2)

    def vis_dtype(self):
        import torch
        return torch.float16 if self.cf16 else torch.float32

    def footprint(self) -> int:
        return rfi_plan_footprint(self.handle)

    def alloc_outputs(self, flags: bool = True, stats: bool = False):
        import torch
        d = self.device
        out = dict(avg=torch.empty((self.B, self.C, 4, 2), dtype=torch.float32, device=d),
                   weight=torch.empty((self.B, self.C), dtype=torch.float32, device=d),
                   flags=torch.empty((self.B, self.G, self.nW), dtype=torch.uint8, device=d) if flags else None,
                   stats=torch.empty((self.B, self.G, self.nW, 3), dtype=torch.float32, device=d) if stats else None)
        return out

    def _check_tensor(self, name, t, shape, dtype):
        if t is None:
            return
        import torch
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, plan is on {self.device}")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != _numel(shape):
            raise ValueError(f"{name} must have {_numel(shape)} elements {shape}, got {tuple(t.shape)}")

    def screen(self, vis, avg, weight, flags=None, stats=None, stream=None) -> None:
        import torch
        self._check_tensor("vis", vis, self.vis_shape, self.vis_dtype())
        self._check_tensor("avg", avg, (self.B, self.C, 4, 2), torch.float32)
        self._check_tensor("weight", weight, (self.B, self.C), torch.float32)
        self._check_tensor("flags", flags, (self.B, self.G, self.nW), torch.uint8)
        self._check_tensor("stats", stats, (self.B, self.G, self.nW, 3), torch.float32)
        rfi_screen(self.handle, vis, avg, weight, flags, stats, stream)

    def state(self):
        """Adaptive state as a numpy structured array [B][C/F] (n, mean[3], m2[3])."""
        import numpy as np
        dt = np.dtype([("n", np.uint64), ("mean", np.float64, 3), ("m2", np.float64, 3), ("reserved", np.uint64)])
        assert dt.itemsize == STATE_RECORD_BYTES
        a = np.zeros((self.B, self.G), dt)
        rfi_state_get(self.handle, a.view(np.uint8))
        return a


def _numel(shape):
    n = 1
    for s in shape:
        n *= s
    return n


# --------------------------------------------------------------------------- serving loop

def rfi_server_create(n_slots: int = 16, hbm_budget: int = 200 << 30, device: int = 0,
                      use_graphs: bool = True, max_graphs: int = 0) -> int:
    cfg = rfi_server_config(device=device, n_slots=n_slots, hbm_budget=hbm_budget,
                            use_graphs=1 if use_graphs else 0, max_graphs=max_graphs)
    h = ctypes.c_void_p()
    _check(load_library().rfi_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def rfi_server_now(server: int) -> float:
    return load_library().rfi_server_now(server)


def rfi_server_submit(server: int, plan: int, vis, avg, weight, flags=None, stats=None,
                      arrival: float = 0.0, tag: int = 0) -> None:
    req = rfi_request(plan=plan, vis=_ptr(vis), avg=_ptr(avg), weight=_ptr(weight),
                      flags=_ptr(flags), stats=_ptr(stats), arrival=arrival, tag=tag)
    _check(load_library().rfi_server_submit(server, ctypes.byref(req)))


def rfi_server_poll(server: int, max_n: int = 256, timeout: float = 0.0):
    buf = (rfi_completion * max_n)()
    n = ctypes.c_int32()
    _check(load_library().rfi_server_poll(server, buf, max_n, ctypes.byref(n), timeout))
    return [dict(tag=c.tag, status=c.status, slot=c.slot, arrival=c.arrival,
                 admitted=c.admitted, done=c.done) for c in buf[:n.value]]


def rfi_server_drain(server: int, timeout: float = 600.0) -> None:
    _check(load_library().rfi_server_drain(server, timeout))


def rfi_server_get_stats(server: int) -> dict:
    st = rfi_server_stats()
    _check(load_library().rfi_server_get_stats(server, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in st._fields_}


def rfi_server_destroy(server: Optional[int]) -> None:
    _check(load_library().rfi_server_destroy(server))


class Server:
    """Serving loop with tensor checks.  Each in-flight request holds its plan and tensors
    until ``poll`` returns its completion: the scheduler thread reads the plan and the kernels
    write its outputs and adaptive state after ``submit`` has returned, so a caller that drops
    its own references early (``srv.submit(Plan(p), ...)``) must not free them."""

    def __init__(self, n_slots: int = 16, hbm_budget: int = 200 << 30, device: int = 0,
                 use_graphs: bool = True, max_graphs: int = 0):
        self.handle = rfi_server_create(n_slots, hbm_budget, device, use_graphs, max_graphs)
        self._live = {}

    def now(self) -> float:
        return rfi_server_now(self.handle)

    def submit(self, plan: "Plan", vis, out: dict, arrival: Optional[float] = None, tag: int = 0):
        import torch
        plan._check_tensor("vis", vis, plan.vis_shape, plan.vis_dtype())
        plan._check_tensor("avg", out["avg"], (plan.B, plan.C, 4, 2), torch.float32)
        plan._check_tensor("weight", out["weight"], (plan.B, plan.C), torch.float32)
        plan._check_tensor("flags", out.get("flags"), (plan.B, plan.G, plan.nW), torch.uint8)
        plan._check_tensor("stats", out.get("stats"), (plan.B, plan.G, plan.nW, 3), torch.float32)
        if tag in self._live:
            raise ValueError(f"tag {tag} is already in flight")
        # the server's streams wait on no other stream: finish whatever produced the inputs
        torch.cuda.current_stream(plan.device).synchronize()
        self._live[tag] = (plan, vis, out)
        try:
            rfi_server_submit(self.handle, plan.handle, vis, out["avg"], out["weight"], out.get("flags"),
                              out.get("stats"), self.now() if arrival is None else arrival, tag)
        except Exception:
            del self._live[tag]
            raise

    def poll(self, max_n: int = 256, timeout: float = 0.0):
        done = rfi_server_poll(self.handle, max_n, timeout)
        for c in done:
            self._live.pop(c["tag"], None)
        return done

    def drain(self, timeout: float = 600.0):
        rfi_server_drain(self.handle, timeout)

    def stats(self) -> dict:
        return rfi_server_get_stats(self.handle)

    def close(self):
        if self.handle is not None:
            rfi_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------- hyperparameters

def rfi_sk_null_moments(W: int, d: float):
    m, v, s = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().rfi_sk_null_moments(W, d, ctypes.byref(m), ctypes.byref(v), ctypes.byref(s)))
    return m.value, v.value, s.value


def rfi_thresholds_from_pfa(W: int, d: float, pfa_sk: float = 0.05, pfa_ds: float = 0.05) -> dict:
    lo, hi, g = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
    _check(load_library().rfi_thresholds_from_pfa(W, d, pfa_sk, pfa_ds, ctypes.byref(lo), ctypes.byref(hi),
                                                  ctypes.byref(g)))
    return dict(sk_low=lo.value, sk_high=hi.value, ds_gamma=g.value)


def rfi_calibrate_from_stats(stats, W: int, d_used: float, pfa_sk: float = 0.05, pfa_ds: float = 0.05) -> dict:
    """stats: host float32 array [..., 3] of (tau, r_re, r_im) from RFI-free data."""
    import numpy as np
    a = np.ascontiguousarray(np.asarray(stats, np.float32).reshape(-1, 3))
    d, lo, hi, g = ctypes.c_float(), ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
    _check(load_library().rfi_calibrate_from_stats(a.ctypes.data, a.shape[0], W, d_used, pfa_sk, pfa_ds,
                                                   ctypes.byref(d), ctypes.byref(lo), ctypes.byref(hi),
                                                   ctypes.byref(g)))
    return dict(sk_d=d.value, sk_low=lo.value, sk_high=hi.value, ds_gamma=g.value)


def calibrate_on_null(params: rfi_params, vis, pfa_sk: float = 0.05, pfa_ds: float = 0.05,
                      device: int = 0) -> dict:
    """Screen RFI-free visibilities ``vis`` (device tensor) with ``params`` on the GPU and
    calibrate d and the thresholds from the kernel's statistics (fine-tuning, Section 2.3)."""
    import torch
    plan = Plan(params, device)
    try:
        out = plan.alloc_outputs(flags=False, stats=True)
        plan.screen(vis, out["avg"], out["weight"], None, out["stats"])
        torch.cuda.synchronize()
        st = out["stats"].cpu().numpy()
    finally:
        plan.close()
    return rfi_calibrate_from_stats(st, params.block_m * params.block_f, params.sk_d, pfa_sk, pfa_ds)

"""Python binding of librxgs (ctypes).  Argument marshalling only: every step
of the render and its backward runs in the library's HIP kernels; PyTorch only
provides device memory (tensors) and the current stream.

The library must be built (``python -m paper_2605_24290_amd.build``); there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_int64, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librxgs.so")

MODE_TX = 0
MODE_RX = 1
MLP_NPARAM = 8706
FEAT_DIM = 32
TILE = 16

EXPORT_BIN, EXPORT_KEYS, EXPORT_OPACITY, EXPORT_ORDER, EXPORT_NVIS, EXPORT_PAIRS, \
    EXPORT_RANGES, EXPORT_RADIANCE, EXPORT_TFINAL, EXPORT_NLAST, EXPORT_RECORDS = range(11)

STATUS = {0: "OK", 1: "E_INVALID", 2: "E_OOM", 3: "E_DEVICE", 4: "E_STATE", 5: "E_BUSY",
          6: "E_TIMEOUT", 7: "E_CANCELLED"}


class RxgsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class CGrid(ctypes.Structure):
    _fields_ = [("H", c_int32), ("W", c_int32), ("reserved", c_int32),
                ("el0", c_double), ("del_el", c_double)]


class CGrads(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p),
                ("logits", c_void_p), ("radiance", c_void_p), ("features", c_void_p),
                ("mlp", c_void_p), ("accumulate", c_int32)]


class CSavedInfo(ctypes.Structure):
    _fields_ = [("K", c_int64), ("K_pad", c_int64), ("V", c_int64), ("N", c_int64),
                ("D", c_int64), ("n_visible", c_int64), ("tiles", c_int64), ("tiles_x", c_int64),
                ("n_composited_px", c_int64), ("n_composited", c_int64), ("n_evaluated_px", c_int64),
                ("n_walked_px", c_int64), ("n_sort_fallbacks", c_int64), ("workspace_bytes", c_int64)]


class CServerOpts(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", c_int64), ("max_rx_per_batch", c_int32), ("max_queries_per_batch", c_int32),
                ("slots", c_int32), ("mode", c_int32), ("queue_capacity", c_int32), ("want_spectra", c_int32)]


class CTicketInfo(ctypes.Structure):
    _fields_ = [("t_submit", c_double), ("t_start", c_double), ("t_done", c_double),
                ("batch_queries", c_int32), ("batch_receivers", c_int32), ("attempts", c_int32),
                ("reserved", c_int32)]


class CServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_int64), ("completed", c_int64), ("cancelled", c_int64), ("rejected", c_int64),
                ("failed", c_int64), ("batches", c_int64), ("receivers", c_int64), ("queued", c_int64),
                ("in_flight", c_int64), ("busy_s", c_double), ("failed_batches", c_int64), ("replayed", c_int64),
                ("peak_slot_bytes", c_int64), ("over_estimate", c_int64)]


class CHostExecutor(ctypes.Structure):
    _fields_ = [("K", c_int64), ("H", c_int32), ("W", c_int32), ("delay_us", c_int32), ("reserved", c_int32),
                ("fail_launch_mask", ctypes.c_uint64), ("fail_device_mask", ctypes.c_uint64)]


class CStageTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", c_int64), ("total_ms", c_double)]


class CWorkCounts(ctypes.Structure):
    _fields_ = [("mlp_items", c_int64), ("mlp_pairs", c_int64), ("mlp_slots", c_int64)]


class CRxCondDesc(ctypes.Structure):
    _fields_ = [("basis", c_int32), ("lmax", c_int32), ("channels", c_int32), ("bands", c_int32),
                ("hidden", c_int32), ("probes", c_int32), ("grid", c_int32), ("reserved", c_int32)]


BASIS_FLE = 0
BASIS_SH = 1
RXCOND_OCCUPANCY = 0
RXCOND_BOX = 1
RXCOND_HIDDEN = 64

ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_int, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, ctypes.c_size_t, c_int, c_void_p)

EXPORTED = ("rxgs_create", "rxgs_create_with_allocator", "rxgs_destroy", "rxgs_last_error", "rxgs_scene_upload", "rxgs_mlp_upload",
            "rxgs_saved_create", "rxgs_saved_destroy", "rxgs_render", "rxgs_render_backward",
            "rxgs_saved_info", "rxgs_saved_export", "rxgs_version", "rxgs_profile_enable",
            "rxgs_profile_read", "rxgs_profile_counts", "rxgs_server_start", "rxgs_server_submit", "rxgs_server_poll",
            "rxgs_server_cancel", "rxgs_server_stats", "rxgs_server_stop", "rxgs_plan_batch",
            "rxgs_workspace_estimate", "rxgs_set_near_cut", "rxgs_views_redone", "rxgs_render_chunked",
            "rxgs_view_flags", "rxgs_rxcond_param_count", "rxgs_rxcond_upload", "rxgs_render_rxcond",
            "rxgs_rxcond_export", "rxgs_render_noalloc", "rxgs_server_start_host", "rxgs_set_deterministic")

_lib = None


def lib():
    """Load librxgs.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2605_24290_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    L.rxgs_create.argtypes = [c_int, POINTER(CGrid), POINTER(vp)]
    L.rxgs_create_with_allocator.argtypes = [c_int, POINTER(CGrid), ALLOC_FN, FREE_FN, vp, POINTER(vp)]
    L.rxgs_create_with_allocator.restype = c_int
    L.rxgs_destroy.argtypes = [vp]
    L.rxgs_destroy.restype = None
    L.rxgs_last_error.argtypes = [vp]
    L.rxgs_last_error.restype = ctypes.c_char_p
    L.rxgs_version.restype = ctypes.c_char_p
    L.rxgs_scene_upload.argtypes = [vp, c_int64, vp, vp, vp, vp, vp, vp, c_int, vp]
    L.rxgs_mlp_upload.argtypes = [vp, vp, c_int, vp]
    L.rxgs_saved_create.argtypes = [vp, POINTER(vp)]
    L.rxgs_saved_destroy.argtypes = [vp]
    L.rxgs_saved_destroy.restype = None
    L.rxgs_render.argtypes = [vp, c_int, c_int, vp, POINTER(c_int32), c_int, vp, vp, vp, vp, vp, vp, vp]
    if hasattr(L, "rxgs_render_backward"):
        L.rxgs_render_backward.argtypes = [vp, vp, vp, vp, vp, vp, POINTER(CGrads), vp]
    L.rxgs_saved_info.argtypes = [vp, POINTER(CSavedInfo)]
    L.rxgs_saved_export.argtypes = [vp, c_int, vp, c_int64, c_int]
    L.rxgs_server_start.argtypes = [vp, POINTER(CServerOpts), POINTER(vp)]
    L.rxgs_server_start_host.argtypes = [POINTER(CServerOpts), POINTER(CHostExecutor), POINTER(vp)]
    L.rxgs_server_start_host.restype = c_int
    L.rxgs_server_submit.argtypes = [vp, vp, c_int32, vp, POINTER(ctypes.c_uint64)]
    L.rxgs_server_poll.argtypes = [vp, ctypes.c_uint64, vp, vp, POINTER(CTicketInfo), c_int32]
    L.rxgs_server_cancel.argtypes = [vp, ctypes.c_uint64]
    L.rxgs_server_stats.argtypes = [vp, POINTER(CServerStats)]
    L.rxgs_server_stop.argtypes = [vp]
    L.rxgs_plan_batch.argtypes = [POINTER(c_int32), c_int32, c_int32, c_int64, c_int32, c_int32, c_int64, c_int32,
                                  c_int32, POINTER(c_int64)]
    L.rxgs_plan_batch.restype = c_int32
    L.rxgs_workspace_estimate.argtypes = [c_int32, c_int32, c_int32, c_int64, c_int32, c_int32]
    L.rxgs_workspace_estimate.restype = c_int64
    for name in ("rxgs_server_start", "rxgs_server_submit", "rxgs_server_poll", "rxgs_server_cancel",
                 "rxgs_server_stats", "rxgs_server_stop"):
        getattr(L, name).restype = c_int
    L.rxgs_render_chunked.argtypes = [vp, c_int, c_int, vp, POINTER(c_int32), c_int, vp, vp, vp, vp, vp, c_int64,
                                      POINTER(c_int32), vp]
    L.rxgs_render_chunked.restype = c_int
    L.rxgs_view_flags.argtypes = [vp, vp, c_int32, POINTER(c_int32)]
    L.rxgs_view_flags.restype = c_int
    L.rxgs_set_deterministic.argtypes = [vp, c_int]
    L.rxgs_set_deterministic.restype = c_int
    L.rxgs_set_near_cut.argtypes = [vp, c_int]
    L.rxgs_set_near_cut.restype = c_int
    L.rxgs_views_redone.argtypes = [vp]
    L.rxgs_views_redone.restype = c_int64
    L.rxgs_render_noalloc.argtypes = [vp, c_int, c_int, vp, POINTER(c_int32), c_int, vp, vp, vp, vp, vp, vp]
    L.rxgs_render_noalloc.restype = c_int
    L.rxgs_rxcond_param_count.argtypes = [POINTER(CRxCondDesc)]
    L.rxgs_rxcond_param_count.restype = c_int64
    L.rxgs_rxcond_upload.argtypes = [vp, POINTER(CRxCondDesc), vp, vp, c_int, vp]
    L.rxgs_rxcond_upload.restype = c_int
    L.rxgs_render_rxcond.argtypes = [vp, c_int, c_int, vp, POINTER(c_int32), c_int, vp, vp, vp, vp, vp, vp, vp]
    L.rxgs_render_rxcond.restype = c_int
    L.rxgs_rxcond_export.argtypes = [vp, c_int, vp, c_int64, c_int]
    L.rxgs_rxcond_export.restype = c_int
    L.rxgs_profile_enable.argtypes = [vp, c_int]
    L.rxgs_profile_read.argtypes = [vp, POINTER(CStageTime), c_int, POINTER(c_int), c_int]
    L.rxgs_profile_counts.argtypes = [vp, POINTER(CWorkCounts), c_int, vp]
    L.rxgs_profile_counts.restype = c_int
    for name in ("rxgs_create", "rxgs_scene_upload", "rxgs_mlp_upload", "rxgs_saved_create", "rxgs_render",
                 "rxgs_saved_info", "rxgs_saved_export", "rxgs_profile_enable", "rxgs_profile_read"):
        getattr(L, name).restype = c_int
    if hasattr(L, "rxgs_render_backward"):
        L.rxgs_render_backward.restype = c_int
    _lib = L
    return L


def _torch():
    import torch
    return torch


def _check(status: int, ctx=None):
    if status != 0:
        msg = lib().rxgs_last_error(ctx)
        raise RxgsError(status, msg.decode() if msg else "")


def _dev_f32(t, device):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t, dtype=np.float32))
    return t.to(device=device, dtype=torch.float32).contiguous()


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


class Saved:
    """Forward state kept for the backward pass (rxgs_saved)."""

    def __init__(self, renderer: "Renderer"):
        self.renderer = renderer
        h = c_void_p()
        _check(lib().rxgs_saved_create(renderer._ctx, byref(h)), renderer._ctx)
        self._h = h

    def info(self) -> dict:
        i = CSavedInfo()
        _check(lib().rxgs_saved_info(self._h, byref(i)), self.renderer._ctx)
        return {f: getattr(i, f) for f, _ in CSavedInfo._fields_}

    def export(self, what: int, dtype, shape) -> np.ndarray:
        out = np.zeros(shape, dtype=dtype)
        if out.size:
            _check(lib().rxgs_saved_export(self._h, what, out.ctypes.data_as(c_void_p), out.nbytes, 0),
                   self.renderer._ctx)
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self.renderer._ctx is not None:
            lib().rxgs_saved_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TorchAllocator:
    """Device memory for a context from PyTorch's caching allocator (the
    allocator callbacks of rxgs_create_with_allocator).  Counts what passes
    through it."""

    def __init__(self):
        self.live = {}          # pointer -> bytes
        self.fail_next = 0      # test hook: this many coming allocations return NULL
        self.n_failed = 0
        self.n_alloc = 0
        self.bytes_alloc = 0
        self.n_free = 0
        self._cb = (ALLOC_FN(self._alloc), FREE_FN(self._free))

    @property
    def live_bytes(self) -> int:
        return sum(self.live.values())

    def _alloc(self, nbytes, device, user):
        if self.fail_next > 0:
            self.fail_next -= 1
            self.n_failed += 1
            return None
        try:
            p = _torch().cuda.caching_allocator_alloc(int(nbytes), int(device))
        except Exception:
            return None
        self.live[int(p)] = int(nbytes)
        self.n_alloc += 1
        self.bytes_alloc += int(nbytes)
        return int(p)

    def _free(self, ptr, nbytes, device, user):
        if ptr is None:
            return
        self.live.pop(int(ptr), None)
        self.n_free += 1
        _torch().cuda.caching_allocator_delete(int(ptr))


class Renderer:
    """One librxgs context on a device, for one angular grid.  allocator: None
    (hipMalloc) or a TorchAllocator (device buffers from PyTorch's caching
    allocator)."""

    def __init__(self, grid, device: int = 0, allocator: TorchAllocator | None = None):
        torch = _torch()
        self.device = torch.device("cuda", device)
        self.grid = grid
        self._cgrid = CGrid(int(grid.H), int(grid.W), 0, float(grid.el0), float(grid.del_el))
        ctx = c_void_p()
        self.allocator = allocator
        if allocator is None:
            _check(lib().rxgs_create(device, byref(self._cgrid), byref(ctx)), None)
        else:
            _check(lib().rxgs_create_with_allocator(device, byref(self._cgrid), allocator._cb[0], allocator._cb[1],
                                                    None, byref(ctx)), None)
        self._ctx = ctx
        self.K = 0
        self.use_mlp = False

    def _stream(self):
        return c_void_p(_torch().cuda.current_stream(self.device).cuda_stream)

    def upload_scene(self, means, log_scales, quats, logits, radiance=None, features=None):
        self._autograd_scene = None   # the autograd wrapper's record of what is resident
        ts = [_dev_f32(x, self.device) for x in (means, log_scales, quats, logits, radiance, features)]
        K = int(ts[0].shape[0])
        self._scene_keep = ts
        _check(lib().rxgs_scene_upload(self._ctx, K, *[_ptr(t) for t in ts], 1, self._stream()), self._ctx)
        self.K = K
        self.use_mlp = features is not None

    def upload_mlp(self, params):
        self._autograd_mlp = None
        if isinstance(params, (list, tuple)):
            params = np.concatenate([np.asarray(p, dtype=np.float32).ravel() for p in params])
        t = _dev_f32(params, self.device).reshape(-1)
        if t.numel() != MLP_NPARAM:
            raise ValueError(f"MLP needs {MLP_NPARAM} parameters")
        _check(lib().rxgs_mlp_upload(self._ctx, _ptr(t), 1, self._stream()), self._ctx)

    def render(self, rx, tx=None, rx_off=None, mode: str = "tx", saved: Saved | None = None,
               want_csum: bool = False, out=None, want_amp: bool = False):
        """Render receivers rx (N x 3).  Returns (C (N,2,H,W), power (N), csum or None), or with
        want_amp=True (C, power, csum or None, amplitude (N,H,W))."""
        torch = _torch()
        rx_t = _dev_f32(rx, self.device).reshape(-1, 3)
        N = int(rx_t.shape[0])
        m = MODE_TX if mode == "tx" else MODE_RX
        if mode not in ("tx", "rx"):
            raise ValueError("mode must be 'tx' or 'rx'")
        tx_t = None
        Q = 0
        off_arr = None
        if m == MODE_TX:
            tx_t = _dev_f32(tx, self.device).reshape(-1, 3)
            Q = int(tx_t.shape[0])
            if rx_off is None:
                if Q != 1:
                    raise ValueError("rx_off is needed with several transmitters")
                rx_off = [0, N]
            off_arr = (c_int32 * (Q + 1))(*[int(x) for x in rx_off])
        H, W = self.grid.H, self.grid.W
        if out is None:
            C = torch.empty((N, 2, H, W), device=self.device, dtype=torch.float32)
            P = torch.empty((N,), device=self.device, dtype=torch.float32)
        else:
            C, P = out
        S = torch.empty((N, 2), device=self.device, dtype=torch.float32) if want_csum else None
        A = torch.empty((N, H, W), device=self.device, dtype=torch.float32) if want_amp else None
        _check(lib().rxgs_render(self._ctx, m, Q, _ptr(tx_t), off_arr, N, _ptr(rx_t), _ptr(C), _ptr(P), _ptr(S),
                                 _ptr(A), None if saved is None else saved._h, self._stream()), self._ctx)
        if want_amp:
            return C, P, S, A
        return C, P, S

    def upload_rxcond(self, model):
        """Upload the paper's conditioning model (rxgs_rxcond_upload): model has kind
        (BASIS_FLE / BASIS_SH), lmax, C, F, H, S, G, coeffs (K, L, C, 2) and params (flat)."""
        self.rxc_desc = CRxCondDesc(int(model.kind), int(model.lmax), int(model.C), int(model.F), int(model.H),
                                    int(model.S), int(model.G), 0)
        n = lib().rxgs_rxcond_param_count(byref(self.rxc_desc))
        if n < 0:
            raise ValueError("invalid conditioning descriptor")
        co = _dev_f32(model.coeffs, self.device).reshape(-1)
        pa = _dev_f32(model.params, self.device).reshape(-1)
        if pa.numel() != n:
            raise ValueError(f"the conditioning model needs {n} parameters, got {pa.numel()}")
        if co.numel() != self.K * (int(model.lmax) + 1) ** 2 * int(model.C) * 2:
            raise ValueError("coefficients must be K x L x C x 2")
        self._rxc_keep = (co, pa)
        _check(lib().rxgs_rxcond_upload(self._ctx, byref(self.rxc_desc), _ptr(co), _ptr(pa), 1, self._stream()),
               self._ctx)
        self.rxc_C = int(model.C)

    def render_rxcond(self, rx, tx=None, rx_off=None, mode: str = "tx", saved: Saved | None = None,
                      want_csum: bool = False, want_amp: bool = False):
        """Render with the conditioned radiance (rxgs_render_rxcond): (C (N, Ch, 2, H, W),
        power (N, Ch), csum (N, Ch, 2) or None, amplitude (N, Ch, H, W) or None)."""
        torch = _torch()
        rx_t = _dev_f32(rx, self.device).reshape(-1, 3)
        N = int(rx_t.shape[0])
        if mode not in ("tx", "rx"):
            raise ValueError("mode must be 'tx' or 'rx'")
        m = MODE_TX if mode == "tx" else MODE_RX
        tx_t, Q, off_arr = None, 0, None
        if m == MODE_TX:
            tx_t = _dev_f32(tx, self.device).reshape(-1, 3)
            Q = int(tx_t.shape[0])
            if rx_off is None:
                if Q != 1:
                    raise ValueError("rx_off is needed with several transmitters")
                rx_off = [0, N]
            off_arr = (c_int32 * (Q + 1))(*[int(x) for x in rx_off])
        H, W, Ch = self.grid.H, self.grid.W, self.rxc_C
        dev = self.device
        C = torch.empty((N, Ch, 2, H, W), device=dev, dtype=torch.float32)
        P = torch.empty((N, Ch), device=dev, dtype=torch.float32)
        S = torch.empty((N, Ch, 2), device=dev, dtype=torch.float32) if want_csum else None
        A = torch.empty((N, Ch, H, W), device=dev, dtype=torch.float32) if want_amp else None
        _check(lib().rxgs_render_rxcond(self._ctx, m, Q, _ptr(tx_t), off_arr, N, _ptr(rx_t), _ptr(C), _ptr(P),
                                        _ptr(S), _ptr(A), None if saved is None else saved._h, self._stream()),
               self._ctx)
        return C, P, S, A

    def rxcond_export(self, what: int):
        """Occupancy grid (G, G, G) f32 indexed [z, y, x], or the grid box (lo (3,), hi (3,))."""
        if what == RXCOND_BOX:
            out = np.zeros(6, dtype=np.float64)
            _check(lib().rxgs_rxcond_export(self._ctx, what, out.ctypes.data_as(c_void_p), out.nbytes, 0), self._ctx)
            return out[:3].copy(), out[3:].copy()
        G = int(self.rxc_desc.grid)
        out = np.zeros((G, G, G), dtype=np.float32)
        _check(lib().rxgs_rxcond_export(self._ctx, what, out.ctypes.data_as(c_void_p), out.nbytes, 0), self._ctx)
        return out

    def render_chunked(self, rx, tx=None, rx_off=None, mode: str = "tx", budget_bytes: int = 0, out=None):
        """Coverage map: the receivers streamed through chunks whose workspace fits
        budget_bytes (0: half the free device memory).  Returns (C, power, chunks)."""
        torch = _torch()
        rx_t = _dev_f32(rx, self.device).reshape(-1, 3)
        N = int(rx_t.shape[0])
        if mode not in ("tx", "rx"):
            raise ValueError("mode must be 'tx' or 'rx'")
        m = MODE_TX if mode == "tx" else MODE_RX
        tx_t, Q, off_arr = None, 0, None
        if m == MODE_TX:
            tx_t = _dev_f32(tx, self.device).reshape(-1, 3)
            Q = int(tx_t.shape[0])
            if rx_off is None:
                if Q != 1:
                    raise ValueError("rx_off is needed with several transmitters")
                rx_off = [0, N]
            off_arr = (c_int32 * (Q + 1))(*[int(x) for x in rx_off])
        H, W = self.grid.H, self.grid.W
        if out is None:
            C = torch.empty((N, 2, H, W), device=self.device, dtype=torch.float32)
            P = torch.empty((N,), device=self.device, dtype=torch.float32)
        else:
            C, P = out
        nch = c_int32(0)
        _check(lib().rxgs_render_chunked(self._ctx, m, Q, _ptr(tx_t), off_arr, N, _ptr(rx_t), _ptr(C), _ptr(P), None,
                                         None, int(budget_bytes), byref(nch), self._stream()), self._ctx)
        return C, P, int(nch.value)

    def backward(self, saved: Saved, C, dC, dP=None, grads: dict | None = None, dA=None,
                 accumulate: bool = False) -> dict:
        """Gradients w.r.t. the scene (and MLP) given dL/dC (or None), dL/dpower and dL/damplitude.
        With accumulate=True the gradients are added into the given `grads` tensors."""
        torch = _torch()
        K = self.K
        dev = self.device
        if grads is None:
            grads = dict(means=torch.empty((K, 3), device=dev), log_scales=torch.empty((K, 3), device=dev),
                         quats=torch.empty((K, 4), device=dev), logits=torch.empty((K,), device=dev))
            if self.use_mlp:
                grads["features"] = torch.empty((K, FEAT_DIM), device=dev)
                grads["mlp"] = torch.empty((MLP_NPARAM,), device=dev)
            else:
                grads["radiance"] = torch.empty((K, 2), device=dev)
        if accumulate and not grads:
            raise ValueError("accumulate needs the gradient tensors to add into")
        cg = CGrads(*[None if grads.get(f) is None else grads[f].data_ptr() for f, _ in CGrads._fields_[:-1]],
                    1 if accumulate else 0)
        dC_t = None if dC is None else dC.contiguous()
        dP_t = None if dP is None else _dev_f32(dP, dev)
        dA_t = None if dA is None else _dev_f32(dA, dev)
        _check(lib().rxgs_render_backward(self._ctx, saved._h, _ptr(C.contiguous()), _ptr(dC_t), _ptr(dP_t),
                                          _ptr(dA_t), byref(cg), self._stream()), self._ctx)
        return grads

    def deterministic(self, on: bool = True):
        """Fixed-order backward sums (rxgs_set_deterministic): bitwise-repeatable gradients."""
        _check(lib().rxgs_set_deterministic(self._ctx, 1 if on else 0), self._ctx)

    def near_cut(self, on: bool = True):
        """Nearest-first emission with the exact fallback (rxgs_set_near_cut; off by default)."""
        _check(lib().rxgs_set_near_cut(self._ctx, 1 if on else 0), self._ctx)

    def view_flags(self) -> np.ndarray:
        """Per-view flags of the last render without saved state (rxgs_view_flags)."""
        n = c_int32(0)
        _check(lib().rxgs_view_flags(self._ctx, None, 0, byref(n)), self._ctx)
        out = np.zeros(max(n.value, 1), dtype=np.uint32)
        _check(lib().rxgs_view_flags(self._ctx, out.ctypes.data, n.value, None), self._ctx)
        return out[:n.value]

    def views_redone(self) -> int:
        """Views redone over all their entries since creation (rxgs_views_redone)."""
        return int(lib().rxgs_views_redone(self._ctx))

    def profile(self, on: bool = True):
        """Turn per-stage event timing on or off."""
        _check(lib().rxgs_profile_enable(self._ctx, 1 if on else 0), self._ctx)

    def profile_read(self, reset: bool = True) -> dict:
        """{stage: (launches, total_ms)} accumulated since the last reset."""
        buf = (CStageTime * 64)()
        n = c_int(0)
        _check(lib().rxgs_profile_read(self._ctx, buf, 64, byref(n), 1 if reset else 0), self._ctx)
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(min(n.value, 64))}

    def profile_counts(self, reset: bool = True) -> dict:
        """Device-counted MLP work of the profiled renders since the last reset
        (rxgs_profile_counts): items, (receiver, position) pairs, 32-slot pairs."""
        c = CWorkCounts()
        _check(lib().rxgs_profile_counts(self._ctx, byref(c), 1 if reset else 0, self._stream()), self._ctx)
        return {"mlp_items": int(c.mlp_items), "mlp_pairs": int(c.mlp_pairs), "mlp_slots": int(c.mlp_slots)}

    def close(self):
        if getattr(self, "_ctx", None) is not None:
            lib().rxgs_destroy(self._ctx)
        self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server on a Renderer (rxgs_server_*), or, with
    renderer=None and host_executor given, the same scheduler against the
    library's host-only executor (rxgs_server_start_host; no GPU)."""

    def __init__(self, renderer: Renderer | None, mode: str = "tx", max_rx_per_batch: int = 2048,
                 max_queries_per_batch: int = 64, slots: int = 2, queue_capacity: int = 1 << 20,
                 want_spectra: bool = False, mem_budget_bytes: int = 0, host_executor: dict | None = None):
        self.renderer = renderer
        self.want_spectra = want_spectra
        o = CServerOpts(mem_budget_bytes, max_rx_per_batch, max_queries_per_batch, slots,
                        MODE_TX if mode == "tx" else MODE_RX, queue_capacity, 1 if want_spectra else 0)
        h = c_void_p()
        if renderer is None:
            he = host_executor or {}
            ex = CHostExecutor(int(he.get("K", 1000)), int(he.get("H", 90)), int(he.get("W", 360)),
                               int(he.get("delay_us", 200)), 0, int(he.get("fail_launch_mask", 0)),
                               int(he.get("fail_device_mask", 0)))
            st = lib().rxgs_server_start_host(byref(o), byref(ex), byref(h))
            if st != 0:
                raise RxgsError(st, "host-executor server rejected its options")
        else:
            _check(lib().rxgs_server_start(renderer._ctx, byref(o), byref(h)), renderer._ctx)
        self._h = h
        self._n = {}

    def submit(self, tx, rx) -> int:
        tx = np.ascontiguousarray(np.asarray(tx, dtype=np.float32).reshape(3))
        rx = np.ascontiguousarray(np.asarray(rx, dtype=np.float32).reshape(-1, 3))
        t = ctypes.c_uint64()
        st = lib().rxgs_server_submit(self._h, tx.ctypes.data_as(c_void_p), rx.shape[0],
                                      rx.ctypes.data_as(c_void_p), byref(t))
        if st != 0:
            raise RxgsError(st, "submit rejected")
        self._n[t.value] = rx.shape[0]
        return t.value

    def poll(self, ticket: int, timeout_ms: int = -1):
        """(power (n,), spectra (n,2,H,W) or None, info dict); raises RxgsError on timeout/failure."""
        n = self._n[ticket]
        power = np.zeros(n, dtype=np.float32)
        C = None
        if self.want_spectra:
            g = self.renderer.grid
            C = np.zeros((n, 2, g.H, g.W), dtype=np.float32)
        info = CTicketInfo()
        st = lib().rxgs_server_poll(self._h, ticket, power.ctypes.data_as(c_void_p),
                                    None if C is None else C.ctypes.data_as(c_void_p), byref(info), timeout_ms)
        d = {f: getattr(info, f) for f, _ in CTicketInfo._fields_}
        if st != 0:
            if st != 6:
                self._n.pop(ticket, None)
            err = RxgsError(st, f"ticket {ticket}")
            err.info = d
            raise err
        self._n.pop(ticket, None)
        return power, C, d

    def cancel(self, ticket: int) -> int:
        return lib().rxgs_server_cancel(self._h, ticket)

    def stats(self) -> dict:
        s = CServerStats()
        _check(lib().rxgs_server_stats(self._h, byref(s)))
        return {f: getattr(s, f) for f, _ in CServerStats._fields_}

    def stop(self):
        if getattr(self, "_h", None) is not None:
            lib().rxgs_server_stop(self._h)
        self._h = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def plan_batch(n_rx, mode: str, K: int, H: int, W: int, budget: int, max_rx: int, max_queries: int):
    """Host batch planner of the server: (queries taken, workspace bytes)."""
    arr = (c_int32 * max(len(n_rx), 1))(*[int(x) for x in n_rx])
    b = c_int64(0)
    take = lib().rxgs_plan_batch(arr, len(n_rx), MODE_TX if mode == "tx" else MODE_RX, K, H, W, budget, max_rx,
                                 max_queries, byref(b))
    return int(take), int(b.value)


def workspace_estimate(mode: str, Q: int, N: int, K: int, H: int, W: int) -> int:
    return int(lib().rxgs_workspace_estimate(MODE_TX if mode == "tx" else MODE_RX, Q, N, K, H, W))


def grid_from(H: int, W: int, el0: float, del_el: float):
    """Plain grid record with the attributes the Renderer needs."""
    from .scenes import Grid
    return Grid(H, W, el0, del_el)


def version() -> str:
    return lib().rxgs_version().decode()


__all__ = ["Renderer", "Saved", "Server", "TorchAllocator", "RxgsError", "lib", "version", "plan_batch",
           "workspace_estimate",
           "MODE_TX", "MODE_RX", "EXPORTED"]

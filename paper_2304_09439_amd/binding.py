"""ctypes binding of liblocc.so (C-ABI in include/locc.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device buffers are torch tensors on the context's device; the
stream is torch's current stream unless one is given.  If the library is not
built this module raises on first use; there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblocc.so")

OK, ERR_INVALID_ARG, ERR_OOM, ERR_HIP, ERR_NOT_READY, ERR_RANGE, ERR_BUSY, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "OOM", -3: "HIP", -4: "NOT_READY", -5: "RANGE", -6: "BUSY",
                -7: "UNSUPPORTED"}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp8": 2, "fp8_encoder": 3}   # fp8_encoder: e4m3 on encoder layer 2 only

EXPORTS = ("locc_version", "locc_last_error", "locc_create", "locc_destroy", "locc_upload_weights",
           "locc_upload_shapes", "locc_detect", "locc_detect_noalloc", "locc_debug_crop", "locc_debug_forward", "locc_device_errors",
           "locc_profile", "locc_profile_read", "locc_set_schedule", "locc_get_schedule", "locc_autotune",
           "locc_reserve", "locc_detect_device_count", "locc_graph_capture", "locc_graph_launch",
           "locc_graph_destroy", "locc_serve_start", "locc_serve_submit", "locc_serve_submit_many", "locc_serve_poll", "locc_serve_get_stats",
           "locc_serve_stop", "locc_calibrate", "locc_set_activation_amax", "locc_broad_phase",
           "locc_reserve_broad_phase", "locc_step_graph_capture", "locc_voxel_weight_count", "locc_voxel_create",
           "locc_voxel_destroy", "locc_voxel_upload_weights", "locc_voxel_upload_shapes", "locc_voxel_embeddings",
           "locc_voxel_detect", "locc_voxel_device_errors", "locc_pose_gradients", "locc_train_step",
           "locc_get_weights")


class Config(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("enc_h1", ctypes.c_int32), ("enc_h2", ctypes.c_int32),
                ("head_h", ctypes.c_int32), ("pad_m", ctypes.c_double), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("wg_per_cu", ctypes.c_int32), ("claim", ctypes.c_int32), ("dynamic", ctypes.c_int32),
                ("split", ctypes.c_int32), ("crop_unroll", ctypes.c_int32), ("chunks", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]

    def as_dict(self):
        return dict(wg_per_cu=self.wg_per_cu, claim=self.claim, dynamic=bool(self.dynamic), split=bool(self.split),
                    crop_unroll=self.crop_unroll, chunks=self.chunks)


class ServeConfig(ctypes.Structure):
    _fields_ = [("max_objects", ctypes.c_int32), ("max_batch_pairs", ctypes.c_int32),
                ("max_batch_updates", ctypes.c_int32), ("slots", ctypes.c_int32), ("batching", ctypes.c_int32),
                ("max_queued_pairs", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_size_t)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("pairs_done", ctypes.c_int64), ("max_batch_pairs", ctypes.c_int64), ("busy_ms", ctypes.c_double)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class LoccError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"locc {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load liblocc.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2304_09439_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    L.locc_version.restype = ctypes.c_char_p
    L.locc_version.argtypes = []
    L.locc_last_error.restype = ctypes.c_char_p
    L.locc_last_error.argtypes = []
    L.locc_create.restype = ctypes.c_int
    L.locc_create.argtypes = [ctypes.POINTER(Config), ctypes.c_int, ctypes.POINTER(vp)]
    L.locc_destroy.restype = None
    L.locc_destroy.argtypes = [vp]
    L.locc_upload_weights.restype = ctypes.c_int
    L.locc_upload_weights.argtypes = [vp, vp, ctypes.c_size_t]
    L.locc_upload_shapes.restype = ctypes.c_int
    L.locc_upload_shapes.argtypes = [vp, i32, vp, vp]
    L.locc_detect.restype = ctypes.c_int
    L.locc_detect.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp]
    L.locc_detect_noalloc.restype = ctypes.c_int
    L.locc_detect_noalloc.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp]
    L.locc_debug_crop.restype = ctypes.c_int
    L.locc_debug_crop.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp]
    L.locc_debug_forward.restype = ctypes.c_int
    L.locc_debug_forward.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp, vp, vp]
    L.locc_device_errors.restype = ctypes.c_int
    L.locc_device_errors.argtypes = [vp, vp, i64p, ctypes.c_int]
    L.locc_profile.restype = ctypes.c_int
    L.locc_profile.argtypes = [vp, ctypes.c_int]
    L.locc_profile_read.restype = ctypes.c_int
    L.locc_profile_read.argtypes = [vp, ctypes.POINTER(KernelTime), i32, ctypes.POINTER(ctypes.c_int32)]
    L.locc_set_schedule.restype = ctypes.c_int
    L.locc_set_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
    L.locc_get_schedule.restype = ctypes.c_int
    L.locc_get_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
    L.locc_autotune.restype = ctypes.c_int
    L.locc_autotune.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp, ctypes.c_char_p, ctypes.POINTER(Schedule),
                                ctypes.POINTER(ctypes.c_double)]
    L.locc_reserve.restype = ctypes.c_int
    L.locc_reserve.argtypes = [vp, i32]
    L.locc_detect_device_count.restype = ctypes.c_int
    L.locc_detect_device_count.argtypes = [vp, vp, i32, vp, vp, i32, vp, vp, vp]
    L.locc_graph_capture.restype = ctypes.c_int
    L.locc_graph_capture.argtypes = [vp, vp, i32, vp, vp, i32, vp, vp, ctypes.POINTER(vp)]
    L.locc_graph_launch.restype = ctypes.c_int
    L.locc_graph_launch.argtypes = [vp, vp]
    L.locc_graph_destroy.restype = None
    L.locc_graph_destroy.argtypes = [vp]
    L.locc_serve_start.restype = ctypes.c_int
    L.locc_serve_start.argtypes = [vp, ctypes.POINTER(ServeConfig), vp, i32, ctypes.POINTER(vp)]
    L.locc_serve_submit.restype = ctypes.c_int
    L.locc_serve_submit.argtypes = [vp, vp, vp, i32, vp, i32, ctypes.POINTER(ctypes.c_uint64)]
    L.locc_serve_submit_many.restype = ctypes.c_int
    L.locc_serve_submit_many.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int32)]
    L.locc_serve_poll.restype = ctypes.c_int
    L.locc_serve_poll.argtypes = [vp, ctypes.c_uint64, vp, vp, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_double)]
    L.locc_serve_get_stats.restype = ctypes.c_int
    L.locc_serve_get_stats.argtypes = [vp, ctypes.POINTER(ServeStats)]
    L.locc_serve_stop.restype = ctypes.c_int
    L.locc_serve_stop.argtypes = [vp]
    L.locc_calibrate.argtypes = [vp, vp, i32, vp, i32, vp, vp]
    L.locc_calibrate.restype = ctypes.c_int
    L.locc_set_activation_amax.argtypes = [vp, vp]
    L.locc_set_activation_amax.restype = ctypes.c_int
    L.locc_broad_phase.argtypes = [vp, vp, i32, vp, i32, vp, i32, vp, vp]
    L.locc_broad_phase.restype = ctypes.c_int
    L.locc_reserve_broad_phase.argtypes = [vp, i32, i32]
    L.locc_reserve_broad_phase.restype = ctypes.c_int
    L.locc_step_graph_capture.argtypes = [vp, vp, i32, vp, i32, vp, i32, vp, vp, vp, ctypes.POINTER(vp)]
    L.locc_step_graph_capture.restype = ctypes.c_int
    L.locc_train_step.argtypes = [vp, vp, i32, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_float, vp, vp, vp]
    L.locc_train_step.restype = ctypes.c_int
    L.locc_get_weights.argtypes = [vp, ctypes.c_int, vp, ctypes.c_size_t]
    L.locc_get_weights.restype = ctypes.c_int
    L.locc_pose_gradients.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp, vp]
    L.locc_pose_gradients.restype = ctypes.c_int
    L.locc_voxel_weight_count.argtypes = []
    L.locc_voxel_weight_count.restype = ctypes.c_size_t
    L.locc_voxel_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    L.locc_voxel_create.restype = ctypes.c_int
    L.locc_voxel_destroy.argtypes = [vp]
    L.locc_voxel_destroy.restype = None
    L.locc_voxel_upload_weights.argtypes = [vp, vp, ctypes.c_size_t]
    L.locc_voxel_upload_weights.restype = ctypes.c_int
    L.locc_voxel_upload_shapes.argtypes = [vp, i32, vp, vp]
    L.locc_voxel_upload_shapes.restype = ctypes.c_int
    L.locc_voxel_embeddings.argtypes = [vp, vp, vp]
    L.locc_voxel_embeddings.restype = ctypes.c_int
    L.locc_voxel_detect.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp, vp]
    L.locc_voxel_detect.restype = ctypes.c_int
    L.locc_voxel_device_errors.argtypes = [vp, vp, i64p, ctypes.c_int]
    L.locc_voxel_device_errors.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        raise LoccError(status, load().locc_last_error().decode(errors="replace"))


def version() -> str:
    return load().locc_version().decode()


def pack_objects(pos, quat, shape) -> np.ndarray:
    """Objects as float32 [n, 8] rows (px, py, pz, shape-id bits, qw, qx, qy, qz): the locc_object layout."""
    pos = np.asarray(pos, np.float32)
    quat = np.asarray(quat, np.float32)
    n = len(pos)
    out = np.empty((n, 8), np.float32)
    out[:, 0:3] = pos
    out[:, 3] = np.asarray(shape, np.int32).view(np.float32)
    out[:, 4:8] = quat
    return out


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


class Context:
    """One library context: configuration, resident shapes and weights."""

    def __init__(self, K: int, widths, pad: float = 0.01, precision: str = "fp32", device: int = 0):
        L = load()
        h1, h2, hh = widths
        self.cfg = Config(K, h1, h2, hh, pad, PRECISIONS[precision], 0)
        self.K, self.h1, self.h2, self.hh = K, h1, h2, hh
        self.device = device
        h = ctypes.c_void_p()
        _check(L.locc_create(ctypes.byref(self.cfg), device, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().locc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------- uploads
    def upload_shapes(self, offsets, points):
        off = np.ascontiguousarray(offsets, np.int64)
        pts = np.ascontiguousarray(points, np.float32)
        if pts.ndim != 2 or pts.shape[1] != 6:
            raise ValueError("points must be float32 [N, 6]")
        _check(load().locc_upload_shapes(self._h, len(off) - 1, off.ctypes.data, pts.ctypes.data))

    def upload_weights(self, flat):
        w = np.ascontiguousarray(flat, np.float32)
        _check(load().locc_upload_weights(self._h, w.ctypes.data, w.size))

    # ------------------------------------------------------------- device calls
    def _stream(self, stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(int(s.cuda_stream))

    def _check_dev(self, name, t, dtype, shape_tail):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.device.index != self.device:
            raise ValueError(f"{name}: expected a tensor on cuda:{self.device}")
        if t.dtype != dtype or not t.is_contiguous() or tuple(t.shape[1:]) != tuple(shape_tail):
            raise ValueError(f"{name}: expected contiguous {dtype} [n, {', '.join(map(str, shape_tail))}], "
                             f"got {t.dtype} {tuple(t.shape)}")

    def _inputs(self, objs, pairs):
        import torch
        self._check_dev("objs", objs, torch.float32, (8,))
        self._check_dev("pairs", pairs, torch.int32, (2,))
        return objs.shape[0], pairs.shape[0]

    def detect(self, objs, pairs, out=None, counts=None, stream=None, want_counts=True):
        """Contacts [P, 8] float32 and counts [P, 2] int32 (torch, on the device)."""
        import torch
        n_objs, P = self._inputs(objs, pairs)
        dev = objs.device
        if out is None:
            out = torch.empty((P, 8), dtype=torch.float32, device=dev)
        if counts is None and want_counts:
            counts = torch.empty((P, 2), dtype=torch.int32, device=dev)
        _check(load().locc_detect(self._h, _ptr(objs), n_objs, _ptr(pairs), P, _ptr(out), _ptr(counts),
                                  self._stream(stream)))
        return out, counts

    def detect_noalloc(self, objs, pairs, out, counts=None, stream=None):
        """locc_detect_noalloc: the detect path with the library's fixed device array as its workspace.
        The caller provides every output buffer (this call allocates nothing)."""
        import torch
        n_objs, P = self._inputs(objs, pairs)
        self._check_dev("out", out, torch.float32, (8,))
        if out.shape[0] < P:
            raise ValueError(f"out: {out.shape[0]} rows for {P} pairs")
        if counts is not None:
            self._check_dev("counts", counts, torch.int32, (2,))
            if counts.shape[0] < P:
                raise ValueError(f"counts: {counts.shape[0]} rows for {P} pairs")
        _check(load().locc_detect_noalloc(self._h, _ptr(objs), n_objs, _ptr(pairs), P, _ptr(out), _ptr(counts),
                                          self._stream(stream)))
        return out, counts

    def debug_crop(self, objs, pairs, stream=None):
        """Selected indices [P, 2, K] and counts [P, 2] (caller order)."""
        import torch
        n_objs, P = self._inputs(objs, pairs)
        idx = torch.empty((P, 2, self.K), dtype=torch.int32, device=objs.device)
        counts = torch.empty((P, 2), dtype=torch.int32, device=objs.device)
        _check(load().locc_debug_crop(self._h, _ptr(objs), n_objs, _ptr(pairs), P, _ptr(idx), _ptr(counts),
                                      self._stream(stream)))
        return idx, counts

    def debug_forward(self, objs, pairs, stream=None):
        """Contacts, counts, pooled features z [P, 2 h2] and raw head output y [P, 8]."""
        import torch
        n_objs, P = self._inputs(objs, pairs)
        dev = objs.device
        out = torch.empty((P, 8), dtype=torch.float32, device=dev)
        counts = torch.empty((P, 2), dtype=torch.int32, device=dev)
        z = torch.empty((P, 2 * self.h2), dtype=torch.float32, device=dev)
        y = torch.empty((P, 8), dtype=torch.float32, device=dev)
        _check(load().locc_debug_forward(self._h, _ptr(objs), n_objs, _ptr(pairs), P, _ptr(out), _ptr(counts),
                                         _ptr(z), _ptr(y), self._stream(stream)))
        return out, counts, z, y

    def set_schedule(self, wg_per_cu: int = 2, claim: int = 4, dynamic: bool = True, split: bool = True,
                     crop_unroll: int = 8, chunks: int = 1):
        sc = Schedule(wg_per_cu, claim, int(dynamic), int(split), crop_unroll, chunks)
        _check(load().locc_set_schedule(self._h, ctypes.byref(sc)))

    def get_schedule(self) -> dict:
        sc = Schedule()
        _check(load().locc_get_schedule(self._h, ctypes.byref(sc)))
        return sc.as_dict()

    def autotune(self, objs, pairs, cache_path=None, stream=None, want_counts=True):
        """Time every schedule on this workload (with or without member counts), install and return the
        fastest: (schedule dict, ms)."""
        import torch
        n_objs, P = self._inputs(objs, pairs)
        out = torch.empty((P, 8), dtype=torch.float32, device=objs.device)
        counts = torch.empty((P, 2), dtype=torch.int32, device=objs.device) if want_counts else None
        sc = Schedule()
        ms = ctypes.c_double()
        path = None if cache_path is None else str(cache_path).encode()
        _check(load().locc_autotune(self._h, _ptr(objs), n_objs, _ptr(pairs), P, _ptr(out), _ptr(counts),
                                    self._stream(stream), path, ctypes.byref(sc), ctypes.byref(ms)))
        return sc.as_dict(), ms.value

    def calibrate(self, objs, pairs, stream=None):
        """FP8: measure and install the activation maxima on this workload; returns them (3 floats)."""
        n_objs, P = self._inputs(objs, pairs)
        amax = np.zeros(3, np.float32)
        _check(load().locc_calibrate(self._h, _ptr(objs), n_objs, _ptr(pairs), P, self._stream(stream),
                                     amax.ctypes.data))
        return amax

    def set_activation_amax(self, amax):
        """FP8: install activation maxima (layer-1 output, pooled features, head layer-1 output)."""
        a = np.ascontiguousarray(amax, np.float32)
        if a.shape != (3,):
            raise ValueError("amax: expected 3 floats")
        _check(load().locc_set_activation_amax(self._h, a.ctypes.data))

    def reserve(self, max_pairs: int):
        _check(load().locc_reserve(self._h, int(max_pairs)))

    def detect_device_count(self, objs, pairs, n_dev, out, counts=None, stream=None):
        """Detect on the first *n_dev pairs (n_dev: int32 [1] device tensor); pairs/out sized for the capacity."""
        n_objs, cap = self._inputs(objs, pairs)
        _check(load().locc_detect_device_count(self._h, _ptr(objs), n_objs, _ptr(pairs), _ptr(n_dev), cap,
                                               _ptr(out), _ptr(counts), self._stream(stream)))
        return out, counts

    def capture_graph(self, objs, pairs, n_dev, out, counts=None) -> "Graph":
        """Capture one step (device pair count) as a HIP graph over these buffers."""
        n_objs, cap = self._inputs(objs, pairs)
        g = ctypes.c_void_p()
        _check(load().locc_graph_capture(self._h, _ptr(objs), n_objs, _ptr(pairs), _ptr(n_dev), cap, _ptr(out),
                                         _ptr(counts), ctypes.byref(g)))
        return Graph(self, g, (objs, pairs, n_dev, out, counts))

    def pose_gradients(self, objs, pairs, grad=None, out=None, stream=None, want_contacts=False,
                       want_argmax=False):
        """d logit / d (p, q) of both objects, float32 [P, 14] (caller order); optionally the contacts and
        the second object's argmax rows uint8 [P, enc_h2]."""
        import torch
        n_objs, P = self._inputs(objs, pairs)
        if grad is None:
            grad = torch.empty((P, 14), dtype=torch.float32, device=objs.device)
        if out is None and want_contacts:
            out = torch.empty((P, 8), dtype=torch.float32, device=objs.device)
        amax = torch.empty((P, self.cfg.enc_h2), dtype=torch.uint8, device=objs.device) if want_argmax else None
        _check(load().locc_pose_gradients(self._h, _ptr(objs), n_objs, _ptr(pairs), P, _ptr(grad), _ptr(out),
                                          _ptr(amax), self._stream(stream)))
        return (grad, out, amax) if want_argmax else (grad, out)

    def train_step(self, objs, pairs, labels, alpha=0.5, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, loss=None,
                   want_argmax=False, stream=None):
        """One Adam step on a labelled batch (FP32 context).  labels: float32 [P] device tensor.
        Returns the loss terms (float32 [2] device tensor: cross-entropy, alpha x feature norm) and
        optionally the argmax rows uint8 [P, 2, enc_h2]."""
        import torch
        n_objs, P = self._inputs(objs, pairs)
        if loss is None:
            loss = torch.empty(2, dtype=torch.float32, device=objs.device)
        amax = torch.empty((P, 2, self.cfg.enc_h2), dtype=torch.uint8, device=objs.device) if want_argmax else None
        _check(load().locc_train_step(self._h, _ptr(objs), n_objs, _ptr(pairs), _ptr(labels), P, alpha, lr, beta1,
                                      beta2, eps, _ptr(loss), _ptr(amax), self._stream(stream)))
        return (loss, amax) if want_argmax else loss

    def get_weights(self, which: int = 0) -> np.ndarray:
        """The flat FP32 weights (0), the last training gradient (1) or the Adam moments (2, 3), host copy."""
        c = self.cfg
        n = (c.enc_h1 * 6 + c.enc_h1 + c.enc_h2 * c.enc_h1 + c.enc_h2 + c.head_h * 2 * c.enc_h2 + c.head_h
             + c.head_h * c.head_h + c.head_h + 8 * c.head_h + 8)
        out = np.empty(n, np.float32)
        _check(load().locc_get_weights(self._h, int(which), out.ctypes.data, n))
        return out

    def broad_phase(self, objs, env_offsets, pairs, count, stream=None):
        """Overlapping pairs per environment into pairs (int32 [capacity, 2], device) and
        count (int32 [2], device: written, total).  env_offsets: int32 [E + 1], device."""
        import torch
        self._check_dev("objs", objs, torch.float32, (8,))
        self._check_dev("pairs", pairs, torch.int32, (2,))
        self._check_dev("env_offsets", env_offsets, torch.int32, ())
        self._check_dev("count", count, torch.int32, ())
        if count.numel() < 2 or env_offsets.numel() < 1:
            raise ValueError("count needs 2 entries, env_offsets at least 1")
        _check(load().locc_broad_phase(self._h, _ptr(objs), objs.shape[0], _ptr(env_offsets),
                                       env_offsets.numel() - 1, _ptr(pairs), pairs.shape[0], _ptr(count),
                                       self._stream(stream)))
        return pairs, count

    def reserve_broad_phase(self, n_objs: int, n_envs: int):
        _check(load().locc_reserve_broad_phase(self._h, int(n_objs), int(n_envs)))

    def capture_step_graph(self, objs, env_offsets, pairs, count, out, counts=None) -> "Graph":
        """Capture broad phase + detect (device count) as one HIP graph over these buffers."""
        import torch
        self._check_dev("objs", objs, torch.float32, (8,))
        self._check_dev("pairs", pairs, torch.int32, (2,))
        self._check_dev("env_offsets", env_offsets, torch.int32, ())
        self._check_dev("count", count, torch.int32, ())
        if count.numel() < 2 or env_offsets.numel() < 1:
            raise ValueError("count needs 2 entries, env_offsets at least 1")
        g = ctypes.c_void_p()
        _check(load().locc_step_graph_capture(self._h, _ptr(objs), objs.shape[0], _ptr(env_offsets),
                                              env_offsets.numel() - 1, _ptr(pairs), pairs.shape[0], _ptr(count),
                                              _ptr(out), _ptr(counts), ctypes.byref(g)))
        return Graph(self, g, (objs, env_offsets, pairs, count, out, counts))

    def profile(self, enable: bool):
        """Start (clearing totals) or stop per-kernel event timing."""
        _check(load().locc_profile(self._h, int(enable)))

    def profile_read(self) -> dict:
        """{kernel name: (launches, total_ms)} recorded while profiling was on."""
        cap = 32
        buf = (KernelTime * cap)()
        n = ctypes.c_int32()
        _check(load().locc_profile_read(self._h, buf, cap, ctypes.byref(n)))
        return {buf[k].name.decode(): (buf[k].launches, buf[k].total_ms) for k in range(min(n.value, cap))}

    def device_errors(self, reset: bool = False, stream=None) -> int:
        n = ctypes.c_int64()
        _check(load().locc_device_errors(self._h, self._stream(stream), ctypes.byref(n), int(reset)))
        return n.value


class Graph:
    """A captured step; keeps its context and buffers alive."""

    def __init__(self, ctx, handle, buffers):
        self.ctx, self._h, self._buffers = ctx, handle, buffers

    def launch(self, stream=None):
        _check(load().locc_graph_launch(self._h, self.ctx._stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            load().locc_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VoxelContext:
    """The voxel-embedding variant (include/locc_voxel.h): shape embeddings computed on the device at
    upload, then per pair cell selection, mean embeddings and the predictor MLPs."""

    def __init__(self, device: int = 0):
        self.device = device
        h = ctypes.c_void_p()
        _check(load().locc_voxel_create(device, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().locc_voxel_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload_weights(self, flat):
        w = np.ascontiguousarray(flat, np.float32)
        _check(load().locc_voxel_upload_weights(self._h, w.ctypes.data, w.size))

    def upload_shapes(self, offsets, points):
        off = np.ascontiguousarray(offsets, np.int64)
        pts = np.ascontiguousarray(points, np.float32)
        _check(load().locc_voxel_upload_shapes(self._h, len(off) - 1, off.ctypes.data, pts.ctypes.data))
        self.n_shapes = len(off) - 1

    def _stream(self, stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(int(s.cuda_stream))

    def embeddings(self, stream=None):
        """float32 [S, 216, 16] (torch, on the device)."""
        import torch
        out = torch.empty((self.n_shapes, 216, 16), dtype=torch.float32, device=f"cuda:{self.device}")
        _check(load().locc_voxel_embeddings(self._h, _ptr(out), self._stream(stream)))
        return out

    def detect(self, objs, pairs, out=None, counts=None, pooled=None, stream=None, want_counts=True,
               want_pooled=False):
        """(logit, probability) float32 [P, 2], counts int32 [P, 2] and pooled float32 [P, 2, 16]."""
        import torch
        for name, t, dt, tail in (("objs", objs, torch.float32, (8,)), ("pairs", pairs, torch.int32, (2,))):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous() \
                    or tuple(t.shape[1:]) != tail:
                raise ValueError(f"{name}: expected a contiguous {dt} [n, {tail[0]}] tensor on the GPU")
        P = pairs.shape[0]
        dev = objs.device
        if out is None:
            out = torch.empty((P, 2), dtype=torch.float32, device=dev)
        if counts is None and want_counts:
            counts = torch.empty((P, 2), dtype=torch.int32, device=dev)
        if pooled is None and want_pooled:
            pooled = torch.empty((P, 2, 16), dtype=torch.float32, device=dev)
        _check(load().locc_voxel_detect(self._h, _ptr(objs), objs.shape[0], _ptr(pairs), P, _ptr(out), _ptr(counts),
                                        _ptr(pooled), self._stream(stream)))
        return out, counts, pooled

    def device_errors(self, reset: bool = False, stream=None) -> int:
        n = ctypes.c_int64()
        _check(load().locc_voxel_device_errors(self._h, self._stream(stream), ctypes.byref(n), int(reset)))
        return n.value


class Server:
    """Continuous-batching request loop on a context (locc_serve_* in locc.h).

    Host numpy arrays in, host numpy arrays out; the context must not be used
    by other calls until stop().
    """

    def __init__(self, ctx: Context, objects, max_objects=None, batching=True, slots=2, max_batch_pairs=0,
                 max_batch_updates=4096, max_queued_pairs=0, hbm_budget_bytes=1 << 30):
        objs = np.ascontiguousarray(objects, np.float32)
        n = len(objs)
        self.cfg = ServeConfig(max_objects or n, max_batch_pairs, max_batch_updates, slots, int(batching),
                               max_queued_pairs, hbm_budget_bytes)
        h = ctypes.c_void_p()
        _check(load().locc_serve_start(ctx._h, ctypes.byref(self.cfg), objs.ctypes.data, n, ctypes.byref(h)))
        self._h, self.ctx = h, ctx
        self._n_pairs = {}

    def submit(self, upd_ids, upd_objects, pairs) -> int:
        ids = np.ascontiguousarray(upd_ids, np.int32)
        upd = np.ascontiguousarray(upd_objects, np.float32)
        pr = np.ascontiguousarray(pairs, np.int32)
        rid = ctypes.c_uint64()
        _check(load().locc_serve_submit(self._h, ids.ctypes.data, upd.ctypes.data, len(ids), pr.ctypes.data,
                                        len(pr), ctypes.byref(rid)))
        self._n_pairs[rid.value] = len(pr)
        return rid.value

    @staticmethod
    def pack_requests(requests):
        """[(upd_ids, upd_objects, pairs), ...] -> the flat arrays submit_many_arrays takes."""
        n = len(requests)
        uo = np.zeros(n + 1, np.int32)
        po = np.zeros(n + 1, np.int32)
        uo[1:] = np.cumsum([len(r[0]) for r in requests])
        po[1:] = np.cumsum([len(r[2]) for r in requests])
        ids = np.concatenate([np.asarray(r[0], np.int32).reshape(-1) for r in requests] + [np.zeros(0, np.int32)])
        upd = np.concatenate([np.asarray(r[1], np.float32).reshape(-1, 8) for r in requests] +
                             [np.zeros((0, 8), np.float32)])
        pr = np.concatenate([np.asarray(r[2], np.int32).reshape(-1, 2) for r in requests] +
                            [np.zeros((0, 2), np.int32)])
        return tuple(np.ascontiguousarray(a) for a in (uo, ids, upd, po, pr))

    def submit_many_arrays(self, upd_offsets, upd_ids, upd_objects, pair_offsets, pairs):
        """locc_serve_submit_many on flat host arrays (see pack_requests); returns the ids of the requests
        queued (all of them unless one was refused: then the call raises after queueing those before it, and
        the exception carries their ids as .accepted_ids)."""
        n = len(upd_offsets) - 1
        out_ids = np.zeros(max(n, 1), np.uint64)
        acc = ctypes.c_int32()
        st = load().locc_serve_submit_many(self._h, n, upd_offsets.ctypes.data, upd_ids.ctypes.data,
                                           upd_objects.ctypes.data, pair_offsets.ctypes.data, pairs.ctypes.data,
                                           out_ids.ctypes.data, ctypes.byref(acc))
        got = [int(x) for x in out_ids[:acc.value]]
        for k, rid in enumerate(got):
            self._n_pairs[rid] = int(pair_offsets[k + 1] - pair_offsets[k])
        if st != OK:
            try:
                _check(st)
            except LoccError as e:
                e.accepted_ids = got
                raise
        return got

    def submit_many(self, requests):
        """Queues [(upd_ids, upd_objects, pairs), ...] in order with one call (see submit_many_arrays)."""
        return self.submit_many_arrays(*self.pack_requests(requests))

    def poll(self, rid: int):
        """None while running; (contacts [P, 8], counts [P, 2], latency_ms) once done."""
        P = self._n_pairs[rid]
        out = np.empty((P, 8), np.float32)
        counts = np.empty((P, 2), np.int32)
        done = ctypes.c_int32()
        lat = ctypes.c_double()
        _check(load().locc_serve_poll(self._h, rid, out.ctypes.data, counts.ctypes.data, ctypes.byref(done),
                                      ctypes.byref(lat)))
        if not done.value:
            return None
        del self._n_pairs[rid]
        return out, counts, lat.value

    def stats(self) -> dict:
        st = ServeStats()
        _check(load().locc_serve_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServeStats._fields_}

    def stop(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(load().locc_serve_stop(h))

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def context_for_scene(scene, K, widths, weights_flat, pad=0.01, precision="fp32", device=0):
    """Create a context, upload the scene's shape library and the weights."""
    ctx = Context(K, widths, pad, precision, device)
    ctx.upload_shapes(scene.lib.offsets, scene.lib.pts)
    ctx.upload_weights(weights_flat)
    return ctx


def scene_tensors(scene, device=0):
    """(objects [n, 8] float32, pairs [P, 2] int32) of a scene, on the device."""
    import torch
    objs = torch.from_numpy(pack_objects(scene.pos, scene.quat, scene.shape)).to(f"cuda:{device}")
    pairs = torch.from_numpy(np.ascontiguousarray(scene.pairs, np.int32)).to(f"cuda:{device}")
    return objs, pairs

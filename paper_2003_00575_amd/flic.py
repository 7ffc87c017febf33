"""Python binding of libflic.so (ctypes): argument marshalling only.

Every step of the clustering runs in the library's HIP kernels; torch is used
for device memory and streams.  If libflic.so is missing the import of this
module still works, but every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
# FLIC_LIB selects another build of the library (the host-sanitizer test
# loads one whose host code is built with AddressSanitizer / UBSan).
LIB_PATH = os.environ.get("FLIC_LIB") or os.path.join(HERE, "libflic.so")

FLIC_OK = 0
FLIC_EINVAL = -1
FLIC_ENOMEM = -2
FLIC_EHIP = -3
MAX_SKIP = 8


class FlicError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"flic status {status}: {message}")
        self.status = status


class _Tables(ctypes.Structure):
    _fields_ = [("cos_v", ctypes.c_void_p), ("cos_h", ctypes.c_void_p)]


class _Scan(ctypes.Structure):
    _fields_ = [("range_img", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("tables", _Tables), ("threshold", ctypes.c_float),
                ("skip_depth", ctypes.c_int32), ("labels_out", ctypes.c_void_p),
                ("min_points", ctypes.c_int32), ("map_connections", ctypes.c_int32)]


class _GroundTables(ctypes.Structure):
    _fields_ = [("sin_a", ctypes.c_void_p), ("cos_a", ctypes.c_void_p), ("tan_lo", ctypes.c_void_p),
                ("tan_hi", ctypes.c_void_p), ("sin_d", ctypes.c_void_p), ("cos_d", ctypes.c_void_p),
                ("sensor_height", ctypes.c_float), ("tan_theta", ctypes.c_float)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("slots_per_sensor", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("hbm_budget", ctypes.c_uint64), ("sim_launch_s", ctypes.c_double),
                ("stage_kernels", ctypes.c_int32)]


class _FrameRecord(ctypes.Structure):
    _fields_ = [("sensor", ctypes.c_int32), ("batch", ctypes.c_int32), ("tag", ctypes.c_int64),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class _Arrival(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("sensor", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("host_range", ctypes.c_void_p), ("host_labels", ctypes.c_void_p)]


# numpy views of the record and arrival structs (same layout)
RECORD_DTYPE = [("sensor", "<i4"), ("batch", "<i4"), ("tag", "<i8"), ("t_arrival", "<f8"),
                ("t_admit", "<f8"), ("t_launch", "<f8"), ("t_done", "<f8")]
ARRIVAL_DTYPE = [("t", "<f8"), ("sensor", "<i4"), ("pad_", "<i4"), ("host_range", "<u8"),
                 ("host_labels", "<u8")]

_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """Load libflic.so (torch first, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(
            f"{LIB_PATH} is not built; run `python -m paper_2003_00575_amd.build`")
    import torch  # noqa: F401  -- loads the HIP runtime the tensors live in
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
    L.flic_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_size_t]
    L.flic_ctx_create.restype = i32
    L.flic_ctx_destroy.argtypes = [vp]
    L.flic_ctx_destroy.restype = None
    L.flic_ground_remove.argtypes = [vp, vp, i32, i32, i32, ctypes.POINTER(_GroundTables), vp, vp, vp]
    L.flic_ground_remove.restype = i32
    L.flic_cluster.argtypes = [vp, i32, i32, ctypes.POINTER(_Tables), f32, i32, vp]
    L.flic_cluster.restype = i32
    L.flic_cluster_async.argtypes = [vp, vp, i32, i32, ctypes.POINTER(_Tables), f32, i32, vp, vp]
    L.flic_cluster_async.restype = i32
    L.flic_cluster_noalloc.argtypes = [vp, i32, i32, ctypes.POINTER(_Tables), f32, i32, vp, vp]
    L.flic_cluster_noalloc.restype = i32
    L.flic_cluster_batched.argtypes = [vp, ctypes.POINTER(_Scan), i32, vp]
    L.flic_cluster_batched.restype = i32
    L.flic_cluster_batched_host.argtypes = [vp, ctypes.POINTER(_Scan), i32, ctypes.POINTER(vp),
                                            ctypes.POINTER(vp), vp]
    L.flic_cluster_batched_host.restype = i32
    L.flic_plan_create.argtypes = [vp, ctypes.POINTER(_Scan), i32, ctypes.POINTER(vp)]
    L.flic_plan_create.restype = i32
    L.flic_plan_launch.argtypes = [vp, ctypes.POINTER(_Scan), i32, vp]
    L.flic_plan_launch.restype = i32
    L.flic_plan_destroy.argtypes = [vp]
    L.flic_plan_destroy.restype = None
    L.flic_set_tile_override.argtypes = [vp, i32]
    L.flic_set_tile_override.restype = i32
    L.flic_ctx_set_tile_rule.argtypes = [vp, i32, i32, i32, i32]
    L.flic_ctx_set_tile_rule.restype = i32
    L.flic_ctx_set_plan_parts.argtypes = [vp, i32]
    L.flic_ctx_set_plan_parts.restype = i32
    L.flic_ctx_tile_for.argtypes = [vp, i32, i32, i32, ctypes.POINTER(i32)]
    L.flic_ctx_tile_for.restype = i32
    L.flic_batch_bytes.argtypes = [vp, ctypes.POINTER(_Scan), i32, ctypes.POINTER(ctypes.c_size_t),
                                   ctypes.POINTER(ctypes.c_size_t)]
    L.flic_batch_bytes.restype = i32
    L.flic_ctx_reserve.argtypes = [vp, ctypes.c_size_t, ctypes.c_size_t]
    L.flic_ctx_reserve.restype = i32
    L.flic_ctx_bytes_in_use.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.flic_ctx_bytes_in_use.restype = i32
    L.flic_ctx_set_pass_timing.argtypes = [vp, i32]
    L.flic_ctx_set_pass_timing.restype = i32
    L.flic_ctx_pass_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i32)]
    L.flic_ctx_pass_times.restype = i32
    L.flic_last_error.argtypes = []
    L.flic_last_error.restype = ctypes.c_char_p
    L.flic_server_create.argtypes = [vp, ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)]
    L.flic_server_create.restype = i32
    L.flic_server_add_sensor.argtypes = [vp, i32, i32, ctypes.POINTER(_Tables), f32, i32, ctypes.POINTER(i32)]
    L.flic_server_add_sensor.restype = i32
    L.flic_server_submit.argtypes = [vp, ctypes.c_double, ctypes.c_double, i32, vp, vp, ctypes.c_int64]
    L.flic_server_submit.restype = i32
    L.flic_server_progress.argtypes = [vp, ctypes.c_double, ctypes.POINTER(i32)]
    L.flic_server_progress.restype = i32
    L.flic_server_replay.argtypes = [vp, vp, i32]
    L.flic_server_replay.restype = i32
    L.flic_server_now.argtypes = [vp]
    L.flic_server_now.restype = ctypes.c_double
    L.flic_server_records.argtypes = [vp, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.flic_server_records.restype = i32
    L.flic_server_clear.argtypes = [vp]
    L.flic_server_clear.restype = i32
    L.flic_server_destroy.argtypes = [vp]
    L.flic_server_destroy.restype = None
    _lib = L
    return L


def _check(status: int) -> None:
    if status != FLIC_OK:
        msg = lib().flic_last_error().decode(errors="replace")
        raise FlicError(status, msg)


def last_error() -> str:
    return lib().flic_last_error().decode(errors="replace")


# ---------------------------------------------------------------------------
# Raw pointer level (ints are device addresses)
# ---------------------------------------------------------------------------

def cluster_raw(range_ptr: int, H: int, W: int, cos_v_ptr: int, cos_h_ptr: int,
                threshold: float, skip_depth: int, labels_ptr: int) -> int:
    """flic_cluster with raw device addresses; returns the status code."""
    t = _Tables(cos_v_ptr, cos_h_ptr)
    return lib().flic_cluster(range_ptr, H, W, ctypes.byref(t), threshold, skip_depth, labels_ptr)


def cluster_async_raw(ctx: int, range_ptr: int, H: int, W: int, cos_v_ptr: int, cos_h_ptr: int,
                      threshold: float, skip_depth: int, labels_ptr: int, stream: int) -> int:
    t = _Tables(cos_v_ptr, cos_h_ptr)
    return lib().flic_cluster_async(ctx, range_ptr, H, W, ctypes.byref(t), threshold,
                                    skip_depth, labels_ptr, stream)


def cluster_noalloc_raw(range_ptr: int, H: int, W: int, cos_v_ptr: int, cos_h_ptr: int,
                        threshold: float, skip_depth: int, labels_ptr: int, stream: int) -> int:
    """flic_cluster_noalloc with raw device addresses; returns the status code."""
    t = _Tables(cos_v_ptr, cos_h_ptr)
    return lib().flic_cluster_noalloc(range_ptr, H, W, ctypes.byref(t), threshold, skip_depth,
                                      labels_ptr, stream)


def batched_raw(ctx: int, scans: Sequence[tuple], stream: int) -> int:
    """scans: (range_ptr, H, W, cos_v_ptr, cos_h_ptr, threshold, N, labels_ptr
    [, min_points])."""
    arr = (_Scan * max(1, len(scans)))()
    for i, sc in enumerate(scans):
        rp, H, W, cv, ch, T, N, lp = sc[:8]
        arr[i] = _Scan(rp, H, W, _Tables(cv, ch), T, N, lp, sc[8] if len(sc) > 8 else 0)
    return lib().flic_cluster_batched(ctx, arr, len(scans), stream)


# ---------------------------------------------------------------------------
# torch level
# ---------------------------------------------------------------------------

def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _check_tensor(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


@dataclasses.dataclass
class DeviceScan:
    """Device tensors of one scan: range [H, W] f32, cos_v [N, H] f32,
    cos_h [N, W] f32, labels [H, W] int32 (output); min_points > 0 applies
    the cluster-size threshold."""
    range_img: "object"
    cos_v: "object"
    cos_h: "object"
    threshold: float
    skip_depth: int
    labels: "object" = None
    min_points: int = 0
    map_connections: int = 0

    def validate(self) -> None:
        import torch
        H, W = self.range_img.shape
        N = self.skip_depth
        _check_tensor(self.range_img, torch.float32, (H, W), "range_img")
        _check_tensor(self.cos_v, torch.float32, (N, H), "cos_v")
        _check_tensor(self.cos_h, torch.float32, (N, W), "cos_h")
        if self.labels is None:
            self.labels = torch.empty((H, W), dtype=torch.int32, device=self.range_img.device)
        _check_tensor(self.labels, torch.int32, (H, W), "labels")

    def to_c(self) -> _Scan:
        H, W = self.range_img.shape
        return _Scan(self.range_img.data_ptr(), H, W,
                     _Tables(self.cos_v.data_ptr(), self.cos_h.data_ptr()),
                     float(self.threshold), int(self.skip_depth), self.labels.data_ptr(),
                     int(self.min_points), int(self.map_connections))


class Context:
    """A flic_ctx on one device (one host thread at a time)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        _check(lib().flic_ctx_create(ctypes.byref(h), int(device), int(hbm_budget_bytes)))
        self.handle = h
        self.device = device

    def close(self) -> None:
        if self.handle:
            lib().flic_ctx_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile_width(self, tile_w: int) -> None:
        """0 restores the built-in choice."""
        _check(lib().flic_set_tile_override(self.handle, int(tile_w)))

    def set_tile_rule(self, H: int, W: int, skip_depth: int, tile_w: int) -> None:
        """Use tile_w columns per tile for scans of exactly this shape (0 removes)."""
        _check(lib().flic_ctx_set_tile_rule(self.handle, int(H), int(W), int(skip_depth), int(tile_w)))

    def set_plan_parts(self, parts: int) -> None:
        """Plans created afterwards split each launch group into up to
        `parts` parallel graph branches (1 = one sequence per group)."""
        _check(lib().flic_ctx_set_plan_parts(self.handle, int(parts)))

    def tile_for(self, H: int, W: int, skip_depth: int) -> int:
        out = ctypes.c_int32()
        _check(lib().flic_ctx_tile_for(self.handle, int(H), int(W), int(skip_depth), ctypes.byref(out)))
        return int(out.value)

    def batch_bytes(self, structs: Sequence[_Scan]):
        """(descriptor bytes, scratch bytes) a batched launch of these scans needs."""
        arr = (_Scan * max(1, len(structs)))(*structs)
        db, sb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().flic_batch_bytes(self.handle, arr, len(structs), ctypes.byref(db), ctypes.byref(sb)))
        return int(db.value), int(sb.value)

    def reserve(self, desc_bytes: int, scratch_bytes: int) -> None:
        """Pre-size every launch slot (no allocation during later launches)."""
        _check(lib().flic_ctx_reserve(self.handle, int(desc_bytes), int(scratch_bytes)))

    def bytes_in_use(self) -> int:
        out = ctypes.c_size_t()
        _check(lib().flic_ctx_bytes_in_use(self.handle, ctypes.byref(out)))
        return int(out.value)

    def cluster_batched_structs(self, structs: Sequence[_Scan], stream=None) -> None:
        """flic_cluster_batched on already marshalled flic_scan structs."""
        arr = (_Scan * max(1, len(structs)))(*structs)
        _check(lib().flic_cluster_batched(self.handle, arr, len(structs), _stream_handle(stream)))

    def cluster_batched_host(self, structs, n: int, host_ranges, host_labels, stream=None) -> None:
        """flic_cluster_batched_host on marshalled arrays: `structs` a ctypes
        array of n flic_scan, host_ranges / host_labels ctypes arrays of n
        host addresses (pinned buffers), or None."""
        _check(lib().flic_cluster_batched_host(self.handle, structs, n, host_ranges, host_labels,
                                               _stream_handle(stream)))

    def cluster_struct_async(self, sc: _Scan, stream=None) -> None:
        """flic_cluster_async on one marshalled flic_scan struct."""
        _check(lib().flic_cluster_async(self.handle, sc.range_img, sc.H, sc.W, ctypes.byref(sc.tables),
                                        sc.threshold, sc.skip_depth, sc.labels_out,
                                        _stream_handle(stream)))

    def set_pass_timing(self, enable: bool) -> None:
        _check(lib().flic_ctx_set_pass_timing(self.handle, int(bool(enable))))

    def pass_times(self):
        """(summed ms of [tile labelling, border merge, relabel], launches)
        since the last call; waits for the timed work."""
        arr = (ctypes.c_float * 3)()
        n = ctypes.c_int32()
        _check(lib().flic_ctx_pass_times(self.handle, arr, ctypes.byref(n)))
        return [float(x) for x in arr], int(n.value)

    def cluster_async(self, scan: DeviceScan, stream=None):
        scan.validate()
        if scan.min_points or scan.map_connections:    # flic_scan fields only
            return self.cluster_batched([scan], stream)[0]
        H, W = scan.range_img.shape
        t = _Tables(scan.cos_v.data_ptr(), scan.cos_h.data_ptr())
        _check(lib().flic_cluster_async(self.handle, scan.range_img.data_ptr(), H, W,
                                        ctypes.byref(t), float(scan.threshold),
                                        int(scan.skip_depth), scan.labels.data_ptr(),
                                        _stream_handle(stream)))
        return scan.labels

    def cluster_batched(self, scans: Sequence[DeviceScan], stream=None):
        arr = self.scan_array(scans)
        _check(lib().flic_cluster_batched(self.handle, arr, len(scans), _stream_handle(stream)))
        return [s.labels for s in scans]

    @staticmethod
    def scan_array(scans: Sequence[DeviceScan]):
        """Marshalled flic_scan[] for repeated cluster_batched_array calls."""
        for s in scans:
            s.validate()
        arr = (_Scan * max(1, len(scans)))()
        for i, s in enumerate(scans):
            arr[i] = s.to_c()
        arr._n = len(scans)
        return arr

    def cluster_batched_array(self, arr, stream=None) -> None:
        _check(lib().flic_cluster_batched(self.handle, arr, arr._n, _stream_handle(stream)))

    def plan(self, scans: Sequence[DeviceScan]) -> "Plan":
        return Plan(self, scans)


class Plan:
    """A hipGraph-captured launch for a fixed list of scan shapes."""

    def __init__(self, ctx: Context, scans: Sequence[DeviceScan]):
        for s in scans:
            s.validate()
        self.ctx = ctx
        self.n = len(scans)
        arr = (_Scan * max(1, self.n))()
        for i, s in enumerate(scans):
            arr[i] = s.to_c()
        h = ctypes.c_void_p()
        _check(lib().flic_plan_create(ctx.handle, arr, self.n, ctypes.byref(h)))
        self.handle = h
        self._arr = arr           # the planned scans, for relaunch()

    def relaunch(self, stream=None) -> None:
        """Launch again on the scans the plan was created with."""
        _check(lib().flic_plan_launch(self.handle, self._arr, self.n, _stream_handle(stream)))

    def launch(self, scans: Sequence[DeviceScan], stream=None):
        arr = (_Scan * max(1, len(scans)))()
        for i, s in enumerate(scans):
            s.validate()
            arr[i] = s.to_c()
        _check(lib().flic_plan_launch(self.handle, arr, len(scans), _stream_handle(stream)))
        return [s.labels for s in scans]

    def close(self) -> None:
        if self.handle:
            lib().flic_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context(device: Optional[int] = None) -> Context:
    import torch
    if device is None:
        device = torch.cuda.current_device()
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def cluster(range_img, cos_v, cos_h, threshold: float, skip_depth: int, out=None, stream=None,
            min_points: int = 0):
    """Labels int32 [H, W] of one scan, enqueued on `stream` (default: the
    current torch stream).  Inputs are device tensors."""
    s = DeviceScan(range_img, cos_v, cos_h, threshold, skip_depth, out, min_points)
    return default_context(range_img.device.index).cluster_async(s, stream)


def cluster_sync(range_img, cos_v, cos_h, threshold: float, skip_depth: int, out=None):
    """flic_cluster: blocking call on the null stream."""
    s = DeviceScan(range_img, cos_v, cos_h, threshold, skip_depth, out)
    s.validate()
    H, W = range_img.shape
    _check(cluster_raw(range_img.data_ptr(), H, W, cos_v.data_ptr(), cos_h.data_ptr(),
                       float(threshold), int(skip_depth), s.labels.data_ptr()))
    return s.labels


def cluster_noalloc(range_img, cos_v, cos_h, threshold: float, skip_depth: int, out=None, stream=None):
    """flic_cluster_noalloc: labels int32 [H, W] of one scan, enqueued on
    `stream` (default: the current torch stream) with the library's fixed
    device scratch (no allocation; calls overlapping on one device race)."""
    s = DeviceScan(range_img, cos_v, cos_h, threshold, skip_depth, out)
    s.validate()
    H, W = range_img.shape
    _check(cluster_noalloc_raw(range_img.data_ptr(), H, W, cos_v.data_ptr(), cos_h.data_ptr(),
                               float(threshold), int(skip_depth), s.labels.data_ptr(),
                               _stream_handle(stream)))
    return s.labels


def cluster_batched(scans: Sequence[DeviceScan], stream=None):
    if not scans:
        return []
    return default_context(scans[0].range_img.device.index).cluster_batched(scans, stream)


@dataclasses.dataclass
class DeviceGroundTables:
    """Device copies (float32 [H] tensors) of one sensor's ground tables."""
    sin_a: "object"
    cos_a: "object"
    tan_lo: "object"
    tan_hi: "object"
    sin_d: "object"
    cos_d: "object"
    sensor_height: float
    tan_theta: float

    @property
    def H(self) -> int:
        return int(self.sin_a.shape[0])

    def to_c(self) -> _GroundTables:
        import torch
        for k in ("sin_a", "cos_a", "tan_lo", "tan_hi", "sin_d", "cos_d"):
            _check_tensor(getattr(self, k), torch.float32, (self.H,), k)
        return _GroundTables(self.sin_a.data_ptr(), self.cos_a.data_ptr(), self.tan_lo.data_ptr(),
                             self.tan_hi.data_ptr(), self.sin_d.data_ptr(), self.cos_d.data_ptr(),
                             float(self.sensor_height), float(self.tan_theta))


def ground_tables_to_device(g, device="cuda") -> DeviceGroundTables:
    """Copy host ground tables (synth.GroundTables) to the device."""
    import torch
    t = {k: torch.from_numpy(getattr(g, k)).to(device)
         for k in ("sin_a", "cos_a", "tan_lo", "tan_hi", "sin_d", "cos_d")}
    return DeviceGroundTables(**t, sensor_height=g.sensor_height, tan_theta=g.tan_theta)


def ground_remove(range_img, tables: DeviceGroundTables, out=None, mask=None, stream=None,
                  ctx: Optional["Context"] = None, with_mask: bool = True):
    """flic_ground_remove on a [H, W] or [n, H, W] float32 device tensor:
    returns (range with ground cells set to 0, uint8 ground mask or None)."""
    import torch
    squeeze = range_img.dim() == 2
    r = range_img.unsqueeze(0) if squeeze else range_img
    n, H, W = r.shape
    _check_tensor(r, torch.float32, (n, H, W), "range_img")
    if out is None:
        out = torch.empty_like(r)
    out = out.view(n, H, W)
    _check_tensor(out, torch.float32, (n, H, W), "out")
    if mask is None and with_mask:
        mask = torch.empty((n, H, W), dtype=torch.uint8, device=r.device)
    if mask is not None:
        mask = mask.view(n, H, W)
        _check_tensor(mask, torch.uint8, (n, H, W), "mask")
    ctx = ctx or default_context(r.device.index)
    t = tables.to_c()
    _check(lib().flic_ground_remove(ctx.handle, r.data_ptr(), n, H, W, ctypes.byref(t), out.data_ptr(),
                                    mask.data_ptr() if mask is not None else None,
                                    _stream_handle(stream)))
    if squeeze:
        return out[0], (mask[0] if mask is not None else None)
    return out, mask


def to_device(scan, device="cuda", min_points: int = 0, map_connections: int = 0) -> DeviceScan:
    """Copy a host scan (synth.Scan) to device tensors."""
    import torch
    d = DeviceScan(torch.from_numpy(scan.range_img).to(device),
                   torch.from_numpy(scan.cos_v).to(device),
                   torch.from_numpy(scan.cos_h).to(device),
                   scan.threshold, scan.skip_depth, min_points=min_points,
                   map_connections=map_connections)
    d.validate()          # allocates the labels tensor
    return d


class Server:
    """The library's serving runtime (flic_server_*): sensors, slots, FIFO
    admission and continuous batching in native code.  ctx None: simulated
    device (each launch takes sim_launch_s; no buffers are touched)."""

    def __init__(self, ctx: Optional["Context"], n_streams: int = 3, max_batch: int = 64,
                 slots_per_sensor: int = 3, max_queue: int = 64, hbm_budget: int = 0,
                 sim_launch_s: float = 0.0, stage_kernels: int = 0):
        self.ctx = ctx
        cfg = _ServerConfig(n_streams, max_batch, slots_per_sensor, max_queue, hbm_budget, sim_launch_s,
                            int(stage_kernels))
        h = ctypes.c_void_p()
        _check(lib().flic_server_create(ctx.handle if ctx is not None else None, ctypes.byref(cfg),
                                        ctypes.byref(h)))
        self.handle = h.value

    def add_sensor(self, H: int, W: int, cos_v, cos_h, threshold: float, skip_depth: int) -> int:
        """cos_v [N][H], cos_h [N][W]: host float32 arrays (copied)."""
        import numpy as np
        cv = np.ascontiguousarray(cos_v, dtype=np.float32)
        chh = np.ascontiguousarray(cos_h, dtype=np.float32)
        sid = ctypes.c_int32()
        t = _Tables(cv.ctypes.data, chh.ctypes.data)
        _check(lib().flic_server_add_sensor(self.handle, H, W, ctypes.byref(t), float(threshold),
                                            int(skip_depth), ctypes.byref(sid)))
        return sid.value

    def now(self) -> float:
        return lib().flic_server_now(self.handle)

    def submit(self, now: float, t_arrival: float, sensor: int, host_range: int = 0, host_labels: int = 0,
               tag: int = 0) -> None:
        _check(lib().flic_server_submit(self.handle, now, t_arrival, sensor, host_range or None,
                                        host_labels or None, tag))

    def progress(self, now: float) -> int:
        n = ctypes.c_int32()
        _check(lib().flic_server_progress(self.handle, now, ctypes.byref(n)))
        return n.value

    def replay(self, arrivals) -> None:
        """arrivals: numpy array of ARRIVAL_DTYPE, times non-decreasing."""
        import numpy as np
        a = np.ascontiguousarray(arrivals, dtype=ARRIVAL_DTYPE)
        assert ctypes.sizeof(_Arrival) == a.dtype.itemsize
        _check(lib().flic_server_replay(self.handle, a.ctypes.data if len(a) else None, len(a)))

    def records(self):
        """(records as a numpy array of RECORD_DTYPE, dropped, launches)."""
        import numpy as np
        n, dropped, launches = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().flic_server_records(self.handle, None, 0, ctypes.byref(n), None, None))
        out = np.zeros(n.value, dtype=RECORD_DTYPE)
        assert ctypes.sizeof(_FrameRecord) == out.dtype.itemsize
        _check(lib().flic_server_records(self.handle, out.ctypes.data if n.value else None, n.value,
                                         ctypes.byref(n), ctypes.byref(dropped), ctypes.byref(launches)))
        return out, dropped.value, launches.value

    def clear(self) -> None:
        _check(lib().flic_server_clear(self.handle))

    def close(self) -> None:
        if self.handle:
            lib().flic_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

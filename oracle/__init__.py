"""CPU oracle for FLIC range-image clustering (ctypes wrapper over flic_oracle.c).

TEST INFRASTRUCTURE ONLY.  Imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; the product package never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flic_oracle.c")
# FLIC_ORACLE_LIB points the wrapper at another build of the same source (the
# sanitizer tests load an AddressSanitizer / UBSan build this way).
_LIB = os.environ.get("FLIC_ORACLE_LIB") or os.path.join(_HERE, "libflic_oracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared"]

_lib: Optional[ctypes.CDLL] = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libflic_oracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        fp = ctypes.POINTER(ctypes.c_float)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.flic_oracle_cluster.restype = ctypes.c_int32
        L.flic_oracle_cluster.argtypes = [fp, ctypes.c_int32, ctypes.c_int32, fp, fp,
                                          ctypes.c_float, ctypes.c_int32, ip]
        L.flic_oracle_cluster_maps.restype = ctypes.c_int32
        L.flic_oracle_cluster_maps.argtypes = [fp, ctypes.c_int32, ctypes.c_int32, fp, fp,
                                               ctypes.c_float, ctypes.c_int32, ctypes.c_int32, ip]
        L.flic_oracle_filter_small.restype = ctypes.c_int32
        L.flic_oracle_filter_small.argtypes = [ip, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ip]
        L.flic_oracle_ground.restype = ctypes.c_int32
        L.flic_oracle_ground.argtypes = [fp, ctypes.c_int32, ctypes.c_int32, fp, fp, fp, fp, fp, fp,
                                         ctypes.c_float, ctypes.c_float,
                                         ctypes.POINTER(ctypes.c_uint8), fp]
        L.flic_oracle_dist2.restype = ctypes.c_float
        L.flic_oracle_dist2.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_float]
        _lib = L
    return _lib


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def dist2(d1: float, d2: float, cos_alpha: float) -> np.float32:
    """Eq. (4) in binary32."""
    return np.float32(lib().flic_oracle_dist2(d1, d2, cos_alpha))


def cluster_status(range_img: np.ndarray, cos_v: np.ndarray, cos_h: np.ndarray,
                   threshold: float, skip_depth: int, H: Optional[int] = None,
                   W: Optional[int] = None):
    """Raw call: returns (status, labels)."""
    r = np.ascontiguousarray(range_img, dtype=np.float32)
    if H is None:
        H, W = r.shape
    cv = np.ascontiguousarray(cos_v, dtype=np.float32)
    ch = np.ascontiguousarray(cos_h, dtype=np.float32)
    out = np.full(max(H * W, 1), -7, dtype=np.int32)
    st = lib().flic_oracle_cluster(_fptr(r), H, W, _fptr(cv), _fptr(ch),
                                   float(threshold), int(skip_depth),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return st, out[: H * W].reshape(H, W) if H * W > 0 else out[:0]


def ground(range_img: np.ndarray, tables) -> tuple:
    """Section III.A ground extraction.  tables: an object with float32 [H]
    arrays sin_a, cos_a, tan_lo, tan_hi, sin_d, cos_d and floats
    sensor_height, tan_theta.  Returns (ground mask uint8 [H, W], range with
    ground cells set to 0)."""
    r = np.ascontiguousarray(range_img, dtype=np.float32)
    H, W = r.shape
    arrs = [np.ascontiguousarray(getattr(tables, k), dtype=np.float32)
            for k in ("sin_a", "cos_a", "tan_lo", "tan_hi", "sin_d", "cos_d")]
    for a in arrs:
        if a.shape != (H,):
            raise ValueError("ground tables must have H entries")
    mask = np.empty((H, W), dtype=np.uint8)
    out = np.empty((H, W), dtype=np.float32)
    st = lib().flic_oracle_ground(_fptr(r), H, W, *[_fptr(a) for a in arrs],
                                  float(tables.sensor_height), float(tables.tan_theta),
                                  mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _fptr(out))
    if st != 0:
        raise ValueError(f"flic_oracle_ground failed with status {st}")
    return mask, out


def filter_small(labels: np.ndarray, min_points: int) -> np.ndarray:
    """Section III.B.1 size threshold: labels of components with fewer than
    min_points pixels become -1."""
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    H, W = lab.shape
    out = np.empty_like(lab)
    ip = ctypes.POINTER(ctypes.c_int32)
    st = lib().flic_oracle_filter_small(lab.ctypes.data_as(ip), H, W, int(min_points),
                                        out.ctypes.data_as(ip))
    if st != 0:
        raise ValueError(f"flic_oracle_filter_small failed with status {st}")
    return out


def cluster(range_img: np.ndarray, cos_v: np.ndarray, cos_h: np.ndarray,
            threshold: float, skip_depth: int, min_points: int = 0, maps: int = 0) -> np.ndarray:
    """Labels int32 [H, W]: minimum linear index of each component, -1 if
    missing or (min_points > 0) in a component of fewer than min_points pixels.
    maps = 1 takes the skip edges from the stride-k maps of Section III.B.2
    instead of every pixel."""
    if maps:
        r = np.ascontiguousarray(range_img, dtype=np.float32)
        H, W = r.shape
        out = np.empty((H, W), dtype=np.int32)
        st = lib().flic_oracle_cluster_maps(_fptr(r), H, W,
                                            _fptr(np.ascontiguousarray(cos_v, dtype=np.float32)),
                                            _fptr(np.ascontiguousarray(cos_h, dtype=np.float32)),
                                            float(threshold), int(skip_depth), int(maps),
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    else:
        st, out = cluster_status(range_img, cos_v, cos_h, threshold, skip_depth)
    if st != 0:
        raise ValueError(f"flic_oracle_cluster failed with status {st}")
    return filter_small(out, min_points) if min_points > 0 else out


def cluster_scan(scan, min_points: int = 0, maps: int = 0) -> np.ndarray:
    return cluster(scan.range_img, scan.cos_v, scan.cos_h, scan.threshold, scan.skip_depth,
                   min_points, maps)

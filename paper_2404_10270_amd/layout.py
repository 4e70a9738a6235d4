"""ctypes binding of libpic_layout (include/pic_layout.h): libpic's FP32
mover pass over one species in four particle layouts, for the layout study.
Argument marshalling only; every step runs in the library's kernels, and the
binding raises when the library is missing or no GPU is present."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpic_layout.so")

PLS_SOA, PLS_AOS, PLS_AOSOA, PLS_CELLPAD = 0, 1, 2, 3
LAYOUTS = {"soa": PLS_SOA, "aos": PLS_AOS, "aosoa": PLS_AOSOA, "cellpad": PLS_CELLPAD}
ABI_SYMBOLS = ("pls_work_bytes", "pls_load", "pls_step", "pls_store")


class pls_soa(C.Structure):
    _fields_ = [("cell", C.c_void_p), ("f", C.c_void_p), ("vx", C.c_void_p), ("vy", C.c_void_p),
                ("vz", C.c_void_p), ("id", C.c_void_p)]


class pls_params(C.Structure):
    _fields_ = [("nc", C.c_int32), ("slack", C.c_int32), ("tx", C.c_float), ("ty", C.c_float),
                ("sx", C.c_float), ("sy", C.c_float), ("key0", C.c_uint32), ("key1", C.c_uint32),
                ("T", C.c_uint64), ("acc", C.c_void_p), ("S", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built (python -m paper_2404_10270_amd.build)")
        L = C.CDLL(LIB)
        i64, vp = C.c_int64, C.c_void_p
        L.pls_work_bytes.argtypes = [C.c_int, i64, C.c_int32, C.c_int32, C.POINTER(C.c_uint64)]
        L.pls_load.argtypes = [C.c_int, C.POINTER(pls_soa), i64, C.c_int32, C.c_int32, vp, vp]
        L.pls_step.argtypes = [C.c_int, C.POINTER(pls_params), i64, i64, i64, vp, vp]
        L.pls_store.argtypes = [C.c_int, vp, i64, C.c_int32, C.c_int32, i64, C.POINTER(pls_soa),
                                C.POINTER(C.c_int64), C.POINTER(C.c_uint64), vp]
        for f in ABI_SYMBOLS:
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed with {rc}")


def _soa(t) -> pls_soa:
    s = pls_soa()
    for k in ("cell", "f", "vx", "vy", "vz", "id"):
        setattr(s, k, t[k].data_ptr())
    return s


class LayoutRun:
    """One species' particles (torch device tensors cell, f, vx, vy, vz, id)
    loaded into a layout's work buffer."""

    def __init__(self, layout: int, soa: dict, nc: int, slack: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libpic_layout needs a GPU")
        self.torch = torch
        self.layout, self.nc, self.slack = layout, int(nc), int(slack)
        self.n = int(soa["id"].numel())
        nb = C.c_uint64()
        _check(lib().pls_work_bytes(layout, self.n, self.nc, self.slack, C.byref(nb)), "pls_work_bytes")
        self.work = torch.zeros(int(nb.value) + 256, dtype=torch.uint8, device=soa["id"].device)
        off = (-self.work.data_ptr()) % 256
        self.wptr = self.work.data_ptr() + off
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.passes = 0
        src = _soa(soa)
        _check(lib().pls_load(layout, C.byref(src), self.n, self.nc, self.slack, self.wptr,
                              self.stream.cuda_stream), "pls_load")

    def step(self, params: pls_params, step: int):
        _check(lib().pls_step(self.layout, C.byref(params), self.n, self.passes, int(step), self.wptr,
                              self.stream.cuda_stream), "pls_step")
        self.passes += 1

    def store(self) -> tuple:
        """(dict of torch tensors, candidates counted) after the passes so far."""
        torch = self.torch
        dev = self.work.device
        out = {"cell": torch.empty(self.n, dtype=torch.int32, device=dev),
               "f": torch.empty(self.n, dtype=torch.float32, device=dev),
               "vx": torch.empty(self.n, dtype=torch.float32, device=dev),
               "vy": torch.empty(self.n, dtype=torch.float32, device=dev),
               "vz": torch.empty(self.n, dtype=torch.float32, device=dev),
               "id": torch.empty(self.n, dtype=torch.int64, device=dev)}
        n_out, n_cand = C.c_int64(), C.c_uint64()
        dst = _soa(out)
        _check(lib().pls_store(self.layout, self.wptr, self.n, self.nc, self.slack, self.passes,
                               C.byref(dst), C.byref(n_out), C.byref(n_cand),
                               self.stream.cuda_stream), "pls_store")
        m = int(n_out.value)
        return {k: v[:m] for k, v in out.items()}, int(n_cand.value)

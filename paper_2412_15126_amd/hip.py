"""Minimal ctypes view of the HIP runtime that libckr.so links (device buffers,
copies, streams, events) -- plumbing for tests and timing.

It binds the same libamdhip64 instance as the library, so buffers, streams
and events are shared with it.
"""
import ctypes as C
import os

import numpy as np

_rt = None


def rt():
    global _rt
    if _rt is None:
        from . import lib
        lib()  # load libckr.so first so its HIP runtime is the one in the process
        rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
        path = os.path.join(rocm, "lib", "libamdhip64.so")
        R = C.CDLL(path)
        vp = C.c_void_p
        for name, args in {
            "hipMalloc": [C.POINTER(vp), C.c_size_t],
            "hipFree": [vp],
            "hipMemcpy": [vp, vp, C.c_size_t, C.c_int],
            "hipDeviceSynchronize": [],
            "hipStreamCreate": [C.POINTER(vp)],
            "hipStreamDestroy": [vp],
            "hipStreamSynchronize": [vp],
            "hipEventCreate": [C.POINTER(vp)],
            "hipEventDestroy": [vp],
            "hipEventRecord": [vp, vp],
            "hipEventSynchronize": [vp],
            "hipEventElapsedTime": [C.POINTER(C.c_float), vp, vp],
            "hipSetDevice": [C.c_int],
        }.items():
            fn = getattr(R, name)
            fn.argtypes = args
            fn.restype = C.c_int
        _rt = R
    return _rt


def _ok(st, what):
    if st != 0:
        raise RuntimeError(f"{what} failed with HIP error {st}")


class DeviceArray:
    """A device allocation holding a copy of a numpy array."""

    def __init__(self, host):
        host = np.ascontiguousarray(host)
        self.shape, self.dtype, self.nbytes = host.shape, host.dtype, host.nbytes
        self.ptr = C.c_void_p()
        _ok(rt().hipMalloc(C.byref(self.ptr), max(self.nbytes, 1)), "hipMalloc")
        _ok(rt().hipMemcpy(self.ptr, host.ctypes.data_as(C.c_void_p), self.nbytes, 1), "hipMemcpy H2D")

    def numpy(self):
        out = np.empty(self.shape, self.dtype)
        _ok(rt().hipMemcpy(out.ctypes.data_as(C.c_void_p), self.ptr, self.nbytes, 2), "hipMemcpy D2H")
        return out

    def free(self):
        if self.ptr:
            rt().hipFree(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        self.free()


def synchronize():
    _ok(rt().hipDeviceSynchronize(), "hipDeviceSynchronize")


class Stream:
    def __init__(self):
        self.h = C.c_void_p()
        _ok(rt().hipStreamCreate(C.byref(self.h)), "hipStreamCreate")

    def synchronize(self):
        _ok(rt().hipStreamSynchronize(self.h), "hipStreamSynchronize")


class Event:
    def __init__(self):
        self.h = C.c_void_p()
        _ok(rt().hipEventCreate(C.byref(self.h)), "hipEventCreate")

    def record(self, stream=None):
        _ok(rt().hipEventRecord(self.h, stream.h if stream else None), "hipEventRecord")

    def synchronize(self):
        _ok(rt().hipEventSynchronize(self.h), "hipEventSynchronize")

    def elapsed_ms(self, end):
        ms = C.c_float()
        _ok(rt().hipEventElapsedTime(C.byref(ms), self.h, end.h), "hipEventElapsedTime")
        return ms.value

"""Device memory and a stream without torch: ctypes over the HIP runtime that
liblee.so itself links (argument marshalling only).

For a process that must hold a single HIP runtime.  torch ships its own
runtime under the same soname; a profiler that preloads the system runtime
before the program starts would then leave two runtimes in one process, with
torch's allocations and the library's launches in different contexts.  A
process that binds its instances through this module never imports torch.
"""
from __future__ import annotations

import ctypes

_hip = None


def _lib():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so.7", mode=ctypes.RTLD_GLOBAL)
        _hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        _hip.hipFree.argtypes = [ctypes.c_void_p]
        _hip.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        _hip.hipStreamDestroy.argtypes = [ctypes.c_void_p]
        _hip.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        _hip.hipSetDevice.argtypes = [ctypes.c_int]
        _hip.hipGetErrorString.restype = ctypes.c_char_p
        _hip.hipGetErrorString.argtypes = [ctypes.c_int]
    return _hip


def _check(e: int, what: str) -> None:
    if e != 0:
        raise RuntimeError(f"{what}: {_lib().hipGetErrorString(e).decode()}")


def set_device(index: int = 0) -> None:
    _check(_lib().hipSetDevice(index), "hipSetDevice")


class DeviceBuffer:
    """hipMalloc'd bytes (256-byte aligned), freed by close()."""

    def __init__(self, nbytes: int):
        p = ctypes.c_void_p()
        _check(_lib().hipMalloc(ctypes.byref(p), max(int(nbytes), 1)), "hipMalloc")
        self.ptr = p.value
        self.nbytes = int(nbytes)

    def close(self) -> None:
        if self.ptr:
            _check(_lib().hipFree(self.ptr), "hipFree")
            self.ptr = None


class Stream:
    """A HIP stream at the default priority, destroyed by close()."""

    def __init__(self):
        s = ctypes.c_void_p()
        _check(_lib().hipStreamCreate(ctypes.byref(s)), "hipStreamCreate")
        self.handle = s.value

    def synchronize(self) -> None:
        _check(_lib().hipStreamSynchronize(self.handle), "hipStreamSynchronize")

    def close(self) -> None:
        if self.handle:
            _check(_lib().hipStreamDestroy(self.handle), "hipStreamDestroy")
            self.handle = None

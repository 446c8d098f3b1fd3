"""The library's C ABI over the CPU emulation build (libsdgp_emu.so, see
build_emu.py): host NumPy arrays stand in for device memory.  Load it in a
process started with the AddressSanitizer runtime preloaded (run_case.py
does that through emu_env())."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from paper_2205_09070_amd import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
DEFAULT_LIB = os.path.join(ROOT, "_build", "emu", "libsdgp_emu.so")


def emu_env(extra=None) -> dict:
    """Environment of a child process that loads the emulation build."""
    from tests.emu import build_emu
    env = dict(os.environ)
    env["LD_PRELOAD"] = build_emu.asan_runtime()
    env["ASAN_OPTIONS"] = ("detect_leaks=0:detect_stack_use_after_return=0:detect_odr_violation=0:"
                           "alloc_dealloc_mismatch=0:abort_on_error=1:halt_on_error=1")
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    if extra:
        env.update(extra)
    return env


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


class EmuContext:
    def __init__(self, path: str = DEFAULT_LIB):
        lib = C.CDLL(path)
        for name, (res, args) in _lib._SIGS.items():
            fn = getattr(lib, name, None)
            if fn is None:      # a build of an older source tree
                continue
            fn.restype = res
            fn.argtypes = args
        self.lib = lib
        h = _lib.VP()
        st = lib.sdgp_create(C.byref(h), 0, None)
        if st != _lib.OK:
            raise _lib.SdgpError(st, lib.sdgp_last_error(None).decode())
        self.h = h
        if lib.sdgp_set_option(h, b"autotune", 0) not in (_lib.OK, _lib.INVALID_ARG):
            raise RuntimeError("sdgp_set_option failed")   # the emulator's clock says nothing about the GPU

    def close(self):
        if self.h is not None:
            self.lib.sdgp_destroy(self.h)
            self.h = None

    def _check(self, st):
        if st != _lib.OK:
            raise _lib.SdgpError(st, self.lib.sdgp_last_error(self.h).decode())

    def set_option(self, name: str, value: int):
        self._check(self.lib.sdgp_set_option(self.h, name.encode(), int(value)))

    def get_option(self, name: str) -> int:
        v = _lib.I64(0)
        self._check(self.lib.sdgp_get_option(self.h, name.encode(), C.byref(v)))
        return int(v.value)

    def lml_grad(self, desc, x, y, h, est):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        hh = np.ascontiguousarray(h, dtype=np.float64)
        d = _lib.desc_of(desc)
        info = _lib.Info()
        v = np.zeros(1)
        g = np.zeros(hh.shape[0])
        self._check(self.lib.sdgp_lml_grad(self.h, C.byref(d), _p(x), _p(y), x.shape[0], _p(hh), C.byref(est),
                                           _p(v), _p(g), C.byref(info)))
        return float(v[0]), g, info

    def lml_grad_batched(self, desc, x, y, H, est):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        H = np.ascontiguousarray(H, dtype=np.float64)
        B, nh = H.shape
        d = _lib.desc_of(desc)
        v = np.zeros(B)
        g = np.zeros((B, nh))
        ms = np.zeros(B, dtype=np.int32)
        infos = (_lib.Info * B)()
        self._check(self.lib.sdgp_lml_grad_batched(self.h, C.byref(d), _p(x), _p(y), x.shape[0], _p(H), B,
                                                   C.byref(est), _p(v), _p(g), _p(ms), C.cast(infos, _lib.VP)))
        return v, g, ms, list(infos)

    def kernel_assemble_sorted(self, desc, x, h, nnz, capacity=None):
        x = np.ascontiguousarray(x, dtype=np.float64)
        hh = np.ascontiguousarray(h, dtype=np.float64)
        n = x.shape[0]
        d = _lib.desc_of(desc)
        rp = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(max(nnz, 1), dtype=np.int32)
        val = np.zeros(max(nnz, 1), dtype=np.float64)
        perm = np.zeros(n, dtype=np.int32)
        out = C.c_int64(0)
        cap = col.shape[0] if capacity is None else capacity
        self._check(self.lib.sdgp_kernel_assemble_sorted(self.h, C.byref(d), _p(x), n, _p(hh), 1, _p(rp), _p(col),
                                                         _p(val), _p(perm), cap, C.byref(out)))
        return rp, col[:out.value], val[:out.value], perm

    def kernel_nnz(self, desc, x, h):
        x = np.ascontiguousarray(x, dtype=np.float64)
        hh = np.ascontiguousarray(h, dtype=np.float64)
        d = _lib.desc_of(desc)
        out = C.c_int64(0)
        self._check(self.lib.sdgp_kernel_nnz(self.h, C.byref(d), _p(x), x.shape[0], _p(hh), C.byref(out)))
        return int(out.value)

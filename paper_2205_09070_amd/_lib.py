"""ctypes binding of libsdgp.so (include/sdgp.h).

Argument marshalling only: every computation runs in the HIP library.  Device
arrays are torch tensors on a ROCm device (their data pointers are passed
through), host arrays are NumPy float64 arrays, and every call enqueues on
torch's current stream for the tensor's device.  If the library has not been
built, or no GPU is present, calls raise instead of falling back.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdgp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sdgp.h")

OK, INVALID_ARG, OOM, NOT_SPD, NOT_CONVERGED, HIP, CAPACITY = range(7)
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "NOT_SPD", 4: "NOT_CONVERGED",
                5: "HIP", 6: "CAPACITY"}
CORE_WENDLAND_C2, CORE_KSTAT = 0, 1
COMBINE_PRODUCT, COMBINE_SUM = 0, 1
PROBE_RADEMACHER, PROBE_IDENTITY = 0, 2
PRECOND_NONE, PRECOND_LOWRANK = 0, 1
OPERATOR_ASSEMBLED, OPERATOR_FACTORED = 0, 1
DE_LML, DE_AUGMENTED, DE_CONSTRAINED = 0, 1, 2


class KernelDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n1", C.c_int32), ("n2", C.c_int32),
                ("core", C.c_int32), ("combine", C.c_int32)]


class Estimator(C.Structure):
    _fields_ = [("probes", C.c_int32), ("lanczos_steps", C.c_int32), ("kind", C.c_int32),
                ("cg_max_iter", C.c_int32), ("seed", C.c_uint64), ("cg_rtol", C.c_double),
                ("precond", C.c_int32), ("operator_form", C.c_int32), ("probe_rtol", C.c_double)]


class Info(C.Structure):
    _fields_ = [("nnz", C.c_int64), ("candidates", C.c_int64), ("cg_iters", C.c_int32),
                ("cg_iters_y", C.c_int32), ("cg_relres_max", C.c_double), ("yKy", C.c_double),
                ("logdet", C.c_double), ("logdet_stderr", C.c_double), ("ritz_min", C.c_double),
                ("ritz_max", C.c_double), ("ms", C.c_double * 8), ("spmm_launches", C.c_int64),
                ("spmm_ms", C.c_double)]

    def to_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "ms"}
        d["ms"] = list(self.ms)
        return d


class DeOptions(C.Structure):
    _fields_ = [("generations", C.c_int32), ("F", C.c_double), ("CR", C.c_double), ("seed", C.c_uint64),
                ("objective", C.c_int32), ("requirement", C.c_double), ("domain_volume", C.c_double)]


class SdgpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None

VP, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
_SIGS = {
    "sdgp_create": (I32, [C.POINTER(VP), C.c_int, VP]),
    "sdgp_destroy": (None, [VP]),
    "sdgp_last_error": (C.c_char_p, [VP]),
    "sdgp_set_timing": (I32, [VP, C.c_int]),
    "sdgp_set_option": (I32, [VP, C.c_char_p, I64]),
    "sdgp_get_option": (I32, [VP, C.c_char_p, C.POINTER(I64)]),
    "sdgp_tune_cache_get": (I32, [C.c_char_p, C.c_char_p, VP]),
    "sdgp_tune_cache_put": (I32, [C.c_char_p, C.c_char_p, VP]),
    "sdgp_num_hyper": (I64, [C.POINTER(KernelDesc)]),
    "sdgp_kernel_nnz": (I32, [VP, C.POINTER(KernelDesc), VP, I64, VP, C.POINTER(I64)]),
    "sdgp_kernel_assemble": (I32, [VP, C.POINTER(KernelDesc), VP, I64, VP, C.c_int, VP, VP, VP, I64,
                                   C.POINTER(I64)]),
    "sdgp_kernel_assemble_sorted": (I32, [VP, C.POINTER(KernelDesc), VP, I64, VP, C.c_int, VP, VP, VP,
                                          VP, I64, C.POINTER(I64)]),
    "sdgp_csr_spmm": (I32, [VP, I64, VP, VP, VP, VP, I32, VP]),
    "sdgp_lml": (I32, [VP, C.POINTER(KernelDesc), VP, VP, I64, VP, C.POINTER(Estimator), VP,
                       C.POINTER(Info)]),
    "sdgp_lml_grad": (I32, [VP, C.POINTER(KernelDesc), VP, VP, I64, VP, C.POINTER(Estimator), VP, VP,
                            C.POINTER(Info)]),
    "sdgp_lml_grad_noalloc": (I32, [VP, C.POINTER(KernelDesc), VP, VP, I64, VP, C.POINTER(Estimator), VP, VP,
                                    C.POINTER(Info)]),
    "sdgp_lml_grad_batched": (I32, [VP, C.POINTER(KernelDesc), VP, VP, I64, VP, I32,
                                    C.POINTER(Estimator), VP, VP, VP, VP]),
    "sdgp_posterior_mean_var": (I32, [VP, C.POINTER(KernelDesc), VP, VP, I64, VP, VP, I64,
                                      C.POINTER(Estimator), VP, VP]),
    "sdgp_logdet_taylor": (I32, [VP, C.POINTER(KernelDesc), VP, I64, VP, I32, I32, C.c_uint64,
                                 C.POINTER(D), C.POINTER(D)]),
    "sdgp_sparsity_bound": (I32, [C.POINTER(KernelDesc), VP, D, C.POINTER(D)]),
    "sdgp_sparsity_objective": (I32, [D, D, D, C.POINTER(D), C.POINTER(I32)]),
    "sdgp_de_trials": (I32, [I32, I32, VP, VP, VP, D, D, C.c_uint64, C.c_uint64, VP]),
    "sdgp_de_select": (I32, [I32, I32, VP, VP, VP, VP, C.POINTER(I32)]),
    "sdgp_train_de": (I32, [VP, C.POINTER(KernelDesc), VP, VP, I64, VP, I32, VP, VP, C.POINTER(Estimator),
                            C.POINTER(DeOptions), VP, VP]),
}


def sparsity_bound(desc, h, domain_volume=1.0) -> float:
    """Sparsity upper bound of eq:sparsity_estimate (host-only library call)."""
    lib = load()
    d = desc_of(desc)
    hh = np.ascontiguousarray(np.asarray(h, dtype=np.float64))
    out = D(0.0)
    st = lib.sdgp_sparsity_bound(C.byref(d), hh.ctypes.data, float(domain_volume), C.byref(out))
    if st != OK:
        raise SdgpError(st, "sdgp_sparsity_bound failed")
    return float(out.value)


def sparsity_objective(lml, s, requirement):
    """(augmented objective, feasible) of Section 2.4 (host-only)."""
    lib = load()
    a = D(0.0)
    f = I32(0)
    st = lib.sdgp_sparsity_objective(float(lml), float(s), float(requirement), C.byref(a), C.byref(f))
    if st != OK:
        raise SdgpError(st, "sdgp_sparsity_objective failed")
    return float(a.value), bool(f.value)


def tune_cache_get(path, key):
    """Autotuner store entry for ``key`` (host-only library call):
    (spmm_blocks, update_blocks, union_spmm, fw_mfma), or None when absent."""
    lib = load()
    v = np.zeros(4, dtype=np.int64)
    st = lib.sdgp_tune_cache_get(None if path is None else str(path).encode(), key.encode(), v.ctypes.data)
    return None if st != OK else tuple(int(t) for t in v)


def tune_cache_put(path, key, values):
    """Stores an autotuner entry (host-only library call); raises on invalid
    values or keys."""
    lib = load()
    v = np.ascontiguousarray(np.asarray(values, dtype=np.int64))
    if v.shape != (4,):
        raise ValueError("values: (spmm_blocks, update_blocks, union_spmm, fw_mfma)")
    st = lib.sdgp_tune_cache_put(None if path is None else str(path).encode(), key.encode(), v.ctypes.data)
    if st != OK:
        raise SdgpError(st, "sdgp_tune_cache_put failed")


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def de_trials(H, lo, hi, F=0.7, CR=0.9, seed=0, generation=1):
    """Trial vectors of one differential-evolution generation (host-only
    library call); H: (B, nh)."""
    lib = load()
    H, lo, hi = _f64(H), _f64(lo), _f64(hi)
    B, nh = H.shape
    T = np.empty_like(H)
    st = lib.sdgp_de_trials(B, nh, H.ctypes.data, lo.ctypes.data, hi.ctypes.data, float(F), float(CR),
                            int(seed), int(generation), T.ctypes.data)
    if st != OK:
        raise SdgpError(st, "sdgp_de_trials failed")
    return T


def de_select(H, fit, T, ft):
    """Selection step; returns (H, fit, replaced) (new arrays)."""
    lib = load()
    H, fit, T, ft = _f64(H).copy(), _f64(fit).copy(), _f64(T), _f64(ft)
    B, nh = H.shape
    rep = I32(0)
    st = lib.sdgp_de_select(B, nh, H.ctypes.data, fit.ctypes.data, T.ctypes.data, ft.ctypes.data, C.byref(rep))
    if st != OK:
        raise SdgpError(st, "sdgp_de_select failed")
    return H, fit, int(rep.value)


def header_functions() -> list:
    """Names of the functions declared in include/sdgp.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sdgp_[a-z_0-9]+)\s*\(", txt)))


def load():
    """Load libsdgp.so (built by build()); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsdgp.so is not built (run __graft_entry__.build() or "
                           "python -m paper_2205_09070_amd.build)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def desc_of(d) -> KernelDesc:
    return KernelDesc(int(d.dim), int(d.n1), int(d.n2), int(d.core), int(d.combine))


def estimator(probes=32, lanczos_steps=0, kind=PROBE_RADEMACHER, cg_max_iter=5000, seed=0,
              cg_rtol=1e-10, precond=PRECOND_NONE, operator_form=OPERATOR_ASSEMBLED,
              probe_rtol=0.0) -> Estimator:
    return Estimator(int(probes), int(lanczos_steps), int(kind), int(cg_max_iter), int(seed),
                     float(cg_rtol), int(precond), int(operator_form), float(probe_rtol))


def exact_estimator(cg_max_iter=20000, cg_rtol=1e-13) -> Estimator:
    """Identity probes: log-det and trace exact up to the CG tolerance."""
    return estimator(probes=0, kind=PROBE_IDENTITY, cg_max_iter=cg_max_iter, cg_rtol=cg_rtol)


def _ptr(t) -> int:
    return t.data_ptr()


def _hptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _dev_f64(t):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("expected a float64 tensor on a ROCm device")
    return t.contiguous()


class Context:
    """A libsdgp context bound to a device and torch's current stream."""

    def __init__(self, device=0, timing=False):
        import torch
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm GPU available: libsdgp has no CPU path")
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        h = VP()
        st = self.lib.sdgp_create(C.byref(h), self.device.index or 0, VP(self.stream.cuda_stream))
        if st != OK:
            raise SdgpError(st, self.lib.sdgp_last_error(None).decode())
        self.h = h
        if timing:
            self.set_timing(True)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.sdgp_destroy(h)
            self.h = None

    def _check(self, st, allow=()):
        if st != OK and st not in allow:
            raise SdgpError(st, self.lib.sdgp_last_error(self.h).decode())
        return st

    def set_timing(self, on: bool):
        self._check(self.lib.sdgp_set_timing(self.h, 1 if on else 0))

    def set_option(self, name: str, value: int):
        self._check(self.lib.sdgp_set_option(self.h, name.encode(), int(value)))

    def get_option(self, name: str) -> int:
        out = I64(0)
        self._check(self.lib.sdgp_get_option(self.h, name.encode(), C.byref(out)))
        return int(out.value)

    def num_hyper(self, desc) -> int:
        d = desc_of(desc)
        return int(self.lib.sdgp_num_hyper(C.byref(d)))

    @staticmethod
    def _h(h) -> np.ndarray:
        return np.ascontiguousarray(np.asarray(h, dtype=np.float64))

    def kernel_nnz(self, desc, x, h) -> int:
        x = _dev_f64(x)
        hh = self._h(h)
        d = desc_of(desc)
        out = I64(0)
        self._check(self.lib.sdgp_kernel_nnz(self.h, C.byref(d), _ptr(x), x.shape[0], _hptr(hh),
                                             C.byref(out)))
        return int(out.value)

    def kernel_assemble(self, desc, x, h, add_noise=True, sorted_order=False, nnz=None):
        """Returns (row_ptr, col, val) device tensors (and perm when
        sorted_order).  nnz: the stored count if already known (sizes the
        outputs without a counting call)."""
        import torch
        x = _dev_f64(x)
        hh = self._h(h)
        d = desc_of(desc)
        n = x.shape[0]
        if nnz is None:
            nnz = self.kernel_nnz(desc, x, hh)
        dev = x.device
        row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
        out = I64(0)
        if sorted_order:
            perm = torch.empty(n, dtype=torch.int32, device=dev)
            self._check(self.lib.sdgp_kernel_assemble_sorted(
                self.h, C.byref(d), _ptr(x), n, _hptr(hh), int(add_noise), _ptr(row_ptr), _ptr(col),
                _ptr(val), _ptr(perm), col.numel(), C.byref(out)))
            return row_ptr, col[:out.value], val[:out.value], perm
        self._check(self.lib.sdgp_kernel_assemble(
            self.h, C.byref(d), _ptr(x), n, _hptr(hh), int(add_noise), _ptr(row_ptr), _ptr(col),
            _ptr(val), col.numel(), C.byref(out)))
        return row_ptr, col[:out.value], val[:out.value]

    def csr_spmm(self, row_ptr, col, val, X, out=None):
        import torch
        X = _dev_f64(X)
        n = row_ptr.shape[0] - 1
        R = 1 if X.dim() == 1 else X.shape[1]
        if out is None:
            out = torch.empty((n,) if X.dim() == 1 else (n, R), dtype=torch.float64, device=X.device)
        self._check(self.lib.sdgp_csr_spmm(self.h, n, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(X), R,
                                           _ptr(out)))
        return out

    def lml(self, desc, x, y, h, est=None, allow_not_converged=False):
        x, y = _dev_f64(x), _dev_f64(y)
        hh = self._h(h)
        d = desc_of(desc)
        e = est or estimator()
        info = Info()
        v = np.zeros(1)
        st = self.lib.sdgp_lml(self.h, C.byref(d), _ptr(x), _ptr(y), x.shape[0], _hptr(hh), C.byref(e),
                               _hptr(v), C.byref(info))
        self._check(st, (NOT_CONVERGED,) if allow_not_converged else ())
        return float(v[0]), info

    def lml_grad(self, desc, x, y, h, est=None, allow_not_converged=False):
        x, y = _dev_f64(x), _dev_f64(y)
        hh = self._h(h)
        d = desc_of(desc)
        e = est or estimator()
        info = Info()
        v = np.zeros(1)
        g = np.zeros(hh.shape[0])
        st = self.lib.sdgp_lml_grad(self.h, C.byref(d), _ptr(x), _ptr(y), x.shape[0], _hptr(hh), C.byref(e),
                                    _hptr(v), _hptr(g), C.byref(info))
        self._check(st, (NOT_CONVERGED,) if allow_not_converged else ())
        return float(v[0]), g, info

    def lml_grad_noalloc(self, desc, x, y, h, est=None, allow_not_converged=False):
        """sdgp_lml_grad_noalloc: lml_grad with the device workspace taken
        from the library's static per-device array (no device allocation)."""
        x, y = _dev_f64(x), _dev_f64(y)
        hh = self._h(h)
        d = desc_of(desc)
        e = est or estimator()
        info = Info()
        v = np.zeros(1)
        g = np.zeros(hh.shape[0])
        st = self.lib.sdgp_lml_grad_noalloc(self.h, C.byref(d), _ptr(x), _ptr(y), x.shape[0], _hptr(hh),
                                            C.byref(e), _hptr(v), _hptr(g), C.byref(info))
        self._check(st, (NOT_CONVERGED,) if allow_not_converged else ())
        return float(v[0]), g, info

    def lml_grad_batched(self, desc, x, y, H, est=None):
        x, y = _dev_f64(x), _dev_f64(y)
        H = np.ascontiguousarray(np.asarray(H, dtype=np.float64))
        B, nh = H.shape
        d = desc_of(desc)
        e = est or estimator()
        v = np.zeros(B)
        g = np.zeros((B, nh))
        ms = np.zeros(B, dtype=np.int32)
        infos = (Info * B)()
        self._check(self.lib.sdgp_lml_grad_batched(self.h, C.byref(d), _ptr(x), _ptr(y), x.shape[0],
                                                   _hptr(H), B, C.byref(e), _hptr(v), _hptr(g), _hptr(ms),
                                                   C.cast(infos, VP)))
        return v, g, ms, list(infos)

    def train_de(self, desc, x, y, H, lo, hi, est=None, generations=10, F=0.7, CR=0.9, seed=0,
                 objective=DE_LML, requirement=1.0, domain_volume=1.0):
        """Differential evolution over the population H (B, nh) with one
        batched evaluation per generation; returns (H, fit, history)."""
        x, y = _dev_f64(x), _dev_f64(y)
        H = _f64(H).copy()
        lo, hi = _f64(lo), _f64(hi)
        B, nh = H.shape
        d = desc_of(desc)
        e = est or estimator()
        o = DeOptions(int(generations), float(F), float(CR), int(seed), int(objective), float(requirement),
                      float(domain_volume))
        fit = np.zeros(B)
        hist = np.zeros(int(generations) + 1)
        self._check(self.lib.sdgp_train_de(self.h, C.byref(d), _ptr(x), _ptr(y), x.shape[0], H.ctypes.data, B,
                                           lo.ctypes.data, hi.ctypes.data, C.byref(e), C.byref(o),
                                           fit.ctypes.data, hist.ctypes.data))
        return H, fit, hist

    def logdet_taylor(self, desc, x, h, probes=32, terms=50, seed=0):
        """Randomised Taylor-series log-det; returns (logdet, alpha)."""
        x = _dev_f64(x)
        hh = self._h(h)
        d = desc_of(desc)
        ld, al = D(0.0), D(0.0)
        self._check(self.lib.sdgp_logdet_taylor(self.h, C.byref(d), _ptr(x), x.shape[0], _hptr(hh), int(probes),
                                                int(terms), int(seed), C.byref(ld), C.byref(al)))
        return float(ld.value), float(al.value)

    def posterior_mean_var(self, desc, x, y, h, x0, est=None):
        import torch
        x, y, x0 = _dev_f64(x), _dev_f64(y), _dev_f64(x0)
        hh = self._h(h)
        d = desc_of(desc)
        e = est or estimator(kind=PROBE_RADEMACHER, probes=1)
        n0 = x0.shape[0]
        mean = torch.empty(n0, dtype=torch.float64, device=x.device)
        var = torch.empty(n0, dtype=torch.float64, device=x.device)
        self._check(self.lib.sdgp_posterior_mean_var(self.h, C.byref(d), _ptr(x), _ptr(y), x.shape[0],
                                                     _hptr(hh), _ptr(x0), n0, C.byref(e), _ptr(mean),
                                                     _ptr(var)))
        return mean, var

"""The C-ABI library loads and exports every function include/sdgp.h
declares (no GPU needed: no compute call is made)."""
import ctypes
import os

import pytest

from paper_2205_09070_amd import _lib


def test_header_declares_the_boundary():
    names = _lib.header_functions()
    for fn in ("sdgp_kernel_assemble", "sdgp_lml", "sdgp_lml_grad", "sdgp_posterior_mean_var",
               "sdgp_lml_grad_batched", "sdgp_create", "sdgp_destroy", "sdgp_last_error"):
        assert fn in names


@pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libsdgp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _lib.header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding's signature table covers the header exactly
    assert sorted(_lib._SIGS) == _lib.header_functions()


@pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libsdgp.so not built")
def test_num_hyper_without_gpu():
    lib = _lib.load()
    d = _lib.KernelDesc(3, 16, 4, 0, 1)
    assert lib.sdgp_num_hyper(ctypes.byref(d)) == 2 + 16 * 4 * 6 + 1
    bad = _lib.KernelDesc(5, 1, 1, 0, 1)
    assert lib.sdgp_num_hyper(ctypes.byref(bad)) == -1
    big = _lib.KernelDesc(2, 65, 1, 0, 1)
    assert lib.sdgp_num_hyper(ctypes.byref(big)) == -1


def test_product_path_refuses_without_gpu(monkeypatch):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libsdgp.so not built")
    with pytest.raises(RuntimeError):
        _lib.Context(0)

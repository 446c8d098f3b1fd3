"""Helpers for GPU tests: context, tensors, CSR conversions, tolerances."""
import sys

import numpy as np
import pytest
import scipy.sparse as ssp

K_REL = 1e-13          # stored K entries, relative
K_ABS_SCALE = 1e-15    # ... or absolute, times max_a K_aa
LML_REL = 1e-6
GRAD_REL = 1e-5


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def ctx(timing=False):
    import paper_2205_09070_amd as sd
    return sd.Context(0, timing=timing)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def csr_to_host(row_ptr, col, val, n):
    rp = row_ptr.cpu().numpy()
    c = col.cpu().numpy()
    v = val.cpu().numpy()
    return rp, c, v, ssp.csr_matrix((v, c, rp), shape=(n, n))


def check_k_entries(got, want, scale):
    err = np.abs(got - want)
    ok = (err <= K_REL * np.abs(want)) | (err <= K_ABS_SCALE * scale)
    return ok


def grad_close(g, g0, rel=GRAD_REL):
    """Per-component relative check with a floor of 1e-6 of the largest
    component (components that are exactly representable zeros compare
    absolutely)."""
    floor = 1e-6 * np.abs(g0).max()
    return np.abs(g - g0) <= rel * np.maximum(np.abs(g0), floor)

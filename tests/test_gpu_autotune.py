"""The CG launch-shape autotuner on the GPU.

* A context with autotune = 2 tunes on its first solve (last_tuned = 2),
  writes the chosen shape to the store (SDGP_TUNE_CACHE), and its LML and
  gradient agree to rounding with the untuned defaults (the shape changes
  only the order of floating-point sums).
* A second context reads the stored shape back (last_tuned = 1) and
  reproduces the tuned result bitwise.
* Explicit launch-shape options switch the tuner off (last_tuned = 0)."""
import json

import numpy as np
import pytest

from paper_2205_09070_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def test_autotune_agrees_with_defaults_and_persists(tmp_path, monkeypatch):
    gu.need_gpu()
    import paper_2205_09070_amd as sd
    store = tmp_path / "autotune.json"
    monkeypatch.setenv("SDGP_TUNE_CACHE", str(store))
    w = wl.random_small(20000, 3, 8, 4, 3, combine=1, per_row=25.0, noise_var=1e-2)
    est = sd.estimator(probes=16, seed=4, cg_rtol=1e-10, cg_max_iter=5000, precond=sd.PRECOND_LOWRANK,
                       operator_form=sd.OPERATOR_FACTORED)
    x, y = gu.dev(w.x), gu.dev(w.y)
    gu.log("autotune off")
    c0 = gu.ctx()
    c0.set_option("autotune", 0)
    v0, g0, i0 = c0.lml_grad(w.desc, x, y, w.h, est)
    assert c0.get_option("last_tuned") == 0
    gu.log("autotune on (trials)")
    c1 = gu.ctx()
    c1.set_option("autotune", 2)
    v1, g1, i1 = c1.lml_grad(w.desc, x, y, w.h, est)
    assert c1.get_option("last_tuned") == 2
    shape = tuple(c1.get_option(k) for k in ("last_spmm_blocks", "last_update_blocks", "last_union_spmm",
                                              "last_fw_mfma"))
    gu.log("  tuned shape %s; lml %.15g vs %.15g, iters %d vs %d" % (shape, v1, v0, i1.cg_iters, i0.cg_iters))
    assert abs(i1.cg_iters - i0.cg_iters) <= 2
    assert abs(v1 - v0) <= 1e-10 * abs(v0)
    assert gu.grad_close(g1, g0, rel=1e-8).all()
    doc = json.load(open(store))
    assert len(doc) == 1
    key, ent = next(iter(doc.items()))
    assert key.startswith("gfx")
    assert (ent["spmm_blocks"], ent["update_blocks"], ent["union_spmm"], ent["fw_mfma"]) == shape
    assert ent["ms_per_iter"] > 0.0 and ent["ms_per_iter"] <= ent["default_ms_per_iter"]
    assert sd.tune_cache_get(str(store), key) == shape
    gu.log("second context reads the store")
    c2 = gu.ctx()
    c2.set_option("autotune", 2)
    v2, g2, _ = c2.lml_grad(w.desc, x, y, w.h, est)
    assert c2.get_option("last_tuned") == 1
    assert v2 == v1 and np.array_equal(g2, g1)
    gu.log("explicit options switch the tuner off")
    c2.set_option("spmm_blocks", 8192)
    c2.lml_grad(w.desc, x, y, w.h, est)
    assert c2.get_option("last_tuned") == 0
    assert c2.get_option("last_spmm_blocks") == min(8192, ((20000 + 15) // 16 + 7) // 8 * 8)
    with pytest.raises(sd.SdgpError):
        c2.set_option("autotune", 3)

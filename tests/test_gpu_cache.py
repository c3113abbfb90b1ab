"""GPU tests of the process-wide device block cache (pmx_device_cache).

A destroyed factor leaves its blocks in the cache, a later factor of the same workload
solves to the same result from reused (not zeroed) blocks, and a limit of 0 empties the
cache.
"""
import numpy as np
import pytest

from oracle import dense
from paper_2603_09381_amd import workloads as W

pytestmark = pytest.mark.gpu


def _solve(pmx, w, **kw):
    import torch
    fac = pmx.Factor(w, pmx.options(w, **kw))
    d = fac.solve_plane_waves(w.angles)
    torch.cuda.synchronize()
    x = pmx.dens_to_numpy(d, w)
    fac.close()
    return x


@pytest.mark.parametrize("form", [dict(precision=0, id_tol=1e-10), dict(precision=1, id_tol=1e-3, ir_tol=1e-10)])
def test_cache_reuse_and_release(pmx, form):
    w = W.sub_grid(W.config2(), 4)
    ref = dense.solve(w)
    pmx.device_cache(0)                  # empties the cache (and sets its limit to 0)
    assert pmx.device_cache() == 0
    pmx.device_cache(8 << 30)            # the default limit: destroyed factors fill it again
    x1 = _solve(pmx, w, **form)
    held = pmx.device_cache()
    print("cache after one factor:", held, "bytes")
    assert held > 0
    x2 = _solve(pmx, w, **form)          # blocks come from the cache
    bound = 5e-9 if form["precision"] == 0 else 1e-8
    assert dense.rel_error(x1, ref) < bound
    assert dense.rel_error(x2, ref) < bound
    assert dense.rel_error(x2, x1) < 1e-12
    pmx.device_cache(0)
    assert pmx.device_cache() == 0
    pmx.device_cache(8 << 30)            # the default limit again

"""The allocation-free far field (pmx_far_field_noalloc) against pmx_far_field.

Both run the same kernels with the same split of the node sum; the allocation-free entry
point keeps its partial sums in the library's static per-GPU array instead of an
allocated buffer.  Two calls in a row, the second smaller, so that what the first left
in the array cannot leak into the second; sizes beyond the array are refused before any
GPU work."""
import numpy as np
import pytest

from paper_2603_09381_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_far_field_noalloc_matches_the_allocating_entry_point(pmx):
    import torch
    w = W.sub_grid(W.config2(), 4)
    fac = pmx.Factor(w)
    dens = fac.solve_plane_waves(w.angles)
    torch.cuda.synchronize()
    cases = [(dens, np.linspace(0.0, 2 * np.pi, 203)),            # 4 right-hand sides, 203 directions
             (dens[1:3].contiguous(), np.linspace(0.1, 3.0, 9))]   # then fewer of both
    for d, dirs in cases:
        print("far field noalloc case", tuple(d.shape), len(dirs), flush=True)
        ref = fac.far_field(d, dirs).cpu().numpy()
        out = torch.full((d.shape[0], len(dirs)), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
        got = fac.far_field_noalloc(d, dirs, out=out)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    fac.close()


def test_far_field_noalloc_refuses_sizes_beyond_its_array(pmx):
    import torch
    w = W.config1()
    fac = pmx.Factor(w)
    dens = fac.solve_plane_waves(w.angles)
    torch.cuda.synchronize()
    dirs = np.linspace(0.0, 2 * np.pi, 600000)    # 600000 pairs x 16 B > 8 MiB
    with pytest.raises(pmx.PmxError, match="PMX_EINVAL"):
        fac.far_field_noalloc(dens, dirs)
    fac.close()

"""Frequency sweep (Sec. 4.3): compressed size, error and time against the angular frequency
at 64 inclusions (8 x 8 stars, 200 nodes each, eps- = 5), CPQR thresholds 1e-6, 1e-9,
1e-12."""
import numpy as np
import pytest

from oracle import dense

pytestmark = pytest.mark.gpu

OMEGAS = (1, 2, 4, 8)
TOLS = (1e-6, 1e-9, 1e-12)


def test_compressed_size_against_frequency(pmx):
    from paper_2603_09381_amd import sweep
    rows, refs = sweep.frequency_sweep(omegas=OMEGAS, tols=TOLS)
    size = {}
    for r in rows:
        print({k: r[k] for k in ("omega", "id_tol", "root_size", "rel_error_vs_ref", "factor_s")}, flush=True)
        size[(r["omega"], r["id_tol"])] = r["root_size"]
        # the threshold bounds the error of the compressed solve (Sec. 4.3, low frequencies)
        assert r["rel_error_vs_ref"] < 1e2 * r["id_tol"]
    for om in OMEGAS:
        # a stricter threshold keeps more skeletons at every frequency
        s = [size[(om, t)] for t in TOLS]
        assert all(b > a for a, b in zip(s, s[1:])), (om, s)
    for tol in TOLS:
        # the frequency half of the O(omega D) bound: doubling omega at most doubles the
        # compressed size
        for a, b in zip(OMEGAS, OMEGAS[1:]):
            assert size[(b, tol)] <= (b / a) * size[(a, tol)], (tol, a, b)
    # each reference (threshold 1e-14) against the oracle's FP64 rows of f - A x
    for om, (w, xr) in refs.items():
        x = pmx.dens_to_numpy(xr, w)
        idx = np.sort(np.random.default_rng(int(om)).choice(w.n_unknowns, size=16, replace=False))
        f = dense.rhs(dense.Geometry(w), w.angles)[idx]
        res = np.linalg.norm(dense.residual_rows(w, x, idx)) / np.linalg.norm(f)
        print("omega", om, "reference sampled residual", res, flush=True)
        assert res < 1e-11

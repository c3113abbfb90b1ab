"""GPU parity of the learned-skeleton form: the network's forward and backward passes against
the numpy oracle, the training labels (leaf IDs, independent of the interior contrast by
the Omit structure), and factorisations whose leaf IDs start from learned proposals (with
the judge and the full-CPQR fallback) against the dense solve."""
import numpy as np
import pytest

from oracle import dense, mlp
from paper_2603_09381_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_mlp_forward_backward_against_oracle(pmx):
    rng = np.random.default_rng(77)
    shape = (20, 64, 3, 8)
    off, npar = mlp.offsets(shape)
    p = np.zeros(npar)
    d = mlp.dims(shape)
    for l in range(len(d) - 1):
        w0, w1 = off[2 * l]
        p[w0:w1] = rng.standard_normal(w1 - w0) * np.sqrt(2.0 / d[l])
        b0, b1 = off[2 * l + 1]
        p[b0:b1] = 0.1 * rng.standard_normal(b1 - b0)
    p = p.astype(np.float32)
    B = 300
    X = rng.standard_normal((B, 20)).astype(np.float32)
    Y = np.concatenate([(rng.random((B, 4)) < 0.4), rng.random((B, 4))], axis=1).astype(np.float32)
    out, grad, loss = pmx.probe_mlp(shape, p, X, Y, wmse=10.0)
    rout, rloss, rgrad = mlp.value_and_grad(p.astype(float), shape, X.astype(float), Y.astype(float), 10.0)
    # FP32 products and sums of <= 300 terms against FP64
    assert np.abs(out - rout).max() < 2e-5 * np.abs(rout).max()
    assert abs(loss - rloss) < 2e-5 * abs(rloss)
    assert np.abs(grad - rgrad).max() < 1e-4 * np.abs(rgrad).max()


def test_leaf_labels_independent_of_contrast(pmx, tmp_path):
    """Leaf IDs use the exterior kernel only (Omit form): changing k- changes one input
    feature and no label."""
    a = W.random_shape_grid(4, 11, 8.0, contrast=1.5)
    b = W.random_shape_grid(4, 11, 8.0, contrast=3.0)
    pa, pb = tmp_path / "a.ids", tmp_path / "b.ids"
    pmx.id_dataset(a, pa)
    pmx.id_dataset(b, pb)
    Xa, Ya = pmx.read_dataset(pa)
    Xb, Yb = pmx.read_dataset(pb)
    assert Xa.shape == (16 * 128, 20) and Ya.shape == (16 * 128, 8)
    assert np.array_equal(Ya, Yb)
    diff = np.flatnonzero(np.any(Xa != Xb, axis=0))
    assert list(diff) == [2]
    # every node label is a 0/1 membership and the skeleton sizes match the rank fractions
    assert set(np.unique(Ya[:, :4])) <= {0.0, 1.0}
    for c in range(16):
        blk = Ya[c * 128:(c + 1) * 128]
        assert np.allclose(blk[:, :4].sum(axis=0) / 128.0, blk[0, 4:])


def _train(pmx, tmp_path, ngeo=6, epochs=40):
    data, model = tmp_path / "train.ids", tmp_path / "model.bin"
    for i in range(ngeo):
        w = W.random_shape_grid(8, 20 + i, 6.0 + 3.0 * i)
        pmx.id_dataset(w, data, append=i > 0)
    loss = pmx.mlp_train(data, model, epochs=epochs, batch=1024, seed=3)
    return model, loss


def _write_model(path, shape, params, mean, istd):
    with open(path, "wb") as f:
        f.write(b"PMXMLP01")
        f.write(np.asarray(shape, np.int32).tobytes())
        f.write(np.asarray(mean, np.float32).tobytes())
        f.write(np.asarray(istd, np.float32).tobytes())
        f.write(np.asarray([len(params)], np.int64).tobytes())
        f.write(np.asarray(params, np.float32).tobytes())


def _solve(pmx, w, **kw):
    import torch
    fac = pmx.Factor(w, pmx.options(w, **kw))
    dens = fac.solve_plane_waves(w.angles)
    torch.cuda.synchronize()
    return fac, pmx.dens_to_numpy(dens, w)


def test_learned_ids_train_and_solve(pmx, tmp_path):
    model, loss = _train(pmx, tmp_path)
    print("final training loss", loss)
    w = W.random_shape_grid(4, 40, 12.0, angles=[0.0, 1.1])
    fac, x = _solve(pmx, w, learned=1, model_path=str(model))
    info = fac.info()
    print("learned cells", info.id_learned, "fallback", info.id_fallback)
    assert info.id_learned + info.id_fallback == 16 and info.id_learned >= 8
    ref = dense.solve(w)
    assert dense.rel_error(x, ref) < 5e-9
    _, xf = _solve(pmx, w)
    assert dense.rel_error(x, xf) < 5e-9
    # predictions for every node, ranks in (0, 1]
    pred = pmx.mlp_predict(model, w)
    assert pred.shape == (w.node_off[-1], 8) and np.isfinite(pred).all()


def test_poor_proposals_fall_back(pmx, tmp_path):
    """A network with random weights proposes poor candidates and small ranks: the judge
    rejects them, the full CPQR takes over and the solution is unchanged."""
    rng = np.random.default_rng(5)
    shape = (20, 32, 1, 8)
    _, npar = mlp.offsets(shape)
    path = tmp_path / "random.bin"
    _write_model(path, shape, 0.05 * rng.standard_normal(npar), np.zeros(20), np.ones(20))
    w = W.random_shape_grid(4, 41, 10.0)
    fac, x = _solve(pmx, w, learned=1, model_path=str(path))
    info = fac.info()
    assert info.id_fallback > 0 and info.id_learned + info.id_fallback == 16
    assert dense.rel_error(x, dense.solve(w)) < 5e-9


def test_learned_rejects_bad_model_file(pmx, tmp_path):
    w = W.random_shape_grid(2, 42, 10.0)
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a model")
    with pytest.raises(pmx.PmxError) as e:
        pmx.Factor(w, pmx.options(w, learned=1, model_path=str(bad)))
    assert e.value.status == 1


def test_learned_gain_is_measured(pmx, tmp_path):
    """What the trained network gains over the full leaf IDs (the adaptive-rank ID of Sec. 3
    at the leaves): a network trained on 2048 seeded cells (eight 16x16 training grids of
    random shapes), then factorisations of a 16x16 grid of other random shapes at
    k+ in {5, 10, 20} with and without it.  The leaf-ID stage time, the leaf QR + CPQR kernel
    time and the factor time of both are reported; the proposals settle most cells, the
    rest fall back, and the solution equals the full one to the ID tolerance."""
    import json
    from paper_2603_09381_amd import skeleton_net
    model = tmp_path / "net.bin"
    loss, t_lab, t_train = skeleton_net.train(model, cells=2048, grid=16, epochs=20, seed=3)
    print("training: loss", loss, "labels s", t_lab, "training s", t_train)
    rows = skeleton_net.gain(model, grid=16, ks=(5.0, 10.0, 20.0), reps=2)
    for r in rows:
        print(json.dumps(r))
        assert r["learned_cells"] + r["fallback_cells"] == 256
        assert r["learned_cells"] >= 128
        assert r["rel_diff"] < 5e-9
        assert r["leaf_id_ms"]["full"] > 0 and r["leaf_id_ms"]["learned"] > 0

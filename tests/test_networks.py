"""The generated min/max networks (csrc/gen_networks.py -> csrc/medtile.inc), on the CPU.

Each tile network must select, for every output, the median of that output's window: by
the 0-1 principle a min/max network that selects rank m on all 0/1 inputs selects it on
all inputs, so random 0/1 vectors with densities spread over [0, 1] (which put the median
boundary everywhere) and small-integer inputs with many ties are checked against a sort of
each window.  The committed medtile.inc must be exactly what the generator writes, so the
kernels compile the networks checked here.  The 25-value sort used by the replacement is
checked on random 0/1 vectors and random floats against numpy's sort.
"""
import os
import sys

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_1008_2192_amd", "csrc")
sys.path.insert(0, CSRC)
import gen_networks  # noqa: E402


@pytest.mark.parametrize("name,k,ty,tx", gen_networks.TILES, ids=[t[0] for t in gen_networks.TILES])
def test_tile_network_selects_every_window_median(name, k, ty, tx):
    tm = gen_networks.TileMedian(k, ty, tx).build()
    assert gen_networks.check_tile(tm, trials=20000, seed=11)
    # and on continuous values with the window medians from numpy
    rng = np.random.default_rng(12)
    X = rng.normal(0.0, 1.0, (4000, tm.ph * tm.pw))
    outs = [tm.outputs[(i, j)] for i in range(ty) for j in range(tx)]
    got = gen_networks.evaluate_np(tm.net, [X[:, i] for i in range(X.shape[1])], outs)
    P = X.reshape(-1, tm.ph, tm.pw)
    for idx, (i, j) in enumerate((i, j) for i in range(ty) for j in range(tx)):
        win = P[:, i:i + k, j:j + k].reshape(len(X), -1)
        np.testing.assert_array_equal(got[idx], np.median(win, axis=1), err_msg=f"{name} {i},{j}")


def test_committed_networks_are_the_generated_ones(tmp_path):
    out = tmp_path / "medtile.inc"
    gen_networks.generate(str(out), verify=False)
    with open(os.path.join(CSRC, "medtile.inc")) as f:
        committed = f.read()
    assert out.read_text() == committed


def _sort_net(X):
    X = X.copy()
    for i, j in gen_networks.batcher_pairs(X.shape[1]):
        a, b = X[:, i].copy(), X[:, j].copy()
        X[:, i] = np.minimum(a, b)
        X[:, j] = np.maximum(a, b)
    return X


def test_sort25_network():
    rng = np.random.default_rng(13)
    p = rng.random((1 << 16, 1))
    Z = (rng.random((1 << 16, 25)) < p).astype(np.int8)
    np.testing.assert_array_equal(_sort_net(Z), np.sort(Z, axis=1))
    F = rng.integers(0, 6, (20000, 25)).astype(np.float64) + rng.normal(0, 1, (20000, 1))
    np.testing.assert_array_equal(_sort_net(F), np.sort(F, axis=1))
    assert len(gen_networks.batcher_pairs(25)) == 138


def test_25_input_networks_on_every_01_vector():
    """Exhaustive 0-1 check of the two 25-input networks: the single-output 5x5 median
    (the work set's med5 of S) and the 25-value sort, over all 2^25 0/1 vectors in chunks
    of 2^20 (the tile networks with 30, 36 and 49 inputs are checked on samples above)."""
    tm = gen_networks.TileMedian(5, 1, 1).build()
    out = [tm.outputs[(0, 0)]]
    pairs = gen_networks.batcher_pairs(25)
    shifts = np.arange(25, dtype=np.uint32)
    for c in range(32):
        idx = np.arange(c << 20, (c + 1) << 20, dtype=np.uint32)
        Z = np.asfortranarray(((idx[:, None] >> shifts[None, :]) & 1).astype(np.int8))
        ones = Z.sum(axis=1, dtype=np.int32)
        med = gen_networks.evaluate_np(tm.net, [Z[:, i] for i in range(25)], out)[0]
        np.testing.assert_array_equal(med, (ones >= 13).astype(np.int8), err_msg=f"chunk {c}")
        S = Z.copy(order="F")
        for i, j in pairs:
            a = S[:, i].copy()
            np.minimum(a, S[:, j], out=S[:, i])
            np.maximum(a, S[:, j], out=S[:, j])
        # sorted 0/1 rows: zeros, then exactly `ones` ones
        np.testing.assert_array_equal(S.sum(axis=1, dtype=np.int32), ones)
        assert bool((np.diff(S, axis=1) >= 0).all()), f"chunk {c}"

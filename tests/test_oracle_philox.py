"""Pins for the counter-based sampler: published Philox4x32-10 known-answer
vectors and the distribution of the Box-Muller normals (Lemma 1 bound on the
sample mean, second moment, antithetic symmetry)."""
import json
import os

import numpy as np
import pytest
import scipy.stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def test_known_answer_vectors():
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")) as f:
        kat = json.load(f)
    for v in kat["vectors"]:
        ctr = [int(c, 16) for c in v["counter"]]
        key = [int(k, 16) for k in v["key"]]
        out = [int(x) for x in philox.philox4x32_10(ctr, key)]
        assert out == [int(x, 16) for x in v["output"]]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_normals_are_standard_gaussian(dtype):
    n, K = 37, 4000
    Z = philox.normals(n, K, seed=12345, stream=7, dtype=dtype)
    assert Z.shape == (n, K)
    flat = Z.reshape(-1)
    # Lemma 1: E|mean| <= sqrt(tr Sigma / count) = 1/sqrt(count); allow 4x
    assert abs(flat.mean()) < 4.0 / np.sqrt(flat.size)
    assert abs(flat.var() - 1.0) < 0.02
    assert scipy.stats.kstest(flat, "norm").pvalue > 1e-4
    # rows are not copies of each other
    assert abs(np.corrcoef(Z[0], Z[1])[0, 1]) < 0.1


def test_antithetic_layout_and_streams_differ():
    W = philox.perturbations(10, 64, 0.5, seed=3, stream=0, dtype="f32")
    np.testing.assert_array_equal(W[:, 32:], -W[:, :32])
    W2 = philox.perturbations(10, 64, 0.5, seed=3, stream=1, dtype="f32")
    assert np.abs(W - W2).max() > 0.1

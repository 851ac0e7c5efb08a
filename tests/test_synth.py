"""Seeded generators: reproducible, in range, with the stated moments."""
import numpy as np

import synth


def test_pair_reproducible_and_ordered():
    A1, B1 = synth.pair(8, 6, 5, seed=0)
    A2, B2 = synth.pair(8, 6, 5, seed=0)
    assert np.array_equal(A1, A2) and np.array_equal(B1, B2)
    assert A1.dtype == np.float32 and A1.shape == (8, 5) and B1.shape == (5, 6)
    # A is drawn first from the stream, then B
    g = synth.rng(0)
    assert np.array_equal(A1, synth.draw(g, (8, 5)))
    assert np.array_equal(B1, synth.draw(g, (5, 6)))


def test_distributions():
    g = synth.rng(1)
    u = synth.draw(g, (200_000,), "uniform")
    assert u.min() >= -1 and u.max() <= 1 and abs(u.mean()) < 0.01 and abs(u.var() - 1 / 3) < 0.01
    z = synth.draw(g, (200_000,), "normal")
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01
    w = synth.draw(g, (200_000,), "wide")
    e = np.log2(np.abs(w.astype(np.float64)))
    assert e.min() >= -8 - 1e-6 and e.max() <= 8 + 1e-6 and abs(np.mean(w > 0) - 0.5) < 0.01
    wi = synth.draw(g, (10_000,), "wide_int")
    ei = np.log2(np.abs(wi.astype(np.float64)))
    assert np.array_equal(ei, np.round(ei))
    r = synth.draw(g, (10_000,), "integers", R=7)
    assert r.min() == -7 and r.max() == 7 and np.array_equal(r, np.round(r))


def test_loguniform_dims_and_arrivals():
    d = synth.loguniform_dims(5000, 32, 1024, seed=0)
    assert d.shape == (5000, 3) and d.min() >= 32 and d.max() <= 1024
    # log-uniform: the median of log(d) sits at the middle of [ln 32, ln 1024]
    assert abs(np.median(np.log(d)) - 0.5 * (np.log(32) + np.log(1024))) < 0.05
    t = synth.poisson_arrivals(20000, 1000.0, seed=0)
    assert t[0] == 0 and np.all(np.diff(t) >= 0)
    assert abs(np.mean(np.diff(t)) - 1e-3) < 3e-5
    mix = synth.dtype_mix(20000, seed=0)
    assert abs(np.mean(mix == 0) - 0.5) < 0.02 and abs(np.mean(mix == 2) - 0.15) < 0.02

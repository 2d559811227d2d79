"""Pins of the Philox generator and checks of the seeded workload data (CPU only)."""
import os

import numpy as np

import workloads as wl
from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    n = 0
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        ctr, key, out = (tuple(int(v, 16) for v in part.split()) for part in line.split("|"))
        got = philox.philox4x32_10(*[np.array([c], np.uint64) for c in ctr], *key)
        assert tuple(int(v[0]) for v in got) == out
        n += 1
    assert n == 3


def test_philox_gaussian_moments():
    Om = philox.gaussian_omega(20001, 8, seed=123, counter=5)
    assert Om.shape == (20001, 8)
    assert abs(Om.mean()) < 0.02 and abs(Om.std() - 1) < 0.02
    assert abs(np.mean(Om ** 4) - 3) < 0.1
    assert not np.allclose(Om, philox.gaussian_omega(20001, 8, seed=123, counter=6))


def test_workloads_deterministic_and_shaped():
    a, b = wl.config("c2", seed=0), wl.config("c2", seed=0)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.g, b.g)
    assert a.n_rows == 4608 and a.n_params == 8577
    assert not np.array_equal(a.X, wl.config("c2", seed=1).X)
    c1 = wl.config("c1")
    assert c1.n_rows == 1020 and c1.n_params == 1185 and c1.lam == 1e-6
    c3 = wl.config("c3")
    assert c3.n_rows == 18432 and c3.n_params == 33921 and c3.ell == 800
    c4 = wl.config("c4")
    assert c4.n_rows == 10240 and c4.n_params == 12801
    for p, meas_b in [(c1, 4.0), (a, 4.0), (c3, 10.0)]:
        inner = p.kind == wl.KIND_INTERIOR
        assert abs(p.w[inner].sum() - 1) < 1e-12 and abs(p.w[~inner].sum() - meas_b) < 1e-12
        assert p.X.min() >= 0 and p.X.max() <= 1
        xb = p.X[~inner]
        assert np.all(np.any((xb == 0) | (xb == 1), axis=1))
    assert np.all(c4.X[c4.kind == wl.KIND_INITIAL][:, 2] == 0)
    th = wl.glorot_theta((2, 64, 64, 1), 0)
    assert th.size == wl.num_params((2, 64, 64, 1)) and np.abs(th).max() <= np.sqrt(6 / 65)  # largest bound: the 64 -> 1 layer

"""Checks of the seeded input generators (no method arithmetic involved)."""

import math

import numpy as np

import workloads


def _min_pair_distance(Y, L):
    from scipy.spatial import cKDTree
    t = cKDTree(np.mod(Y, L), boxsize=L)
    d, _ = t.query(np.mod(Y, L), k=2)
    return d[:, 1].min()


def test_small_workload_is_seeded_and_non_overlapping():
    w1 = workloads.workload(0)
    w2 = workloads.workload(0)
    assert np.array_equal(w1["Y"], w2["Y"]) and np.array_equal(w1["F"], w2["F"])
    assert w1["N"] == 64 and w1["grid"] == 32 and w1["M_G"] == 12
    assert _min_pair_distance(w1["Y"], w1["L"]) >= 2.0 - 1e-12
    assert np.abs(w1["F"].sum(0)).max() < 1e-12          # net force removed
    assert w1["R_c"] < w1["L"] / 2


def test_dilute_workload_fraction_and_overlap():
    w = workloads.workload(1, N=2000)
    phi = w["N"] * 4 * math.pi / 3 / w["L"] ** 3
    assert abs(phi - 0.01) < 1e-12
    assert _min_pair_distance(w["Y"], w["L"]) >= 2.0 - 1e-12
    assert np.all((w["Y"] >= 0) & (w["Y"] < w["L"]))


def test_rod_workload_geometry():
    w = workloads.workload(3, N=300)
    Y = w["Y"]
    assert Y.shape == (300, 3)
    assert np.all(Y[:, 0] >= 0) and np.all(Y[:, 0] < w["L"] / 2)
    rods = Y.reshape(-1, 30, 3)
    d = np.diff(rods, axis=1)
    d -= w["L"] * np.round(d / w["L"])
    assert np.allclose(np.linalg.norm(d, axis=2), 2.0)
    assert _min_pair_distance(Y, w["L"]) >= 2.0 - 1e-9
    assert np.all(w["T"] == 0)


def test_serving_stream_draws():
    reqs = workloads.serving_stream(n_requests=64, rate=100.0)
    Ns = np.array([r["N"] for r in reqs])
    assert Ns.min() >= 1000 and Ns.max() <= 200_000
    for r in reqs:
        g = r["grid"]
        assert g % 2 == 0 and g >= 1.5 * r["L"] / r["Sigma"]
        m = g
        while m % 2 == 0:
            m //= 2
        while m % 3 == 0:
            m //= 3
        assert m == 1
        assert r["R_c"] < r["L"] / 2
    arr = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(arr) >= 0)

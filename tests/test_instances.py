"""The seeded Monte Carlo input generator."""
import math

import numpy as np

from paper_2404_18034_amd import instances as I


def test_splitmix64_published_vector():
    # SplitMix64 seeded with 1234567 (reference sequence of the generator's authors)
    g = 0x9E3779B97F4A7C15
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    got = [int(I.splitmix64(np.uint64((1234567 + i * g) % 2 ** 64))) for i in range(5)]
    assert got == want


def test_instances_are_counter_based():
    a = I.make_instances("C2", B=64)
    b = I.make_instances("C2", ids=[5, 63, 17])
    for k in ("x0", "xf", "params", "K"):
        np.testing.assert_array_equal(a[k][[5, 63, 17]], b[k])


def test_dispersion_ranges_and_tilt():
    inst = I.make_instances("C1", B=2000)
    x0 = inst["x0"]
    assert np.all(np.abs(x0[:, 1:4] - [4, 4, 0]) <= 0.5 + 1e-6)
    assert np.all(np.abs(x0[:, 4:7] - [-1, -2, 0]) <= 0.2 + 1e-6)
    assert np.all(np.abs(x0[:, 0] - 2.0) <= 0.05 + 1e-6)
    np.testing.assert_array_equal(inst["params"][:, 0], x0[:, 0])
    # tilt = angle between body x axis and vertical: cos(tilt) = C11 = 1 - 2 (q2^2 + q3^2)
    q = x0[:, 7:11]
    c11 = 1 - 2 * (q[:, 2] ** 2 + q[:, 3] ** 2)
    tilt = np.degrees(np.arccos(np.clip(c11, -1, 1)))
    assert tilt.max() <= 10.0 + 1e-3 and tilt.max() > 9.0
    assert np.all(q[:, 1] == 0.0)                          # rotation about a horizontal axis
    np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-7)
    # uniform: mean of a U(-0.5, 0.5) dispersion is near 0
    assert abs(np.mean(x0[:, 1] - 4.0)) < 0.03


def test_uneven_k_and_inertia_dispersion():
    c2 = I.make_instances("C2", B=3000)
    vals, counts = np.unique(c2["K"], return_counts=True)
    assert list(vals) == [10, 20, 30] and counts.min() > 900
    c4 = I.make_instances("C4", B=500)
    J = c4["params"][:, 6:9]
    assert np.all(np.abs(J / 0.01 - 1) <= 0.1 + 1e-6) and np.std(J[:, 0]) > 0
    assert np.all(c4["params"][:, 10:12] == 0.0)          # lateral r_T stays zero


def test_fp32_configs_are_float32_exact():
    inst = I.make_instances("C1", B=50)
    for k in ("x0", "xf", "params"):
        np.testing.assert_array_equal(inst[k], inst[k].astype(np.float32).astype(np.float64))
    c0 = I.make_instances("C0")
    assert c0["x0"][0, 1] == 4.0 and c0["params"][0, 14] == math.radians(20.0)

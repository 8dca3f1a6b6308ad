"""The seeded input generators (no arithmetic of the method): shapes,
determinism, and the distributions they claim."""
import numpy as np

from paper_1405_7487_amd import workloads as W


def test_sphere_surface_is_uniform_on_the_unit_sphere():
    x, q, _ = W.sphere_surface(200_000, 5)
    r = np.linalg.norm(x, axis=1)
    assert np.max(np.abs(r - 1.0)) < 1e-14
    # uniform on the sphere: every coordinate is uniform in [-1, 1] (mean 0, variance 1/3)
    assert np.all(np.abs(x.mean(axis=0)) < 0.01)
    assert np.all(np.abs((x * x).mean(axis=0) - 1.0 / 3.0) < 0.01)
    # octants hold equal shares
    octant = (x[:, 0] > 0) * 4 + (x[:, 1] > 0) * 2 + (x[:, 2] > 0)
    share = np.bincount(octant, minlength=8) / x.shape[0]
    assert np.all(np.abs(share - 0.125) < 0.005)
    assert q.min() >= -1.0 and q.max() < 1.0


def test_generators_are_deterministic_and_configs_resolve():
    for name in W.CONFIGS:
        a = W.make_config(name, n=1000)
        b = W.make_config(name, n=1000)
        assert a[0].shape == (1000, 3) and a[1].shape == (1000,)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert W.CONFIGS["sphere4m"] == dict(n=1 << 22, dist="sphere", p=10, theta=0.4, ncrit=512)

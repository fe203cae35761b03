"""Seeded input generators: placements are non-overlapping hard spheres inside the
lysosome (Sec. III.1), axes are unit vectors, and the configuration samplers respect
their stated ranges."""
import numpy as np

from paper_1407_2737_amd import workloads as W


def _min_pair_distance(p):
    d = np.linalg.norm(p[:, None, :] - p[None, :, :], axis=2)
    d[np.arange(len(p)), np.arange(len(p))] = np.inf
    return d.min()


def test_random_placement_hard_spheres():
    n, R, d = 800, 120e-9, 12e-9
    p = W.place_random(n, R, d, 3)
    assert p.shape == (n, 3)
    assert np.all(np.linalg.norm(p, axis=1) <= R - d / 2 + 1e-18)
    assert _min_pair_distance(p) >= d * (1 - 1e-12)
    assert np.array_equal(p, W.place_random(n, R, d, 3))          # seeded
    assert abs(W.volume_fraction(n, R, d) - n * (d / (2 * R)) ** 3) < 1e-15


def test_lattice_with_maximal_disorder():
    n, R, d = 600, 120e-9, 12e-9
    p = W.place_lattice_disorder(n, R, d, 4)
    assert p.shape == (n, 3)
    assert np.all(np.linalg.norm(p, axis=1) <= R - d / 2 + 1e-15)
    assert _min_pair_distance(p) >= d * (1 - 1e-9)


def test_axes_are_unit_and_isotropic():
    a = W.axes_random_3d(20000, 5)
    assert np.allclose(np.linalg.norm(a, axis=1), 1.0)
    assert np.all(np.abs(a.mean(axis=0)) < 0.03)
    assert abs(np.mean(a[:, 0] ** 2) - 1 / 3) < 0.01
    b = W.axes_random_2d(1000, 6)
    assert np.allclose(b[:, 2], 0.0) and np.allclose(np.linalg.norm(b, axis=1), 1.0)


def test_config_samplers():
    c1 = W.lysosome_n100()
    assert c1.n == 100 and abs(c1.meta["phi"] - 0.0422) < 1e-3
    ps = W.uneven_batch_params()
    assert len(ps) == 256 and all(200 <= p["n"] <= 8000 for p in ps)
    d4 = W.replica_batch_geometry()[1]
    assert abs(d4 - 11.60e-9) < 0.01e-9
    reqs = W.request_stream(count=200)
    assert all(100 <= q["n"] <= 8000 and 3 <= q["P"] <= 10 for q in reqs)
    assert all(np.diff([q["t"] for q in reqs]) > 0)


def test_request_stream_prefix_does_not_depend_on_count():
    """The served bench takes its phases as slices of one stream: the first k requests
    (parameters and arrival times) are the same whatever the stream's length."""
    short, long = W.request_stream(count=18), W.request_stream(count=40)
    for a, b in zip(short, long):
        assert a == b

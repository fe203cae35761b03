"""Pins of the Stoner-Wohlfarth extremum search (Eq. 2, Sec. II.1 steps iv-v).

Closed forms (Stoner and Wohlfarth 1948): with the field along the axis (phi = 0) and
h < 1 the minima are theta = 0 and pi, the maxima cos theta = -h, the barriers
(1 + h)^2 and (1 - h)^2 in units of K V; with the field across the axis the minima
are arcsin h and pi - arcsin h; in zero field the barrier is K V; the switching field
at 45 degrees is h = 1/2, and two minima exist exactly inside the astroid."""
import numpy as np
import pytest

from oracle import sw


def test_field_along_axis():
    for h in (0.0, 0.1, 0.37, 0.8, 0.999):
        th, mn, cnt = sw.stationary_points(np.array([h]), np.array([0.0]))
        assert cnt[0] == 4
        mins = np.sort(th[0][mn[0]])
        maxs = np.sort(th[0][~mn[0]])
        assert np.allclose(np.cos(mins), [1.0, -1.0], atol=1e-12)
        assert np.allclose(np.cos(maxs), [-h, -h], atol=1e-12)
        tc, ec, to, eo, e3, two = sw.classify(np.array([0.0]), th, mn, cnt,
                                              np.array([h]), np.array([0.0]))
        assert two[0]
        assert abs((e3[0] - ec[0]) - (1 + h) ** 2) < 1e-12
        assert abs((e3[0] - eo[0]) - (1 - h) ** 2) < 1e-12
    for h in (1.0 + 1e-9, 1.5, 3.0):
        th, mn, cnt = sw.stationary_points(np.array([h]), np.array([0.0]))
        assert cnt[0] == 2


def test_field_across_axis():
    for h in (0.05, 0.4, 0.9):
        th, mn, cnt = sw.stationary_points(np.array([0.0]), np.array([h]))
        assert cnt[0] == 4
        mins = np.sort(th[0][mn[0]])
        assert np.allclose(mins, [np.arcsin(h), np.pi - np.arcsin(h)], atol=1e-12)
        maxs = np.sort(th[0][~mn[0]])
        assert np.allclose(maxs, [-np.pi / 2, np.pi / 2], atol=1e-12)


def test_zero_field_barrier_is_KV():
    th, mn, cnt = sw.stationary_points(np.array([0.0]), np.array([0.0]))
    tc, ec, to, eo, e3, two = sw.classify(np.array([0.2]), th, mn, cnt, np.zeros(1), np.zeros(1))
    assert two[0] and abs(e3[0] - ec[0] - 1.0) < 1e-14 and abs(tc[0]) < 1e-14


def test_switching_field_45_degrees():
    c = np.cos(np.pi / 4)
    for h, want in ((0.5 * (1 - 1e-6), 4), (0.5 * (1 + 1e-6), 2), (0.49, 4), (0.51, 2)):
        th, mn, cnt = sw.stationary_points(np.array([h * c]), np.array([h * c]))
        assert cnt[0] == want, h


def test_random_fields_are_exact_extrema():
    rng = np.random.default_rng(11)
    n = 4000
    h = rng.uniform(0, 2.0, n)
    phi = rng.uniform(-np.pi, np.pi, n)
    hx, hy = h * np.cos(phi), h * np.sin(phi)
    th, mn, cnt = sw.stationary_points(hx, hy)
    assert np.array_equal(cnt, np.where(sw.astroid_bistable(hx, hy), 4, 2))
    for i in range(n):
        t = th[i, :cnt[i]]
        assert np.all(np.abs(sw.g(t, hx[i], hy[i])) < 1e-13)
        # e''/2 = cos 2t + hx cos t + hy sin t is positive at minima, negative at maxima
        e2 = np.cos(2 * t) + hx[i] * np.cos(t) + hy[i] * np.sin(t)
        assert np.all((e2 > 0) == mn[i, :cnt[i]])
        # minima and maxima alternate around the circle
        assert np.all(mn[i, :cnt[i]] != np.roll(mn[i, :cnt[i]], 1))


def test_close_pair_near_astroid_is_found():
    # just inside the astroid at phi = 30 degrees: the metastable minimum and the
    # saddle are far closer than the scan spacing
    phi = np.radians(30.0)
    hsw = (np.cos(phi) ** (2 / 3) + np.sin(phi) ** (2 / 3)) ** -1.5
    for eps in (1e-6, 1e-9):
        h = hsw * (1 - eps)
        th, mn, cnt = sw.stationary_points(np.array([h * np.cos(phi)]), np.array([h * np.sin(phi)]))
        assert cnt[0] == 4
        t = th[0]
        gap = np.min(np.abs(np.diff(np.sort(t))))
        assert gap < 2 * np.pi / sw.SCAN


def test_fall_rules():
    hx, hy = np.array([0.3]), np.array([0.2])
    th, mn, cnt = sw.stationary_points(hx, hy)
    mins = th[0][mn[0]]
    maxs = th[0][~mn[0]]
    for x in np.linspace(-np.pi + 1e-3, np.pi, 97):
        tc, ec, to, eo, e3, two = sw.classify(np.array([x]), th, mn, cnt, hx, hy)
        # descend from x along -e' with tiny steps: ends at tc
        y = x
        for _ in range(20000):
            y -= 0.01 * sw.g(y, hx[0], hy[0])
        assert abs(np.angle(np.exp(1j * (y - tc[0])))) < 1e-6
        assert to[0] != tc[0] and to[0] in mins
    # exactly on a maximum: lower-energy minimum wins
    e = sw.energy(mins, hx[0], hy[0])
    for x in maxs:
        tc, *_ = sw.classify(np.array([x]), th, mn, cnt, hx, hy)
        assert tc[0] == mins[np.argmin(e)]


def test_scan200_matches_exact_away_from_switching():
    """The paper's literal 200-point scan + Newton finds the same stationary points as the
    exact search wherever the astroid margin is not small."""
    rng = np.random.default_rng(21)
    h = rng.uniform(0, 2.0, 3000)
    phi = rng.uniform(0, np.pi, 3000)
    hx, hy = h * np.cos(phi), h * np.sin(phi)
    a = hx * hx + hy * hy - 1.0
    margin = np.abs(a ** 3 + 27 * hx * hx * hy * hy)
    keep = margin > 0.05
    hx, hy = hx[keep], hy[keep]
    t1, m1, c1 = sw.stationary_points(hx, hy)
    t2, m2, c2 = sw.stationary_points_scan200(hx, hy)
    assert np.array_equal(c1, c2)
    assert np.array_equal(m1, m2)
    assert np.nanmax(np.abs(t1 - t2)) < 1e-12


def test_scan200_misses_close_pair_near_switching_field():
    """With the field 10 deg off the easy axis at 0.9999 of the astroid's switching field,
    the saddle and the metastable minimum (2.6223 and 2.6387 rad) both fall inside grid
    cell 83 of the 200-point scan (width 2 pi / 200): the literal scan has no sign change
    there and keeps only the stable pair.  At 0.999 of it they are 0.05 rad apart and
    both are found, identical to the exact search."""
    phi = np.deg2rad(10.0)
    h_sw = (np.cos(phi) ** (2 / 3) + np.sin(phi) ** (2 / 3)) ** -1.5
    for f, want in ((0.9999, 2), (0.999, 4)):
        hx, hy = np.array([f * h_sw * np.cos(phi)]), np.array([f * h_sw * np.sin(phi)])
        t1, m1, c_exact = sw.stationary_points(hx, hy)
        t2, m2, c_scan = sw.stationary_points_scan200(hx, hy)
        assert c_exact[0] == 4
        assert c_scan[0] == want
        # the stable minimum and the maximum it keeps are the exact ones either way
        assert np.allclose(t2[0, :2], t1[0, :2], atol=1e-13, rtol=0)
        assert np.array_equal(m2[0, :2], m1[0, :2])
    # the lost pair leaves a single well: every start falls to the one minimum
    hx = np.array([0.9999 * h_sw * np.cos(phi)])
    hy = np.array([0.9999 * h_sw * np.sin(phi)])
    t2, m2, c2 = sw.stationary_points_scan200(hx, hy)
    assert m2[0, :2].sum() == 1

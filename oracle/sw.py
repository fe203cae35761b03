"""Stoner-Wohlfarth extrema of one particle in its working plane (Sec. II.1, Eq. 2,
steps iv-v).

Energy in units of K_eff V, with h = |B_tot| / (mu0 H_K), mu0 H_K = 2 K_eff / M_S and
(hx, hy) = h (cos phi, sin phi) the field components along the easy axis and across
it in the working plane:

    e(theta) = sin^2 theta - 2 (hx cos theta + hy sin theta)

(Eq. 2 divided by K_eff V, since mu0 M_S V H_tot = 2 h K_eff V). Stationary points are
the zeros of g = e'/2 = sin theta cos theta + hx sin theta - hy cos theta.

The paper scans 200 points and refines with Newton (step iv). The oracle keeps the
idea but makes it exact: a dense scan, bisection of every sign change down to
adjacent doubles, and a rescan at finer resolution whenever fewer stationary points
are found than the Stoner-Wohlfarth astroid demands (two minima exactly when
(hx^2 + hy^2 - 1)^3 + 27 hx^2 hy^2 < 0), so pairs of extrema closer than the grid
spacing near the switching field are not lost. stationary_points_scan200 is the
paper's search taken literally (a selectable mode), with the loss of such pairs.
"""
import math

import numpy as np

SCAN = 256


def g(theta, hx, hy):
    s, c = np.sin(theta), np.cos(theta)
    return s * c + hx * s - hy * c


def energy(theta, hx, hy):
    """e(theta), Eq. 2 in units of K_eff V."""
    s, c = np.sin(theta), np.cos(theta)
    return s * s - 2.0 * (hx * c + hy * s)


def astroid_bistable(hx, hy):
    """True where the field lies strictly inside the Stoner-Wohlfarth astroid."""
    a = hx * hx + hy * hy - 1.0
    return a * a * a + 27.0 * hx * hx * hy * hy < 0.0


def _bisect(a, b, hx, hy, neg_a):
    """Vectorised bisection of g on [a, b] (one root per row), sign of g(a) given."""
    for _ in range(200):
        mid = 0.5 * (a + b)
        done = (mid == a) | (mid == b)
        if np.all(done):
            break
        gm = g(mid, hx, hy)
        same = (gm < 0.0) == neg_a
        a = np.where(~done & same, mid, a)
        b = np.where(~done & ~same, mid, b)
    ga, gb = np.abs(g(a, hx, hy)), np.abs(g(b, hx, hy))
    return np.where(ga <= gb, a, b)


def _scan_rows(hx, hy, m):
    """Sign changes of g on an m-point grid of (-pi, pi]; returns (row, left, right, neg_left)."""
    th = -np.pi + 2.0 * np.pi * np.arange(m) / m
    G = g(th[None, :], hx[:, None], hy[:, None])
    G = np.concatenate([G, G[:, :1]], axis=1)          # exact wrap-around
    neg = G < 0.0
    row, k = np.nonzero(neg[:, :-1] != neg[:, 1:])
    left = th[k]
    right = np.where(k + 1 < m, th[np.minimum(k + 1, m - 1)], np.pi)
    return row, left, right, neg[row, k]


def stationary_points(hx, hy):
    """All stationary points of e on (-pi, pi] for arrays hx, hy (shape (N,)).

    Returns ``theta`` (N,4) sorted ascending (unused slots NaN), ``is_min`` (N,4) bool
    and ``count`` (N,) in {2, 4}.
    """
    hx = np.atleast_1d(np.asarray(hx, dtype=np.float64))
    hy = np.atleast_1d(np.asarray(hy, dtype=np.float64))
    n = hx.shape[0]
    row, a, b, neg_a = _scan_rows(hx, hy, SCAN)
    roots = _bisect(a, b, hx[row], hy[row], neg_a)
    theta = np.full((n, 4), np.nan)
    is_min = np.zeros((n, 4), dtype=bool)
    count = np.bincount(row, minlength=n)
    want = np.where(astroid_bistable(hx, hy), 4, 2)
    good = (count == want)
    # rows come out of the scan in order, so the slot of a root is its rank in its row
    first = np.concatenate([[0], np.cumsum(count)[:-1]])
    slot = np.arange(row.shape[0]) - first[row]
    sel = good[row]
    theta[row[sel], slot[sel]] = roots[sel]
    is_min[row[sel], slot[sel]] = neg_a[sel]     # g goes - -> +: e'' > 0, a minimum
    for r in np.nonzero(~good)[0]:
        t, mn = _refine_row(hx[r], hy[r], want[r])
        theta[r, :len(t)] = t
        is_min[r, :len(t)] = mn
        count[r] = len(t)
    # order each row by angle
    key = np.where(np.isnan(theta), np.inf, theta)
    order = np.argsort(key, axis=1, kind="stable")
    theta = np.take_along_axis(theta, order, axis=1)
    is_min = np.take_along_axis(is_min, order, axis=1)
    return theta, is_min, count


SCAN_PAPER = 200


def _wrap(x):
    """Angle into (-pi, pi] through the IEEE remainder by 2 pi."""
    r = np.array([math.remainder(float(v), 2.0 * np.pi) for v in np.ravel(x)])
    return np.where(r == -np.pi, np.pi, r)


def stationary_points_scan200(hx, hy):
    """The paper's step iv taken literally (paper-literal mode): g on the 200 angles
    theta_j = 2 pi j / 200 of [0, 2 pi), each sign change between neighbours (cyclically)
    marks an extremum, refined by Newton's method on g from the middle of its interval
    (at most 50 steps, stopping once a step is below 1e-13); a minimum where g goes from
    negative to positive. Pairs of extrema closer than the grid spacing near the
    switching field are missed, as with the paper's scan. Same output layout as
    stationary_points (count in {2, 4})."""
    hx = np.atleast_1d(np.asarray(hx, dtype=np.float64))
    hy = np.atleast_1d(np.asarray(hy, dtype=np.float64))
    n = hx.shape[0]
    j = np.arange(SCAN_PAPER + 1)
    t = 2.0 * np.pi * j / 200.0
    G = g(t[None, :SCAN_PAPER], hx[:, None], hy[:, None])
    G = np.concatenate([G, G[:, :1]], axis=1)           # the value at 2 pi is the one at 0
    neg = G < 0.0
    change = neg[:, :-1] != neg[:, 1:]
    count = np.minimum(change.sum(axis=1), 4).astype(np.int64)
    # the first four sign changes of each row, in grid order
    rank = np.cumsum(change, axis=1) - 1
    slot = np.where(change & (rank < 4), rank, 4)
    k_of = np.full((n, 5), -1, dtype=np.int64)
    rows = np.broadcast_to(np.arange(n)[:, None], slot.shape)
    k_of[rows[slot < 4], slot[slot < 4]] = np.broadcast_to(j[None, :SCAN_PAPER],
                                                           slot.shape)[slot < 4]
    k_of = k_of[:, :4]
    valid = k_of >= 0
    kk = np.where(valid, k_of, 0)
    # Newton on g from each interval's middle; an element stops after the first step
    # below 1e-13 (that step is still taken), or after 50 steps
    x = 0.5 * (t[kk] + t[kk + 1])
    live = valid.copy()
    HX, HY = hx[:, None], hy[:, None]
    for _ in range(50):
        if not live.any():
            break
        sn, cs = np.sin(x), np.cos(x)
        f = sn * cs + HX * sn - HY * cs
        d = (cs * cs - sn * sn) + HX * cs + HY * sn
        dx = np.where(live, f / np.where(live, d, 1.0), 0.0)
        x = np.where(live, x - dx, x)
        live &= ~(np.abs(dx) < 1e-13)
    theta = np.where(valid, _wrap(x).reshape(n, 4), np.nan)
    is_min = valid & np.take_along_axis(neg, kk, axis=1)
    key = np.where(np.isnan(theta), np.inf, theta)
    order = np.argsort(key, axis=1, kind="stable")
    return (np.take_along_axis(theta, order, axis=1), np.take_along_axis(is_min, order, axis=1),
            count)


def _refine_row(hx, hy, want):
    """Rescan one particle at finer grids until the astroid count is met."""
    hxa, hya = np.array([hx]), np.array([hy])
    best = None
    for m in (SCAN * 64, SCAN * 4096, 1 << 22):
        row, a, b, neg_a = _scan_rows(hxa, hya, m)
        roots = _bisect(a, b, np.full(a.shape, hx), np.full(a.shape, hy), neg_a)
        best = (list(roots), list(neg_a))
        if len(roots) == want:
            break
    if len(best[0]) > 4:
        raise RuntimeError("more than four stationary points: impossible for Eq. 2")
    return best


def classify(theta0, theta, is_min, count, hx, hy):
    """Step v: the minimum the moment at ``theta0`` falls into, and the other one.

    Returns (theta_c, e_c, theta_o, e_o, e3, two) where ``two`` flags two minima and
    e3 is the energy of the lower maximum. With one minimum, theta_o = theta_c.
    With two minima the circle is cut by the four stationary points into arcs that
    each join one minimum and one maximum; the moment falls into the minimum at the
    end of its arc. A moment sitting exactly on a maximum goes to the lower-energy
    minimum, then to the nearer one.
    """
    n = theta0.shape[0]
    rows = np.arange(n)
    th = np.where(np.isnan(theta), 0.0, theta)
    E = energy(th, hx[:, None], hy[:, None])
    two = count == 4
    # one minimum: rows with count 2 keep it in whichever slot is flagged
    k1 = np.argmax(is_min & ~np.isnan(theta), axis=1)
    # two minima: arc of theta0 among the sorted stationary points
    j = np.sum(np.where(np.isnan(theta), False, theta < theta0[:, None]), axis=1)
    left, right = (j - 1) % 4, j % 4
    c4 = np.where(is_min[rows, left], left, right)
    c = np.where(two, c4, k1)
    # the other minimum: the flagged slot that is not c
    m2 = is_min.copy()
    m2[rows, c] = False
    o = np.where(two, np.argmax(m2, axis=1), c)
    e3 = np.where(two, np.min(np.where(~is_min & two[:, None], E, np.inf), axis=1), np.nan)
    # exact hits on a stationary point
    hit = two & np.any(theta == theta0[:, None], axis=1)
    for i in np.nonzero(hit)[0]:
        kk = int(np.nonzero(theta[i] == theta0[i])[0][0])
        if is_min[i, kk]:
            ci = kk
        else:
            a, b = np.nonzero(is_min[i])[0]
            if E[i, a] != E[i, b]:
                ci = a if E[i, a] < E[i, b] else b
            else:
                da = abs(np.angle(np.exp(1j * (theta0[i] - theta[i, a]))))
                db = abs(np.angle(np.exp(1j * (theta0[i] - theta[i, b]))))
                ci = a if da <= db else b
        c[i] = ci
        mins = np.nonzero(is_min[i])[0]
        o[i] = mins[0] if mins[1] == ci else mins[1]
    return th[rows, c], E[rows, c], th[rows, o], E[rows, o], e3, two

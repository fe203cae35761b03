"""Seeded synthetic inputs: nanoparticle placements, easy axes and run configurations.

This module holds no arithmetic of the simulation method itself. It only draws the
inputs that the paper's workloads are made of (Sec. II.1 and Sec. III.1):

* monodisperse hard spheres of diameter ``d`` placed at random, without overlap,
  inside a spherical lysosome (random sequential addition);
* the same spheres on a cubic lattice, each node displaced by a random vector of
  length at most the largest value that cannot create an overlap;
* easy axes drawn uniformly on the unit sphere (random 3-D) or uniformly in a plane
  that contains the applied field (random 2-D, Fig. 1 caption).

Both the oracle-side tests and the GPU path are fed from here, so the two sides
always see identical inputs. Lengths are in metres.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np


# ----------------------------------------------------------------------------
# placements
# ----------------------------------------------------------------------------

def place_random(n: int, radius: float, d: float, seed: int, max_tries: int = 2000) -> np.ndarray:
    """Random sequential addition of ``n`` hard spheres (diameter ``d``) fully inside
    a sphere of radius ``radius``: centres satisfy ``|r| <= radius - d/2`` and every
    pair is at least ``d`` apart (random non-overlapping placement, Sec. III.1).

    A uniform cell list keeps each insertion O(1). Raises ``RuntimeError`` when the
    requested packing cannot be reached within ``max_tries`` attempts per sphere.
    """
    if n <= 0:
        return np.zeros((0, 3))
    rin = radius - 0.5 * d
    if rin < 0:
        raise ValueError("lysosome radius smaller than one particle radius")
    rng = np.random.default_rng(seed)
    cell = d
    ncell = max(1, int(math.ceil(2 * rin / cell)) + 1)
    grid: dict[tuple[int, int, int], list[int]] = {}
    pos = np.empty((n, 3))
    d2 = d * d
    count = 0
    batch = 4096
    while count < n:
        cand = rng.uniform(-rin, rin, size=(batch, 3))
        cand = cand[np.einsum("ij,ij->i", cand, cand) <= rin * rin]
        for c in cand:
            key = tuple(int(v) for v in np.floor((c + rin) / cell))
            ok = True
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        lst = grid.get((key[0] + dx, key[1] + dy, key[2] + dz))
                        if not lst:
                            continue
                        for j in lst:
                            q = pos[j] - c
                            if q[0] * q[0] + q[1] * q[1] + q[2] * q[2] < d2:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                pos[count] = c
                grid.setdefault(key, []).append(count)
                count += 1
                if count == n:
                    break
        max_tries -= 1
        if max_tries <= 0 and count < n:
            raise RuntimeError(f"random placement stalled at {count}/{n} spheres")
    del ncell
    return pos


def place_lattice_disorder(n: int, radius: float, d: float, seed: int) -> np.ndarray:
    """Cubic lattice cut by the lysosome, then maximal disorder (Sec. III.1).

    The lattice constant ``a`` is the largest one for which at least ``n`` nodes lie
    within ``radius - d/2 - delta`` of the centre, with ``delta = (a - d)/2`` the largest
    displacement that cannot make two neighbours overlap (two nodes ``a`` apart that
    each move ``delta`` towards the other end up exactly ``d`` apart). The ``n`` nodes
    closest to the centre are kept and each moves by a vector drawn uniformly in the
    ball of radius ``delta``.
    """
    if n <= 0:
        return np.zeros((0, 3))
    rng = np.random.default_rng(seed)
    rin = radius - 0.5 * d

    def nodes_for(a: float):
        delta = 0.5 * (a - d)
        lim = rin - delta
        m = int(math.floor(lim / a)) + 1
        g = np.arange(-m, m + 1) * a
        X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
        P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        r = np.linalg.norm(P, axis=1)
        return P[r <= lim], r[r <= lim], delta

    lo, hi = d, 2 * rin + d
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        P, _, _ = nodes_for(mid)
        if len(P) >= n:
            lo = mid
        else:
            hi = mid
    P, r, delta = nodes_for(lo)
    if len(P) < n:
        raise RuntimeError("lattice placement could not fit the requested number of spheres")
    order = np.argsort(r, kind="stable")[:n]
    P = P[order]
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    rad = delta * rng.uniform(0.0, 1.0, size=n) ** (1.0 / 3.0)
    return P + v * rad[:, None]


def axes_random_3d(n: int, seed: int) -> np.ndarray:
    """Easy axes uniform on the unit sphere (normalised Gaussian triples)."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def axes_random_2d(n: int, seed: int) -> np.ndarray:
    """Easy axes uniform in the x-y plane, which contains the applied field (Fig. 1 caption)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 2.0 * np.pi, size=n)
    return np.stack([np.cos(a), np.sin(a), np.zeros(n)], axis=1)


def volume_fraction(n: int, radius: float, d: float) -> float:
    """Volume concentration of ``n`` spheres of diameter ``d`` in a sphere of ``radius``."""
    return n * (d / (2.0 * radius)) ** 3


# ----------------------------------------------------------------------------
# run configurations
# ----------------------------------------------------------------------------

@dataclass
class Material:
    """Per-assembly material, field and protocol parameters (SI units)."""
    Ms: float = 4.0e5          # A/m
    Keff: float = 1.3e4        # J/m^3
    d: float = 12e-9           # m
    T: float = 300.0           # K (0 disables thermal jumps)
    tau0: float = 1e-10        # s, attempt time 1/nu0
    rho: float = 5200.0        # kg/m^3
    f: float = 1e5             # Hz
    mu0Hmax: float = 0.02      # T
    steps_per_period: int = 2000
    n_periods: int = 3
    n_discard: int = 2
    dt_override: float = 0.0   # >0: constant field mu0Hmax along x, step dt_override
    prob_form: int = 0         # 0: two-state Eq. 5; 1: single rate 1-exp(-nu_c dt)
    interactions: int = 1

    def as_dict(self):
        return asdict(self)


@dataclass
class Assembly:
    pos: np.ndarray
    axes: np.ndarray
    mat: Material
    radius: float = 0.0
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def lysosome_n100(seed_offset: int = 0) -> Assembly:
    """N=100 in an 80 nm lysosome, d=12 nm, random placement and 3-D axes, 20 mT,
    100 kHz, 2000 steps, 3 periods with the last one kept (FP64 end to end)."""
    c = 1
    n, R, d = 100, 80e-9, 12e-9
    pos = place_random(n, R, d, 1000 + c + seed_offset)
    ax = axes_random_3d(n, 2000 + c + seed_offset)
    mat = Material(d=d, mu0Hmax=0.02, n_periods=3, n_discard=2)
    return Assembly(pos, ax, mat, R, 3000 + c + seed_offset,
                    {"phi": volume_fraction(n, R, d)})


def lysosome_n5000(mu0Hmax: float = 0.02, n_periods: int = 5) -> Assembly:
    """N=5000 in a 250 nm lysosome, d=12 nm (phi=6.9 %), random 3-D axes, 100 kHz,
    2000 steps per period, 5 periods with the first discarded."""
    c = 2
    n, R, d = 5000, 250e-9, 12e-9
    pos = place_random(n, R, d, 1000 + c)
    ax = axes_random_3d(n, 2000 + c)
    mat = Material(d=d, mu0Hmax=mu0Hmax, n_periods=n_periods, n_discard=min(1, n_periods - 1))
    return Assembly(pos, ax, mat, R, 3000 + c, {"phi": volume_fraction(n, R, d)})


def uneven_batch_params(count: int = 256, seed: int = 1003):
    """Draws of the uneven batch: radius U(100,250) nm, phi U(1,20) %, d U(10,16) nm,
    Keff U(0.8,2.0)e4, mu0Hmax U(5,40) mT, N = round(phi (2R/d)^3) kept when
    200 <= N <= 8000."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        R = rng.uniform(100e-9, 250e-9)
        phi = rng.uniform(0.01, 0.20)
        d = rng.uniform(10e-9, 16e-9)
        K = rng.uniform(0.8e4, 2.0e4)
        H = rng.uniform(0.005, 0.040)
        n = int(round(phi * (2 * R / d) ** 3))
        if 200 <= n <= 8000:
            out.append(dict(R=R, phi=phi, d=d, K=K, H=H, n=n))
    return out


def uneven_batch(count: int = 256, n_periods: int = 3) -> list[Assembly]:
    out = []
    for a, p in enumerate(uneven_batch_params(count)):
        pos = place_random(p["n"], p["R"], p["d"], 100000 + a)
        ax = axes_random_3d(p["n"], 200000 + a)
        mat = Material(d=p["d"], Keff=p["K"], mu0Hmax=p["H"], n_periods=n_periods,
                       n_discard=n_periods - 1)
        out.append(Assembly(pos, ax, mat, p["R"], 300000 + a, {"phi": p["phi"]}))
    return out


def replica_batch_geometry():
    """N=4096 in a 200 nm lysosome at phi=10 %: d = 2R (phi/N)^(1/3) = 11.60 nm."""
    n, R, phi = 4096, 200e-9, 0.10
    d = 2 * R * (phi / n) ** (1.0 / 3.0)
    pos = place_random(n, R, d, 1004)
    return pos, d, R


def replica_batch_n4096(n_axes_sets: int = 512) -> Assembly:
    """Replica-batched form: shared positions, one set of random 3-D axes per replica
    (the paper's averaging over axis orientations, Sec. III.1), 20 mT, 100 kHz,
    3 periods with the last kept."""
    pos, d, R = replica_batch_geometry()
    n = pos.shape[0]
    rng_seed = 2004
    axes = np.concatenate([axes_random_3d(n, rng_seed + 7919 * s) for s in range(n_axes_sets)])
    mat = Material(d=d, mu0Hmax=0.02, n_periods=3, n_discard=2)
    return Assembly(pos, axes, mat, R, 3004, {"phi": 0.10, "n_axes_sets": n_axes_sets})


def request_stream(count: int = 1000, seed: int = 1005, rate_hz: float = 1.0):
    """Poisson arrivals of loop requests: N log-uniform in [100, 8000], radius
    U(80,300) nm, phi U(1,20) % (d derived), f log-uniform in [1e5, 1e6] Hz, mu0Hmax
    U(5,50) mT, periods U{3..10} with one discarded."""
    # request parameters and arrival gaps from separate generators, so that the first k
    # requests are the same whatever the count
    rng = np.random.default_rng(seed)
    t = np.cumsum(np.random.default_rng(seed + 1).exponential(1.0 / rate_hz, size=count))
    reqs = []
    for q in range(count):
        n = int(round(math.exp(rng.uniform(math.log(100), math.log(8000)))))
        R = rng.uniform(80e-9, 300e-9)
        phi = rng.uniform(0.01, 0.20)
        d = 2 * R * (phi / n) ** (1.0 / 3.0)
        f = math.exp(rng.uniform(math.log(1e5), math.log(1e6)))
        H = rng.uniform(0.005, 0.050)
        P = int(rng.integers(3, 11))
        reqs.append(dict(t=float(t[q]), n=n, R=R, phi=phi, d=d, f=f, H=H, P=P,
                         seed=500000 + q))
    return reqs

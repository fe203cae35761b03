"""Kinetic Monte-Carlo hysteresis loops, written out step by step in FP64 (Sec. II.1
steps i-viii, Eqs. 1-5; loop protocol Sec. III.1; SAR conversion Sec. III.2.a).

Readings of points the paper leaves open (applied identically by the GPU library):

* Eq. 1 sums over the other particles j != i; the result mu0 H_dip is in tesla.
* Field H_k = H_max cos(2 pi k / S) along a fixed unit direction e_H (x unless
  field_dir says otherwise; (0, 0, 0) means x), constant during step k (steps of
  equal length dt = 1/(f S)); a run is n_periods periods starting at +H_max; the first
  n_discard periods are thrown away (Sec. III.1). Loop, area and Eq. 6 use the
  components along e_H, which is x in the paper.
* Working plane (step iii): u1 = easy axis n, u2 = the unit part of B_tot normal to
  n. When that part vanishes (|B_perp| <= 1e-12 max(|B|, mu0 H_K)) u2 is the unit
  part of the previous moment normal to n, else the normalised n x e, with e the
  coordinate axis least aligned with n.
* Initial moments m_i = sign(n_i . e_H) n_i with sign(0) = +1.
* Eq. 5 is read as the probability to leave the current well c for the other well o:
  P = nu_c/(nu_c+nu_o) (1 - exp(-(nu_c+nu_o) dt)), nu = nu0 exp(-(E3-E)/kT); it is
  evaluated as sigma(a_o - a_c) * (-expm1(-nu0 dt (e^-a_c + e^-a_o))), which is the
  same expression rearranged so that it cannot overflow. Jump iff u < P.
  prob_form=1 selects the single-rate form 1 - exp(-nu_c dt) instead.
* T = 0: steps vi-vii are skipped; K_eff = 0: the moment aligns with B_tot.
* Area: A = M_S sum_k mu0H_k (m_H,k - m_H,k-1) over the kept steps (work done at
  constant field per step; m_H = m . e_H), J/m^3; SAR = A f / rho.
* Eq. 6: the dipolar field "at +mu0 H_max" (-mu0 H_max) is the e_H component of the Eq. 1
  field acting in the step whose applied field is +H_max (-H_max), k = 0 (S/2) mod S,
  i.e. computed from that step's start-of-step moments; Delta-_Hdip per particle is
  its difference, averaged over the kept periods.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import philox
from . import sw

MU0 = 4e-7 * np.pi
KB = 1.380649e-23


@dataclass
class Params:
    Ms: float = 4.0e5
    Keff: float = 1.3e4
    d: float = 12e-9
    T: float = 300.0
    tau0: float = 1e-10
    rho: float = 5200.0
    f: float = 1e5
    mu0Hmax: float = 0.02
    steps_per_period: int = 2000
    n_periods: int = 3
    n_discard: int = 2
    dt_override: float = 0.0
    prob_form: int = 0
    interactions: int = 1
    extrema_mode: int = 0    # 0: exact stationary points; 1: the paper's 200-point scan
    field_dir: tuple = (1.0, 0.0, 0.0)   # direction of the applied field

    @classmethod
    def from_dict(cls, d):
        return cls(**{k: d[k] for k in cls.__dataclass_fields__ if k in d})


def derived(p: Params):
    """Sec. II.1 quantities: V, C = mu0 Ms V / 4pi, mu0 H_K = 2K/Ms, beta = K V / kT,
    nu0 dt with dt = 1/(f S) (or dt_override)."""
    V = np.pi * p.d ** 3 / 6.0
    C = MU0 * p.Ms * V / (4.0 * np.pi)
    BK = 2.0 * p.Keff / p.Ms if p.Keff > 0 else 0.0
    beta = p.Keff * V / (KB * p.T) if p.T > 0 else np.inf
    dt = p.dt_override if p.dt_override > 0 else 1.0 / (p.f * p.steps_per_period)
    return dict(V=V, C=C, BK=BK, beta=beta, dt=dt, nu0dt=dt / p.tau0)


def field_unit(p: Params) -> np.ndarray:
    """The unit direction e_H of the applied field: field_dir normalised, x for (0, 0, 0)."""
    d = np.asarray(p.field_dir, dtype=np.float64)
    nd = np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
    return np.array([1.0, 0.0, 0.0]) if nd == 0.0 else d / nd


def applied_field(k: int, p: Params) -> float:
    """mu0 H_ext at step k (its component along e_H), Sec. II.1 and Sec. III.1."""
    if p.dt_override > 0:
        return p.mu0Hmax
    return p.mu0Hmax * np.cos(2.0 * np.pi * k / p.steps_per_period)


def dipolar_field(pos: np.ndarray, m: np.ndarray, C: float, chunk: int = 512) -> np.ndarray:
    """Eq. 1: mu0 H_dip,i = C sum_{j != i} [3 (m_j . e_ij) e_ij - m_j] / r_ij^3, exact,
    no cutoff. pos (N,3) in m, m (N,3) unit vectors; returns (N,3) in tesla."""
    n = pos.shape[0]
    out = np.zeros((n, 3))
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        r = pos[None, :, :] - pos[s:e, None, :]            # r_j - r_i
        d2 = np.einsum("ijk,ijk->ij", r, r)
        idx = np.arange(s, e)
        d2[idx - s, idx] = np.inf                           # j == i excluded
        inv = 1.0 / np.sqrt(d2)
        eu = r * inv[:, :, None]
        md = np.einsum("jk,ijk->ij", m, eu)
        term = (3.0 * md[:, :, None] * eu - m[None, :, :]) * (inv ** 3)[:, :, None]
        out[s:e] = term.sum(axis=1)
    return C * out


def working_plane(B: np.ndarray, n: np.ndarray, m: np.ndarray, BK: float):
    """Step iii: in-plane frame (n, u2), reduced field (hx, hy) and theta0 of the
    previous moment projected into the plane."""
    bpar = np.einsum("ij,ij->i", B, n)
    Bp = B - bpar[:, None] * n
    bp = np.linalg.norm(Bp, axis=1)
    Bn = np.linalg.norm(B, axis=1)
    deg = bp <= 1e-12 * np.maximum(Bn, BK)
    u2 = np.zeros_like(B)
    ok = ~deg
    u2[ok] = Bp[ok] / bp[ok, None]
    if np.any(deg):
        v = m - np.einsum("ij,ij->i", m, n)[:, None] * n
        vn = np.linalg.norm(v, axis=1)
        for i in np.nonzero(deg)[0]:
            if vn[i] > 1e-12:
                u2[i] = v[i] / vn[i]
            else:
                c = int(np.argmin(np.abs(n[i])))
                e = np.zeros(3)
                e[c] = 1.0
                w = np.cross(n[i], e)
                u2[i] = w / np.linalg.norm(w)
    hx = bpar / BK
    hy = np.where(deg, 0.0, bp / BK)
    theta0 = np.arctan2(np.einsum("ij,ij->i", m, u2), np.einsum("ij,ij->i", m, n))
    return u2, hx, hy, theta0


def transition_probability(a_c, a_o, nu0dt, prob_form: int = 0):
    """Eq. 5 (prob_form 0) or the single-rate form (prob_form 1); a = barrier / kT."""
    if prob_form == 1:
        return -np.expm1(-nu0dt * np.exp(-a_c))
    with np.errstate(over="ignore"):
        sig = 1.0 / (1.0 + np.exp(a_c - a_o))
    return sig * (-np.expm1(-nu0dt * (np.exp(-a_c) + np.exp(-a_o))))


@dataclass
class StepInfo:
    B: np.ndarray
    hx: np.ndarray
    hy: np.ndarray
    theta0: np.ndarray
    theta_c: np.ndarray
    theta_o: np.ndarray
    e_c: np.ndarray
    e_o: np.ndarray
    e3: np.ndarray
    two: np.ndarray
    P: np.ndarray
    u: np.ndarray
    jump: np.ndarray
    u2: np.ndarray | None = None
    Bdip: np.ndarray | None = None   # the Eq. 1 part of B (zeros without interactions)


def step(pos, axes, m, k, p: Params, seed: int, stream: int, B_override=None):
    """One synchronous step (steps ii-vii) for every particle from the start-of-step
    moments ``m`` (Sec. II.2: fields are computed once per step). Returns (m_new, info)."""
    dv = derived(p)
    n = pos.shape[0]
    Bx = applied_field(k, p)
    Bdip = None
    if B_override is not None:
        B = np.array(B_override, dtype=np.float64)
    else:
        B = np.zeros((n, 3))
        if p.interactions and n > 1:
            B += dipolar_field(pos, m, dv["C"])
        Bdip = B.copy()
        B += Bx * field_unit(p)[None, :]
    if p.Keff <= 0:
        Bn = np.linalg.norm(B, axis=1)
        m_new = np.where(Bn[:, None] > 0, B / np.where(Bn > 0, Bn, 1.0)[:, None], m)
        z = np.zeros(n)
        return m_new, StepInfo(B, z, z, z, z, z, z, z, z, np.zeros(n, bool), z, z,
                               np.zeros(n, bool), None, Bdip)
    u2, hx, hy, theta0 = working_plane(B, axes, m, dv["BK"])
    scan = sw.stationary_points_scan200 if p.extrema_mode == 1 else sw.stationary_points
    theta, is_min, count = scan(hx, hy)
    th_c, e_c, th_o, e_o, e3, two = sw.classify(theta0, theta, is_min, count, hx, hy)
    th_new = th_c.copy()
    P = np.zeros(n)
    u = np.full(n, np.nan)
    jump = np.zeros(n, dtype=bool)
    if p.T > 0:
        u = philox.uniforms(seed, stream, k, n)
        a_c = dv["beta"] * (e3 - e_c)
        a_o = dv["beta"] * (e3 - e_o)
        P = np.where(two, transition_probability(np.where(two, a_c, 0.0),
                                                 np.where(two, a_o, 0.0),
                                                 dv["nu0dt"], p.prob_form), 0.0)
        jump = two & (u < P)
        th_new = np.where(jump, th_o, th_c)
    m_new = np.cos(th_new)[:, None] * axes + np.sin(th_new)[:, None] * u2
    info = StepInfo(B, hx, hy, theta0, th_c, th_o, e_c, e_o, e3, two, P, u, jump, u2, Bdip)
    return m_new, info


def initial_moments(axes: np.ndarray, e_H=(1.0, 0.0, 0.0)) -> np.ndarray:
    """m_i = sign(n_i . e_H) n_i, sign(0) = +1: saturated along the field at +H_max."""
    e = np.asarray(e_H, dtype=np.float64)
    s = np.where(axes @ e >= 0.0, 1.0, -1.0)
    return axes * s[:, None]


@dataclass
class LoopResult:
    H: np.ndarray                  # (S,) mu0 H_k, tesla
    M: np.ndarray                  # (n_kept, S) M_S <m . e_H> after each step, A/m
    area_per_np: np.ndarray        # (N,) J/m^3, mean over kept periods
    area: float                    # J/m^3
    sar: float                     # W/kg
    m_final: np.ndarray
    jumps: int = 0
    trace: list = field(default_factory=list)
    dhdip_per_np: np.ndarray | None = None   # (N,) Eq. 6, T, mean over kept periods


def simulate(pos, axes, p: Params, seed: int, stream: int = 0, n_steps: int | None = None,
             keep_trace: bool = False, m0=None) -> LoopResult:
    """Whole run: n_periods x steps_per_period synchronous steps (Sec. III.1)."""
    S = p.steps_per_period
    total = p.n_periods * S if n_steps is None else n_steps
    kept0 = p.n_discard * S
    n_kept = max(0, p.n_periods - p.n_discard)
    eH = field_unit(p)
    m = initial_moments(axes, eH) if m0 is None else np.array(m0, dtype=np.float64)
    n = pos.shape[0]
    area = np.zeros(n)
    dhdip = np.zeros(n)
    Mrec = np.zeros((max(n_kept, 1), S))
    Hrec = np.array([applied_field(k, p) for k in range(S)])
    jumps = 0
    trace = []
    for k in range(total):
        m_new, info = step(pos, axes, m, k, p, seed, stream)
        jumps += int(info.jump.sum())
        if k >= kept0 and info.Bdip is not None and k % S in (0, S // 2):
            # Eq. 6: dipolar field along e_H at +H_max minus at -H_max
            bh = info.Bdip @ eH
            dhdip += bh if k % S == 0 else -bh
        if k >= kept0:
            area += p.Ms * applied_field(k, p) * (m_new @ eH - m @ eH)
            Mrec[(k - kept0) // S, k % S] = p.Ms * (m_new @ eH).mean()
        if keep_trace:
            trace.append(info)
        m = m_new
    area_np = area / max(n_kept, 1)
    A = float(area_np.mean()) if n else 0.0
    return LoopResult(Hrec, Mrec[:n_kept], area_np, A, A * p.f / p.rho, m, jumps, trace,
                      dhdip / max(n_kept, 1))


def replica_stats(areas):
    """Mean loop area over independent replicas and its standard error (Sec. III.1: a
    result is the average over loops that differ only in their random draws and axes).
    The replicas are independent, so the error of the mean is the sample standard
    deviation (ddof = 1) over sqrt(R); one replica has no spread and gives 0."""
    a = np.asarray(areas, dtype=np.float64)
    R = a.shape[0]
    mean = float(a.sum() / R)
    if R < 2:
        return mean, 0.0
    return mean, float(np.sqrt(((a - mean) ** 2).sum() / (R - 1) / R))


def sar_from_area(area, f, rho=5200.0):
    """Sec. III.2.a: SAR = A f / rho (W/kg) for an area A in J/m^3."""
    return area * f / rho

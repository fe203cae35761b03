"""The device-side step logic (csrc/mh_device.hpp), compiled for the host, against the
oracle: Philox words, Stoner-Wohlfarth extrema and basins (Eq. 2, steps iv-v), and the
whole per-particle update with its Eq. 5 draw (steps iii-vii). Runs without a GPU, so
the CPU suite checks the kernels' arithmetic; the GPU parity tests check the same
functions as compiled for gfx950."""
import ctypes as C
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import kmc, master, philox, sw

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hostshim", "device_logic.cpp")


@pytest.fixture(scope="module")
def dl():
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tempfile.mkdtemp()
    so = os.path.join(d, "device_logic.so")
    r = subprocess.run([cxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-I/opt/rocm/include", SRC,
                        "-o", so], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    L = C.CDLL(so)
    dp = C.POINTER(C.c_double)
    u64p = C.POINTER(C.c_uint64)
    L.dl_philox.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, u64p, u64p]
    L.dl_sw.argtypes = [C.c_int64, dp, dp, dp, dp]
    L.dl_sw_scan200.argtypes = [C.c_int64, dp, dp, dp, dp]
    L.dl_update.argtypes = [C.c_int64, dp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_int,
                            C.c_int, C.c_uint64, C.c_uint64, C.c_int64, C.c_int, dp]
    L.dl_master.argtypes = [C.c_int64, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                            C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int,
                            dp, dp, dp]
    u64p2 = C.POINTER(C.c_uint64)
    L.dl_mul128.argtypes = [C.c_int64, u64p2, u64p2]
    return L


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def test_philox_words(dl):
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2**63, size=(300, 4), dtype=np.int64).astype(np.uint64)
    out = np.empty_like(ctr)
    p = C.POINTER(C.c_uint64)
    dl.dl_philox(2**63 + 9, 77, ctr.shape[0], ctr.ctypes.data_as(p), out.ctypes.data_as(p))
    assert np.array_equal(out, philox.raw_words(2**63 + 9, 77, ctr))


def test_sw_fall_matches_oracle(dl):
    rng = np.random.default_rng(6)
    n = 30000
    h = rng.uniform(0, 2.0, n) ** 1.5
    phi = rng.uniform(0, np.pi, n)
    hx, hy = h * np.cos(phi), h * np.sin(phi)
    hx[:300] = rng.uniform(-1.5, 1.5, 300)
    hy[:300] = 0.0
    hx[300:600] = 0.0
    hy[300:600] = rng.uniform(0, 1.5, 300)
    # near the astroid: close min/max pairs
    psi = rng.uniform(0.05, np.pi / 2 - 0.05, 400)
    hsw = (np.cos(psi) ** (2 / 3) + np.sin(psi) ** (2 / 3)) ** -1.5
    hh = hsw * (1 - 10 ** rng.uniform(-9, -3, 400))
    hx[600:1000], hy[600:1000] = hh * np.cos(psi), hh * np.sin(psi)
    th0 = rng.uniform(-np.pi, np.pi, n)
    out = np.empty((n, 6))
    dl.dl_sw(n, _p(hx), _p(hy), _p(th0), _p(out))
    th, mn, cnt = sw.stationary_points(hx, hy)
    tc, ec, to, eo, e3, two = sw.classify(th0, th, mn, cnt, hx, hy)
    assert np.array_equal(out[:, 5] == 1.0, two)
    dc = np.abs(np.angle(np.exp(1j * (out[:, 0] - tc))))
    assert dc.max() < 1e-9, dc.max()
    do = np.abs(np.angle(np.exp(1j * (out[:, 2] - to))))
    assert do[two].max() < 1e-9, do[two].max()
    assert np.abs(out[:, 1] - ec).max() < 1e-12
    assert np.abs(out[two, 3] - eo[two]).max() < 1e-12
    assert np.abs(out[two, 4] - e3[two]).max() < 1e-12


def test_sw_fall_scan200_matches_oracle(dl):
    """The paper-literal search (200-point scan + Newton) against the oracle's, over
    the same field mix as above: pair counts decided identically, including the pairs
    the scan misses next to the astroid, which fall back to the one stable well."""
    rng = np.random.default_rng(16)
    n = 20000
    h = rng.uniform(0, 2.0, n) ** 1.5
    phi = rng.uniform(0, np.pi, n)
    hx, hy = h * np.cos(phi), h * np.sin(phi)
    hx[:300] = rng.uniform(-1.5, 1.5, 300)
    hy[:300] = 0.0
    hx[300:600] = 0.0
    hy[300:600] = rng.uniform(0, 1.5, 300)
    psi = rng.uniform(0.05, np.pi / 2 - 0.05, 1000)
    hsw = (np.cos(psi) ** (2 / 3) + np.sin(psi) ** (2 / 3)) ** -1.5
    hh = hsw * (1 - 10 ** rng.uniform(-7, -1, 1000))
    hx[600:1600], hy[600:1600] = hh * np.cos(psi), hh * np.sin(psi)
    th0 = rng.uniform(-np.pi, np.pi, n)
    out = np.empty((n, 6))
    dl.dl_sw_scan200(n, _p(hx), _p(hy), _p(th0), _p(out))
    th, mn, cnt = sw.stationary_points_scan200(hx, hy)
    tc, ec, to, eo, e3, two = sw.classify(th0, th, mn, cnt, hx, hy)
    _, _, cnt_exact = sw.stationary_points(hx, hy)
    missed = (cnt_exact == 4) & (cnt == 2)
    assert missed[600:1600].sum() > 100          # the scan's known loss near h_sw
    assert np.array_equal(out[:, 5] == 1.0, two)
    dc = np.abs(np.angle(np.exp(1j * (out[:, 0] - tc))))
    assert dc.max() < 1e-12, dc.max()
    do = np.abs(np.angle(np.exp(1j * (out[:, 2] - to))))
    assert do[two].max() < 1e-12, do[two].max()
    assert np.abs(out[:, 1] - ec).max() < 1e-12
    assert np.abs(out[two, 3] - eo[two]).max() < 1e-12
    assert np.abs(out[two, 4] - e3[two]).max() < 1e-12


@pytest.mark.parametrize("prob_form,scan", [(0, 0), (1, 0), (0, 1)])
def test_update_matches_oracle_step(dl, prob_form, scan):
    rng = np.random.default_rng(7 + prob_form)
    n = 4000
    p = kmc.Params(Ms=4e5, Keff=1.3e4, d=12e-9, T=300.0, mu0Hmax=0.02, interactions=0,
                   prob_form=prob_form, extrema_mode=scan)
    dv = kmc.derived(p)
    axes = rng.normal(size=(n, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    m = rng.normal(size=(n, 3))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    B = rng.normal(size=(n, 3)) * rng.uniform(0, 0.08, size=(n, 1))
    k = 1234
    m_new, info = kmc.step(np.zeros((n, 3)), axes, m, k, p, 4321, 3, B_override=B)
    out = np.empty((n, 6))
    dl.dl_update(n, _p(B), _p(axes), _p(m), dv["BK"], dv["beta"], dv["nu0dt"], prob_form, 1,
                 4321, 3, k, scan, _p(out))
    assert np.array_equal(out[:, 5] == 1.0, info.two)
    assert np.array_equal(out[:, 4] == 1.0, info.jump)
    assert np.abs(out[:, 3] - info.P).max() < 1e-12
    assert np.abs(out[:, :3] - m_new).max() < 1e-9


@pytest.mark.parametrize("T,prob_form,static,tilt", [(300.0, 0, 0, 0), (300.0, 1, 0, 0),
                                                     (0.0, 0, 0, 0), (300.0, 0, 1, 0),
                                                     (300.0, 0, 0, 1)])
def test_master_step_matches_oracle(dl, T, prob_form, static, tilt):
    """The mean-magnetisation step (weights over two wells, Sec. II.3) against the
    oracle's master-equation loop: loop record and area to rounding; tilt applies the
    field along (1, 2, -2)/3 instead of x."""
    rng = np.random.default_rng(11 + prob_form + 2 * static)
    n = 60
    axes = rng.normal(size=(n, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    axes[:5, 2] = 0.0       # axes in the field plane: degenerate plane at zero field
    axes[:5] /= np.linalg.norm(axes[:5], axis=1, keepdims=True)
    S, P, D = 100, 3, 1
    p = kmc.Params(Ms=4e5, Keff=1.3e4, d=12e-9, T=T, mu0Hmax=0.03, steps_per_period=S,
                   n_periods=P, n_discard=D, interactions=0, prob_form=prob_form,
                   dt_override=2e-10 if static else 0.0,
                   field_dir=(1.0, 2.0, -2.0) if tilt else (1.0, 0.0, 0.0))
    dv = kmc.derived(p)
    H, M, A = master.mean_loop(axes, p)
    Mg = np.empty((P - D) * S)
    Ag = np.empty(1)
    eh = kmc.field_unit(p)
    dl.dl_master(n, _p(axes), p.Ms, dv["BK"], dv["beta"], dv["nu0dt"], prob_form,
                 1 if T > 0 else 0, p.mu0Hmax, S, P, D, static, _p(eh), _p(Mg), _p(Ag))
    assert np.abs(Mg - M.ravel()).max() < 1e-9 * np.abs(M).max()
    assert abs(Ag[0] - A) < 1e-9 * max(abs(A), 1.0), (Ag[0], A)


def test_eq5_where_both_rates_underflow(dl):
    """Fig. 1(d) at T = 5 K (beta = 13107): barriers of about 0.055 K V put both
    e^-a terms of Eq. 5 near 1e-310, where a reciprocal of their sum overflows. The
    step must give P (within 1e-12 of the oracle's, which is below 1e-290 there) and
    the oracle's jump decisions, and the mean loop must stay finite and equal. At this
    beta an energy rounding of a few ulps moves a = beta * barrier by ~beta * 4e-16,
    so P is held to 5e-16 beta instead of 1e-12, and a decision may differ only
    where u lies that close to P."""
    rng = np.random.default_rng(41)
    n = 6000
    p = kmc.Params(Ms=1e6, Keff=1e6, d=12e-9, T=5.0, mu0Hmax=2.5, interactions=0,
                   steps_per_period=200, n_periods=2, n_discard=1)
    dv = kmc.derived(p)
    axes = rng.normal(size=(n, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    m = axes.copy()
    # fields just inside the switching field of each particle, opposite to its moment,
    # so the metastable barrier sweeps through 0..0.2 K V
    ph = rng.uniform(0.05, np.pi / 2 - 0.05, n)
    hsw = (np.cos(ph) ** (2 / 3) + np.sin(ph) ** (2 / 3)) ** -1.5
    h = hsw * (1 - rng.uniform(0.0, 0.6, n) ** 2)
    perp = np.cross(axes, rng.normal(size=(n, 3)))
    perp /= np.linalg.norm(perp, axis=1, keepdims=True)
    B = dv["BK"] * h[:, None] * (-np.cos(ph)[:, None] * axes + np.sin(ph)[:, None] * perp)
    m_new, info = kmc.step(np.zeros((n, 3)), axes, m, 77, p, 9, 0, B_override=B)
    a_c = dv["beta"] * (info.e3 - info.e_c)
    a_o = dv["beta"] * (info.e3 - info.e_o)
    band = info.two & (np.exp(-a_c) + np.exp(-a_o) < 2.2e-308) & (np.exp(-a_c) > 0)
    assert band.sum() > 10, band.sum()
    out = np.empty((n, 6))
    dl.dl_update(n, _p(B), _p(axes), _p(m), dv["BK"], dv["beta"], dv["nu0dt"], 0, 1, 9, 0, 77,
                 0, _p(out))
    assert np.all(np.isfinite(out))
    tol = 5e-16 * dv["beta"]
    assert np.abs(out[:, 3] - info.P).max() < tol
    dif = (out[:, 4] == 1.0) != info.jump
    assert np.all((np.abs(info.u - info.P) < tol)[dif])
    # the mean loop through the same regime
    n2 = 60
    ax2 = axes[:n2].copy()
    H, M, A = master.mean_loop(ax2, p)
    Mg = np.empty(p.steps_per_period)
    Ag = np.empty(1)
    eh = kmc.field_unit(p)
    dl.dl_master(n2, _p(ax2), p.Ms, dv["BK"], dv["beta"], dv["nu0dt"], 0, 1, p.mu0Hmax,
                 p.steps_per_period, 2, 1, 0, _p(eh), _p(Mg), _p(Ag))
    assert np.all(np.isfinite(Mg)) and np.isfinite(Ag[0])
    assert np.abs(Mg - M.ravel()).max() < 1e-9 * np.abs(M).max()
    assert abs(Ag[0] - A) < 1e-9 * abs(A)


def test_mul128_is_the_exact_product(dl):
    """The Philox rounds' 128-bit product (four 32 x 32 -> 64 multiply-adds with the
    carries folded in) equals the exact integer product, for random words and the
    edge cases 0, 1, 2^32 - 1, 2^32 and 2^64 - 1."""
    rng = np.random.default_rng(11)
    x = rng.integers(0, 2**63, size=2000, dtype=np.int64).astype(np.uint64) * np.uint64(2)
    x[1::2] += np.uint64(1)
    edge = np.array([0, 1, 2**32 - 1, 2**32, 2**64 - 1, 2**63, 2**63 - 1], dtype=np.uint64)
    x = np.concatenate([edge, x])
    out = np.zeros((len(x), 4), dtype=np.uint64)
    p = C.POINTER(C.c_uint64)
    dl.dl_mul128(len(x), x.ctypes.data_as(p), out.ctypes.data_as(p))
    for q, xv in enumerate(x.tolist()):
        for m, (lo, hi) in zip((0xD2E7470EE14C6C93, 0xCA5A826395121157),
                               ((out[q, 0], out[q, 1]), (out[q, 2], out[q, 3]))):
            prod = m * int(xv)
            assert int(lo) == prod & (2**64 - 1) and int(hi) == prod >> 64, (q, xv)

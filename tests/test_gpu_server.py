"""Continuous-batching server: a request's result is the same alone and when it runs
interleaved with other requests of different sizes and forms (it is also the same as a
direct run of the same replicas), and requests that can never fit the device-memory
budget are refused at submission."""
import time

import numpy as np
import pytest

from paper_1407_2737_amd import workloads as W

pytestmark = pytest.mark.gpu


def _req(lib, n, prec, seed, S=100, P=2):
    d = 12e-9
    R = d / 2 * (n / 0.05) ** (1 / 3)
    pos = W.place_random(n, R, d, seed)
    axes = W.axes_random_3d(n, seed + 1)
    kw = dict(Ms=4e5, Keff=1.3e4, d=d, T=300.0, tau0=1e-10, rho=5200.0, f=1e5, mu0Hmax=0.02,
              steps_per_period=S, n_periods=P, n_discard=1)
    return pos, axes, lib.Params.make(prec, **kw)


def _wait(srv, ids, timeout=240):
    out = {}
    t0 = time.time()
    while len(out) < len(ids):
        for i in ids:
            if i not in out:
                r = srv.poll(i)
                if r is not None:
                    out[i] = r
        assert time.time() - t0 < timeout, "server did not finish in time"
        time.sleep(0.01)
    return out


def test_alone_equals_mix(lib):
    ctx = lib.Context(0)
    A = _req(lib, 150, lib.FP32_FIELD, 11)
    srv = lib.Server(ctx, 8 << 30)
    ia = srv.submit(*A, seed=7, target_rel_err=0.02, min_replicas=64, max_replicas=128)
    alone = _wait(srv, [ia])[ia]
    srv.close()
    assert alone["status"] == 0 and alone["replicas"] in (64, 128)

    srv = lib.Server(ctx, 8 << 30)
    others = [_req(lib, 900, lib.FP32_FIELD, 21, S=60, P=3), _req(lib, 300, lib.BF16X3_WM, 31),
              _req(lib, 60, lib.FP64, 41, S=140), _req(lib, 2000, lib.FP32_FIELD, 51, S=40)]
    ids = [srv.submit(*others[0], seed=1, max_replicas=64),
           srv.submit(*others[1], seed=2, max_replicas=256)]
    time.sleep(0.05)                       # A arrives while the others run
    ib = srv.submit(*A, seed=7, target_rel_err=0.02, min_replicas=64, max_replicas=128)
    ids += [srv.submit(*others[2], seed=3, max_replicas=64),
            srv.submit(*others[3], seed=4, max_replicas=64)]
    res = _wait(srv, ids + [ib])
    srv.close()
    mix = res[ib]
    for key in ("area_Jm3", "area_se", "sar_Wkg", "sar_se", "replicas", "loops", "status"):
        assert mix[key] == alone[key], (key, mix[key], alone[key])
    assert all(res[i]["status"] == 0 for i in ids)
    assert mix["start_ns"] >= mix["submit_ns"] and mix["done_ns"] > mix["start_ns"]

    # the same replicas run directly give the same area
    a = lib.Assembly(ctx, A[0], A[1], A[2])
    a.run(alone["replicas"], seed=7)
    a.sync()
    direct = a.sar()
    assert direct["area"] == alone["area_Jm3"] and direct["area_se"] == alone["area_se"]


def test_budget_refusal(lib):
    ctx = lib.Context(0)
    srv = lib.Server(ctx, 1 << 20)          # 1 MiB
    pos, axes, p = _req(lib, 2000, lib.FP32_FIELD, 61)
    with pytest.raises(lib.MHError) as e:
        srv.submit(pos, axes, p, seed=1)
    assert e.value.code == -7
    srv.close()


def test_budget_counts_axis_sets_and_state(lib):
    """Admission counts every buffer a request's runs allocate: here 64 axis sets of
    5000 particles (10 MB) alone exceed an 8 MiB budget although the per-replica state
    of a one-replica round fits; with one axis set the same request is admitted and
    finishes."""
    ctx = lib.Context(0)
    n, d = 5000, 12e-9
    pos = W.place_lattice_disorder(n, d / 2 * (n / 0.05) ** (1 / 3), d, 71)
    kw = dict(Ms=4e5, Keff=1.3e4, d=d, T=300.0, tau0=1e-10, rho=5200.0, f=1e5, mu0Hmax=0.02,
              steps_per_period=100, n_periods=2, n_discard=1)
    p = lib.Params.make(lib.FP32_FIELD, **kw)
    srv = lib.Server(ctx, 8 << 20)
    with pytest.raises(lib.MHError) as e:
        srv.submit(pos, W.axes_random_3d(64 * n, 72), p, seed=1, min_replicas=1, max_replicas=1,
                   n_axes_sets=64)
    assert e.value.code == -7
    i = srv.submit(pos, W.axes_random_3d(n, 73), p, seed=1, min_replicas=1, max_replicas=1)
    r = _wait(srv, [i])[i]
    assert r["status"] == 0 and r["replicas"] == 1
    assert srv.progress(i) == 1      # a finished request reports all its replicas
    srv.close()


def test_submit_while_the_server_captures(lib):
    """Requests are submitted from the caller's thread while the server thread captures
    and replays the graphs of earlier requests (each admission changes the plan, so the
    server captures again): every submission must be accepted and every request must
    finish. The assembly upload of a submission runs on a non-blocking stream, so it
    takes no implicit dependency on the server's capturing stream."""
    ctx = lib.Context(0)
    srv = lib.Server(ctx, 32 << 30)
    forms = [lib.BF16X3_WM, lib.FP32_FIELD, lib.BF16X3_WM, lib.FP64]
    ids = []
    for q in range(24):
        n = (120, 500, 260, 80)[q % 4] + 7 * q
        req = _req(lib, n, forms[q % 4], 300 + q, S=100, P=3)
        ids.append(srv.submit(*req, seed=q, target_rel_err=0.5, min_replicas=64,
                              max_replicas=256 if forms[q % 4] == lib.BF16X3_WM else 64))
        time.sleep(0.002 * (q % 5))
    res = _wait(srv, ids, timeout=300)
    srv.close()
    assert all(res[i]["status"] == 0 for i in ids)
    assert all(res[i]["replicas"] >= 64 for i in ids)

"""GPU: the request loop (npb_server_*).  Requests of different sizes are
admitted by workspace size into the server's arena and batched; every
result must equal the single solve of the same request bit for bit (same
kernels, same launch shapes), and admission must refuse what cannot fit."""
import sys
import time

import numpy as np
import pytest

from paper_1410_2788_amd import inputs

pytestmark = pytest.mark.gpu


def _npb():
    from paper_1410_2788_amd import npb
    return npb


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wait(sv, tickets, timeout_s=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = sv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout_s, "server did not finish in time"
        time.sleep(0.002)
    return out


def test_server_results_equal_single_solves():
    npb = _npb()
    reqs = [inputs.small_globular(seed=40 + i, n=n, n_atoms=na, n_steps=3, precision="f32")
            for i, (n, na) in enumerate([(29, 50), (41, 120), (35, 80), (45, 150), (31, 60)])]
    ws = [npb.npb_workspace_bytes(npb.Molecule(w.molecule.xyz, w.molecule.q, w.molecule.radius).c,
                                  npb.make_grid(w.grid), npb.make_params(w.params)) for w in reqs]
    # arena for about three of them: admission splits the stream into batches
    budget = int(sum(sorted(ws)[-3:]) + 4096)
    sv = npb.Server(budget, max_batch=4, max_queue=16)
    try:
        tickets = [sv.submit(w.molecule, w.grid, w.params) for w in reqs]
        res = _wait(sv, tickets)
        st = sv.stats()
        _say("server stats:", st)
        assert st["completed"] == len(reqs) and st["batches"] >= 2
        for t, w in zip(tickets, reqs):
            status, r = res[t]
            assert status == npb.NPB_OK
            one = npb.solve(w.molecule, w.grid, w.params)
            assert r["dG"] == one["dG"] and r["G_m"] == one["G_m"], (r["dG"], one["dG"])
        with pytest.raises(npb.NPBError) as ei:
            sv.poll(tickets[0])  # released after its result was taken
        assert ei.value.status == npb.NPB_EINVAL
    finally:
        sv.close()


def test_server_refuses_what_cannot_fit_and_bad_requests():
    npb = _npb()
    small = inputs.small_globular(seed=50, n=25, n_atoms=20, n_steps=2, precision="f32")
    big = inputs.small_globular(seed=51, n=61, n_atoms=200, n_steps=2, precision="f32")
    wb = npb.npb_workspace_bytes(npb.Molecule(small.molecule.xyz, small.molecule.q,
                                              small.molecule.radius).c,
                                 npb.make_grid(small.grid), npb.make_params(small.params))
    sv = npb.Server(wb + 1024, max_batch=2, max_queue=4)
    try:
        with pytest.raises(npb.NPBError) as ei:
            sv.submit(big.molecule, big.grid, big.params)
        assert ei.value.status == npb.NPB_EBUSY
        bad = inputs.Molecule(np.array([[100.0, 0.0, 0.0]]), np.array([1.0]), np.array([1.0]))
        with pytest.raises(npb.NPBError) as ei:
            sv.submit(bad, small.grid, small.params)
        assert ei.value.status == npb.NPB_ERANGE
        t = sv.submit(small.molecule, small.grid, small.params)
        status, r = _wait(sv, [t])[t]
        assert status == npb.NPB_OK and np.isfinite(r["dG"])
    finally:
        sv.close()


def test_request_joining_mid_loop_finishes_first():
    """Continuous batching: a 103^3 request submitted while a 257^3 request
    (60 / 120 steps) is mid-loop joins the running launches and finishes
    first; both results equal their single solves bit for bit."""
    import dataclasses
    npb = _npb()
    big = inputs.serve_requests(1, precision="f32")[0]
    big.params = dataclasses.replace(big.params, n_steps=60)
    small = inputs.small_globular(seed=81, n_atoms=500, n=103, n_steps=20, precision="f32")
    _say(f"case server join: {big.grid.nx}^3 60/120 steps, then {small.grid.nx}^3 20/40 steps")
    ref_big = npb.solve(big.molecule, big.grid, big.params)
    ref_small = npb.solve(small.molecule, small.grid, small.params)
    sv = npb.Server(2 << 30, max_batch=4, max_queue=8)
    try:
        tb = sv.submit(big.molecule, big.grid, big.params)
        t0 = time.time()
        while sv.stats()["batches"] < 3:
            assert time.time() - t0 < 30.0, "the first request did not start"
            time.sleep(0.0005)
        ts = sv.submit(small.molecule, small.grid, small.params)
        order, out = [], {}
        while len(out) < 2:
            for t in (tb, ts):
                if t not in out:
                    r = sv.poll(t)
                    if r is not None:
                        out[t] = r
                        order.append(t)
            assert time.time() - t0 < 60.0, "server did not finish in time"
            time.sleep(0.0005)
        st = sv.stats()
    finally:
        sv.close()
    _say(f"  completion order {'small, big' if order == [ts, tb] else 'big, small'}; stats {st}")
    assert order == [ts, tb]
    for t, ref in ((tb, ref_big), (ts, ref_small)):
        status, r = out[t]
        assert status == npb.NPB_OK
        for k in ("dG", "dG_plain", "G_m", "G_0", "n_charge_nodes", "steps_done",
                  "grid_point_updates", "dG_err_est"):
            assert r[k] == ref[k], k

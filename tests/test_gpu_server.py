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

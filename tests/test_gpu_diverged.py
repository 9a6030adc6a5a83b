"""GPU: a run whose field holds a value that is not finite after a step is
reported as diverged (NPB_EDIVERGED, finite = 0): the paper's sign of an
unstable run is a non-finite result (Sec. 4.2).  The condition comes from
the inputs (a NaN in a caller-given initial field, or explicit Euler far
beyond its stability limit, whose iterates overflow) through ordinary
floating-point arithmetic; no kernel faults.  In a batch or the request
loop the diverged problem is reported alone: the other problems' results
equal their single solves bit for bit."""
import math
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


@pytest.mark.parametrize("scheme,where", [("LODIE2", "interior"), ("LODIE2", "shell"),
                                          ("AOSIE2", "interior"), ("MAOSIE", "interior"),
                                          ("LODCN2", "interior"), ("EULER", "interior")])
def test_nan_in_the_initial_field_is_reported_as_diverged(scheme, where):
    npb = _npb()
    b = inputs.sphere_benchmark(0.5)
    u0 = b.u0.copy()
    n = u0.shape[0]
    if where == "interior":
        u0[n // 2 + 2, n // 2 - 1, n // 2 + 1] = float("nan")
    else:
        u0[0, n // 2, n // 2] = float("nan")
    dt, steps = (1e-4, 5) if scheme == "EULER" else (0.05, 3)
    _say(f"case NaN in u0 ({where}) scheme={scheme} grid={n}^3 dt={dt} steps={steps}")
    p = npb.make_params_raw(b.eps_in, b.eps_out, b.kbar_sq, 1.0, dt, steps, scheme=scheme,
                            precision="f64")
    with pytest.raises(npb.NPBError) as ei:
        npb.FieldsSolver(b.solute, b.grid, p, u0, b.rho).run()
    assert ei.value.status == npb.NPB_EDIVERGED
    assert ei.value.result.finite == 0
    # the same problem without the NaN is finite
    ok = npb.FieldsSolver(b.solute, b.grid, p, b.u0, b.rho).run()
    assert ok["finite"]


def _unstable_euler():
    # tau = dt / alpha = 0.025, about fifty times the explicit limit
    # h^2 / (6 eps_out) at h = 0.5: the iterates grow ~47-fold per step and
    # overflow within a few hundred steps
    return inputs.small_globular(seed=61, n_atoms=10, n=21, precision="f64", scheme="EULER",
                                 n_steps=400, dt=1e-3)


def test_unstable_explicit_euler_is_reported_as_diverged():
    npb = _npb()
    w = _unstable_euler()
    _say("case unstable explicit Euler 21^3, tau 0.025, 400 / 800 steps")
    with pytest.raises(npb.NPBError) as ei:
        npb.solve(w.molecule, w.grid, w.params)
    assert ei.value.status == npb.NPB_EDIVERGED


def test_server_reports_the_diverged_request_alone():
    npb = _npb()
    good = [inputs.small_globular(seed=70 + i, n=n, n_atoms=na, n_steps=3, precision="f64")
            for i, (n, na) in enumerate([(29, 40), (25, 20), (33, 60)])]
    bad = _unstable_euler()
    singles = [npb.solve(w.molecule, w.grid, w.params) for w in good]
    _say("case server: 3 FP64 LODIE2 requests and one unstable explicit Euler request")
    sv = npb.Server(1 << 30, max_batch=8, max_queue=16)
    try:
        reqs = [good[0], bad, good[1], good[2]]
        tickets = [sv.submit(w.molecule, w.grid, w.params) for w in reqs]
        out = {}
        t0 = time.time()
        while len(out) < len(tickets):
            for t in tickets:
                if t not in out:
                    r = sv.poll(t)
                    if r is not None:
                        out[t] = r
            assert time.time() - t0 < 60.0, "server did not finish in time"
            time.sleep(0.002)
    finally:
        sv.close()
    st_bad, r_bad = out[tickets[1]]
    assert st_bad == npb.NPB_EDIVERGED and not r_bad["finite"]
    for t, ref in zip([tickets[0], tickets[2], tickets[3]], singles):
        st, r = out[t]
        assert st == npb.NPB_OK
        for k in ("dG", "dG_plain", "G_m", "G_0", "n_charge_nodes", "dG_err_est"):
            assert r[k] == ref[k], k

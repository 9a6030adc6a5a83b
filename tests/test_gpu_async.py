"""GPU checks of npb_solve_async (result delivered into page-locked host
memory, no host wait) and of the field_units switch, through the C ABI."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1410_2788_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_async_result_matches_the_synchronous_solve():
    import torch
    from paper_1410_2788_amd import npb
    w = inputs.small_globular(n=33, n_atoms=20, n_steps=6, seed=11)
    _say(f"case async grid=33^3 atoms=20 steps=6 scheme={w.params.scheme}")
    s = npb.Solver(w.molecule, w.grid, w.params, want_field=True)
    sync = s.run()
    phi_sync = s.field.cpu().numpy().copy()
    s.field.zero_()
    out = npb.AsyncResult()
    npb.solve_async(s, out)
    torch.cuda.current_stream().synchronize()
    got = out.result()
    for k in ("dG", "dG_plain", "G_m", "G_0", "grid_point_updates", "steps_done",
              "n_charge_nodes"):
        assert got[k] == sync[k], k
    assert math.isnan(got["device_ms"])
    assert got["finite"] == 1
    np.testing.assert_array_equal(s.field.cpu().numpy(), phi_sync)
    # a second problem enqueued behind the first on the same stream
    w2 = inputs.small_globular(n=29, n_atoms=12, n_steps=4, seed=12)
    s2 = npb.Solver(w2.molecule, w2.grid, w2.params)
    ref2 = s2.run()
    a, b = npb.AsyncResult(), npb.AsyncResult()
    npb.solve_async(s, a)
    npb.solve_async(s2, b)
    torch.cuda.current_stream().synchronize()
    assert a.result()["dG"] == sync["dG"] and b.result()["dG"] == ref2["dG"]


def test_async_rejects_pageable_result_memory():
    from paper_1410_2788_amd import npb
    w = inputs.small_globular(n=25, n_atoms=6, n_steps=2, seed=3)
    s = npb.Solver(w.molecule, w.grid, w.params)
    import ctypes
    buf = (ctypes.c_uint8 * ctypes.sizeof(npb.npb_result))()
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    with pytest.raises(npb.NPBError):
        npb.npb_solve_async(s.ctx, s.mol.c, s.grid, s.params, s.ws.data_ptr(), s.ws_bytes, None,
                            stream, ctypes.addressof(buf))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_dimensionless_field_is_the_kcal_field_over_kT(precision):
    import dataclasses
    from paper_1410_2788_amd import npb
    w = inputs.small_globular(n=31, n_atoms=15, n_steps=5, seed=5)
    w.params = dataclasses.replace(w.params, precision=precision)
    _say(f"case units prec={precision}")
    kcal = npb.solve(w.molecule, w.grid, w.params, want_field=True)
    dim = npb.solve(w.molecule, w.grid, w.params, want_field=True, field_units="dimensionless")
    assert dim["dG"] == kcal["dG"]
    kT = oracle.thermal_energy(w.params.temperature_K)
    np.testing.assert_allclose(dim["phi"] * kT, kcal["phi"], rtol=1e-14,
                               atol=1e-14 * np.max(np.abs(kcal["phi"])))


def test_async_solves_on_two_streams_sharing_one_context():
    """Solvers share one context per device; asynchronous solves queued on
    two streams, back to back with no host wait between them, each equal
    to its synchronous result (the context's staging buffers and launch
    tables are reused only after the enqueues that read them are done)."""
    import torch
    from paper_1410_2788_amd import npb
    w1 = inputs.small_globular(n=33, n_atoms=20, n_steps=6, seed=31, precision="f32")
    w2 = inputs.small_globular(n=29, n_atoms=12, n_steps=4, seed=32, precision="f32")
    _say("case async two streams: 33^3 and 29^3 f32, 3 rounds")
    s1 = npb.Solver(w1.molecule, w1.grid, w1.params)
    s2 = npb.Solver(w2.molecule, w2.grid, w2.params)
    ref1, ref2 = s1.run(), s2.run()
    st1, st2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for _ in range(3):
        a, b = npb.AsyncResult(), npb.AsyncResult()
        with torch.cuda.stream(st1):
            npb.solve_async(s1, a)
        with torch.cuda.stream(st2):
            npb.solve_async(s2, b)
        outs.append((a, b))
    torch.cuda.synchronize()
    for a, b in outs:
        for k in ("dG", "dG_plain", "G_m", "G_0", "n_charge_nodes"):
            assert a.result()[k] == ref1[k], k
            assert b.result()[k] == ref2[k], k

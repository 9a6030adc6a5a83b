"""GPU checks of npb_solve_noalloc (workspace and launch tables in the
library's static device scratch, no allocation at call time) against
npb_solve on the same inputs, through the C ABI: two calls in a row, the
second on a smaller problem, each equal to its npb_solve result bit for bit
(the same kernels on the same bytes; only the workspace address differs)."""
import sys

import numpy as np
import pytest

from paper_1410_2788_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(w, field_select=0):
    """(npb_solve result and field, npb_solve_noalloc result and field)."""
    import torch
    from paper_1410_2788_amd import npb
    s = npb.Solver(w.molecule, w.grid, w.params, want_field=True, field_select=field_select)
    ref = s.run()
    phi_ref = s.field.cpu().numpy().copy()
    del s
    params = npb.make_params(w.params, field_select=field_select)
    mol = npb.Molecule(w.molecule.xyz, w.molecule.q, w.molecule.radius)
    field = torch.full((w.grid.nz, w.grid.ny, w.grid.nx), float("nan"), dtype=torch.float64,
                       device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    res = npb.npb_solve_noalloc(npb.context(0), mol.c, npb.make_grid(w.grid), params,
                                field.data_ptr(), stream)
    return ref, phi_ref, npb.result_dict(res), field.cpu().numpy()


def _same(ref, got):
    bad = []
    for k in ("dG", "dG_plain", "G_m", "G_0", "grid_point_updates", "steps_done",
              "n_charge_nodes", "finite"):
        if ref[k] != got[k]:
            bad.append((k, ref[k], got[k]))
    return bad


def test_noalloc_matches_npb_solve_twice_then_smaller():
    # first call: FP32 RE+V on a ragged 45 x 41 x 37 grid, solvated field
    w1 = inputs.small_globular(seed=21, n_atoms=60, n=45, ny=41, nz=37, n_steps=5,
                               precision="f32")
    _say("case noalloc call 1: 45x41x37 f32 LODIE2 RE+V, 60 atoms")
    ref, phi_ref, got, phi = _pair(w1)
    bad = _same(ref, got)
    assert not bad, bad
    np.testing.assert_array_equal(phi, phi_ref)
    # second call on the same scratch: a smaller FP64 AOSIE2 problem, vacuum field
    w2 = inputs.small_globular(seed=22, n_atoms=15, n=29, n_steps=4, precision="f64",
                               scheme="AOSIE2")
    _say("case noalloc call 2: 29^3 f64 AOSIE2 RE+V, 15 atoms, vacuum field")
    ref2, phi_ref2, got2, phi2 = _pair(w2, field_select=1)
    bad = _same(ref2, got2)
    assert not bad, bad
    np.testing.assert_array_equal(phi2, phi_ref2)


def test_noalloc_refuses_a_problem_beyond_the_scratch():
    import torch
    from paper_1410_2788_amd import npb
    w = inputs.large_complex(precision="f32")
    params = npb.make_params(w.params)
    mol = npb.Molecule(w.molecule.xyz, w.molecule.q, w.molecule.radius)
    _say("case noalloc refusal: 321^3 f32 (619 MiB workspace)")
    with pytest.raises(npb.NPBError) as ei:
        npb.npb_solve_noalloc(npb.context(0), mol.c, npb.make_grid(w.grid), params, None,
                              torch.cuda.current_stream().cuda_stream)
    assert ei.value.status == npb.NPB_EINVAL
    assert "static scratch" in str(ei.value)

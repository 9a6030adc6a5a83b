"""GPU: batches of uneven problems through npb_solve_batch.

Every problem of a batch runs exactly the arithmetic it runs alone (the
same launch shape per grid, the same kernels), so batch results must equal
single solves bit for bit; small batches are also checked against the FP64
oracle with the single-solve tolerances (energies 1e-9 relative in FP64).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1410_2788_amd import inputs

pytestmark = pytest.mark.gpu


def _npb():
    from paper_1410_2788_amd import npb
    return npb


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mixed_batch(precision, schemes=("LODIE2",), steps=(4,), rich=(True,), vac=(True,)):
    probs = []
    sizes = [(29, 60), (37, 90), (45, 150), (53, 120), (33, 40), (41, 100)]
    for i, (n, na) in enumerate(sizes):
        w = inputs.small_globular(seed=20 + i, n=n, n_atoms=na, n_steps=steps[i % len(steps)],
                                  precision=precision, scheme=schemes[i % len(schemes)])
        w.params.richardson = rich[i % len(rich)]
        w.params.vacuum = vac[i % len(vac)]
        probs.append(w)
    return probs


def _check_against_singles(probs, fields=True):
    npb = _npb()
    bs = npb.BatchSolver([(w.molecule, w.grid, w.params) for w in probs], want_field=fields)
    _say("batch of", len(probs), "grids", [(w.grid.nx, w.grid.ny, w.grid.nz) for w in probs],
         "schemes", [w.params.scheme for w in probs])
    res = bs.run()
    for i, w in enumerate(probs):
        one = npb.solve(w.molecule, w.grid, w.params, want_field=fields)
        for k in ("dG", "dG_plain", "G_m", "G_0", "n_charge_nodes", "steps_done"):
            a, b = res[i][k], one[k]
            same = (a == b) or (isinstance(a, float) and np.isnan(a) and np.isnan(b))
            assert same, (i, k, a, b)
        if fields:
            f = bs.fields[i].cpu().numpy()
            assert np.array_equal(f, one["phi"]), (i, float(np.max(np.abs(f - one["phi"]))))
    return res


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_uneven_batch_equals_single_solves(precision):
    _check_against_singles(_mixed_batch(precision))


def test_batch_mixing_schemes_steps_and_flags():
    probs = _mixed_batch("f64", schemes=("LODIE2", "AOSIE2", "LODIE1", "AOSIE1"),
                         steps=(3, 5, 2), rich=(True, False), vac=(True, True, False))
    _check_against_singles(probs, fields=True)


def test_batch_replays_and_new_molecules():
    """Graph replay across calls, and new atom positions of the same sizes
    (re-staged, same graph) give the single-solve answers."""
    npb = _npb()
    probs = _mixed_batch("f32")[:3]
    bs = npb.BatchSolver([(w.molecule, w.grid, w.params) for w in probs])
    r1 = bs.run()
    r2 = bs.run()
    assert [r["dG"] for r in r1] == [r["dG"] for r in r2]
    # same sizes, other seeds: the staged atoms change, the launch shapes do not
    other = [inputs.small_globular(seed=90 + i, n=w.grid.nx, n_atoms=w.molecule.n_atoms,
                                   n_steps=w.params.n_steps, precision="f32")
             for i, w in enumerate(probs)]
    for i, w in enumerate(other):
        bs.mols[i] = npb.Molecule(w.molecule.xyz, w.molecule.q, w.molecule.radius)
    r3 = bs.run()
    for i, w in enumerate(other):
        one = npb.solve(w.molecule, w.grid, w.params)
        assert r3[i]["dG"] == one["dG"], (i, r3[i]["dG"], one["dG"])


def test_batch_against_oracle_fp64():
    npb = _npb()
    probs = _mixed_batch("f64")[:3]
    res = npb.BatchSolver([(w.molecule, w.grid, w.params) for w in probs]).run()
    for i, w in enumerate(probs):
        o = oracle.solve(w.molecule, w.grid, w.params)
        _say(f"problem {i}: dG gpu {res[i]['dG']!r} oracle {o['dG']!r}")
        for k in ("dG", "dG_plain"):
            assert abs(res[i][k] - o[k]) <= max(1e-8, 1e-9 * abs(o[k])), (i, k)


def test_batch_errors_name_the_problem():
    npb = _npb()
    probs = _mixed_batch("f64")[:2]
    bad = inputs.Molecule(np.array([[100.0, 0.0, 0.0]]), np.array([1.0]), np.array([1.0]))
    with pytest.raises(npb.NPBError) as ei:
        npb.BatchSolver([(probs[0].molecule, probs[0].grid, probs[0].params),
                         (bad, probs[1].grid, probs[1].params)])
    assert ei.value.status == npb.NPB_ERANGE

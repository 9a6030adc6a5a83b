"""GPU: npb_autotune picks line-solver launch shapes by timing; solves on
the tuned shapes still meet the oracle tolerances (a different chunk
partition changes rounding only)."""
import json
import os
import sys

import pytest

import oracle
from paper_1410_2788_amd import inputs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _npb():
    from paper_1410_2788_amd import npb
    return npb


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_autotune_small_fp64_against_oracle():
    npb = _npb()
    w = inputs.small_globular(seed=61, n=61, n_atoms=150, n_steps=3, precision="f64")
    s = npb.Solver(w.molecule, w.grid, w.params)
    before = npb.npb_launch_shapes(s.ctx, s.grid, s.params)
    ms = s.autotune()
    after = npb.npb_launch_shapes(s.ctx, s.grid, s.params)
    _say("shapes before", before, "after", after, "ms", ms)
    assert all(t > 0 for t in ms)
    for M, P, lw, thr in after:
        assert M * P >= 59 and thr == lw * P
    r = s.run()
    o = oracle.solve(w.molecule, w.grid, w.params)
    for k in ("dG", "dG_plain"):
        assert abs(r[k] - o[k]) <= max(1e-8, 1e-9 * abs(o[k])), (k, r[k], o[k])


def test_autotune_full_size_fp32_meets_energy_contract():
    npb = _npb()
    w = inputs.globular_2000(precision="f32")
    ref = json.load(open(os.path.join(GOLDEN, "globular_2000_161.json")))
    s = npb.Solver(w.molecule, w.grid, w.params)
    ms = s.autotune()
    shapes = npb.npb_launch_shapes(s.ctx, s.grid, s.params)
    r = s.run()
    tol = max(1e-3, 1e-5 * abs(ref["dG"]))
    _say("tuned shapes", shapes, "ms", ms, "dG err", r["dG"] - ref["dG"], "tol", tol)
    assert abs(r["dG"] - ref["dG"]) <= tol

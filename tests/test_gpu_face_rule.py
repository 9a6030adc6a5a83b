"""GPU parity of the face rule by location (npb_face_rule NPB_FACE_LOCATION:
eps at each half point from the half point's own position, the paper's
rule applied to the union of balls) against the FP64 oracle with
face_rule "location", through the C ABI.

Tolerances as in the other parity tests: FP64 field max|d phi| <= 1e-11
max|phi|, energies 1e-9 relative (1e-8 kcal/mol absolute); FP32 energies
max(1e-3 kcal/mol, 1e-5 |E|), field 2e-5 max|phi|."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
from paper_1410_2788_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _close(got, ref, rel, abs_):
    return abs(got - ref) <= max(abs_, rel * abs(ref))


def _case(scheme, precision="f64", n=41, ny=None, nz=None, n_atoms=120, seed=17, n_steps=6,
          dt=0.2, richardson=True):
    w = inputs.small_globular(seed=seed, n=n, ny=ny, nz=nz, n_atoms=n_atoms, n_steps=n_steps,
                              scheme=scheme, precision=precision, richardson=richardson, dt=dt)
    w.params = dataclasses.replace(w.params, face_rule="location")
    return w


def _compare(w):
    from paper_1410_2788_amd import npb
    p = w.params
    _say(f"case face=location scheme={p.scheme} prec={p.precision} "
         f"grid=({w.grid.nx},{w.grid.ny},{w.grid.nz}) atoms={w.molecule.n_atoms}")
    g = npb.solve(w.molecule, w.grid, p, want_field=True)
    o = oracle.solve(w.molecule, w.grid, p, want_fields=True)
    f64 = p.precision == "f64"
    rel, abs_ = (1e-9, 1e-8) if f64 else (1e-5, 1e-3)
    for k in ("dG", "dG_plain"):
        assert _close(g[k], o[k], rel, abs_), (k, g[k], o[k])
    for lv in range(2 if p.richardson else 1):
        assert _close(g["G_m"][lv], o["G_m"][lv], rel, abs_), ("G_m", lv)
        assert _close(g["G_0"][lv], o["G_0"][lv], rel, abs_), ("G_0", lv)
    err = float(np.max(np.abs(g["phi"] - o["phi_m"])) / np.max(np.abs(o["phi_m"])))
    _say(f"  dG gpu {g['dG']:.9f} oracle {o['dG']:.9f} field rel err {err:.3e}")
    assert err <= (1e-11 if f64 else 2e-5)
    return g, o


@pytest.mark.parametrize("scheme", ["LODIE2", "LODIE1", "AOSIE2", "AOSIE1", "LODCN2", "AOSCN2",
                                    "MAOSIE", "MAOSCN"])
def test_location_rule_matches_oracle_fp64(scheme):
    _compare(_case(scheme))


def test_location_rule_ragged_grid_and_fp32():
    _compare(_case("LODIE2", n=37, ny=33, nz=31, n_atoms=90, seed=19))
    _compare(_case("LODIE2", precision="f32"))
    _compare(_case("AOSIE2", precision="f32", seed=23))


def test_location_rule_explicit_euler():
    w = _case("EULER", n=29, n_atoms=40, n_steps=25, dt=1e-5, seed=29)
    _compare(w)


def test_location_rule_changes_the_answer():
    # the two rules differ only at the solute surface, which a molecule
    # always has: the energies must differ (both against their oracles)
    from paper_1410_2788_amd import npb
    w = _case("LODIE2")
    loc = npb.solve(w.molecule, w.grid, w.params)
    harm = npb.solve(w.molecule, w.grid, dataclasses.replace(w.params, face_rule="harmonic"))
    assert abs(loc["dG"] - harm["dG"]) > 1e-3 * abs(harm["dG"])


def test_location_rule_on_caller_given_fields():
    from paper_1410_2788_amd import npb
    b = inputs.sphere_benchmark(0.25, H=20.0)
    dt, n = 0.05, 20
    _say(f"case sphere fields face=location h=0.25 dt={dt} n={n}")
    p = npb.make_params_raw(b.eps_in, b.eps_out, b.kbar_sq, 1.0, dt, n, scheme="LODIE2",
                            face_rule="location")
    g = npb.FieldsSolver(b.solute, b.grid, p, b.u0, b.rho).run()
    pb = oracle.problem_from_fields(b.grid, b.solute, b.eps_in, b.eps_out, b.kbar_sq, b.rho, b.u0,
                                    face_rule="location")
    o = oracle.run(pb, dt, 1.0, n, "LODIE2")
    err = float(np.max(np.abs(g["u"] - o)) / np.max(np.abs(o)))
    _say("  rel err", err)
    assert err <= 1e-11

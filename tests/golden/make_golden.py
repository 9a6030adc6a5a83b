"""Write stored oracle results for full-size GPU parity checks.

Calls only the FP64 oracle (and the seeded input generators); nothing here
comes from the HIP library.

Usage:  python tests/golden/make_golden.py [name ...]
        names: globular_2000, globular_2000_direct, globular_2000_euler,
               large_complex_lod04,
               large_complex_lod02, large_complex_aos04, batch_mix_samples,
               serve_samples
        (no name: all of them; each writes its own JSON file)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1410_2788_amd import inputs  # noqa: E402

# field samples per solve: random interior nodes, random boundary-shell
# nodes, and the nodes of largest |phi| (at the charges)
N_INTERIOR, N_SHELL, N_PEAK = 192, 48, 16


def _stencil_nodes(w):
    """Distinct nodes touched by the trilinear stencils (zero weights included)."""
    g = w.grid
    nodes = set()
    for a in range(w.molecule.n_atoms):
        i0 = [int(np.floor((w.molecule.xyz[a, d] - g.origin[d]) / g.h)) for d in range(3)]
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    nodes.add(((i0[2] + cz) * g.ny + i0[1] + cy) * g.nx + i0[0] + cx)
    return len(nodes)


def _sample_nodes(g, phi, seed):
    """Flat (z, y, x) node indices: random interior, random shell, peaks."""
    rng = np.random.default_rng(seed)
    shape = (g.nz, g.ny, g.nx)
    inner = np.stack([rng.integers(1, n - 1, N_INTERIOR) for n in shape], axis=1)
    shell = np.stack([rng.integers(0, n, N_SHELL) for n in shape], axis=1)
    face = rng.integers(0, 3, N_SHELL)
    side = rng.integers(0, 2, N_SHELL)
    for k in range(N_SHELL):
        shell[k, face[k]] = 0 if side[k] == 0 else shape[face[k]] - 1
    idx = [np.ravel_multi_index(tuple(p), shape) for p in np.concatenate([inner, shell])]
    peaks = np.argsort(np.abs(phi).ravel())[-N_PEAK:]
    return sorted(set(int(i) for i in idx) | set(int(i) for i in peaks))


def _record(w, source, want_fields=True, seed=0):
    t = time.time()
    r = oracle.solve(w.molecule, w.grid, w.params, want_fields=want_fields)
    out = {
        "_source": source,
        "dG": r["dG"], "dG_plain": r["dG_plain"], "G_m": r["G_m"], "G_0": r["G_0"],
        "n_charge_nodes": int(_stencil_nodes(w)),
    }
    if want_fields:
        nodes = _sample_nodes(w.grid, r["phi_m"], seed)
        out["field_nodes"] = nodes
        out["phi_m"] = [float(r["phi_m"].ravel()[i]) for i in nodes]
        out["phi_0"] = [float(r["phi_0"].ravel()[i]) for i in nodes]
        out["phi_m_absmax"] = float(np.max(np.abs(r["phi_m"])))
        out["phi_0_absmax"] = float(np.max(np.abs(r["phi_0"])))
    out["oracle_seconds"] = time.time() - t
    return out


def _write(name, obj):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(obj, f, indent=1)
    print(name, {k: v for k, v in obj.items() if not isinstance(v, (list, dict))}, flush=True)


def globular_2000():
    w = inputs.globular_2000(precision="f64")
    out = _record(w, "oracle.solve on inputs.globular_2000() (seed 2, 161^3, RE+V, "
                     "dt 0.2/0.1, 20/40 steps)", want_fields=False)
    _write("globular_2000_161.json", out)


def globular_2000_direct():
    """The benchmark workload with the direct vacuum solve: Eq. (deltaG2)
    energy and sampled nodes of phi_0^direct and of the recovered potential."""
    w = inputs.globular_2000(precision="f64")
    t = time.time()
    r = oracle.solve(w.molecule, w.grid, w.params, want_fields=True, vacuum_direct=True)
    nodes = _sample_nodes(w.grid, r["phi_0_direct"], 2)
    out = {"_source": "oracle.solve(..., vacuum_direct=True) on inputs.globular_2000() (seed 2, "
                      "161^3, RE+V, dt 0.2/0.1, 20/40 steps)",
           "dG": r["dG"], "dG_direct": r["dG_direct"], "field_nodes": nodes,
           "phi_0_direct": [float(r["phi_0_direct"].ravel()[i]) for i in nodes],
           "phi_rec": [float(r["phi_rec"].ravel()[i]) for i in nodes],
           "phi_0_direct_absmax": float(np.max(np.abs(r["phi_0_direct"]))),
           "phi_rec_absmax": float(np.max(np.abs(r["phi_rec"]))),
           "oracle_seconds": time.time() - t}
    _write("globular_2000_161_direct.json", out)


def globular_2000_euler():
    """40 explicit Euler steps (dt 1e-5, alpha 1/25) of the benchmark
    molecule with the direct vacuum solve: G_m, Eq. (deltaG2) energy and
    sampled nodes of phi_m."""
    w = inputs.globular_2000_euler(n_steps=40)
    t = time.time()
    r = oracle.solve(w.molecule, w.grid, w.params, want_fields=True, vacuum_direct=True)
    nodes = _sample_nodes(w.grid, r["phi_m"], 3)
    out = {"_source": "oracle.solve(..., vacuum_direct=True) on inputs.globular_2000_euler("
                      "n_steps=40) (seed 2, 161^3, explicit Euler, dt 1e-5, alpha 1/25)",
           "G_m": r["G_m"], "dG_direct": r["dG_direct"], "field_nodes": nodes,
           "phi_m": [float(r["phi_m"].ravel()[i]) for i in nodes],
           "phi_m_absmax": float(np.max(np.abs(r["phi_m"]))),
           "oracle_seconds": time.time() - t}
    _write("globular_2000_161_euler40.json", out)


def _large(scheme, dt, n_steps, tag):
    w = inputs.large_complex(precision="f64", scheme=scheme, dt=dt, n_steps=n_steps)
    out = _record(w, f"oracle.solve on inputs.large_complex(scheme={scheme!r}, dt={dt}, "
                     f"n_steps={n_steps}) (seed 5, 30000 atoms, 321^3, h 0.35, RE+V)", seed=5)
    out.update(scheme=scheme, dt=dt, n_steps=n_steps)
    _write(f"large_complex_321_{tag}.json", out)


def large_complex_lod04():
    _large("LODIE2", 0.4, 20, "lodie2_dt04")


def large_complex_lod02():
    _large("LODIE2", 0.2, 40, "lodie2_dt02")


def large_complex_aos04():
    _large("AOSIE2", 0.4, 20, "aosie2_dt04")


BATCH_SAMPLES = (2, 44, 9)     # the smallest (79^3), a middle (127^3) and the largest (193^3) grid
SERVE_SAMPLES = (47, 37)       # 111^3 and 257^3 (19029 atoms)


def batch_mix_samples():
    out = {"_source": "oracle.solve on members of inputs.batch_mix(64) (seeds (3, i)), "
                      "LODIE2 and AOSIE2, RE+V, dt 0.2/0.1, 20/40 steps", "members": {}}
    for scheme in ("LODIE2", "AOSIE2"):
        ws = inputs.batch_mix(64, precision="f64", scheme=scheme)
        for i in BATCH_SAMPLES:
            out["members"][f"{scheme}:{i}"] = _record(ws[i], f"batch_mix(64)[{i}] {scheme}",
                                                      seed=300 + i)
    _write("batch_mix_64_samples.json", out)


def serve_samples():
    out = {"_source": "oracle.solve on members of inputs.serve_requests(48) (seeds (4, i)), "
                      "LODIE2 RE+V, dt 0.2/0.1, 20/40 steps", "members": {}}
    ws = inputs.serve_requests(48, precision="f64")
    for i in SERVE_SAMPLES:
        out["members"][str(i)] = _record(ws[i], f"serve_requests(48)[{i}]", seed=400 + i)
    _write("serve_48_samples.json", out)


ALL = [globular_2000, globular_2000_direct, globular_2000_euler, large_complex_lod04, large_complex_lod02, large_complex_aos04,
       batch_mix_samples, serve_samples]

if __name__ == "__main__":
    names = sys.argv[1:] or [f.__name__ for f in ALL]
    table = {f.__name__: f for f in ALL}
    for n in names:
        table[n]()

"""Python binding of libnpb.so: the C ABI of include/npb.h, one function per
entry point with the same name, plus `solve`, which allocates the device
workspace (a torch uint8 tensor) and the optional field, and marshals a
seeded workload into the C structs.  Every step of the computation runs in
the HIP library; this module only moves arguments.
"""
from __future__ import annotations

import ctypes as C
import os
import re
import threading
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnpb.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "npb.h")

NPB_OK, NPB_EINVAL, NPB_ERANGE, NPB_ENOMEM, NPB_EDEVICE, NPB_EDIVERGED, NPB_EBUSY = range(7)
STATUS_NAMES = {0: "NPB_OK", 1: "NPB_EINVAL", 2: "NPB_ERANGE", 3: "NPB_ENOMEM",
                4: "NPB_EDEVICE", 5: "NPB_EDIVERGED", 6: "NPB_EBUSY"}
SCHEMES = {"LODIE2": 0, "LODIE1": 1, "AOSIE2": 2, "AOSIE1": 3, "LODCN1": 4, "LODCN2": 5,
           "AOSCN1": 6, "AOSCN2": 7, "MAOSIE": 8, "MAOSCN": 9, "EULER": 10}
PRECISIONS = {"f64": 0, "f32": 1, "f32x": 2}
KERNEL_CLASSES = ["sweep_x", "sweep_y", "sweep_z", "setup", "init", "energy", "other", "direct",
                  "euler"]
# sweep launches split again by the kernel that ran them (npb_sweep_kernel)
SWEEP_KERNELS = ["x", "yz_plain", "yz_flow", "yz_general", "euler"]
ABI_VERSION = 7


class npb_molecule(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("xyz", C.POINTER(C.c_double)),
                ("q", C.POINTER(C.c_double)), ("radius", C.POINTER(C.c_double))]


class npb_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad_", C.c_int32),
                ("h", C.c_double), ("origin", C.c_double * 3)]


class npb_params(C.Structure):
    _fields_ = [("eps_in", C.c_double), ("eps_out", C.c_double), ("kappa_bar_sq", C.c_double),
                ("temperature_K", C.c_double), ("alpha", C.c_double), ("dt", C.c_double),
                ("n_steps", C.c_int32), ("scheme", C.c_int32), ("precision", C.c_int32),
                ("richardson", C.c_int32), ("vacuum", C.c_int32), ("field_select", C.c_int32),
                ("vacuum_direct", C.c_int32), ("field_units", C.c_int32),
                ("face_rule", C.c_int32)]


class npb_result(C.Structure):
    _fields_ = [("dG", C.c_double), ("dG_plain", C.c_double), ("G_m", C.c_double * 2),
                ("G_0", C.c_double * 2), ("grid_point_updates", C.c_double),
                ("device_ms", C.c_double), ("steps_done", C.c_int32),
                ("n_charge_nodes", C.c_int32), ("finite", C.c_int32), ("reserved", C.c_int32),
                ("dG_direct", C.c_double), ("dG_err_est", C.c_double)]


class npb_kernel_times(C.Structure):
    _fields_ = [("count", C.c_int64 * 12), ("ms", C.c_double * 12), ("bytes", C.c_double * 12),
                ("kcount", C.c_int64 * 8), ("kms", C.c_double * 8), ("kbytes", C.c_double * 8)]


class npb_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("refused", C.c_int64), ("batches", C.c_int64), ("queued", C.c_int64),
                ("busy_ms", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double)]


class NPBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_lib_lock = threading.Lock()


def load_library(path: str = LIB_PATH):
    """Load libnpb.so; raises if it has not been built (no fallback)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_1410_2788_amd.build`")
        # torch ships its own HIP runtime with the same soname as ROCm's;
        # loading torch first makes libnpb bind to that one, so the process
        # holds a single HIP runtime (two would each claim the device).
        import torch  # noqa: F401
        lib = C.CDLL(path)
        P = C.POINTER
        lib.npb_abi_version.restype = C.c_int
        if lib.npb_abi_version() != ABI_VERSION:
            raise ImportError(f"{path} has ABI version {lib.npb_abi_version()}, this binding "
                              f"expects {ABI_VERSION}: rebuild it")
        lib.npb_last_error.restype = C.c_char_p
        lib.npb_kappa_bar_sq.restype = C.c_double
        lib.npb_kappa_bar_sq.argtypes = [C.c_double, C.c_double]
        lib.npb_ctx_create.restype = C.c_int
        lib.npb_ctx_create.argtypes = [C.c_int, P(C.c_void_p)]
        lib.npb_ctx_destroy.restype = None
        lib.npb_ctx_destroy.argtypes = [C.c_void_p]
        lib.npb_ctx_set_timing.restype = C.c_int
        lib.npb_ctx_set_timing.argtypes = [C.c_void_p, C.c_int]
        lib.npb_ctx_set_graph.restype = C.c_int
        lib.npb_ctx_set_graph.argtypes = [C.c_void_p, C.c_int]
        lib.npb_ctx_get_kernel_times.restype = C.c_int
        lib.npb_ctx_get_kernel_times.argtypes = [C.c_void_p, P(npb_kernel_times)]
        lib.npb_validate.restype = C.c_int
        lib.npb_validate.argtypes = [P(npb_molecule), P(npb_grid), P(npb_params)]
        lib.npb_workspace_bytes.restype = C.c_int
        lib.npb_workspace_bytes.argtypes = [P(npb_molecule), P(npb_grid), P(npb_params),
                                            P(C.c_size_t)]
        lib.npb_solve_batch.restype = C.c_int
        lib.npb_solve_batch.argtypes = [C.c_void_p, C.c_int, P(npb_molecule), P(npb_grid),
                                        P(npb_params), P(C.c_void_p), P(C.c_size_t),
                                        P(C.c_void_p), C.c_void_p, P(npb_result)]
        lib.npb_server_create.restype = C.c_int
        lib.npb_server_create.argtypes = [C.c_void_p, C.c_size_t, C.c_int, C.c_int,
                                          P(C.c_void_p)]
        lib.npb_submit.restype = C.c_int
        lib.npb_submit.argtypes = [C.c_void_p, P(npb_molecule), P(npb_grid), P(npb_params),
                                   P(C.c_uint64)]
        lib.npb_poll.restype = C.c_int
        lib.npb_poll.argtypes = [C.c_void_p, C.c_uint64, P(npb_result), P(C.c_int)]
        lib.npb_server_get_stats.restype = C.c_int
        lib.npb_server_get_stats.argtypes = [C.c_void_p, P(npb_server_stats)]
        lib.npb_server_reset_stats.restype = C.c_int
        lib.npb_server_reset_stats.argtypes = [C.c_void_p]
        lib.npb_server_destroy.restype = None
        lib.npb_server_destroy.argtypes = [C.c_void_p]
        lib.npb_autotune.restype = C.c_int
        lib.npb_autotune.argtypes = [C.c_void_p, P(npb_molecule), P(npb_grid), P(npb_params),
                                     C.c_void_p, C.c_size_t, C.c_void_p, P(C.c_double)]
        lib.npb_launch_shapes.restype = C.c_int
        lib.npb_launch_shapes.argtypes = [C.c_void_p, P(npb_grid), P(npb_params), P(C.c_int32)]
        lib.npb_solve.restype = C.c_int
        lib.npb_solve.argtypes = [C.c_void_p, P(npb_molecule), P(npb_grid), P(npb_params),
                                  C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, P(npb_result)]
        lib.npb_solve_noalloc.restype = C.c_int
        lib.npb_solve_noalloc.argtypes = [C.c_void_p, P(npb_molecule), P(npb_grid),
                                          P(npb_params), C.c_void_p, C.c_void_p, P(npb_result)]
        lib.npb_solve_async.restype = C.c_int
        lib.npb_solve_async.argtypes = [C.c_void_p, P(npb_molecule), P(npb_grid), P(npb_params),
                                        C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                        C.c_void_p]
        lib.npb_default_grid.restype = C.c_int
        lib.npb_default_grid.argtypes = [P(npb_molecule), C.c_double, C.c_double, P(npb_grid)]
        lib.npb_fields_workspace_bytes.restype = C.c_int
        lib.npb_fields_workspace_bytes.argtypes = [P(npb_molecule), P(npb_grid), P(npb_params),
                                                   P(C.c_size_t)]
        lib.npb_solve_fields.restype = C.c_int
        lib.npb_solve_fields.argtypes = [C.c_void_p, P(npb_molecule), P(npb_grid), P(npb_params),
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                         C.c_void_p, C.c_void_p, P(npb_result)]
        _lib = lib
        return lib


def header_functions(path: str = HEADER_PATH):
    """Names of the functions include/npb.h declares."""
    text = re.sub(r"/\*.*?\*/", " ", open(path).read(), flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return sorted(set(re.findall(r"\b(npb_[a-z_0-9]+)\s*\(", text)))


def _check(status: int):
    if status != NPB_OK:
        raise NPBError(status, npb_last_error())


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)

def npb_abi_version() -> int:
    return load_library().npb_abi_version()


def npb_last_error() -> str:
    return load_library().npb_last_error().decode()


def npb_kappa_bar_sq(ionic_molar: float, temperature_K: float) -> float:
    return load_library().npb_kappa_bar_sq(ionic_molar, temperature_K)


def npb_ctx_create(device: int = 0) -> C.c_void_p:
    ctx = C.c_void_p()
    _check(load_library().npb_ctx_create(device, C.byref(ctx)))
    return ctx


def npb_ctx_destroy(ctx) -> None:
    load_library().npb_ctx_destroy(ctx)


def npb_ctx_set_timing(ctx, enable: bool) -> None:
    _check(load_library().npb_ctx_set_timing(ctx, 1 if enable else 0))


def npb_ctx_set_graph(ctx, enable: bool) -> None:
    _check(load_library().npb_ctx_set_graph(ctx, 1 if enable else 0))


def npb_ctx_get_kernel_times(ctx) -> dict:
    t = npb_kernel_times()
    _check(load_library().npb_ctx_get_kernel_times(ctx, C.byref(t)))
    out = {name: {"count": int(t.count[i]), "ms": float(t.ms[i]), "bytes": float(t.bytes[i])}
           for i, name in enumerate(KERNEL_CLASSES)}
    out["by_kernel"] = {name: {"count": int(t.kcount[i]), "ms": float(t.kms[i]),
                               "bytes": float(t.kbytes[i])}
                        for i, name in enumerate(SWEEP_KERNELS)}
    return out


def npb_validate(mol: npb_molecule, grid: npb_grid, params: npb_params) -> int:
    """Returns the status code (does not raise)."""
    return load_library().npb_validate(C.byref(mol), C.byref(grid), C.byref(params))


def npb_workspace_bytes(mol: npb_molecule, grid: npb_grid, params: npb_params) -> int:
    n = C.c_size_t()
    _check(load_library().npb_workspace_bytes(C.byref(mol), C.byref(grid), C.byref(params),
                                              C.byref(n)))
    return int(n.value)


def npb_solve(ctx, mol: npb_molecule, grid: npb_grid, params: npb_params, d_ws: int,
              ws_bytes: int, d_field_out: Optional[int], stream: int) -> npb_result:
    res = npb_result()
    st = load_library().npb_solve(ctx, C.byref(mol), C.byref(grid), C.byref(params),
                                  C.c_void_p(d_ws), ws_bytes,
                                  C.c_void_p(d_field_out) if d_field_out else None,
                                  C.c_void_p(stream), C.byref(res))
    if st != NPB_OK:
        err = NPBError(st, npb_last_error())
        err.result = res
        raise err
    return res


def npb_solve_noalloc(ctx, mol: npb_molecule, grid: npb_grid, params: npb_params,
                      d_field_out: Optional[int], stream: int) -> npb_result:
    """npb_solve with the workspace in the library's static device scratch."""
    res = npb_result()
    st = load_library().npb_solve_noalloc(ctx, C.byref(mol), C.byref(grid), C.byref(params),
                                          C.c_void_p(d_field_out) if d_field_out else None,
                                          C.c_void_p(stream), C.byref(res))
    if st != NPB_OK:
        err = NPBError(st, npb_last_error())
        err.result = res
        raise err
    return res


def npb_solve_batch(ctx, mols, grids, params, d_ws, ws_bytes, d_field_out, stream) -> list:
    """Arrays of C structs / pointers in, a list of npb_result out."""
    n = len(mols)
    M = (npb_molecule * n)(*mols)
    G = (npb_grid * n)(*grids)
    Pp = (npb_params * n)(*params)
    W = (C.c_void_p * n)(*[C.c_void_p(p) for p in d_ws])
    B = (C.c_size_t * n)(*ws_bytes)
    F = None
    if d_field_out is not None:
        F = (C.c_void_p * n)(*[C.c_void_p(p) if p else None for p in d_field_out])
    R = (npb_result * n)()
    st = load_library().npb_solve_batch(ctx, n, M, G, Pp, W, B, F, C.c_void_p(stream), R)
    if st != NPB_OK:
        err = NPBError(st, npb_last_error())
        err.results = list(R)
        raise err
    return list(R)


def npb_autotune(ctx, mol: npb_molecule, grid: npb_grid, params: npb_params, d_ws: int,
                 ws_bytes: int, stream: int) -> list:
    ms = (C.c_double * 3)()
    _check(load_library().npb_autotune(ctx, C.byref(mol), C.byref(grid), C.byref(params),
                                       C.c_void_p(d_ws), ws_bytes, C.c_void_p(stream), ms))
    return list(ms)


def npb_launch_shapes(ctx, grid: npb_grid, params: npb_params) -> list:
    """[(M, P, lines or tile width, threads) for x, y, z]."""
    out = (C.c_int32 * 12)()
    _check(load_library().npb_launch_shapes(ctx, C.byref(grid), C.byref(params), out))
    return [tuple(out[4 * d:4 * d + 4]) for d in range(3)]


def npb_solve_async(ctx, mol: npb_molecule, grid: npb_grid, params: npb_params, d_ws: int,
                    ws_bytes: int, d_field_out: Optional[int], stream: int,
                    pinned_out: int) -> None:
    """Enqueue a solve; the npb_result lands at pinned_out (page-locked host
    memory) when the stream's work completes."""
    _check(load_library().npb_solve_async(ctx, C.byref(mol), C.byref(grid), C.byref(params),
                                          d_ws, ws_bytes, d_field_out, stream, pinned_out))


def npb_default_grid(mol: npb_molecule, h: float, margin: float) -> npb_grid:
    g = npb_grid()
    _check(load_library().npb_default_grid(C.byref(mol), h, margin, C.byref(g)))
    return g


def npb_fields_workspace_bytes(mol: npb_molecule, grid: npb_grid, params: npb_params) -> int:
    n = C.c_size_t()
    _check(load_library().npb_fields_workspace_bytes(C.byref(mol), C.byref(grid),
                                                     C.byref(params), C.byref(n)))
    return int(n.value)


def npb_solve_fields(ctx, solute: npb_molecule, grid: npb_grid, params: npb_params, d_u0: int,
                     d_rho: int, d_ws: int, ws_bytes: int, d_u_out: Optional[int],
                     stream: int) -> npb_result:
    res = npb_result()
    st = load_library().npb_solve_fields(ctx, C.byref(solute), C.byref(grid), C.byref(params),
                                         d_u0, d_rho, d_ws, ws_bytes, d_u_out, stream,
                                         C.byref(res))
    if st != NPB_OK:
        err = NPBError(st, npb_last_error())
        err.result = res
        raise err
    return res


def npb_server_create(ctx, hbm_budget: int, max_batch: int = 16, max_queue: int = 256):
    sv = C.c_void_p()
    _check(load_library().npb_server_create(ctx, hbm_budget, max_batch, max_queue,
                                            C.byref(sv)))
    return sv


def npb_submit(server, mol: npb_molecule, grid: npb_grid, params: npb_params) -> int:
    t = C.c_uint64()
    _check(load_library().npb_submit(server, C.byref(mol), C.byref(grid), C.byref(params),
                                     C.byref(t)))
    return int(t.value)


def npb_poll(server, ticket: int):
    """(done, status, npb_result or None); raises NPBError for an unknown ticket."""
    res = npb_result()
    done = C.c_int()
    st = load_library().npb_poll(server, ticket, C.byref(res), C.byref(done))
    if not done.value:
        _check(st)
        return False, NPB_OK, None
    return True, st, res


def npb_server_get_stats(server) -> dict:
    s = npb_server_stats()
    _check(load_library().npb_server_get_stats(server, C.byref(s)))
    return {k: getattr(s, k) for k, _ in npb_server_stats._fields_}


def npb_server_reset_stats(server) -> None:
    _check(load_library().npb_server_reset_stats(server))


def npb_server_destroy(server) -> None:
    load_library().npb_server_destroy(server)


# ---------------------------------------------------------------------------
# marshalling helpers

class Molecule:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, xyz, q, radius):
        self.xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
        self.q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1))
        self.radius = np.ascontiguousarray(np.asarray(radius, dtype=np.float64).reshape(-1))
        dp = C.POINTER(C.c_double)
        self.c = npb_molecule(self.q.shape[0], self.xyz.ctypes.data_as(dp),
                              self.q.ctypes.data_as(dp), self.radius.ctypes.data_as(dp))


def make_grid(g) -> npb_grid:
    o = (C.c_double * 3)(*[float(v) for v in g.origin])
    return npb_grid(int(g.nx), int(g.ny), int(g.nz), 0, float(g.h), o)


FIELD_UNITS = {"kcal": 0, "dimensionless": 1}
FACE_RULES = {"harmonic": 0, "location": 1}


def make_params(p, field_select: int = 0, vacuum_direct: bool = False,
                field_units: str = "kcal") -> npb_params:
    kb2 = npb_kappa_bar_sq(p.ionic_molar, p.temperature_K)
    return npb_params(float(p.eps_in), float(p.eps_out), kb2, float(p.temperature_K),
                      float(p.alpha), float(p.dt), int(p.n_steps), SCHEMES[p.scheme],
                      PRECISIONS[p.precision], 1 if p.richardson else 0, 1 if p.vacuum else 0,
                      int(field_select), 1 if vacuum_direct else 0, FIELD_UNITS[field_units],
                      FACE_RULES[getattr(p, "face_rule", "harmonic")])


_ctx_cache = {}


def context(device: int = 0):
    if device not in _ctx_cache:
        _ctx_cache[device] = npb_ctx_create(device)
    return _ctx_cache[device]


class Solver:
    """Reusable device state for one problem shape: the workspace and the
    optional field buffer are allocated once (torch), then `run` calls
    npb_solve on the current torch stream."""

    def __init__(self, mol, grid, params, device: int = 0, want_field: bool = False,
                 field_select: int = 0, vacuum_direct: bool = False, field_units: str = "kcal"):
        import torch
        self.torch = torch
        self.device = device
        self.mol = Molecule(mol.xyz, mol.q, mol.radius)
        self.grid = make_grid(grid)
        self.params = make_params(params, field_select, vacuum_direct, field_units)
        self.ctx = context(device)
        self.ws_bytes = npb_workspace_bytes(self.mol.c, self.grid, self.params)
        dev = torch.device("cuda", device)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.field = None
        if want_field:
            self.field = torch.empty((grid.nz, grid.ny, grid.nx), dtype=torch.float64, device=dev)

    def autotune(self) -> list:
        """Tune this problem's launch shapes on its own workspace (ctx-wide)."""
        stream = self.torch.cuda.current_stream(self.device).cuda_stream
        return npb_autotune(self.ctx, self.mol.c, self.grid, self.params, self.ws.data_ptr(),
                            self.ws_bytes, stream)

    def run(self) -> dict:
        torch = self.torch
        stream = torch.cuda.current_stream(self.device).cuda_stream
        res = npb_solve(self.ctx, self.mol.c, self.grid, self.params, self.ws.data_ptr(),
                        self.ws_bytes, self.field.data_ptr() if self.field is not None else None,
                        stream)
        return result_dict(res)


class FieldsSolver:
    """npb_solve_fields on caller-given dense fields (numpy [nz][ny][nx],
    dimensionless): the initial field u0 (its shell is the Dirichlet data)
    and the source rho; `solute` gives the solute balls.  `params` is an
    npb_params (built with make_params or make_params_raw)."""

    def __init__(self, solute, grid, params: npb_params, u0, rho, device: int = 0,
                 graphs: bool = True):
        import numpy as np
        import torch
        self.torch = torch
        self.device = device
        self.mol = Molecule(solute.xyz, solute.q, solute.radius)
        self.grid = make_grid(grid)
        self.params = params
        self.ctx = context(device)
        dev = torch.device("cuda", device)
        self.u0 = torch.from_numpy(np.ascontiguousarray(u0, dtype=np.float64)).to(dev)
        self.rho = torch.from_numpy(np.ascontiguousarray(rho, dtype=np.float64)).to(dev)
        self.ws_bytes = npb_fields_workspace_bytes(self.mol.c, self.grid, self.params)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.u = torch.empty_like(self.u0)
        self.graphs = graphs

    def run(self) -> dict:
        stream = self.torch.cuda.current_stream(self.device).cuda_stream
        npb_ctx_set_graph(self.ctx, self.graphs)
        try:
            res = npb_solve_fields(self.ctx, self.mol.c, self.grid, self.params,
                                   self.u0.data_ptr(), self.rho.data_ptr(), self.ws.data_ptr(),
                                   self.ws_bytes, self.u.data_ptr(), stream)
        finally:
            npb_ctx_set_graph(self.ctx, True)
        out = result_dict(res)
        out["u"] = self.u.cpu().numpy()
        return out


def make_params_raw(eps_in, eps_out, kappa_bar_sq, alpha, dt, n_steps, scheme="LODIE2",
                    precision="f64", richardson=False, temperature_K=298.0,
                    face_rule="harmonic") -> npb_params:
    """npb_params with kbar^2 given directly (Angstrom^-2 or dimensionless)."""
    return npb_params(float(eps_in), float(eps_out), float(kappa_bar_sq), float(temperature_K),
                      float(alpha), float(dt), int(n_steps), SCHEMES[scheme],
                      PRECISIONS[precision], 1 if richardson else 0, 0, 0, 0, 0,
                      FACE_RULES[face_rule])


class AsyncResult:
    """A page-locked npb_result filled by npb_solve_async."""

    def __init__(self):
        import torch
        self.buf = torch.zeros(C.sizeof(npb_result), dtype=torch.uint8).pin_memory()

    def result(self) -> dict:
        return result_dict(npb_result.from_address(self.buf.data_ptr()))


def solve_async(solver: "Solver", out: AsyncResult) -> None:
    """Enqueue solver's solve on the current torch stream without waiting;
    out.result() is valid once the stream has completed."""
    stream = solver.torch.cuda.current_stream(solver.device).cuda_stream
    npb_solve_async(solver.ctx, solver.mol.c, solver.grid, solver.params, solver.ws.data_ptr(),
                    solver.ws_bytes,
                    solver.field.data_ptr() if solver.field is not None else None, stream,
                    out.buf.data_ptr())


class BatchSolver:
    """Device state for a batch of problems (any mix of sizes): one
    workspace per problem, allocated once; `run` solves them all together
    with npb_solve_batch on the current torch stream."""

    def __init__(self, problems, device: int = 0, want_field: bool = False):
        import torch
        self.torch = torch
        self.device = device
        self.mols = [Molecule(m.xyz, m.q, m.radius) for m, _, _ in problems]
        self.grids = [make_grid(g) for _, g, _ in problems]
        self.params = [make_params(p) for _, _, p in problems]
        self.ctx = context(device)
        dev = torch.device("cuda", device)
        self.ws_bytes = [npb_workspace_bytes(m.c, g, p)
                         for m, g, p in zip(self.mols, self.grids, self.params)]
        self.ws = [torch.empty(b, dtype=torch.uint8, device=dev) for b in self.ws_bytes]
        self.fields = None
        if want_field:
            self.fields = [torch.empty((g.nz, g.ny, g.nx), dtype=torch.float64, device=dev)
                           for _, g, _ in problems]

    def run(self) -> list:
        torch = self.torch
        stream = torch.cuda.current_stream(self.device).cuda_stream
        res = npb_solve_batch(self.ctx, [m.c for m in self.mols], self.grids, self.params,
                              [w.data_ptr() for w in self.ws], self.ws_bytes,
                              [f.data_ptr() for f in self.fields] if self.fields else None,
                              stream)
        return [result_dict(r) for r in res]


class Server:
    """The request loop of include/npb.h: submit molecules as they arrive,
    poll for results.  hbm_budget bytes of device memory are held until
    close()."""

    def __init__(self, hbm_budget: int, max_batch: int = 16, max_queue: int = 256,
                 device: int = 0):
        self.handle = npb_server_create(context(device), hbm_budget, max_batch, max_queue)

    def submit(self, mol, grid, params) -> int:
        m = Molecule(mol.xyz, mol.q, mol.radius)  # copied by the library before returning
        return npb_submit(self.handle, m.c, make_grid(grid), make_params(params))

    def poll(self, ticket: int):
        """None while pending, else (status, result dict)."""
        done, st, res = npb_poll(self.handle, ticket)
        return None if not done else (st, result_dict(res))

    def stats(self) -> dict:
        return npb_server_get_stats(self.handle)

    def reset_stats(self) -> None:
        npb_server_reset_stats(self.handle)

    def close(self) -> None:
        if self.handle:
            npb_server_destroy(self.handle)
            self.handle = None


def result_dict(res: npb_result) -> dict:
    return {"dG": res.dG, "dG_plain": res.dG_plain, "G_m": [res.G_m[0], res.G_m[1]],
            "G_0": [res.G_0[0], res.G_0[1]], "grid_point_updates": res.grid_point_updates,
            "device_ms": res.device_ms, "steps_done": res.steps_done,
            "n_charge_nodes": res.n_charge_nodes, "finite": bool(res.finite),
            "dG_direct": res.dG_direct, "dG_err_est": res.dG_err_est}


def solve(mol, grid, params, device: int = 0, want_field: bool = False,
          field_select: int = 0, vacuum_direct: bool = False, field_units: str = "kcal") -> dict:
    """One solve; with want_field the result also holds 'phi' (numpy, FP64,
    [nz][ny][nx], kcal/mol/e or dimensionless) as chosen by field_select."""
    s = Solver(mol, grid, params, device, want_field, field_select, vacuum_direct, field_units)
    out = s.run()
    if want_field:
        out["phi"] = s.field.cpu().numpy()
    return out

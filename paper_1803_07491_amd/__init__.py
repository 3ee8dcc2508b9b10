"""MI355X (gfx950) analytic-BOP energy path — Python binding.

Thin ctypes layer over ``libbop.so`` (C ABI in ``include/bop.h``): it checks
tensor dtypes, devices and contiguity, passes device pointers and the current
HIP stream, and allocates the caller-side buffers the ABI asks for.  Every
step of the computation runs in the library's HIP kernels; if the library is
not built this module raises instead of computing anything itself.

Entry points mirror the ABI: ``build_neighbours``, ``build_H``,
``moments_plan`` / ``moments``, ``recursion``, ``energy``, ``scf_step``;
``EnergyPath`` strings them together for a structure.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbop.so")

BOP_OK, BOP_E_ARG, BOP_E_CAPACITY, BOP_E_HIP, BOP_E_UNSUPPORTED, BOP_E_NOT_CONVERGED = 0, -1, -2, -3, -4, -5
F64, F32, BF16, F16 = 0, 1, 2, 3
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}
MAX_SPECIES = 3
N_CHANNELS = 14
CHANNELS = ("sss", "sps", "pss", "sds", "dss", "pps", "ppp",
            "pds", "dps", "pdp", "dpp", "dds", "ddp", "ddd")

FLAG_BREAKDOWN, FLAG_NONFINITE, FLAG_OUTSIDE, FLAG_NARROW, FLAG_DIVERGENT = 1, 2, 4, 8, 16


class BopError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bop error {code}: {msg}")
        self.code = code


class Model(C.Structure):
    _fields_ = [
        ("n_species", C.c_int),
        ("n_orb", C.c_int),
        ("r_cut", C.c_double),
        ("d_cut", C.c_double),
        ("onsite", (C.c_double * 3) * MAX_SPECIES),
        ("form", (C.c_ubyte * N_CHANNELS) * (MAX_SPECIES * MAX_SPECIES)),
        ("beta0", (C.c_double * N_CHANNELS) * (MAX_SPECIES * MAX_SPECIES)),
        ("r0", (C.c_double * N_CHANNELS) * (MAX_SPECIES * MAX_SPECIES)),
        ("q", (C.c_double * N_CHANNELS) * (MAX_SPECIES * MAX_SPECIES)),
    ]


MAX_NMAX = 40


class Tuning(C.Structure):
    _fields_ = [("tile_atoms", C.c_int), ("block_threads", C.c_int), ("batch_tiles", C.c_int),
                ("chunk_rows", C.c_int), ("plan_search", C.c_int)]


class Plan(C.Structure):
    _fields_ = [("n_atoms", C.c_int), ("n_orb", C.c_int), ("n_max", C.c_int), ("dtype", C.c_int),
                ("tile_atoms", C.c_int), ("n_tiles", C.c_int), ("block_threads", C.c_int),
                ("batch_tiles", C.c_int), ("chunk_rows", C.c_int), ("deg_max", C.c_int),
                ("rows_cap", C.c_int), ("rows_k", C.c_int * (MAX_NMAX // 2 + 1)),
                ("search", C.c_int), ("ws_bytes", C.c_size_t), ("r_max", C.c_double)]


class PathRadius(C.Structure):
    _fields_ = [("r_max", C.c_double), ("r_cut", C.c_double), ("cell", C.c_double * 9), ("pos", C.c_void_p)]


def path_radius(r_max, r_cut, cell, pos):
    """The ABI's path-radius struct (``pos`` a device tensor that must stay
    alive while the plan is used), or None for r_max <= 0."""
    if not r_max or r_max <= 0:
        return None
    r = PathRadius()
    r.r_max, r.r_cut = float(r_max), float(r_cut)
    for e, v in enumerate(np.ascontiguousarray(cell, np.float64).reshape(9)):
        r.cell[e] = float(v)
    r.pos = pos.data_ptr()
    return r


P = C.c_void_p


class System(C.Structure):
    _fields_ = [
        ("model", Model),
        ("n_atoms", C.c_int), ("n_max", C.c_int), ("n_exp", C.c_int), ("dtype", C.c_int),
        ("method", C.c_int),
        ("species", P), ("n0", P), ("row_ptr", P), ("nbr_j", P), ("order", P),
        ("n_pairs", C.c_long),
        ("H_on", P), ("H_bond", P),
        ("plan", Plan),
        ("moments_ws", P), ("moments_ws_bytes", C.c_size_t),
        ("mu", P), ("a", P), ("b", P), ("a_inf", P), ("b_inf", P), ("flags", P),
        ("energy_ws", P), ("energy_ws_bytes", C.c_size_t),
        ("n_elec", C.c_double),
        ("E_F", P), ("N_atom", P), ("U_atom", P), ("dos_atom", P), ("U_total", P),
    ]


class Magnetism(C.Structure):
    _fields_ = [("stoner", C.c_double * MAX_SPECIES), ("B_z", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(the BOP path has no CPU fallback)")
    lib = C.CDLL(path)
    lib.bop_last_error.argtypes = [C.c_char_p, C.c_size_t]
    lib.bop_neighbours_workspace_size.restype = C.c_size_t
    lib.bop_neighbours_workspace_size.argtypes = [C.c_int, P, C.c_double]
    lib.bop_build_neighbours.argtypes = [C.c_int, P, P, C.c_double, C.c_long, P, P, P, P, P,
                                         C.POINTER(C.c_long), P, C.c_size_t, P]
    lib.bop_build_H.argtypes = [C.POINTER(Model), C.c_int, P, P, P, P, P, C.c_long, C.c_int, P, P, P]
    lib.bop_moments_plan_scratch_size.restype = C.c_size_t
    lib.bop_moments_plan_scratch_size.argtypes = [C.c_int]
    lib.bop_moments_plan.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, P, P, C.POINTER(Tuning),
                                     C.POINTER(PathRadius), P, C.c_size_t, C.POINTER(Plan), P]
    lib.bop_moments_prepare.argtypes = [C.POINTER(Plan), P, P, P, C.POINTER(PathRadius), P, C.c_size_t, P]
    lib.bop_moments.argtypes = [C.POINTER(Plan), P, P, P, P, P, C.c_size_t, P]
    lib.bop_recursion.argtypes = [C.c_int, C.c_int, P, C.c_int, C.c_double, C.c_double, P, P, P, P, P, P]
    lib.bop_energy_workspace_size.restype = C.c_size_t
    lib.bop_energy_workspace_size.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.bop_energy.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, P, P, P, P, P, C.c_double, C.c_int,
                               P, P, P, P, P, P, P, C.c_size_t, P]
    lib.bop_energy_noalloc.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, P, P, P, P, P, C.c_double, C.c_int,
                                       P, P, P, P, P, P, P]
    lib.bop_scf_step.argtypes = [C.POINTER(System), C.c_double, C.c_double, C.c_double, P, P, P, P, P]
    lib.bop_broyden_workspace_size.restype = C.c_size_t
    lib.bop_broyden_workspace_size.argtypes = [C.c_int, C.c_int]
    lib.bop_scf_step_broyden.argtypes = [C.POINTER(System), C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                         P, P, P, P, P, C.c_size_t, P]
    lib.bop_spin_shifts.argtypes = [C.c_int, P, C.POINTER(Magnetism), P, P, P, P]
    lib.bop_mag_energy.argtypes = [C.POINTER(System), C.POINTER(Magnetism), P, P, P, P, P]
    lib.bop_mag_scf_step.argtypes = [C.POINTER(System), C.POINTER(Magnetism), C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_double, P, P, P, P, P, P, P, P]
    lib.bop_features.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, P]
    lib.bop_mlp_forward.argtypes = [C.c_int, P, P, P, P]
    lib.bop_feature_stats.argtypes = [C.c_int, P, P, P, P]
    lib.bop_standardise.argtypes = [C.c_int, P, P, P, P, P]
    lib.bop_mlp_shift.argtypes = [C.c_int, P, P, P, P]
    lib.bop_mlp_train_workspace_size.restype = C.c_size_t
    lib.bop_mlp_train_workspace_size.argtypes = [C.c_int]
    lib.bop_mlp_train_step.argtypes = [C.c_int, P, P, P, P, P, P, C.c_int, C.c_float, P, P, P, C.c_size_t, P]
    lib.bop_mlp_backward.argtypes = [C.c_int, P, P, P, P, P, P, P, C.c_size_t, P]
    lib.bop_mlp_adam.argtypes = [P, P, P, P, C.c_int, C.c_float, P]
    lib.bop_atom_average.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, P]
    lib.bop_energy_atom_averaged.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, P, P, P, P, P, C.c_double,
                                             C.c_int, P, P, P, P, P, P, P, C.c_size_t, P]
    lib.bop_weights_workspace_size.restype = C.c_size_t
    lib.bop_weights_workspace_size.argtypes = [C.c_int, C.c_int]
    lib.bop_weights.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, P, C.c_size_t, P]
    lib.bop_bond_derivatives.argtypes = [C.POINTER(Model), C.c_int, P, P, P, P, C.c_long, P, P]
    lib.bop_forces_workspace_size.restype = C.c_size_t
    lib.bop_forces_workspace_size.argtypes = [C.POINTER(Plan), C.c_long, C.c_int]
    lib.bop_forces.argtypes = [C.POINTER(Plan), P, P, P, P, C.c_long, P, P, P, P, C.c_int, P, P, P, C.c_size_t, P]
    lib.bop_scf_target.argtypes = [C.c_int, C.c_int, P, P, P, P]
    lib.bop_moments_batched.argtypes = [C.POINTER(Plan), C.c_int, P, P, P, P, P, P, P, P, P, P, P, P, C.c_size_t, P]
    _lib = lib
    return lib


def _check(rc):
    if rc != BOP_OK:
        buf = C.create_string_buffer(512)
        _lib.bop_last_error(buf, 512)
        raise BopError(rc, buf.value.decode())


def _torch():
    import torch
    return torch


def _dev(t, dtype=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    if t is None:
        return None
    p = t.data_ptr()
    if p == 0 and t.numel() == 0:
        # torch reports NULL for empty views; keep the storage's address so an
        # empty array still passes as a valid pointer
        p = t.untyped_storage().data_ptr()
    return C.c_void_p(p) if p else None


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _bytes(n, device):
    torch = _torch()
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------
def model_struct(model: dict) -> Model:
    """Fill the ABI's model struct from a plain model dict (onsite levels,
    bond-integral tables per ordered species pair and channel)."""
    m = Model()
    ns = model["n_species"]
    if ns > MAX_SPECIES:
        raise ValueError(f"at most {MAX_SPECIES} species")
    m.n_species = ns
    m.n_orb = model["n_orb"]
    m.r_cut = model["r_cut"]
    m.d_cut = model.get("d_cut", 0.0)
    for s in range(ns):
        for l in range(3):
            m.onsite[s][l] = model["onsite"][s][l]
    for pr in range(MAX_SPECIES * MAX_SPECIES):
        for c in range(N_CHANNELS):
            m.r0[pr][c] = 1.0
    for (si, sj), chans in model["bonds"].items():
        pr = si * ns + sj
        for name, (f, b0, r0, q) in chans.items():
            c = CHANNELS.index(name)
            m.form[pr][c] = f
            m.beta0[pr][c] = b0
            m.r0[pr][c] = r0
            m.q[pr][c] = q
    return m


@dataclass
class Neighbours:
    row_ptr: object
    nbr_j: object
    nbr_shift: object
    nbr_d: object
    order: object
    n_pairs: int


def build_neighbours(pos, cell, r_cut, capacity=None) -> Neighbours:
    """Periodic neighbour list on the GPU (``bop_build_neighbours``).
    ``pos`` [N,3] float64 device tensor, ``cell`` 3x3 (host, rows = a1..a3)."""
    torch = _torch()
    lib = load()
    _dev(pos, torch.float64, "pos")
    n = pos.shape[0]
    dev = pos.device
    cell_np = np.ascontiguousarray(cell, dtype=np.float64).reshape(3, 3)
    cptr = cell_np.ctypes.data_as(C.c_void_p)
    wsb = lib.bop_neighbours_workspace_size(n, cptr, float(r_cut))
    if wsb == 0:
        raise ValueError("invalid cell or cutoff")
    ws = _bytes(wsb, dev)
    if capacity is None:
        vol = abs(np.linalg.det(cell_np))
        dens = n / vol if vol > 0 else 0.0
        capacity = int(n * (4.0 / 3.0 * np.pi * r_cut ** 3 * dens * 1.5 + 16))
    row_ptr = torch.empty(n + 1, dtype=torch.int32, device=dev)
    order = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    for _ in range(2):
        nbr_j = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        nbr_shift = torch.empty((max(capacity, 1), 3), dtype=torch.int32, device=dev)
        nbr_d = torch.empty((max(capacity, 1), 3), dtype=torch.float64, device=dev)
        npairs = C.c_long(0)
        rc = lib.bop_build_neighbours(n, _ptr(pos), cptr, float(r_cut), capacity, _ptr(row_ptr), _ptr(nbr_j),
                                      _ptr(nbr_shift), _ptr(nbr_d), _ptr(order), C.byref(npairs), _ptr(ws),
                                      wsb, _stream())
        if rc == BOP_E_CAPACITY and npairs.value > capacity:
            capacity = int(npairs.value)
            continue
        _check(rc)
        P_ = int(npairs.value)
        return Neighbours(row_ptr, nbr_j[:P_], nbr_shift[:P_], nbr_d[:P_], order[:n], P_)
    raise RuntimeError("neighbour capacity retry failed")


D_PACKED = 16   # values per packed d-d block (BOP_D_PACKED)


def build_H(model: dict, species, nl: Neighbours, shift=None, dtype="f64", H_on=None, H_bond=None):
    """Onsite levels [N, n_orb] (float64) and bond blocks in ``dtype``
    (``bop_build_H``): [P, 16] packed symmetric d-d blocks for n_orb = 5 in
    FP64/FP32, else [P, n_orb, ld]."""
    torch = _torch()
    lib = load()
    _dev(species, torch.int32, "species")
    n = species.shape[0]
    no = model["n_orb"]
    dev = species.device
    # f16 (FP16 storage of the Lanczos vectors) uses FP32 blocks
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float32}[dtype]
    if H_on is None:
        H_on = torch.empty((n, no), dtype=torch.float64, device=dev)
    if H_bond is None and nl is not None:
        ld = (8 if no <= 8 else 16) if dtype == "bf16" else no
        shape = (D_PACKED,) if (no == 5 and dtype != "bf16") else (no, ld)
        # at least one row, so the pointer is valid when there are no pairs
        H_bond = torch.empty((max(nl.n_pairs, 1),) + shape, dtype=tdt, device=dev)[: nl.n_pairs]
    m = model_struct(model)
    if shift is not None:
        _dev(shift, torch.float64, "shift")
    _check(lib.bop_build_H(C.byref(m), n, _ptr(species), _ptr(shift),
                           _ptr(nl.row_ptr) if nl else None, _ptr(nl.nbr_j) if nl else None,
                           _ptr(nl.nbr_d) if nl else None, nl.n_pairs if nl else 0, DTYPES[dtype],
                           _ptr(H_on), _ptr(H_bond), _stream()))
    return H_on, H_bond


def moments_plan(n_atoms, n_orb, n_max, dtype, nl: Neighbours, tuning=None, use_order=True, radius=None) -> Plan:
    """Breadth-first sizing of the moment tiles (``bop_moments_plan``);
    ``radius`` a ``PathRadius`` (maximum path radius) or None."""
    torch = _torch()
    lib = load()
    dev = nl.row_ptr.device
    sb = lib.bop_moments_plan_scratch_size(n_atoms)
    scratch = _bytes(sb, dev)
    plan = Plan()
    t = None
    if tuning:
        t = Tuning(int(tuning.get("tile_atoms", 0)), int(tuning.get("block_threads", 0)),
                   int(tuning.get("batch_tiles", 0)), int(tuning.get("chunk_rows", 0)),
                   int(tuning.get("plan_search", 0)))
    _check(lib.bop_moments_plan(n_atoms, n_orb, n_max, DTYPES[dtype], _ptr(nl.row_ptr), _ptr(nl.nbr_j),
                                _ptr(nl.order) if use_order else None, C.byref(t) if t else None,
                                C.byref(radius) if radius else None, _ptr(scratch), sb, C.byref(plan), _stream()))
    del scratch
    return plan


def moments_prepare(plan: Plan, nl: Neighbours, ws=None, use_order=True, radius=None):
    """Store every tile's support in the moment workspace
    (``bop_moments_prepare``); returns the workspace tensor."""
    lib = load()
    if ws is None:
        ws = _bytes(plan.ws_bytes, nl.row_ptr.device)
    _check(lib.bop_moments_prepare(C.byref(plan), _ptr(nl.row_ptr), _ptr(nl.nbr_j),
                                   _ptr(nl.order) if use_order else None, C.byref(radius) if radius else None,
                                   _ptr(ws), ws.numel(), _stream()))
    return ws


def moments(plan: Plan, nl: Neighbours, H_on, H_bond, mu=None, ws=None, use_order=True):
    """Orbital moments mu [N, n_orb, n_max+1] float64 (``bop_moments``).
    Without ``ws`` the supports are prepared first."""
    torch = _torch()
    lib = load()
    dev = H_on.device
    if mu is None:
        mu = torch.empty((plan.n_atoms, plan.n_orb, plan.n_max + 1), dtype=torch.float64, device=dev)
    if ws is None:
        ws = moments_prepare(plan, nl, use_order=use_order)
    _check(lib.bop_moments(C.byref(plan), _ptr(nl.row_ptr), _ptr(H_on), _ptr(H_bond), _ptr(mu),
                           _ptr(ws), ws.numel(), _stream()))
    return mu


def lanczos(plan: Plan, nl: Neighbours, H_on, H_bond, out=None, ws=None, use_order=True):
    """Recursion coefficients a [R, n_a], b [R, n_b+1] and flags [R] straight
    from the H.X products (``bop_lanczos``); R = N * n_orb."""
    torch = _torch()
    lib = load()
    dev = H_on.device
    R = plan.n_atoms * plan.n_orb
    o = out or {}
    a = o.get("a", torch.empty((R, n_a(plan.n_max)), dtype=torch.float64, device=dev))
    b = o.get("b", torch.empty((R, n_b(plan.n_max) + 1), dtype=torch.float64, device=dev))
    fl = o.get("flags", torch.empty(R, dtype=torch.int32, device=dev))
    if ws is None:
        ws = moments_prepare(plan, nl, use_order=use_order)
    _check(lib.bop_lanczos(C.byref(plan), _ptr(nl.row_ptr), _ptr(H_on), _ptr(H_bond), _ptr(a), _ptr(b), _ptr(fl),
                           _ptr(ws), ws.numel(), _stream()))
    return {"a": a, "b": b, "flags": fl}


BW_MODES = {"gershgorin": 0, "global": 1, "lowest": 2, "highest": 3, "average": 4, "average_highest": 5,
            "minmax": 6, "weighted": 7}


def _bw_args(global_ab, bw, beta):
    if global_ab is not None:
        return 1, float(global_ab[0]), float(global_ab[1])
    return BW_MODES[bw], (float(beta) if bw == "weighted" else 0.0), 0.0


def terminator(rec, n_max, global_ab=None, bw="gershgorin", beta=1.0):
    """a_inf, b_inf (and terminator flags) for coefficients from ``lanczos``
    (``bop_recursion`` with mu = NULL); updates and returns ``rec``."""
    torch = _torch()
    R = rec["a"].shape[0] if n_a(n_max) else rec["b"].shape[0]
    dev = rec["b"].device
    for k in ("a_inf", "b_inf"):
        if k not in rec:
            rec[k] = torch.empty(R, dtype=torch.float64, device=dev)
    mode, ag, bg = _bw_args(global_ab, bw, beta)
    _check(load().bop_recursion(R, n_max, None, mode, ag, bg, _ptr(rec["a"]), _ptr(rec["b"]), _ptr(rec["a_inf"]),
                                _ptr(rec["b_inf"]), _ptr(rec["flags"]), _stream()))
    return rec


def n_a(n_max):
    return (n_max - 1) // 2 + 1 if n_max >= 1 else 0


def n_b(n_max):
    return n_max // 2


def recursion(mu_rows, n_max, global_ab=None, out=None, bw="gershgorin", beta=1.0):
    """Recursion coefficients a [R, n_a], b [R, n_b+1], a_inf, b_inf, flags
    (``bop_recursion``); ``bw`` selects the band centre/width estimate."""
    torch = _torch()
    lib = load()
    mu_rows = _dev(mu_rows.reshape(-1, n_max + 1), torch.float64, "mu")
    R = mu_rows.shape[0]
    dev = mu_rows.device
    o = out or {}
    a = o.get("a", torch.empty((R, n_a(n_max)), dtype=torch.float64, device=dev))
    b = o.get("b", torch.empty((R, n_b(n_max) + 1), dtype=torch.float64, device=dev))
    ai = o.get("a_inf", torch.empty(R, dtype=torch.float64, device=dev))
    bi = o.get("b_inf", torch.empty(R, dtype=torch.float64, device=dev))
    fl = o.get("flags", torch.empty(R, dtype=torch.int32, device=dev))
    mode, ag, bg = _bw_args(global_ab, bw, beta)
    _check(lib.bop_recursion(R, n_max, _ptr(mu_rows), mode, ag, bg, _ptr(a), _ptr(b), _ptr(ai), _ptr(bi),
                             _ptr(fl), _stream()))
    return {"a": a, "b": b, "a_inf": ai, "b_inf": bi, "flags": fl}


def energy(mu, rec, H_on, n_elec, n_max, n_exp=200, E_F=None, ws=None):
    """Fermi level (bisection, unless ``E_F`` is given as a float or a
    1-element device tensor), per-atom N, U, n(E_F) and U_total
    (``bop_energy``)."""
    torch = _torch()
    lib = load()
    n, no = H_on.shape
    dev = H_on.device
    if ws is None:
        ws = _bytes(lib.bop_energy_workspace_size(n, no, n_exp), dev)
    ef_mode = 0
    if E_F is None:
        ef = torch.zeros(1, dtype=torch.float64, device=dev)
    else:
        ef_mode = 1
        ef = E_F if isinstance(E_F, torch.Tensor) else torch.tensor([float(E_F)], dtype=torch.float64, device=dev)
    out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("N_atom", "U_atom", "dos_atom")}
    ut = torch.zeros(1, dtype=torch.float64, device=dev)
    _check(lib.bop_energy(n, no, n_max, n_exp, _ptr(mu), _ptr(rec["a"]), _ptr(rec["b"]), _ptr(rec["a_inf"]),
                          _ptr(rec["b_inf"]), _ptr(H_on), float(n_elec), ef_mode, _ptr(ef), _ptr(out["N_atom"]),
                          _ptr(out["U_atom"]), _ptr(out["dos_atom"]), _ptr(ut), _ptr(rec["flags"]), _ptr(ws),
                          ws.numel(), _stream()))
    out["E_F"] = ef
    out["U_total"] = ut
    return out


def energy_atom_averaged(mu, H_on, n_elec, n_max, n_exp=200, bw="gershgorin", beta=1.0, E_F=None, ws=None):
    """The atom-averaged mode: one chain per atom from the orbital-averaged
    moments (``bop_atom_average``, ``bop_recursion``,
    ``bop_energy_atom_averaged``).  Returns the energy outputs plus the
    averaged moments and chain coefficients."""
    torch = _torch()
    lib = load()
    n, no = H_on.shape
    dev = H_on.device
    mu_avg = torch.empty((n, n_max + 1), dtype=torch.float64, device=dev)
    H_avg = torch.empty(n, dtype=torch.float64, device=dev)
    _check(lib.bop_atom_average(n, no, n_max, _ptr(mu), _ptr(H_on), _ptr(mu_avg), _ptr(H_avg), _stream()))
    rec = recursion(mu_avg, n_max, bw=bw, beta=beta)
    if ws is None:
        ws = _bytes(lib.bop_energy_workspace_size(n, 1, n_exp), dev)
    ef_mode = 0
    if E_F is None:
        ef = torch.zeros(1, dtype=torch.float64, device=dev)
    else:
        ef_mode = 1
        ef = E_F if isinstance(E_F, torch.Tensor) else torch.tensor([float(E_F)], dtype=torch.float64, device=dev)
    out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("N_atom", "U_atom", "dos_atom")}
    ut = torch.zeros(1, dtype=torch.float64, device=dev)
    _check(lib.bop_energy_atom_averaged(n, no, n_max, n_exp, _ptr(mu_avg), _ptr(rec["a"]), _ptr(rec["b"]),
                                        _ptr(rec["a_inf"]), _ptr(rec["b_inf"]), _ptr(H_avg), float(n_elec), ef_mode,
                                        _ptr(ef), _ptr(out["N_atom"]), _ptr(out["U_atom"]), _ptr(out["dos_atom"]),
                                        _ptr(ut), _ptr(rec["flags"]), _ptr(ws), ws.numel(), _stream()))
    out.update({"E_F": ef, "U_total": ut, "mu_avg": mu_avg, "H_avg": H_avg, "rec": rec})
    return out


def energy_noalloc(mu, rec, H_on, n_elec, n_max, n_exp=200, E_F=None, out=None):
    """``energy`` through ``bop_energy_noalloc``: the library's fixed scratch
    array instead of a workspace.  Output tensors may be passed in ``out``
    (keys N_atom, U_atom, dos_atom, E_F, U_total) so that the call allocates
    nothing."""
    torch = _torch()
    lib = load()
    n, no = H_on.shape
    dev = H_on.device
    o = dict(out or {})
    for k in ("N_atom", "U_atom", "dos_atom"):
        if k not in o:
            o[k] = torch.empty(n, dtype=torch.float64, device=dev)
    if "U_total" not in o:
        o["U_total"] = torch.zeros(1, dtype=torch.float64, device=dev)
    ef_mode = 0
    if E_F is not None:
        ef_mode = 1
        o["E_F"] = E_F if isinstance(E_F, torch.Tensor) else torch.tensor([float(E_F)], dtype=torch.float64,
                                                                          device=dev)
    elif "E_F" not in o:
        o["E_F"] = torch.zeros(1, dtype=torch.float64, device=dev)
    _check(lib.bop_energy_noalloc(n, no, n_max, n_exp, _ptr(mu), _ptr(rec["a"]), _ptr(rec["b"]), _ptr(rec["a_inf"]),
                                  _ptr(rec["b_inf"]), _ptr(H_on), float(n_elec), ef_mode, _ptr(o["E_F"]),
                                  _ptr(o["N_atom"]), _ptr(o["U_atom"]), _ptr(o["dos_atom"]), _ptr(o["U_total"]),
                                  _ptr(rec["flags"]), _stream()))
    return o


def weights(mu, H_on, E_F, n_max, n_exp=200, out=None, ws=None):
    """w [R, n_max+1] = dU_bond/dmu (both spins) at the self-determined Fermi
    level ``E_F`` (1-element device tensor), ``bop_weights``."""
    torch = _torch()
    lib = load()
    mu_rows = _dev(mu.reshape(-1, n_max + 1), torch.float64, "mu")
    R = mu_rows.shape[0]
    dev = mu_rows.device
    if out is None:
        out = torch.empty((R, n_max + 1), dtype=torch.float64, device=dev)
    if ws is None:
        ws = _bytes(lib.bop_weights_workspace_size(R, n_max), dev)
    _check(lib.bop_weights(R, n_max, n_exp, _ptr(mu_rows), _ptr(H_on), _ptr(E_F), _ptr(out), _ptr(ws), ws.numel(),
                           _stream()))
    return out


def bond_derivatives(model: dict, species, nl: Neighbours, out=None):
    """dH [P, 3, 16]: derivatives of the packed d-d blocks with respect to the
    bond vector (``bop_bond_derivatives``)."""
    torch = _torch()
    lib = load()
    dev = species.device
    if out is None:
        out = torch.empty((max(nl.n_pairs, 1), 3, D_PACKED), dtype=torch.float64, device=dev)[: nl.n_pairs]
    m = model_struct(model)
    _check(lib.bop_bond_derivatives(C.byref(m), species.shape[0], _ptr(species), _ptr(nl.row_ptr), _ptr(nl.nbr_j),
                                    _ptr(nl.nbr_d), nl.n_pairs, _ptr(out), _stream()))
    return out


def forces_workspace(plan: Plan, nl: Neighbours, batch_tiles=0):
    """Device workspace for ``forces`` with this plan and batch."""
    lib = load()
    return _bytes(lib.bop_forces_workspace_size(C.byref(plan), nl.n_pairs, int(batch_tiles)), nl.row_ptr.device)


def forces(plan: Plan, mws, nl: Neighbours, H_on, H_bond, dH, w, batch_tiles=0, F=None, ws=None, theta_on=None):
    """F [N, 3] = -dU_bond/dr (``bop_forces``) from the moment plan and its
    prepared workspace ``mws``, the blocks in the plan's dtype, their
    derivatives and the weights.  With ``theta_on`` (an [N, n_orb] FP64
    device tensor) the onsite elements Theta~_(ia,ia) are written too."""
    torch = _torch()
    lib = load()
    dev = H_on.device
    if F is None:
        F = torch.empty((plan.n_atoms, 3), dtype=torch.float64, device=dev)
    if ws is None:
        ws = forces_workspace(plan, nl, batch_tiles)
    _check(lib.bop_forces(C.byref(plan), _ptr(mws), _ptr(nl.row_ptr), _ptr(nl.nbr_j), _ptr(nl.nbr_shift), nl.n_pairs,
                          _ptr(H_on), _ptr(H_bond), _ptr(dH), _ptr(w), int(batch_tiles), _ptr(F), _ptr(theta_on),
                          _ptr(ws), ws.numel(), _stream()))
    return F


def scf_target(theta_on, N_atom, delta=None):
    """Delta_i = sum_a Theta~_(ia,ia) - N_i = dU/d(shift_i) (``bop_scf_target``)."""
    torch = _torch()
    n, no = theta_on.shape
    if delta is None:
        delta = torch.empty(n, dtype=torch.float64, device=theta_on.device)
    _check(load().bop_scf_target(n, no, _ptr(theta_on), _ptr(N_atom), _ptr(delta), _stream()))
    return delta


class EnergyPath:
    """Neighbours -> H -> moments -> recursion -> energy for one structure,
    with every buffer allocated once (device tensors) and reused."""

    def __init__(self, pos, cell, species, model: dict, n_max: int, n_exp: int = 200, dtype: str = "f64",
                 tuning=None, device="cuda", method: str = "moments", bw: str = "gershgorin", beta: float = 1.0,
                 r_max: float = 0.0):
        torch = _torch()
        load()
        self.r_max = float(r_max)
        if bw not in BW_MODES or bw == "global":
            raise ValueError(f"bw must be one of {sorted(k for k in BW_MODES if k != 'global')}")
        self.bw, self.beta = bw, float(beta)
        if method not in ("moments", "lanczos"):
            raise ValueError("method must be 'moments' or 'lanczos'")
        self.method = method
        self.device = torch.device(device)
        self.model = model
        self.n_max, self.n_exp, self.dtype = int(n_max), int(n_exp), dtype
        self.pos = torch.as_tensor(np.ascontiguousarray(pos, np.float64), device=self.device)
        self.cell = np.ascontiguousarray(cell, np.float64)
        self.species = torch.as_tensor(np.ascontiguousarray(species, np.int32), device=self.device)
        self.n = self.pos.shape[0]
        self.no = model["n_orb"]
        self.tuning = tuning
        self.nl = build_neighbours(self.pos, self.cell, model["r_cut"])
        self.H_on, self.H_bond = build_H(model, self.species, self.nl, dtype=dtype)
        self.radius = path_radius(self.r_max, model["r_cut"], self.cell, self.pos)
        self.plan = moments_plan(self.n, self.no, self.n_max, dtype, self.nl, tuning, radius=self.radius)
        self.mws = moments_prepare(self.plan, self.nl, radius=self.radius)
        self.mu = torch.empty((self.n, self.no, self.n_max + 1), dtype=torch.float64, device=self.device)
        R = self.n * self.no
        self.rec = {"a": torch.empty((R, n_a(self.n_max)), dtype=torch.float64, device=self.device),
                    "b": torch.empty((R, n_b(self.n_max) + 1), dtype=torch.float64, device=self.device),
                    "a_inf": torch.empty(R, dtype=torch.float64, device=self.device),
                    "b_inf": torch.empty(R, dtype=torch.float64, device=self.device),
                    "flags": torch.empty(R, dtype=torch.int32, device=self.device)}
        self.ews = _bytes(load().bop_energy_workspace_size(self.n, self.no, self.n_exp), self.device)

    def rebuild(self, shift=None):
        """Neighbour list, H and the moment plan again, reusing buffers."""
        self.nl = build_neighbours(self.pos, self.cell, self.model["r_cut"], capacity=self.nl.n_pairs)
        if self.H_bond.shape[0] != self.nl.n_pairs:
            self.H_bond = None
        self.H_on, self.H_bond = build_H(self.model, self.species, self.nl, shift=shift, dtype=self.dtype,
                                         H_on=self.H_on, H_bond=self.H_bond)
        self.plan = moments_plan(self.n, self.no, self.n_max, self.dtype, self.nl, self.tuning, radius=self.radius)
        if self.plan.ws_bytes > self.mws.numel():
            self.mws = None
        self.mws = moments_prepare(self.plan, self.nl, ws=self.mws, radius=self.radius)

    def step(self, n_elec, E_F=None):
        """The whole path for the structure: neighbours, H, plan, moments,
        recursion, expansion, Fermi level, energies."""
        self.rebuild()
        return self.run(n_elec, E_F)

    def run_moments(self):
        """The H.X passes: moments, or with method 'lanczos' the recursion
        coefficients."""
        if self.method == "lanczos":
            return lanczos(self.plan, self.nl, self.H_on, self.H_bond, out=self.rec, ws=self.mws)
        return moments(self.plan, self.nl, self.H_on, self.H_bond, mu=self.mu, ws=self.mws)

    def run_tail(self, n_elec, E_F=None):
        if self.method == "lanczos":
            terminator(self.rec, self.n_max, bw=self.bw, beta=self.beta)
            return energy(None, self.rec, self.H_on, n_elec, self.n_max, self.n_exp, E_F=E_F, ws=self.ews)
        recursion(self.mu, self.n_max, out=self.rec, bw=self.bw, beta=self.beta)
        return energy(self.mu, self.rec, self.H_on, n_elec, self.n_max, self.n_exp, E_F=E_F, ws=self.ews)

    def run(self, n_elec, E_F=None):
        self.run_moments()
        return self.run_tail(n_elec, E_F)

    def forces(self, n_elec, batch_tiles=0, scf_target=False):
        """Energy and forces of the current structure: the moment form of the
        path (FP64 or FP32 vectors as the path's dtype), then the weights at
        its Fermi level, the block derivatives and F = -dU_bond/dr [N, 3].
        With ``scf_target`` also the onsite Theta~ [N, n_orb] and the
        per-atom target of Eq. BOP_SCF (out["theta_on"], out["delta"])."""
        if self.method != "moments":
            raise ValueError("forces need the moment form")
        out = self.run(n_elec)
        self.w = weights(self.mu, self.H_on, out["E_F"], self.n_max, self.n_exp)
        self.dH = bond_derivatives(self.model, self.species, self.nl)
        th = None
        if scf_target:
            th = _torch().empty((self.n, self.no), dtype=_torch().float64, device=self.device)
        out["F"] = forces(self.plan, self.mws, self.nl, self.H_on, self.H_bond, self.dH, self.w,
                          batch_tiles=batch_tiles, theta_on=th)
        if scf_target:
            out["theta_on"] = th
            out["delta"] = globals()["scf_target"](th, out["N_atom"])
        return out


class SCFPath(EnergyPath):
    """Local-charge-neutrality self-consistency (``bop_scf_step``): one onsite
    shift per atom, updated on the device until max |N_i - n0_i| < tol."""

    def __init__(self, pos, cell, species, model, n_max, n0, n_exp=200, dtype="f64", tuning=None, device="cuda",
                 method="moments", mixer="linear", hist=20):
        super().__init__(pos, cell, species, model, n_max, n_exp, dtype, tuning, device, method)
        torch = _torch()
        if mixer not in ("linear", "broyden"):
            raise ValueError("mixer must be 'linear' or 'broyden'")
        self.mixer, self.hist, self.iter = mixer, int(hist), 0
        self.bws = _bytes(load().bop_broyden_workspace_size(self.n, self.hist), self.device) \
            if mixer == "broyden" else None
        self.n0 = torch.as_tensor(np.ascontiguousarray(n0, np.float64), device=self.device)
        self.n_elec = float(np.sum(n0))
        self.shift = torch.zeros(self.n, dtype=torch.float64, device=self.device)
        self.q = torch.zeros(self.n, dtype=torch.float64, device=self.device)
        self.max_dq = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.converged = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.out = {k: torch.zeros(self.n, dtype=torch.float64, device=self.device)
                    for k in ("N_atom", "U_atom", "dos_atom")}
        self.out["E_F"] = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.out["U_total"] = torch.zeros(1, dtype=torch.float64, device=self.device)
        s = System()
        s.model = model_struct(model)
        s.n_atoms, s.n_max, s.n_exp, s.dtype = self.n, self.n_max, self.n_exp, DTYPES[dtype]
        s.method = 1 if method == "lanczos" else 0
        s.species, s.n0 = _ptr(self.species), _ptr(self.n0)
        s.mu = _ptr(self.mu)
        for k in ("a", "b", "a_inf", "b_inf", "flags"):
            setattr(s, k, _ptr(self.rec[k]))
        s.energy_ws, s.energy_ws_bytes = _ptr(self.ews), self.ews.numel()
        s.n_elec = self.n_elec
        for k in ("E_F", "N_atom", "U_atom", "dos_atom", "U_total"):
            setattr(s, k, _ptr(self.out[k]))
        self.sys = s
        self._point_at_structure()

    def _point_at_structure(self):
        """The system's neighbour list, H and moment plan (after a rebuild)."""
        s = self.sys
        s.row_ptr, s.nbr_j, s.order = _ptr(self.nl.row_ptr), _ptr(self.nl.nbr_j), _ptr(self.nl.order)
        s.n_pairs = self.nl.n_pairs
        s.H_on, s.H_bond = _ptr(self.H_on), _ptr(self.H_bond)
        s.plan = self.plan
        s.moments_ws, s.moments_ws_bytes = _ptr(self.mws), self.mws.numel()

    def set_positions(self, pos):
        """Move the atoms (an MD or relaxation step): neighbour list, bonds and
        moment plan are rebuilt; the shifts stay, so the next cycle starts from
        the previous step's converged onsite levels (Sec. III "Speed-ups" (ii))."""
        torch = _torch()
        self.pos.copy_(torch.as_tensor(np.ascontiguousarray(pos, np.float64), device=self.device))
        self.rebuild()
        self._point_at_structure()

    def set_shift(self, shift):
        """Start a new cycle from ``shift`` (the Broyden history starts again)."""
        self.shift.copy_(_torch().as_tensor(shift, dtype=_torch().float64, device=self.device))
        self.iter = 0

    def step(self, mix=0.5, n_floor=1e-3, tol=1e-4):
        if self.mixer == "broyden":
            _check(load().bop_scf_step_broyden(C.byref(self.sys), float(mix), float(n_floor), float(tol), self.iter,
                                               self.hist, _ptr(self.shift), _ptr(self.q), _ptr(self.max_dq),
                                               _ptr(self.converged), _ptr(self.bws), self.bws.numel(), _stream()))
        else:
            _check(load().bop_scf_step(C.byref(self.sys), float(mix), float(n_floor), float(tol), _ptr(self.shift),
                                       _ptr(self.q), _ptr(self.max_dq), _ptr(self.converged), _stream()))
        self.iter += 1

    def run_scf(self, mix=0.5, n_floor=1e-3, tol=1e-4, max_iter=200):
        """Iterate from the current shifts until converged (a new cycle: the
        Broyden history starts again); returns (iterations, history of max|q|)."""
        self.iter = 0
        hist = []
        for it in range(max_iter):
            self.step(mix, n_floor, tol)
            mq = float(self.max_dq.item())
            hist.append(mq)
            if int(self.converged.item()):
                return it + 1, hist
        raise BopError(BOP_E_NOT_CONVERGED, f"SCF not converged in {max_iter} iterations (max|q| {hist[-1]:.3e})")


class MagneticPath:
    """Collinear-magnetic energy path and Stoner / charge-neutrality cycle
    (``bop_mag_energy``, ``bop_mag_scf_step``): both spin channels share the
    neighbour list, bonds and moment plan; every per-row and per-atom buffer
    holds the up channel's atoms followed by the down channel's."""

    def __init__(self, pos, cell, species, model, n_max, n0, stoner, B_z=0.0, n_exp=200, dtype="f64",
                 method="moments", tuning=None, device="cuda"):
        torch = _torch()
        lib = load()
        if method not in ("moments", "lanczos"):
            raise ValueError("method must be 'moments' or 'lanczos'")
        self.device = torch.device(device)
        self.model, self.n_max, self.n_exp, self.dtype, self.method = model, int(n_max), int(n_exp), dtype, method
        self.pos = torch.as_tensor(np.ascontiguousarray(pos, np.float64), device=self.device)
        self.cell = np.ascontiguousarray(cell, np.float64)
        self.species = torch.as_tensor(np.ascontiguousarray(species, np.int32), device=self.device)
        n = self.n = self.pos.shape[0]
        no = self.no = model["n_orb"]
        self.mag = Magnetism()
        st = list(stoner) if np.ndim(stoner) else [float(stoner)] * model["n_species"]
        for k, v in enumerate(st):
            self.mag.stoner[k] = float(v)
        self.mag.B_z = float(B_z)
        self.nl = build_neighbours(self.pos, self.cell, model["r_cut"])
        self.H_on1, self.H_bond = build_H(model, self.species, self.nl, dtype=dtype)
        self.plan = moments_plan(n, no, self.n_max, dtype, self.nl, tuning)
        self.mws = moments_prepare(self.plan, self.nl)
        f64 = dict(dtype=torch.float64, device=self.device)
        R2 = 2 * n * no
        self.H_on = torch.empty((2 * n, no), **f64)
        self.mu = torch.empty((2 * n, no, self.n_max + 1), **f64)
        self.rec = {"a": torch.empty((R2, n_a(self.n_max)), **f64), "b": torch.empty((R2, n_b(self.n_max) + 1), **f64),
                    "a_inf": torch.empty(R2, **f64), "b_inf": torch.empty(R2, **f64),
                    "flags": torch.empty(R2, dtype=torch.int32, device=self.device)}
        self.ews = _bytes(lib.bop_energy_workspace_size(2 * n, no, self.n_exp), self.device)
        self.out = {k: torch.zeros(2 * n, **f64) for k in ("N_atom", "U_atom", "dos_atom")}
        self.out["E_F"] = torch.zeros(1, **f64)
        self.out["U_total"] = torch.zeros(1, **f64)
        self.n0 = torch.as_tensor(np.ascontiguousarray(n0, np.float64) * np.ones(n), device=self.device)
        self.shift = torch.zeros(n, **f64)
        self.moment = torch.zeros(n, **f64)
        self.m_out = torch.zeros(n, **f64)
        self.q = torch.zeros(n, **f64)
        self.U_X = torch.zeros(1, **f64)
        self.max_d = torch.zeros(2, **f64)
        self.converged = torch.zeros(1, dtype=torch.int32, device=self.device)
        sy = System()
        sy.model = model_struct(model)
        sy.n_atoms, sy.n_max, sy.n_exp, sy.dtype = n, self.n_max, self.n_exp, DTYPES[dtype]
        sy.method = 1 if method == "lanczos" else 0
        sy.species, sy.n0 = _ptr(self.species), _ptr(self.n0)
        sy.row_ptr, sy.nbr_j, sy.order = _ptr(self.nl.row_ptr), _ptr(self.nl.nbr_j), _ptr(self.nl.order)
        sy.n_pairs = self.nl.n_pairs
        sy.H_on, sy.H_bond = _ptr(self.H_on), _ptr(self.H_bond)
        sy.plan = self.plan
        sy.moments_ws, sy.moments_ws_bytes = _ptr(self.mws), self.mws.numel()
        sy.mu = _ptr(self.mu)
        for k in ("a", "b", "a_inf", "b_inf", "flags"):
            setattr(sy, k, _ptr(self.rec[k]))
        sy.energy_ws, sy.energy_ws_bytes = _ptr(self.ews), self.ews.numel()
        sy.n_elec = float(self.n0.sum().item())
        for k in ("E_F", "N_atom", "U_atom", "dos_atom", "U_total"):
            setattr(sy, k, _ptr(self.out[k]))
        self.sys = sy

    def set_state(self, shift=None, moment=None):
        torch = _torch()
        if shift is not None:
            self.shift.copy_(torch.as_tensor(shift, dtype=torch.float64, device=self.device))
        if moment is not None:
            self.moment.copy_(torch.as_tensor(moment, dtype=torch.float64, device=self.device))

    def energy(self):
        """Both channels at the current shifts and moments (``bop_mag_energy``);
        returns the output dict (per-channel rows in N_atom, U_atom, dos_atom)."""
        _check(load().bop_mag_energy(C.byref(self.sys), C.byref(self.mag), _ptr(self.shift), _ptr(self.moment),
                                     _ptr(self.m_out), _ptr(self.U_X), _stream()))
        return self.out

    def step(self, mix=0.5, mix_m=0.5, n_floor=1e-3, tol=1e-4, tol_m=1e-4):
        _check(load().bop_mag_scf_step(C.byref(self.sys), C.byref(self.mag), float(mix), float(mix_m),
                                       float(n_floor), float(tol), float(tol_m), _ptr(self.shift),
                                       _ptr(self.moment), _ptr(self.m_out), _ptr(self.q), _ptr(self.U_X),
                                       _ptr(self.max_d), _ptr(self.converged), _stream()))

    def run_scf(self, mix=0.5, mix_m=0.5, n_floor=1e-3, tol=1e-4, tol_m=1e-4, max_iter=300):
        """Iterate until converged; returns (iterations, history of (max|q|, max|dm|))."""
        hist = []
        for it in range(max_iter):
            self.step(mix, mix_m, n_floor, tol, tol_m)
            hist.append(tuple(self.max_d.cpu().numpy().tolist()))
            if int(self.converged.item()):
                return it + 1, hist
        raise BopError(BOP_E_NOT_CONVERGED, f"magnetic SCF not converged in {max_iter} iterations ({hist[-1]})")


MLP_NPARAM = 4673
MLP_SHAPES = ((64, 6), (64,), (64, 64), (64,), (1, 64), (1,))


def features(mu, n_orb, n_max, mean=None, std=None):
    """Standardised per-atom moment traces mu_1..mu_6 (``bop_features``)."""
    torch = _torch()
    n = mu.shape[0]
    x = torch.empty((n, 6), dtype=torch.float32, device=mu.device)
    _check(load().bop_features(n, n_orb, n_max, _ptr(mu), _ptr(mean), _ptr(std), _ptr(x), _stream()))
    return x


def mlp_forward(params, x):
    torch = _torch()
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    _check(load().bop_mlp_forward(x.shape[0], _ptr(params), _ptr(x), _ptr(y), _stream()))
    return y


def feature_stats(x):
    """Column mean and std (n - 1) of the features x [n, 6] (``bop_feature_stats``)."""
    torch = _torch()
    mean = torch.empty(6, dtype=torch.float32, device=x.device)
    std = torch.empty(6, dtype=torch.float32, device=x.device)
    _check(load().bop_feature_stats(x.shape[0], _ptr(_dev(x, torch.float32, "x")), _ptr(mean), _ptr(std),
                                    _stream()))
    return mean, std


def standardise(x, mean, std, out=None):
    """(x - mean) / std per feature column (``bop_standardise``)."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(x)
    _check(load().bop_standardise(x.shape[0], _ptr(_dev(x, torch.float32, "x")), _ptr(mean), _ptr(std), _ptr(out),
                                  _stream()))
    return out


def mlp_shift(params, x):
    """Gauge-fixed warm-start shifts (FP64, mean removed) for standardised
    features x (``bop_mlp_shift``)."""
    torch = _torch()
    y = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
    _check(load().bop_mlp_shift(x.shape[0], _ptr(params), _ptr(_dev(x, torch.float32, "x")), _ptr(y), _stream()))
    return y


def mlp_pack(arrays, device="cuda"):
    """Flatten (W1, b1, W2, b2, W3, b3) into the ABI's parameter array."""
    torch = _torch()
    flat = np.concatenate([np.asarray(a, np.float32).reshape(-1) for a in arrays])
    assert flat.size == MLP_NPARAM
    return torch.as_tensor(flat, device=device)


def mlp_unpack(params):
    flat = params.detach().cpu().numpy().astype(np.float64)
    out, o = [], 0
    for shp in MLP_SHAPES:
        k = int(np.prod(shp))
        out.append(flat[o:o + k].reshape(shp))
        o += k
    return out


class MLP:
    """The warm-start network with Adam state on the device; every training
    step runs ``bop_mlp_train_step``."""

    def __init__(self, seed=0, device="cuda"):
        torch = _torch()
        rng = np.random.default_rng(seed)
        arrs = []
        for shp in MLP_SHAPES:
            if len(shp) == 2:                       # Xavier uniform
                lim = np.sqrt(6.0 / (shp[0] + shp[1]))
                arrs.append(rng.uniform(-lim, lim, size=shp))
            else:
                arrs.append(np.zeros(shp))
        self.device = device
        self.params = mlp_pack(arrs, device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.mean = torch.zeros(6, dtype=torch.float32, device=device)
        self.std = torch.ones(6, dtype=torch.float32, device=device)
        self._ws = None
        self._wsb = 0

    def grad(self, x, t):
        """Loss and gradient at the current parameters, no update
        (``bop_mlp_backward``)."""
        torch = _torch()
        B = x.shape[0]
        ws = _bytes(load().bop_mlp_train_workspace_size(B), x.device)
        g = torch.empty_like(self.params)
        loss = torch.zeros(1, dtype=torch.float32, device=x.device)
        _check(load().bop_mlp_backward(B, None, _ptr(x), _ptr(t), _ptr(self.params), _ptr(loss), _ptr(g), _ptr(ws),
                                       ws.numel(), _stream()))
        return loss, g

    def adam(self, g, lr=1e-3):
        """One Adam update of the parameters from a gradient (``bop_mlp_adam``)."""
        self.t += 1
        _check(load().bop_mlp_adam(_ptr(g), _ptr(self.params), _ptr(self.m), _ptr(self.v), self.t, float(lr),
                                   _stream()))

    def train(self, x, t, epochs=50, batch=4096, lr=1e-3, seed=0, log_every=0):
        """Minibatch Adam over (x, t) device tensors; returns per-epoch mean loss."""
        torch = _torch()
        n = x.shape[0]
        B = min(batch, n)
        need = load().bop_mlp_train_workspace_size(B)
        if self._wsb < need:
            self._ws, self._wsb = _bytes(need, x.device), need
        rng = np.random.default_rng(seed)
        loss = torch.zeros(1, dtype=torch.float32, device=x.device)
        hist = []
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(n).astype(np.int32), device=x.device)
            tot, nb = 0.0, 0
            for s0 in range(0, n - B + 1, B):
                self.t += 1
                _check(load().bop_mlp_train_step(B, _ptr(perm[s0:s0 + B]), _ptr(x), _ptr(t), _ptr(self.params),
                                                 _ptr(self.m), _ptr(self.v), self.t, float(lr), _ptr(loss), None,
                                                 _ptr(self._ws), self._wsb, _stream()))
                tot += float(loss.item()) if (log_every and nb % log_every == 0) else 0.0
                nb += 1
            hist.append(tot)
        return hist

    def predict(self, x):
        return mlp_forward(self.params, x)

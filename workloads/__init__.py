"""Seeded synthetic inputs for analytic-BOP energy calculations.

This module only builds *inputs*: atom positions, periodic cells, species
labels and tight-binding parameter tables written as plain numbers.  It holds
none of the method's arithmetic (no neighbour search, no Hamiltonian, no
moments), so the CPU oracle and the HIP library can both be fed from it
without sharing any of the computation they are compared on.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.  Positions
are wrapped into the cell (fractional coordinates in [0, 1)).

Workloads (the paper publishes no dataset; these stand in for the model
systems it discusses, e.g. the canonical d-band model named among its
parametrisations and the bcc transition-metal example of its Appendix B):

* ``bcc_small``   : bcc 4x4x4 (128 atoms, a = 2.87 A), Gaussian displacements
                    sigma = 0.05 A, canonical d band, cutoff 3.5 A, 9 moments,
                    N_d = 6.5.
* ``bcc_large``   : bcc 40^3 (128,000 atoms, a = 3.16 A), sigma = 0.08 A,
                    canonical d band, cutoff 3.8 A (two shells), 18 moments,
                    N_d = 4.5.
* ``fcc_alloy_spd``: fcc 30^3 binary random alloy (108,000 atoms), 9-orbital
                    s,p,d blocks with exponential bond integrals, cutoff 4.2 A,
                    20 moments.
* ``bcc_alloy_scf``: bcc binary random alloy for local charge neutrality,
                    onsite levels 0 / +0.8 eV, N_d = 6.0 / 5.0, 16 moments.
* ``ragged_batch``: many periodic structures of uneven size (bcc, fcc, hcp,
                    random dense packing), cutoff 3.6 A, 14 moments.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

# Slater-Koster channel names, in a fixed order used by both sides' parameter
# tables.  The first orbital letter belongs to the atom the bond starts at,
# the second to the atom it points to; the last letter is the bond symmetry
# (s = sigma, p = pi, d = delta).
CHANNELS = ("sss", "sps", "pss", "sds", "dss", "pps", "ppp",
            "pds", "dps", "pdp", "dpp", "dds", "ddp", "ddd")
FORM_POWER = 0   # beta(r) = beta0 * (r0 / r) ** q
FORM_EXP = 1     # beta(r) = beta0 * exp(-q * (r - r0))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# lattices
# ----------------------------------------------------------------------------
_BASIS = {
    "sc": np.array([[0.0, 0.0, 0.0]]),
    "bcc": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]),
    "fcc": np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5],
                     [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]]),
}


def cubic_lattice(kind: str, a: float, reps) -> tuple[np.ndarray, np.ndarray]:
    """Conventional cubic cells of ``kind`` repeated ``reps`` = (n1, n2, n3).

    Atoms are ordered cell by cell (x slowest), basis atom fastest.
    Returns ``(pos [N,3], cell [3,3])`` with the rows of ``cell`` the lattice
    vectors a1, a2, a3."""
    n1, n2, n3 = (reps, reps, reps) if np.isscalar(reps) else reps
    basis = _BASIS[kind]
    g = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3),
                             indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    frac = (g[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    pos = frac * a
    cell = np.diag([n1 * a, n2 * a, n3 * a]).astype(np.float64)
    return pos, cell


def hcp_lattice(a: float, reps) -> tuple[np.ndarray, np.ndarray]:
    """Ideal hcp (c/a = sqrt(8/3)) in its orthorhombic 4-atom cell
    (a x a*sqrt(3) x c), repeated ``reps``."""
    n1, n2, n3 = reps
    c = a * math.sqrt(8.0 / 3.0)
    b = a * math.sqrt(3.0)
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0],
                      [0.5, 1.0 / 6.0, 0.5], [0.0, 2.0 / 3.0, 0.5]])
    g = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3),
                             indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    frac = (g[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    pos = frac * np.array([a, b, c])
    cell = np.diag([n1 * a, n2 * b, n3 * c]).astype(np.float64)
    return pos, cell


def wrap(pos: np.ndarray, cell: np.ndarray) -> np.ndarray:
    """Wrap positions into the cell: fractional coordinates in [0, 1)."""
    frac = pos @ np.linalg.inv(cell)
    frac -= np.floor(frac)
    frac[frac >= 1.0] = 0.0
    return frac @ cell


def displace(pos, cell, sigma, rng) -> np.ndarray:
    """i.i.d. Gaussian displacement N(0, sigma^2) per Cartesian component,
    then wrap into the cell."""
    if sigma > 0:
        pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    return wrap(pos, cell)


def random_species(n: int, counts, rng) -> np.ndarray:
    """Exact-composition random labelling: ``counts[s]`` atoms of species s,
    placed by a seeded random permutation."""
    lab = np.concatenate([np.full(c, s, dtype=np.int32) for s, c in enumerate(counts)])
    assert lab.size == n
    return lab[rng.permutation(n)].astype(np.int32)


_PACK = None


def _packing_lib():
    """The C accept/reject loop (workloads/_packing.c), built with the host
    compiler on first use; None (pure Python loop) if that is not possible."""
    global _PACK
    if _PACK is not None:
        return _PACK or None
    import ctypes
    import shutil
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    so = os.path.join(here, "_packing.so")
    src = os.path.join(here, "_packing.c")
    try:
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
            gcc = shutil.which("gcc")
            if gcc is None:
                _PACK = False
                return None
            tmp = so + f".{os.getpid()}.tmp"
            subprocess.run([gcc, "-O2", "-shared", "-fPIC", "-o", tmp, src, "-lm"], check=True)
            os.replace(tmp, so)
        _PACK = ctypes.CDLL(so)
    except (OSError, subprocess.CalledProcessError):
        _PACK = False
        return None
    return _PACK


def random_dense_packing(n: int, density: float, dmin: float, rng,
                         sweeps: int = 200) -> tuple[np.ndarray, np.ndarray]:
    """Hard-sphere Monte Carlo in a cubic box: start from a simple-cubic
    arrangement at the target density, then ``sweeps`` sweeps of random
    single-particle moves (periodic minimum image).  A move is accepted if the
    particle keeps ``dmin`` from every other one, or, while the start-up
    arrangement is still closer than ``dmin``, if it strictly increases the
    particle's nearest distance; the smallest separation never decreases.
    The accept/reject loop runs in C when a host compiler is available (same
    random numbers, same result)."""
    L = (n / density) ** (1.0 / 3.0)
    # start: n random sites of the simple-cubic, bcc or fcc arrangement of the
    # box with the largest nearest-neighbour distance
    best = None
    for basis, nn in ((np.zeros((1, 3)), 1.0),
                      (np.array([[0, 0, 0], [0.5, 0.5, 0.5]]), math.sqrt(3.0) / 2.0),
                      (np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]), 1.0 / math.sqrt(2.0))):
        mm = int(math.ceil((n / len(basis)) ** (1.0 / 3.0) - 1e-9))
        if best is None or L / mm * nn > best[0]:
            best = (L / mm * nn, mm, basis)
    _, m, basis = best
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    sites = (g[:, None, :] + basis[None, :, :] + 0.25).reshape(-1, 3) * (L / m)
    pos = sites[np.sort(rng.permutation(len(sites))[:n])]
    cell = np.diag([L, L, L])
    # bin grid for overlap checks
    nb = max(1, int(L // dmin))
    w = L / nb
    step = 0.1 * dmin

    def bins_of(p):
        return np.minimum((p // w).astype(int), nb - 1)

    def min_sep(p):
        out = np.inf
        for i0 in range(0, n, 512):
            d = p[i0:i0 + 512, None, :] - p[None, :, :]
            d -= L * np.round(d / L)
            r2 = (d * d).sum(-1)
            r2[np.arange(min(512, n - i0)), np.arange(i0, min(i0 + 512, n))] = np.inf
            out = min(out, float(r2.min()))
        return math.sqrt(out)

    lib = _packing_lib()
    if lib is not None:
        import ctypes as C
        done = 0
        # the given sweeps, then more (at most 2000) while a pair is still closer than dmin
        while done < sweeps or (done < sweeps + 2000 and done % 50 == 0 and min_sep(pos) < dmin) \
                or (sweeps < done < sweeps + 2000 and done % 50 != 0):
            perm = np.ascontiguousarray(rng.permutation(n), dtype=np.int64)
            disp = np.ascontiguousarray(rng.uniform(-step, step, (n, 3)))
            pos = np.ascontiguousarray(pos, dtype=np.float64)
            lib.rdp_sweeps(C.c_int(n), C.c_double(L), C.c_double(dmin), C.c_int(nb), C.c_int(1),
                           perm.ctypes.data_as(C.c_void_p), disp.ctypes.data_as(C.c_void_p),
                           pos.ctypes.data_as(C.c_void_p))
            done += 1
        return wrap(pos, cell), cell

    b = bins_of(pos)
    from collections import defaultdict
    grid = defaultdict(list)
    for i in range(n):
        grid[tuple(b[i])].append(i)

    def nearest(i, t, tb, stop):
        best = 1e300
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    key = ((tb[0] + dx) % nb, (tb[1] + dy) % nb, (tb[2] + dz) % nb)
                    for j in grid.get(key, ()):
                        if j == i:
                            continue
                        d = t - pos[j]
                        d -= L * np.round(d / L)
                        r2 = float(d @ d)
                        best = min(best, r2)
                        if best < stop:
                            return best
        return best

    done = 0
    while done < sweeps or (done < sweeps + 2000 and done % 50 == 0 and min_sep(pos) < dmin) \
            or (sweeps < done < sweeps + 2000 and done % 50 != 0):
        done += 1
        perm = rng.permutation(n)
        disp = rng.uniform(-step, step, (n, 3))
        for q, i in enumerate(perm):
            trial = (pos[i] + disp[q]) % L
            tb = bins_of(trial[None])[0]
            mt = nearest(i, trial, tb, dmin * dmin)
            ok = mt >= dmin * dmin
            if not ok:
                ok = nearest(i, trial, tb, -1.0) > nearest(i, pos[i], b[i], -1.0)
            if ok:
                ob = tuple(b[i])
                grid[ob].remove(i)
                pos[i] = trial
                b[i] = tb
                grid[tuple(tb)].append(i)
    return wrap(pos, cell), cell


# ----------------------------------------------------------------------------
# tight-binding parameter tables (plain data)
# ----------------------------------------------------------------------------
def canonical_d_model(r_cut: float, onsite_d=(0.0,), d_cut: float = 0.0) -> dict:
    """Canonical d band: dd sigma : dd pi : dd delta = -6 : 4 : -1 with a
    power law r^-5, scaled so that dd sigma = -1 eV at r = 2.48 A.
    ``onsite_d`` gives the d level of each species (eV)."""
    ns = len(onsite_d)
    bonds = {}
    for si in range(ns):
        for sj in range(ns):
            bonds[(si, sj)] = {
                "dds": (FORM_POWER, -1.0, 2.48, 5.0),
                "ddp": (FORM_POWER, 4.0 / 6.0, 2.48, 5.0),
                "ddd": (FORM_POWER, -1.0 / 6.0, 2.48, 5.0),
            }
    return {"n_orb": 5, "n_species": ns, "r_cut": float(r_cut), "d_cut": float(d_cut),
            "onsite": [[0.0, 0.0, float(e)] for e in onsite_d], "bonds": bonds}


# synthetic s,p,d bond-integral prefactors (eV) for species pair A-A, for the
# exponential form beta0 * exp(-1.8 (r - 2.5)); reversed channels follow the
# parity rule V(l'l m) = (-1)^(l+l') V(l l' m).
_SPD_AA = {"sss": -1.2, "sps": 1.5, "sds": -0.8, "pps": 2.0, "ppp": -0.6,
           "pds": -1.1, "pdp": 0.5, "dds": -0.9, "ddp": 0.5, "ddd": -0.1}
_PARITY_REVERSED = {"pss": ("sps", -1.0), "dss": ("sds", 1.0),
                    "dps": ("pds", -1.0), "dpp": ("pdp", -1.0)}


def spd_alloy_model(r_cut: float = 4.2, lam: float = 1.8, r0: float = 2.5) -> dict:
    """Two-species s,p,d model.  B-B integrals are 0.9 x A-A; A-B are the
    geometric mean with the sign kept.  Onsite (s, p, d): A = (-4, 2, 0),
    B = (-3.5, 2.5, 0.5) eV."""
    scale = {(0, 0): 1.0, (1, 1): 0.9, (0, 1): math.sqrt(0.9), (1, 0): math.sqrt(0.9)}
    bonds = {}
    for pair, f in scale.items():
        ch = {}
        for name, v in _SPD_AA.items():
            ch[name] = (FORM_EXP, f * v, r0, lam)
        for name, (src, sgn) in _PARITY_REVERSED.items():
            ch[name] = (FORM_EXP, sgn * f * _SPD_AA[src], r0, lam)
        bonds[pair] = ch
    return {"n_orb": 9, "n_species": 2, "r_cut": float(r_cut), "d_cut": 0.0,
            "onsite": [[-4.0, 2.0, 0.0], [-3.5, 2.5, 0.5]], "bonds": bonds}


def model_arrays(model: dict):
    """Flatten a model dict into dense arrays indexed [pair = si*ns+sj][channel]:
    ``form`` (int32), ``beta0``, ``r0``, ``q`` (float64); absent channels have
    beta0 = 0.  Also returns ``onsite`` [ns, 3] (s, p, d levels)."""
    ns = model["n_species"]
    form = np.zeros((ns * ns, len(CHANNELS)), np.int32)
    beta0 = np.zeros((ns * ns, len(CHANNELS)))
    r0 = np.ones((ns * ns, len(CHANNELS)))
    q = np.zeros((ns * ns, len(CHANNELS)))
    for (si, sj), chans in model["bonds"].items():
        for name, (f, b, rr, qq) in chans.items():
            c = CHANNELS.index(name)
            form[si * ns + sj, c] = f
            beta0[si * ns + sj, c] = b
            r0[si * ns + sj, c] = rr
            q[si * ns + sj, c] = qq
    onsite = np.asarray(model["onsite"], np.float64).reshape(ns, 3)
    return form, beta0, r0, q, onsite


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    pos: np.ndarray
    cell: np.ndarray
    species: np.ndarray
    model: dict
    n_max: int
    n_exp: int
    n_elec: np.ndarray            # valence electrons per atom (both spins)
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])


def bcc_small(seed: int = 1) -> Workload:
    rng = _rng(seed)
    pos, cell = cubic_lattice("bcc", 2.87, 4)
    pos = displace(pos, cell, 0.05, rng)
    n = pos.shape[0]
    return Workload("bcc_small", pos, cell, np.zeros(n, np.int32),
                    canonical_d_model(3.5), n_max=9, n_exp=200,
                    n_elec=np.full(n, 6.5), meta={"seed": seed, "a": 2.87, "reps": 4})


def bcc_large(seed: int = 2, reps: int = 40) -> Workload:
    rng = _rng(seed)
    pos, cell = cubic_lattice("bcc", 3.16, reps)
    pos = displace(pos, cell, 0.08, rng)
    n = pos.shape[0]
    return Workload("bcc_large", pos, cell, np.zeros(n, np.int32),
                    canonical_d_model(3.8), n_max=18, n_exp=200,
                    n_elec=np.full(n, 4.5), meta={"seed": seed, "a": 3.16, "reps": reps})


def fcc_alloy_spd(seed: int = 3, reps: int = 30) -> Workload:
    rng = _rng(seed)
    pos, cell = cubic_lattice("fcc", 3.5355, reps)
    pos = wrap(pos, cell)
    n = pos.shape[0]
    spc = random_species(n, [n // 2, n - n // 2], rng)
    val = np.where(spc == 0, 9.0, 8.0)
    return Workload("fcc_alloy_spd", pos, cell, spc, spd_alloy_model(),
                    n_max=20, n_exp=200, n_elec=val,
                    meta={"seed": seed, "a": 3.5355, "reps": reps})


def bcc_alloy_scf(seed: int = 5, reps: int = 50, a: float = 2.87) -> Workload:
    rng = _rng(seed)
    pos, cell = cubic_lattice("bcc", a, reps)
    pos = wrap(pos, cell)
    n = pos.shape[0]
    spc = random_species(n, [n // 2, n - n // 2], rng)
    val = np.where(spc == 0, 6.0, 5.0)
    return Workload("bcc_alloy_scf", pos, cell, spc,
                    canonical_d_model(3.5, onsite_d=(0.0, 0.8)),
                    n_max=16, n_exp=200, n_elec=val,
                    meta={"seed": seed, "a": a, "reps": reps})


def ragged_structure(s: int, base_seed: int = 4000) -> Workload:
    """Structure ``s`` of the ragged batch: size drawn log-uniformly in
    [50, 5000], kind uniform in {bcc, fcc, hcp, random}, all at a density of
    0.085 atoms / A^3."""
    rng = _rng(base_seed + s)
    target = int(round(math.exp(rng.uniform(math.log(50.0), math.log(5000.0)))))
    kind = ("bcc", "fcc", "hcp", "random")[int(rng.integers(0, 4))]
    rho = 0.085
    if kind in ("bcc", "fcc"):
        nb = 2 if kind == "bcc" else 4
        a = (nb / rho) ** (1.0 / 3.0)
        m = max(1, int(round((target / nb) ** (1.0 / 3.0))))
        pos, cell = cubic_lattice(kind, a, (m, m, m))
        pos = displace(pos, cell, 0.05, rng)
    elif kind == "hcp":
        a = (math.sqrt(2.0) / rho) ** (1.0 / 3.0)
        # 4-atom orthorhombic cell a x a*sqrt3 x c; pick near-cubic repeats
        b, c = a * math.sqrt(3.0), a * math.sqrt(8.0 / 3.0)
        best = None
        for n1 in range(1, 30):
            for n2 in range(1, 20):
                for n3 in range(1, 20):
                    N = 4 * n1 * n2 * n3
                    L = np.array([n1 * a, n2 * b, n3 * c])
                    cost = abs(N - target) / target + 0.2 * (L.max() / L.min() - 1.0)
                    if best is None or cost < best[0]:
                        best = (cost, (n1, n2, n3))
        pos, cell = hcp_lattice(a, best[1])
        pos = displace(pos, cell, 0.05, rng)
    else:
        pos, cell = random_dense_packing(target, rho, 2.2, rng, sweeps=20)
    n = pos.shape[0]
    return Workload(f"ragged_{s}", pos, cell, np.zeros(n, np.int32),
                    canonical_d_model(3.6), n_max=14, n_exp=200,
                    n_elec=np.full(n, 6.5), meta={"kind": kind, "target": target})


def dimer(d: float = 2.6, box: float = 30.0, direction=(0.0, 0.0, 1.0)) -> Workload:
    """Two d-only atoms at distance ``d`` along ``direction`` in a large cubic
    box (no periodic image within the cutoff)."""
    u = np.asarray(direction, float)
    u = u / np.linalg.norm(u)
    c = np.array([box / 2] * 3)
    pos = np.stack([c - 0.5 * d * u, c + 0.5 * d * u])
    cell = np.diag([box] * 3)
    return Workload("dimer", wrap(pos, cell), cell, np.zeros(2, np.int32),
                    canonical_d_model(3.5), n_max=9, n_exp=200,
                    n_elec=np.full(2, 6.5))


NAMED = {
    "bcc_small": bcc_small,
    "bcc_large": bcc_large,
    "fcc_alloy_spd": fcc_alloy_spd,
    "bcc_alloy_scf": bcc_alloy_scf,
}


def md_trajectory(wl: Workload, n_steps: int, step_sigma: float = 0.02, seed: int = 6000) -> list:
    """A seeded stand-in for the positions of successive MD steps: each step
    adds i.i.d. normal displacements (step_sigma per component, Angstrom) to
    the previous positions, wrapped into the cell.  Returns n_steps position
    arrays, the first being the workload's own."""
    rng = _rng(seed)
    out = [np.array(wl.pos, np.float64)]
    for _ in range(n_steps - 1):
        out.append(wrap(out[-1] + rng.normal(scale=step_sigma, size=out[-1].shape), wl.cell))
    return out

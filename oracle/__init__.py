"""CPU oracle for the analytic-BOP energy path — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The HIP product path never imports,
links or calls it, and this package imports nothing from the product.

The numerics live in ``bop_oracle.c`` (plain FP64 C, OpenMP over atoms), each
function citing the passage of arXiv:1803.07491 it follows; this module only
marshals NumPy arrays into it.  The MLP reference (forward, backward, Adam)
is written here in NumPy FP64.

Functions whose results have no independent pin are marked "parity unpinned"
in their docstring.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bop_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAXSP = 4
NCH = 14


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [
        ("n_species", C.c_int),
        ("n_orb", C.c_int),
        ("r_cut", C.c_double),
        ("d_cut", C.c_double),
        ("onsite", (C.c_double * 3) * MAXSP),
        ("form", (C.c_int * NCH) * (MAXSP * MAXSP)),
        ("beta0", (C.c_double * NCH) * (MAXSP * MAXSP)),
        ("r0", (C.c_double * NCH) * (MAXSP * MAXSP)),
        ("q", (C.c_double * NCH) * (MAXSP * MAXSP)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        _lib.or_neighbours.restype = C.c_long
        _lib.or_neighbours.argtypes = [C.c_int, P, P, C.c_double, C.c_int, C.c_long, P, P, P, P]
        _lib.or_build_H.argtypes = [P, C.c_int, P, P, P, P, P, P, P]
        _lib.or_moments.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, C.c_int, P, P]
        _lib.or_moments_radius.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, C.c_double, P, P, C.c_int, P, P]
        _lib.or_recursion.argtypes = [C.c_int, C.c_int, P, C.c_int, C.c_double, C.c_double, P, P, P, P, P]
        _lib.or_jackson.argtypes = [C.c_int, P]
        _lib.or_dos_coeffs.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, P, P, P]
        _lib.or_orbital_NU.argtypes = [C.c_int, P, C.c_double, C.c_double, C.c_double, C.c_double, P, P, P]
        _lib.or_count.restype = C.c_double
        _lib.or_count.argtypes = [C.c_int, C.c_int, P, P, P, C.c_double]
        _lib.or_fermi.restype = C.c_double
        _lib.or_fermi.argtypes = [C.c_int, C.c_int, P, P, P, C.c_double]
        _lib.or_energy.restype = C.c_double
        _lib.or_energy.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, C.c_double, P, P, P]
        _lib.or_scf_step.restype = C.c_double
        _lib.or_scf_step.argtypes = [C.c_int, P, P, P, C.c_double, C.c_double, C.c_double, P, P, P]
        _lib.or_rotation.argtypes = [P, P, P]
        _lib.or_n_a.argtypes = [C.c_int]
        _lib.or_n_b.argtypes = [C.c_int]
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def num_threads() -> int:
    return int(lib().or_num_threads())


def model_struct(model: dict) -> _Model:
    """Fill the oracle's own model struct from a plain model dict
    (``workloads`` format)."""
    from workloads import CHANNELS  # plain data names only
    m = _Model()
    ns = model["n_species"]
    assert ns <= MAXSP
    m.n_species = ns
    m.n_orb = model["n_orb"]
    m.r_cut = model["r_cut"]
    m.d_cut = model.get("d_cut", 0.0)
    for s in range(ns):
        for l in range(3):
            m.onsite[s][l] = model["onsite"][s][l]
    for pr in range(MAXSP * MAXSP):
        for c in range(NCH):
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


# --------------------------------------------------------------------------
def neighbours(pos, cell, r_cut, brute=False):
    """Periodic neighbour list (CSR).  Returns dict(row_ptr, nbr_j, nbr_shift,
    nbr_d)."""
    pos = _c(pos, np.float64)
    cell = _c(cell, np.float64)
    n = pos.shape[0]
    rp = np.zeros(n + 1, np.int32)
    need = lib().or_neighbours(n, _p(pos), _p(cell), r_cut, int(brute), 0, _p(rp), None, None, None)
    nj = np.zeros(need, np.int32)
    ns = np.zeros((need, 3), np.int32)
    nd = np.zeros((need, 3), np.float64)
    got = lib().or_neighbours(n, _p(pos), _p(cell), r_cut, int(brute), need, _p(rp), _p(nj), _p(ns), _p(nd))
    assert got == need
    return {"row_ptr": rp, "nbr_j": nj, "nbr_shift": ns, "nbr_d": nd}


def build_H(model, species, nl, shift=None):
    """Onsite levels [N, n_orb] and bond blocks [P, n_orb, n_orb] (FP64)."""
    m = model_struct(model)
    species = _c(species, np.int32)
    n = species.shape[0]
    no = model["n_orb"]
    P = nl["nbr_j"].shape[0]
    H_on = np.zeros((n, no))
    H_bond = np.zeros((P, no, no))
    sh = None if shift is None else _c(shift, np.float64)
    lib().or_build_H(C.byref(m), n, _p(species), _p(sh), _p(nl["row_ptr"]), _p(nl["nbr_j"]),
                     _p(nl["nbr_d"]), _p(H_on), _p(H_bond))
    return H_on, H_bond


def moments(nl, H_on, H_bond, n_max, sel=None, r_max=0.0):
    """Orbital moments mu[s, a, n] = <i a|H^n|i a> for i = sel[s]; with
    r_max > 0 only paths that stay within r_max of atom i (Sec. III
    "Speed-ups" (iii))."""
    n, no = H_on.shape
    sel = np.arange(n, dtype=np.int32) if sel is None else _c(sel, np.int32)
    mu = np.zeros((sel.shape[0], no, n_max + 1))
    if r_max > 0.0:
        lib().or_moments_radius(n, no, n_max, _p(nl["row_ptr"]), _p(nl["nbr_j"]), _p(_c(nl["nbr_d"], np.float64)),
                                float(r_max), _p(_c(H_on, np.float64)), _p(_c(H_bond, np.float64)), sel.shape[0],
                                _p(sel), _p(mu))
    else:
        lib().or_moments(n, no, n_max, _p(nl["row_ptr"]), _p(nl["nbr_j"]), _p(_c(H_on, np.float64)),
                         _p(_c(H_bond, np.float64)), sel.shape[0], _p(sel), _p(mu))
    return mu


def n_a(n_max):
    return int(lib().or_n_a(n_max))


def n_b(n_max):
    return int(lib().or_n_b(n_max))


BW_MODES = {"gershgorin": 0, "global": 1, "lowest": 2, "highest": 3, "average": 4, "average_highest": 5,
            "minmax": 6, "weighted": 7}


def recursion(mu_rows, n_max, global_ab=None, bw="gershgorin", beta=1.0):
    """Recursion coefficients and terminator per row (orbital).  ``mu_rows``
    [R, n_max+1]; ``bw`` one of BW_MODES (App. B.5 options i-v, vii, viii and
    the weighted average of Eq. weighted with ``beta``).  Returns dict(a, b,
    a_inf, b_inf, flags)."""
    mu_rows = _c(mu_rows, np.float64).reshape(-1, n_max + 1)
    R = mu_rows.shape[0]
    a = np.zeros((R, n_a(n_max)))
    b = np.zeros((R, n_b(n_max) + 1))
    ai = np.zeros(R)
    bi = np.zeros(R)
    fl = np.zeros(R, np.int32)
    if global_ab is not None:
        mode, p1, p2 = 1, global_ab[0], global_ab[1]
    else:
        mode, p1, p2 = BW_MODES[bw], (beta if bw == "weighted" else 0.0), 0.0
    lib().or_recursion(R, n_max, _p(mu_rows), mode, p1, p2, _p(a), _p(b), _p(ai), _p(bi), _p(fl))
    return {"a": a, "b": b, "a_inf": ai, "b_inf": bi, "flags": fl}


def jackson(n_exp):
    g = np.zeros(n_exp + 1)
    lib().or_jackson(n_exp, _p(g))
    return g


def dos_coeffs(mu_rows, rec, n_max, n_exp, with_chain=False):
    """g_m sigma_m [R, n_exp+1]; with ``with_chain`` also the chain route's
    sigma_m for m <= n_max [R, n_max+1]."""
    mu_rows = _c(mu_rows, np.float64).reshape(-1, n_max + 1)
    R = mu_rows.shape[0]
    gs = np.zeros((R, n_exp + 1))
    sc = np.zeros((R, n_max + 1)) if with_chain else None
    lib().or_dos_coeffs(R, n_max, n_exp, _p(mu_rows), _p(rec["a"]), _p(rec["b"]), _p(rec["a_inf"]),
                        _p(rec["b_inf"]), _p(gs), _p(sc))
    return (gs, sc) if with_chain else gs


def orbital_NU(gsig_row, a_inf, b_inf, e_on, E):
    n_exp = gsig_row.shape[0] - 1
    N, U, D = C.c_double(), C.c_double(), C.c_double()
    lib().or_orbital_NU(n_exp, _p(_c(gsig_row, np.float64)), a_inf, b_inf, e_on, E,
                        C.byref(N), C.byref(U), C.byref(D))
    return N.value, U.value, D.value


def count(gsig, a_inf, b_inf, E):
    R, ne1 = gsig.shape
    return lib().or_count(R, ne1 - 1, _p(gsig), _p(a_inf), _p(b_inf), E)


def fermi(gsig, a_inf, b_inf, n_elec):
    R, ne1 = gsig.shape
    return lib().or_fermi(R, ne1 - 1, _p(_c(gsig, np.float64)), _p(_c(a_inf, np.float64)),
                          _p(_c(b_inf, np.float64)), float(n_elec))


def energy(gsig, a_inf, b_inf, H_on, E_F):
    """Per-atom N_i, U_i, n_i(E_F) (both spins) and U_total."""
    n, no = H_on.shape
    Na = np.zeros(n)
    Ua = np.zeros(n)
    Da = np.zeros(n)
    tot = lib().or_energy(n, no, gsig.shape[1] - 1, _p(_c(gsig, np.float64)), _p(_c(a_inf, np.float64)),
                          _p(_c(b_inf, np.float64)), _p(_c(H_on, np.float64)), E_F, _p(Na), _p(Ua), _p(Da))
    return {"N_atom": Na, "U_atom": Ua, "dos_atom": Da, "U_total": tot}


def scf_step(N_atom, dos_atom, n0, shift, mix=0.5, n_floor=1e-3, tol=1e-4):
    shift = np.array(shift, dtype=np.float64, copy=True)
    q = np.zeros_like(shift)
    conv = C.c_int()
    mq = lib().or_scf_step(shift.shape[0], _p(_c(N_atom, np.float64)), _p(_c(dos_atom, np.float64)),
                           _p(_c(n0, np.float64)), mix, n_floor, tol, _p(shift), _p(q), C.byref(conv))
    return shift, q, mq, bool(conv.value)


def rotation(u):
    Rp = np.zeros((3, 3))
    Rd = np.zeros((5, 5))
    lib().or_rotation(_p(_c(u, np.float64)), _p(Rp), _p(Rd))
    return Rp, Rd


# --------------------------------------------------------------------------
def energy_pipeline(wl, shift=None, sel=None, n_max=None, n_exp=None, E_F=None, nl=None, bw="gershgorin",
                    beta=1.0, r_max=0.0):
    """Whole path for a workload: neighbours -> H -> moments -> recursion ->
    DOS coefficients -> Fermi level (unless given) -> energies.  With ``sel``
    only those atoms' moments and energies are computed and ``E_F`` must be
    given."""
    n_max = wl.n_max if n_max is None else n_max
    n_exp = wl.n_exp if n_exp is None else n_exp
    if nl is None:
        nl = neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    H_on, H_bond = build_H(wl.model, wl.species, nl, shift)
    mu = moments(nl, H_on, H_bond, n_max, sel, r_max=r_max)
    no = H_on.shape[1]
    rows = mu.reshape(-1, n_max + 1)
    rec = recursion(rows, n_max, bw=bw, beta=beta)
    gs = dos_coeffs(rows, rec, n_max, n_exp)
    Hs = H_on if sel is None else H_on[np.asarray(sel)]
    if E_F is None:
        assert sel is None
        E_F = fermi(gs, rec["a_inf"], rec["b_inf"], float(np.sum(wl.n_elec)))
    en = energy(gs, rec["a_inf"], rec["b_inf"], Hs, E_F)
    return {"nl": nl, "H_on": H_on, "H_bond": H_bond, "mu": mu, "rec": rec, "gsig": gs,
            "E_F": E_F, **en}


def energy_pipeline_avg(wl, shift=None, n_max=None, n_exp=None, E_F=None, nl=None):
    """Atom-averaged mode of the energy path (the per-atom reading of the
    moments): one recursion chain per atom, from its orbital-averaged moments
    mu_i / n_orb = sum_a mu_ia / n_orb and the averaged onsite level, each
    chain standing for n_orb orbitals in the electron count and the energies
    (N_i = 2 n_orb N_chain, U_i = 2 n_orb U_chain).  Where all orbitals of an
    atom share one local DOS (e.g. equal bond integrals in every channel) it
    equals the orbital-resolved path."""
    n_max = wl.n_max if n_max is None else n_max
    n_exp = wl.n_exp if n_exp is None else n_exp
    if nl is None:
        nl = neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    H_on, H_bond = build_H(wl.model, wl.species, nl, shift)
    mu = moments(nl, H_on, H_bond, n_max)
    n, no = H_on.shape
    mu_avg = mu.reshape(n, no, n_max + 1).mean(axis=1)
    e_avg = H_on.mean(axis=1)
    rec = recursion(mu_avg, n_max)
    gs = dos_coeffs(mu_avg, rec, n_max, n_exp)
    if E_F is None:
        E_F = fermi(gs, rec["a_inf"], rec["b_inf"], float(np.sum(wl.n_elec)) / no)
    en = energy(gs, rec["a_inf"], rec["b_inf"], e_avg[:, None], E_F)
    return {"mu_avg": mu_avg, "H_avg": e_avg, "rec": rec, "E_F": E_F, "N_atom": no * en["N_atom"],
            "U_atom": no * en["U_atom"], "dos_atom": no * en["dos_atom"], "U_total": no * en["U_total"]}


def scf(wl, shift0=None, mix=0.5, tol=1e-4, max_iter=200, n_floor=1e-3, n_max=None):
    """Plain local-charge-neutrality cycle; returns (shift, history)."""
    n = wl.n_atoms
    shift = np.zeros(n) if shift0 is None else np.array(shift0, float)
    nl = neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    hist = []
    for it in range(max_iter):
        r = energy_pipeline(wl, shift=shift, nl=nl, n_max=n_max)
        shift_new, q, mq, conv = scf_step(r["N_atom"], r["dos_atom"], wl.n_elec, shift, mix, n_floor, tol)
        hist.append({"it": it, "max_dq": mq, "U_total": r["U_total"], "E_F": r["E_F"]})
        if conv:
            return shift, hist, r
        shift = shift_new
    return shift, hist, r


# --------------------------------------------------------------------------
# Collinear magnetism (Sec. II "Hamiltonian": one loop over the two spin
# channels; App. A.2.2 collinear onsite levels; App. A.1 Eq. TB-UX).
# --------------------------------------------------------------------------
def spin_shifts(shift, moment, species, stoner, B_z=0.0):
    """Onsite shifts of the two spin channels (collinear form of the onsite
    levels, App. A.2.2): E_iav = H0 + shift_i - (-1)^v B_z + (1/2) (-1)^v I_i m_i.
    Reading: (-1)^v = -1 for the up channel, so that the majority channel
    (m_i > 0 means more up electrons) is lowered by I_i m_i / 2 (Stoner)."""
    I = np.asarray(stoner, np.float64)[np.asarray(species)]
    shift = np.asarray(shift, np.float64)
    moment = np.asarray(moment, np.float64)
    return shift + B_z - 0.5 * I * moment, shift - B_z + 0.5 * I * moment


def energy_pipeline_mag(wl, stoner, shift=None, moment=None, B_z=0.0, n_max=None, n_exp=None, nl=None):
    """Collinear-magnetic energy path: both spin channels share the bonds and
    differ in their onsite levels; one Fermi level with sum over channels,
    orbitals and atoms of N_iav = N_e; per channel N_iv = sum_a N_iav and the
    onsite bond energy U_iv = sum_a int^E_F (E - E_iav) n_iav dE (Eq.
    TB-Ubond with the spin index); moments m_i = N_iup - N_idown; exchange
    energy U_X = -1/4 sum_i I_i m_i^2 (Eq. TB-UX) of these moments.
    The channels' rows are stacked (up atoms then down atoms) and handed to
    the non-magnetic count and energy routines, which count both spins of a
    row (factor 2): the Fermi level of the stacked rows for 2 N_e electrons is
    the one of the channels for N_e, and their per-atom outputs are halved."""
    n = wl.n_atoms
    n_max = wl.n_max if n_max is None else n_max
    n_exp = wl.n_exp if n_exp is None else n_exp
    shift = np.zeros(n) if shift is None else np.asarray(shift, np.float64)
    moment = np.zeros(n) if moment is None else np.asarray(moment, np.float64)
    if nl is None:
        nl = neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    s_up, s_dn = spin_shifts(shift, moment, wl.species, stoner, B_z)
    H_up, H_bond = build_H(wl.model, wl.species, nl, s_up)
    H_dn, _ = build_H(wl.model, wl.species, nl, s_dn)
    mu = np.concatenate([moments(nl, H_up, H_bond, n_max), moments(nl, H_dn, H_bond, n_max)])
    rows = mu.reshape(-1, n_max + 1)
    rec = recursion(rows, n_max)
    gs = dos_coeffs(rows, rec, n_max, n_exp)
    n_e = float(np.sum(wl.n_elec))
    E_F = fermi(gs, rec["a_inf"], rec["b_inf"], 2.0 * n_e)
    en = energy(gs, rec["a_inf"], rec["b_inf"], np.concatenate([H_up, H_dn]), E_F)
    N_sp = en["N_atom"].reshape(2, n) / 2.0
    U_sp = en["U_atom"].reshape(2, n) / 2.0
    D_sp = en["dos_atom"].reshape(2, n) / 2.0
    m_out = N_sp[0] - N_sp[1]
    I = np.asarray(stoner, np.float64)[np.asarray(wl.species)]
    return {"E_F": E_F, "N_spin": N_sp, "U_spin": U_sp, "dos_spin": D_sp, "N_atom": N_sp.sum(0),
            "U_atom": U_sp.sum(0), "dos_atom": D_sp.sum(0), "moment": m_out,
            "U_bond": float(U_sp.sum()), "U_X": float(-0.25 * np.sum(I * m_out * m_out)), "mu": mu, "rec": rec}


def scf_mag(wl, stoner, moment0, shift0=None, B_z=0.0, mix=0.5, mix_m=0.5, tol=1e-4, tol_m=1e-4, max_iter=200,
            n_floor=1e-3, n_max=None):
    """Self-consistent collinear magnetism with local charge neutrality: the
    shifts follow the linear charge-neutrality cycle (total DOS at E_F), the
    moments are mixed linearly, m_i <- m_i + mix_m (m_i^out - m_i) (a Stoner
    cycle).  Converged when max |q_i| < tol and max |m_i^out - m_i| < tol_m;
    then nothing is updated.  Returns (shift, moment, history, last result)."""
    n = wl.n_atoms
    shift = np.zeros(n) if shift0 is None else np.array(shift0, float)
    m = np.array(moment0, float) * np.ones(n)
    nl = neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    hist = []
    for it in range(max_iter):
        r = energy_pipeline_mag(wl, stoner, shift, m, B_z, n_max=n_max, nl=nl)
        q = r["N_atom"] - wl.n_elec
        dm = r["moment"] - m
        mq, mdm = float(np.max(np.abs(q))), float(np.max(np.abs(dm)))
        hist.append({"it": it, "max_dq": mq, "max_dm": mdm, "m_mean": float(r["moment"].mean())})
        if mq < tol and mdm < tol_m:
            return shift, m, hist, r
        shift = shift + mix * q / np.maximum(r["dos_atom"], n_floor)
        shift = shift - shift.mean()
        m = m + mix_m * dm
    return shift, m, hist, r


class Broyden:
    """Broyden's second method (Broyden 1965, the update of the inverse
    Jacobian) for F(x) = 0, as a mixer of the self-consistency cycle (Sec. II
    "Self-consistency", mixer (ii)).

    H_0 = -eta I, so the first step x + eta F is linear mixing.  With s =
    x_n - x_(n-1) and y = F_n - F_(n-1):
        H_n = H_(n-1) + (s - H_(n-1) y) y^T / (y^T y),
        x_(n+1) = x_n - H_n F_n.
    H is kept as -eta I + sum_k u_k y_k^T with u_k = (s - H_(k-1) y) / (y^T y).
    After ``hist`` updates the history is cleared (a restart from H_0).
    Readings (the paper names the method only): F is the Newton-like output
    step q_i / max(n_i(E_F), n_floor) of the linear mixer, and the mean of x
    is removed after each step (the gauge of the charge-neutrality cycle)."""

    def __init__(self, eta=0.5, hist=20, gauge=True):
        self.eta, self.hist, self.gauge = float(eta), int(hist), gauge
        self.u, self.y = [], []
        self.x_prev = self.F_prev = None

    def apply_H(self, v):
        out = -self.eta * v
        for u, y in zip(self.u, self.y):
            out = out + u * np.dot(y, v)
        return out

    def step(self, x, F):
        x = np.asarray(x, np.float64)
        F = np.asarray(F, np.float64)
        if self.x_prev is not None and len(self.u) >= self.hist:
            self.u, self.y, self.x_prev, self.F_prev = [], [], None, None     # restart
        if self.x_prev is not None:
            s = x - self.x_prev
            y = F - self.F_prev
            yy = np.dot(y, y)
            # an unchanged F (y = 0) gives no information: a zero update
            self.u.append((s - self.apply_H(y)) / yy if yy > 0.0 else np.zeros_like(x))
            self.y.append(y)
        self.x_prev, self.F_prev = x.copy(), F.copy()
        xn = x - self.apply_H(F)
        if self.gauge:
            xn = xn - xn.mean()
        return xn


def scf_broyden(wl, shift0=None, mix=0.5, tol=1e-4, max_iter=200, n_floor=1e-3, n_max=None, hist=20):
    """Charge-neutrality cycle with Broyden mixing; returns (shift, history,
    last pipeline result).  Convergence test as in the linear cycle: stop,
    with the shifts unchanged, once max |q_i| < tol."""
    n = wl.n_atoms
    shift = np.zeros(n) if shift0 is None else np.array(shift0, float)
    nl = neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    mixer = Broyden(mix, hist)
    hist_out = []
    for it in range(max_iter):
        r = energy_pipeline(wl, shift=shift, nl=nl, n_max=n_max)
        q = r["N_atom"] - wl.n_elec
        mq = float(np.max(np.abs(q)))
        hist_out.append({"it": it, "max_dq": mq, "U_total": r["U_total"], "E_F": r["E_F"]})
        if mq < tol:
            return shift, hist_out, r
        F = q / np.maximum(r["dos_atom"], n_floor)
        shift = mixer.step(shift, F)
    return shift, hist_out, r


# --------------------------------------------------------------------------
# MLP reference (NumPy FP64).  Network: x (6) -> tanh(W1 x + b1) (64)
# -> tanh(W2 h1 + b2) (64) -> W3 h2 + b3 (1); loss = mean squared error.
# Not from the paper (its warm start of onsite levels, Sec. III "Speed-ups"
# (ii), is the idea this replaces).  Pins: the gradients by central finite
# differences of the loss; Adam by hand-worked steps and the constant-gradient
# invariant of its bias correction (Kingma & Ba, Algorithm 1).
# --------------------------------------------------------------------------
def mlp_forward(params, x):
    W1, b1, W2, b2, W3, b3 = params
    z1 = x @ W1.T + b1
    h1 = np.tanh(z1)
    z2 = h1 @ W2.T + b2
    h2 = np.tanh(z2)
    y = h2 @ W3.T + b3
    return y[:, 0], (x, h1, h2)


def mlp_loss_grad(params, x, t):
    W1, b1, W2, b2, W3, b3 = params
    y, (x, h1, h2) = mlp_forward(params, x)
    B = x.shape[0]
    r = y - t
    loss = np.mean(r * r)
    gy = (2.0 / B) * r[:, None]            # dL/dy
    gW3 = gy.T @ h2
    gb3 = gy.sum(0)
    gh2 = gy @ W3
    gz2 = gh2 * (1.0 - h2 * h2)
    gW2 = gz2.T @ h1
    gb2 = gz2.sum(0)
    gh1 = gz2 @ W2
    gz1 = gh1 * (1.0 - h1 * h1)
    gW1 = gz1.T @ x
    gb1 = gz1.sum(0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def feature_stats(x):
    """Column means and standard deviations (n - 1 normalisation, floored at
    1e-12) of the feature rows x [n, 6]."""
    x = np.asarray(x, np.float64)
    return x.mean(0), np.maximum(x.std(0, ddof=1), 1e-12)


def mlp_shift(params, x):
    """Warm-start shifts: the network's outputs minus their mean (the gauge of
    the charge-neutrality cycle)."""
    y, _ = mlp_forward(params, x)
    return y - y.mean()


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, Algorithm 1): moment estimates, bias
    correction by 1 - beta^t, eps added outside the square root."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** t)
        vh = vv / (1 - b2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


# --------------------------------------------------------------------------
# Forces of the bond energy (App. C.1-C.2: dU/dLambda through the weights
# w = dU/dmu, Eq. weights; the bond-order-like Theta~ = dU/dH, Eq.
# Theta_tilde_BOP; F_k = -sum Theta~ grad_k H, Eq. F_k), for the d band.
#
# Written out from the definitions, for cells small enough for dense matrices:
#  * the weights are the exact derivatives of the bond energy with respect to
#    every orbital's moments at the self-determined Fermi level.  The
#    per-orbital part (recursion, terminator, expansion with its chain,
#    damping, N and U at E_F) is evaluated here in complex arithmetic and
#    differentiated by the complex step (Squire & Trapp 1998: f'(x) =
#    Im f(x + ih)/h, exact to rounding for h = 1e-30).  The Fermi level
#    moves with the moments so that the electron count stays N_e, which adds
#    -(E_F - E_bar) dN/dmu with E_bar = sum E_r n_r(E_F) / sum n_r(E_F);
#  * Theta~ = sum_n sum_(l=0..n-1) H^l diag(w_n) H^(n-1-l), the derivative of
#    mu_n = diag(H^n) with respect to the folded Hamiltonian H, by dense
#    matrix powers;
#  * the bond blocks' derivatives with respect to the bond vector are complex
#    steps through the direction-cosine form of the two-centre blocks (the
#    same blocks as App. D's rotation, without its polar singularity);
#  * F_k = -sum over directed pairs p = (i -> j) of Theta~_(i a, j b)
#    dH_p,ab/dd (d_p = r_j + S - r_i, so +1 for k = j and -1 for k = i).
# Onsite levels do not depend on positions, and no repulsive term is modelled.
# Pinned by central finite differences of the bond energy.
# --------------------------------------------------------------------------
def _sk_dd(l, m, n, Vs, Vp, Vd):
    """d-d bond block from the direction cosines (l, m, n) of the bond and its
    three bond integrals, the two-centre table of Slater & Koster (Phys. Rev.
    94, 1498 (1954), Table I), in the orbital order z2, zx, yz, x2-y2, xy of
    App. D.  Polynomial in l, m, n, so it is smooth for every direction
    (including the polar axis, where the angle form of App. D is singular) and
    takes complex arrays for the complex step."""
    s3 = np.sqrt(3.0)
    l2, m2, n2 = l * l, m * m, n * n
    dlm = l2 - m2
    E = {}
    E[4, 4] = 3 * l2 * m2 * Vs + (l2 + m2 - 4 * l2 * m2) * Vp + (n2 + l2 * m2) * Vd
    E[2, 2] = 3 * m2 * n2 * Vs + (m2 + n2 - 4 * m2 * n2) * Vp + (l2 + m2 * n2) * Vd
    E[1, 1] = 3 * n2 * l2 * Vs + (n2 + l2 - 4 * n2 * l2) * Vp + (m2 + n2 * l2) * Vd
    E[4, 2] = 3 * l * m2 * n * Vs + l * n * (1 - 4 * m2) * Vp + l * n * (m2 - 1) * Vd
    E[2, 1] = 3 * m * n2 * l * Vs + m * l * (1 - 4 * n2) * Vp + m * l * (n2 - 1) * Vd
    E[4, 1] = 3 * l2 * m * n * Vs + m * n * (1 - 4 * l2) * Vp + m * n * (l2 - 1) * Vd
    E[4, 3] = 1.5 * l * m * dlm * Vs - 2 * l * m * dlm * Vp + 0.5 * l * m * dlm * Vd
    E[2, 3] = 1.5 * m * n * dlm * Vs - m * n * (1 + 2 * dlm) * Vp + m * n * (1 + 0.5 * dlm) * Vd
    E[1, 3] = 1.5 * n * l * dlm * Vs + n * l * (1 - 2 * dlm) * Vp - n * l * (1 - 0.5 * dlm) * Vd
    zz = n2 - 0.5 * (l2 + m2)
    E[4, 0] = s3 * l * m * zz * Vs - 2 * s3 * l * m * n2 * Vp + 0.5 * s3 * l * m * (1 + n2) * Vd
    E[2, 0] = s3 * m * n * zz * Vs + s3 * m * n * (l2 + m2 - n2) * Vp - 0.5 * s3 * m * n * (l2 + m2) * Vd
    E[1, 0] = s3 * l * n * zz * Vs + s3 * l * n * (l2 + m2 - n2) * Vp - 0.5 * s3 * l * n * (l2 + m2) * Vd
    E[3, 3] = 0.75 * dlm * dlm * Vs + (l2 + m2 - dlm * dlm) * Vp + (n2 + 0.25 * dlm * dlm) * Vd
    E[3, 0] = 0.5 * s3 * dlm * zz * Vs - s3 * n2 * dlm * Vp + 0.25 * s3 * (1 + n2) * dlm * Vd
    E[0, 0] = zz * zz * Vs + 3 * n2 * (l2 + m2) * Vp + 0.75 * (l2 + m2) ** 2 * Vd
    B = np.empty(np.shape(l) + (5, 5), dtype=np.result_type(l, Vs, 1.0))
    for (a, b), v in E.items():
        B[..., a, b] = v
        B[..., b, a] = v
    return B


def _dd_blocks(model, species, nl, d):
    """d-d bond blocks of the directed pairs of ``nl`` for bond vectors d [P, 3]
    (complex allowed), by the direction-cosine table."""
    ns = model["n_species"]
    i_of = np.repeat(np.arange(len(nl["row_ptr"]) - 1), np.diff(nl["row_ptr"]))
    pair = species[i_of] * ns + species[nl["nbr_j"]]
    r = np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])
    V = np.zeros((d.shape[0], 3), dtype=r.dtype)
    for k, ch in enumerate(("dds", "ddp", "ddd")):
        for (si, sj), chans in model["bonds"].items():
            if ch not in chans:
                continue
            f, b0, r0, q = chans[ch]
            sel = pair == si * ns + sj
            v = b0 * (r0 / r[sel]) ** q if f == 0 else b0 * np.exp(-q * (r[sel] - r0))
            V[sel, k] = v
    assert model.get("d_cut", 0.0) == 0.0, "forces: hard cutoff only"
    u = d / r[:, None]
    return _sk_dd(u[:, 0], u[:, 1], u[:, 2], V[:, 0], V[:, 1], V[:, 2])


def _tail_c(mu, n_max, n_exp, E_F, e_on):
    """Per-orbital energy path in complex arithmetic, the steps of the C
    oracle's recursion, Gershgorin terminator, expansion coefficients (moment
    route and chain) and N, U at the given E_F.  mu [R, n_max+1] complex.
    Returns (N, U, n(E_F)) [R] complex."""
    R = mu.shape[0]
    na, nb = n_a(n_max), n_b(n_max)
    m = mu / mu[:, :1]
    a = np.zeros((R, na), complex)
    b = np.zeros((R, nb + 1), complex)
    var = (m[:, 2] - m[:, 1] ** 2).real if n_max >= 2 else np.zeros(R)
    for r in range(R):
        cprev = np.zeros(n_max + 2, complex)
        ccur = np.zeros(n_max + 2, complex)
        ccur[0] = 1.0
        broke = False
        for n in range(na):
            if broke:
                a[r, n] = a[r, n - 1]
                continue
            idx = np.add.outer(np.arange(n + 1), np.arange(n + 1)) + 1
            a[r, n] = np.sum(np.outer(ccur[:n + 1], ccur[:n + 1]) * m[r][idx])
            if n + 1 > nb:
                break
            dv = np.zeros(n + 2, complex)
            dv[1:] += ccur[:n + 1]
            dv[:n + 1] -= a[r, n] * ccur[:n + 1] + b[r, n] * cprev[:n + 1]
            idx2 = np.add.outer(np.arange(n + 2), np.arange(n + 2))
            b2 = np.sum(np.outer(dv, dv) * m[r][idx2])
            if b2.real <= 1e-14 * var[r]:
                b[r, n + 1:] = 0.0
                broke = True
                continue
            b[r, n + 1] = np.sqrt(b2)
            cprev[:n + 2] = ccur[:n + 2]
            ccur[:n + 2] = dv / b[r, n + 1]
    # Gershgorin terminator (values decide the extremes)
    lo = np.zeros(R, complex)
    hi = np.zeros(R, complex)
    for n in range(na):
        bl = b[:, n] if 1 <= n <= nb else np.zeros(R)
        bh = b[:, n + 1] if n + 1 <= nb else np.zeros(R)
        e0, e1 = a[:, n] - bl - bh, a[:, n] + bl + bh
        if n == 0:
            lo, hi = e0.copy(), e1.copy()
        else:
            lo = np.where(e0.real < lo.real, e0, lo)
            hi = np.where(e1.real > hi.real, e1, hi)
    ai = 0.5 * (hi + lo)
    bi = 0.25 * (hi - lo)
    bi = np.where(bi.real < 1e-6, 1e-6 + 0j, bi)
    # expansion coefficients
    g = jackson(n_exp)
    M = n_max + 1
    p = np.zeros((M, M))
    p[0, 0] = 1.0
    if M > 1:
        p[1, 1] = 2.0
    for mm in range(1, M - 1):
        for n in range(mm + 2):
            p[mm + 1, n] = (2.0 * p[mm, n - 1] if n >= 1 else 0.0) - (p[mm - 1, n] if n <= mm - 1 else 0.0)
    from math import comb
    gs = np.zeros((R, n_exp + 1), complex)
    mh = np.zeros((R, M), complex)
    for n in range(M):
        s = sum(comb(n, l) * (-ai) ** l * m[:, n - l] for l in range(n + 1))
        mh[:, n] = s / (2.0 * bi) ** n
    n_mom = np.where(bi.real > 1e-6, n_max, 0)
    gs[:, 0] = 1.0
    for mm in range(min(n_max, n_exp) + 1):
        val = mh[:, :mm + 1] @ p[mm, :mm + 1]
        gs[:, mm] = np.where(mm <= n_mom, val, gs[:, mm])
    depth = n_exp + 3
    ah = np.zeros((R, depth), complex)
    bh = np.zeros((R, depth), complex)
    for k in range(depth):
        if k < na:
            ah[:, k] = (a[:, k] - ai) / (2.0 * bi)
        bh[:, k] = 0.0 if k == 0 else (b[:, k] / (2.0 * bi) if k <= nb else 0.5)
    z0 = np.zeros((R, depth), complex)
    z1 = np.zeros((R, depth), complex)
    z1[:, 0] = 1.0
    for mm in range(n_exp):
        zm = np.zeros_like(z1)
        zm[:, 1:] = z1[:, :-1]
        zp = np.zeros_like(z1)
        zp[:, :-1] = z1[:, 1:]
        bh1 = np.zeros_like(bh)
        bh1[:, :-1] = bh[:, 1:]
        z2 = 2.0 * (ah * z1 + bh * zm + bh1 * zp) - z0
        z0, z1 = z1, z2
        k = mm + 1
        gs[:, k] = np.where(k > n_mom, z1[:, 0], gs[:, k])
    gs = gs * g[None, :]
    # N, U and the DOS at E_F
    eps = (E_F - ai) / (2.0 * bi)
    inside = (eps.real > -1.0) & (eps.real < 1.0)
    c = np.where(inside, eps, np.where(eps.real <= -1.0, -1.0 + 0j, 1.0 + 0j))
    phi = np.arccos(c)

    def chi(k):
        if k == 0:
            return np.zeros(R, complex)
        if k == 1:
            return 1.0 - phi / np.pi + np.sin(2.0 * phi) / (2.0 * np.pi)
        return (np.sin((k + 1) * phi) / (k + 1) - np.sin((k - 1) * phi) / (k - 1)) / np.pi

    chis = [chi(k) for k in range(n_exp + 3)]
    N = sum(gs[:, k] * chis[k + 1] for k in range(n_exp + 1))
    U = bi * sum(gs[:, k] * (chis[k + 2] + chis[k]) for k in range(n_exp + 1)) + (ai - e_on) * N
    D = sum(gs[:, k] * np.sin((k + 1) * phi) for k in range(n_exp + 1))
    D = np.where(inside, D / (np.pi * bi), 0.0)
    return N, U, D


def weights(mu_rows, n_max, n_exp, E_F, e_on, h=1e-30):
    """w[r, n] = dU_total/dmu_(r,n) (both spins) at the self-determined Fermi
    level, by the complex step; also returns (dU/dmu, dN/dmu) per spin."""
    mu_rows = np.asarray(mu_rows, np.float64)
    R = mu_rows.shape[0]
    N0, U0, D0 = _tail_c(mu_rows.astype(complex), n_max, n_exp, E_F, e_on)
    dU = np.zeros((R, n_max + 1))
    dN = np.zeros((R, n_max + 1))
    for n in range(1, n_max + 1):
        muc = mu_rows.astype(complex)
        muc[:, n] += 1j * h
        Nc, Uc, _ = _tail_c(muc, n_max, n_exp, E_F, e_on)
        dU[:, n] = Uc.imag / h
        dN[:, n] = Nc.imag / h
    D = D0.real
    E_bar = float(np.sum(e_on * D) / np.sum(D))
    w = 2.0 * (dU - (E_F - E_bar) * dN)
    return w, dU, dN


def forces(wl, nl=None, n_max=None, n_exp=None):
    """Forces F [N, 3] (eV/A) on every atom from the bond energy of the
    non-magnetic d-band path, and the energy pipeline's result."""
    n_max = wl.n_max if n_max is None else n_max
    n_exp = wl.n_exp if n_exp is None else n_exp
    assert wl.model["n_orb"] == 5, "forces: d band only"
    if nl is None:
        nl = neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    r = energy_pipeline(wl, nl=nl, n_max=n_max, n_exp=n_exp)
    H_on, H_b = r["H_on"], r["H_bond"]
    n = wl.n_atoms
    no = 5
    rows = r["mu"].reshape(-1, n_max + 1)
    w, _, _ = weights(rows, n_max, n_exp, r["E_F"], H_on.reshape(-1))
    # dense folded H and Theta~
    H = np.diag(H_on.reshape(-1)).astype(np.float64)
    i_of = np.repeat(np.arange(n), np.diff(nl["row_ptr"]))
    for p in range(len(nl["nbr_j"])):
        i, j = i_of[p], nl["nbr_j"][p]
        H[no * i:no * i + no, no * j:no * j + no] += H_b[p]
    powers = [np.eye(n * no)]
    for l in range(1, n_max):
        powers.append(powers[-1] @ H)
    Theta = np.zeros_like(H)
    for l in range(n_max):
        Q = np.zeros_like(H)
        for lp in range(n_max - l):
            Q += w[:, l + lp + 1][:, None] * powers[lp]
        Theta += powers[l] @ Q
    # block derivatives by the complex step in each Cartesian direction
    spc = np.asarray(wl.species)
    dH = np.zeros((len(nl["nbr_j"]), 3, no, no))
    for c in range(3):
        d = nl["nbr_d"].astype(complex)
        d[:, c] += 1e-30j
        dH[:, c] = _dd_blocks(wl.model, spc, nl, d).imag / 1e-30
    F = np.zeros((n, 3))
    for p in range(len(nl["nbr_j"])):
        i, j = i_of[p], nl["nbr_j"][p]
        T = Theta[no * i:no * i + no, no * j:no * j + no]
        gp = np.einsum("ab,cab->c", T, dH[p])
        F[j] -= gp
        F[i] += gp
    # onsite elements Theta~_(ia,ia) = dU/dE_ia through the moments; with the
    # explicit -N_ia of the onsite reference they give the derivative of the
    # bond energy with respect to an onsite level, the self-consistency
    # target of Eq. BOP_SCF: Delta_ia = Theta~_(ia,ia) - N_ia
    r["theta_onsite"] = np.diag(Theta).reshape(n, no).copy()
    return F, r, w

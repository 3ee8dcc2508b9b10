"""The Lanczos form (bop_lanczos): recursion coefficients straight from the
H.X products, against the oracle's coefficients from the moments (App. B.3)
and its energies; FP32 and BF16 within stated bounds; breakdown on an
isolated atom; tiling invariance; SCF in FP32."""
import numpy as np
import pytest

import oracle as O
import workloads as W

from test_gpu_parity import STRUCTS, _np

pytestmark = pytest.mark.gpu


def _wl(name):
    pos, cell, spc, model, n_max = STRUCTS[name]
    n = pos.shape[0]
    nel = {"fcc_spd": np.where(spc == 0, 9.0, 8.0)}.get(name, np.full(n, 6.5))
    return W.Workload(name, pos, cell, spc, model, n_max, 200, nel)


def _run(bop, wl, dtype, tuning=None, E_F=None):
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, dtype, tuning=tuning,
                       method="lanczos")
    out = p.run(float(np.sum(wl.n_elec)), E_F=E_F)
    return p, out


# FP64: the moment route loses about 1e-16 times the condition number of the
# moments-to-coefficients map (up to ~1e5 at these orders); 1e-9 eV covers it.
@pytest.mark.parametrize("name", ["bcc_small", "fcc_spd", "bcc_alloy", "dimer", "hcp", "bcc_2cell"])
def test_lanczos_fp64_matches_oracle(bop, name):
    wl = _wl(name)
    ref = O.energy_pipeline(wl)
    p, out = _run(bop, wl, "f64")
    rec = p.rec
    np.testing.assert_allclose(_np(rec["a"]), ref["rec"]["a"], atol=1e-9)
    np.testing.assert_allclose(_np(rec["b"]), ref["rec"]["b"], atol=1e-9)
    np.testing.assert_allclose(_np(rec["a_inf"]), ref["rec"]["a_inf"], atol=1e-9)
    np.testing.assert_allclose(_np(rec["b_inf"]), ref["rec"]["b_inf"], atol=1e-9)
    assert np.array_equal(_np(rec["flags"]) & ~(4 | 16), ref["rec"]["flags"] & ~(4 | 16))
    assert abs(float(_np(out["E_F"])[0]) - ref["E_F"]) < 1e-8
    np.testing.assert_allclose(_np(out["N_atom"]), ref["N_atom"], atol=1e-8)
    np.testing.assert_allclose(_np(out["U_atom"]), ref["U_atom"], atol=1e-8)
    assert abs(float(_np(out["U_total"])[0]) - ref["U_total"]) < 1e-9 * abs(ref["U_total"])


# FP32 vectors: coefficients within 1e-5 eV, energies within 1e-5 relative.
@pytest.mark.parametrize("name", ["bcc_small", "fcc_spd", "bcc_alloy", "hcp"])
def test_lanczos_fp32(bop, name):
    wl = _wl(name)
    ref = O.energy_pipeline(wl)
    p, out = _run(bop, wl, "f32")
    np.testing.assert_allclose(_np(p.rec["a"]), ref["rec"]["a"], atol=1e-5)
    np.testing.assert_allclose(_np(p.rec["b"]), ref["rec"]["b"], atol=1e-5)
    u = float(_np(out["U_total"])[0])
    assert abs(u - ref["U_total"]) < 1e-5 * abs(ref["U_total"])
    np.testing.assert_allclose(_np(out["N_atom"]), ref["N_atom"], atol=1e-4)


# BF16 vectors and blocks on MFMA: the stated bound is 0.1 eV on a_n, b_n and
# 2e-3 relative on the total bond energy (unit roundoff 2^-9 per stored value).
@pytest.mark.parametrize("name", ["bcc_small", "bcc_alloy", "fcc_spd"])
def test_lanczos_bf16_bound(bop, name):
    wl = _wl(name)
    ref = O.energy_pipeline(wl)
    p, out = _run(bop, wl, "bf16")
    ea = np.max(np.abs(_np(p.rec["a"]) - ref["rec"]["a"]))
    eb = np.max(np.abs(_np(p.rec["b"]) - ref["rec"]["b"]))
    u = float(_np(out["U_total"])[0])
    eu = abs(u - ref["U_total"]) / abs(ref["U_total"])
    print(f"{name}: bf16 a {ea:.2e} b {eb:.2e} U rel {eu:.2e} ({abs(u - ref['U_total']) / wl.n_atoms * 1e3:.3f} meV/atom)")
    assert ea < 0.1 and eb < 0.1
    assert eu < 2e-3


def test_lanczos_isolated_atoms_break_down(bop):
    """Atoms without neighbours: b_1 = 0, the chain ends at level 1, a_n
    repeat the onsite level; same flags as the moment route."""
    pos = np.array([[1.0, 1.0, 1.0], [9.0, 9.0, 9.0]])
    cell = np.eye(3) * 20.0
    spc = np.array([0, 1], np.int32)
    wl = W.Workload("iso", pos, cell, spc, W.canonical_d_model(3.5, onsite_d=(0.0, 0.8)), 6, 200,
                    np.array([6.0, 5.0]))
    ref = O.energy_pipeline(wl)
    for method in ("moments", "lanczos"):
        p = bop.EnergyPath(pos, cell, spc, wl.model, 6, 200, "f64", method=method)
        out = p.run(11.0)
        assert np.array_equal(_np(p.rec["flags"]) & 0xff01, ref["rec"]["flags"] & 0xff01), method
        np.testing.assert_allclose(_np(p.rec["a"]), ref["rec"]["a"], atol=1e-12)
        np.testing.assert_allclose(_np(p.rec["b"]), ref["rec"]["b"], atol=1e-12)
        np.testing.assert_allclose(_np(out["N_atom"]), ref["N_atom"], atol=1e-9)


@pytest.mark.parametrize("tuning", [{"tile_atoms": 1}, {"tile_atoms": 7, "block_threads": 1024, "batch_tiles": 8,
                                                         "chunk_rows": 8}])
def test_lanczos_tilings(bop, tuning):
    wl = _wl("bcc_alloy")
    p0, _ = _run(bop, wl, "f64")
    p1, _ = _run(bop, wl, "f64", tuning=tuning)
    np.testing.assert_allclose(_np(p1.rec["a"]), _np(p0.rec["a"]), atol=1e-12)
    np.testing.assert_allclose(_np(p1.rec["b"]), _np(p0.rec["b"]), atol=1e-12)


def test_lanczos_high_order_spd_fp32(bop):
    """20 levels' worth of coefficients (n_max 20) on the s,p,d alloy, where
    FP32 moments are useless: FP32 Lanczos stays within 1e-4 eV of FP64
    Lanczos."""
    wl = W.fcc_alloy_spd(reps=3)
    wl.n_max = 20
    p64, o64 = _run(bop, wl, "f64")
    p32, o32 = _run(bop, wl, "f32")
    np.testing.assert_allclose(_np(p32.rec["a"]), _np(p64.rec["a"]), atol=1e-4)
    np.testing.assert_allclose(_np(p32.rec["b"]), _np(p64.rec["b"]), atol=1e-4)
    du = abs(float(_np(o32["U_total"])[0]) - float(_np(o64["U_total"])[0])) / wl.n_atoms
    assert du < 1e-5


def test_lanczos_high_order_spd_bf16_bound(bop):
    """BF16 at the precision workload's order: 20 moments on the s,p,d alloy
    (108 atoms), against the oracle.  Bound: each level's coefficients take
    the BF16 rounding (2^-9) of blocks and vectors of spectral radius ~20 eV,
    about 0.04 eV, and the ten levels accumulate it: 0.5 eV on a_n, b_n; the
    bond energy keeps the BF16 form's 2e-3 relative.  The per-atom energy
    error is reported, not bounded by 1 meV (BF16 s-s hoppings of ~5 eV carry
    about 1e-2 eV of rounding each)."""
    wl = W.fcc_alloy_spd(reps=3)
    wl.n_max = 20
    ref = O.energy_pipeline(wl)
    p, out = _run(bop, wl, "bf16")
    ea = np.max(np.abs(_np(p.rec["a"]) - ref["rec"]["a"]))
    eb = np.max(np.abs(_np(p.rec["b"]) - ref["rec"]["b"]))
    u = float(_np(out["U_total"])[0])
    eu = abs(u - ref["U_total"]) / abs(ref["U_total"])
    print(f"s,p,d 20 moments: bf16 a {ea:.2e} b {eb:.2e} U rel {eu:.2e} "
          f"({abs(u - ref['U_total']) / wl.n_atoms * 1e3:.3f} meV/atom)")
    assert ea < 0.5 and eb < 0.5
    assert eu < 2e-3


def test_lanczos_scf_fp32_matches_oracle(bop):
    from test_gpu_scf import _alloy
    wl = _alloy()
    shift_ref, hist_ref, r_ref = O.scf(wl, mix=0.5, tol=1e-4, max_iter=100)
    s = bop.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, 200, "f32", method="lanczos")
    iters, hist = s.run_scf(mix=0.5, tol=1e-4, max_iter=100)
    assert abs(iters - len(hist_ref)) <= 1
    np.testing.assert_allclose(s.shift.cpu().numpy(), shift_ref, atol=1e-4)


# FP16 storage of the Lanczos vectors (FP32 H and arithmetic): unit roundoff
# 2^-11 per stored value times the spectral radius of these Hamiltonians
# (about 10 eV) bounds a_n, b_n by 5e-3 eV.  A coefficient error d moves the
# band by at most d, so U_ia by at most about N_ia d: 5e-3 relative in the
# worst case; errors of different levels and orbitals largely cancel, and U is
# held to 2e-4 relative (measured up to 1.1e-4 on the alloy: the fused level
# pass rebuilds H r_(j-1) from the stored y'_j, one more FP16 rounding per
# level than a separate update pass, which measured 1.0e-4).
@pytest.mark.parametrize("name", ["bcc_small", "bcc_alloy", "fcc_spd", "hcp"])
def test_lanczos_fp16_storage_bound(bop, name):
    wl = _wl(name)
    ref = O.energy_pipeline(wl)
    p, out = _run(bop, wl, "f16")
    ea = np.max(np.abs(_np(p.rec["a"]) - ref["rec"]["a"]))
    eb = np.max(np.abs(_np(p.rec["b"]) - ref["rec"]["b"]))
    u = float(_np(out["U_total"])[0])
    eu = abs(u - ref["U_total"]) / abs(ref["U_total"])
    print(f"{name}: f16 a {ea:.2e} b {eb:.2e} U rel {eu:.2e} ({abs(u - ref['U_total']) / wl.n_atoms * 1e3:.4f} meV/atom)")
    assert ea < 5e-3 and eb < 5e-3
    assert eu < 2e-4


def test_moments_reject_fp16_storage(bop):
    wl = _wl("bcc_small")
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, 200, "f16", method="moments")
    with pytest.raises(bop.BopError) as e:
        p.run_moments()
    assert e.value.code == bop.BOP_E_UNSUPPORTED


# FP32 step kernels stage each row's H blocks in LDS unless the slice (waves x
# deg_max blocks) exceeds a workgroup's LDS; then they read them with scalar
# loads, as FP64 always does.  fcc s,p,d with three shells inside the cutoff
# (42 neighbours) at 1024 threads needs 16 x 42 x 81 x 4 B = 218 KB, more than
# any workgroup can hold, so this runs the scalar-load form in FP32.
def test_fp32_wide_rows_read_h_with_scalar_loads(bop):
    rng = np.random.default_rng(33)
    pos, cell = W.cubic_lattice("fcc", 3.5355, 3)
    spc = W.random_species(108, [54, 54], rng)
    model = W.spd_alloy_model(r_cut=4.5)
    wl = W.Workload("fcc_spd_3shell", W.displace(pos, cell, 0.04, rng), cell, spc, model, 6, 200,
                    np.where(spc == 0, 9.0, 8.0))
    ref_nl = O.neighbours(wl.pos, wl.cell, model["r_cut"])
    assert np.diff(ref_nl["row_ptr"]).max() >= 40
    ref = O.energy_pipeline(wl)
    wide = {"block_threads": 1024}
    p, out = _run(bop, wl, "f32", tuning=wide)
    np.testing.assert_allclose(_np(p.rec["a"]), ref["rec"]["a"], atol=1e-5)
    np.testing.assert_allclose(_np(p.rec["b"]), ref["rec"]["b"], atol=1e-5)
    m = bop.EnergyPath(wl.pos, wl.cell, wl.species, model, wl.n_max, wl.n_exp, "f32", tuning=wide)
    m.run_moments()
    from test_gpu_parity import _mu_err
    assert _mu_err(_np(m.mu), O.moments(ref_nl, *O.build_H(model, spc, ref_nl), wl.n_max)) < 1e-5


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n_max", [2, 4])
def test_lanczos_breakdown_at_last_level(bop, dtype, n_max):
    """A dimer along z with onsite level e: each d orbital couples only to the
    same orbital of the other atom, so every chain spans two states: a_0 = a_1
    = e, b_1 = |hopping| and b_2 = 0 exactly.  For an even n_max the last
    level's b_K comes from the product pass's partial sums (|r|^2 = |y'|^2 -
    2a^2 + a^2 s^2 |r_prev|^2): n_max = 4 puts the breakdown on that level
    (every orbital flagged at level 2), n_max = 2 takes b_1 from it.  The
    oracle's moment route is used for a and b_1 only: at b_2 it stops at its
    rounding level (6e-8 on the weak delta bonds), which the closed form
    replaces."""
    e = 0.7
    d = W.dimer(2.6, direction=(0.0, 0.0, 1.0))
    wl = W.Workload("dimer_z", d.pos, d.cell, d.species, W.canonical_d_model(3.5, onsite_d=(e,)), n_max, 200,
                    d.n_elec)
    ref = O.energy_pipeline(wl)
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, n_max, wl.n_exp, dtype, method="lanczos")
    p.run(float(np.sum(wl.n_elec)))
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16": 0.1}[dtype]
    a, b, fl = _np(p.rec["a"]), _np(p.rec["b"]), _np(p.rec["flags"])
    np.testing.assert_allclose(a, e, atol=tol)
    np.testing.assert_allclose(b[:, 1], ref["rec"]["b"][:, 1], atol=tol)
    assert np.all(b[:, 1] > 0.1)
    if n_max == 4:
        assert np.all(b[:, 2] == 0.0)
        assert np.all((fl & 0xff01) == 0x201)
    else:
        assert np.all((fl & 0xff01) == 0)

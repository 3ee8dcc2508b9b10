"""Terminator and band-width options (App. B.5 options i-v, vii, viii; App. B.1
Eq. weighted) and Broyden mixing of the charge-neutrality cycle (Sec. II
"Self-consistency"), through the C ABI against the oracle.  FP64: 1e-10."""
import numpy as np
import pytest

import oracle as O
import workloads as W

from test_gpu_parity import STRUCTS, _np

pytestmark = pytest.mark.gpu

MODES = ["lowest", "highest", "average", "average_highest", "minmax", "weighted"]


def _wl(name):
    pos, cell, spc, model, n_max = STRUCTS[name]
    n_elec = np.full(len(spc), 6.5 if model["n_orb"] == 5 else 8.5)
    return W.Workload(name, pos, cell, spc, model, n_max, 200, n_elec)


@pytest.mark.parametrize("name", ["bcc_small", "fcc_spd", "hcp", "dimer"])
@pytest.mark.parametrize("bw", MODES)
def test_band_options_match_oracle(bop, name, bw):
    """Terminator, Fermi level and energies with each estimate: moments route
    (FP64) against the oracle at 1e-10 (a_inf, b_inf, E_F in eV; N and U
    relative); the Lanczos route's a_inf, b_inf at 1e-9 eV (its coefficients
    carry 1e-10 eV of rounding, which the averages pass on)."""
    wl = _wl(name)
    ref = O.energy_pipeline(wl, bw=bw, beta=1.5)
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64", bw=bw, beta=1.5)
    out = p.run(float(np.sum(wl.n_elec)))
    np.testing.assert_allclose(_np(p.rec["a_inf"]), ref["rec"]["a_inf"], atol=1e-10)
    np.testing.assert_allclose(_np(p.rec["b_inf"]), ref["rec"]["b_inf"], atol=1e-10)
    fl = _np(p.rec["flags"])
    assert np.array_equal(fl & ~20, ref["rec"]["flags"] & ~20)
    # an estimate narrower than the band (e.g. b_1 alone) leaves states far
    # outside [a_inf - 2 b_inf, a_inf + 2 b_inf]: the expansion diverges; such
    # rows are flagged (|g_m sigma_m| > 1e4 in the oracle's coefficients) and
    # their energies have no meaning to compare
    div = np.max(np.abs(ref["gsig"]), axis=1) > 1e4
    assert np.array_equal((fl & 16) != 0, div)
    if not div.any():
        assert abs(float(_np(out["E_F"])[0]) - ref["E_F"]) < 1e-10
        np.testing.assert_allclose(_np(out["N_atom"]), ref["N_atom"], rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(_np(out["U_atom"]), ref["U_atom"], rtol=1e-10, atol=1e-10)
    pl = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64", method="lanczos",
                        bw=bw, beta=1.5)
    pl.run(float(np.sum(wl.n_elec)))
    np.testing.assert_allclose(_np(pl.rec["a_inf"]), ref["rec"]["a_inf"], atol=1e-9)
    np.testing.assert_allclose(_np(pl.rec["b_inf"]), ref["rec"]["b_inf"], atol=1e-9)


def test_band_options_reject_bad_arguments(bop):
    import torch
    mu = torch.ones((4, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(bop.BopError):
        bop.recursion(mu, 9, bw="weighted", beta=-1.0)
    lib = bop.load()
    out = {k: torch.empty(4, dtype=torch.float64, device="cuda") for k in ("a_inf", "b_inf")}
    a = torch.empty((4, 5), dtype=torch.float64, device="cuda")
    b = torch.empty((4, 5), dtype=torch.float64, device="cuda")
    fl = torch.empty(4, dtype=torch.int32, device="cuda")
    rc = lib.bop_recursion(4, 9, bop._ptr(mu), 8, 0.0, 0.0, bop._ptr(a), bop._ptr(b), bop._ptr(out["a_inf"]),
                           bop._ptr(out["b_inf"]), bop._ptr(fl), bop._stream())
    assert rc == bop.BOP_E_ARG


def _alloy54():
    rng = np.random.default_rng(5)
    pos, cell = W.cubic_lattice("bcc", 2.87, 3)
    spc = W.random_species(54, [27, 27], rng)
    return W.Workload("a54", W.wrap(pos, cell), cell, spc, W.canonical_d_model(3.5, onsite_d=(0.0, 0.8)),
                      8, 200, np.where(spc == 0, 6.0, 5.0))


@pytest.mark.parametrize("hist", [20, 3])
def test_broyden_scf_matches_oracle(bop, hist):
    """Broyden cycle (FP64) against the oracle's: the same number of
    iterations and the same shifts at every checked point (1e-9 eV); hist = 3
    exercises the restarts."""
    wl = _alloy54()
    shift_ref, hist_ref, r_ref = O.scf_broyden(wl, mix=0.5, tol=1e-4, max_iter=100, hist=hist)
    s = bop.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, "f64",
                    mixer="broyden", hist=hist)
    it, h = s.run_scf(mix=0.5, tol=1e-4, max_iter=100)
    assert it == len(hist_ref), (it, len(hist_ref))
    np.testing.assert_allclose(h, [x["max_dq"] for x in hist_ref], rtol=1e-6, atol=1e-10)
    np.testing.assert_allclose(_np(s.shift), shift_ref, atol=1e-9)
    assert abs(float(_np(s.out["U_total"])[0]) - r_ref["U_total"]) < 1e-9 * abs(r_ref["U_total"])


def test_broyden_beats_linear_on_large_alloy(bop):
    """250,000-atom alloy (16 moments, FP64): Broyden reaches max|q| < 1e-4 in
    fewer iterations than linear mixing, at the same energy (1e-3 meV/atom)."""
    wl = W.bcc_alloy_scf()
    lin = bop.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, "f64")
    it_l, _ = lin.run_scf(tol=1e-4, max_iter=100)
    u_l = float(_np(lin.out["U_total"])[0])
    del lin
    bro = bop.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, "f64",
                      mixer="broyden")
    it_b, _ = bro.run_scf(tol=1e-4, max_iter=100)
    u_b = float(_np(bro.out["U_total"])[0])
    print(f"linear {it_l} iterations, Broyden {it_b}; dU {abs(u_b - u_l) / wl.n_atoms * 1e3:.2e} meV/atom")
    assert it_b < it_l
    assert abs(u_b - u_l) / wl.n_atoms * 1e3 < 1e-3


@pytest.mark.parametrize("name", ["bcc_small", "fcc_spd", "hcp", "bcc_alloy"])
def test_atom_averaged_mode_matches_oracle(bop, name):
    """Atom-averaged mode (one chain per atom from mu_i / n_orb, each standing
    for n_orb orbitals): averaged moments, coefficients, terminator, Fermi
    level and per-atom energies against the oracle's averaged path, FP64
    1e-10 (coefficients and levels in eV, N and U relative)."""
    wl = _wl(name)
    ref = O.energy_pipeline_avg(wl)
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
    p.run_moments()
    out = bop.energy_atom_averaged(p.mu, p.H_on, float(np.sum(wl.n_elec)), wl.n_max, wl.n_exp)
    mu = _np(out["mu_avg"])
    assert np.max(np.abs(mu - ref["mu_avg"]) / np.abs(ref["mu_avg"]).max(axis=1, keepdims=True)) < 1e-12
    np.testing.assert_allclose(_np(out["H_avg"]), ref["H_avg"], atol=1e-14)
    np.testing.assert_allclose(_np(out["rec"]["a"]), ref["rec"]["a"], atol=1e-10)
    np.testing.assert_allclose(_np(out["rec"]["b"]), ref["rec"]["b"], atol=1e-10)
    np.testing.assert_allclose(_np(out["rec"]["a_inf"]), ref["rec"]["a_inf"], atol=1e-10)
    np.testing.assert_allclose(_np(out["rec"]["b_inf"]), ref["rec"]["b_inf"], atol=1e-10)
    assert abs(float(_np(out["E_F"])[0]) - ref["E_F"]) < 1e-10
    np.testing.assert_allclose(_np(out["N_atom"]), ref["N_atom"], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(_np(out["U_atom"]), ref["U_atom"], rtol=1e-10, atol=1e-10)
    assert abs(float(_np(out["N_atom"]).sum()) - float(np.sum(wl.n_elec))) < 1e-8 * float(np.sum(wl.n_elec))

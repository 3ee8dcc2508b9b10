"""Parity at the benchmark sizes, in the configurations bench.py times.

The oracle cannot run whole 10^5-atom cells in a test, so each case computes
the oracle's own neighbour list and H for the full cell and its moments (and
recursion, expansion and energies at the GPU's Fermi level) for a seeded
sample of atoms, and compares them element by element with the GPU.  The
global quantities are checked through properties that hold at any size: the
Fermi level makes the total electron count equal N_e, and a converged
charge-neutrality cycle has every |N_i - N0_i| below the tolerance.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

from test_gpu_parity import _mu_err, _np

pytestmark = pytest.mark.gpu


def _sample(n, m, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=m, replace=False)).astype(np.int32)


# bcc 40^3, 128,000 atoms, 18 moments: the headline step (neighbours, H, plan,
# supports, H.X, FP64 tail) with the default tiling.  FP64: moments 1e-10,
# per-atom N and U at the GPU's E_F 1e-9 (electrons, eV).  FP32 H.X: moments
# 1e-5; the moments-to-coefficients map at 18 moments amplifies their FP32
# rounding (about 1e-7 relative) by the conditioning of the Hankel matrix, up
# to ~1e4, so per-atom N and U are held to 2e-3 (measured up to 6.6e-4), while
# the errors of different atoms cancel in the totals (1e-4 meV/atom).
@pytest.mark.parametrize("dtype,tol_mu,tol_e", [("f32", 1e-5, 2e-3), ("f64", 1e-10, 1e-9)])
def test_bcc_large_sampled_atoms(bop, dtype, tol_mu, tol_e):
    wl = W.bcc_large()
    ne = float(np.sum(wl.n_elec))
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, dtype)
    out = p.step(ne)
    E_F = float(_np(out["E_F"])[0])
    N = _np(out["N_atom"])
    assert abs(N.sum() - ne) < 1e-8 * ne
    sel = _sample(wl.n_atoms, 48, 101)
    ref = O.energy_pipeline(wl, sel=sel, E_F=E_F)
    assert _mu_err(_np(p.mu)[sel], ref["mu"]) < tol_mu
    np.testing.assert_allclose(N[sel], ref["N_atom"], atol=tol_e)
    np.testing.assert_allclose(_np(out["U_atom"])[sel], ref["U_atom"], atol=tol_e)


# bcc 40^3: the neighbour list of the headline cell (33 cell-list bins per
# axis, Hilbert-ordered fine grid) against the oracle's, bit for bit.
def test_bcc_large_neighbours_bit_exact(bop):
    import torch
    wl = W.bcc_large()
    pos = torch.as_tensor(wl.pos, device="cuda")
    nl = bop.build_neighbours(pos, wl.cell, wl.model["r_cut"])
    ref = O.neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    np.testing.assert_array_equal(_np(nl.row_ptr), ref["row_ptr"])
    np.testing.assert_array_equal(_np(nl.nbr_j), ref["nbr_j"])
    np.testing.assert_array_equal(_np(nl.nbr_shift), ref["nbr_shift"])
    assert np.array_equal(_np(nl.nbr_d).view(np.int64), np.ascontiguousarray(ref["nbr_d"]).view(np.int64))
    order = np.sort(_np(nl.order))
    np.testing.assert_array_equal(order, np.arange(wl.n_atoms))


# bcc 40^3, FP32 Lanczos form (the headline): per-atom N_i and U_i of 48
# sampled atoms against the oracle (FP64 moments -> recursion -> expansion) at
# the GPU's Fermi level, within 1e-5 relative.  The vectors stay orthonormal,
# so FP32 rounding enters a_n, b_n at about 6e-8 |H| per level instead of being
# amplified by the Hankel map of the moment route.
def test_bcc_large_lanczos_fp32_per_atom(bop):
    wl = W.bcc_large()
    ne = float(np.sum(wl.n_elec))
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f32", method="lanczos")
    out = p.step(ne)
    E_F = float(_np(out["E_F"])[0])
    N = _np(out["N_atom"])
    U = _np(out["U_atom"])
    assert abs(N.sum() - ne) < 1e-8 * ne
    sel = _sample(wl.n_atoms, 48, 105)
    ref = O.energy_pipeline(wl, sel=sel, E_F=E_F)
    eN = np.max(np.abs(N[sel] - ref["N_atom"]) / np.abs(ref["N_atom"]))
    eU = np.max(np.abs(U[sel] - ref["U_atom"]) / np.abs(ref["U_atom"]))
    print(f"FP32 Lanczos per-atom relative error: N {eN:.3e}, U {eU:.3e}")
    assert eN < 1e-5 and eU < 1e-5, (eN, eU)


# bcc 40^3, the 16-bit Lanczos forms on MFMA (packed rows, bench.py --dtype
# bf16 / f16): per-atom N_i and U_i of 48 sampled atoms against the oracle at
# the GPU's Fermi level.  Each level's coefficients take one rounding of the
# stored vectors (unit roundoff u = 2^-9 BF16, 2^-11 FP16) times |H|, and the
# per-atom energies move by about u relative: the bound is u (measured over
# every atom against the FP64 path: BF16 U 9.4e-4, N 2.6e-4; FP16 U 1.3e-4,
# N 3.8e-5).
@pytest.mark.parametrize("dtype,u", [("bf16", 2.0 ** -9), ("f16", 2.0 ** -11)])
def test_bcc_large_lanczos_16bit_per_atom(bop, dtype, u):
    wl = W.bcc_large()
    ne = float(np.sum(wl.n_elec))
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, dtype, method="lanczos")
    out = p.step(ne)
    E_F = float(_np(out["E_F"])[0])
    N = _np(out["N_atom"])
    U = _np(out["U_atom"])
    assert abs(N.sum() - ne) < 1e-8 * ne
    sel = _sample(wl.n_atoms, 48, 107)
    ref = O.energy_pipeline(wl, sel=sel, E_F=E_F)
    eN = np.max(np.abs(N[sel] - ref["N_atom"]) / np.abs(ref["N_atom"]))
    eU = np.max(np.abs(U[sel] - ref["U_atom"]) / np.abs(ref["U_atom"]))
    print(f"{dtype} Lanczos per-atom relative error: N {eN:.3e}, U {eU:.3e} (bound {u:.2e})")
    assert eN < u and eU < u, (eN, eU)


# fcc A/B s,p,d alloy 30^3, 108,000 atoms, 20 moments: the FP32 Lanczos form
# (the fastest form within 1 meV/atom) against the oracle's coefficients from
# FP64 moments.  The FP32 rounding of the vectors (6e-8 times |H| of up to
# ~15 eV, 1e-6 eV per level) grows as the chain loses orthogonality over its
# ten levels; the bound is 5e-4 eV (measured up to 1.3e-4 eV, on level 9 of an
# s orbital with |a| ~ 6 eV).  FP64 moments of the same atoms: 1e-10.
def test_spd_alloy_sampled_atoms(bop):
    wl = W.fcc_alloy_spd()
    sel = _sample(wl.n_atoms, 12, 202)
    nl = O.neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    H_on, H_b = O.build_H(wl.model, wl.species, nl)
    mu_ref = O.moments(nl, H_on, H_b, wl.n_max, sel)
    rec_ref = O.recursion(mu_ref.reshape(-1, wl.n_max + 1), wl.n_max)

    p64 = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
    p64.run_moments()
    assert _mu_err(_np(p64.mu)[sel], mu_ref) < 1e-10
    del p64

    p32 = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f32", method="lanczos")
    p32.run_moments()
    rows = (sel[:, None] * 9 + np.arange(9)[None, :]).ravel()
    np.testing.assert_allclose(_np(p32.rec["a"])[rows], rec_ref["a"], atol=5e-4)
    np.testing.assert_allclose(_np(p32.rec["b"])[rows], rec_ref["b"], atol=5e-4)


# 512 ragged structures, 517,928 atoms, 14 moments, FP32: the captured launch
# sequence bench.py replays, against the oracle on every atom of six seeded
# structures of at most 1,500 atoms (1e-5, the FP32 bar).
def test_batch_sampled_structures(bop):
    import torch
    from paper_1803_07491_amd.batch import BatchedMoments
    structs = [W.ragged_structure(s) for s in range(512)]
    model = W.canonical_d_model(3.6)
    b = BatchedMoments(structs, model, 14, "f32")
    b.capture()
    for _ in range(2):
        b.replay()
    torch.cuda.synchronize()
    small = [s for s in range(512) if structs[s].n_atoms <= 1500]
    pick = np.random.default_rng(303).choice(small, size=6, replace=False)
    for s in pick:
        wl = structs[s]
        nl = O.neighbours(wl.pos, wl.cell, model["r_cut"])
        ref = O.moments(nl, *O.build_H(model, wl.species, nl), 14)
        assert _mu_err(_np(b.structure_mu(int(s))), ref) < 1e-5, int(s)


# bcc A/B alloy 50^3, 250,000 atoms, 16 moments: the plain FP64 charge-
# neutrality cycle from zero shifts converges (every |q_i| < 1e-4), and at the
# converged shifts the oracle's N_i of sampled atoms match the GPU's (1e-9).
def test_scf_alloy_converges_and_matches_sampled_atoms(bop):
    wl = W.bcc_alloy_scf()
    s = bop.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, "f64")
    it, hist = s.run_scf(tol=1e-4, max_iter=60)
    N = _np(s.out["N_atom"])
    assert np.max(np.abs(N - wl.n_elec)) < 1e-4
    sel = _sample(wl.n_atoms, 32, 404)
    ref = O.energy_pipeline(wl, shift=_np(s.shift), sel=sel, E_F=float(_np(s.out["E_F"])[0]))
    np.testing.assert_allclose(N[sel], ref["N_atom"], atol=1e-9)

"""Collinear magnetism (two spin channels, one Fermi level, Stoner exchange)
through the C ABI against the oracle: energies at a given state of shifts and
moments (FP64 moments 1e-10; Lanczos form FP64 1e-9, FP32 1e-5 relative) and
the self-consistent Stoner / charge-neutrality cycle (same iteration count,
final moments and shifts 1e-9)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

from test_gpu_parity import STRUCTS, _np

pytestmark = pytest.mark.gpu


def _case(name):
    pos, cell, spc, model, n_max = STRUCTS[name]
    n = len(spc)
    rng = np.random.default_rng(31)
    n0 = np.full(n, 6.5 if model["n_orb"] == 5 else 8.5)
    stoner = [0.8, 0.5][: model["n_species"]]
    wl = W.Workload(name, pos, cell, spc, model, n_max, 200, n0)
    shift = rng.normal(scale=0.1, size=n)
    moment = 1.5 + rng.normal(scale=0.3, size=n)
    return wl, stoner, shift - shift.mean(), moment


@pytest.mark.parametrize("name", ["bcc_small", "fcc_spd", "bcc_alloy", "hcp"])
@pytest.mark.parametrize("method,dtype,tol", [("moments", "f64", 1e-10), ("lanczos", "f64", 1e-9),
                                              ("lanczos", "f32", 1e-5)])
def test_magnetic_energy_matches_oracle(bop, name, method, dtype, tol):
    wl, stoner, shift, moment = _case(name)
    if dtype == "f32" and wl.model["n_orb"] == 9:
        # s,p,d in FP32: the vectors' rounding (6e-8 times |H| ~ 15 eV per
        # level) leaves up to ~1e-4 eV in a_n, b_n of the s rows (the bound of
        # the full-size s,p,d test is 5e-4 eV), which moves an orbital's count
        # by its DOS at E_F times that: counts and energies within 5e-4
        tol = 5e-4
    ref = O.energy_pipeline_mag(wl, stoner, shift, moment, B_z=0.05)
    p = bop.MagneticPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, stoner, B_z=0.05,
                         dtype=dtype, method=method)
    p.set_state(shift, moment)
    out = p.energy()
    n = wl.n_atoms
    assert abs(float(_np(out["E_F"])[0]) - ref["E_F"]) < tol * max(1.0, abs(ref["E_F"]))
    N = _np(out["N_atom"]).reshape(2, n)
    U = _np(out["U_atom"]).reshape(2, n)
    print(f"{name} {method} {dtype}: N {np.max(np.abs(N - ref['N_spin']) / np.abs(ref['N_spin'])):.2e} "
          f"U {np.max(np.abs(U - ref['U_spin']) / np.abs(ref['U_spin'])):.2e} "
          f"m {np.max(np.abs(_np(p.m_out) - ref['moment'])):.2e} E_F {abs(float(_np(out['E_F'])[0]) - ref['E_F']):.2e}")
    np.testing.assert_allclose(N, ref["N_spin"], rtol=tol, atol=tol)
    np.testing.assert_allclose(U, ref["U_spin"], rtol=tol, atol=tol)
    np.testing.assert_allclose(_np(p.m_out), ref["moment"], atol=tol * 10)
    assert abs(float(_np(out["U_total"])[0]) - ref["U_bond"]) < tol * abs(ref["U_bond"])
    assert abs(float(_np(p.U_X)[0]) - ref["U_X"]) < tol * abs(ref["U_X"]) + tol
    if method == "moments":
        assert np.max(np.abs(_np(p.mu).reshape(ref["mu"].shape) - ref["mu"]) / np.abs(ref["mu"]).max()) < 1e-12


def test_spin_shifts_closed_form(bop):
    """Up: shift + B_z - I m / 2; down: shift - B_z + I m / 2, I per species."""
    import torch
    spc = np.array([0, 1, 1, 0], np.int32)
    sh = np.array([0.1, -0.2, 0.3, 0.0])
    m = np.array([2.0, -1.0, 0.5, 0.0])
    mag = bop.Magnetism()
    mag.stoner[0], mag.stoner[1], mag.B_z = 0.8, 0.4, 0.05
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    # the device arrays stay referenced until the kernel has run
    d_spc = torch.tensor(spc, dtype=torch.int32, device="cuda")
    d_sh = torch.tensor(sh, dtype=torch.float64, device="cuda")
    d_m = torch.tensor(m, dtype=torch.float64, device="cuda")
    rc = bop.load().bop_spin_shifts(4, bop._ptr(d_spc), bop.C.byref(mag), bop._ptr(d_sh), bop._ptr(d_m),
                                    bop._ptr(out), bop._stream())
    assert rc == 0
    torch.cuda.synchronize()
    I = np.array([0.8, 0.4, 0.4, 0.8])
    want = np.concatenate([sh + 0.05 - 0.5 * I * m, sh - 0.05 + 0.5 * I * m])
    np.testing.assert_allclose(out.cpu().numpy(), want, atol=1e-15)


def test_magnetic_scf_matches_oracle(bop):
    """16-atom bcc cell (8 moments; n_sigma(E_F) = 0.88 per eV there, so I =
    1.3 eV makes I n_sigma > 1, ferromagnetic): same iteration count as the
    oracle's cycle from m = 1 (34), final moments and shifts within 1e-9."""
    pos, cell = W.cubic_lattice("bcc", 2.87, 2)
    pos = W.displace(pos, cell, 0.05, np.random.default_rng(8))
    n = pos.shape[0]
    wl = W.Workload("fe16", pos, cell, np.zeros(n, np.int32), W.canonical_d_model(3.5), 8, 200, np.full(n, 6.5))
    sh_ref, m_ref, hist_ref, r_ref = O.scf_mag(wl, [1.3], 1.0, mix=0.5, mix_m=0.8, max_iter=200)
    p = bop.MagneticPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, [1.3])
    p.set_state(np.zeros(n), np.ones(n))
    it, hist = p.run_scf(mix=0.5, mix_m=0.8, max_iter=200)
    assert it == len(hist_ref), (it, len(hist_ref))
    np.testing.assert_allclose(_np(p.moment), m_ref, atol=1e-9)
    np.testing.assert_allclose(_np(p.shift), sh_ref, atol=1e-9)
    assert abs(float(_np(p.U_X)[0]) - r_ref["U_X"]) < 1e-9 * abs(r_ref["U_X"])
    assert np.mean(_np(p.moment)) > 1.0            # the ferromagnetic solution

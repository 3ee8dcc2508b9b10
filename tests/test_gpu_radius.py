"""Maximum path radius (Sec. III "Speed-ups" (iii)) through the C ABI against
the oracle, whose truncated moments are pinned by cluster matrix powers:
moments FP64 1e-10, Lanczos coefficients FP64 1e-9 and FP32 1e-5, energies."""
import numpy as np
import pytest

import oracle as O
import workloads as W

from test_gpu_parity import _mu_err, _np

pytestmark = pytest.mark.gpu


def _bcc6(alloy=False, reps=6):
    rng = np.random.default_rng(12)
    pos, cell = W.cubic_lattice("bcc", 2.87, reps)           # 432 atoms, L = 17.22 A (reps 6)
    pos = W.displace(pos, cell, 0.05, rng)
    n = len(pos)
    if alloy:
        spc = W.random_species(n, [n // 2, n - n // 2], rng)
        model = W.canonical_d_model(3.5, onsite_d=(0.0, 0.8))
        n0 = np.where(spc == 0, 6.0, 5.0)
    else:
        spc = np.zeros(n, np.int32)
        model = W.canonical_d_model(3.5)
        n0 = np.full(n, 6.5)
    return W.Workload("bcc6", pos, cell, spc, model, 9, 200, n0)


def _gap_ok(wl, r_max):
    """no atom within 0.05 A of r_max from any atom (the two sides' distances
    differ in rounding only)"""
    inv = np.linalg.inv(wl.cell)
    for i in range(0, wl.n_atoms, 7):
        f = (wl.pos - wl.pos[i]) @ inv
        f -= np.rint(f)
        dist = np.linalg.norm(f @ wl.cell, axis=1)
        assert np.min(np.abs(dist - r_max)) > 0.05


# r_max + r_cut must stay below half the cell height: 4.45 A on 6^3 cells
# (8.61 A), 5.35 A on 7^3 cells (10.05 A)
@pytest.mark.parametrize("r_max,reps", [(4.45, 6), (5.35, 7)])
@pytest.mark.parametrize("alloy", [False, True])
def test_radius_moments_and_energy_match_oracle(bop, r_max, reps, alloy):
    wl = _bcc6(alloy, reps)
    _gap_ok(wl, r_max)
    ref = O.energy_pipeline(wl, r_max=r_max)
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64", r_max=r_max)
    out = p.run(float(np.sum(wl.n_elec)))
    assert _mu_err(_np(p.mu), ref["mu"]) < 1e-10
    assert abs(float(_np(out["E_F"])[0]) - ref["E_F"]) < 1e-10
    # a cut cluster can leave states outside the estimated band: those rows'
    # expansions diverge (flagged where the oracle's |g_m sigma_m| > 1e4) and
    # their energies are compared only through the flag
    div = (np.max(np.abs(ref["gsig"]), axis=1) > 1e4).reshape(wl.n_atoms, -1)
    assert np.array_equal((_np(p.rec["flags"]).reshape(wl.n_atoms, -1) & 16) != 0, div)
    ok = ~div.any(axis=1)
    assert ok.sum() >= 150
    np.testing.assert_allclose(_np(out["U_atom"])[ok], ref["U_atom"][ok], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(_np(out["N_atom"])[ok], ref["N_atom"][ok], rtol=1e-10, atol=1e-10)
    full = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
    assert p.plan.rows_cap < full.plan.rows_cap          # smaller tile supports
    for dtype, tol in (("f64", 1e-9), ("f32", 1e-5)):
        pl = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, dtype, method="lanczos",
                            r_max=r_max)
        pl.run_moments()
        np.testing.assert_allclose(_np(pl.rec["a"]), ref["rec"]["a"], atol=tol)
        np.testing.assert_allclose(_np(pl.rec["b"]), ref["rec"]["b"], atol=tol)


def test_radius_beyond_reach_changes_nothing(bop):
    """4 moments reach two hops (at most 7 A): r_max = 7.5 A gives the
    untruncated moments (8^3 cells, half height 11.48 A)."""
    wl = _bcc6(reps=8)
    a = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, 4, 200, "f64", r_max=7.5)
    b = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, 4, 200, "f64")
    a.run_moments()
    b.run_moments()
    assert _mu_err(_np(a.mu), _np(b.mu)) < 1e-14


def test_radius_rejections(bop):
    wl = _bcc6()
    with pytest.raises(bop.BopError) as e:           # r_max + r_cut above half the cell height
        bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, 9, 200, "f64", r_max=6.0)
    assert e.value.code == bop.BOP_E_ARG
    with pytest.raises(bop.BopError) as e:
        bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, 9, 200, "bf16", r_max=4.45)
    assert e.value.code == bop.BOP_E_UNSUPPORTED

"""GPU local-charge-neutrality SCF (bop_scf_step) against the oracle's SCF
loop: same update rule, so the same iteration count and the same converged
shifts and energies."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _alloy(reps=(3, 3, 3), seed=5):
    rng = np.random.default_rng(seed)
    pos, cell = W.cubic_lattice("bcc", 2.87, reps)
    n = pos.shape[0]
    spc = W.random_species(n, [n // 2, n - n // 2], rng)
    return W.Workload("a", W.wrap(pos, cell), cell, spc, W.canonical_d_model(3.5, onsite_d=(0.0, 0.8)),
                      8, 200, np.where(spc == 0, 6.0, 5.0))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_scf_matches_oracle(bop, dtype):
    wl = _alloy()
    shift_ref, hist_ref, r_ref = O.scf(wl, mix=0.5, tol=1e-4, max_iter=100)
    s = bop.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, 200, dtype)
    iters, hist = s.run_scf(mix=0.5, tol=1e-4, max_iter=100)
    assert abs(iters - len(hist_ref)) <= (0 if dtype == "f64" else 2)
    tol = 1e-9 if dtype == "f64" else 1e-4
    np.testing.assert_allclose(s.shift.cpu().numpy(), shift_ref, atol=tol)
    np.testing.assert_allclose(s.out["U_atom"].cpu().numpy(), r_ref["U_atom"], atol=tol * 10)
    assert abs(float(s.shift.mean())) < 1e-12
    assert float(s.max_dq.item()) < 1e-4


def test_scf_iteration_cap_reports_not_converged(bop):
    wl = _alloy()
    s = bop.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, 200, "f64")
    with pytest.raises(bop.BopError) as e:
        s.run_scf(max_iter=1)
    assert e.value.code == bop.BOP_E_NOT_CONVERGED


def test_md_warm_start_matches_oracle(bop):
    """Sec. III "Speed-ups" (ii): along a seeded 4-step trajectory of the
    54-atom alloy, each cycle starts from the previous step's converged shifts.
    The GPU (FP64) and the oracle take the same number of iterations at every
    step and reach the same shifts (1e-9 eV), and the warm cycles need fewer
    iterations in total than cycles from zero shifts."""
    rng = np.random.default_rng(5)
    pos, cell = W.cubic_lattice("bcc", 2.87, 3)
    spc = W.random_species(54, [27, 27], rng)
    wl = W.Workload("a54", W.displace(pos, cell, 0.04, rng), cell, spc,
                    W.canonical_d_model(3.5, onsite_d=(0.0, 0.8)), 8, 200, np.where(spc == 0, 6.0, 5.0))
    traj = W.md_trajectory(wl, 4, step_sigma=0.03)
    s = bop.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, "f64")
    cold = bop.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, "f64")
    shift_ref = None
    warm_total = cold_total = 0
    for t, p in enumerate(traj):
        wt = W.Workload("a54", p, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, wl.n_elec)
        shift_ref, hist_ref, _ = O.scf(wt, shift0=shift_ref, mix=0.5, tol=1e-4, max_iter=100)
        if t > 0:
            s.set_positions(p)
            cold.set_positions(p)
        it, _ = s.run_scf(tol=1e-4, max_iter=100)
        assert it == len(hist_ref), (t, it, len(hist_ref))
        np.testing.assert_allclose(s.shift.cpu().numpy(), shift_ref, atol=1e-9)
        cold.set_shift(np.zeros(wl.n_atoms))
        it_c, _ = cold.run_scf(tol=1e-4, max_iter=100)
        warm_total += it
        cold_total += it_c
    assert warm_total < cold_total, (warm_total, cold_total)

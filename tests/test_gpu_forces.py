"""GPU forces of the d-band bond energy (weights, block derivatives, Theta~
passes and the force sum, through the C ABI) against the oracle's
(complex-step weights, dense Theta~, direction-cosine block derivatives),
which is pinned on the CPU by finite differences of its own energy.

Bars: FP64 forces within 1e-10 of max(1, max|F|) eV/A; FP32 vectors (weights
and block derivatives FP64) within 1e-5 of it.  Weights: every moment order's
column within 1e-9 of its largest entry (both sides exact derivatives; the
difference is the rounding of two moment computations carried through the
recursion, up to the Hankel conditioning of the 9-moment map, ~1e4)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _bcc54(sigma=0.05, n_max=8):
    rng = np.random.default_rng(14)
    pos, cell = W.cubic_lattice("bcc", 2.87, 3)
    if sigma:
        pos = W.displace(pos, cell, sigma, rng)
    return W.Workload("b54", pos, cell, np.zeros(54, np.int32), W.canonical_d_model(3.5), n_max, 200,
                      np.full(54, 6.5))


def _gpu_forces(bop, wl, dtype="f64"):
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
    out = p.forces(float(np.sum(wl.n_elec)))
    if dtype == "f64":
        return p, out, _np(out["F"])
    # FP32 vectors for the Theta~ passes; weights and derivatives from FP64
    H_on, H32 = bop.build_H(wl.model, p.species, p.nl, dtype="f32")
    plan = bop.moments_plan(p.n, 5, wl.n_max, "f32", p.nl)
    mws = bop.moments_prepare(plan, p.nl)
    F = bop.forces(plan, mws, p.nl, H_on, H32, p.dH, p.w)
    return p, out, _np(F)


@pytest.mark.parametrize("case", ["bcc54_n8", "bcc54_n5", "bcc128_n9"])
def test_weights_match_oracle(bop, case):
    wl = {"bcc54_n8": lambda: _bcc54(n_max=8), "bcc54_n5": lambda: _bcc54(n_max=5),
          "bcc128_n9": W.bcc_small}[case]()
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
    out = p.run(float(np.sum(wl.n_elec)))
    E_F = float(_np(out["E_F"])[0])
    w = _np(bop.weights(p.mu, p.H_on, out["E_F"], wl.n_max, wl.n_exp))
    ref = O.energy_pipeline(wl, E_F=E_F)
    w_ref, _, _ = O.weights(ref["mu"].reshape(-1, wl.n_max + 1), wl.n_max, wl.n_exp, E_F, ref["H_on"].reshape(-1))
    assert np.all(w[:, 0] == 0.0)
    for n in range(1, wl.n_max + 1):
        scale = np.abs(w_ref[:, n]).max()
        err = np.abs(w[:, n] - w_ref[:, n]).max()
        assert err <= 1e-9 * scale, (case, n, err, scale)


def test_bond_derivatives_match_oracle(bop):
    """dH/dd of every pair of a displaced bcc cell and of a dimer along z (the
    polar axis) against the complex step of the oracle's blocks (1e-12 of the
    largest entry)."""
    import torch
    for wl in (_bcc54(), W.dimer(direction=(0.0, 0.0, 1.0)), W.dimer(direction=(1.0, -2.0, 0.5))):
        pos = torch.as_tensor(wl.pos, device="cuda")
        sp = torch.as_tensor(wl.species, device="cuda")
        nl = bop.build_neighbours(pos, wl.cell, wl.model["r_cut"])
        dH = _np(bop.bond_derivatives(wl.model, sp, nl))
        onl = O.neighbours(wl.pos, wl.cell, wl.model["r_cut"])
        ref = np.zeros((len(onl["nbr_j"]), 3, 5, 5))
        for c in range(3):
            d = onl["nbr_d"].astype(complex)
            d[:, c] += 1e-30j
            ref[:, c] = O._dd_blocks(wl.model, np.asarray(wl.species), onl, d).imag / 1e-30
        idx = np.array([[min(a, b) * 5 - min(a, b) * (min(a, b) - 1) // 2 + abs(b - a) for b in range(5)]
                        for a in range(5)])
        got = dH[:, :, idx]
        np.testing.assert_array_equal(_np(nl.nbr_j), onl["nbr_j"])
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.all(dH[:, :, 15] == 0.0)


@pytest.mark.parametrize("case", ["bcc54_n8", "bcc54_n5", "bcc128_n9", "bcc54_n4"])
def test_forces_match_oracle_fp64(bop, case):
    """Displaced bcc cells: 54 atoms (four 12-atom tiles and a ragged one of 6)
    at 8, 5 and 4 moments, 128 atoms at 9."""
    wl = {"bcc54_n8": lambda: _bcc54(n_max=8), "bcc54_n5": lambda: _bcc54(n_max=5),
          "bcc128_n9": W.bcc_small, "bcc54_n4": lambda: _bcc54(n_max=4)}[case]()
    _, out, F = _gpu_forces(bop, wl)
    F_ref, _, _ = O.forces(wl)
    scale = max(1.0, np.abs(F_ref).max())
    err = np.abs(F - F_ref).max()
    print(f"{case}: max |F - F_ref| = {err:.3e} eV/A (max |F| {np.abs(F_ref).max():.3f})")
    assert err <= 1e-10 * scale, err
    assert np.abs(F.sum(axis=0)).max() <= 1e-10 * scale


def test_forces_fp32_vectors_match_oracle(bop):
    wl = _bcc54(n_max=8)
    _, _, F = _gpu_forces(bop, wl, "f32")
    F_ref, _, _ = O.forces(wl)
    scale = max(1.0, np.abs(F_ref).max())
    err = np.abs(F - F_ref).max()
    print(f"FP32 vectors: max |F - F_ref| = {err:.3e} eV/A")
    assert err <= 1e-5 * scale, err


def test_forces_perfect_lattice_and_polar_dimer(bop):
    """Every atom of the perfect bcc lattice is a centre of inversion (F = 0);
    with one moment nothing depends on the bonds (F = 0); a dimer along z
    (bonds on the polar axis, a recursion that breaks down) has equal and
    opposite forces along z, equal to the oracle's."""
    _, _, F = _gpu_forces(bop, _bcc54(sigma=0.0))
    assert np.abs(F).max() < 1e-10
    # one moment: mu_1 is the onsite level, which no bond changes
    _, _, F = _gpu_forces(bop, _bcc54(n_max=1))
    assert np.all(F == 0.0)
    wl = W.dimer(direction=(0.0, 0.0, 1.0))
    _, _, F = _gpu_forces(bop, wl)
    F_ref, _, _ = O.forces(wl)
    assert np.abs(F - F_ref).max() <= 1e-10 * max(1.0, np.abs(F_ref).max())
    assert np.abs(F[:, :2]).max() < 1e-12 and abs(F[0, 2] + F[1, 2]) < 1e-12


def _fullsize(bop):
    wl = W.bcc_large()
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
    out = p.forces(float(np.sum(wl.n_elec)))
    return wl, p, _np(out["F"])


def test_forces_fullsize_properties(bop):
    """bcc 40^3, 128,000 atoms, 18 moments (the bench cell), in the launch
    configuration bench.py times: the forces sum to zero (translation
    invariance, 1e-9 eV/A per component of the sum) and two sampled
    components match central differences of the FP64 energy path (h = 2e-3 A:
    truncation h^2 F'''/6 ~ 1e-5, rounding of U_total ~1e-10 eV / 4e-3 A;
    bound 5e-5 eV/A)."""
    wl, p, F = _fullsize(bop)
    ne = float(np.sum(wl.n_elec))
    assert np.isfinite(F).all()
    assert np.abs(F.sum(axis=0)).max() < 1e-9
    del p
    h = 2e-3
    rng = np.random.default_rng(31)
    for _ in range(2):
        k, c = int(rng.integers(wl.n_atoms)), int(rng.integers(3))
        u = []
        for sgn in (1.0, -1.0):
            pos = wl.pos.copy()
            pos[k, c] += sgn * h
            q = bop.EnergyPath(pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
            u.append(float(q.run(ne)["U_total"].item()))
            del q
        fd = -(u[0] - u[1]) / (2 * h)
        print(f"atom {k} component {c}: F {F[k, c]:.8f}, central difference {fd:.8f}")
        assert abs(F[k, c] - fd) < 5e-5, (k, c, F[k, c], fd)


# FP32 vectors in the Theta~ passes against the FP64 forces at 128,000 atoms.
# Theta~ = sum_n w_n dmu_n/dH inherits the conditioning of the moment route
# (the weights carry the Hankel map's derivatives), so FP32 rounding of the
# vectors grows with n_max and with the number of columns reaching a bond:
# at 8 moments the 1e-5 bar holds (measured 7.2e-6 eV/A at max|F| 10.3); at
# the bench's 18 moments the bound is 1e-3 of max|F| (measured 5.5e-3 eV/A
# at max|F| 9.7, about the same for every atom, none of them flagged).  The
# rounding of the FP32 blocks alone accounts for 3e-6 eV/A of it.
@pytest.mark.parametrize("n_max,bound", [(8, 1e-5), (18, 1e-3)])
def test_forces_fullsize_fp32_vectors(bop, n_max, bound):
    wl = W.bcc_large()
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, n_max, wl.n_exp, "f64")
    F = _np(p.forces(float(np.sum(wl.n_elec)))["F"])
    H_on, H32 = bop.build_H(wl.model, p.species, p.nl, dtype="f32")
    plan = bop.moments_plan(p.n, 5, n_max, "f32", p.nl)
    mws = bop.moments_prepare(plan, p.nl)
    F32 = _np(bop.forces(plan, mws, p.nl, H_on, H32, p.dH, p.w))
    e32 = np.abs(F32 - F).max()
    print(f"FP32 vectors vs FP64, 128,000 atoms, {n_max} moments: {e32:.3e} eV/A (max |F| {np.abs(F).max():.3f})")
    assert e32 <= bound * max(1.0, np.abs(F).max())


def test_forces_batches_and_rejections(bop):
    """The force passes over several tile batches (batch of 8 tiles: 11 tiles
    of bcc 4^3 in two batches) give the same forces as one batch, to rounding
    of the atomic sums; unsupported inputs are rejected with
    BOP_E_UNSUPPORTED before anything runs: an s,p,d model, BF16 vectors, a
    path radius, more than 20 moments."""
    import torch
    wl = W.bcc_small()
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
    F1 = _np(p.forces(float(np.sum(wl.n_elec)))["F"])
    F8 = _np(bop.forces(p.plan, p.mws, p.nl, p.H_on, p.H_bond, p.dH, p.w, batch_tiles=8))
    assert p.plan.n_tiles > 8
    assert np.abs(F8 - F1).max() < 1e-12
    # BF16 plan
    _, Hb = bop.build_H(wl.model, p.species, p.nl, dtype="bf16")
    plan_b = bop.moments_plan(p.n, 5, wl.n_max, "bf16", p.nl)
    mws_b = bop.moments_prepare(plan_b, p.nl)
    with pytest.raises(bop.BopError) as e:
        bop.forces(plan_b, mws_b, p.nl, p.H_on, Hb, p.dH, p.w)
    assert e.value.code == bop.BOP_E_UNSUPPORTED
    # a plan with a path radius
    wl7 = W.bcc_large(reps=7)
    p7 = bop.EnergyPath(wl7.pos, wl7.cell, wl7.species, wl7.model, 6, wl7.n_exp, "f64", r_max=5.0)
    w7 = torch.zeros((p7.n * 5, 7), dtype=torch.float64, device="cuda")
    dH7 = bop.bond_derivatives(wl7.model, p7.species, p7.nl)
    with pytest.raises(bop.BopError) as e:
        bop.forces(p7.plan, p7.mws, p7.nl, p7.H_on, p7.H_bond, dH7, w7)
    assert e.value.code == bop.BOP_E_UNSUPPORTED
    # s,p,d model: the block derivatives are d-d only
    from test_gpu_parity import STRUCTS
    pos, cell, spc, model, _ = STRUCTS["fcc_spd"]
    sp = torch.as_tensor(spc, device="cuda")
    nl = bop.build_neighbours(torch.as_tensor(pos, device="cuda"), cell, model["r_cut"])
    with pytest.raises(bop.BopError) as e:
        bop.bond_derivatives(model, sp, nl)
    assert e.value.code == bop.BOP_E_UNSUPPORTED
    # weights beyond 20 moments
    mu = torch.ones((4, 22), dtype=torch.float64, device="cuda")
    with pytest.raises(bop.BopError) as e:
        bop.weights(mu, torch.zeros(4, dtype=torch.float64, device="cuda"),
                    torch.zeros(1, dtype=torch.float64, device="cuda"), 21, 200)
    assert e.value.code == bop.BOP_E_UNSUPPORTED


@pytest.mark.parametrize("case", ["bcc54_n8", "bcc54_n5", "bcc128_n9"])
def test_onsite_theta_and_scf_target_match_oracle(bop, case):
    """The onsite elements Theta~_(ia,ia) of the backward passes and the
    per-atom target of Eq. BOP_SCF (sum_a Theta~_(ia,ia) - N_i) against the
    oracle's dense Theta~ diagonal, within 1e-10 of max(1, max|Theta~|); the
    same values from two tile batches (batch of 8 tiles) to rounding of the
    atomic sums, and from FP32 vectors within 1e-5."""
    import torch
    wl = {"bcc54_n8": lambda: _bcc54(n_max=8), "bcc54_n5": lambda: _bcc54(n_max=5),
          "bcc128_n9": W.bcc_small}[case]()
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
    out = p.forces(float(np.sum(wl.n_elec)), scf_target=True)
    th, delta = _np(out["theta_on"]), _np(out["delta"])
    _, r, _ = O.forces(wl)
    th_ref = r["theta_onsite"]
    d_ref = th_ref.sum(axis=1) - r["N_atom"]
    scale = max(1.0, np.abs(th_ref).max())
    err = np.abs(th - th_ref).max()
    print(f"{case}: max |theta - theta_ref| = {err:.3e} (max |theta| {np.abs(th_ref).max():.3f}), "
          f"max |delta - delta_ref| = {np.abs(delta - d_ref).max():.3e}")
    assert err <= 1e-10 * scale, err
    assert np.abs(delta - d_ref).max() <= 1e-9 * scale
    th8 = torch.empty_like(out["theta_on"])
    bop.forces(p.plan, p.mws, p.nl, p.H_on, p.H_bond, p.dH, p.w, batch_tiles=8, theta_on=th8)
    assert np.abs(_np(th8) - th).max() < 1e-12 * scale
    H_on, H32 = bop.build_H(wl.model, p.species, p.nl, dtype="f32")
    plan = bop.moments_plan(p.n, 5, wl.n_max, "f32", p.nl)
    mws = bop.moments_prepare(plan, p.nl)
    th32 = torch.empty_like(out["theta_on"])
    bop.forces(plan, mws, p.nl, H_on, H32, p.dH, p.w, theta_on=th32)
    assert np.abs(_np(th32) - th_ref).max() <= 1e-5 * scale


def test_scf_target_fullsize_matches_energy_differences(bop):
    """bcc 40^3, 128,000 atoms, 18 moments: Delta_i = sum_a Theta~_(ia,ia) -
    N_i at two sampled atoms equals the central difference of the FP64 energy
    path in that atom's onsite shift, the Fermi level following (h = 1e-3 eV;
    rounding of U_total ~1e-10 eV / 2e-3 eV; bound 5e-5)."""
    import torch
    wl = W.bcc_large()
    ne = float(np.sum(wl.n_elec))
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
    out = p.forces(ne, scf_target=True)
    delta = _np(out["delta"])
    assert np.isfinite(delta).all()
    h = 1e-3
    rng = np.random.default_rng(37)
    for k in rng.integers(wl.n_atoms, size=2):
        u = []
        for sgn in (1.0, -1.0):
            s = torch.zeros(p.n, dtype=torch.float64, device="cuda")
            s[int(k)] = sgn * h
            p.rebuild(shift=s)
            u.append(float(p.run(ne)["U_total"].item()))
        fd = (u[0] - u[1]) / (2 * h)
        print(f"atom {k}: delta {delta[k]:.8f}, central difference {fd:.8f}")
        assert abs(delta[k] - fd) < 5e-5, (int(k), delta[k], fd)


_FCC = {}


def _fcc108():
    """fcc a = 3.6 A, 3^3 cells (108 atoms), sigma = 0.05 A (seed 21), the
    canonical d band with a 3.8 A cutoff (both first shells), 6 moments; the
    oracle's forces computed once."""
    if not _FCC:
        rng = np.random.default_rng(21)
        pos, cell = W.cubic_lattice("fcc", 3.6, 3)
        pos = W.displace(pos, cell, 0.05, rng)
        n = pos.shape[0]
        wl = W.Workload("fcc108", pos, cell, np.zeros(n, np.int32), W.canonical_d_model(3.8), 6, 200,
                        np.full(n, 6.5))
        _FCC["wl"] = wl
        _FCC["F"] = O.forces(wl)[0]
    return _FCC["wl"], _FCC["F"]


@pytest.mark.parametrize("dtype,bar", [("f64", 1e-10), ("f32", 1e-5)])
def test_forces_fcc_eighteen_neighbours_match_oracle(bop, dtype, bar):
    """fcc with the first two shells inside the cutoff (18 neighbours per
    atom): rows with more slot groups than the bcc cells, and (FP32 vectors)
    the L2 touches of the next group's blocks."""
    wl, F_ref = _fcc108()
    n = wl.n_atoms
    p, _, F = _gpu_forces(bop, wl, dtype)
    deg = np.diff(_np(p.nl.row_ptr))
    assert deg.min() == deg.max() == 18
    scale = max(1.0, np.abs(F_ref).max())
    err = np.abs(F - F_ref).max()
    print(f"fcc108 {dtype}: max |F - F_ref| = {err:.3e} eV/A (max |F| {np.abs(F_ref).max():.3f})")
    assert err <= bar * scale, err
    assert np.abs(F.sum(axis=0)).max() <= 1e-9 * max(1.0, np.abs(F).max() * n)


def test_weights_twenty_moments_from_the_oracle_moments(bop):
    """The weights kernel's deeper chain (n_max 19-20) against the oracle's
    weights from the same moments (the oracle's own), so that only the tail
    differs: moments to recursion, band, expansion, N and U at E_F in dual
    numbers against the complex step.  At 20 moments the map from moments is
    ill-conditioned, so the bar is 1e-6 of each column's largest entry; a
    wrong index in the chain would be an error of order one."""
    import torch
    wl = _bcc54(n_max=20)
    ref = O.energy_pipeline(wl)
    rows = ref["mu"].reshape(-1, 21)
    H_on = ref["H_on"].reshape(-1)
    mu = torch.as_tensor(np.ascontiguousarray(rows), dtype=torch.float64, device="cuda")
    H = torch.as_tensor(np.ascontiguousarray(ref["H_on"]), dtype=torch.float64, device="cuda")
    E_F = torch.tensor([ref["E_F"]], dtype=torch.float64, device="cuda")
    w = _np(bop.weights(mu, H, E_F, 20, wl.n_exp))
    w_ref, _, _ = O.weights(rows, 20, wl.n_exp, ref["E_F"], H_on)
    assert np.all(w[:, 0] == 0.0)
    worst = 0.0
    for n in range(1, 21):
        scale = np.abs(w_ref[:, n]).max()
        err = np.abs(w[:, n] - w_ref[:, n]).max()
        worst = max(worst, err / scale)
        assert err <= 1e-6 * scale, (n, err, scale)
    print(f"20 moments: largest column error {worst:.2e} of the column's largest entry")

"""Edge cases through the C ABI: empty input, the smallest and largest
moment orders, rejected sizes, the neighbour-capacity retry."""
import numpy as np
import pytest

import oracle as O
import workloads as W

from test_gpu_parity import STRUCTS, _np

pytestmark = pytest.mark.gpu


def test_empty_structure(bop):
    import torch
    pos = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    nl = bop.build_neighbours(pos, np.eye(3) * 10.0, 3.5)
    assert nl.n_pairs == 0
    assert int(nl.row_ptr.cpu()[0]) == 0
    sp = torch.zeros(0, dtype=torch.int32, device="cuda")
    m = W.canonical_d_model(3.5)
    H_on, H_bond = bop.build_H(m, sp, nl)
    plan = bop.moments_plan(0, 5, 8, "f64", nl)
    assert plan.n_tiles == 0
    mu = bop.moments(plan, nl, H_on, H_bond)
    assert mu.shape == (0, 5, 9)


@pytest.mark.parametrize("n_max", [1, 2, 3])
@pytest.mark.parametrize("method", ["moments", "lanczos"])
def test_lowest_orders(bop, n_max, method):
    pos, cell, spc, model, _ = STRUCTS["bcc_alloy"]
    wl = W.Workload("x", pos, cell, spc, model, n_max, 200, np.full(pos.shape[0], 6.5))
    ref = O.energy_pipeline(wl)
    p = bop.EnergyPath(pos, cell, spc, model, n_max, 200, "f64", method=method)
    out = p.run(float(wl.n_elec.sum()))
    np.testing.assert_allclose(_np(p.rec["a"]), ref["rec"]["a"], atol=1e-10)
    np.testing.assert_allclose(_np(p.rec["b"]), ref["rec"]["b"], atol=1e-10)
    np.testing.assert_allclose(_np(out["U_atom"]), ref["U_atom"], atol=1e-8)


def test_highest_order(bop):
    """n_max = 40 (the largest supported): FP64 moments of a small cell
    against the oracle, odd moments on the Cauchy-Schwarz scale."""
    from test_gpu_parity import _mu_err
    wl = W.bcc_small()
    nl = O.neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    H_on, H_b = O.build_H(wl.model, wl.species, nl)
    ref = O.moments(nl, H_on, H_b, 40)
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, 40, 200, "f64")
    p.run_moments()
    assert _mu_err(_np(p.mu), ref) < 1e-10


def test_unsupported_sizes_are_rejected(bop):
    wl = W.bcc_small()
    with pytest.raises(bop.BopError) as e:
        bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, 41, 200, "f64")
    assert e.value.code == bop.BOP_E_UNSUPPORTED
    # more than 64 neighbours in a row
    big = W.canonical_d_model(6.5)
    with pytest.raises(bop.BopError) as e:
        bop.EnergyPath(wl.pos, wl.cell, wl.species, big, 4, 200, "f64")
    assert e.value.code == bop.BOP_E_UNSUPPORTED


def test_neighbour_capacity_retry(bop):
    import torch
    wl = W.bcc_small()
    pos = torch.as_tensor(wl.pos, device="cuda")
    full = bop.build_neighbours(pos, wl.cell, wl.model["r_cut"])
    small = bop.build_neighbours(pos, wl.cell, wl.model["r_cut"], capacity=10)
    assert small.n_pairs == full.n_pairs
    assert torch.equal(small.nbr_j, full.nbr_j)
    assert torch.equal(small.row_ptr, full.row_ptr)


def test_recursion_register_and_generic_kernels(bop):
    """bop_recursion keeps its arrays in registers up to n_max = 20 and
    indexes them at run time above.  Level n uses only the moments up to
    2n + 1, so the coefficients that n_max = 20 and n_max = 21 share are the
    same arithmetic in the two kernels and must agree bit for bit; both are
    compared with the oracle's recursion on the same (oracle) moments."""
    import torch
    wl = W.bcc_small()
    nl = O.neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    H_on, H_b = O.build_H(wl.model, wl.species, nl)
    mu21 = O.moments(nl, H_on, H_b, 21).reshape(-1, 22)
    got = {}
    for n_max in (20, 21):
        mu = np.ascontiguousarray(mu21[:, :n_max + 1])
        got[n_max] = {k: _np(v) for k, v in bop.recursion(torch.as_tensor(mu, device="cuda"), n_max).items()}
        ref = O.recursion(mu, n_max)
        for k in ("a", "b"):
            err = np.max(np.abs(got[n_max][k] - ref[k]))
            assert err < 1e-9, (n_max, k, err)
        assert np.array_equal(got[n_max]["flags"] & 0xff, ref["flags"] & 0xff)
    assert np.array_equal(got[21]["a"][:, :10], got[20]["a"])
    assert np.array_equal(got[21]["b"][:, :11], got[20]["b"])


@pytest.mark.parametrize("search", [1, 2])
def test_plan_outgrown_by_neighbour_list(bop, search):
    """A plan made for one neighbour list and used with another whose rows
    have more neighbours than the plan's deg_max: the tiles that meet such a
    row get NaN moments (the documented failure), nothing is written past the
    planned rows, and the atoms of every other tile still match the oracle.
    Two 16-atom bcc blocks far apart (at most 11 neighbours) are the planned
    structure; the same blocks joined face to face (12 at the junction) the
    used one."""
    import torch
    a = 2.87
    blk, _ = W.cubic_lattice("bcc", a, 2)
    box = np.eye(3) * 40.0
    apart = np.vstack([blk + 2.0, blk + 20.0])
    joined = np.vstack([blk + 2.0, blk + 2.0 + np.array([2 * a, 0.0, 0.0])])
    m = W.canonical_d_model(3.5)
    spc = np.zeros(32, np.int32)
    species = torch.as_tensor(spc, device="cuda")
    nl_a = bop.build_neighbours(torch.as_tensor(apart, device="cuda"), box, 3.5)
    nl_b = bop.build_neighbours(torch.as_tensor(joined, device="cuda"), box, 3.5)
    plan = bop.moments_plan(32, 5, 6, "f64", nl_a, {"plan_search": search})
    deg_b = np.diff(_np(nl_b.row_ptr))
    assert plan.deg_max == 11 and deg_b.max() == 12
    H_on, H_b = bop.build_H(m, species, nl_b, dtype="f64")
    ws = bop.moments_prepare(plan, nl_b)
    mu = _np(bop.moments(plan, nl_b, H_on, H_b, ws=ws))
    bad = np.isnan(mu).all(axis=(1, 2))
    assert bad.any()
    assert np.isfinite(mu[~bad]).all()
    ref_nl = O.neighbours(joined, box, 3.5)
    ref = O.moments(ref_nl, *O.build_H(m, spc, ref_nl), 6)
    if (~bad).any():
        from test_gpu_parity import _mu_err
        assert _mu_err(mu[~bad], ref[~bad]) < 1e-10

"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.  Bars: neighbour lists bit-exact; FP64 moments and
energies within 1e-10 relative; FP32 moments within 1e-5 (scale-normalised
for odd moments, which can vanish)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


# position of entry (a, b) of a 5 x 5 symmetric block in the packed layout
_D_PACKED_INDEX = np.array([[min(a, b) * 5 - min(a, b) * (min(a, b) - 1) // 2 + abs(b - a)
                             for b in range(5)] for a in range(5)])


def _np(t):
    return t.detach().cpu().numpy()


def _mu_err(mu, ref):
    """max over rows/orders of |d mu_n| / scale_n.  Even moments are sums of
    squares (mu_2k = |X^k|^2 > 0): scale = mu_n (relative error).  Odd moments
    are merged path sums <X^(k-1), X^k> that can vanish; their natural scale is
    the Cauchy-Schwarz bound sqrt(mu_(n-1) mu_(n+1)), with mu_(n+1) for the top
    odd order extrapolated as mu_(n-1)^2 / mu_(n-3) (mu_2 when n = 1)."""
    mu = mu.reshape(-1, mu.shape[-1])
    ref = ref.reshape(-1, ref.shape[-1])
    nm = ref.shape[1] - 1
    scale = np.abs(ref).copy()
    for o in range(1, nm + 1, 2):
        lo = ref[:, o - 1]
        if o + 1 <= nm:
            hi = ref[:, o + 1]
        elif o >= 3:
            hi = lo * lo / np.maximum(ref[:, o - 3], 1e-300)
        else:
            hi = lo * np.maximum(ref[:, 2] if nm >= 2 else lo, 1e-300)
        scale[:, o] = np.sqrt(np.abs(lo * hi))
    scale = np.maximum(scale, 1e-300)
    return float(np.max(np.abs(mu - ref) / scale))


def _structures():
    rng = np.random.default_rng(21)
    out = {}
    wl = W.bcc_small()
    out["bcc_small"] = (wl.pos, wl.cell, wl.species, wl.model, 9)
    pos, cell = W.cubic_lattice("bcc", 2.87, 1)              # self images, all-pairs search
    out["bcc_1cell"] = (W.displace(pos, cell, 0.05, rng), cell, np.zeros(2, np.int32),
                        W.canonical_d_model(3.5, onsite_d=(0.3,)), 7)
    pos, cell = W.cubic_lattice("bcc", 2.87, 2)              # all-pairs search
    out["bcc_2cell"] = (W.displace(pos, cell, 0.05, rng), cell, np.zeros(16, np.int32),
                        W.canonical_d_model(3.5), 8)
    pos, cell = W.hcp_lattice(2.5529, (3, 2, 2))
    out["hcp"] = (W.displace(pos, cell, 0.05, rng), cell, np.zeros(pos.shape[0], np.int32),
                  W.canonical_d_model(3.6), 10)
    pos, cell = W.cubic_lattice("fcc", 3.5355, 3)
    spc = W.random_species(108, [54, 54], rng)
    out["fcc_spd"] = (W.displace(pos, cell, 0.06, rng), cell, spc, W.spd_alloy_model(), 9)
    pos, cell = W.cubic_lattice("bcc", 2.87, (5, 4, 3))     # 120 atoms: ragged last tile
    spc = W.random_species(120, [60, 60], rng)
    out["bcc_alloy"] = (W.displace(pos, cell, 0.05, rng), cell, spc,
                        W.canonical_d_model(3.5, onsite_d=(0.0, 0.8)), 12)
    wl = W.dimer(2.6, direction=(0.3, -0.5, 0.8))
    out["dimer"] = (wl.pos, wl.cell, wl.species, wl.model, 9)
    return out


STRUCTS = _structures()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


@pytest.mark.parametrize("name", sorted(STRUCTS))
def test_neighbours_bit_exact(bop, torch_mod, name):
    pos, cell, spc, model, _ = STRUCTS[name]
    ref = O.neighbours(pos, cell, model["r_cut"])
    nl = bop.build_neighbours(torch_mod.tensor(pos, device="cuda"), cell, model["r_cut"])
    assert np.array_equal(_np(nl.row_ptr), ref["row_ptr"])
    assert np.array_equal(_np(nl.nbr_j), ref["nbr_j"])
    assert np.array_equal(_np(nl.nbr_shift), ref["nbr_shift"])
    assert np.array_equal(_np(nl.nbr_d).view(np.uint64), ref["nbr_d"].view(np.uint64))
    order = np.sort(_np(nl.order))
    assert np.array_equal(order, np.arange(pos.shape[0]))


@pytest.mark.parametrize("name", sorted(STRUCTS))
def test_hamiltonian(bop, torch_mod, name):
    pos, cell, spc, model, _ = STRUCTS[name]
    ref_nl = O.neighbours(pos, cell, model["r_cut"])
    sh = np.linspace(-0.2, 0.3, pos.shape[0])
    Hon_r, Hb_r = O.build_H(model, spc, ref_nl, shift=sh)
    nl = bop.build_neighbours(torch_mod.tensor(pos, device="cuda"), cell, model["r_cut"])
    species = torch_mod.tensor(spc, dtype=torch_mod.int32, device="cuda")
    shift = torch_mod.tensor(sh, device="cuda")
    for dt, tol in (("f64", 1e-13), ("f32", 2e-7), ("bf16", 8e-3)):
        H_on, H_b = bop.build_H(model, species, nl, shift=shift, dtype=dt)
        np.testing.assert_allclose(_np(H_on), Hon_r, atol=1e-15)
        hb = _np(H_b.double())
        no = Hb_r.shape[1]
        if no == 5 and dt != "bf16":
            # packed symmetric d-d blocks: upper triangle row-major, then a zero
            assert hb.shape == (Hb_r.shape[0], 16)
            assert np.all(hb[:, 15] == 0.0)
            hb = hb[:, _D_PACKED_INDEX]
        err = np.abs(hb[:, :, :no] - Hb_r).max() / np.abs(Hb_r).max()
        assert err < tol, (dt, err)
        assert np.all(hb[:, :, no:] == 0.0)


def _gpu_moments(bop, torch_mod, pos, cell, spc, model, n_max, dtype="f64", tuning=None, use_order=True):
    nl = bop.build_neighbours(torch_mod.tensor(pos, device="cuda"), cell, model["r_cut"])
    species = torch_mod.tensor(spc, dtype=torch_mod.int32, device="cuda")
    H_on, H_b = bop.build_H(model, species, nl, dtype=dtype)
    plan = bop.moments_plan(pos.shape[0], model["n_orb"], n_max, dtype, nl, tuning, use_order=use_order)
    mu = bop.moments(plan, nl, H_on, H_b, use_order=use_order)
    torch_mod.cuda.synchronize()
    return mu, nl, H_on, H_b, plan


@pytest.mark.parametrize("name", sorted(STRUCTS))
def test_moments_fp64(bop, torch_mod, name):
    pos, cell, spc, model, n_max = STRUCTS[name]
    ref_nl = O.neighbours(pos, cell, model["r_cut"])
    ref = O.moments(ref_nl, *O.build_H(model, spc, ref_nl), n_max)
    mu, *_ = _gpu_moments(bop, torch_mod, pos, cell, spc, model, n_max)
    assert _mu_err(_np(mu), ref) < 1e-10


@pytest.mark.parametrize("tuning", [{"tile_atoms": 1}, {"tile_atoms": 5, "block_threads": 512},
                                    {"tile_atoms": 7, "block_threads": 1024, "batch_tiles": 8, "chunk_rows": 8},
                                    {"block_threads": 256, "batch_tiles": 8, "chunk_rows": 1}])
def test_moments_tilings(bop, torch_mod, tuning):
    pos, cell, spc, model, n_max = STRUCTS["bcc_alloy"]
    ref_nl = O.neighbours(pos, cell, model["r_cut"])
    ref = O.moments(ref_nl, *O.build_H(model, spc, ref_nl), n_max)
    for use_order in (True, False):
        mu, *_ = _gpu_moments(bop, torch_mod, pos, cell, spc, model, n_max, tuning=tuning, use_order=use_order)
        assert _mu_err(_np(mu), ref) < 1e-10


@pytest.mark.parametrize("name", ["bcc_small", "fcc_spd", "hcp"])
def test_moments_fp32(bop, torch_mod, name):
    pos, cell, spc, model, n_max = STRUCTS[name]
    ref_nl = O.neighbours(pos, cell, model["r_cut"])
    ref = O.moments(ref_nl, *O.build_H(model, spc, ref_nl), n_max)
    mu, *_ = _gpu_moments(bop, torch_mod, pos, cell, spc, model, n_max, dtype="f32")
    assert _mu_err(_np(mu), ref) < 1e-5


@pytest.mark.parametrize("name", ["bcc_small", "fcc_spd", "hcp", "bcc_alloy"])
def test_moments_bf16_mfma(bop, torch_mod, name):
    """BF16 H and X on MFMA with FP32 accumulation.  Stated bound: each step
    rounds X^k to BF16 (relative 2^-9) and multiplies by BF16 H, so the
    scale-normalised moment error grows about linearly with the order; 2e-2
    at n_max <= 12 covers it with margin (measured values are reported by
    the precision benchmark)."""
    pos, cell, spc, model, n_max = STRUCTS[name]
    ref_nl = O.neighbours(pos, cell, model["r_cut"])
    ref = O.moments(ref_nl, *O.build_H(model, spc, ref_nl), n_max)
    mu, *_ = _gpu_moments(bop, torch_mod, pos, cell, spc, model, n_max, dtype="bf16")
    m = _np(mu)
    assert np.all(np.isfinite(m))
    np.testing.assert_array_equal(m[..., 0], 1.0)
    assert _mu_err(m, ref) < 2e-2


def test_moments_deterministic(bop, torch_mod):
    pos, cell, spc, model, n_max = STRUCTS["bcc_alloy"]
    a, *_ = _gpu_moments(bop, torch_mod, pos, cell, spc, model, n_max, tuning={"batch_tiles": 8})
    b, *_ = _gpu_moments(bop, torch_mod, pos, cell, spc, model, n_max, tuning={"batch_tiles": 16})
    assert np.array_equal(_np(a).view(np.uint64), _np(b).view(np.uint64))


def test_dimer_closed_form_on_gpu(bop, torch_mod):
    pos, cell, spc, model, n_max = STRUCTS["dimer"]
    mu, *_ = _gpu_moments(bop, torch_mod, pos, cell, spc, model, n_max)
    f = (2.48 / 2.6) ** 5
    V = np.array([-1.0, 4 / 6, 4 / 6, -1 / 6, -1 / 6]) * f
    m = _np(mu)[0]
    for k in range(5):                      # traces are basis independent
        assert abs(m[:, 2 * k].sum() - np.sum(V ** (2 * k))) < 1e-13 * max(1.0, np.sum(V ** (2 * k)))
        assert np.max(np.abs(m[:, 2 * k + 1])) < 1e-15


@pytest.mark.parametrize("name", ["bcc_small", "fcc_spd", "bcc_alloy", "dimer", "hcp"])
def test_energy_path_fp64(bop, torch_mod, name):
    pos, cell, spc, model, n_max = STRUCTS[name]
    n = pos.shape[0]
    nel = {"fcc_spd": np.where(spc == 0, 9.0, 8.0)}.get(name, np.full(n, 6.5))
    wl = W.Workload(name, pos, cell, spc, model, n_max, 200, nel)
    ref = O.energy_pipeline(wl)
    path = bop.EnergyPath(pos, cell, spc, model, n_max, 200, "f64")
    out = path.run(float(nel.sum()))
    torch_mod.cuda.synchronize()
    rec = path.rec
    np.testing.assert_allclose(_np(rec["a"]), ref["rec"]["a"], atol=1e-10, rtol=1e-10)
    np.testing.assert_allclose(_np(rec["b"]), ref["rec"]["b"], atol=1e-10, rtol=1e-10)
    np.testing.assert_allclose(_np(rec["a_inf"]), ref["rec"]["a_inf"], atol=1e-10)
    np.testing.assert_allclose(_np(rec["b_inf"]), ref["rec"]["b_inf"], atol=1e-10)
    assert np.array_equal(_np(rec["flags"]) & ~(4 | 16), ref["rec"]["flags"] & ~(4 | 16))
    assert abs(float(_np(out["E_F"])[0]) - ref["E_F"]) < 1e-10 * max(1.0, abs(ref["E_F"]))
    np.testing.assert_allclose(_np(out["N_atom"]), ref["N_atom"], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(_np(out["U_atom"]), ref["U_atom"], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(_np(out["dos_atom"]), ref["dos_atom"], rtol=1e-9, atol=1e-9)
    assert abs(float(_np(out["U_total"])[0]) - ref["U_total"]) < 1e-10 * abs(ref["U_total"])


def test_energy_at_given_fermi_level(bop, torch_mod):
    pos, cell, spc, model, n_max = STRUCTS["bcc_alloy"]
    nel = np.full(pos.shape[0], 6.5)
    wl = W.Workload("x", pos, cell, spc, model, n_max, 200, nel)
    for ef in (-1.0, 0.4, 5.0):          # 5 eV: above every band (all full)
        ref = O.energy_pipeline(wl, E_F=ef, sel=np.arange(pos.shape[0], dtype=np.int32))
        path = bop.EnergyPath(pos, cell, spc, model, n_max, 200, "f64")
        out = path.run(float(nel.sum()), E_F=ef)
        np.testing.assert_allclose(_np(out["N_atom"]), ref["N_atom"], rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(_np(out["U_atom"]), ref["U_atom"], rtol=1e-10, atol=1e-10)


def test_divergent_expansion_is_flagged(bop, torch_mod):
    """A 2-atom cell with self images has a local DOS of a few sharp peaks;
    with 7 moments the terminated chain has states far outside the
    Gershgorin band, so sigma_m grows geometrically (in the oracle as well).
    The device flags such rows instead of returning silent garbage."""
    pos, cell, spc, model, n_max = STRUCTS["bcc_1cell"]
    path = bop.EnergyPath(pos, cell, spc, model, n_max, 200, "f64")
    path.run(13.0)
    fl = _np(path.rec["flags"])
    assert np.all(fl & bop.FLAG_DIVERGENT)
    ok = bop.EnergyPath(*STRUCTS["bcc_small"][:4], 9, 200, "f64")
    ok.run(6.5 * 128)
    assert not np.any(_np(ok.rec["flags"]) & bop.FLAG_DIVERGENT)


# The support search runs on bitmaps in LDS (structures up to 524,288 atoms)
# or on per-workgroup maps in memory, in the plan and in the prepare pass;
# both must give the same plan and the same supports, hence the same moments
# up to the order of the rows within a layer.
@pytest.mark.parametrize("name", ["bcc_small", "fcc_spd", "bcc_alloy", "bcc_1cell"])
def test_plan_searches_agree(bop, torch_mod, name):
    pos, cell, spc, model, n_max = STRUCTS[name]
    mus, plans = [], []
    for search in (1, 2, 1):
        mu, nl, H_on, H_b, plan = _gpu_moments(bop, torch_mod, pos, cell, spc, model, n_max,
                                               tuning={"plan_search": search})
        assert plan.search == search
        mus.append(_np(mu))
        plans.append((plan.rows_cap, list(plan.rows_k), plan.deg_max, plan.n_tiles, plan.ws_bytes))
    # the same supports; the bitmap search lists each layer in ascending atom
    # index, the map search in order of discovery, so the moments agree to
    # rounding, and each search is deterministic
    assert plans[0] == plans[1] == plans[2]
    assert _mu_err(mus[1], mus[0]) < 1e-13
    assert np.array_equal(mus[0], mus[2])


# The tile order follows a Hilbert curve over a grid a third of the cell-list
# width: a permutation, the same on every build, and compact.  Groups of 12
# consecutive atoms of a displaced bcc 20^3 cell (a = 3.16 A) span under 9.5 A
# on average (the cell-list order gives about 11 A).
def test_tile_order_is_compact_permutation(bop, torch_mod):
    rng = np.random.default_rng(55)
    pos, cell = W.cubic_lattice("bcc", 3.16, 20)
    pos = W.displace(pos, cell, 0.08, rng)
    t = torch_mod.as_tensor(pos, device="cuda")
    o1 = _np(bop.build_neighbours(t, cell, 3.8).order)
    o2 = _np(bop.build_neighbours(t, cell, 3.8).order)
    assert np.array_equal(np.sort(o1), np.arange(pos.shape[0]))
    assert np.array_equal(o1, o2)
    L = np.diag(cell)
    p = np.mod(pos, L)
    ext = []
    for g in range(0, pos.shape[0] // 12):
        q = p[o1[12 * g:12 * g + 12]]
        d = q[:, None] - q[None]
        d -= L * np.round(d / L)
        ext.append(np.sqrt((d ** 2).sum(-1)).max())
    assert np.mean(ext) < 9.5

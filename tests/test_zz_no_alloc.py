"""bop_energy_noalloc (the energy call whose workspace is the library's fixed
device array) against bop_energy with a caller workspace: same kernels, so the
outputs must agree bit for bit, on two calls in a row, the second with a
smaller structure, with the Fermi level found and given; oversized inputs are
rejected before anything is enqueued."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("E_F", "N_atom", "U_atom", "dos_atom", "U_total")


def _path(bop, wl, method):
    p = bop.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64", method=method)
    p.run_moments()
    if method == "lanczos":
        bop.terminator(p.rec, p.n_max)
        mu = None
    else:
        bop.recursion(p.mu, p.n_max, out=p.rec)
        mu = p.mu
    return p, mu


def _compare(bop, wl, method, E_F=None):
    import torch
    p, mu = _path(bop, wl, method)
    ne = float(np.sum(wl.n_elec))
    flags0 = p.rec["flags"].clone()
    ref = bop.energy(mu, p.rec, p.H_on, ne, p.n_max, p.n_exp, E_F=E_F)
    flags_ref = p.rec["flags"].clone()
    p.rec["flags"].copy_(flags0)
    got = bop.energy_noalloc(mu, p.rec, p.H_on, ne, p.n_max, p.n_exp, E_F=E_F)
    torch.cuda.synchronize()
    for k in KEYS:
        a, b = got[k].cpu().numpy(), ref[k].cpu().numpy()
        assert np.array_equal(a.view(np.int64), b.view(np.int64)), k
    assert torch.equal(p.rec["flags"], flags_ref)
    return ref


def test_noalloc_energy_matches_workspace_call_twice(bop):
    big = W.bcc_small()                                    # 128 atoms, 9 moments
    pos, cell = W.cubic_lattice("bcc", 2.87, 2)            # 16 atoms: the smaller second call
    rng = np.random.default_rng(5)
    small = W.Workload("bcc16", W.displace(pos, cell, 0.05, rng), cell, np.zeros(16, np.int32),
                       W.canonical_d_model(3.5), n_max=8, n_exp=200, n_elec=np.full(16, 6.5))
    r1 = _compare(bop, big, "moments")
    r2 = _compare(bop, small, "lanczos")
    assert small.n_atoms < big.n_atoms
    # given Fermi levels, again large then small
    _compare(bop, big, "moments", E_F=float(r1["E_F"].item()) + 0.05)
    _compare(bop, small, "lanczos", E_F=float(r2["E_F"].item()) - 0.05)


def test_noalloc_energy_rejects_oversized_input(bop):
    wl = W.bcc_small()
    p, mu = _path(bop, wl, "moments")
    lib = bop.load()
    import ctypes as C
    o = {k: p.mu.new_zeros(1) for k in KEYS}
    # 20,000 atoms x 5 orbitals x 201 coefficients x 8 bytes > 64 MiB: refused on
    # the host before anything is enqueued (the tensors are never read)
    rc = lib.bop_energy_noalloc(20000, 5, p.n_max, 200, bop._ptr(mu), bop._ptr(p.rec["a"]), bop._ptr(p.rec["b"]),
                                bop._ptr(p.rec["a_inf"]), bop._ptr(p.rec["b_inf"]), bop._ptr(p.H_on), 100.0, 0,
                                bop._ptr(o["E_F"]), bop._ptr(o["N_atom"]), bop._ptr(o["U_atom"]),
                                bop._ptr(o["dos_atom"]), bop._ptr(o["U_total"]), bop._ptr(p.rec["flags"]),
                                bop._stream())
    assert rc == bop.BOP_E_CAPACITY
    buf = C.create_string_buffer(512)
    lib.bop_last_error(buf, 512)
    assert b"64" in buf.value or b"fixed" in buf.value

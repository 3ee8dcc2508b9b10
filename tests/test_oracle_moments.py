"""Pins for the oracle's moments (CPU only): exact diagonalisation and matrix
powers of the folded Hamiltonian, explicit self-returning path sums, closed
forms for the lowest moments, and the bipartite and dimer special cases."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _dense(nl, H_on, H_b):
    n, no = H_on.shape
    H = np.zeros((n * no, n * no))
    for i in range(n):
        H[i * no:(i + 1) * no, i * no:(i + 1) * no] += np.diag(H_on[i])
        for p in range(nl["row_ptr"][i], nl["row_ptr"][i + 1]):
            j = nl["nbr_j"][p]
            H[i * no:(i + 1) * no, j * no:(j + 1) * no] += H_b[p]
    return H


def _scaled_err(mu, ref):
    s = np.sqrt(np.abs(ref[..., 2]) / ref[..., :1][..., 0])[..., None]
    n = np.arange(mu.shape[-1])
    return np.max(np.abs(mu - ref) / (ref[..., :1] * s ** n))


def _cases():
    rng = np.random.default_rng(2)
    out = {}
    wl = W.bcc_small()
    out["bcc_small"] = (wl.pos, wl.cell, wl.species, wl.model, 9)
    pos, cell = W.cubic_lattice("fcc", 3.5355, 2)
    pos = W.displace(pos, cell, 0.08, rng)
    spc = W.random_species(32, [16, 16], rng)
    out["fcc_spd"] = (pos, cell, spc, W.spd_alloy_model(), 8)
    pos, cell = W.cubic_lattice("bcc", 2.87, 1)          # self images
    out["bcc_tiny"] = (W.displace(pos, cell, 0.05, rng), cell, np.zeros(2, np.int32),
                       W.canonical_d_model(3.5, onsite_d=(0.3,)), 7)
    pos, cell = W.cubic_lattice("bcc", 2.87, 3)          # two species, onsite levels
    spc = W.random_species(54, [27, 27], rng)
    out["bcc_alloy"] = (W.displace(pos, cell, 0.05, rng), cell, spc,
                        W.canonical_d_model(3.5, onsite_d=(0.0, 0.8)), 10)
    return out


CASES = _cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_moments_vs_exact_diagonalisation(name):
    pos, cell, spc, model, n_max = CASES[name]
    nl = O.neighbours(pos, cell, model["r_cut"])
    H_on, H_b = O.build_H(model, spc, nl)
    mu = O.moments(nl, H_on, H_b, n_max)
    H = _dense(nl, H_on, H_b)
    w, V = np.linalg.eigh(H)
    ref = np.stack([(V ** 2) @ (w ** k) for k in range(n_max + 1)], -1).reshape(mu.shape)
    rho = np.abs(w).max()                  # error scale of both sides: |H|^n
    assert np.max(np.abs(mu - ref) / rho ** np.arange(n_max + 1)) < 1e-12
    # matrix powers, independent of eigh
    P = np.eye(H.shape[0])
    for k in range(n_max + 1):
        np.testing.assert_allclose(mu.reshape(-1, n_max + 1)[:, k], np.diag(P),
                                   atol=1e-11 * max(1.0, np.abs(np.diag(P)).max()))
        P = P @ H


def test_moments_explicit_path_sums():
    """Eq. (momDOS), second line: sum over every self-returning path
    i a -> j1 b1 -> ... -> i a, enumerated explicitly on a 2-atom cell."""
    pos, cell, spc, model, _ = CASES["bcc_tiny"]
    nl = O.neighbours(pos, cell, model["r_cut"])
    H_on, H_b = O.build_H(model, spc, nl)
    H = _dense(nl, H_on, H_b)
    mu = O.moments(nl, H_on, H_b, 4).reshape(-1, 5)
    D = H.shape[0]
    for n in range(1, 5):
        for ia in range(D):
            tot = 0.0
            for path in itertools.product(range(D), repeat=n - 1):
                seq = (ia,) + path + (ia,)
                term = 1.0
                for s in range(n):
                    term *= H[seq[s], seq[s + 1]]
                tot += term
            assert abs(tot - mu[ia, n]) < 1e-12 * max(1.0, abs(tot))


def test_lowest_moments_closed_forms():
    """mu0 = 1, mu1 = onsite level, and the per-atom trace of mu2 = sum of
    squared onsite levels + sum over bonds of |H_ij|_F^2, where for d-d bonds
    |H_ij|_F^2 = dds^2 + 2 ddp^2 + 2 ddd^2 from the distance alone."""
    pos, cell, spc, model, n_max = CASES["bcc_alloy"]
    nl = O.neighbours(pos, cell, model["r_cut"])
    H_on, H_b = O.build_H(model, spc, nl)
    mu = O.moments(nl, H_on, H_b, 4)
    np.testing.assert_array_equal(mu[..., 0], 1.0)
    np.testing.assert_allclose(mu[..., 1], H_on, atol=1e-14)
    for i in range(pos.shape[0]):
        tr = np.sum(H_on[i] ** 2)
        for p in range(nl["row_ptr"][i], nl["row_ptr"][i + 1]):
            f = (2.48 / np.linalg.norm(nl["nbr_d"][p])) ** 5
            tr += f * f * (1.0 + 2 * (4 / 6) ** 2 + 2 * (1 / 6) ** 2)
        assert abs(mu[i, :, 2].sum() - tr) < 1e-12


def test_bipartite_odd_moments_vanish():
    """bcc first shell only (cutoff 2.7 A at a = 2.87), zero onsite: the
    graph is bipartite so every odd moment is zero."""
    rng = np.random.default_rng(4)
    pos, cell = W.cubic_lattice("bcc", 2.87, 4)
    pos = W.displace(pos, cell, 0.01, rng)
    model = W.canonical_d_model(2.7)
    nl = O.neighbours(pos, cell, 2.7)
    assert np.all(np.diff(nl["row_ptr"]) == 8)
    H_on, H_b = O.build_H(model, np.zeros(128, np.int32), nl)
    mu = O.moments(nl, H_on, H_b, 11)
    scale = mu[..., 2:3] ** (np.arange(12) / 2.0)
    assert np.max(np.abs(mu[..., 1::2]) / scale[..., 1::2]) < 1e-14
    rec = O.recursion(mu.reshape(-1, 12), 11)
    assert np.max(np.abs(rec["a"])) < 1e-6 * np.max(rec["b"])


def test_dimer_moments():
    """Two d atoms: each bond-frame orbital pairs only with its partner, so
    mu_2k = V^2k (V = dds, ddp or ddd), odd moments vanish, b_1 = |V| and the
    chain breaks down at level 2."""
    wl = W.dimer(d=2.6, direction=(0.0, 0.0, 1.0))
    nl = O.neighbours(wl.pos, wl.cell, 3.5)
    H_on, H_b = O.build_H(wl.model, wl.species, nl)
    mu = O.moments(nl, H_on, H_b, 9)
    f = (2.48 / 2.6) ** 5
    V = np.array([-1.0, 4 / 6, 4 / 6, -1 / 6, -1 / 6]) * f
    for k in range(5):
        np.testing.assert_allclose(mu[0, :, 2 * k], V ** (2 * k), rtol=1e-13)
        np.testing.assert_allclose(mu[0, :, 2 * k + 1], 0.0, atol=1e-15)
    rec = O.recursion(mu[0], 9)
    np.testing.assert_allclose(rec["b"][:, 1], np.abs(V), rtol=1e-13)
    assert np.all(rec["flags"] & 1)
    assert np.all((rec["flags"] >> 8) == 2)


def _bcc6():
    rng = np.random.default_rng(12)
    pos, cell = W.cubic_lattice("bcc", 2.87, 6)              # 432 atoms, L = 17.22 A
    return W.displace(pos, cell, 0.05, rng), cell


def test_path_radius_large_and_tiny_limits():
    """A radius beyond every path's reach changes nothing (4 moments: two hops
    of at most 3.5 A each, r_max = 7.5 A); a radius below the nearest-neighbour
    distance leaves the start atom alone: mu_n = E^n."""
    pos, cell = _bcc6()
    model = W.canonical_d_model(3.5, onsite_d=(0.3,))
    spc = np.zeros(len(pos), np.int32)
    nl = O.neighbours(pos, cell, 3.5)
    H_on, H_b = O.build_H(model, spc, nl)
    sel = np.array([0, 17, 431], np.int32)
    full = O.moments(nl, H_on, H_b, 4, sel)
    np.testing.assert_allclose(O.moments(nl, H_on, H_b, 4, sel, r_max=7.5), full, rtol=1e-15, atol=1e-15)
    tiny = O.moments(nl, H_on, H_b, 6, sel, r_max=2.0)
    np.testing.assert_allclose(tiny, np.broadcast_to(0.3 ** np.arange(7), tiny.shape), rtol=1e-14)


def test_path_radius_matches_cluster_matrix_powers():
    """Brute force: the atoms within r_max of the start atom (minimum image)
    form a cluster; its dense Hamiltonian keeps the bonds whose target lies
    within r_max; the truncated moments are the diagonal of its matrix powers.
    r_max = 4.45 A sits in the gap between the third and fourth bcc shells
    (4.06 and 4.76 A, broadened by the displacements), asserted here."""
    pos, cell = _bcc6()
    model = W.canonical_d_model(3.5)
    spc = np.zeros(len(pos), np.int32)
    nl = O.neighbours(pos, cell, 3.5)
    H_on, H_b = O.build_H(model, spc, nl)
    r_max, n_max = 4.45, 9
    inv = np.linalg.inv(cell)
    for i in (0, 101, 250):
        d = pos - pos[i]
        f = d @ inv
        f -= np.rint(f)
        dist = np.linalg.norm(f @ cell, axis=1)
        assert np.min(np.abs(dist - r_max)) > 0.05
        inside = np.nonzero(dist <= r_max)[0]
        rel = (f @ cell)[inside]
        idx = {a: k for k, a in enumerate(inside)}
        Hc = np.zeros((5 * len(inside), 5 * len(inside)))
        for k, a in enumerate(inside):
            Hc[5 * k:5 * k + 5, 5 * k:5 * k + 5] = np.diag(H_on[a])
            for p in range(nl["row_ptr"][a], nl["row_ptr"][a + 1]):
                j = nl["nbr_j"][p]
                if j in idx and np.linalg.norm(rel[k] + nl["nbr_d"][p]) <= r_max:
                    kj = idx[j]
                    Hc[5 * k:5 * k + 5, 5 * kj:5 * kj + 5] += H_b[p]
        s = idx[i]
        want = np.array([[np.linalg.matrix_power(Hc, n)[5 * s + al, 5 * s + al] for n in range(n_max + 1)]
                         for al in range(5)])
        got = O.moments(nl, H_on, H_b, n_max, np.array([i], np.int32), r_max=r_max)[0]
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-13)
        full = O.moments(nl, H_on, H_b, n_max, np.array([i], np.int32))[0]
        assert np.max(np.abs(got - full)[:, 2::2] / full[:, 2::2]) > 1e-3    # the truncation does bite

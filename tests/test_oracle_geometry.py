"""Pins for the oracle's neighbour list, rotation matrices and Hamiltonian
blocks (CPU only).  Each check compares against something other than the
oracle's own formulas: brute-force enumeration, textbook Slater-Koster closed
forms, the rotation group itself, or invariances of the spectrum."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _numpy_pairs(pos, cell, rc, smax=3):
    """Brute force in NumPy over all (i, j) and all shifts in a box; the pair
    vector is formed in the same fixed order as the criterion defines."""
    out = []
    n = pos.shape[0]
    rng = range(-smax, smax + 1)
    for i in range(n):
        rows = []
        for j in range(n):
            for s1 in rng:
                for s2 in rng:
                    for s3 in rng:
                        sv = (s1 * cell[0] + s2 * cell[1]) + s3 * cell[2]
                        d = (pos[j] - pos[i]) + sv
                        r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
                        if 0.0 < r2 < rc * rc:
                            rows.append((j, s1, s2, s3, d[0], d[1], d[2]))
        rows.sort(key=lambda t: t[:4])
        out.append(rows)
    return out


@pytest.mark.parametrize("case", ["bcc1", "bcc2_tricl", "hcp"])
def test_neighbours_vs_numpy_bruteforce(case):
    rng = np.random.default_rng(7)
    if case == "bcc1":          # 2-atom cell smaller than the cutoff: self images
        pos, cell = W.cubic_lattice("bcc", 2.87, 1)
        pos = W.displace(pos, cell, 0.05, rng)
        rc = 3.5
    elif case == "bcc2_tricl":  # sheared cell
        pos, cell = W.cubic_lattice("bcc", 2.87, 2)
        cell = cell.copy()
        cell[1, 0] = 1.3
        cell[2, 1] = -0.7
        pos = W.displace(pos @ np.linalg.inv(np.diag([5.74] * 3)) @ cell, cell, 0.05, rng)
        rc = 3.5
    else:
        pos, cell = W.hcp_lattice(2.55, (2, 1, 1))
        pos = W.displace(pos, cell, 0.05, rng)
        rc = 3.6
    nl = O.neighbours(pos, cell, rc)
    ref = _numpy_pairs(pos, cell, rc)
    for i, rows in enumerate(ref):
        lo, hi = nl["row_ptr"][i], nl["row_ptr"][i + 1]
        assert hi - lo == len(rows)
        got = [(int(nl["nbr_j"][p]), *map(int, nl["nbr_shift"][p]), *nl["nbr_d"][p]) for p in range(lo, hi)]
        for g, r in zip(got, rows):
            assert g[:4] == r[:4]
            assert g[4:] == r[4:]          # bit-exact pair vectors


def test_neighbours_binned_equals_brute_and_counts():
    wl = W.bcc_small()
    a = O.neighbours(wl.pos, wl.cell, 3.5)
    b = O.neighbours(wl.pos, wl.cell, 3.5, brute=True)
    for k in a:
        assert np.array_equal(a[k], b[k])
    # bcc at a = 2.87: 8 first + 6 second neighbours inside 3.5 A
    assert np.all(np.diff(a["row_ptr"]) == 14)


def test_neighbours_reverse_pairs_exact():
    """Every (i, j, S) has (j, i, -S) with exactly the negated vector."""
    wl = W.bcc_small()
    nl = O.neighbours(wl.pos, wl.cell, 3.5)
    idx = {}
    for i in range(wl.n_atoms):
        for p in range(nl["row_ptr"][i], nl["row_ptr"][i + 1]):
            idx[(i, int(nl["nbr_j"][p]), *map(int, nl["nbr_shift"][p]))] = p
    for (i, j, s1, s2, s3), p in idx.items():
        q = idx[(j, i, -s1, -s2, -s3)]
        assert np.array_equal(nl["nbr_d"][q], -nl["nbr_d"][p])


# ---------------------------------------------------------------------------
def _frame(u):
    """Bond frame (x', y', z') = (theta-hat, phi-hat, u) built from the unit
    vector with trigonometry, independently of the oracle."""
    th = math.acos(max(-1.0, min(1.0, u[2])))
    ph = math.atan2(u[1], u[0]) if abs(u[2]) < 1 else 0.0
    xt = np.array([math.cos(th) * math.cos(ph), math.cos(th) * math.sin(ph), -math.sin(th)])
    yp = np.array([-math.sin(ph), math.cos(ph), 0.0])
    return np.stack([xt, yp, np.asarray(u)])


def _dquad():
    """Real d orbitals as symmetric traceless 3x3 quadratic forms, Frobenius
    normalised, order 3z^2-r^2, zx, yz, x^2-y^2, xy (x, y, z = 0, 1, 2)."""
    Q = np.zeros((5, 3, 3))
    Q[0] = np.diag([-1.0, -1.0, 2.0]) / math.sqrt(6.0)
    Q[1][0, 2] = Q[1][2, 0] = 1.0 / math.sqrt(2.0)
    Q[2][1, 2] = Q[2][2, 1] = 1.0 / math.sqrt(2.0)
    Q[3] = np.diag([1.0, -1.0, 0.0]) / math.sqrt(2.0)
    Q[4][0, 1] = Q[4][1, 0] = 1.0 / math.sqrt(2.0)
    return Q


def _random_dirs(n, seed=3):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return np.concatenate([v, [[0, 0, 1.0], [1.0, 0, 0], [0, 1.0, 0], [0, 0, -1.0]]])


def test_rotation_matrices_are_the_group_representation():
    Q = _dquad()
    for u in _random_dirs(40):
        Rp, Rd = O.rotation(u)
        F = _frame(u)                      # rows: x', y', z' in (x, y, z)
        # p: bond-frame p_z', p_x', p_y' expressed in global p_z, p_x, p_y
        order = [2, 0, 1]
        Fp = F[[2, 0, 1]][:, order]
        np.testing.assert_allclose(Rp, Fp, atol=1e-14)
        # d: rotate each quadratic form into the bond frame and project
        U = F.T                            # columns: bond axes in global coords
        M = np.array([[np.sum((U @ Q[a] @ U.T) * Q[b]) for b in range(5)] for a in range(5)])
        np.testing.assert_allclose(Rd, M, atol=1e-14)
        np.testing.assert_allclose(Rd @ Rd.T, np.eye(5), atol=1e-14)
    Rp, Rd = O.rotation(np.array([0.0, 0.0, 1.0]))
    np.testing.assert_array_equal(Rp, np.eye(3))
    np.testing.assert_array_equal(Rd, np.eye(5))


def _dimer_H(model, u, r, species=(0, 0)):
    pos = np.array([[10.0, 10.0, 10.0], [10.0, 10.0, 10.0]]) + np.array([[0, 0, 0], r * np.asarray(u)])
    cell = np.diag([40.0] * 3)
    nl = O.neighbours(pos, cell, model["r_cut"])
    H_on, H_b = O.build_H(model, np.array(species, np.int32), nl)
    return nl, H_on, H_b


def test_dd_blocks_textbook_closed_forms():
    """d-d block: the d_{3z'^2-r^2} combination along the bond is an
    eigenvector with eigenvalue dd-sigma (Slater-Koster), the spectrum is
    {sigma, pi, pi, delta, delta}, and |H|_F^2 = s^2 + 2 p^2 + 2 d^2."""
    model = W.canonical_d_model(3.5)
    for u in _random_dirs(20, seed=11):
        r = 2.6
        nl, H_on, H_b = _dimer_H(model, u, r)
        H = H_b[0]
        f = (2.48 / r) ** 5
        s, p, d = -f, 4.0 / 6.0 * f, -f / 6.0
        l, m, n = u
        v = np.array([(3 * n * n - 1) / 2, math.sqrt(3) * n * l, math.sqrt(3) * m * n,
                      math.sqrt(3) / 2 * (l * l - m * m), math.sqrt(3) * l * m])
        np.testing.assert_allclose(H @ v, s * v, atol=1e-13)
        np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(H)), np.sort([s, p, p, d, d]), atol=1e-13)
        assert abs(np.sum(H * H) - (s * s + 2 * p * p + 2 * d * d)) < 1e-13


def test_dd_blocks_are_symmetric():
    """Every d-d block is a symmetric matrix, H_ij[a][b] = H_ij[b][a] (the
    bond-frame block is diagonal, and its rotation R^T D R stays symmetric),
    also for an A-B pair of different species: the premise of storing d-d
    blocks as their upper triangle."""
    model = W.canonical_d_model(3.5, onsite_d=(0.0, 0.8))
    ab = {"dds": (W.FORM_EXP, -1.3, 2.5, 1.7), "ddp": (W.FORM_EXP, 0.7, 2.5, 1.7),
          "ddd": (W.FORM_EXP, -0.2, 2.5, 1.7)}
    model["bonds"][(0, 1)] = model["bonds"][(1, 0)] = ab
    model["bonds"][(1, 1)] = {k: (f, 0.9 * b, r0, q) for k, (f, b, r0, q) in ab.items()}
    rng = np.random.default_rng(17)
    pos, cell = W.cubic_lattice("bcc", 2.87, 3)
    pos = W.displace(pos, cell, 0.08, rng)
    spc = W.random_species(pos.shape[0], [27, 27], rng)
    nl = O.neighbours(pos, cell, model["r_cut"])
    _, H_b = O.build_H(model, spc, nl)
    assert H_b.shape[1:] == (5, 5) and H_b.shape[0] > 0
    assert np.max(np.abs(H_b - H_b.transpose(0, 2, 1))) <= 1e-15 * np.max(np.abs(H_b))


def test_spd_blocks_textbook_closed_forms_and_hermiticity():
    """s-s, s-p and p-p elements against the Slater-Koster table
    E_ss = V_sss, E_s,x = l V_sps, E_x,x = l^2 V_pps + (1-l^2) V_ppp,
    E_x,y = l m (V_pps - V_ppp); and H_ji(-S) = H_ij(S)^T for an A-B pair."""
    model = W.spd_alloy_model()
    r = 2.7
    for u in _random_dirs(12, seed=5):
        nl, H_on, H_b = _dimer_H(model, u, r, species=(0, 1))
        H01 = H_b[0] if nl["nbr_j"][0] == 1 else None
        p10 = nl["row_ptr"][1]
        H10 = H_b[p10]
        np.testing.assert_allclose(H10, H01.T, atol=1e-14)
        e = math.exp(-1.8 * (r - 2.5)) * math.sqrt(0.9)
        V = {k: v * e for k, v in {"sss": -1.2, "sps": 1.5, "pps": 2.0, "ppp": -0.6}.items()}
        l, m, n = u
        gl = {1: n, 2: l, 3: m}                       # p_z, p_x, p_y
        assert abs(H01[0, 0] - V["sss"]) < 1e-14
        for a in (1, 2, 3):
            assert abs(H01[0, a] - gl[a] * V["sps"]) < 1e-14
            for b in (1, 2, 3):
                ref = gl[a] * gl[b] * (V["pps"] - V["ppp"]) + (V["ppp"] if a == b else 0.0)
                assert abs(H01[a, b] - ref) < 1e-14
    # onsite levels
    assert np.allclose(H_on[0], [-4.0, 2, 2, 2, 0, 0, 0, 0, 0])
    assert np.allclose(H_on[1], [-3.5, 2.5, 2.5, 2.5, 0.5, 0.5, 0.5, 0.5, 0.5])


def _dense(nl, H_on, H_b):
    n, no = H_on.shape
    H = np.zeros((n * no, n * no))
    for i in range(n):
        H[i * no:(i + 1) * no, i * no:(i + 1) * no] += np.diag(H_on[i])
        for p in range(nl["row_ptr"][i], nl["row_ptr"][i + 1]):
            j = nl["nbr_j"][p]
            H[i * no:(i + 1) * no, j * no:(j + 1) * no] += H_b[p]
    return H


def test_spectrum_invariant_under_rotation_and_inversion():
    rng = np.random.default_rng(1)
    pos, cell = W.cubic_lattice("fcc", 3.5355, 2)
    pos = W.displace(pos, cell, 0.08, rng)
    spc = W.random_species(pos.shape[0], [16, 16], rng)
    model = W.spd_alloy_model()
    nl = O.neighbours(pos, cell, model["r_cut"])
    H = _dense(nl, *O.build_H(model, spc, nl))
    assert np.abs(H - H.T).max() < 1e-14
    ev = np.linalg.eigvalsh(H)
    # random proper rotation of positions and cell together
    A = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    for T in (A, -np.eye(3)):
        pos2, cell2 = pos @ T.T, cell @ T.T
        nl2 = O.neighbours(pos2, cell2, model["r_cut"])
        ev2 = np.linalg.eigvalsh(_dense(nl2, *O.build_H(model, spc, nl2)))
        np.testing.assert_allclose(ev2, ev, atol=1e-12)


def test_cosine_cutoff_taper():
    model = W.canonical_d_model(3.5, d_cut=0.5)
    for r, f in ((2.9, 1.0), (3.0, 1.0), (3.25, 0.5), (3.49, 0.5 * (math.cos(math.pi * 0.98) + 1))):
        nl, H_on, H_b = _dimer_H(model, (0, 0, 1.0), r)
        assert abs(H_b[0][0, 0] - (-(2.48 / r) ** 5 * f)) < 1e-13

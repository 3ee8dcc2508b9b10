"""Pins for the oracle's recursion coefficients, band edges, expansion
coefficients, electron counts, bond energies and Fermi level (CPU only).
References: direct Lanczos on the dense Hamiltonian, the closed forms of the
lowest moments, the semicircle (constant chain) special case, direct kernel
polynomial expansion, numerical quadrature of the expanded DOS, and the exact
tight-binding energy of the same periodic cell."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O
import workloads as W

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _dense(nl, H_on, H_b):
    n, no = H_on.shape
    H = np.zeros((n * no, n * no))
    for i in range(n):
        H[i * no:(i + 1) * no, i * no:(i + 1) * no] += np.diag(H_on[i])
        for p in range(nl["row_ptr"][i], nl["row_ptr"][i + 1]):
            j = nl["nbr_j"][p]
            H[i * no:(i + 1) * no, j * no:(j + 1) * no] += H_b[p]
    return H


def _lanczos(H, start, steps):
    """Lanczos with full reorthogonalisation from the unit vector e_start."""
    D = H.shape[0]
    V = np.zeros((steps + 2, D))
    V[0, start] = 1.0
    a, b = [], [0.0]
    for n in range(steps + 1):
        w = H @ V[n] - b[-1] * (V[n - 1] if n > 0 else 0.0)
        a.append(V[n] @ w)
        w -= a[-1] * V[n]
        for _ in range(2):
            w -= V[: n + 1].T @ (V[: n + 1] @ w)
        b.append(np.linalg.norm(w))
        V[n + 1] = w / b[-1]
    return np.array(a), np.array(b)


@pytest.fixture(scope="module")
def bcc432():
    rng = np.random.default_rng(9)
    pos, cell = W.cubic_lattice("bcc", 3.16, 6)
    pos = W.displace(pos, cell, 0.08, rng)
    model = W.canonical_d_model(3.8)
    nl = O.neighbours(pos, cell, 3.8)
    H_on, H_b = O.build_H(model, np.zeros(432, np.int32), nl)
    return pos, cell, model, nl, H_on, H_b, _dense(nl, H_on, H_b)


@pytest.mark.parametrize("n_max", [9, 18])
def test_recursion_vs_direct_lanczos(bcc432, n_max):
    pos, cell, model, nl, H_on, H_b, H = bcc432
    sel = np.array([0, 17, 230], np.int32)
    mu = O.moments(nl, H_on, H_b, n_max, sel).reshape(-1, n_max + 1)
    rec = O.recursion(mu, n_max)
    na, nb = O.n_a(n_max), O.n_b(n_max)
    tol = 1e-12 if n_max <= 9 else 1e-9
    for r in range(mu.shape[0]):
        i, al = sel[r // 5], r % 5
        a, b = _lanczos(H, 5 * i + al, na)
        np.testing.assert_allclose(rec["a"][r], a[:na], atol=tol)
        np.testing.assert_allclose(rec["b"][r, 1:nb + 1], b[1:nb + 1], atol=tol)
    # closed forms of App. B.3 for the lowest moments
    a0, a1, b1 = rec["a"][:, 0], rec["a"][:, 1], rec["b"][:, 1]
    np.testing.assert_allclose(mu[:, 1], a0, atol=1e-13)
    np.testing.assert_allclose(mu[:, 2], a0 ** 2 + b1 ** 2, atol=1e-13)
    np.testing.assert_allclose(mu[:, 3], a0 ** 3 + 2 * a0 * b1 ** 2 + a1 * b1 ** 2, atol=1e-13)


def _semicircle_moments(bb, n_max, centre=0.0):
    """Moments of a semicircle of half-width 2b about ``centre``:
    mu_2k = Catalan(k) b^2k (centred), shifted binomially."""
    c = [math.comb(2 * k, k) // (k + 1) for k in range(n_max + 1)]
    cen = np.array([c[n // 2] * bb ** n if n % 2 == 0 else 0.0 for n in range(n_max + 1)])
    return np.array([sum(math.comb(n, l) * centre ** (n - l) * cen[l] for l in range(n + 1))
                     for n in range(n_max + 1)])


def test_semicircle_special_case():
    """Constant chain a_n = c, b_n = b: its moments give back the constants,
    the Gershgorin terminator equals the chain, sigma_m = delta_m0, and at
    E_F = c the orbital is half filled with U = -4b/(3 pi)."""
    gold = dict(l.split() for l in open(f"{GOLDEN}/semicircle.txt") if l.strip() and not l.startswith("#"))
    bb, c, n_max, n_exp = 0.8, 0.3, 12, 200
    mu = _semicircle_moments(bb, n_max, centre=c)[None]
    rec = O.recursion(mu, n_max)
    np.testing.assert_allclose(rec["a"], c, atol=1e-12)
    np.testing.assert_allclose(rec["b"][0, 1:], bb, atol=1e-12)
    assert abs(rec["a_inf"][0] - c) < 1e-12 and abs(rec["b_inf"][0] - bb) < 1e-12
    gs = O.dos_coeffs(mu, rec, n_max, n_exp)
    assert abs(gs[0, 0] - 1.0) < 1e-12 and np.max(np.abs(gs[0, 1:])) < 1e-10
    N, U, D = O.orbital_NU(gs[0], rec["a_inf"][0], rec["b_inf"][0], c, c)
    assert abs(N - float(gold["N_half"])) < 1e-12
    assert abs(U - float(gold["U_half_per_b"]) * bb) < 1e-12
    assert abs(D - 1.0 / (math.pi * bb)) < 1e-10


def test_gershgorin_contains_chain_spectrum(bcc432):
    pos, cell, model, nl, H_on, H_b, H = bcc432
    n_max = 18
    mu = O.moments(nl, H_on, H_b, n_max, np.arange(0, 432, 37, dtype=np.int32)).reshape(-1, n_max + 1)
    rec = O.recursion(mu, n_max)
    na, nb = O.n_a(n_max), O.n_b(n_max)
    for r in range(mu.shape[0]):
        T = np.diag(rec["a"][r]) + np.diag(rec["b"][r, 1:na], 1) + np.diag(rec["b"][r, 1:na], -1)
        ev = np.linalg.eigvalsh(T)
        lo = rec["a_inf"][r] - 2 * rec["b_inf"][r]
        hi = rec["a_inf"][r] + 2 * rec["b_inf"][r]
        assert ev.min() >= lo - 1e-12 and ev.max() <= hi + 1e-12


def test_expansion_coefficients_vs_direct_kpm_and_chain(bcc432):
    """sigma_m for m <= n_max by the moment route equals <e|U_m(H^)|e> from a
    direct Chebyshev vector recursion on the dense Hamiltonian, and equals the
    chain route; the Jackson factors run from 1 to 0."""
    pos, cell, model, nl, H_on, H_b, H = bcc432
    n_max, n_exp = 9, 200
    sel = np.array([3, 100], np.int32)
    mu = O.moments(nl, H_on, H_b, n_max, sel).reshape(-1, n_max + 1)
    rec = O.recursion(mu, n_max)
    gs, sc = O.dos_coeffs(mu, rec, n_max, n_exp, with_chain=True)
    g = O.jackson(n_exp)
    assert g[0] == 1.0 and abs(g[-1]) < 1e-15 and np.all(np.diff(g) <= 1e-15)
    sig = gs[:, : n_max + 1] / g[: n_max + 1]
    np.testing.assert_allclose(sc, sig, atol=1e-11)
    for r in range(mu.shape[0]):
        i, al = sel[r // 5], r % 5
        Hh = (H - rec["a_inf"][r] * np.eye(H.shape[0])) / (2 * rec["b_inf"][r])
        u0 = np.zeros(H.shape[0]); u0[5 * i + al] = 1.0
        um1, u = np.zeros_like(u0), u0.copy()
        for m in range(n_max + 1):
            assert abs(u0 @ u - sig[r, m]) < 1e-11
            um1, u = u, 2 * Hh @ u - um1


def test_counts_and_energies_vs_quadrature(bcc432):
    """N and U per orbital equal the numerical integral of the expanded DOS
    n(eps) = (2/pi) sqrt(1 - eps^2) sum_m g_m sigma_m U_m(eps) (Eq. nialpha),
    and the DOS is non-negative."""
    pos, cell, model, nl, H_on, H_b, H = bcc432
    n_max, n_exp = 9, 200
    mu = O.moments(nl, H_on, H_b, n_max, np.array([11], np.int32)).reshape(-1, n_max + 1)
    rec = O.recursion(mu, n_max)
    gs = O.dos_coeffs(mu, rec, n_max, n_exp)
    ai, bi = rec["a_inf"][0], rec["b_inf"][0]
    m = np.arange(n_exp + 1)

    def n_eps(e):
        return 2 / np.pi * np.sqrt(max(0.0, 1 - e * e)) * np.sum(gs[0] * special.eval_chebyu(m, e))

    grid = np.linspace(-0.999, 0.999, 801)
    assert min(n_eps(e) for e in grid) > -1e-10
    for E in (ai - 1.5 * bi, ai + 0.3 * bi, ai + 1.9 * bi):
        ef = (E - ai) / (2 * bi)
        N_q = integrate.quad(n_eps, -1, ef, limit=400, epsabs=1e-13)[0]
        U_q = integrate.quad(lambda e: (ai + 2 * bi * e - H_on[0, 0]) * n_eps(e), -1, ef,
                             limit=400, epsabs=1e-13)[0] * 1.0
        N, U, D = O.orbital_NU(gs[0], ai, bi, H_on[0, 0], E)
        assert abs(N - N_q) < 1e-9
        assert abs(U - U_q) < 1e-9
        assert abs(D - n_eps(ef) / (2 * bi)) < 1e-9
    # outside the band: empty / full, U over the whole band
    N, U, _ = O.orbital_NU(gs[0], ai, bi, 0.0, ai - 3 * bi)
    assert abs(N) < 1e-14 and abs(U) < 1e-14
    N, U, _ = O.orbital_NU(gs[0], ai, bi, 0.0, ai + 3 * bi)
    U_q = integrate.quad(lambda e: (ai + 2 * bi * e) * n_eps(e), -1, 1, limit=400, epsabs=1e-13)[0]
    assert abs(N - 1.0) < 1e-12 and abs(U - U_q) < 1e-9


def test_fermi_level_and_gauge():
    wl = W.bcc_small()
    r = O.energy_pipeline(wl)
    ne = float(np.sum(wl.n_elec))
    assert abs(O.count(r["gsig"], r["rec"]["a_inf"], r["rec"]["b_inf"], r["E_F"]) - ne) < 1e-10 * ne
    assert abs(r["N_atom"].sum() - ne) < 1e-10 * ne
    # monotone electron count
    Es = np.linspace(r["E_F"] - 1, r["E_F"] + 1, 21)
    cnt = [O.count(r["gsig"], r["rec"]["a_inf"], r["rec"]["b_inf"], E) for E in Es]
    assert np.all(np.diff(cnt) >= 0)
    # a uniform onsite shift c moves E_F by c and leaves N_i and U_i unchanged
    r2 = O.energy_pipeline(wl, shift=np.full(wl.n_atoms, 0.37))
    assert abs(r2["E_F"] - r["E_F"] - 0.37) < 1e-9
    np.testing.assert_allclose(r2["U_atom"], r["U_atom"], atol=1e-8)
    np.testing.assert_allclose(r2["N_atom"], r["N_atom"], atol=1e-8)


def test_bond_energy_converges_to_exact_tight_binding(bcc432):
    """As the number of moments grows, the BOP bond energy of a displaced
    432-atom bcc cell approaches the exact Gamma-point tight-binding energy
    2 sum_occ e_k (zero onsite levels; fractional filling at E_F)."""
    pos, cell, model, nl, H_on, H_b, H = bcc432
    ne = 4.5 * 432
    w = np.linalg.eigvalsh(H)
    nocc = ne / 2.0
    full = int(math.floor(nocc))
    U_tb = 2 * (np.sum(w[:full]) + (nocc - full) * w[full])
    errs = []
    for n_max in (5, 9, 13, 17):
        wl = W.Workload("c", pos, cell, np.zeros(432, np.int32), model, n_max, 200, np.full(432, 4.5))
        r = O.energy_pipeline(wl, nl=nl)
        errs.append(abs(r["U_total"] - U_tb) / 432)
    assert errs[-1] < errs[0]
    assert errs[-1] < 0.02          # eV / atom


def test_scf_fixed_point_and_invariants():
    rng = np.random.default_rng(5)
    pos, cell = W.cubic_lattice("bcc", 2.87, 3)
    spc = W.random_species(54, [27, 27], rng)
    wl = W.Workload("a", W.wrap(pos, cell), cell, spc, W.canonical_d_model(3.5, onsite_d=(0.0, 0.8)),
                    8, 200, np.where(spc == 0, 6.0, 5.0))
    shift, hist, r = O.scf(wl, mix=0.5, tol=1e-4, max_iter=100)
    assert hist[-1]["max_dq"] < 1e-4 and len(hist) < 100
    assert abs(np.mean(shift)) < 1e-12
    assert abs(r["N_atom"].sum() - wl.n_elec.sum()) < 1e-8
    # the B atoms (higher bare level, fewer electrons wanted) end up lower
    assert np.mean(shift[spc == 1]) < np.mean(shift[spc == 0])


def test_scf_broyden_reaches_the_linear_fixed_point():
    """The Broyden cycle converges (max |q| < 1e-4) in fewer iterations than
    linear mixing on the 54-atom alloy, to the same fixed point: shifts agree
    within 1e-3 eV (both stop within 1e-4 electrons of charge neutrality; the
    per-atom DOS at E_F is ~1 state/eV)."""
    rng = np.random.default_rng(5)
    pos, cell = W.cubic_lattice("bcc", 2.87, 3)
    spc = W.random_species(54, [27, 27], rng)
    wl = W.Workload("a", W.wrap(pos, cell), cell, spc, W.canonical_d_model(3.5, onsite_d=(0.0, 0.8)),
                    8, 200, np.where(spc == 0, 6.0, 5.0))
    s_lin, h_lin, _ = O.scf(wl, mix=0.5, tol=1e-4, max_iter=100)
    s_bro, h_bro, r = O.scf_broyden(wl, mix=0.5, tol=1e-4, max_iter=100)
    assert h_bro[-1]["max_dq"] < 1e-4 and len(h_bro) < len(h_lin)
    assert abs(np.mean(s_bro)) < 1e-12
    assert np.max(np.abs(s_bro - s_lin)) < 1e-3


def test_mlp_gradients_vs_finite_differences():
    rng = np.random.default_rng(0)
    sizes = [(64, 6), (64,), (64, 64), (64,), (1, 64), (1,)]
    params = [rng.normal(scale=0.3, size=s) for s in sizes]
    x = rng.normal(size=(37, 6))
    t = rng.normal(size=37)
    loss, grads = O.mlp_loss_grad(params, x, t)
    h = 1e-6
    for k, p in enumerate(params):
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = O.mlp_loss_grad(params, x, t)
            flat[idx] = old - h
            lm, _ = O.mlp_loss_grad(params, x, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            g = grads[k].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-7 * max(1.0, abs(g))


def test_adam_step_properties_and_hand_values():
    """Adam (Kingma & Ba, Algorithm 1: bias-corrected first and second moment
    estimates, eps added to the square root of the second).  Pins: (1) from
    zero moments a constant gradient g moves a parameter by lr g / (|g| + eps)
    at every step, whatever |g| (the bias corrections make both estimates
    exactly g and g^2), so n steps move it by n lr; a missing or misplaced bias
    correction breaks this.  (2) A gradient of 1e-8 with eps = 1e-8 moves it by
    lr / 2 (eps outside the root; inside the root the step would be ~1e-4 lr).
    (3) Two steps worked by hand: p0 = 1, g1 = 2, g2 = -1, lr = 0.1:
    m1 = 0.2, v1 = 0.004 -> p1 = 1 - 0.1 * 2 / (2 + 1e-8);
    m2 = 0.08, v2 = 0.004996, bias factors 0.19 and 0.001999 ->
    p2 = p1 - 0.1 * (0.08 / 0.19) / (sqrt(0.004996 / 0.001999) + 1e-8)."""
    for g in (3.0, -0.25, 7e-3):
        p, m, v = [np.array([1.5])], [np.zeros(1)], [np.zeros(1)]
        for t in range(1, 6):
            p, m, v = O.adam_step(p, [np.array([g])], m, v, t, lr=0.01)
            step = 0.01 * abs(g) / (abs(g) + 1e-8)
            assert abs(p[0][0] - (1.5 - np.sign(g) * t * step)) < 1e-14
    p, _, _ = O.adam_step([np.array([0.0])], [np.array([1e-8])], [np.zeros(1)], [np.zeros(1)], 1, lr=0.1)
    assert abs(p[0][0] + 0.05) < 1e-15
    p, m, v = O.adam_step([np.array([1.0])], [np.array([2.0])], [np.zeros(1)], [np.zeros(1)], 1, lr=0.1)
    p1 = 1.0 - 0.2 / (2.0 + 1e-8)
    assert abs(p[0][0] - p1) < 1e-15 and abs(m[0][0] - 0.2) < 1e-15 and abs(v[0][0] - 0.004) < 1e-15
    p, m, v = O.adam_step(p, [np.array([-1.0])], m, v, 2, lr=0.1)
    assert abs(m[0][0] - 0.08) < 1e-15 and abs(v[0][0] - 0.004996) < 1e-15
    p2 = p1 - 0.1 * (0.08 / 0.19) / (np.sqrt(0.004996 / 0.001999) + 1e-8)
    assert abs(p[0][0] - p2) < 1e-14
    assert abs(p2 - 0.8733662967) < 1e-9          # the same value evaluated by hand to 10 digits


def test_feature_stats_and_gauge_closed_forms():
    """Column statistics of 0, 1, ..., n-1 (scaled per column): mean (n-1)/2 and
    sample variance n (n+1) / 12.  The gauge-fixed shifts sum to zero and keep
    every difference of the network's outputs."""
    n = 1001
    x = np.arange(n, dtype=np.float64)[:, None] * np.array([1.0, 2.0, -0.5, 3.0, 0.25, 10.0])[None, :]
    mean, std = O.feature_stats(x)
    scale = np.array([1.0, 2.0, 0.5, 3.0, 0.25, 10.0])
    assert np.allclose(mean, (n - 1) / 2 * np.array([1.0, 2.0, -0.5, 3.0, 0.25, 10.0]), rtol=1e-14)
    assert np.allclose(std, np.sqrt(n * (n + 1) / 12.0) * scale, rtol=1e-13)
    mean1, std1 = O.feature_stats(np.ones((5, 6)))
    assert np.all(std1 == 1e-12) and np.all(mean1 == 1.0)
    rng = np.random.default_rng(1)
    params = [rng.normal(scale=0.3, size=sh) for sh in [(64, 6), (64,), (64, 64), (64,), (1, 64), (1,)]]
    xs = rng.normal(size=(50, 6))
    y, _ = O.mlp_forward(params, xs)
    d = O.mlp_shift(params, xs)
    assert abs(d.sum()) < 1e-12
    assert np.allclose(d[1:] - d[:-1], y[1:] - y[:-1], atol=1e-14)


def _chain_moments(a, b, n_max):
    """Site-0 moments of a finite tridiagonal chain (a_0.., b_1..)."""
    J = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    return np.array([np.linalg.matrix_power(J, n)[0, 0] for n in range(n_max + 1)])


def test_band_centre_and_width_options_hand_values():
    """App. B.5 options i-v, vii and the weighted average of Eq. (weighted) on a
    chain with a = (0.5, -1, 2, 0.25), b = (1, 2, 0.5, 1.5), 8 moments (four
    levels of each), worked by hand:
      (i)   a_0, b_1                            -> 0.5, 1
      (ii)  a_3, b_4                            -> 0.25, 1.5
      (iii) mean a = 1.75/4, sqrt(mean b^2) = sqrt(7.5/4)
      (iv)  mean a, b_4                         -> 0.4375, 1.5
      (v)   (2 - 1)/2, (2 + 1 + 4*2)/4          -> 0.5, 2.75
      (vii) edges -4 and 4.5 (rows 1 and 2)     -> 0.25, 2.125
      weighted, beta = 1: w = 1/4, 1/3, 1/2, 1 for both a and b:
            (0.125 - 1/3 + 1 + 0.25) / (25/12) = 0.5,
            (0.25 + 2/3 + 0.25 + 1.5) / (25/12) = 1.28."""
    a = [0.5, -1.0, 2.0, 0.25, 0.7]          # a_4 does not enter 8 moments
    b = [1.0, 2.0, 0.5, 1.5]
    mu = _chain_moments(a, b, 8)[None, :]
    want = {"lowest": (0.5, 1.0), "highest": (0.25, 1.5), "average": (0.4375, math.sqrt(1.875)),
            "average_highest": (0.4375, 1.5), "minmax": (0.5, 2.75), "gershgorin": (0.25, 2.125),
            "weighted": (0.5, 1.28)}
    for mode, (A, B) in want.items():
        r = O.recursion(mu, 8, bw=mode, beta=1.0)
        assert np.allclose(r["a"][0], a[:4], atol=1e-12) and np.allclose(r["b"][0, 1:], b, atol=1e-12)
        assert abs(r["a_inf"][0] - A) < 1e-12 and abs(r["b_inf"][0] - B) < 1e-12, mode
    # weighted with beta = 0: plain averages of a and of b
    r = O.recursion(mu, 8, bw="weighted", beta=0.0)
    assert abs(r["a_inf"][0] - 0.4375) < 1e-12 and abs(r["b_inf"][0] - 1.25) < 1e-12


def test_band_options_use_only_levels_before_a_breakdown():
    """A two-level chain (a = (1, -0.5), b_1 = 2, nothing beyond) at 6 moments:
    the recursion breaks down at level 2; options i-v and the weighted average
    see a_0, a_1, b_1 only: (ii) gives a_1 = -0.5 and b_1 = 2, (iii) gives 0.25
    and 2, (v) gives 0.25 and (1.5 + 8)/4."""
    mu = _chain_moments([1.0, -0.5], [2.0], 6)[None, :]
    r = O.recursion(mu, 6, bw="highest")
    assert r["flags"][0] & 1 and (r["flags"][0] >> 8) == 2
    assert abs(r["a_inf"][0] + 0.5) < 1e-12 and abs(r["b_inf"][0] - 2.0) < 1e-12
    r = O.recursion(mu, 6, bw="average")
    assert abs(r["a_inf"][0] - 0.25) < 1e-12 and abs(r["b_inf"][0] - 2.0) < 1e-12
    r = O.recursion(mu, 6, bw="minmax")
    assert abs(r["a_inf"][0] - 0.25) < 1e-12 and abs(r["b_inf"][0] - 9.5 / 4) < 1e-12


def test_broyden_linear_system_secant_and_linear_limit():
    """Broyden's second method on F(x) = b - A x (A symmetric positive definite,
    6 x 6): (1) it reaches A^-1 b within 2n = 12 steps (Gay 1979: Broyden's
    updates terminate on linear systems in at most 2n steps); (2) after every
    update the secant condition H_n y_n = s_n holds; (3) with no history it is
    linear mixing, x + eta F."""
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.normal(size=(6, 6)))
    A = Q @ np.diag([0.5, 0.8, 1.0, 1.7, 2.5, 3.0]) @ Q.T
    bvec = rng.normal(size=6)
    x_star = np.linalg.solve(A, bvec)
    m = O.Broyden(eta=0.3, hist=50, gauge=False)
    x = np.zeros(6)
    for it in range(13):
        F = bvec - A @ x
        x_new = m.step(x, F)
        if m.u:
            assert np.allclose(m.apply_H(m.y[-1]), x - m_prev, atol=1e-12)
        m_prev = x.copy()
        x = x_new
    assert np.max(np.abs(x - x_star)) < 1e-8
    lin = O.Broyden(eta=0.3, hist=0, gauge=False)
    x = np.zeros(6)
    for it in range(5):
        F = bvec - A @ x
        xn = lin.step(x, F)
        assert np.allclose(xn, x + 0.3 * F, atol=1e-15)
        x = xn


def test_isolated_atoms_are_delta_bands():
    """Atoms without neighbours have a delta-function local DOS at their
    onsite level: the chain ends at level 1 (breakdown), b_inf sits at its
    floor and the expansion must reproduce a filled d shell (10 electrons) on
    the deeper atom and the remaining electron on the other, with zero bond
    energy (U is measured from the onsite level)."""
    pos = np.array([[1.0, 1.0, 1.0], [9.0, 9.0, 9.0]])
    cell = np.eye(3) * 20.0
    spc = np.array([0, 1], np.int32)
    wl = W.Workload("iso", pos, cell, spc, W.canonical_d_model(3.5, onsite_d=(0.0, 0.8)), 6, 200,
                    np.array([6.0, 5.0]))
    r = O.energy_pipeline(wl)
    assert np.all(r["rec"]["flags"] & 1)
    assert np.all((r["rec"]["flags"] >> 8) == 1)
    np.testing.assert_allclose(r["N_atom"], [10.0, 1.0], atol=1e-6)
    np.testing.assert_allclose(r["U_atom"], [0.0, 0.0], atol=1e-6)
    assert abs(r["E_F"] - 0.8) < 1e-5


def test_magnetic_channels_reduce_to_the_non_magnetic_path():
    """With no exchange (I = 0) and no field both spin channels are the
    non-magnetic problem: same Fermi level, N_i, U_i, and zero moments."""
    wl = W.bcc_small()
    r0 = O.energy_pipeline(wl)
    rm = O.energy_pipeline_mag(wl, [0.0], moment=np.linspace(-1, 1, wl.n_atoms))
    assert abs(rm["E_F"] - r0["E_F"]) < 1e-12
    np.testing.assert_allclose(rm["N_atom"], r0["N_atom"], atol=1e-12)
    np.testing.assert_allclose(rm["U_atom"], r0["U_atom"], atol=1e-12)
    assert np.max(np.abs(rm["moment"])) < 1e-12 and rm["U_X"] == 0.0


def test_magnetic_linear_response_is_the_stoner_factor():
    """A small uniform moment m splits the channels by I m; at fixed E_F
    (unchanged to first order by symmetry) the output moment is
    m_out = I n_sigma(E_F) m, n_sigma the non-magnetic DOS per spin and atom at
    E_F: the Stoner enhancement.  It pins the sign and the factor 1/2 of the
    spin splitting."""
    wl = W.bcc_small()
    r0 = O.energy_pipeline(wl)
    m0 = 1e-5
    rm = O.energy_pipeline_mag(wl, [0.8], moment=np.full(wl.n_atoms, m0))
    want = 0.8 * r0["dos_atom"] / 2.0
    np.testing.assert_allclose(rm["moment"] / m0, want, rtol=1e-4)


def test_magnetic_isolated_atoms_closed_form():
    """Isolated atoms with 6.5 d electrons and exchange splitting I m = 1 eV:
    the lowered (up) shell fills (5 electrons), the down shell holds 1.5, so
    m_out = 3.5 whatever the input moment's size, U_X = -1/4 I m_out^2, and
    the Fermi level sits on the down level, H0 + I m / 2."""
    pos = np.array([[1.0, 1.0, 1.0], [9.0, 9.0, 9.0]])
    cell = np.eye(3) * 20.0
    wl = W.Workload("iso", pos, cell, np.zeros(2, np.int32), W.canonical_d_model(3.5), 6, 200,
                    np.array([6.5, 6.5]))
    rm = O.energy_pipeline_mag(wl, [1.0], moment=np.array([1.0, 1.0]))
    np.testing.assert_allclose(rm["N_spin"][0], [5.0, 5.0], atol=1e-6)
    np.testing.assert_allclose(rm["N_spin"][1], [1.5, 1.5], atol=1e-6)
    np.testing.assert_allclose(rm["moment"], [3.5, 3.5], atol=1e-6)
    assert abs(rm["U_X"] + 0.25 * 2 * 3.5 ** 2) < 1e-5
    assert abs(rm["E_F"] - 0.5) < 1e-5


def _bcc54(sigma=0.05, n_max=8):
    rng = np.random.default_rng(14)
    pos, cell = W.cubic_lattice("bcc", 2.87, 3)
    if sigma:
        pos = W.displace(pos, cell, sigma, rng)
    return W.Workload("b54", pos, cell, np.zeros(54, np.int32), W.canonical_d_model(3.5), n_max, 200,
                      np.full(54, 6.5))


def test_direction_cosine_blocks_match_rotation_blocks_and_invariants():
    """The direction-cosine d-d blocks the force oracle differentiates: equal to
    the C oracle's App. D rotation blocks for generic bonds (1e-13), equal to
    diag(Vs, Vp, Vp, Vd, Vd) for a bond along z (the bond frame itself), with
    eigenvalues {Vs, Vp, Vp, Vd, Vd} in every direction, including the polar
    axis where the angle form is singular."""
    rng = np.random.default_rng(0)
    model = W.canonical_d_model(10.0)
    for _ in range(6):
        d = rng.normal(size=3)
        d *= 2.6 / np.linalg.norm(d)
        pos = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0] + d])
        nl = O.neighbours(pos, np.eye(3) * 30.0, 3.0)
        _, Hb = O.build_H(model, np.zeros(2, np.int32), nl)
        B = O._dd_blocks(model, np.zeros(2, np.int32), nl, nl["nbr_d"])
        assert np.max(np.abs(B - Hb)) < 1e-13 * np.max(np.abs(Hb))
    Vs, Vp, Vd = -1.3, 0.7, -0.2
    B = O._sk_dd(np.array(0.0), np.array(0.0), np.array(1.0), Vs, Vp, Vd)
    np.testing.assert_allclose(B, np.diag([Vs, Vp, Vp, Vd, Vd]), atol=1e-15)
    for u in [np.array([0.0, 0.0, -1.0]), np.array([1.0, 0.0, 0.0]), rng.normal(size=3)]:
        u = u / np.linalg.norm(u)
        B = O._sk_dd(u[0], u[1], u[2], Vs, Vp, Vd)
        np.testing.assert_allclose(B, B.T, atol=0)
        np.testing.assert_allclose(np.linalg.eigvalsh(B), np.sort([Vs, Vp, Vp, Vd, Vd]), atol=1e-14)


def test_forces_match_finite_differences_of_the_energy():
    """The oracle's analytic forces (weights, Theta~, block derivatives)
    against central differences of its own bond energy (neighbours, H,
    moments, recursion, expansion and the Fermi bisection redone at r +- h,
    h = 1e-4 A; truncation error ~h^2 F''' ~ 1e-8 eV/A), for even and odd
    n_max (odd 5: at 7, 9 and 11 some orbitals' Gershgorin-terminated
    expansions diverge on this cell); the forces sum to zero."""
    for n_max in (8, 5):
        wl = _bcc54(n_max=n_max)
        F, r, _ = O.forces(wl)
        assert np.max(np.abs(F.sum(axis=0))) < 1e-10
        h = 1e-4
        rng = np.random.default_rng(n_max)
        for _ in range(4):
            k, c = int(rng.integers(54)), int(rng.integers(3))
            pp, pm = wl.pos.copy(), wl.pos.copy()
            pp[k, c] += h
            pm[k, c] -= h
            up = O.energy_pipeline(W.Workload("p", pp, wl.cell, wl.species, wl.model, n_max, 200, wl.n_elec))
            um = O.energy_pipeline(W.Workload("m", pm, wl.cell, wl.species, wl.model, n_max, 200, wl.n_elec))
            fd = -(up["U_total"] - um["U_total"]) / (2 * h)
            assert abs(F[k, c] - fd) < 1e-6 * max(1.0, abs(fd)), (n_max, k, c, F[k, c], fd)


def test_forces_vanish_on_a_perfect_lattice_and_weights_match_differences():
    """Every atom of a perfect bcc lattice is a centre of inversion: F = 0.
    The weights dU/dmu (complex step, with the Fermi level's response) match
    central differences of the oracle's energy in one orbital's moment."""
    wl = _bcc54(sigma=0.0)
    F, _, _ = O.forces(wl)
    assert np.max(np.abs(F)) < 1e-10
    wl = _bcc54()
    nl = O.neighbours(wl.pos, wl.cell, 3.5)
    r = O.energy_pipeline(wl, nl=nl)
    rows = r["mu"].reshape(-1, 9)
    w, _, _ = O.weights(rows, 8, 200, r["E_F"], r["H_on"].reshape(-1))

    def U_of(rows_):
        rec = O.recursion(rows_, 8)
        gs = O.dos_coeffs(rows_, rec, 8, 200)
        ef = O.fermi(gs, rec["a_inf"], rec["b_inf"], float(np.sum(wl.n_elec)))
        return O.energy(gs, rec["a_inf"], rec["b_inf"], r["H_on"], ef)["U_total"]

    for (row, n) in ((3, 2), (40, 5), (200, 8)):
        h = 1e-6 * abs(rows[row, n]) + 1e-7
        p, m = rows.copy(), rows.copy()
        p[row, n] += h
        m[row, n] -= h
        fd = (U_of(p) - U_of(m)) / (2 * h)
        assert abs(w[row, n] - fd) < 1e-5 * max(1e-3, abs(fd)), (row, n, w[row, n], fd)


def test_atom_averaged_mode_equals_orbital_mode_for_isotropic_bonds():
    """With equal d-d bond integrals in every channel each bond block is V I,
    so all five orbitals of an atom have the same local DOS and the atom-
    averaged chain is each orbital's chain: both modes give the same E_F and
    energies.  With the canonical channels they differ (the averaged DOS is a
    different approximation) while the electron count stays N_e."""
    rng = np.random.default_rng(21)
    pos, cell = W.cubic_lattice("bcc", 2.87, 3)
    pos = W.displace(pos, cell, 0.05, rng)
    model = W.canonical_d_model(3.5)
    b = dict(model["bonds"][(0, 0)])
    b["ddp"] = b["dds"]
    b["ddd"] = b["dds"]
    iso = dict(model, bonds={(0, 0): b})
    wl = W.Workload("iso", pos, cell, np.zeros(54, np.int32), iso, 8, 200, np.full(54, 6.5))
    r = O.energy_pipeline(wl)
    ra = O.energy_pipeline_avg(wl)
    assert abs(ra["E_F"] - r["E_F"]) < 1e-12
    np.testing.assert_allclose(ra["N_atom"], r["N_atom"], atol=1e-12)
    np.testing.assert_allclose(ra["U_atom"], r["U_atom"], atol=1e-12)
    wl2 = W.Workload("can", pos, cell, np.zeros(54, np.int32), model, 8, 200, np.full(54, 6.5))
    r2 = O.energy_pipeline(wl2)
    ra2 = O.energy_pipeline_avg(wl2)
    assert abs(ra2["N_atom"].sum() - 54 * 6.5) < 1e-9
    assert abs(ra2["U_total"] - r2["U_total"]) > 1e-3


def test_onsite_theta_is_the_onsite_derivative_of_the_energy():
    """Eq. BOP_SCF: dU/dE_i (all orbitals of atom i shifted together) =
    sum_a Theta~_(ia,ia) - N_i, with E_F following; central differences of the
    oracle's energy in one atom's onsite shift (h = 1e-5 eV)."""
    wl = _bcc54(n_max=8)
    _, r, _ = O.forces(wl)
    delta = r["theta_onsite"].sum(axis=1) - r["N_atom"]
    h = 1e-5
    for k in (0, 17, 40):
        sp = np.zeros(54)
        sm = np.zeros(54)
        sp[k] = h
        sm[k] = -h
        fd = (O.energy_pipeline(wl, shift=sp)["U_total"] - O.energy_pipeline(wl, shift=sm)["U_total"]) / (2 * h)
        assert abs(delta[k] - fd) < 1e-7 * max(1.0, abs(fd)), (k, delta[k], fd)

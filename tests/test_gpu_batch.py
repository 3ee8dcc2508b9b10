"""Batched form: ragged structures joined into one block-diagonal graph give
each structure the moments of its own cell (against per-structure runs and,
for small structures, the oracle); the captured graph replays reproduce the
eager result bit for bit, with eager work between replays."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _batch():
    structs = [W.ragged_structure(s) for s in (1, 3, 9, 11, 8, 6)]       # hcp, random, bcc, fcc, random, fcc
    structs = [s for s in structs if s.n_atoms <= 600]
    d = W.dimer(2.6, direction=(0.3, -0.5, 0.8))                          # a 2-atom structure
    structs.append(d)
    return structs


def _model():
    return W.canonical_d_model(3.6)


def test_batched_equals_per_structure_and_oracle(bop):
    from paper_1803_07491_amd.batch import BatchedMoments, PerStructure
    structs = _batch()
    m = _model()
    b = BatchedMoments(structs, m, 10, "f64")
    b.run()
    ps = PerStructure(structs, m, 10, "f64")
    ps.run()
    for s, wl in enumerate(structs):
        mu_b = b.structure_mu(s).cpu().numpy()
        mu_s = ps.items[s][4].cpu().numpy()
        scale = np.maximum(np.abs(mu_s), 1e-12 * np.abs(mu_s).max())
        assert np.max(np.abs(mu_b - mu_s) / scale) < 1e-12, s
        if wl.n_atoms <= 200:
            nl = O.neighbours(wl.pos, wl.cell, m["r_cut"])
            H_on, H_bond = O.build_H(m, wl.species, nl)
            ref = O.moments(nl, H_on, H_bond, 10)
            assert np.max(np.abs(mu_b - ref) / np.maximum(np.abs(ref), 1e-12 * np.abs(ref).max())) < 1e-10, s


def test_moments_batched_one_call_and_its_graph(bop):
    """bop_moments_batched (join, supports and moments in one enqueue-only
    call) gives the moments of the separate calls bit for bit, and a graph
    captured around it replays them, with the join and the supports redone
    from cleared outputs at every replay."""
    import torch
    from paper_1803_07491_amd.batch import BatchedMoments
    b = BatchedMoments(_batch(), _model(), 14, "f32")
    b.run()
    torch.cuda.synchronize()
    eager = b.mu.clone()
    b.mu.fill_(-7.0)
    b.step()
    torch.cuda.synchronize()
    assert torch.equal(b.mu, eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.step()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.step()
    for r in range(3):
        b.mu.fill_(-7.0)
        b.nl.nbr_j.fill_(-1)
        b.nl.row_ptr.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(b.mu, eager), r
        x = torch.randn(1 << 20, device="cuda")            # eager work between replays
        float(x.sum())


@pytest.mark.parametrize("method", ["moments", "lanczos"])
def test_graph_replays_match_eager(bop, method):
    import torch
    from paper_1803_07491_amd.batch import BatchedMoments
    structs = _batch()
    b = BatchedMoments(structs, _model(), 14, "f32", method=method)
    b.run()
    torch.cuda.synchronize()
    key = "a" if method == "lanczos" else None
    eager = (b.rec["a"] if key else b.mu).clone()
    eager_b = b.rec["b"].clone() if key else None
    b.capture()
    for r in range(4):
        (b.rec["a"] if key else b.mu).fill_(-7.0)
        b.replay()
        torch.cuda.synchronize()
        out = b.rec["a"] if key else b.mu
        assert torch.equal(out, eager), r
        if key:
            assert torch.equal(b.rec["b"], eager_b), r
        x = torch.randn(1 << 20, device="cuda")            # eager work between replays
        float(x.sum())
    b.run()                                                # eager again after the replays
    torch.cuda.synchronize()
    assert torch.equal(b.rec["a"] if key else b.mu, eager)


def test_autotune_keeps_a_valid_tiling(bop):
    from paper_1803_07491_amd.batch import BatchedMoments, autotune
    structs = _batch()
    b = BatchedMoments(structs, _model(), 8, "f32")
    b.run()
    ref = b.mu.clone()
    best, times = autotune(b, candidates=[dict(tile_atoms=0, block_threads=256, chunk_rows=16),
                                          dict(tile_atoms=6, block_threads=512, chunk_rows=64)], reps=1)
    assert len(times) == 2
    b.run()
    np.testing.assert_allclose(b.mu.cpu().numpy(), ref.cpu().numpy(), rtol=1e-5, atol=1e-5 * float(ref.abs().max()))


def test_autotune_coordinate_search_and_cache(bop, tmp_path):
    """The coordinate search starts from the default tiling, keeps a tiling
    only when it is faster, leaves the batch on the pick (results unchanged
    up to FP32 rounding), and a second call with the cache returns the same
    pick without timing anything."""
    from paper_1803_07491_amd.batch import BatchedMoments, autotune, _key, DEFAULT
    structs = _batch()
    b = BatchedMoments(structs, _model(), 8, "f32")
    b.run()
    ref = b.mu.clone()
    cache = str(tmp_path / "tune.json")
    space = {"tile_atoms": [0, 6], "chunk_rows": [16, 64], "plan_search": [0, 2]}
    best, times = autotune(b, reps=1, space=space, rounds=1, cache=cache)
    assert _key(DEFAULT) in times
    assert times[_key(best)] <= times[_key(DEFAULT)]
    b.run()
    np.testing.assert_allclose(b.mu.cpu().numpy(), ref.cpu().numpy(), rtol=1e-5, atol=1e-5 * float(ref.abs().max()))
    again, t2 = autotune(b, reps=1, space=space, rounds=1, cache=cache)
    assert again == best and t2 == {}

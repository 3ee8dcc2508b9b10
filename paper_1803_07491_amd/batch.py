"""Batched moments over many ragged periodic structures.

The structures' neighbour lists are built one by one (each on its own cell)
and joined by ``bop_batch_concat`` into one block-diagonal graph; one moment
plan and one prepare pass then cover the batch, and the moment launch
sequence (``bop_moments`` or ``bop_lanczos``) is captured once in a HIP graph
and replayed.  ``PerStructure`` is the plain alternative: one plan and one
launch sequence per structure.  ``autotune`` times candidate tilings on the
batch itself and keeps the fastest.

Everything numeric runs in the HIP library; this module only sequences calls
and marshals arguments.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import (BOP_E_CAPACITY, BOP_E_UNSUPPORTED, BopError, Neighbours, build_H, build_neighbours, lanczos,
               load, moments, moments_plan, moments_prepare, n_a, n_b, _check, _ptr, _stream, _torch)


class BatchedMoments:
    def __init__(self, structures, model, n_max, dtype="f32", tuning=None, method="moments", device="cuda"):
        torch = _torch()
        load()
        self.device = torch.device(device)
        self.model, self.n_max, self.dtype, self.method = model, int(n_max), dtype, method
        nls, species, sizes = [], [], []
        for wl in structures:
            pos = torch.as_tensor(np.ascontiguousarray(wl.pos, np.float64), device=self.device)
            nls.append(build_neighbours(pos, wl.cell, model["r_cut"]))
            species.append(np.asarray(wl.species, np.int32))
            sizes.append(len(wl.species))
        self.sizes = np.array(sizes)
        self.n_structs = len(structures)
        atom_off = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int32)
        pair_off = np.concatenate([[0], np.cumsum([nl.n_pairs for nl in nls])]).astype(np.int32)
        self.atom_off, self.pair_off = atom_off, pair_off
        self.n = int(atom_off[-1])
        P = int(pair_off[-1])
        cat = lambda ts: torch.cat(ts) if ts else None
        row_ptr_local = cat([nl.row_ptr for nl in nls])
        nbr_j_local = cat([nl.nbr_j for nl in nls])
        order_local = cat([nl.order for nl in nls])
        nbr_d = cat([nl.nbr_d for nl in nls])
        d_atom_off = torch.as_tensor(atom_off, device=self.device)
        d_pair_off = torch.as_tensor(pair_off, device=self.device)
        row_ptr = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        nbr_j = torch.empty(max(P, 1), dtype=torch.int32, device=self.device)[:P]
        order = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)[: self.n]
        _check(load().bop_batch_concat(self.n_structs, self.n, _ptr(d_atom_off), _ptr(d_pair_off), _ptr(row_ptr_local),
                                       _ptr(nbr_j_local), _ptr(order_local), _ptr(row_ptr), _ptr(nbr_j), _ptr(order),
                                       _stream()))
        self.local = (d_atom_off, d_pair_off, row_ptr_local, nbr_j_local, order_local)
        self.nl = Neighbours(row_ptr, nbr_j, None, nbr_d, order, P)
        self.species = torch.as_tensor(np.concatenate(species), device=self.device)
        self.H_on, self.H_bond = build_H(model, self.species, self.nl, dtype=dtype)
        self.no = model["n_orb"]
        self.set_tuning(tuning)
        self.graph = None

    def set_tuning(self, tuning):
        torch = _torch()
        self.tuning = tuning
        self.plan = moments_plan(self.n, self.no, self.n_max, self.dtype, self.nl, tuning)
        self.ws = moments_prepare(self.plan, self.nl)
        R = self.n * self.no
        self.mu = torch.empty((self.n, self.no, self.n_max + 1), dtype=torch.float64, device=self.device)
        self.rec = {"a": torch.empty((R, n_a(self.n_max)), dtype=torch.float64, device=self.device),
                    "b": torch.empty((R, n_b(self.n_max) + 1), dtype=torch.float64, device=self.device),
                    "flags": torch.empty(R, dtype=torch.int32, device=self.device)}
        self.graph = None

    def run(self):
        """One launch sequence over the whole batch (eager)."""
        if self.method == "lanczos":
            return lanczos(self.plan, self.nl, self.H_on, self.H_bond, out=self.rec, ws=self.ws)
        return moments(self.plan, self.nl, self.H_on, self.H_bond, mu=self.mu, ws=self.ws)

    def step(self):
        """The whole batch step in one library call (``bop_moments_batched``):
        join the per-structure lists, prepare the supports, moments."""
        d_atom_off, d_pair_off, row_ptr_local, nbr_j_local, order_local = self.local
        _check(load().bop_moments_batched(C.byref(self.plan), self.n_structs, _ptr(d_atom_off), _ptr(d_pair_off),
                                          _ptr(row_ptr_local), _ptr(nbr_j_local), _ptr(order_local),
                                          _ptr(self.nl.row_ptr), _ptr(self.nl.nbr_j), _ptr(self.nl.order),
                                          _ptr(self.H_on), _ptr(self.H_bond), _ptr(self.mu), _ptr(self.ws),
                                          self.ws.numel(), _stream()))
        return self.mu

    def capture(self):
        """Record the launch sequence in a HIP graph (after one eager run on
        the capture stream)."""
        torch = _torch()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()

    def structure_mu(self, s):
        return self.mu[self.atom_off[s]:self.atom_off[s + 1]]


class PerStructure:
    """One plan and one moment launch sequence per structure.  Every
    structure keeps its own prepared workspace, so each plan's batch is
    capped (64 tiles unless ``tuning`` says otherwise): the 512-structure
    workload would otherwise hold X buffers for all of its tiles at once."""

    def __init__(self, structures, model, n_max, dtype="f32", tuning=None, device="cuda"):
        torch = _torch()
        tuning = dict(tuning or {})
        tuning.setdefault("batch_tiles", 64)
        self.items = []
        for wl in structures:
            pos = torch.as_tensor(np.ascontiguousarray(wl.pos, np.float64), device=device)
            nl = build_neighbours(pos, wl.cell, model["r_cut"])
            sp = torch.as_tensor(np.asarray(wl.species, np.int32), device=device)
            H_on, H_bond = build_H(model, sp, nl, dtype=dtype)
            plan = moments_plan(len(wl.species), model["n_orb"], n_max, dtype, nl, tuning)
            ws = moments_prepare(plan, nl)
            mu = torch.empty((len(wl.species), model["n_orb"], n_max + 1), dtype=torch.float64, device=device)
            self.items.append((plan, nl, H_on, H_bond, mu, ws))

    def run(self):
        for plan, nl, H_on, H_bond, mu, ws in self.items:
            moments(plan, nl, H_on, H_bond, mu=mu, ws=ws)


# the autotuner's search space: tile size (atoms per 64 columns; 0 = as many
# as fit one wavefront), workgroup size, rows per workgroup and step, tiles
# whose vectors are live at once (0 = the memory-sized default) and the
# support search of the plan (0 automatic, 1 LDS bitmap, 2 global map)
SPACE = {"tile_atoms": [0, 4, 6, 8, 10], "block_threads": [256, 512, 1024], "chunk_rows": [16, 32, 64, 128],
         "batch_tiles": [0, 256, 1024], "plan_search": [0, 2]}
DEFAULT = {"tile_atoms": 0, "block_threads": 512, "chunk_rows": 64, "batch_tiles": 0, "plan_search": 0}

# kept for callers that time an explicit list
CANDIDATES = [dict(tile_atoms=ta, block_threads=bt, chunk_rows=cr)
              for ta in (0, 6) for bt in (256, 512, 1024) for cr in (16, 32, 64, 128)]


def _key(cand):
    return "_".join(f"{k}{cand.get(k, DEFAULT[k])}" for k in DEFAULT)


def _time(batch, cand, reps, times, log):
    """Graph-replay time of one tiling (ms), or None if the plan rejects it."""
    torch = _torch()
    key = _key(cand)
    if key in times:
        return times[key]
    try:
        batch.set_tuning(cand)
    except BopError as e:
        # a tiling the plan rejects; any other failure (a HIP error that may
        # have left the stream unusable) propagates
        if e.code not in (BOP_E_UNSUPPORTED, BOP_E_CAPACITY):
            raise
        if log:
            log(f"skip {key}: {e}")
        times[key] = None
        return None
    batch.capture()
    batch.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        batch.replay()
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    times[key] = ms
    if log:
        log(f"{key}: {ms:.2f} ms")
    return ms


def autotune(batch: BatchedMoments, candidates=None, reps=2, log=None, space=None, rounds=2, cache=None):
    """Pick the fastest tiling for this batch by timing graph replays.

    With ``candidates`` (a list of tuning dicts) every one is timed.  Otherwise
    a coordinate search over ``space`` (default SPACE): starting from the
    default tiling, each parameter in turn is swept with the others fixed and
    the best value kept, for ``rounds`` passes or until a pass changes
    nothing.  ``cache`` (a JSON file path) stores the pick per workload
    signature (atoms, pairs, moments, dtype, form) and is consulted first.
    Returns (best tuning dict, {tiling: ms})."""
    import json
    import os
    sig = f"n{batch.n}_p{batch.nl.n_pairs}_m{batch.n_max}_{batch.dtype}_{batch.method}"
    if cache and os.path.exists(cache):
        known = json.load(open(cache))
        if sig in known:
            best = known[sig]
            batch.set_tuning(best)
            return best, {}
    times = {}
    if candidates is not None:
        scored = [(c, _time(batch, c, reps, times, log)) for c in candidates]
        scored = [(c, t) for c, t in scored if t is not None]
        if not scored:
            raise RuntimeError("autotune: the plan rejected every candidate tiling")
        best = min(scored, key=lambda ct: ct[1])[0]
    else:
        space = space or SPACE
        best = dict(DEFAULT)
        best_ms = _time(batch, best, reps, times, log)
        if best_ms is None:
            raise RuntimeError("autotune: the plan rejected the default tiling")
        for _ in range(rounds):
            changed = False
            for name, values in space.items():
                for v in values:
                    if v == best[name]:
                        continue
                    cand = dict(best, **{name: v})
                    ms = _time(batch, cand, reps, times, log)
                    if ms is not None and ms < best_ms:
                        best, best_ms, changed = cand, ms, True
            if not changed:
                break
    batch.set_tuning(best)
    if cache:
        known = json.load(open(cache)) if os.path.exists(cache) else {}
        known[sig] = best
        with open(cache, "w") as f:
            json.dump(known, f, indent=1)
    return best, times

#!/usr/bin/env python3
"""Benchmark of the analytic-BOP energy path on one MI355X.

Workload: bcc 40x40x40 supercell (128,000 atoms, a = 3.16 A), Gaussian
displacements sigma = 0.08 A (seed 2), canonical d band (dd sigma : pi : delta =
-6 : 4 : -1, r^-5, dd sigma = -1 eV at 2.48 A), two-shell cutoff 3.8 A
(14 neighbours), 18 moments, N_d = 4.5, one energy evaluation.

A step is one pass of the whole path with inputs resident on the GPU:
neighbour list -> Hamiltonian -> moment plan -> moments (H.X in the compute
dtype, FP64 accumulation) -> recursion -> expansion coefficients -> Fermi level
-> energies.  The metric is atom-moments/s = N_atoms * n_max / step time.

Printed: one JSON line with the metric, a roofline object for the moment
kernel (algorithmic flops on the exact k-hop supports / measured kernel time)
and a CPU baseline from the FP64 oracle on a bounded sample of atoms.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0}   # MI355X peaks: vector FP32 (incl. packed), FP64, dense BF16 MFMA
PEAK_NONPACKED_F32 = 78.6                     # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_flops_per_atom(row_ptr, nbr_j, n_orb, n_max, sample):
    """H.X flops one atom's n_orb columns need on exact supports: for each step
    k = 1..K, every row s of the (k-1)-hop support feeds its deg(s) neighbours
    with an n_orb x n_orb block (2 n_orb^2 flops per column) and itself with
    the diagonal onsite level (2 n_orb); an odd n_max adds H X^K restricted to
    the K-hop support."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import dijkstra
    n = row_ptr.shape[0] - 1
    deg = np.diff(row_ptr)
    A = sp.csr_matrix((np.ones(nbr_j.shape[0]), nbr_j, row_ptr), shape=(n, n))
    K = n_max // 2
    dist = dijkstra(A, indices=sample, unweighted=True, limit=K + 0.5)
    out = []
    for d in dist:
        f = 0.0
        for k in range(1, K + 1):
            s = d <= k - 1
            f += n_orb * (2 * n_orb * n_orb * deg[s].sum() + 2 * n_orb * s.sum())
        if n_max % 2:
            inK = d <= K
            rows = np.nonzero(inK)[0]
            inner = sum(int(np.sum(inK[nbr_j[row_ptr[r]:row_ptr[r + 1]]])) for r in rows)
            f += n_orb * (2 * n_orb * n_orb * inner + 2 * n_orb * inK.sum())
        out.append(f)
    return np.array(out)


def kernel_source_hash():
    h = hashlib.sha256()
    p = os.path.join(ROOT, "paper_1803_07491_amd", "csrc", "moments.hip")
    h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def read_traffic(dtype):
    """HBM bytes per launch of the moment kernel measured with rocprofv3
    counters (FETCH_SIZE + WRITE_SIZE, scaled by a copy-kernel calibration),
    if recorded for the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_moments_bcc_large_{dtype}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(wl, target_s=12.0):
    """The FP64 oracle on the host cores: full neighbour list and H, then
    moments, recursion, expansion and energies (at a fixed Fermi level) for a
    seeded sample of atoms sized to take about `target_s` seconds."""
    import oracle as O
    t0 = time.perf_counter()
    nl = O.neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    H_on, H_b = O.build_H(wl.model, wl.species, nl)
    t_nlh = time.perf_counter() - t0
    rng = np.random.default_rng(123)

    def run(m):
        sel = np.sort(rng.choice(wl.n_atoms, size=m, replace=False)).astype(np.int32)
        t = time.perf_counter()
        mu = O.moments(nl, H_on, H_b, wl.n_max, sel)
        rows = mu.reshape(-1, wl.n_max + 1)
        rec = O.recursion(rows, wl.n_max)
        gs = O.dos_coeffs(rows, rec, wl.n_max, wl.n_exp)
        O.energy(gs, rec["a_inf"], rec["b_inf"], H_on[sel], 0.0)
        return time.perf_counter() - t

    t_probe = run(16)
    m = int(max(16, min(wl.n_atoms, 16 * target_s / max(t_probe, 1e-3))))
    t_s = run(m)
    t_tot = t_s + t_nlh * m / wl.n_atoms
    return {"value": m * wl.n_max / t_tot, "unit": "atom-moments/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": (f"{m} of {wl.n_atoms} atoms (seeded): FP64 moments, recursion, expansion and energies "
                       f"at a fixed Fermi level; full-cell neighbour list + H ({t_nlh:.2f} s) charged pro rata; "
                       f"Fermi bisection excluded (needs every atom)"),
            "seconds": round(t_s + t_nlh, 2)}


def timed_steps(path, n_elec, steps, warmup, torch):
    for _ in range(warmup):
        path.step(n_elec)
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        path.rebuild()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        path.run_moments()
        b.record()
        out = path.run_tail(n_elec)
        evs.append((a, b))
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    kms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    return t, kms, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64", "bf16"])
    ap.add_argument("--method", default="moments", choices=["moments", "lanczos"],
                    help="moments then FP64 recursion, or the recursion straight from the H.X products")
    ap.add_argument("--reps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (for scaling HBM counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4}))
        return

    import paper_1803_07491_amd as P
    import workloads as W
    P.load()
    wl = W.bcc_large(reps=args.reps)
    n_elec = float(wl.n_elec.sum())
    log(f"workload bcc {args.reps}^3: {wl.n_atoms} atoms, n_max {wl.n_max}, dtype {args.dtype}, {args.method}")
    path = P.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, args.dtype,
                        method=args.method)
    log(f"plan: tile {path.plan.tile_atoms} atoms, {path.plan.n_tiles} tiles, rows_cap {path.plan.rows_cap}, "
        f"workspace {path.plan.ws_bytes / 2**30:.2f} GiB, batch {path.plan.batch_tiles} tiles, chunk {path.plan.chunk_rows} rows x "
        f"{path.plan.block_threads}")
    t_step, t_mom_ms, out = timed_steps(path, n_elec, args.steps, args.warmup, torch)
    log(f"{args.dtype}: {t_step * 1e3:.2f} ms/step, moment kernel {t_mom_ms:.2f} ms, "
        f"E_F {float(out['E_F'].cpu()[0]):.8f} eV, U {float(out['U_total'].cpu()[0]) / wl.n_atoms:.8f} eV/atom")

    rp = path.nl.row_ptr.cpu().numpy()
    nj = path.nl.nbr_j.cpu().numpy()
    sample = np.random.default_rng(7).choice(wl.n_atoms, size=8, replace=False)
    fpa = algorithmic_flops_per_atom(rp, nj, path.no, wl.n_max, sample)
    flops = float(fpa.mean()) * wl.n_atoms
    achieved = flops / (t_mom_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.dtype]
    traffic = read_traffic(args.dtype)
    res = {
        "metric": "atom-moments/s",
        "value": wl.n_atoms * wl.n_max / t_step,
        "unit": "atom-moments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"bcc {args.reps}^3 supercell, {wl.n_atoms} atoms, a=3.16 A, sigma=0.08 A, "
                               f"canonical d band, cutoff 3.8 A, {wl.n_max} moments, N_d=4.5, single energy",
                   "n_atoms": wl.n_atoms, "n_max": wl.n_max, "n_exp": wl.n_exp,
                   "method": args.method, "hx_dtype": args.dtype, "tail_dtype": "f64",
                   "tile_atoms": path.plan.tile_atoms, "block_threads": path.plan.block_threads,
                   "batch_tiles": path.plan.batch_tiles, "chunk_rows": path.plan.chunk_rows},
        "roofline": {"bound": "mfma" if args.dtype == "bf16" else "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": "k_step (all H.X launches of one pass)", "kernel_ms": t_mom_ms,
                     "algorithmic_flops_per_launch": flops,
                     "flops_per_atom": float(fpa.mean()), "flops_per_atom_spread": float(np.ptp(fpa))},
    }
    if args.dtype == "f32":
        res["roofline"]["frac_nonpacked_fp32"] = achieved / PEAK_NONPACKED_F32
    if not args.no_f64 and (args.dtype != "f64" or args.method != "moments"):
        # the plain FP64 path (moments, FP64 recursion) as the reference
        p64 = P.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
        t64, k64, o64 = timed_steps(p64, n_elec, args.steps, 1, torch)
        u32 = float(out["U_total"].cpu()[0])
        u64 = float(o64["U_total"].cpu()[0])
        res["f64_path"] = {"value": wl.n_atoms * wl.n_max / t64, "ms_per_step": t64 * 1e3, "kernel_ms": k64,
                           "achieved_tflops": flops / (k64 * 1e-3) / 1e12,
                           "energy_err_meV_per_atom": abs(u32 - u64) / wl.n_atoms * 1e3}
        log(f"f64: {t64 * 1e3:.2f} ms/step, moment kernel {k64:.2f} ms, |dU| "
            f"{res['f64_path']['energy_err_meV_per_atom']:.3e} meV/atom")
        del p64
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(wl)
        log(f"cpu: {res['cpu_baseline']['value']:.3e} atom-moments/s on {res['cpu_baseline']['cores']} threads")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

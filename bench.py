#!/usr/bin/env python3
"""Benchmark of the analytic-BOP energy path on one MI355X.

Workload: bcc 40x40x40 supercell (128,000 atoms, a = 3.16 A), Gaussian
displacements sigma = 0.08 A (seed 2), canonical d band (dd sigma : pi : delta =
-6 : 4 : -1, r^-5, dd sigma = -1 eV at 2.48 A), two-shell cutoff 3.8 A
(14 neighbours), 18 moments, N_d = 4.5, one energy evaluation.

A step is one pass of the whole path with inputs resident on the GPU:
neighbour list -> Hamiltonian -> moment plan -> H.X passes in the compute
dtype with FP64 sums (by default the Lanczos form, which gives the recursion
coefficients of the 18 moments directly; --method moments computes the moments
and the FP64 recursion) -> terminator -> expansion coefficients -> Fermi level
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

# MI355X peaks: vector FP32 (incl. packed), FP64, dense BF16 and FP16 MFMA (the 16-bit H.X forms of the
# d band run on MFMA)
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "f16": 2500.0}
PEAK_NONPACKED_F32 = 78.6                     # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_HBM_TBPS = 8.0


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


def algorithmic_flops_per_atom_radius(pos, cell, row_ptr, nbr_j, n_orb, n_max, sample, r_max):
    """The same count with a maximum path radius: the supports and degrees are
    those of the graph restricted to the atoms within r_max (minimum image) of
    the column's atom, since a path leaving that ball is dropped."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import dijkstra
    n = row_ptr.shape[0] - 1
    inv = np.linalg.inv(cell)
    i_of = np.repeat(np.arange(n), np.diff(row_ptr))
    K = n_max // 2
    out = []
    for c in sample:
        f = (pos - pos[c]) @ inv
        f -= np.round(f)
        inb = np.linalg.norm(f @ cell, axis=1) <= r_max
        keep = inb[i_of] & inb[nbr_j]
        A = sp.csr_matrix((np.ones(int(keep.sum())), (i_of[keep], nbr_j[keep])), shape=(n, n))
        deg = np.asarray(A.sum(axis=1)).ravel()
        d = dijkstra(A, indices=[c], unweighted=True, limit=K + 0.5)[0]
        fl = 0.0
        for k in range(1, K + 1):
            s_ = d <= k - 1
            fl += n_orb * (2 * n_orb * n_orb * deg[s_].sum() + 2 * n_orb * s_.sum())
        if n_max % 2:
            inK = d <= K
            inner = A[inK][:, inK].sum()
            fl += n_orb * (2 * n_orb * n_orb * inner + 2 * n_orb * inK.sum())
        out.append(fl)
    return np.array(out)


def cpu_baseline_forces(W, reps=4):
    """The oracle's force path on a small cell of the headline recipe (bcc
    a = 3.16 A, sigma = 0.08 A, seed 2, the same model and moments): energy,
    weights, Theta~ from dense matrix powers of the folded H, block
    derivatives.  Dense in the cell, so its cost grows as N^3."""
    import oracle as O
    wl = W.bcc_large(reps=reps)
    t = time.perf_counter()
    O.forces(wl)
    sec = time.perf_counter() - t
    return {"value": wl.n_atoms / sec, "unit": "atoms/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": (f"energy and forces of a {wl.n_atoms}-atom cell (bcc {reps}^3, same lattice, displacements, "
                       f"model and {wl.n_max} moments) by the oracle's dense path (its cost grows as N^3)"),
            "seconds": round(sec, 2)}


def cpu_baseline_scf(wl, kind, n_target, stoner=None, mix_m=0.8, traj_steps=0):
    """The oracle's self-consistent cycle on a small cell: LCN with linear
    mixing ("linear"), Broyden mixing ("broyden"), or collinear magnetism
    from m = 1 ("magnetic"); with traj_steps > 0, that many seeded MD-like
    steps, each started from the previous converged shifts (the metric is then
    per step).  Also reported scaled to n_target atoms, assuming a cost linear
    in the atoms (the oracle's per-atom moments) at the sample's iteration
    count."""
    import oracle as O
    import workloads as W_
    t = time.perf_counter()
    if kind == "magnetic":
        O.scf_mag(wl, stoner, np.ones(wl.n_atoms), mix=0.5, mix_m=mix_m, max_iter=800)
        n_scf = 1
    elif traj_steps:
        shift = None
        for pos in W_.md_trajectory(wl, traj_steps, step_sigma=0.02):
            w = W_.Workload(wl.name, pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, wl.n_elec, wl.meta)
            fn = O.scf_broyden if kind == "broyden" else O.scf
            shift, _, _ = fn(w, shift0=shift, tol=1e-4, max_iter=300)
        n_scf = traj_steps
    else:
        (O.scf_broyden if kind == "broyden" else O.scf)(wl, tol=1e-4, max_iter=300)
        n_scf = 1
    sec = time.perf_counter() - t
    return {"value": sec / n_scf, "unit": "s", "cores": O.num_threads(), "kind": "oracle",
            "scaled_to_workload_s": sec / n_scf * n_target / wl.n_atoms,
            "sample": (f"the oracle's {kind} cycle on a {wl.n_atoms}-atom cell of the same recipe"
                       + (f", {traj_steps} warm-started MD-like steps" if traj_steps else "")
                       + " (FP64, every atom's moments each iteration)"),
            "seconds": round(sec, 2)}


def kernel_source_hash(source="moments.hip"):
    """Hash of a kernel file's code: the source without // comments and
    blank lines, so that a change of comments keeps recorded counters valid."""
    p = os.path.join(ROOT, "paper_1803_07491_amd", "csrc", source)
    lines = []
    for ln in open(p, encoding="utf-8").read().splitlines():
        code = ln.split("//", 1)[0].rstrip()
        if code:
            lines.append(code)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def read_traffic(dtype, method, source="moments.hip"):
    """HBM bytes of one H.X pass (or force pass) measured with rocprofv3
    counters (FETCH_SIZE + WRITE_SIZE, scaled by a copy-kernel calibration),
    if recorded for the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_{method}_bcc_large_{dtype}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_sha256_16") != kernel_source_hash(source):
        return None
    return d.get("bytes_per_launch")


def per_atom_errors(out, ref):
    """Largest relative per-atom differences of N_i and U_i."""
    eN = ((out["N_atom"] - ref["N_atom"]).abs() / ref["N_atom"].abs()).max().item()
    eU = ((out["U_atom"] - ref["U_atom"]).abs() / ref["U_atom"].abs()).max().item()
    return {"N": eN, "U": eU}


def cpu_baseline(wl, target_s=12.0, r_max=0.0):
    """The FP64 oracle on the host cores: full neighbour list and H, then
    moments (with a maximum path radius if r_max > 0), recursion, expansion
    and energies (at a fixed Fermi level) for a seeded sample of atoms sized
    to take about `target_s` seconds."""
    import oracle as O
    t0 = time.perf_counter()
    nl = O.neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    H_on, H_b = O.build_H(wl.model, wl.species, nl)
    t_nlh = time.perf_counter() - t0
    rng = np.random.default_rng(123)

    def run(m):
        sel = np.sort(rng.choice(wl.n_atoms, size=m, replace=False)).astype(np.int32)
        t = time.perf_counter()
        mu = O.moments(nl, H_on, H_b, wl.n_max, sel, r_max=r_max)
        rows = mu.reshape(-1, wl.n_max + 1)
        rec = O.recursion(rows, wl.n_max)
        gs = O.dos_coeffs(rows, rec, wl.n_max, wl.n_exp)
        O.energy(gs, rec["a_inf"], rec["b_inf"], H_on[sel], 0.0)
        return time.perf_counter() - t

    # two probes: the first (16 atoms) is dominated by start-up costs, so the
    # second, sized to about a tenth of the target, sets the sample
    t_probe = run(16)
    m1 = int(max(16, min(wl.n_atoms, 16 * 0.1 * target_s / max(t_probe, 1e-3))))
    t_probe = run(m1)
    m = int(max(16, min(wl.n_atoms, m1 * target_s / max(t_probe, 1e-3))))
    t_s = run(m)
    t_tot = t_s + t_nlh * m / wl.n_atoms
    return {"value": m * wl.n_max / t_tot, "unit": "atom-moments/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": (f"{m} of {wl.n_atoms} atoms (seeded): FP64 moments"
                       + (f" (paths within {r_max:g} A)" if r_max > 0 else "")
                       + ", recursion, expansion and energies "
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


def stage_times(path, n_elec, P, torch):
    """One more step, after the timed ones, with HIP events between its
    stages: a1 neighbour list, a2 H, the moment plan and supports, the H.X
    passes, the tail (a4-a8).  The neighbour list and the plan read a count
    back to the host, so their intervals include that round trip."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    ev[0].record()
    path.nl = P.build_neighbours(path.pos, path.cell, path.model["r_cut"], capacity=path.nl.n_pairs)
    ev[1].record()
    path.H_on, path.H_bond = P.build_H(path.model, path.species, path.nl, dtype=path.dtype, H_on=path.H_on,
                                       H_bond=path.H_bond)
    ev[2].record()
    path.plan = P.moments_plan(path.n, path.no, path.n_max, path.dtype, path.nl, path.tuning, radius=path.radius)
    path.mws = P.moments_prepare(path.plan, path.nl, ws=path.mws, radius=path.radius)
    ev[3].record()
    path.run_moments()
    ev[4].record()
    path.run_tail(n_elec)
    ev[5].record()
    torch.cuda.synchronize()
    names = ("a1_neighbours", "a2_H", "plan_and_supports", "hx_passes", "tail_a4_a8")
    return {k: ev[i].elapsed_time(ev[i + 1]) for i, k in enumerate(names)}


def hx_roofline(P, wl, dtype, method, torch):
    """The H.X pass of one energy evaluation of the workload's cell, with the
    dtype and form its cycle uses, against the compute peak on exact per-atom
    supports (a cycle runs this pass once per iteration, per spin channel in
    a collinear one)."""
    p = P.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, dtype, method=method)
    _, kms, _ = timed_steps(p, float(np.sum(wl.n_elec)), 2, 1, torch)
    rp, nj = p.nl.row_ptr.cpu().numpy(), p.nl.nbr_j.cpu().numpy()
    fpa = algorithmic_flops_per_atom(rp, nj, p.no, wl.n_max,
                                     np.random.default_rng(7).choice(wl.n_atoms, 8, replace=False))
    del p
    torch.cuda.empty_cache()
    flops = float(fpa.mean()) * wl.n_atoms
    ach = flops / (kms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": ach, "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
            "frac": ach / PEAK_TFLOPS[dtype], "traffic": None,
            "kernel": f"k_step ({method}, {dtype}): the H.X launches of one energy pass of the cell",
            "kernel_ms": kms, "algorithmic_flops_per_launch": flops, "flops_per_atom": float(fpa.mean())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64", "bf16", "f16"],
                    help="H.X arithmetic/storage; f16 = FP16 vectors with FP32 H and arithmetic (Lanczos form)")
    ap.add_argument("--method", default="lanczos", choices=["moments", "lanczos"],
                    help="recursion coefficients straight from the H.X products (Lanczos, default), or moments "
                         "then the FP64 recursion")
    ap.add_argument("--reps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--workload", default="energy",
                    choices=["energy", "batch", "scf", "precision", "radius", "md", "magnetic", "forces",
                             "terminators", "mlp"],
                    help="energy: bcc 40^3 single energy (default); batch: 512 ragged structures; "
                         "scf: 250,000-atom alloy SCF with MLP warm start (and Broyden mixing); precision: s,p,d "
                         "alloy, 20 moments; radius: bcc 40^3 with maximum path radii; md: alloy SCF along a "
                         "trajectory, warm against cold starts; magnetic: collinear ferromagnetic bcc Stoner cycle; forces: "
                         "energy and forces of the bcc 40^3 cell")
    ap.add_argument("--md-steps", type=int, default=5)
    ap.add_argument("--reps-md", type=int, default=30)
    ap.add_argument("--reps-mag", type=int, default=12)
    ap.add_argument("--n-structs", type=int, default=512)
    ap.add_argument("--n-train", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=50)
    ap.add_argument("--reps-scf", type=int, default=50)
    ap.add_argument("--reps-spd", type=int, default=30)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy (for scaling HBM counters)")
    ap.add_argument("--copy-gib", type=int, default=1, help="size of the calibration copy in GiB")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        x = torch.ones(args.copy_gib << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4}))
        return

    import paper_1803_07491_amd as P
    import workloads as W
    P.load()
    if args.workload != "energy":
        {"batch": bench_batch, "scf": bench_scf, "precision": bench_precision, "radius": bench_radius,
         "md": bench_md, "magnetic": bench_magnetic, "forces": bench_forces,
         "terminators": bench_terminators, "mlp": bench_mlp}[args.workload](args, torch, P, W)
        return
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

    out = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in out.items()}
    rp = path.nl.row_ptr.cpu().numpy()
    nj = path.nl.nbr_j.cpu().numpy()
    sample = np.random.default_rng(7).choice(wl.n_atoms, size=8, replace=False)
    fpa = algorithmic_flops_per_atom(rp, nj, path.no, wl.n_max, sample)
    flops = float(fpa.mean()) * wl.n_atoms
    achieved = flops / (t_mom_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.dtype]
    traffic = read_traffic(args.dtype, args.method)
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
        "roofline": {"bound": "mfma" if args.dtype in ("bf16", "f16") else "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": ("k_lstep16" if args.dtype in ("bf16", "f16") and args.method == "lanczos" else "k_step")
                               + " (all H.X launches of one pass)", "kernel_ms": t_mom_ms,
                     "algorithmic_flops_per_launch": flops,
                     "flops_per_atom": float(fpa.mean()), "flops_per_atom_spread": float(np.ptp(fpa))},
    }
    if traffic:
        # the second ceiling: measured HBM bytes of the pass over its time
        res["roofline"]["achieved_hbm_TBps"] = traffic / (t_mom_ms * 1e-3) / 1e12
        res["roofline"]["hbm_frac"] = res["roofline"]["achieved_hbm_TBps"] / PEAK_HBM_TBPS
    if args.dtype == "f32":
        res["roofline"]["frac_nonpacked_fp32"] = achieved / PEAK_NONPACKED_F32
    # where one step's time goes (one more step, outside the timed ones)
    res["stages_ms"] = stage_times(path, n_elec, P, torch)
    res["a1_a2_ms"] = res["stages_ms"]["a1_neighbours"] + res["stages_ms"]["a2_H"]
    log(f"stages (ms): {res['stages_ms']}")
    if not args.no_f64 and (args.dtype != "f64" or args.method != "moments"):
        # the plain FP64 path (moments, FP64 recursion) as the reference
        p64 = P.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
        t64, k64, o64 = timed_steps(p64, n_elec, args.steps, 1, torch)
        u32 = float(out["U_total"].cpu()[0])
        u64 = float(o64["U_total"].cpu()[0])
        # per-atom accuracy of the timed form: its energies at the FP64 path's
        # Fermi level against the FP64 path's, every atom
        o_at = path.run_tail(n_elec, E_F=o64["E_F"].clone())
        res["accuracy_vs_f64"] = {"max_atom_rel_err": per_atom_errors(o_at, o64), "bar": 1e-5,
                                  "energy_err_meV_per_atom": abs(u32 - u64) / wl.n_atoms * 1e3,
                                  "E_F_diff_eV": abs(float(out["E_F"].cpu()[0]) - float(o64["E_F"].cpu()[0]))}
        res["f64_path"] = {"value": wl.n_atoms * wl.n_max / t64, "ms_per_step": t64 * 1e3, "kernel_ms": k64,
                           "achieved_tflops": flops / (k64 * 1e-3) / 1e12}
        log(f"f64: {t64 * 1e3:.2f} ms/step, moment kernel {k64:.2f} ms; timed form vs f64: {res['accuracy_vs_f64']}")
        if args.method == "lanczos" and args.dtype == "f32":
            # the FP32 moment form, for comparison: faster, but the moments-to-
            # coefficients map amplifies its rounding beyond the FP32 bar per atom
            del path
            pm = P.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f32", method="moments")
            tm, km, om = timed_steps(pm, n_elec, args.steps, 1, torch)
            om_at = pm.run_tail(n_elec, E_F=o64["E_F"].clone())
            res["moments_f32_path"] = {"value": wl.n_atoms * wl.n_max / tm, "ms_per_step": tm * 1e3,
                                       "kernel_ms": km, "achieved_tflops": flops / (km * 1e-3) / 1e12,
                                       "frac": flops / (km * 1e-3) / 1e12 / peak,
                                       "max_atom_rel_err": per_atom_errors(om_at, o64),
                                       "meets_fp32_bar": False}
            res["moments_f32_path"]["meets_fp32_bar"] = max(res["moments_f32_path"]["max_atom_rel_err"].values()) < 1e-5
            log(f"moments f32: {tm * 1e3:.2f} ms/step, kernel {km:.2f} ms, {res['moments_f32_path']['max_atom_rel_err']}")
            del pm
        del p64
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(wl)
        log(f"cpu: {res['cpu_baseline']['value']:.3e} atom-moments/s on {res['cpu_baseline']['cores']} threads")
    print(json.dumps(res), flush=True)


# ---------------------------------------------------------------------------
# other workloads (each prints its own JSON line)
# ---------------------------------------------------------------------------
def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _launches(plan):
    """Kernel launches in one moment launch sequence: per batch of tiles the
    unit columns, one step per level (plus the odd pass) and the reduction."""
    K = plan.n_max // 2
    steps = K + (plan.n_max & 1)
    n_batches = -(-plan.n_tiles // max(plan.batch_tiles, 1))
    return n_batches * (steps + 2)


def bench_batch(args, torch, P, W):
    """512 ragged structures (bcc/fcc/hcp/random dense packing, 50-5000 atoms,
    0.085 atoms/A^3), d band, cutoff 3.6 A, 14 moments, FP32 H.X: the batch as
    one captured launch sequence (default and autotuned tiling) against one
    launch sequence per structure."""
    from paper_1803_07491_amd.batch import BatchedMoments, PerStructure, autotune
    import oracle as O
    t0 = time.perf_counter()
    structs = [W.ragged_structure(s) for s in range(args.n_structs)]
    model = W.canonical_d_model(3.6)
    n_max = 14
    N = sum(w.n_atoms for w in structs)
    log(f"batch: {len(structs)} structures, {N} atoms, generated in {time.perf_counter() - t0:.1f} s")
    b = BatchedMoments(structs, model, n_max, args.dtype)

    def time_replays(reps):
        b.replay()
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        e0.record()
        for _ in range(reps):
            b.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    b.capture()
    t_def = time_replays(args.steps)
    log(f"batched, default tiling: {t_def:.2f} ms")
    ps = PerStructure(structs, model, n_max, args.dtype)
    ps.run()
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(args.steps):
        ps.run()
    e1.record()
    torch.cuda.synchronize()
    t_loop = e0.elapsed_time(e1) / args.steps
    log(f"per-structure loop: {t_loop:.2f} ms")
    # per-structure results vs the batched ones (same dtype; only the tiling differs)
    # scale-normalised error |d mu_n| / (mu_0 s^n) per orbital, s = max over even
    # m of (mu_m / mu_0)^(1/m), the spectral radius estimate of the orbital's DOS
    err = 0.0
    nn = torch.arange(n_max + 1, device=b.mu.device, dtype=torch.float64)
    ev = torch.arange(2, n_max + 1, 2, device=b.mu.device)
    for s in range(len(structs)):
        a_ = b.structure_mu(s)
        r_ = ps.items[s][4]
        rad = ((r_[..., ev] / r_[..., :1]).clamp_min(1e-300) ** (1.0 / ev.double())).amax(-1, keepdim=True)
        sc = r_[..., :1] * rad ** nn
        err = max(err, float(((a_ - r_).abs() / sc).max()))
    del ps
    best, times = autotune(b, reps=max(1, args.steps // 2), log=log)
    b.capture()
    t_best = time_replays(args.steps)
    log(f"batched, autotuned {best}: {t_best:.2f} ms")
    # algorithmic flops: exact supports of two sampled atoms per structure
    rng = np.random.default_rng(11)
    flops = 0.0
    for w in structs:
        nl = O.neighbours(w.pos, w.cell, model["r_cut"])
        smp = rng.choice(w.n_atoms, size=min(2, w.n_atoms), replace=False)
        flops += float(algorithmic_flops_per_atom(nl["row_ptr"], nl["nbr_j"], 5, n_max, smp).mean()) * w.n_atoms
    achieved = flops / (t_best * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.dtype]
    res = {
        "metric": "atom-moments/s", "value": N * n_max / (t_best * 1e-3), "unit": "atom-moments/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": t_best, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"{len(structs)} ragged periodic structures (bcc/fcc/hcp/random dense packing, "
                               f"50-5000 atoms log-uniform, 0.085 atoms/A^3), {N} atoms, d band, cutoff 3.6 A, "
                               f"{n_max} moments, moments only (one captured launch sequence)",
                   "n_atoms": N, "n_structs": len(structs), "n_max": n_max, "autotuned": best},
        "launches_per_replay": _launches(b.plan),
        "batched_default_ms": t_def, "per_structure_loop_ms": t_loop,
        "speedup_vs_loop": t_loop / t_best, "autotune_gain": t_def / t_best, "autotune_ms": times,
        "batched_vs_per_structure_max_scaled_err": err,
        "roofline": {"bound": "mfma" if args.dtype == "bf16" else "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "algorithmic_flops_per_launch": flops},
    }
    if not args.no_cpu:
        t = time.perf_counter()
        done = 0
        sel = rng.choice(len(structs), size=len(structs), replace=False)
        for s in sel:
            w = structs[s]
            nl = O.neighbours(w.pos, w.cell, model["r_cut"])
            H_on, H_b = O.build_H(model, w.species, nl)
            O.moments(nl, H_on, H_b, n_max)
            done += w.n_atoms
            if time.perf_counter() - t > 12.0:
                break
        dt = time.perf_counter() - t
        res["cpu_baseline"] = {"value": done * n_max / dt, "unit": "atom-moments/s", "cores": O.num_threads(),
                               "kind": "oracle", "sample": f"whole structures in seeded random order until 12 s: "
                                                           f"{done} atoms (neighbours, H, FP64 moments)"}
    print(json.dumps(res), flush=True)


def bench_scf(args, torch, P, W):
    """Learned form: 250,000-atom bcc A/B alloy (eps_B = 0.8 eV, N_d 6/5), 16
    moments, LCN self-consistency to max|q| < 1e-4.  Plain FP64 cycle from
    zero shifts against the MLP warm start (trained here on 200 converged
    2,000-atom alloys), with the FP64 cycle or the FP32 Lanczos cycle."""
    from paper_1803_07491_amd import warmstart as WS
    t0 = time.perf_counter()
    train = [W.bcc_alloy_scf(seed=5001 + s, reps=10) for s in range(args.n_train)]
    xs, ts, its = [], [], []
    for k, w in enumerate(train):
        x = WS.zero_shift_features(w)
        sp, it, _, _ = WS.converge(w, dtype="f64")
        xs.append(x)
        ts.append(sp.shift.float())
        its.append(it)
        del sp
        if k % 40 == 0:
            log(f"training structure {k}: {it} iterations")
    n_fit = int(round(0.9 * len(train)))
    rows_fit = sum(w.n_atoms for w in train[:n_fit])
    x = torch.cat(xs)
    t = torch.cat(ts)
    t_data = time.perf_counter() - t0
    t1 = time.perf_counter()
    model = WS.fit(x[:rows_fit], t[:rows_fit], epochs=args.epochs, batch=4096, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    xv = P.standardise(x[rows_fit:].contiguous(), model.mean, model.std)
    yv = model.predict(xv).double()
    # gauge: compare mean-free predictions per validation structure
    off = rows_fit
    se, cnt = 0.0, 0
    for w in train[n_fit:]:
        pv = yv[off - rows_fit: off - rows_fit + w.n_atoms]
        tv = t[off: off + w.n_atoms].double()
        se += float((((pv - pv.mean()) - (tv - tv.mean())) ** 2).sum())
        cnt += w.n_atoms
        off += w.n_atoms
    rmse = (se / max(cnt, 1)) ** 0.5
    log(f"training data {t_data:.1f} s, fit {t_train:.1f} s, validation rmse {rmse:.3e} eV")

    wl = W.bcc_alloy_scf(seed=5, reps=args.reps_scf)
    log(f"scf workload: {wl.n_atoms} atoms")
    # plain FP64 from zero
    plain, it_p, t_p, _ = WS.converge(wl, dtype="f64")
    u_p = float(plain.out["U_total"].item())
    log(f"plain FP64: {it_p} iterations, {t_p:.2f} s")
    bro = P.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, "f64", mixer="broyden")
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    it_b, _ = bro.run_scf(tol=1e-4, max_iter=300)
    torch.cuda.synchronize()
    broyden = {"iterations": it_b, "seconds": time.perf_counter() - tb0,
               "energy_diff_meV_per_atom": abs(float(bro.out["U_total"].item()) - u_p) / wl.n_atoms * 1e3}
    log(f"Broyden FP64: {broyden}")
    del bro
    shift_p = plain.shift.clone()
    del plain

    def warm(dtype, method):
        s = P.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, dtype, method=method)
        torch.cuda.synchronize()
        ts_ = time.perf_counter()
        d0 = WS.predict_shift(model, wl)          # feature pass + inference, inside the timing
        s.set_shift(d0)
        it, _ = s.run_scf(tol=1e-4, max_iter=300)
        torch.cuda.synchronize()
        sec = time.perf_counter() - ts_
        # the plain FP64 path judges the result: its energy at the converged shifts
        chk = P.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
        chk.H_on, _ = P.build_H(wl.model, chk.species, chk.nl, shift=s.shift, dtype="f64", H_on=chk.H_on,
                                H_bond=chk.H_bond)
        o = chk.run(float(np.sum(wl.n_elec)))
        du = abs(float(o["U_total"].item()) - u_p) / wl.n_atoms * 1e3
        rms = float(((s.shift - shift_p) ** 2).mean().sqrt())
        d0rms = float(((d0 - shift_p) ** 2).mean().sqrt())
        del s, chk
        return {"iterations": it, "seconds": sec, "energy_err_meV_per_atom": du, "shift_rms_vs_plain": rms,
                "initial_shift_rms": d0rms}

    w64 = warm("f64", "moments")
    log(f"warm FP64: {w64}")
    w32 = warm("f32", "lanczos")
    log(f"warm FP32 Lanczos: {w32}")
    best = w32 if (w32["seconds"] < w64["seconds"] and w32["energy_err_meV_per_atom"] <= 1.0) else w64
    res = {
        "metric": "s per converged SCF", "value": best["seconds"], "unit": "s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": best["seconds"] * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if best is w32 else "f64", "data": "synthetic",
        "config": {"workload": f"bcc A/B random alloy {args.reps_scf}^3 cells, {wl.n_atoms} atoms, a=2.87 A, "
                               f"eps_B=0.8 eV, N_d 6/5, d band cutoff 3.5 A, 16 moments, LCN SCF to max|q|<1e-4, "
                               f"MLP warm start",
                   "n_atoms": wl.n_atoms, "n_max": wl.n_max, "mix": 0.5},
        "plain_fp64": {"iterations": it_p, "seconds": t_p}, "broyden_fp64": broyden,
        "warm_fp64": w64, "warm_fp32_lanczos": w32,
        "speedup_vs_plain": t_p / best["seconds"],
        "mlp": {"train_structures": n_fit, "val_structures": len(train) - n_fit, "rows": int(x.shape[0]),
                "epochs": args.epochs, "val_rmse_eV": rmse, "train_seconds": t_train,
                "data_seconds": t_data, "train_iterations_mean": float(np.mean(its))},
    }
    res["roofline"] = hx_roofline(P, wl, "f32" if best is w32 else "f64", "lanczos" if best is w32 else "moments",
                                  torch)
    if not args.no_cpu:
        # the oracle's plain cycle from zero shifts on a small cell of the recipe
        res["cpu_baseline"] = cpu_baseline_scf(W.bcc_alloy_scf(seed=5, reps=4), "linear", wl.n_atoms)
    print(json.dumps(res), flush=True)


def bench_precision(args, torch, P, W):
    """Precision form: fcc A/B alloy 30^3 (108,000 atoms), s,p,d blocks with
    exponential bond integrals, cutoff 4.2 A, 20 moments: FP64 / FP32 / BF16
    H.X, moments and Lanczos forms, and Lanczos with FP16 vector storage;
    energy error against the FP64 path."""
    import oracle as O
    wl = W.fcc_alloy_spd(reps=args.reps_spd)
    ne = float(np.sum(wl.n_elec))
    out = {}
    ref = None
    for method, dtype in (("moments", "f64"), ("moments", "f32"), ("moments", "bf16"),
                          ("lanczos", "f64"), ("lanczos", "f32"), ("lanczos", "bf16"), ("lanczos", "f16")):
        p = P.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, dtype, method=method)
        t_step, t_k, o = timed_steps(p, ne, args.steps, 1, torch)
        u = float(o["U_total"].item())
        rec = {"ms_per_step": t_step * 1e3, "hx_ms": t_k, "U_eV_per_atom": u / wl.n_atoms,
               "atom_moments_per_s": wl.n_atoms * wl.n_max / t_step,
               "flagged_rows": int((p.rec["flags"] & ~4).ne(0).sum().item())}
        if ref is None:
            ref = (u, o["N_atom"].clone(), p.mu.clone())
        else:
            rec["energy_err_meV_per_atom"] = abs(u - ref[0]) / wl.n_atoms * 1e3
            rec["max_N_err"] = float((o["N_atom"] - ref[1]).abs().max())
        out[f"{method}_{dtype}"] = rec
        log(f"{method} {dtype}: {rec}")
        del p
    # FP64 moments of a seeded sample against the oracle
    sel = np.sort(np.random.default_rng(17).choice(wl.n_atoms, size=64, replace=False)).astype(np.int32)
    nl = O.neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    H_on, H_b = O.build_H(wl.model, wl.species, nl)
    t = time.perf_counter()
    mu_o = O.moments(nl, H_on, H_b, wl.n_max, sel)
    t_o = time.perf_counter() - t
    mu_g = ref[2][torch.as_tensor(sel, device=ref[2].device)].cpu().numpy()
    rel = float(np.max(np.abs(mu_g - mu_o) / np.maximum(np.abs(mu_o), 1e-12 * np.abs(mu_o).max())))
    best = min((v for k, v in out.items() if v.get("energy_err_meV_per_atom", 9) <= 1.0 and k != "moments_f64"),
               key=lambda v: v["ms_per_step"], default=out["moments_f64"])
    bname = [k for k, v in out.items() if v is best][0]
    res = {
        "metric": "atom-moments/s", "value": best["atom_moments_per_s"], "unit": "atom-moments/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": best["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": bname.split("_")[1], "data": "synthetic",
        "config": {"workload": f"fcc A/B alloy {args.reps_spd}^3 cells, {wl.n_atoms} atoms, a=3.5355 A, s,p,d "
                               f"Slater-Koster blocks, exponential bond integrals, cutoff 4.2 A, 20 moments; "
                               f"fastest form within 1 meV/atom of FP64: {bname}",
                   "n_atoms": wl.n_atoms, "n_max": wl.n_max},
        "forms": out,
        "roofline": None,
        "fp64_vs_oracle_sample": {"atoms": 64, "max_rel_err_moments": rel},
        "cpu_baseline": {"value": 64 * wl.n_max / t_o, "unit": "atom-moments/s", "cores": O.num_threads(),
                         "kind": "oracle", "sample": "64 seeded atoms, FP64 moments only"},
    }
    # the chosen form's H.X pass against the peak of its dtype, exact supports
    fpa = algorithmic_flops_per_atom(nl["row_ptr"], nl["nbr_j"], 9, wl.n_max,
                                     np.random.default_rng(7).choice(wl.n_atoms, 4, replace=False))
    flops = float(fpa.mean()) * wl.n_atoms
    dt = bname.split("_")[1]
    ach = flops / (best["hx_ms"] * 1e-3) / 1e12
    res["roofline"] = {"bound": "mfma" if dt == "bf16" else "alu", "achieved": ach, "peak": PEAK_TFLOPS[dt],
                       "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS[dt], "traffic": None,
                       "kernel": f"H.X launches of one {bname} pass (9 orbitals)", "kernel_ms": best["hx_ms"],
                       "algorithmic_flops_per_launch": flops, "flops_per_atom": float(fpa.mean())}
    print(json.dumps(res), flush=True)


def bench_radius(args, torch, P, W):
    """Maximum path radius (Sec. III "Speed-ups" (iii)) on the headline
    workload, FP32 Lanczos: step time and energy error against the paths of
    every length, per radius."""
    wl = W.bcc_large(reps=args.reps)
    ne = float(wl.n_elec.sum())
    full = P.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f32", method="lanczos")
    t0, k0, o0 = timed_steps(full, ne, args.steps, 1, torch)
    ref = {k: v.clone() for k, v in o0.items()}
    rows0 = full.plan.rows_cap
    del full
    forms = {}
    for r_max in (7.0, 10.0, 13.0, 16.0, 19.0):
        p = P.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f32", method="lanczos",
                         r_max=r_max)
        t, k, o = timed_steps(p, ne, args.steps, 1, torch)
        du = abs(float(o["U_total"].item()) - float(ref["U_total"].item())) / wl.n_atoms * 1e3
        forms[f"{r_max:g}"] = {"ms_per_step": t * 1e3, "hx_ms": k, "rows_cap": p.plan.rows_cap,
                               "energy_diff_meV_per_atom": du,
                               "max_atom_U_diff_eV": float((o["U_atom"] - ref["U_atom"]).abs().max()),
                               "atom_moments_per_s": wl.n_atoms * wl.n_max / t,
                               "diverging_rows": int(((p.rec["flags"] & 16) != 0).sum().item())}
        log(f"r_max {r_max}: {forms[f'{r_max:g}']}")
        del p
    within = [kv for kv in forms.items() if kv[1]["energy_diff_meV_per_atom"] <= 1.0]
    # the fastest radius within 1 meV/atom of all paths, else the widest one
    best = min(within, key=lambda kv: kv[1]["ms_per_step"]) if within else list(forms.items())[-1]
    res = {"metric": "atom-moments/s", "value": best[1]["atom_moments_per_s"], "unit": "atom-moments/s",
           "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": best[1]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": (f"bcc {args.reps}^3 ({wl.n_atoms} atoms), 18 moments, FP32 Lanczos, maximum "
                                   f"path radius {best[0]} A ("
                                   + ("the fastest within 1 meV/atom of all paths)" if within else
                                      "none tested is within 1 meV/atom of all paths; the widest)")),
                      "n_atoms": wl.n_atoms, "n_max": wl.n_max},
           "all_paths": {"ms_per_step": t0 * 1e3, "hx_ms": k0, "rows_cap": rows0}, "radii": forms}
    # the chosen radius's H.X pass against the FP32 peak, on exact per-atom
    # supports restricted to the radius
    nlc = P.build_neighbours(torch.as_tensor(np.asarray(wl.pos, float), device="cuda"), wl.cell, wl.model["r_cut"])
    rp, nj = nlc.row_ptr.cpu().numpy(), nlc.nbr_j.cpu().numpy()
    r_b = float(best[0])
    fpa = algorithmic_flops_per_atom_radius(np.asarray(wl.pos, float), wl.cell, rp, nj, 5,
                                            wl.n_max, np.random.default_rng(7).choice(wl.n_atoms, 4, replace=False),
                                            r_b)
    flops = float(fpa.mean()) * wl.n_atoms
    ach = flops / (best[1]["hx_ms"] * 1e-3) / 1e12
    res["roofline"] = {"bound": "alu", "achieved": ach, "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                       "frac": ach / PEAK_TFLOPS["f32"], "traffic": None,
                       "kernel": f"k_step with a path radius of {best[0]} A (all H.X launches of one pass)",
                       "kernel_ms": best[1]["hx_ms"], "algorithmic_flops_per_launch": flops,
                       "flops_per_atom": float(fpa.mean())}
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(wl, r_max=r_b)
    print(json.dumps(res), flush=True)


def bench_md(args, torch, P, W):
    """Sec. III "Speed-ups" (ii): the alloy's charge-neutrality cycle along a
    seeded trajectory, each step started from the previous converged shifts
    (warm) or from zero (cold); linear and Broyden mixing, FP64; then the
    better mixer's warm run with the FP32 Lanczos form, judged by the FP64
    path's energy at its converged shifts."""
    wl = W.bcc_alloy_scf(reps=args.reps_md)
    traj = W.md_trajectory(wl, args.md_steps, step_sigma=0.02)
    res_m = {}
    for mixer in ("linear", "broyden"):
        out = {}
        for mode in ("cold", "warm"):
            s = P.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, "f64", mixer=mixer)
            its, secs = [], []
            for t, pos in enumerate(traj):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if t > 0:
                    s.set_positions(pos)
                if mode == "cold":
                    s.set_shift(np.zeros(wl.n_atoms))
                it, _ = s.run_scf(tol=1e-4, max_iter=300)
                torch.cuda.synchronize()
                its.append(it)
                secs.append(time.perf_counter() - t0)
            out[mode] = {"iterations": its, "seconds": secs, "total_s": float(np.sum(secs)),
                         "U_last_eV_per_atom": float(s.out["U_total"].item()) / wl.n_atoms}
            log(f"{mixer} {mode}: {out[mode]['iterations']} iterations, {out[mode]['total_s']:.2f} s")
            del s
        res_m[mixer] = out
    best = min((m for m in res_m), key=lambda m: res_m[m]["warm"]["total_s"])
    # the same warm run with the FP32 Lanczos form, judged by the FP64 path's
    # energy at its converged shifts of the last step
    s = P.SCFPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_elec, wl.n_exp, "f32", method="lanczos",
                  mixer=best)
    its, secs = [], []
    for t, pos in enumerate(traj):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if t > 0:
            s.set_positions(pos)
        it, _ = s.run_scf(tol=1e-4, max_iter=300)
        torch.cuda.synchronize()
        its.append(it)
        secs.append(time.perf_counter() - t0)
    chk = P.EnergyPath(traj[-1], wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
    chk.H_on, _ = P.build_H(wl.model, chk.species, chk.nl, shift=s.shift, dtype="f64", H_on=chk.H_on,
                            H_bond=chk.H_bond)
    o = chk.run(float(np.sum(wl.n_elec)))
    du = abs(float(o["U_total"].item()) / wl.n_atoms - res_m[best]["warm"]["U_last_eV_per_atom"]) * 1e3
    del s, chk
    w32 = {"iterations": its, "seconds": secs, "total_s": float(np.sum(secs)), "energy_err_meV_per_atom": du}
    log(f"{best} warm FP32 Lanczos: {its} iterations, {w32['total_s']:.2f} s, {du:.2e} meV/atom")
    use32 = w32["total_s"] < res_m[best]["warm"]["total_s"] and du <= 1.0
    tot = w32["total_s"] if use32 else res_m[best]["warm"]["total_s"]
    res = {"metric": "s per converged SCF", "value": tot / args.md_steps, "unit": "s",
           "n_gpus": 1, "steps": args.md_steps, "warmup": 0,
           "ms_per_step": tot / args.md_steps * 1e3, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if use32 else "f64", "data": "synthetic",
           "config": {"workload": f"bcc A/B alloy {args.reps_md}^3 cells ({wl.n_atoms} atoms), 16 moments, LCN SCF "
                                  f"to max|q|<1e-4 along {args.md_steps} seeded MD-like steps (0.02 A per step), "
                                  f"warm start from the previous step; {best} mixing"
                                  + ("; FP32 Lanczos form (FP64 tail)" if use32 else "; FP64"),
                      "n_atoms": wl.n_atoms, "n_max": wl.n_max},
           "mixers": res_m, "warm_fp32_lanczos": w32,
           "speedup_warm_vs_cold": res_m[best]["cold"]["total_s"] / res_m[best]["warm"]["total_s"]}
    res["roofline"] = hx_roofline(P, wl, "f32" if use32 else "f64", "lanczos" if use32 else "moments", torch)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline_scf(W.bcc_alloy_scf(reps=4), best, wl.n_atoms, traj_steps=3)
    print(json.dumps(res), flush=True)


def bench_magnetic(args, torch, P, W):
    """Collinear magnetism: ferromagnetic bcc (a = 2.87 A, 6.5 d electrons,
    Stoner I = 0.8 eV), 16 moments; the Stoner / charge-neutrality cycle from
    m = 1, with the FP64 moment route and the FP32 Lanczos form, which is
    judged by the FP64 path's energies at its converged state."""
    import workloads as W_
    rng = np.random.default_rng(9)
    pos, cell = W_.cubic_lattice("bcc", 2.87, args.reps_mag)
    pos = W_.displace(pos, cell, 0.03, rng)
    n = pos.shape[0]
    model = W_.canonical_d_model(3.5)
    spc = np.zeros(n, np.int32)
    n0 = np.full(n, 6.5)
    out = {}
    for method, dtype in (("moments", "f64"), ("lanczos", "f32")):
        p = P.MagneticPath(pos, cell, spc, model, 16, n0, [0.8], dtype=dtype, method=method)
        p.set_state(np.zeros(n), np.ones(n))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, hist = p.run_scf(mix=0.5, mix_m=0.8, max_iter=800)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        rec = {"iterations": it, "seconds": sec, "ms_per_iteration": sec / it * 1e3,
               "m_mean": float(p.moment.mean().item()), "U_bond_eV_per_atom": float(p.out["U_total"].item()) / n,
               "U_X_eV_per_atom": float(p.U_X.item()) / n, "shift": p.shift.clone(), "moment": p.moment.clone()}
        out[f"{method}_{dtype}"] = rec
        log(f"{method} {dtype}: {it} iterations, {sec:.2f} s, m {rec['m_mean']:.4f}")
        del p
    # the FP64 path at the FP32 cycle's converged state judges it
    r32 = out["lanczos_f32"]
    chk = P.MagneticPath(pos, cell, spc, model, 16, n0, [0.8], dtype="f64", method="moments")
    chk.set_state(r32["shift"], r32["moment"])
    chk.energy()
    e64 = (float(chk.out["U_total"].item()) + float(chk.U_X.item())) / n
    e32 = r32["U_bond_eV_per_atom"] + r32["U_X_eV_per_atom"]
    r32["energy_err_meV_per_atom"] = abs(e64 - e32) * 1e3
    ref = out["moments_f64"]
    r32["energy_diff_vs_f64_cycle_meV_per_atom"] = abs(
        (ref["U_bond_eV_per_atom"] + ref["U_X_eV_per_atom"]) - e32) * 1e3
    for v in out.values():
        v.pop("shift")
        v.pop("moment")
    best = "lanczos_f32" if (r32["seconds"] < ref["seconds"] and r32["energy_err_meV_per_atom"] <= 1.0) \
        else "moments_f64"
    res = {"metric": "s per converged SCF", "value": out[best]["seconds"], "unit": "s", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": out[best]["seconds"] * 1e3, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if best == "lanczos_f32" else "f64", "data": "synthetic",
           "config": {"workload": f"collinear ferromagnetic bcc {args.reps_mag}^3 ({n} atoms), a=2.87 A, sigma=0.03 A, "
                                  f"canonical d band, 6.5 d electrons, Stoner I=0.8 eV, 16 moments, Stoner/LCN cycle "
                                  f"from m=1 to max|q|,|dm|<1e-4",
                      "n_atoms": n, "n_max": 16},
           "forms": out}
    # one spin channel's pass is the non-magnetic pass over the same cell
    res["roofline"] = hx_roofline(P, W_.Workload("magnetic_bcc", pos, cell, spc, model, 16, 200, n0),
                                  "f32" if best == "lanczos_f32" else "f64",
                                  "lanczos" if best == "lanczos_f32" else "moments", torch)
    if not args.no_cpu:
        ps, cs = W_.cubic_lattice("bcc", 2.87, 4)
        ps = W_.displace(ps, cs, 0.03, np.random.default_rng(9))
        small = W_.Workload("magnetic_bcc", ps, cs, np.zeros(ps.shape[0], np.int32), model, 16, 200,
                            np.full(ps.shape[0], 6.5))
        res["cpu_baseline"] = cpu_baseline_scf(small, "magnetic", n, stoner=[0.8], mix_m=0.8)
    print(json.dumps(res), flush=True)


def bench_mlp(args, torch, P, W):
    """Warm-start network training: 6-64-64-1, minibatch Adam over 400,000
    seeded feature rows (standard normal; smooth seeded targets of the shift
    scale), batch 4,096; a step is one bop_mlp_train_step (row gather,
    forward, backward, Adam).  Then forward passes over all rows.  The
    roofline counts 2 (6*64 + 64*64 + 64) flops per row forward and three
    times that per training row against the FP32 matrix peak."""
    import oracle as O
    rng = np.random.default_rng(3)
    n, B, epochs = 400000, 4096, 10
    x = rng.normal(size=(n, 6))
    t = np.tanh(x @ rng.normal(size=6)) * 0.2
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    m = P.MLP(seed=0)
    m.train(xd, td, epochs=1, batch=B, lr=1e-3)          # warm-up epoch
    torch.cuda.synchronize()
    steps = epochs * (n // B)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    m.train(xd, td, epochs=epochs, batch=B, lr=1e-3)
    b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = a.elapsed_time(b) / steps
    loss, _ = m.grad(xd, td)
    y = P.mlp_forward(m.params, xd)
    torch.cuda.synchronize()
    a.record()
    for _ in range(10):
        y = P.mlp_forward(m.params, xd)
    b.record()
    torch.cuda.synchronize()
    ms_fwd = a.elapsed_time(b) / 10
    f_row = 2.0 * (6 * 64 + 64 * 64 + 64)
    ach = 3.0 * f_row * B / (ms_step * 1e-3) / 1e12
    res = {"metric": "training rows/s", "value": B / (ms_step * 1e-3), "unit": "rows/s", "n_gpus": 1,
           "steps": steps, "warmup": n // B, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": (f"6-64-64-1 tanh MLP, Adam (lr 1e-3), {n} seeded rows of 6 features, batch {B}, "
                                   f"{epochs} epochs"), "rows": n, "batch": B},
           "loss": float(loss.item()), "wall_s": wall, "forward_ms_all_rows": ms_fwd,
           "forward_rows_per_s": n / (ms_fwd * 1e-3),
           "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                        "frac": ach / PEAK_TFLOPS["f32"], "traffic": None,
                        "kernel": "one training step (row gather, forward and backward tiles on MFMA, gradients, "
                                  "Adam)", "kernel_ms": ms_step, "algorithmic_flops_per_launch": 3.0 * f_row * B}}
    if not args.no_cpu:
        # the oracle's NumPy step (forward, gradient, Adam) on the same rows
        r2 = np.random.default_rng(0)
        params = []
        for shp in P.MLP_SHAPES:
            lim = np.sqrt(6.0 / (shp[0] + shp[1])) if len(shp) == 2 else 0.0
            params.append(r2.uniform(-lim, lim, size=shp) if len(shp) == 2 else np.zeros(shp))
        mo = [np.zeros_like(q) for q in params]
        vo = [np.zeros_like(q) for q in params]
        k, tc = 0, time.perf_counter()
        while time.perf_counter() - tc < 5.0:
            idx = r2.integers(0, n, B)
            _, g = O.mlp_loss_grad(params, x[idx], t[idx])
            k += 1
            params, mo, vo = O.adam_step(params, g, mo, vo, k)
        sec = time.perf_counter() - tc
        res["cpu_baseline"] = {"value": k * B / sec, "unit": "rows/s", "cores": O.num_threads(), "kind": "oracle",
                               "sample": f"{k} training steps of batch {B} (NumPy forward, gradient and Adam)",
                               "seconds": round(sec, 2)}
    print(json.dumps(res), flush=True)


BW_OPTIONS = ("gershgorin", "lowest", "highest", "average", "average_highest", "minmax", "weighted")


def bench_terminators(args, torch, P, W):
    """Terminators and band-width estimates (App. B.5 options (i)-(v),
    Gershgorin, the weighted-average terminator of App. B.1) on the headline
    cell: the FP32 Lanczos coefficients once, then per option the tail
    (a_inf, b_inf, expansion coefficients, Fermi level, energies), timed live;
    energy differences to the Gershgorin estimate.  The tail is bound by the
    Fermi passes, each of which reads every row's expansion coefficients."""
    import oracle as O
    wl = W.bcc_large(reps=args.reps)
    ne = float(wl.n_elec.sum())
    p = P.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f32", method="lanczos")
    p.run(ne)
    torch.cuda.synchronize()
    # the tail ORs its conditions into the flags of the Lanczos pass, so each
    # option starts from the pass's own flags
    flags0 = p.rec["flags"].clone()
    R = wl.n_atoms * p.no
    forms = {}
    u_ref = None
    for mode in BW_OPTIONS:
        p.bw = mode
        p.rec["flags"].copy_(flags0)
        out = p.run_tail(ne)
        ts = []
        for _ in range(args.steps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            p.rec["flags"].copy_(flags0)
            a.record()
            out = p.run_tail(ne)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        u = float(out["U_total"].item()) / wl.n_atoms
        if u_ref is None:
            u_ref = u
        # an estimate that puts the band inside the chain's spectrum makes
        # the chain's expansion diverge (flag 16); its energies mean nothing
        div = int(((p.rec["flags"] & 16) != 0).sum().item())
        forms[mode] = {"tail_ms": float(np.median(ts)), "U_eV_per_atom": u if div == 0 else None,
                       "E_F": float(out["E_F"].cpu()[0]),
                       "dU_vs_gershgorin_meV_per_atom": abs(u - u_ref) * 1e3 if div == 0 else None,
                       "divergent_rows": div, "floor_rows": int(((p.rec["flags"] & 8) != 0).sum().item())}
        log(f"{mode}: {forms[mode]}")
    g = forms["gershgorin"]
    e_f = g["E_F"]
    n_pass = 16    # 64 halvings, four per pass
    bytes_f = n_pass * R * (wl.n_exp + 1) * 8.0
    res = {"metric": "orbital-tails/s", "value": R / (g["tail_ms"] * 1e-3), "unit": "orbital-tails/s",
           "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": g["tail_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": (f"bcc {args.reps}^3 ({wl.n_atoms} atoms, {R} orbital rows), 18 moments, "
                                   f"FP32 Lanczos coefficients, FP64 tail per terminator option"),
                      "n_atoms": wl.n_atoms, "n_max": wl.n_max, "n_exp": wl.n_exp},
           "roofline": {"bound": "hbm", "achieved": bytes_f / (g["tail_ms"] * 1e-3) / 1e9, "peak": PEAK_HBM_TBPS * 1e3,
                        "unit": "GB/s", "frac": bytes_f / (g["tail_ms"] * 1e-3) / 1e12 / PEAK_HBM_TBPS,
                        "traffic": None, "kernel": "the tail (Gershgorin): its 16 Fermi passes' reads of the "
                                                   "expansion coefficients over the whole tail's time",
                        "kernel_ms": g["tail_ms"], "algorithmic_bytes_per_launch": bytes_f},
           "options": forms}
    del p
    if not args.no_cpu:
        # the oracle's tail per option on the moments of seeded atoms, at the
        # GPU's Fermi level (a bisection needs every atom)
        nl = O.neighbours(wl.pos, wl.cell, wl.model["r_cut"])
        H_on, H_b = O.build_H(wl.model, wl.species, nl)
        sel = np.sort(np.random.default_rng(123).choice(wl.n_atoms, 512, replace=False)).astype(np.int32)
        rows = O.moments(nl, H_on, H_b, wl.n_max, sel).reshape(-1, wl.n_max + 1)
        per = {}
        for mode in BW_OPTIONS:
            t = time.perf_counter()
            rec = O.recursion(rows, wl.n_max, bw=mode)
            gs = O.dos_coeffs(rows, rec, wl.n_max, wl.n_exp)
            O.energy(gs, rec["a_inf"], rec["b_inf"], H_on[sel], e_f)
            per[mode] = rows.shape[0] / (time.perf_counter() - t)
        res["cpu_baseline"] = {"value": per["gershgorin"], "unit": "orbital-tails/s", "cores": O.num_threads(),
                               "kind": "oracle", "per_option": per,
                               "sample": (f"the {rows.shape[0]} orbital rows of 512 seeded atoms: recursion from "
                                          f"the moments, terminator, expansion and energies at the GPU's Fermi "
                                          f"level (the moments themselves not timed)")}
    print(json.dumps(res), flush=True)


def algorithmic_force_flops_per_atom(row_ptr, nbr_j, n_max, sample):
    """Theta~ flops one atom's 5 columns need on exact supports (the
    diamond: X^l and G^k on the atoms within min(l, n - l) hops): per level,
    every kept row s and each neighbour t whose operand is kept costs one 5x5
    block times a column (50 flops), plus the onsite level (10); the backward
    passes add per (s, t) the outer product X^k[s] G^(k+1)[t] (50) contracted
    with the three symmetric derivative blocks (90)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import dijkstra
    n = row_ptr.shape[0] - 1
    A = sp.csr_matrix((np.ones(nbr_j.shape[0]), nbr_j, row_ptr), shape=(n, n))
    K = n_max // 2
    dist = dijkstra(A, indices=sample, unweighted=True, limit=K + 0.5)
    deg = np.diff(row_ptr)
    owner = np.repeat(np.arange(n), deg)
    out = []
    for d in dist:
        keep = np.isfinite(d[owner]) & np.isfinite(d[nbr_j])
        ds, dt = d[owner][keep], d[nbr_j][keep]
        f = 0.0
        for lev in range(1, n_max):           # forward X^lev
            Lc, Lp = min(lev, n_max - lev, K), min(lev - 1, n_max - lev + 1, K)
            f += 50 * np.count_nonzero((ds <= Lc) & (dt <= Lp)) + 10 * np.count_nonzero(d <= Lc)
        for lev in range(n_max - 1, -1, -1):  # backward G^lev and the contraction
            Lc, Lg = min(lev, n_max - lev, K), min(lev + 1, n_max - lev - 1, K)
            v = np.count_nonzero((ds <= Lc) & (dt <= Lg))
            f += 140 * v + ((50 * v + 10 * np.count_nonzero(d <= Lc)) if lev >= 1 else 0)
        out.append(5 * f)
    return np.asarray(out)


def bench_forces(args, torch, P, W):
    """Energy and forces of the headline cell: the FP64 moment path (its
    moments feed the weights), the weights, the block derivatives and the
    Theta~ passes with FP32 or FP64 vectors; the metric counts atoms whose
    energy and forces one step delivers."""
    wl = W.bcc_large(reps=args.reps)
    ne = float(wl.n_elec.sum())
    vec = "f32" if args.dtype in ("f32", "f16", "bf16") else "f64"
    p = P.EnergyPath(wl.pos, wl.cell, wl.species, wl.model, wl.n_max, wl.n_exp, "f64")
    stream = torch.cuda.current_stream()

    def setup():
        p.rebuild()
        if vec == "f64":
            return p.plan, p.mws, p.H_bond
        _, H32 = P.build_H(wl.model, p.species, p.nl, dtype="f32")
        plan32 = P.moments_plan(p.n, 5, wl.n_max, "f32", p.nl)
        return plan32, P.moments_prepare(plan32, p.nl), H32

    plan, mws, Hb = setup()
    fws = P.forces_workspace(plan, p.nl)
    log(f"forces bcc {args.reps}^3: {wl.n_atoms} atoms, n_max {wl.n_max}, vectors {vec}, rows_cap {plan.rows_cap}, "
        f"force workspace {fws.numel() / 2**30:.2f} GiB")

    def one():
        out = p.run(ne)
        w = P.weights(p.mu, p.H_on, out["E_F"], wl.n_max, wl.n_exp)
        dH = P.bond_derivatives(wl.model, p.species, p.nl)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        F = P.forces(plan, mws, p.nl, p.H_on, Hb, dH, w, ws=fws)
        b.record(stream)
        return out, F, (a, b)

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = []
    for _ in range(args.steps):
        out, F, ev = one()
        evs.append(ev)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    kms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    Fn = F.cpu().numpy()
    rp = p.nl.row_ptr.cpu().numpy()
    nj = p.nl.nbr_j.cpu().numpy()
    sample = np.random.default_rng(7).choice(wl.n_atoms, size=4, replace=False)
    fpa = algorithmic_force_flops_per_atom(rp, nj, wl.n_max, sample)
    flops = float(fpa.mean()) * wl.n_atoms
    achieved = flops / (kms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[vec]
    res = {"metric": "atom-forces/s", "value": wl.n_atoms / t, "unit": "atoms/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": vec, "data": "synthetic",
           "config": {"workload": f"bcc {args.reps}^3 supercell, {wl.n_atoms} atoms, a=3.16 A, sigma=0.08 A, "
                                  f"canonical d band, cutoff 3.8 A, {wl.n_max} moments, N_d=4.5: energy (FP64 "
                                  f"moments) and forces ({vec} Theta~ vectors)",
                      "n_atoms": wl.n_atoms, "n_max": wl.n_max, "rows_cap": plan.rows_cap},
           "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                        "frac": achieved / peak, "traffic": read_traffic(vec, "forces", "forces.hip"),
                        "kernel": "force passes (k_finit, k_fstep forward and backward, all batches)",
                        "kernel_ms": kms, "algorithmic_flops_per_launch": flops,
                        "flops_per_atom": float(fpa.mean())},
           "sum_F": float(np.abs(Fn.sum(axis=0)).max()), "max_abs_F": float(np.abs(Fn).max()),
           "U_eV_per_atom": float(out["U_total"].item()) / wl.n_atoms}
    if res["roofline"]["traffic"]:
        res["roofline"]["achieved_hbm_TBps"] = res["roofline"]["traffic"] / (kms * 1e-3) / 1e12
        res["roofline"]["hbm_frac"] = res["roofline"]["achieved_hbm_TBps"] / PEAK_HBM_TBPS
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline_forces(W)
    log(f"forces: {t * 1e3:.1f} ms/step, force passes {kms:.1f} ms, {achieved:.2f} TFLOP/s")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

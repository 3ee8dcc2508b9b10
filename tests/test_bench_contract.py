"""CPU-side checks of bench.py's contract: it refuses more than one GPU with a
message, and the committed bench line for the headline workload carries every
field of the JSON line, the roofline object and the timed oracle baseline.
No kernel is launched."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == ""          # no JSON line for a configuration it does not run


def test_committed_bench_line_has_every_field():
    j = json.load(open(os.path.join(ROOT, "profiles", "bench_bcc_large_f32.json")))
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in j, key
    assert j["metric"] == j["unit"] == "atom-moments/s"
    assert j["n_gpus"] == 1 and j["higher_is_better"] is True and j["data"] == "synthetic"
    assert "workload" in j["config"] and j["config"]["n_atoms"] == 128000 and j["config"]["n_max"] == 18
    # value is atom-moments per second of one whole step
    assert abs(j["value"] - 128000 * 18 / (j["ms_per_step"] * 1e-3)) < 1e-6 * j["value"]
    r = j["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in r, key
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    assert abs(r["achieved"] - r["algorithmic_flops_per_launch"] / (r["kernel_ms"] * 1e-3) / 1e12) < 1e-9 * r["achieved"]
    c = j["cpu_baseline"]
    for key in ("value", "unit", "cores", "kind", "sample"):
        assert key in c, key
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["unit"] == j["unit"]


def test_committed_bench_line_states_its_accuracy():
    """The headline form carries its own per-atom accuracy against the FP64
    path, and it meets the FP32 bar (1e-5 relative on every atom's N and U);
    the faster FP32 moment form is reported beside it with its own error."""
    j = json.load(open(os.path.join(ROOT, "profiles", "bench_bcc_large_f32.json")))
    acc = j["accuracy_vs_f64"]
    assert acc["bar"] == 1e-5
    assert max(acc["max_atom_rel_err"].values()) < acc["bar"]
    assert j["config"]["method"] == "lanczos" and j["dtype"] == "f32"
    m = j["moments_f32_path"]
    assert m["meets_fp32_bar"] == (max(m["max_atom_rel_err"].values()) < 1e-5)
    r = j["roofline"]
    if r["traffic"]:
        assert abs(r["achieved_hbm_TBps"] - r["traffic"] / (r["kernel_ms"] * 1e-3) / 1e12) < 1e-9


def test_radius_flop_count_reduces_to_the_unrestricted_one():
    """The path-radius roofline's work count: with a radius beyond every
    support it equals the unrestricted count atom by atom, and a radius below
    the supports' extent removes work."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    import oracle as O
    import workloads as W
    wl = W.bcc_large(reps=6)
    nl = O.neighbours(wl.pos, wl.cell, wl.model["r_cut"])
    smp = np.array([0, 7, 100])
    full = bench.algorithmic_flops_per_atom(nl["row_ptr"], nl["nbr_j"], 5, wl.n_max, smp)
    wide = bench.algorithmic_flops_per_atom_radius(wl.pos, wl.cell, nl["row_ptr"], nl["nbr_j"], 5, wl.n_max, smp,
                                                   1e3)
    small = bench.algorithmic_flops_per_atom_radius(wl.pos, wl.cell, nl["row_ptr"], nl["nbr_j"], 5, wl.n_max, smp,
                                                    7.0)
    np.testing.assert_array_equal(wide, full)
    assert np.all(small < full) and np.all(small > 0)
    # odd n_max adds the last product on the K-hop support; the same identity holds
    f17 = bench.algorithmic_flops_per_atom(nl["row_ptr"], nl["nbr_j"], 5, 17, smp)
    w17 = bench.algorithmic_flops_per_atom_radius(wl.pos, wl.cell, nl["row_ptr"], nl["nbr_j"], 5, 17, smp, 1e3)
    np.testing.assert_array_equal(w17, f17)

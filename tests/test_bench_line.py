"""The benchmark's stdout line (CPU only): built from a canned result of a
full run with every report, it must parse, carry the headline, roofline and
CPU-baseline fields, and stay far below what a log tail keeps."""
import json
import tempfile

import numpy as np

import bench
import oracle
import synth


def _canned():
    spmv = {"height": 32, "schedule": "colblock4", "ms": 0.15123, "gbs_plus": 1449.9, "eta_plus": 0.1812,
            "eta_minus": 0.2877, "gflops": 221.9, "cold_ms": 0.15234, "cold_eta_plus": 0.1799}
    ex = {
        "selector": {"this_workload": {"tune_ratio": 1.0, "predicted": "h32_colblock4", "exhaustive_best": "h32_colblock4"},
                     "fresh": {"regret": 0.0098, "regret_default_h8_group": 0.08},
                     "held_out": {"regret": 0.0243}},
        "precision": {**{dt: {"height": 16, "schedule": "split", "spmv_cold_ms": 0.1394, "gbs_plus": 1356.2, "frac_of_hbm_peak": 0.1695,
                           "max_err_over_bound": 0.238, "rows_over_bound": 0, "extra": list(range(50))}
                         for dt in ("f64", "f32", "bf16")},
                      "ceiling_f64": {"stream_read_gbs": 6012.3, "stream_read_ms": 0.02601, "random_gathers_ms": 0.1234,
                                      "own_column_gathers_ms": 0.0712}},
        "residual": {f"{low}_inner_{r}_residual": {"final_rel_err": 1.234e-16, "rel_err_every_5": [1e-3] * 4}
                     for low in ("f32", "bf16") for r in ("f64", low)},
        "batched": {dt: {"graph_persistent_ms": 6.896, "separate_launches_ms": 7.505, "speedup_vs_separate": 1.088,
                         "frac_of_hbm_peak": 0.2825, "tuning": {"tile_nnz": 32768}} for dt in ("f64", "f32")},
        "structured": {k: {"f64": {"eta_plus": 0.57}, "f32": {"eta_plus": 0.7}} for k in ("stencil27", "band_bw40")},
        "padded": {f"h{h}": {"memory_overhead": 0.123, "speedup_vs_best_plain": 0.8, "padded_nnz": 1} for h in (8, 16, 32)},
        "padded_small_mu": {k: {"mu": 1.0, "best_plain": {"height": 8, "variant": "auto", "cold_ms": 0.05},
                                "padded_h8": {"cold_ms": 0.06, "memory_overhead": 2.1, "speedup_vs_best_plain": 0.8},
                                "padded_h16": {"cold_ms": 0.06, "memory_overhead": 3.1, "speedup_vs_best_plain": 0.7}}
                            for k in ("permutation", "poisson2", "poisson4", "laplace2d_1024")},
        "model": {"mu": 16.0, "rows": [{"dtype": dt, "height": h, "a_lambda128_b4": 1.5, "a_lambda64_b4": 1.2,
                                        "a_lambda128_bval": 1.3, "measured_wave": 1.4, "measured_best": 1.6}
                                       for dt in ("f64", "f32") for h in (1, 2, 4, 8, 16, 32)]},
    }
    return {
        "metric": bench.METRIC, "value": 1449.9, "unit": "GB/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "ms_per_step": 0.81234, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "poisson16 n=1048576: row lengths max(1,Poisson(16)), distinct uniform columns, "
                               "N(0,1) values and x, seed 0", "rows": 1048576, "nnz": 16780095,
                   "value_is": "SpMV beta+ GB/s (Eq. 6.1) in the timed steps; a step is CSR->CMRS sorted + SpMV + "
                               "CMRS->CSR"},
        "roofline": {"bound": "hbm", "kernel": "SpMV f64 h=32 colblock4", "achieved": 1449.9, "peak": 8000.0,
                     "unit": "GB/s", "frac": 0.1812, "traffic": 1330000000, "alg_bytes_per_launch": 219268000,
                     "launch_ms": 0.15123},
        "cpu_baseline": {"value": 9.5, "unit": "GB/s", "cores": 16, "kind": "oracle",
                         "sample": "CSR y=Ax, fp64, the full 1048576-row workload matrix, 11 calls, longest dropped, "
                                   "mean of 10; beta+ of the CSR arrays (223469000 B)",
                         "ms": 23.5, "ms_std": 0.4, "serial": {"value": 2.1, "cores": 1, "ms": 105.0, "ms_std": 1.0},
                         "cpu_model": "AMD EPYC 9575F 64-Core Processor", "os_cpu_count": 256,
                         "build": "gcc -O3 -march=native -ffp-contract=off -fopenmp", "parallel_equals_serial_bits": True},
        "spmv": {"f64": spmv, "f32": dict(spmv)},
        "step": {"f64": {"ms": 0.812, "gbs": 2583.0, "calls": "from_csr_sorted + colblock_plan + spmv + to_csr"},
                 "f32": {"ms": 0.7, "gbs": 2000.0},
                 "kernels_f64_ms": {"from_csr_sorted": 0.44, "colblock_plan": 0.03, "spmv": 0.151, "to_csr": 0.16}},
        "ceiling": {"stream_read_gbs": 6219.5, "gathers_per_s": 106.3, "gather_floor_over_spmv": 0.86},
        "extras": ex, "detail_file": "bench_detail.json",
    }


def test_line_is_short_and_complete():
    txt = bench.compact_line(_canned())
    assert len(txt) < 4000, len(txt)
    assert "\n" not in txt
    d = json.loads(txt)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert set(d["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert set(d["cpu_baseline"]) >= {"value", "unit", "cores", "kind", "sample"}
    assert d["roofline"]["frac"] == round(d["roofline"]["achieved"] / d["roofline"]["peak"], 4)
    assert set(d["reports"]) == {"selector", "precision_zipf", "batched", "structured", "padded", "model_eq52_f64",
                                 "residual_refinement", "padded_small_mu"}
    assert "extras" not in d and "sweep" not in d


def test_line_refuses_to_grow():
    r = _canned()
    r["config"]["workload"] = "x" * 5000
    try:
        bench.compact_line(r)
    except ValueError:
        return
    raise AssertionError("an oversized line was printed")


def test_baseline_build_matches_oracle_bits():
    """The CPU-baseline build (-O3 -march=native -fopenmp) of the oracle gives
    the test build's y bit for bit, serially and over 1..8 threads."""
    lib = oracle._load(oracle.build_baseline(tempfile.mkdtemp(prefix="cmrs_cpu_test_")))
    A = synth.random_csr(3000, 2500, max_row=40, seed=5)
    x = synth.normal_vector(A.cols, seed=6)
    ref = oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x)
    assert np.array_equal(oracle.csr_spmv(A.row_ptr, A.col_ind, A.val, x, lib=lib).view(np.uint64), ref.view(np.uint64))
    for t in (1, 2, 3, 8):
        y, used = oracle.csr_spmv_par(A.row_ptr, A.col_ind, A.val, x, t, lib=lib)
        assert 1 <= used <= t
        assert np.array_equal(y.view(np.uint64), ref.view(np.uint64))
    E = synth.Csr(5, 3, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0))
    y, _ = oracle.csr_spmv_par(E.row_ptr, E.col_ind, E.val, np.ones(3), 4, lib=lib)
    assert np.all(y == 0)


def test_line_drops_reports_before_growing():
    r = _canned()
    r["extras"]["structured"] = {f"m{i}": {"f64": {"eta_plus": 0.5}, "f32": {"eta_plus": 0.6}} for i in range(60)}
    txt = bench.compact_line(r)
    assert len(txt) <= bench.LINE_SOFT_LIMIT, len(txt)
    d = json.loads(txt)
    assert "structured" not in d.get("reports", {})
    assert "precision_zipf" in d["reports"] and "batched" in d["reports"]

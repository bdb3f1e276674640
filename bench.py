"""Benchmark of the CMRS hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--height H] [--dtype f64|f32]

Workload: square n = 2^20 matrix, row lengths max(1, Poisson(16)), distinct
uniform columns, N(0,1) values and x (seeded, synthetic).  One step is one
pass of the whole hot path over it: CSR -> CMRS with the in-strip reorder,
y = A x, CMRS -> CSR, every buffer preallocated and resident in HBM.

Before the timed steps the SpMV alone is characterised for every strip height
1..32, fp64 and fp32, both kernel variants, with the paper's protocol (11 calls,
the longest dropped, mean and std of the rest; Sec. 6.3), cold (L2 and MALL
flushed by a 1 GiB write before each call) and warm (back to back).  Unless
--height is given, the timed steps use the height with the best cold fp64 SpMV
time.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CMRS SpMV GB/s & % HBM roofline (FP64/FP32); learned-vs-exhaustive tune ratio"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--height", type=int, default=0, help="strip height for the timed steps (0: best from sweep)")
    p.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    p.add_argument("--no-sweep", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--rows", type=int, default=1 << 20)
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the CMRS path here is single-GPU; multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    if os.environ.get("WORLD_SIZE", "1") not in ("", "1"):
        print("bench.py is single-process; WORLD_SIZE > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1203_2946_amd import cmrs, model

    assert torch.cuda.is_available(), "needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    props = torch.cuda.get_device_properties(dev)
    log("device", props.name, getattr(props, "gcnArchName", ""), "CUs", props.multi_processor_count)

    t0 = time.time()
    A = synth.poisson_rows(args.rows, 16.0, seed=0)
    x64 = synth.normal_vector(A.cols, seed=1)
    log(f"matrix {A.name}: rows={A.rows} nnz={A.nnz} ({time.time() - t0:.1f}s)")

    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col_ind).to(dev)
    v64 = torch.from_numpy(A.val).to(dev)
    v32 = v64.float()
    x_d = {"f64": torch.from_numpy(x64).to(dev), "f32": torch.from_numpy(x64).to(dev).float()}
    v_d = {"f64": v64, "f32": v32}
    flush_buf = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def flush():
        flush_buf.fill_(1)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def protocol(fn, cold: bool, reps: int = 11):
        """Sec. 6.3: 11 calls, drop the longest, mean and std of the other 10."""
        pairs = []
        for _ in range(reps):
            if cold:
                flush()
            s, e = ev(), ev()
            s.record(stream)
            fn()
            e.record(stream)
            pairs.append((s, e))
        torch.cuda.synchronize()
        t = sorted(s.elapsed_time(e) for s, e in pairs)[:-1]
        return float(np.mean(t)), float(np.std(t)), float(np.median(t))

    sizes = {"f64": (8, 8, 8), "f32": (4, 4, 4)}

    def spmv_bytes(M, dt):
        s_v, s_x, s_y = sizes[dt]
        return (model.beta_plus(M.nnz, M.rows, M.cols, M.strips, s_v, s_x, s_y),
                model.beta_minus(M.nnz, M.rows, M.cols, M.strips, s_v, s_x, s_y))

    # ---------------------------------------------------------------- sweep
    sweep = []
    if not args.no_sweep:
        for dt in ("f64", "f32"):
            for h in (1, 2, 4, 8, 16, 32):
                M = cmrs.from_csr(rp, ci, v_d[dt], A.cols, h, sort=True)
                y = torch.empty(A.rows, dtype=x_d[dt].dtype, device=dev)
                bp, bm = spmv_bytes(M, dt)
                for var in ("lds", "reg"):
                    if var == "reg" and h > 8:
                        continue
                    fn = lambda: cmrs.spmv(M, x_d[dt], out=y, variant=var)  # noqa: E731
                    fn()
                    cm, cs, cmed = protocol(fn, cold=True)
                    wm, ws, _ = protocol(fn, cold=False)
                    row = {"dtype": dt, "height": h, "variant": var, "cold_ms": round(cm, 5),
                           "cold_std_ms": round(cs, 5), "warm_ms": round(wm, 5),
                           "gbs_plus_cold": round(bp / cm / 1e6, 1), "eta_plus_cold": round(bp / cm / 1e6 / HBM_PEAK_GBS, 4),
                           "gbs_minus_cold": round(bm / cm / 1e6, 1),
                           "gflops_cold": round(model.flops(M.nnz, M.rows) / cm / 1e6, 1),
                           "gbs_plus_warm": round(bp / wm / 1e6, 1)}
                    sweep.append(row)
                    log(f"sweep {dt} h={h:2d} {var}: cold {cm * 1e3:7.1f} us ({row['gbs_plus_cold']:7.1f} GB/s, "
                        f"eta+ {row['eta_plus_cold']:.3f})  warm {wm * 1e3:7.1f} us")
                del M, y

    dt = args.dtype
    if args.height:
        h = args.height
    elif sweep:
        best = min((r for r in sweep if r["dtype"] == dt and r["variant"] == "lds"), key=lambda r: r["cold_ms"])
        h = best["height"]
    else:
        h = 8
    log(f"timed steps: dtype={dt} height={h}")

    # ---------------------------------------------------------------- timed steps
    vv = v_d[dt]
    M = cmrs.from_csr(rp, ci, vv, A.cols, h, sort=True)
    ws_bytes = cmrs.from_csr_workspace_bytes(A.rows, A.nnz, h, True)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    y = torch.empty(A.rows, dtype=x_d[dt].dtype, device=dev)
    rp2 = torch.empty_like(rp)
    ci2 = torch.empty_like(ci)
    v2 = torch.empty_like(vv)
    xx = x_d[dt]

    def step(evs=None):
        if evs is not None:
            evs[0].record(stream)
        cmrs.from_csr(rp, ci, vv, A.cols, h, sort=True, workspace=ws, out=M)
        if evs is not None:
            evs[1].record(stream)
        cmrs.spmv(M, xx, out=y)
        if evs is not None:
            evs[2].record(stream)
        cmrs.to_csr(M, out=(rp2, ci2, v2))
        if evs is not None:
            evs[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    all_evs = [[ev() for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(all_evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / args.steps
    seg = np.array([[e[k].elapsed_time(e[k + 1]) for k in range(3)] for e in all_evs])
    seg_ms = seg.mean(axis=0)

    s_v = sizes[dt][0]
    b_from = model.from_csr_bytes(A.nnz, A.rows, M.strips, s_v)
    b_spmv, b_spmv_minus = spmv_bytes(M, dt)
    b_to = model.to_csr_bytes(A.nnz, A.rows, M.strips, s_v)
    b_step = b_from + b_spmv + b_to
    value = b_step / (ms_per_step * 1e-3) / 1e9
    kern = {
        "from_csr_sorted": {"ms": round(float(seg_ms[0]), 5), "alg_bytes": b_from,
                            "gbs": round(b_from / seg_ms[0] / 1e6, 1)},
        "spmv": {"ms": round(float(seg_ms[1]), 5), "alg_bytes": b_spmv,
                 "gbs": round(b_spmv / seg_ms[1] / 1e6, 1)},
        "to_csr": {"ms": round(float(seg_ms[2]), 5), "alg_bytes": b_to, "gbs": round(b_to / seg_ms[2] / 1e6, 1)},
    }
    dom_name = max(kern, key=lambda k: kern[k]["ms"])
    dom = kern[dom_name]
    ach = dom["alg_bytes"] / dom["ms"] / 1e6
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    log(f"step {ms_per_step * 1e3:.1f} us (events: from {seg_ms[0] * 1e3:.1f}, spmv {seg_ms[1] * 1e3:.1f}, "
        f"to {seg_ms[2] * 1e3:.1f} us) -> {value:.1f} GB/s")

    # SpMV alone at the chosen height (cold, paper protocol)
    fn = lambda: cmrs.spmv(M, xx, out=y)  # noqa: E731
    cm, cs, cmed = protocol(fn, cold=True)
    wm, wsd, _ = protocol(fn, cold=False)
    spmv = {"height": h, "dtype": dt, "cold_ms": round(cm, 5), "cold_std_ms": round(cs, 5), "warm_ms": round(wm, 5),
            "beta_plus_bytes": b_spmv, "beta_minus_bytes": b_spmv_minus,
            "gbs_plus_cold": round(b_spmv / cm / 1e6, 1), "eta_plus_cold": round(b_spmv / cm / 1e6 / HBM_PEAK_GBS, 4),
            "gbs_minus_cold": round(b_spmv_minus / cm / 1e6, 1),
            "eta_minus_cold": round(b_spmv_minus / cm / 1e6 / HBM_PEAK_GBS, 4),
            "gflops_cold": round(model.flops(A.nnz, A.rows) / cm / 1e6, 1),
            "gbs_plus_warm": round(b_spmv / wm / 1e6, 1)}

    # ---------------------------------------------------------------- CPU oracle baseline
    cpu = None
    if not args.no_cpu:
        import oracle
        hv = A.val if dt == "f64" else synth.round_to_f32(A.val)
        xs = x64 if dt == "f64" else synth.round_to_f32(x64).astype(np.float64)

        def cpu_step():
            sp_, w_, vo_ = oracle.csr_to_cmrs(A.row_ptr, A.col_ind, hv, A.cols, h, sorted_=True)
            oracle.csr_spmv(A.row_ptr, A.col_ind, hv.astype(np.float64), xs)
            oracle.cmrs_to_csr(sp_, w_, vo_, A.rows, h)

        t1 = time.perf_counter()
        cpu_step()
        first = time.perf_counter() - t1
        reps = max(1, min(8, int(15.0 / max(first, 1e-3))))
        t1 = time.perf_counter()
        for _ in range(reps):
            cpu_step()
        tc = (time.perf_counter() - t1) / reps
        cpu = {"value": round(b_step / tc / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the full workload matrix, one step (oracle CSR->CMRS sorted, CSR SpMV, CMRS->CSR) "
                         f"timed {reps}x after one untimed pass; {tc:.2f} s per step",
               "ms_per_step": round(tc * 1e3, 1)}
        log(f"cpu oracle: {tc:.2f} s/step -> {cpu['value']} GB/s")

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dt, "data": "synthetic",
        "config": {"workload": f"poisson16 n={A.rows} (row lengths max(1,Poisson(16)), distinct uniform columns, "
                               f"N(0,1) values and x, seed 0)", "rows": A.rows, "nnz": A.nnz, "height": h,
                   "sorted": True, "step": "from_csr(sorted) + spmv + to_csr", "alg_bytes_per_step": b_step},
        "roofline": roofline, "cpu_baseline": cpu, "spmv": spmv, "kernels": kern, "sweep": sweep,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the CMRS hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--height H] [--schedule S] [--dtype f64|f32]

Workload: square n = 2^20 matrix, row lengths max(1, Poisson(16)), distinct
uniform columns, N(0,1) values and x (seeded, synthetic).  One step is one
pass of the whole hot path over it: CSR -> CMRS with the in-strip reorder, the
SpMV y = A x (for the column-blocked schedules including the plan that
locates each strip's column-block runs), and CMRS -> CSR, with every buffer
preallocated and resident in HBM.

Before the timed steps every strip height 1..32 and SpMV schedule is measured
with the paper's protocol (11 calls, the longest dropped, mean and std of the
rest; Sec. 6.3), cold (L2 and MALL flushed by a 1 GiB write before each call)
and warm, for fp64 and fp32.  Unless --height / --schedule are given, the timed
steps use the (height, schedule) with the shortest fp64 step.

Prints one JSON line on stdout; progress goes to stderr.
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

METRIC = "CMRS SpMV GB/s & % HBM roofline (FP64/FP32); learned-vs-exhaustive tune ratio"
HBM_PEAK_GBS = 8000.0
SCHEDULES = {
    "group": ("auto", None),            # strip groups, non-temporal stream loads (library default)
    "wave": ("lds", None),              # one wave per strip, LDS partials (Algorithm 1 as printed)
    "colblock4": ("auto", 4),           # column-blocked, one launch, 4 blocks
    "colblock8": ("auto", 8),           # column-blocked, one launch, 8 blocks (one per XCD)
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--height", type=int, default=0, help="strip height of the timed steps (0: from the sweep)")
    p.add_argument("--schedule", choices=list(SCHEDULES), default=None)
    p.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    p.add_argument("--no-sweep", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--rows", type=int, default=1 << 20)
    return p.parse_args()


def kernel_source_hash() -> str:
    d = os.path.join(ROOT, "paper_1203_2946_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(kernel_tag: str):
    """HBM bytes per dispatch of `kernel_tag` from the committed counter
    summary (profiles/traffic.txt), or None if it was taken from other kernel
    sources than the ones built now."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    src = kernel_source_hash()
    for line in open(path):
        f = dict(kv.split("=", 1) for kv in line.split() if "=" in kv)
        if f.get("tag") == kernel_tag and f.get("src") == src:
            return int(f["fetch_bytes"]) + int(f["write_bytes"])
    return None


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
    v_d = {"f64": v64, "f32": v64.float()}
    x_d = {"f64": torch.from_numpy(x64).to(dev), "f32": torch.from_numpy(x64).to(dev).float()}
    flush_buf = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    sizes = {"f64": 8, "f32": 4}

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
        return float(np.mean(t)), float(np.std(t))

    class Pipeline:
        """Preallocated buffers of one (dtype, height, schedule) and its step."""

        def __init__(self, dt, h, sched):
            self.dt, self.h, self.sched = dt, h, sched
            self.variant, self.nb = SCHEDULES[sched]
            self.v = v_d[dt]
            self.x = x_d[dt]
            self.M = cmrs.from_csr(rp, ci, self.v, A.cols, h, sort=True)
            self.ws = torch.empty(max(1, cmrs.from_csr_workspace_bytes(A.rows, A.nnz, h, True)), dtype=torch.uint8,
                                  device=dev)
            self.y = torch.empty(A.rows, dtype=self.x.dtype, device=dev)
            self.out = (torch.empty_like(rp), torch.empty_like(ci), torch.empty_like(self.v))
            if self.nb:
                self.plan = cmrs.colblock_plan(self.M, self.nb)
                self.cws = torch.empty(max(1, cmrs.spmv_colblock_workspace_bytes(self.M, self.nb, "concurrent")),
                                       dtype=torch.uint8, device=dev)

        def convert(self):
            cmrs.from_csr(rp, ci, self.v, A.cols, self.h, sort=True, workspace=self.ws, out=self.M)

        def make_plan(self):
            if self.nb:
                d = self.M.desc()
                st = cmrs.lib.cmrs_colblock_plan(cmrs.ctypes.byref(d), self.nb, self.plan.split.data_ptr(),
                                                 self.plan.nbytes, stream.cuda_stream)
                cmrs._check(st, "cmrs_colblock_plan")

        def spmv(self):
            if self.nb:
                cmrs.spmv_colblock(self.M, self.plan, self.x, out=self.y, variant=self.variant,
                                   schedule="concurrent", workspace=self.cws)
            else:
                cmrs.spmv(self.M, self.x, out=self.y, variant=self.variant)

        def back(self):
            cmrs.to_csr(self.M, out=self.out)

        def bytes(self):
            s_v = sizes[self.dt]
            b_from = model.from_csr_bytes(A.nnz, A.rows, self.M.strips, s_v)
            b_plan = (4 * A.nnz + 4 * (self.M.strips + 1) + 4 * self.M.strips * (self.nb - 1)) if self.nb else 0
            bp = model.beta_plus(A.nnz, A.rows, A.cols, self.M.strips, s_v, s_v, s_v)
            bm = model.beta_minus(A.nnz, A.rows, A.cols, self.M.strips, s_v, s_v, s_v)
            b_to = model.to_csr_bytes(A.nnz, A.rows, self.M.strips, s_v)
            return b_from, b_plan, bp, bm, b_to

    # ---------------------------------------------------------------- sweep
    sweep = []
    if not args.no_sweep:
        for dt in ("f64", "f32"):
            for h in (1, 2, 4, 8, 16, 32):
                row_conv = None
                for sched in SCHEDULES:
                    P = Pipeline(dt, h, sched)
                    b_from, b_plan, bp, bm, b_to = P.bytes()
                    if row_conv is None:
                        tf, _ = protocol(P.convert, cold=True)
                        tt, _ = protocol(P.back, cold=True)
                        row_conv = (tf, tt)
                    tf, tt = row_conv
                    tp = protocol(P.make_plan, cold=True)[0] if P.nb else 0.0
                    P.spmv()
                    cm, cs = protocol(P.spmv, cold=True)
                    wm, _ = protocol(P.spmv, cold=False)
                    r = {"dtype": dt, "height": h, "schedule": sched, "spmv_cold_ms": round(cm, 5),
                         "spmv_cold_std_ms": round(cs, 5), "spmv_warm_ms": round(wm, 5),
                         "gbs_plus_cold": round(bp / cm / 1e6, 1), "eta_plus_cold": round(bp / cm / 1e6 / HBM_PEAK_GBS, 4),
                         "gbs_minus_cold": round(bm / cm / 1e6, 1),
                         "gflops_cold": round(model.flops(A.nnz, A.rows) / cm / 1e6, 1),
                         "from_csr_ms": round(tf, 5), "plan_ms": round(tp, 5), "to_csr_ms": round(tt, 5),
                         "step_ms": round(tf + tp + cm + tt, 5)}
                    sweep.append(r)
                    log(f"sweep {dt} h={h:2d} {sched:9s}: spmv cold {cm * 1e3:7.1f} us ({r['gbs_plus_cold']:7.1f} GB/s, "
                        f"eta+ {r['eta_plus_cold']:.3f}) warm {wm * 1e3:7.1f} us | step {r['step_ms'] * 1e3:7.1f} us")
                    del P

    dt = args.dtype
    cand = [r for r in sweep if r["dtype"] == dt]
    if args.height and args.schedule:
        h, sched = args.height, args.schedule
    elif cand:
        pool = [r for r in cand if (not args.height or r["height"] == args.height)
                and (not args.schedule or r["schedule"] == args.schedule)]
        best = min(pool, key=lambda r: r["step_ms"])
        h, sched = best["height"], best["schedule"]
    else:
        h, sched = args.height or 8, args.schedule or "group"
    log(f"timed steps: dtype={dt} height={h} schedule={sched}")

    # ---------------------------------------------------------------- timed steps
    P = Pipeline(dt, h, sched)
    names = ["from_csr_sorted", "colblock_plan", "spmv", "to_csr"] if P.nb else ["from_csr_sorted", "spmv", "to_csr"]
    calls = [P.convert, P.make_plan, P.spmv, P.back] if P.nb else [P.convert, P.spmv, P.back]

    def step(evs=None):
        for k, fn in enumerate(calls):
            if evs is not None:
                evs[k].record(stream)
            fn()
        if evs is not None:
            evs[len(calls)].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    all_evs = [[ev() for _ in range(len(calls) + 1)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(all_evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / args.steps
    seg_ms = np.array([[e[k].elapsed_time(e[k + 1]) for k in range(len(calls))] for e in all_evs]).mean(axis=0)

    b_from, b_plan, b_spmv, b_spmv_minus, b_to = P.bytes()
    algb = {"from_csr_sorted": b_from, "colblock_plan": b_plan, "spmv": b_spmv, "to_csr": b_to}
    b_step = sum(algb[n] for n in names)
    value = b_step / (ms_per_step * 1e-3) / 1e9
    kern = {n: {"ms": round(float(seg_ms[k]), 5), "alg_bytes": algb[n],
                "gbs": round(algb[n] / seg_ms[k] / 1e6, 1)} for k, n in enumerate(names)}
    dom_name = max(kern, key=lambda k: kern[k]["ms"])
    dom = kern[dom_name]
    ach = dom["alg_bytes"] / dom["ms"] / 1e6
    tag = f"{dom_name}:{dt}:h{h}:{sched}"
    traffic = read_traffic(tag)
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic}
    log(f"step {ms_per_step * 1e3:.1f} us (" + ", ".join(f"{n} {seg_ms[k] * 1e3:.1f}" for k, n in enumerate(names))
        + f" us) -> {value:.1f} GB/s")

    # SpMV alone at the chosen configuration, paper protocol
    cm, cs = protocol(P.spmv, cold=True)
    wm, _ = protocol(P.spmv, cold=False)
    spmv = {"height": h, "schedule": sched, "dtype": dt, "cold_ms": round(cm, 5), "cold_std_ms": round(cs, 5),
            "warm_ms": round(wm, 5), "beta_plus_bytes": b_spmv, "beta_minus_bytes": b_spmv_minus,
            "gbs_plus_cold": round(b_spmv / cm / 1e6, 1), "eta_plus_cold": round(b_spmv / cm / 1e6 / HBM_PEAK_GBS, 4),
            "gbs_minus_cold": round(b_spmv_minus / cm / 1e6, 1),
            "eta_minus_cold": round(b_spmv_minus / cm / 1e6 / HBM_PEAK_GBS, 4),
            "gflops_cold": round(model.flops(A.nnz, A.rows) / cm / 1e6, 1),
            "gbs_plus_warm": round(b_spmv / wm / 1e6, 1)}

    # Achievable ceilings: read-only pass over the streams (Sec. 6.3) and the random-gather rate into x.
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    ts, _ = protocol(lambda: cmrs.calib_stream_read(P.M, h, sink), cold=True)
    stream_bytes = (4 + sizes[dt]) * A.nnz
    idx = torch.from_numpy(np.random.default_rng(2).integers(0, A.cols, A.nnz).astype(np.int32)).to(dev)
    tg, _ = protocol(lambda: cmrs.calib_gather(idx, P.x, sink), cold=True)
    ceiling = {"stream_read_gbs": round(stream_bytes / ts / 1e6, 1),
               "stream_read_frac_of_peak": round(stream_bytes / ts / 1e6 / HBM_PEAK_GBS, 4),
               "random_gathers_per_s": round(A.nnz / (tg * 1e-3), 1),
               "random_gather_ms_for_nnz": round(tg, 5),
               "spmv_eta_plus_vs_stream_ceiling": round(b_spmv / cm / 1e6 / (stream_bytes / ts / 1e6), 4)}
    log(f"ceilings: stream {ceiling['stream_read_gbs']} GB/s, gathers {ceiling['random_gathers_per_s'] / 1e9:.1f} G/s")

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
        b_cpu = b_from + b_spmv + b_to
        cpu = {"value": round(b_cpu / tc / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the full workload matrix, one step (oracle CSR->CMRS sorted, CSR SpMV, CMRS->CSR; "
                         f"{b_cpu} algorithmic bytes) timed {reps}x after one untimed pass; {tc:.2f} s per step",
               "ms_per_step": round(tc * 1e3, 1)}
        log(f"cpu oracle: {tc:.2f} s/step -> {cpu['value']} GB/s")

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dt, "data": "synthetic",
        "config": {"workload": f"poisson16 n={A.rows} (row lengths max(1,Poisson(16)), distinct uniform columns, "
                               f"N(0,1) values and x, seed 0)", "rows": A.rows, "nnz": A.nnz, "height": h,
                   "schedule": sched, "sorted": True,
                   "step": " + ".join(names), "alg_bytes_per_step": b_step},
        "roofline": roofline, "cpu_baseline": cpu, "spmv": spmv, "ceiling": ceiling, "kernels": kern,
        "kernel_src": kernel_source_hash(), "sweep": sweep,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

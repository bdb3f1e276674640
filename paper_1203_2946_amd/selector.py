"""Learned choice of strip height and SpMV schedule.

The paper tunes the strip height and kernel options by brute-force search over
measured SpMV times (Sec. 6.3) and quantifies what per-matrix tuning could
still gain over its fixed defaults (Sec. 6.8).  This module turns that search
into training data: for seeded synthetic matrices it measures every class
(6 heights x 4 schedules = 24) and trains, on the GPU with the library's own
HIP kernels (cmrs_mlp_forward / cmrs_mlp_backward / cmrs_adam_step), an MLP
40 -> 64 -> 64 -> 24 that predicts each class's log2 time relative to the
fastest from the features of cmrs_features.  Selection takes the class with
the lowest prediction; `autotune(..., top_k)` times the k best predictions
and keeps the fastest (k = 24 is exhaustive search, the fallback and the
yardstick the regret is measured against).

    python -m paper_1203_2946_amd.selector collect OUT.npz [--count N] [--start K] [--max-seconds S]
    python -m paper_1203_2946_amd.selector merge OUT.npz PART1.npz PART2.npz ...
    python -m paper_1203_2946_amd.selector train DATA.npz WEIGHTS.npz
"""
from __future__ import annotations

import math
import os
import sys
import time

import numpy as np
import torch

from . import cmrs

HEIGHTS = (1, 2, 4, 8, 16, 32)
SCHEDULES = ("wave", "wave_nt", "group", "colblock4")
CLASSES = [(h, s) for h in HEIGHTS for s in SCHEDULES]
N_FEATURES, N_CLASSES, N_PARAMS = 40, 24, 8344
HIDDEN = 64
DEFAULT_CLASS = CLASSES.index((8, "group"))
_HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_PATH = os.path.join(_HERE, "data", "selector_weights.npz")
DATA_PATH = os.path.join(_HERE, "data", "selector_timings.npz")

_L = cmrs.lib


def _s():
    return torch.cuda.current_stream().cuda_stream


def _p(t):
    return t.data_ptr()


# ----------------------------------------------------------------- features
def features(row_ptr: torch.Tensor, col_ind: torch.Tensor, cols: int) -> torch.Tensor:
    """The 40 selection features of a device CSR structure (fp32, device)."""
    rows = row_ptr.numel() - 1
    out = torch.empty(N_FEATURES, dtype=torch.float32, device=row_ptr.device)
    ws = torch.empty(64, dtype=torch.int32, device=row_ptr.device)
    st = _L.cmrs_features(rows, cols, col_ind.numel(), _p(row_ptr), cmrs._ptr(col_ind), _p(out), _p(ws), 256, _s())
    cmrs._check(st, "cmrs_features")
    return out


# ----------------------------------------------------------------- MLP on the GPU
def init_params(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-uniform weights, zero biases, packed W1 b1 W2 b2 W3 b3."""
    g = np.random.default_rng(seed)
    parts = []
    for nin, nout in ((N_FEATURES, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, N_CLASSES)):
        lim = math.sqrt(6.0 / nin)
        parts.append(g.uniform(-lim, lim, nin * nout))
        parts.append(np.zeros(nout))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == N_PARAMS
    return torch.from_numpy(p).to(device)


class Mlp:
    def __init__(self, params: torch.Tensor):
        assert params.numel() == N_PARAMS and params.dtype == torch.float32 and params.is_cuda
        self.params = params

    def forward(self, X: torch.Tensor):
        b = X.shape[0]
        dev = X.device
        H1 = torch.empty(b, HIDDEN, device=dev)
        H2 = torch.empty(b, HIDDEN, device=dev)
        Y = torch.empty(b, N_CLASSES, device=dev)
        cmrs._check(_L.cmrs_mlp_forward(b, _p(X), _p(self.params), _p(H1), _p(H2), _p(Y), _s()), "cmrs_mlp_forward")
        return H1, H2, Y

    def grads(self, X: torch.Tensor, T: torch.Tensor):
        """Parameter gradients of mean((Y - T)^2) over all batch x class entries."""
        b = X.shape[0]
        H1, H2, Y = self.forward(X)
        dY = torch.empty_like(Y)
        cmrs._check(_L.cmrs_mse_grad(Y.numel(), _p(Y), _p(T), _p(dY), 2.0 / Y.numel(), _s()), "cmrs_mse_grad")
        dH2 = torch.empty_like(H2)
        dH1 = torch.empty_like(H1)
        g = torch.empty_like(self.params)
        cmrs._check(_L.cmrs_mlp_backward(b, _p(X), _p(self.params), _p(H1), _p(H2), _p(dY), _p(dH2), _p(dH1), _p(g),
                                         _s()), "cmrs_mlp_backward")
        return Y, g

    def train(self, X: torch.Tensor, T: torch.Tensor, steps: int = 4000, lr: float = 2e-3, log_every: int = 0):
        """Full-batch Adam; returns the loss history (host floats, every step)."""
        m = torch.zeros_like(self.params)
        v = torch.zeros_like(self.params)
        hist = []
        for k in range(1, steps + 1):
            Y, g = self.grads(X, T)
            cmrs._check(_L.cmrs_adam_step(N_PARAMS, _p(self.params), _p(g), _p(m), _p(v), lr, 0.9, 0.999, 1e-8, k,
                                          _s()), "cmrs_adam_step")
            if log_every and (k % log_every == 0 or k == 1):
                loss = float(((Y - T) ** 2).mean())
                hist.append((k, loss))
        return hist

    def predict(self, X: torch.Tensor) -> torch.Tensor:
        return self.forward(X)[2]


def load(path: str = WEIGHTS_PATH, device="cuda") -> Mlp:
    d = np.load(path, allow_pickle=False)
    return Mlp(torch.from_numpy(d["params"].astype(np.float32)).to(device))


# ----------------------------------------------------------------- running a class
class ClassRunner:
    """One CMRS matrix per height and the buffers to run every class on it."""

    def __init__(self, row_ptr, col_ind, val, cols, heights=HEIGHTS):
        self.rows = row_ptr.numel() - 1
        self.cols = cols
        self.x = torch.randn(cols, dtype=val.dtype, device=val.device)
        self.y = torch.empty(self.rows, dtype=val.dtype, device=val.device)
        self.mats, self.plans, self.ws = {}, {}, {}
        for h in heights:
            M = cmrs.from_csr(row_ptr, col_ind, val, cols, h, sort=True)
            self.mats[h] = M
            self.plans[h] = cmrs.colblock_plan(M, 4)
            self.ws[h] = torch.empty(max(1, cmrs.spmv_colblock_workspace_bytes(M, 4, "concurrent")),
                                     dtype=torch.uint8, device=val.device)

    def run(self, c: int):
        h, s = CLASSES[c]
        M = self.mats[h]
        if s == "colblock4":
            cmrs.spmv_colblock(M, self.plans[h], self.x, out=self.y, schedule="concurrent", workspace=self.ws[h])
        else:
            cmrs.spmv(M, self.x, out=self.y, variant={"wave": "lds", "wave_nt": "lds_nt", "group": "group_nt"}[s])

    def time_classes(self, classes=None, reps: int = 5) -> np.ndarray:
        """Median time (ms) of each class, warm, HIP events on the stream."""
        classes = list(range(N_CLASSES)) if classes is None else list(classes)
        evs = {}
        for c in classes:
            self.run(c)
            pairs = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                self.run(c)
                b.record()
                pairs.append((a, b))
            evs[c] = pairs
        torch.cuda.synchronize()
        out = np.full(N_CLASSES, np.nan)
        for c, pairs in evs.items():
            out[c] = float(np.median([a.elapsed_time(b) for a, b in pairs]))
        return out


def targets(times: np.ndarray) -> np.ndarray:
    """log2(time / fastest time) per class (0 for the best)."""
    return np.log2(times / times.min(axis=1, keepdims=True)).astype(np.float32)


def regret(times: np.ndarray, choice: np.ndarray) -> float:
    """Geometric-mean slowdown of the chosen classes against the fastest, minus 1."""
    t = times[np.arange(times.shape[0]), choice]
    return float(np.exp(np.mean(np.log(t / times.min(axis=1)))) - 1.0)


def autotune(runner: ClassRunner, feat: torch.Tensor, model: Mlp | None, top_k: int = 1):
    """Class for one matrix: the model's best prediction (top_k = 1), the
    fastest of its top_k predictions when timed, or exhaustive search
    (model None or top_k = 24)."""
    if model is None or top_k >= N_CLASSES:
        t = runner.time_classes()
        return int(np.nanargmin(t))
    pred = model.predict(feat.reshape(1, -1)).cpu().numpy()[0]
    order = np.argsort(pred)[:top_k]
    if top_k == 1:
        return int(order[0])
    t = runner.time_classes(order)
    return int(order[np.nanargmin(t[order])])


# ----------------------------------------------------------------- data set
def sample_matrix(idx: int, seed: int, dev, max_nnz: int = 40_000_000):
    """Matrix idx of the data set: family idx % 5 with its parameters drawn
    at random, rows log-uniform in [10^4, 4 * 10^6], capped so that the
    expected nnz stays below max_nnz."""
    from synth import gpu_families as F
    g = torch.Generator(device=dev)
    g.manual_seed(seed * 1_000_003 + idx)
    fam = F.FAMILIES[idx % len(F.FAMILIES)]
    u = torch.rand(3, generator=g, device=dev).tolist()
    n = int(10 ** (4 + u[0] * (math.log10(4e6) - 4)))
    if fam == "banded":
        kw = {"bandwidth": 8 + int(u[1] * 57)}
        per_row = 0.6 * (2 * kw["bandwidth"] + 1) + 0.4
    elif fam == "poisson":
        kw = {"mean": math.exp(math.log(2) + u[1] * (math.log(64) - math.log(2)))}
        per_row = kw["mean"] + 1
    elif fam == "zipf":
        kw = {"a": 1.8 + 0.8 * u[1]}
        per_row = 16
    elif fam == "dblock":
        kw = {"per_row": 1 + int(u[1] * 4)}
        per_row = 32 * kw["per_row"]
    else:
        kw, per_row = {}, 27
    n = max(10_000, min(n, int(max_nnz / per_row)))
    rp, ci, val, cols = getattr(F, fam)(n, g, **kw)
    return fam, rp, ci, val, cols


def collect(out_path: str, count: int = 2000, seed: int = 0, reps: int = 5, log=print, max_seconds: float = 1e9,
            start: int = 0):
    """Time all classes on matrices start..count-1 of the data set; saves
    every 50 matrices and stops early (keeping what it has) after
    max_seconds.  Parts collected from different starts are joined with
    `merge`."""
    dev = torch.device("cuda:0")
    n = max(0, count - start)
    feats = np.zeros((n, N_FEATURES), np.float32)
    times = np.zeros((n, N_CLASSES), np.float64)
    meta_rows = np.zeros(n, np.int64)
    meta_nnz = np.zeros(n, np.int64)
    fams = []
    t0 = time.time()
    done = 0
    for k in range(n):
        if time.time() - t0 > max_seconds:
            break
        fam, rp, ci, val, cols = sample_matrix(start + k, seed, dev)
        feats[k] = features(rp, ci, cols).cpu().numpy()
        runner = ClassRunner(rp, ci, val, cols)
        times[k] = runner.time_classes(reps=reps)
        meta_rows[k], meta_nnz[k] = rp.numel() - 1, ci.numel()
        fams.append(fam)
        done = k + 1
        del runner, rp, ci, val
        if done % 50 == 0:
            log(f"[collect] {start + done}/{count} matrices ({time.time() - t0:.0f}s)")
            _save(out_path, feats, times, meta_rows, meta_nnz, fams, done)
    _save(out_path, feats, times, meta_rows, meta_nnz, fams, done)
    log(f"[collect] done: matrices {start}..{start + done - 1} ({time.time() - t0:.0f}s)")
    return out_path


def merge(out_path: str, parts) -> str:
    """Join data files collected from consecutive starts, in the order given."""
    ds = [np.load(p, allow_pickle=False) for p in parts]
    keys = ("features", "times_ms", "rows", "nnz", "family")
    np.savez(out_path, **{k: np.concatenate([d[k] for d in ds]) for k in keys}, classes=ds[0]["classes"])
    return out_path


def _save(path, feats, times, rows, nnz, fams, n):
    np.savez(path, features=feats[:n], times_ms=times[:n], rows=rows[:n], nnz=nnz[:n], family=np.array(fams[:n]),
             classes=np.array([f"h{h}_{s}" for h, s in CLASSES]))


def split(n: int, n_train: int):
    return np.arange(n_train), np.arange(n_train, n)


def train_from_data(data_path: str, steps: int = 4000, lr: float = 2e-3, seed: int = 0, n_train: int | None = None):
    d = np.load(data_path, allow_pickle=False)
    X, times = d["features"], d["times_ms"]
    n = X.shape[0]
    n_train = int(n * 0.75) if n_train is None else n_train
    tr, te = split(n, n_train)
    dev = torch.device("cuda:0")
    Xt = torch.from_numpy(X[tr]).to(dev)
    Tt = torch.from_numpy(targets(times[tr])).to(dev)
    model = Mlp(init_params(seed, dev))
    hist = model.train(Xt, Tt, steps=steps, lr=lr, log_every=max(1, steps // 10))
    pred = model.predict(torch.from_numpy(X).to(dev)).cpu().numpy()
    choice = pred.argmin(axis=1)
    report = {
        "n_train": int(tr.size), "n_test": int(te.size), "loss_history": hist,
        "regret_test": regret(times[te], choice[te]), "regret_train": regret(times[tr], choice[tr]),
        "regret_default_test": regret(times[te], np.full(te.size, DEFAULT_CLASS)),
        "regret_best_fixed_test": min(regret(times[te], np.full(te.size, c)) for c in range(N_CLASSES)),
        "exact_best_test": float(np.mean(choice[te] == times[te].argmin(axis=1))),
    }
    return model, report


def main(argv):
    if len(argv) >= 2 and argv[0] == "collect":
        count = int(argv[argv.index("--count") + 1]) if "--count" in argv else 2000
        secs = float(argv[argv.index("--max-seconds") + 1]) if "--max-seconds" in argv else 1e9
        start = int(argv[argv.index("--start") + 1]) if "--start" in argv else 0
        collect(argv[1], count=count, max_seconds=secs, start=start,
                log=lambda s: print(s, file=sys.stderr, flush=True))
    elif len(argv) >= 3 and argv[0] == "merge":
        merge(argv[1], argv[2:])
    elif len(argv) >= 3 and argv[0] == "train":
        model, rep = train_from_data(argv[1])
        np.savez(argv[2], params=model.params.cpu().numpy(), n_train=rep["n_train"])
        print({k: v for k, v in rep.items() if k != "loss_history"})
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))

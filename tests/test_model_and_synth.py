"""CPU tests of the byte/perf models and of the seeded input generators."""
import json
import os

import numpy as np
import pytest

import synth
from paper_1203_2946_amd import model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")


def test_eq51_printed_values():
    """Sec. 5: h=1, lambda=128, b=4, mu=2 gives f = 16.5; h=16 gives about 2."""
    pm = json.load(open(GOLDEN))["perf_model"]
    assert model.f_model(1, pm["mu"], pm["lambda"], pm["b"]) == pm["f_h1"]
    f16 = model.f_model(16, pm["mu"], pm["lambda"], pm["b"])
    assert abs(f16 - pm["f_h16_approx"]) < 0.05


def test_eq52_approximation_close_to_ratio():
    # b / lambda = 1/32, the case discussed after Eq. (5.2)
    for h in (2, 4, 8, 16):
        for mu in (1, 2, 5, 20, 100):
            ex = model.a_model(h, mu, 128, 4)
            ap = model.a_model_approx(h, mu, 128, 4)
            assert abs(ex - ap) / ex < 0.05
    # small mu and small h: a(h, mu) is close to h
    assert abs(model.a_model(4, 1, 128, 4) - 4) < 0.5


@pytest.mark.parametrize("lam,b", [(128, 4), (128, 8), (256, 8), (64, 4)])
def test_appendix_a_segment_count_by_enumeration(lam, b):
    """Count the segments touched by every b-aligned placement of an n-byte
    chunk and compare the mean with 1 + (n - b) / lambda."""
    for n in range(b, 6 * lam, b):
        counts = []
        for start in range(0, lam, b):
            first = start // lam
            last = (start + n - 1) // lam
            counts.append(last - first + 1)
        assert abs(np.mean(counts) - model.expected_segments(n, lam, b)) < 1e-12


def test_beta_models():
    # paper form, square matrix: beta- - beta+ = s_v (nnz - rows)
    bm, bp = model.paper_beta(1000, 100, 25, 8)
    assert bm - bp == 8 * (1000 - 100)
    # generalised form reduces to the paper's for square matrices, up to the +1 strip pointer
    gp = model.beta_plus(1000, 100, 100, 25, 8, 8, 8)
    assert gp == bp + 4
    assert model.beta_minus(1000, 100, 100, 25, 8, 8, 8) - gp == 8 * (1000 - 100)
    assert model.flops(1000, 100) == 1900


def test_generators_deterministic_and_canonical():
    a = synth.poisson_rows(5000, mean=16, seed=3)
    b = synth.poisson_rows(5000, mean=16, seed=3)
    assert np.array_equal(a.col_ind, b.col_ind) and np.array_equal(a.val, b.val)
    for A in (a, synth.zipf_clustered(20000, seed=1), synth.laplace2d(16), synth.stencil27(5, 4, 3),
              synth.banded(300, 9, seed=2), synth.dense_blocks(100, 32, 2, seed=1)):
        assert A.row_ptr[0] == 0 and A.row_ptr[-1] == A.nnz
        assert np.all(np.diff(A.row_ptr) >= 0)
        assert A.col_ind.min() >= 0 and A.col_ind.max() < A.cols
        d = np.diff(A.col_ind.astype(np.int64))
        inner = np.ones(max(A.nnz - 1, 0), bool)
        starts = A.row_ptr[1:-1]
        inner[starts[(starts > 0) & (starts < A.nnz)] - 1] = False
        assert np.all(d[inner] > 0), A.name


def test_poisson_row_lengths():
    A = synth.poisson_rows(200000, mean=16, seed=0)
    k = A.row_lengths()
    assert k.min() >= 1
    assert abs(k.mean() - 16) < 0.05


def test_zipf_structure():
    A = synth.zipf_clustered(200000, seed=0)
    k = A.row_lengths()
    assert k.min() >= 1 and k.max() <= 10000
    rows = np.repeat(np.arange(A.rows), k)
    near = np.abs(A.col_ind.astype(np.int64) - rows) <= 512
    short = np.repeat(k <= 1000, k)   # rows whose near share is not capped by the band
    frac = near[short].mean()
    assert 0.68 < frac < 0.76


def test_laplace_counts():
    A = synth.laplace2d(64)
    assert A.rows == 4096 and A.nnz == 20224
    assert set(np.unique(A.val).tolist()) == {-1.0, 4.0}


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""

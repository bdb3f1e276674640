"""GPU parity of the selector kernels against oracle/selector_ref.py.

Features: bin fractions bit-exact (same integer counts, one fp32 division);
the four log2 scalars within 4 ulp.  MLP: forward within the rounding bound
of fp32 dot products (Higham's gamma_n on |in| |W| + |b|, propagated through
the layers), gradients and Adam within fp32 accumulation bounds derived in
each test.
"""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import selector_ref as R

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _sel():
    from paper_1203_2946_amd import selector
    return selector


def _feat_case(A):
    S = _sel()
    rp = torch.from_numpy(A.row_ptr).cuda()
    ci = torch.from_numpy(A.col_ind).cuda()
    got = S.features(rp, ci, A.cols).cpu().numpy()
    ref = R.features(A.row_ptr, A.col_ind, A.cols)
    np.testing.assert_array_equal(got[:36], ref[:36])
    np.testing.assert_allclose(got[36:], ref[36:], rtol=4 * U * 2, atol=0)


@pytest.mark.parametrize("case", ["laplace", "poisson", "zipf", "random_rect", "identity", "dense", "banded",
                                  "blocks", "empty_rows"])
def test_features_match_reference(case):
    A = {
        "laplace": lambda: synth.laplace2d(70, 33),
        "poisson": lambda: synth.poisson_rows(20_000, 12.0, 3),
        "zipf": lambda: synth.zipf_clustered(30_000, seed=4),
        "random_rect": lambda: synth.random_csr(1_777, 50_000, 70, seed=5),
        "identity": lambda: synth.identity(4097),
        "dense": lambda: synth.dense_as_sparse(150, seed=6),
        "banded": lambda: synth.banded(9_000, 40, seed=7),
        "blocks": lambda: synth.dense_blocks(4096, 32, 3, seed=8),
        "empty_rows": lambda: synth.random_csr(3_001, 3_001, 3, seed=9),
    }[case]()
    _feat_case(A)


def test_features_no_entries_and_no_rows():
    S = _sel()
    rp = torch.zeros(65, dtype=torch.int32, device="cuda")
    ci = torch.zeros(0, dtype=torch.int32, device="cuda")
    got = S.features(rp, ci, 10).cpu().numpy()
    np.testing.assert_array_equal(got, R.features(np.zeros(65, np.int64), np.zeros(0, np.int64), 10))
    rp0 = torch.zeros(1, dtype=torch.int32, device="cuda")
    got0 = S.features(rp0, ci, 0).cpu().numpy()
    assert not np.any(np.isnan(got0)) and np.all(got0[:36] == 0)


def _forward_bound(X, p):
    """Entrywise bound on |fp32 forward - exact| for the fp32-representable
    inputs X, p: each layer adds gamma_{n+1} (|in| |W| + |b|) and carries the
    input error through |W| (ReLU is 1-Lipschitz)."""
    e = np.zeros_like(X)
    a = X
    for k, (W, b) in enumerate(R.unpack(p)):
        n = W.shape[0]
        g = (n + 1) * U / (1 - (n + 1) * U)
        e = g * (np.abs(a) @ np.abs(W) + np.abs(b)) + e @ np.abs(W) * (1 + g)
        a = a @ W + b
        if k < 2:
            a = np.maximum(a, 0)
    return e


def _rand_model(seed, batch):
    g = np.random.default_rng(seed)
    X = g.uniform(0, 1, (batch, 40)).astype(np.float32)
    p = _sel().init_params(seed, "cpu").numpy()
    p = (p + g.normal(0, 0.05, p.size)).astype(np.float32)
    return X, p


@pytest.mark.parametrize("batch", [1, 7, 64, 300, 1500])
def test_mlp_forward(batch):
    S = _sel()
    X, p = _rand_model(batch, batch)
    m = S.Mlp(torch.from_numpy(p).cuda())
    H1, H2, Y = m.forward(torch.from_numpy(X).cuda())
    rH1, rH2, rY = R.mlp_forward(X.astype(np.float64), p.astype(np.float64))
    bound = _forward_bound(X.astype(np.float64), p.astype(np.float64))
    err = np.abs(Y.cpu().numpy().astype(np.float64) - rY)
    assert np.all(err <= bound + 1e-30), float((err / (bound + 1e-30)).max())
    # Hidden activations too (first layer: single rounding bound).
    W1, b1 = R.unpack(p.astype(np.float64))[0]
    b_h1 = 41 * U * (np.abs(X.astype(np.float64)) @ np.abs(W1) + np.abs(b1)) * 1.01
    assert np.all(np.abs(H1.cpu().numpy() - rH1) <= b_h1 + 1e-30)


def _abs_backward(p, H1, H2, X, dY_abs):
    """Gradient of the same network with every factor replaced by its absolute
    value, seeded with dY_abs: it bounds the sums whose rounding the fp32
    backward incurs, and carries an error in dY through the layers."""
    (W1, b1), (W2, b2), (W3, b3) = R.unpack(p)
    gW3 = np.abs(H2).T @ dY_abs
    dH2 = (dY_abs @ np.abs(W3).T) * (H2 > 0)
    gW2 = np.abs(H1).T @ dH2
    dH1 = (dH2 @ np.abs(W2).T) * (H1 > 0)
    gW1 = np.abs(X).T @ dH1
    return np.concatenate([gW1.ravel(), dH1.sum(0), gW2.ravel(), dH2.sum(0), gW3.ravel(), dY_abs.sum(0)])


@pytest.mark.parametrize("batch", [1, 5, 64, 257, 1500])
def test_mlp_backward(batch):
    S = _sel()
    X, p = _rand_model(100 + batch, batch)
    T = np.random.default_rng(batch).normal(0, 1, (batch, 24)).astype(np.float32)
    m = S.Mlp(torch.from_numpy(p).cuda())
    Y, g = m.grads(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    X64, p64, T64 = X.astype(np.float64), p.astype(np.float64), T.astype(np.float64)
    H1, H2, _ = R.mlp_forward(X64, p64)
    # Mask disagreements (an activation within rounding of 0) make the
    # comparison meaningless; the random inputs keep them out.
    gH1, gH2, _ = m.forward(torch.from_numpy(X).cuda())
    assert np.array_equal(gH1.cpu().numpy() > 0, H1 > 0) and np.array_equal(gH2.cpu().numpy() > 0, H2 > 0)
    ref, dY, _, _ = R.mlp_backward(X64, T64, p64)
    # Each gradient is a sum of at most batch (weights) or 64 (inputs) fp32
    # products over three layers, fed by activations that carry their own
    # forward rounding (at most 3 * 41 units): 4 (batch + 3 * 64 + 3 * 41) u
    # times the absolute-value gradient; the forward error of Y enters dY as
    # 2 |dY error| / (batch * 24) and is carried through the same graph.
    k = 4 * (batch + 3 * 64 + 3 * 41) * U
    dY_err = 2.0 * _forward_bound(X64, p64) / dY.size
    bound = k * _abs_backward(p64, H1, H2, X64, np.abs(dY)) + 2 * _abs_backward(p64, H1, H2, X64, dY_err)
    err = np.abs(g.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= bound + 1e-30), float((err / (bound + 1e-30)).max())


def test_adam_steps():
    S = _sel()
    g = np.random.default_rng(11)
    n = S.N_PARAMS
    p = g.normal(size=n).astype(np.float32)
    m = np.zeros(n)
    v = np.zeros(n)
    tp = torch.from_numpy(p).cuda()
    tm = torch.zeros(n, device="cuda")
    tv = torch.zeros(n, device="cuda")
    pr = p.astype(np.float64)
    # The kernel receives the hyper-parameters as fp32: the reference takes
    # the same rounded values (1 - fp32(0.999) differs from 0.001 by 1.3e-5).
    lr, b1, b2, eps = (float(np.float32(c)) for c in (1e-3, 0.9, 0.999, 1e-8))
    for step in range(1, 6):
        gr = g.normal(size=n).astype(np.float32)
        st = S._L.cmrs_adam_step(n, tp.data_ptr(), torch.from_numpy(gr).cuda().data_ptr(), tm.data_ptr(),
                                 tv.data_ptr(), lr, b1, b2, eps, step, S._s())
        assert st == 0
        pr, m, v = R.adam(pr, gr.astype(np.float64), m, v, lr, b1, b2, eps, step)
    torch.cuda.synchronize()
    # Each step moves a parameter by at most about lr; fp32 rounding of the
    # moments and the update stays far below 1e-3 of that per step.
    np.testing.assert_allclose(tp.cpu().numpy(), pr, rtol=0, atol=5 * 1e-3 * 1e-3 + 5 * 2 * U * np.abs(pr).max())
    np.testing.assert_allclose(tm.cpu().numpy(), m, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(tv.cpu().numpy(), v, rtol=1e-5, atol=1e-9)


def test_training_fits_a_known_target():
    """Targets from a random teacher network: 600 full-batch Adam steps
    through the HIP kernels must cut the loss by 10x."""
    S = _sel()
    g = np.random.default_rng(21)
    X = g.uniform(0, 1, (256, 40)).astype(np.float32)
    teacher = S.init_params(99, "cpu").numpy().astype(np.float64)
    T = R.mlp_forward(X.astype(np.float64), teacher)[2].astype(np.float32)
    m = S.Mlp(S.init_params(1, "cuda"))
    Xt, Tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    first = float(((m.predict(Xt) - Tt) ** 2).mean())
    m.train(Xt, Tt, steps=600, lr=2e-3)
    last = float(((m.predict(Xt) - Tt) ** 2).mean())
    assert last < first / 10, (first, last)


DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1203_2946_amd", "data")


@pytest.mark.skipif(not os.path.exists(os.path.join(DATA, "selector_weights.npz")), reason="no trained weights")
def test_committed_selector_regret_on_gpu():
    """The HIP forward with the committed weights picks, on the held-out
    matrices of the committed timing set, classes within 5 % (geometric mean)
    of the exhaustive best, and better than any single fixed class."""
    S = _sel()
    d = np.load(os.path.join(DATA, "selector_timings.npz"), allow_pickle=False)
    w = np.load(os.path.join(DATA, "selector_weights.npz"), allow_pickle=False)
    te = np.arange(int(w["n_train"]), d["features"].shape[0])
    m = S.load(os.path.join(DATA, "selector_weights.npz"))
    pred = m.predict(torch.from_numpy(d["features"][te]).cuda()).cpu().numpy()
    t = d["times_ms"][te]
    r = S.regret(t, pred.argmin(axis=1))
    fixed = min(S.regret(t, np.full(te.size, c)) for c in range(S.N_CLASSES))
    assert r <= 0.05 and r < fixed, (r, fixed)


def test_class_runner_matches_oracle():
    """Every one of the 24 classes computes the same y = A x (fp64, within
    the CRS error bound) on a GPU-generated matrix of each family."""
    S = _sel()
    import oracle
    from synth import gpu_families as F
    for i, fam in enumerate(F.FAMILIES):
        gen = torch.Generator(device="cuda")
        gen.manual_seed(500 + i)
        rp, ci, val, cols = F.generate(fam, 6000, gen)
        run = S.ClassRunner(rp, ci, val, cols)
        hrp, hci, hv, hx = (t.cpu().numpy() for t in (rp, ci, val, run.x))
        ref = oracle.csr_spmv(hrp, hci, hv, hx)
        bound = oracle.spmv_bound(hrp, hci, hv, hx, 2.0 ** -53, 4.0)
        for c in range(S.N_CLASSES):
            run.y.fill_(float("nan"))
            run.run(c)
            torch.cuda.synchronize()
            err = np.abs(run.y.cpu().numpy() - ref)
            assert np.all(err <= bound), (fam, S.CLASSES[c])


def test_autotune_paths():
    """autotune: exhaustive (no model) returns the fastest measured class;
    top-k timing returns one of the model's k best predictions."""
    S = _sel()
    from synth import gpu_families as F
    gen = torch.Generator(device="cuda")
    gen.manual_seed(77)
    rp, ci, val, cols = F.generate("poisson", 40_000, gen)
    run = S.ClassRunner(rp, ci, val, cols)
    c_ex = S.autotune(run, None, None)
    assert 0 <= c_ex < S.N_CLASSES
    model = S.Mlp(S.init_params(5, "cuda"))
    feat = S.features(rp, ci, cols)
    pred = model.predict(feat.reshape(1, -1)).cpu().numpy()[0]
    c3 = S.autotune(run, feat, model, top_k=3)
    assert c3 in set(np.argsort(pred)[:3].tolist())
    assert S.autotune(run, feat, model, top_k=1) == int(np.argmin(pred))

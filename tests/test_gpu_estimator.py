"""GPU parity of the learned selectivity estimator against the CPU reference.

Histograms are exact (a sort); features are bfloat16 roundings of the same fractions
(at most one bfloat16 unit apart when float32 and float64 land on opposite sides of a
rounding midpoint); network outputs, losses and gradients use bfloat16 operands with
float32 accumulation on the GPU and float64 sums of the same bfloat16 operands in the
reference.  Labels are exact counts.  Orderings chosen from estimates never change a
result.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import estimator_ref as er
from paper_1801_03644_amd import datagen as dg
from paper_1801_03644_amd import mdrq
from tests.gpu_helpers import run

pytestmark = pytest.mark.gpu

BF16_ULP = 2.0 ** -8  # relative spacing of bfloat16 values (8 significant bits)


def _print(*a):
    print(*a, flush=True)


def bits_to_float(b: np.ndarray) -> np.ndarray:
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def sample_bounds(raw, m):
    n = len(raw[0])
    rows = (np.arange(m, dtype=np.uint64) * np.uint64(n)) // np.uint64(m)
    return np.stack([er.boundaries(np.sort(c[rows].astype(np.float64))) for c in raw])


def c4_small(n_rows):
    w = dg.workload("c4", n_rows)
    return w, w.columns()


def queries_with_edges(w, n, seed):
    qs = dg.workload_queries(w, n, sampler=w.sampler(sample_rows=1 << 15), seed=seed)
    qs[0] = dg.make_query([(3, 0.7, 0.2)])                               # empty interval
    qs[1] = dg.make_query([(0, -np.inf, np.inf), (5, 0.1, 0.4)])         # partial match entry
    qs[2] = dg.make_query([(7, -5.0, 5.0)])                              # beyond the data range
    qs[3] = dg.make_query([(9, 0.5, 0.5), (19, -np.inf, 0.3)])           # point and half-open
    return qs


def random_params(est, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in est._shapes():
        if name.startswith("W"):
            a = scale * math.sqrt(6.0 / (shape[0] + shape[1]))
            p[name] = rng.uniform(-a, a, size=shape).astype(np.float32)
        else:
            p[name] = rng.normal(0, 0.1, size=shape).astype(np.float32)
    return p


@pytest.mark.parametrize("m", [2, 1000, 16384])
def test_histograms_are_equi_depth_boundaries_of_the_sample(m):
    w, raw = c4_small(70_001)
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds, sample_rows=m) as est:
        got = est.histograms().astype(np.float64)
    want = sample_bounds(raw, m)
    assert np.array_equal(got, want)


def test_features_match_reference():
    w, raw = c4_small(50_000)
    qs = queries_with_edges(w, 300, seed=5)
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds) as est:
        b = est.histograms().astype(np.float64)
        got = bits_to_float(est.features(qs))
    want = np.stack([er.bf16_round(er.features(q, b, 50_000)) for q in qs])
    diff = np.abs(got - want)
    assert (diff <= BF16_ULP * np.abs(want) + 1e-30).all()
    assert (diff == 0).mean() > 0.999


def base_ref(bounds, qs, n_rows):
    return np.stack([er.base(q, bounds, n_rows) for q in qs])


def forward_ref(est, params, X, bounds, n_rows, qs):
    Y, _ = er.forward(params, X, base_ref(bounds, qs, n_rows))
    s = er.selectivity_from_output(Y, n_rows)
    for i, (dims, lo, hi) in enumerate(qs):
        restricted = {int(j) for j, a, c in zip(dims, lo, hi) if not (a == -np.inf and c == np.inf)}
        for j in range(est.n_dims):
            if j not in restricted:
                s[i, j] = 1.0
    return Y, s


def _abs_products(A, B):
    return np.abs(A) @ np.abs(B)


def test_forward_matches_reference():
    """Layer by layer, each GPU layer against the reference fed the GPU's own inputs to
    that layer (its bfloat16 hidden activations), so that a rounding flip upstream cannot
    move the comparison: a hidden activation is within half a bfloat16 unit of GELU of the
    exact pre-activation (plus float32 accumulation), and the output layer, which rounds
    nothing, agrees to 1e-5 on the log scale."""
    w, raw = c4_small(40_000)
    qs = queries_with_edges(w, 333, seed=6)  # ragged: not a multiple of the 16-row tile
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds, hidden=48) as est:
        b = est.histograms().astype(np.float64)
        untrained = est.predict(qs).astype(np.float64)
        p = random_params(est, 1, scale=2.0)
        est.set_params(p)
        X = bits_to_float(est.features(qs))
        got = est.predict(qs).astype(np.float64)
        h1, h2, y = est.activations(qs)
    H1g, H2g, y = bits_to_float(h1), bits_to_float(h2), y.astype(np.float64)
    # untrained: the output layer is zero, the estimate is the histogram base
    _, base_s = forward_ref(est, {k: np.zeros_like(v) for k, v in p.items()}, X, b, 40_000, qs)
    assert np.allclose(untrained, base_s, rtol=1e-5, atol=0)
    W1, W2, W3 = (er.bf16_round(p[k]) for k in ("W1", "W2", "W3"))
    b1, b2, b3 = (p[k].astype(np.float64) for k in ("b1", "b2", "b3"))
    eps32 = 2.0 ** -24
    for Hg, Hin, W, bias in ((H1g, X, W1, b1), (H2g, H1g, W2, b2)):
        Z = Hin @ W + bias
        exact = er.gelu(Z)
        # float32 pre-activation: accumulation error; float32 GELU: 0.5 z (1 + erf) loses
        # up to 2^-23 |z| absolute where 1 + erf cancels (z < 0); then half a bfloat16 unit
        acc = Hin.shape[1] * eps32 * (_abs_products(Hin, W) + np.abs(bias))
        bound = (1.01 * 2.0 ** -8 * np.maximum(np.abs(exact), np.abs(Hg)) + 1.2 * acc
                 + 2.0 ** -22 * (np.abs(Z) + np.abs(exact)) + 1e-30)
        assert (np.abs(Hg - exact) <= bound).all(), np.abs(Hg - exact).max()
        clear = Z > -1.0   # no cancellation in the GELU: rounding flips are rare
        assert (Hg == er.bf16_round(exact.astype(np.float32)))[clear].mean() > 0.99
    want_y = H2g @ W3 + b3 + base_ref(b, qs, 40_000)
    dy = np.abs(y - want_y)
    _print("output layer max |dy|", dy.max())
    assert dy.max() <= 1e-5
    # the prediction is the clamped output layer on the selectivity scale
    s = er.selectivity_from_output(y, 40_000)
    for i, (dims, lo, hi) in enumerate(qs):
        restricted = {int(j) for j, a, c in zip(dims, lo, hi) if not (a == -np.inf and c == np.inf)}
        for j in range(est.n_dims):
            if j not in restricted:
                s[i, j] = 1.0
    assert np.allclose(got, s, rtol=1e-5, atol=0)


def test_one_query_graph_replays_match_eager_prediction():
    """A single query is predicted by replaying a captured HIP graph; every replay must
    equal the eager (many-query) prediction of the same query, also after training has
    changed the weights between replays."""
    w, raw = c4_small(30_000)
    qs = queries_with_edges(w, 40, seed=12)
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds, seed=2) as est:
        p = random_params(est, 6)
        est.set_params(p)
        sel = ds.label_selectivities(qs)
        for rep in range(3):
            eager = est.predict(qs)
            for i in range(12):
                one = est.predict([qs[i]])
                assert np.array_equal(one[0], eager[i]), (rep, i)
            est.train(qs, sel, epochs=1, batch=16, lr=1e-2, seed=rep)


def test_estimated_order_is_exact_on_every_query_shape():
    """Single queries in estimated order (the order computed on the device, ahead of
    the scan on the same stream): ids, bitmap and count equal the oracle's for empty,
    one-predicate, partial-match and all-20-dimension queries; repeated calls replay
    the estimator's graph."""
    from tests.gpu_helpers import bitmap_to_ids

    w, raw = c4_small(60_001)
    cols = oracle.prepare(raw)
    qs = queries_with_edges(w, 40, seed=13)
    rng = np.random.default_rng(13)
    for _ in range(6):
        preds = []
        for j in range(20):
            lo = float(rng.uniform(0, 0.2))
            preds.append((j, lo, lo + float(rng.uniform(0.6, 0.8))))
        qs.append(dg.make_query(preds))
    qs.append(dg.make_query([]))
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds, seed=4) as est:
        est.set_params(random_params(est, 9))
        ds.attach_estimator(est)
        for rep in range(2):
            for i, q in enumerate(qs):
                st, cnt, want = oracle.query(cols, q)
                a, ids = run(ds, q, flags=mdrq.Q_ORDER_ESTIMATED)
                assert a.count == cnt and np.array_equal(ids, want), (rep, i)
                a, words = run(ds, q, mode="bitmap", flags=mdrq.Q_ORDER_ESTIMATED)
                assert np.array_equal(bitmap_to_ids(words, ds.n_rows)[0], want), (rep, i)
                assert run(ds, q, mode="count", flags=mdrq.Q_ORDER_ESTIMATED)[0].count == cnt
        ds.attach_estimator(None)


def test_parameters_round_trip_and_invalid():
    w, raw = c4_small(10_000)
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds, hidden=32, seed=3) as est:
        p = est.get_params()
        assert p["W1"].shape == (20 * 19, 32) and p["W3"].shape == (32, 21)
        assert (p["b1"] == 0).all() and np.abs(p["W2"]).max() <= math.sqrt(6 / 64) + 1e-6
        assert (p["W3"] == 0).all() and (p["b3"] == 0).all() and np.abs(p["W1"]).max() > 0
        q = random_params(est, 2)
        est.set_params(q)
        r = est.get_params()
        for k in q:
            assert np.array_equal(q[k], r[k])
        q["W2"][0, 0] = np.nan
        with pytest.raises(mdrq.MdrqError) as e:
            est.set_params(q)
        assert e.value.code == mdrq.EINVAL
        with pytest.raises(mdrq.MdrqError):
            mdrq.Estimator(ds, hidden=40)
        with pytest.raises(mdrq.MdrqError):
            est.predict([dg.make_query([(0, np.nan, 1.0)])])


def test_labels_are_exact_counts():
    w, raw = c4_small(30_011)
    cols = oracle.prepare(raw)
    qs = queries_with_edges(w, 120, seed=7)
    with mdrq.Dataset.from_host(raw) as ds:
        sel = ds.label_selectivities(qs)
    n = 30_011
    for i, (dims, lo, hi) in enumerate(qs):
        want = np.full(21, -1.0, dtype=np.float32)
        for j, a, c in zip(dims, lo, hi):
            if a == -np.inf and c == np.inf:
                continue
            want[j] = np.float32(oracle.count(cols, dg.make_query([(j, a, c)])) / n)
        want[20] = np.float32(oracle.count(cols, (dims, lo, hi)) / n)
        assert np.array_equal(sel[i], want), i


def test_gradient_matches_reference():
    """Backward kernels against the float64 reference backward, fed the GPU's own forward
    activations and output (so only the backward's own roundings can differ).  Per
    tensor the relative error norm is at most 1e-4; per element the error is within the
    bfloat16 unit of the operand magnitudes that reach it (one rounding flip per layer
    of the chain) plus float32 accumulation."""
    w, raw = c4_small(40_000)
    qs = queries_with_edges(w, 301, seed=8)
    n = 40_000
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds) as est:
        sel = ds.label_selectivities(qs)
        p = random_params(est, 4)
        est.set_params(p)
        X = bits_to_float(est.features(qs))
        b = est.histograms().astype(np.float64)
        loss, g = est.gradient(qs, sel)
        h1, h2, y = est.activations(qs)
    H1g, H2g, Yg = bits_to_float(h1), bits_to_float(h2), y.astype(np.float64)
    T, M = [], []
    for row in sel.astype(np.float64):
        d = {j: row[j] for j in range(20) if row[j] >= 0}
        t, m = er.targets(d, row[20], 20, n)
        T.append(t)
        M.append(m)
    T, M = np.array(T), np.array(M)
    W1, W2, W3 = (er.bf16_round(p[k]) for k in ("W1", "W2", "W3"))
    Z1 = X @ W1 + p["b1"].astype(np.float64)
    Z2 = H1g @ W2 + p["b2"].astype(np.float64)
    cache = {"X": X, "W1": W1, "W2": W2, "W3": W3, "Z1": Z1, "H1": H1g, "Z2": Z2, "H2": H2g}
    want_loss, dY = er.loss_and_grad_y(Yg, T, M)
    want = er.backward(cache, dY)
    assert abs(loss - want_loss) <= 1e-5 * want_loss
    bound = _backward_error_bound(cache, dY, M, p, len(qs))
    for k in want:
        a, r = g[k].astype(np.float64), want[k]
        rel = np.linalg.norm(a - r) / np.linalg.norm(r)
        err = np.abs(a - r)
        _print(k, "relative error", rel, "worst element / bound", (err / (bound[k] + 1e-30)).max())
        assert rel <= 1e-4, (k, rel)
        assert (err <= bound[k] + 1e-30).all(), k


def _backward_error_bound(cache, dY, M, p, rows):
    """Per-element bound on |GPU gradient - reference gradient| when both start from the
    same forward values: every bfloat16-rounded gradient operand may land one bfloat16
    unit (2^-7 relative) away from the reference's, the float32 targets y(s) carry up to
    2^-21 absolute into dY = 2 (Y - T) / count, float32 products and column sums add
    K * 2^-24 of the magnitudes they sum, GELU' in float32 loses up to 2^-22 absolute
    (cancellation in 0.5 (1 + erf)) and moves by at most 0.8 times the float32 error of
    the pre-activation it is taken at."""
    f = 2.0 ** -7
    acc = lambda k: k * 2.0 ** -24
    X, W1, W2, W3 = cache["X"], cache["W1"], cache["W2"], cache["W3"]
    H1, H2, Z1, Z2 = cache["H1"], cache["H2"], cache["Z1"], cache["Z2"]
    F, H, O = W1.shape[0], W1.shape[1], W3.shape[1]
    aX, aH1, aH2 = np.abs(X), np.abs(H1), np.abs(H2)
    aW1, aW2, aW3 = np.abs(W1), np.abs(W2), np.abs(W3)
    dYr = er.bf16_round(dY.astype(np.float32))
    e_dY = 2.0 ** -22 * np.abs(dY) + 2.0 * 2.0 ** -21 * M / M.sum()
    e_dYr = f * np.abs(dY) + e_dY
    dH2 = dYr @ W3.T
    e_dH2 = e_dYr @ aW3.T + acc(O) * (np.abs(dYr) @ aW3.T)
    g2 = er.gelu_grad(Z2)
    e_Z2 = acc(H) * (aH1 @ aW2 + np.abs(p["b2"]))
    dZ2 = dH2 * g2
    e_dZ2 = e_dH2 * np.abs(g2) + np.abs(dH2) * (2.0 ** -22 + 0.8 * e_Z2)
    dZ2r = er.bf16_round(dZ2.astype(np.float32))
    e_dZ2r = e_dZ2 + f * np.abs(dZ2)
    dH1 = dZ2r @ W2.T
    e_dH1 = e_dZ2r @ aW2.T + acc(H) * (np.abs(dZ2r) @ aW2.T)
    g1 = er.gelu_grad(Z1)
    e_Z1 = acc(F) * (aX @ aW1 + np.abs(p["b1"]))
    dZ1 = dH1 * g1
    e_dZ1 = e_dH1 * np.abs(g1) + np.abs(dH1) * (2.0 ** -22 + 0.8 * e_Z1)
    dZ1r = er.bf16_round(dZ1.astype(np.float32))
    e_dZ1r = e_dZ1 + f * np.abs(dZ1)
    a = acc(rows)
    return {"W3": aH2.T @ e_dYr + a * (aH2.T @ np.abs(dYr)),
            "b3": a * np.abs(dY).sum(axis=0) + e_dY.sum(axis=0),
            "W2": aH1.T @ e_dZ2r + a * (aH1.T @ np.abs(dZ2r)),
            "b2": e_dZ2.sum(axis=0) + a * np.abs(dZ2).sum(axis=0),
            "W1": aX.T @ e_dZ1r + a * (aX.T @ np.abs(dZ1r)),
            "b1": e_dZ1.sum(axis=0) + a * np.abs(dZ1).sum(axis=0)}


def test_adam_steps_match_reference():
    w, raw = c4_small(20_000)
    qs = queries_with_edges(w, 200, seed=9)
    lr = 1e-2
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds, hidden=32) as est:
        sel = ds.label_selectivities(qs)
        p0 = random_params(est, 5)
        est.set_params(p0)
        _, g0 = est.gradient(qs, sel)
        est.train(qs, sel, epochs=1, batch=len(qs), lr=lr)
        p1 = est.get_params()
        _, g1 = est.gradient(qs, sel)
        est.train(qs, sel, epochs=1, batch=len(qs), lr=lr)
        p2 = est.get_params()
    for k in p0:
        m0 = np.zeros_like(p0[k], dtype=np.float64)
        r1, m1, v1 = er.adam_step(p0[k].astype(np.float64), g0[k].astype(np.float64), m0, m0, 1, lr)
        r2, _, _ = er.adam_step(p1[k].astype(np.float64), g1[k].astype(np.float64), m1, v1, 2, lr)
        # the training step sums its batch in another order than the gradient call:
        # steps of size about lr may differ where a gradient is within rounding of 0
        bad1 = np.abs(p1[k] - r1) > 1e-4 * lr + 1e-6
        bad2 = np.abs(p2[k] - r2) > 1e-4 * lr + 1e-6
        assert bad1.sum() <= 1e-3 * bad1.size and bad2.sum() <= 1e-3 * bad2.size, k


def independence(bounds, q, n_rows):
    """The histogram independence product (the base estimate) as a selectivity."""
    return er.selectivity_from_output(er.base(q, bounds, n_rows)[-1:], n_rows)[0]


def test_training_learns_and_beats_the_independence_product():
    """c4 shape (pairs of correlated columns) at 2*10^6 rows, trained on 80000 labelled
    queries: on 3000 held-out queries the learned joint estimate has a lower held-out
    loss, geometric-mean q-error and 90th-percentile q-error than the product of the
    per-dimension histogram estimates (the base it corrects)."""
    n = 2_000_000
    w, raw = c4_small(n)
    samp = w.sampler(sample_rows=1 << 17)
    train_q = dg.workload_queries(w, 80000, sampler=samp, seed=11)
    test_q = dg.workload_queries(w, 3000, sampler=samp, seed=12)
    val_q = dg.workload_queries(w, 3000, sampler=samp, seed=13)
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds, seed=1) as est:
        _print("labelling")
        s_train = ds.label_selectivities(train_q)
        s_test = ds.label_selectivities(test_q)
        s_val = ds.label_selectivities(val_q)
        base_pred = est.predict(test_q)   # untrained: the histogram estimates
        _print("training")
        before, _ = est.gradient(test_q, s_test)
        losses = est.train(train_q, s_train, epochs=30, batch=256, lr=1e-3, seed=3)
        after, _ = est.gradient(test_q, s_test)
        _print("epoch losses", losses[0], losses[-1], "held-out loss", before, after)
        ungated = est.predict(test_q)
        kept = est.gate(val_q, s_val)
        _print("outputs kept after gating on the validation split", np.flatnonzero(kept).tolist())
        pred = est.predict(test_q)
        b = est.histograms().astype(np.float64)
    # gating keeps the joint correction, and a removed output returns the base estimate
    assert kept[20]
    for j in np.flatnonzero(~kept):
        assert np.array_equal(pred[:, j], base_pred[:, j]), j
    for j in np.flatnonzero(kept):
        assert np.array_equal(pred[:, j], ungated[:, j]), j
    learned = er.qerror(pred[:, 20], s_test[:, 20], n)
    indep = er.qerror([independence(b, q, n) for q in test_q], s_test[:, 20], n)
    for name, qe in (("learned", learned), ("independence", indep)):
        _print(name, "q-error median", np.median(qe), "p90", np.percentile(qe, 90),
               "geometric mean", np.exp(np.log(qe).mean()))
    assert np.isfinite(losses).all() and losses[-1] < losses[0]
    assert after < 0.8 * before
    assert np.log(learned).mean() < np.log(indep).mean()
    assert np.percentile(learned, 90) < np.percentile(indep, 90)
    assert np.median(learned) < 1.5
    # per-dimension estimates after gating are no worse than the histogram's on the
    # test split (the network never adds noise to an output it does not improve)
    mask = s_test[:, :20] >= 0
    per_dim = er.qerror(pred[:, :20][mask], s_test[:, :20][mask], n)
    hist = er.qerror(base_pred[:, :20][mask], s_test[:, :20][mask], n)
    _print("per-dimension q-error median / p90: gated", np.median(per_dim), np.percentile(per_dim, 90),
           "histogram", np.median(hist), np.percentile(hist, 90))
    assert np.median(per_dim) <= np.median(hist) * 1.01
    assert np.percentile(per_dim, 90) <= np.percentile(hist, 90) * 1.01


def test_estimated_order_gives_identical_results_and_is_faster():
    """Queries whose given order starts with a wide predicate and ends with a narrow
    one: evaluated in estimated order they read fewer column bytes (the early break
    skips more tiles), with the same results."""
    n = 32_000_000
    raw = [dg.column(31, j, dg.uniform(), n) for j in range(6)]
    cols = oracle.prepare(raw)
    rng = np.random.default_rng(3)
    qs = []
    for _ in range(24):
        dims = rng.permutation(6)[:4]
        widths = [0.95, 0.9, 0.8, 2e-5]
        preds = []
        for j, wd in zip(dims, widths):
            lo = float(rng.uniform(0, 1 - wd))
            preds.append((int(j), lo, lo + wd))
        qs.append(dg.make_query(preds))
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds) as est:
        tq = []
        for _ in range(3000):
            k = int(rng.integers(1, 5))
            dims = rng.permutation(6)[:k]
            preds = []
            for j in dims:
                wd = float(np.exp(rng.uniform(np.log(1e-5), 0)))
                lo = float(rng.uniform(0, 1 - wd))
                preds.append((int(j), lo, lo + wd))
            tq.append(dg.make_query(preds))
        est.train(tq, ds.label_selectivities(tq), epochs=15, batch=256, lr=2e-3)
        ds.attach_estimator(est)
        times = {}
        for name, flags in (("given", mdrq.Q_ORDER_GIVEN), ("estimated", mdrq.Q_ORDER_ESTIMATED)):
            for q in qs[:2]:
                run(ds, q, flags=flags)  # warm up
            ds.set_profiling(True)
            ds.reset_profile()
            for q in qs:
                a, ids = run(ds, q, flags=flags)
                st, cnt, want = oracle.query(cols, q)
                assert a.count == cnt and np.array_equal(ids, want)
            times[name] = ds.profile()[1]
            ds.set_profiling(False)
        _print("scan ms given", times["given"], "estimated", times["estimated"])
        assert times["estimated"] < 0.6 * times["given"]
        # batched path with estimated order: same answers
        outs = [None] * len(qs)
        a1 = ds.query_batch(qs, outs, "count", flags=mdrq.Q_ORDER_ESTIMATED)
        for q, a in zip(qs, a1):
            assert a.count == oracle.count(cols, q)
        ds.attach_estimator(None)


def test_trained_order_is_no_slower_on_correlated_data():
    """c4-shaped data (correlated column pairs), 4*10^6 rows: single queries in the order
    of a trained and gated estimator take no more scan time than in the order of the
    untrained one (the histogram estimates), with identical, oracle-exact results."""
    n = 4_000_000
    w, raw = c4_small(n)
    cols = oracle.prepare(raw)
    samp = w.sampler(sample_rows=1 << 16)
    train_q = dg.workload_queries(w, 20000, sampler=samp, seed=21)
    val_q = dg.workload_queries(w, 2000, sampler=samp, seed=22)
    test_q = dg.workload_queries(w, 64, sampler=samp, seed=23)
    want = [oracle.query(cols, q) for q in test_q]
    times = {}
    with mdrq.Dataset.from_host(raw) as ds:
        for name in ("histogram", "trained"):
            with mdrq.Estimator(ds, seed=5) as est:
                if name == "trained":
                    est.train(train_q, ds.label_selectivities(train_q), epochs=10, batch=256, lr=1e-3, seed=1)
                    est.gate(val_q, ds.label_selectivities(val_q))
                ds.attach_estimator(est)
                for q in test_q[:4]:
                    run(ds, q, flags=mdrq.Q_ORDER_ESTIMATED)   # warm-up
                best = None
                for rep in range(3):
                    ds.set_profiling(True)
                    ds.reset_profile()
                    for q, (st, cnt, ids) in zip(test_q, want):
                        a, got = run(ds, q, flags=mdrq.Q_ORDER_ESTIMATED)
                        assert a.count == cnt and np.array_equal(got, ids)
                    t = ds.profile()[1]
                    ds.set_profiling(False)
                    best = t if best is None else min(best, t)
                times[name] = best
                ds.attach_estimator(None)
    _print("scan ms in estimated order: histogram", times["histogram"], "trained", times["trained"])
    assert times["trained"] <= 1.05 * times["histogram"] + 0.05


def test_full_size_c4_batched_estimated_order_sampled():
    """The learned workload's shape at full size (10^8 x 20, correlated pairs), as the
    bench runs its held-out set: shared scans with estimated order (an untrained
    estimator: the histogram ranking), whose grouping splits the 20-column union into
    register-sized scans.  Every count and a sample of identifier lists equal the
    oracle's."""
    import torch

    from tests.gpu_helpers import device, oracle_counts

    w = dg.workload("c4")
    _print("c4 full size: generating")
    raw = w.columns()
    cols = oracle.prepare(raw)
    qs = dg.workload_queries(w, 64)   # held-out mix: k 3..10
    with mdrq.Dataset.from_host(raw) as ds, mdrq.Estimator(ds) as est:
        ds.attach_estimator(est)
        outs = [torch.full((ds.n_rows,), -1, dtype=torch.int32, device=device()) if i in (0, 9, 33)
                else None for i in range(len(qs))]
        modes = ["ids" if o is not None else "count" for o in outs]
        _print("c4 full size: batch of", len(qs))
        ans = ds.query_batch(qs, outs, modes, flags=mdrq.Q_ORDER_ESTIMATED)
        _print("c4 full size: oracle counts of all", len(qs))
        assert [a.count for a in ans] == oracle_counts(cols, qs)
        for i in (0, 9, 33):
            _print("c4 full size: oracle", i)
            st, cnt, want = oracle.query(cols, qs[i])
            assert ans[i].count == cnt
            got = outs[i][:ans[i].written].cpu().numpy().view(np.uint32)
            assert np.array_equal(got, want), i
        ds.attach_estimator(None)

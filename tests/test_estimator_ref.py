"""Pins for the estimator's CPU reference (oracle/estimator_ref.py): closed forms, known
values, brute-force derivatives and invariants, none of which reuse its formulas."""
import math

import numpy as np
import pytest

from oracle import estimator_ref as er


def test_bf16_rounding_known_bit_patterns():
    f = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, -2.5, 3.0e38, 1e-40],
                 dtype=np.float32)
    r = er.bf16_round(f)
    bits = r.astype(np.float32).view(np.uint32)
    assert (bits & 0xFFFF == 0).all()
    assert r[0] == 1.0
    assert r[1] == 1.0                    # tie, even upper half stays
    assert r[2] == 1 + 4 * 2 ** -8        # tie, odd upper half rounds up
    assert r[3] == 1.0                    # below half
    assert r[4] == -2.5
    # nearest: no other bfloat16 value is closer
    for x, y in zip(f.astype(np.float64), r):
        up = np.float32(y).view(np.uint32) + np.uint32(0x10000)
        dn = np.float32(y).view(np.uint32) - np.uint32(0x10000)
        for z in (up, dn):
            zz = float(np.uint32(z).view(np.float32))
            if np.isfinite(zz):
                assert abs(zz - x) >= abs(y - x)


def test_gelu_known_values_and_derivative():
    assert er.gelu(np.array([0.0]))[0] == 0.0
    assert abs(er.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(er.gelu(np.array([-1.0]))[0] + 0.15865525393145707) < 1e-15
    assert abs(er.gelu(np.array([8.0]))[0] - 8.0) < 1e-12
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (er.gelu(z + h) - er.gelu(z - h)) / (2 * h)
    assert np.allclose(er.gelu_grad(z), fd, atol=1e-8)


def _params(rng, K=12, H=8, O=5, scale=0.5):
    return {"W1": rng.normal(0, scale, (K, H)), "b1": rng.normal(0, 0.1, H),
            "W2": rng.normal(0, scale, (H, H)), "b2": rng.normal(0, 0.1, H),
            "W3": rng.normal(0, scale, (H, O)), "b3": rng.normal(0, 0.1, O)}


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    p = _params(rng)
    X = rng.uniform(-1, 1, (7, 12))
    T = rng.uniform(0, 1, (7, 5))
    M = (rng.uniform(0, 1, (7, 5)) < 0.7).astype(float)
    M[:, -1] = 1.0

    def loss(pp):
        Y, _ = er.forward(pp, X, rounding=False)
        return er.loss_and_grad_y(Y, T, M)[0]

    Y, cache = er.forward(p, X, rounding=False)
    _, dY = er.loss_and_grad_y(Y, T, M)
    g = er.backward(cache, dY, round_like_gpu=False)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            pp = {k: v.copy() for k, v in p.items()}
            pp[name].reshape(-1)[idx] += h
            lp = loss(pp)
            pp[name].reshape(-1)[idx] -= 2 * h
            lm = loss(pp)
            fd = (lp - lm) / (2 * h)
            assert abs(g[name].reshape(-1)[idx] - fd) < 1e-6 * max(1.0, abs(fd)), (name, idx)


def test_adam_first_steps_closed_form():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 0.01
    q, m, v = er.adam_step(p, g, m, v, 1, lr, eps=0.0)
    assert np.allclose(q, p - lr * np.sign(g))
    # a constant gradient moves every coordinate by lr per step
    for t in range(2, 6):
        q, m, v = er.adam_step(q, g, m, v, t, lr, eps=0.0)
    assert np.allclose(q, p - 5 * lr * np.sign(g))


def test_histogram_boundaries_cdf_and_coverage():
    s = np.arange(1600, dtype=np.float64)
    b = er.boundaries(s)
    assert b.tolist() == [100.0 * i for i in range(16)] + [1599.0]
    for i in range(16):
        assert er.hist_cdf(b, 100.0 * i) == i / 16
    assert er.hist_cdf(b, -1) == 0.0 and er.hist_cdf(b, 1599) == 1.0
    xs = np.linspace(-10, 1700, 500)
    cdf = [er.hist_cdf(b, x) for x in xs]
    assert all(a <= c for a, c in zip(cdf, cdf[1:]))
    assert (er.coverage(b, 0, 1599) == 1).all()
    assert (er.coverage(b, 2000, 3000) == 0).all()
    c = er.coverage(b, 150, 349)
    assert c[1] == 0.5 and c[2] == 1.0 and abs(c[3] - 0.49) < 1e-12 and c[4] == 0


def test_features_unqueried_and_uniform_data():
    rng = np.random.default_rng(1)
    sample = np.sort(rng.uniform(0, 1, 16384))
    b = np.stack([er.boundaries(sample)] * 3)
    N = 10**6
    f = er.features((np.array([1]), np.array([0.25]), np.array([0.75])), b, N).reshape(3, 19)
    assert (f[0, :2] == -1).all() and f[0, 2] == 0 and (f[0, 3:] == 1).all()
    assert (f[2, :2] == -1).all()
    assert abs(f[1, 0] - 0.25) < 0.02 and abs(f[1, 1] - 0.75) < 0.02
    assert abs(f[1, 2] - math.log(2) / math.log(N)) < 0.01
    assert abs(f[1, 3:].sum() / 16 - 0.5) < 0.02
    # the partial-match interval [-inf, +inf] restricts nothing: same as no predicate
    g = er.features((np.array([0, 1]), np.array([-np.inf, 0.25]), np.array([np.inf, 0.75])), b, N)
    assert np.array_equal(g, f.reshape(-1))
    # an empty interval (lo > hi) covers nothing, has H(lo) > H(hi) and the smallest
    # representable selectivity 1/N
    e = er.features((np.array([2]), np.array([0.6]), np.array([0.4])), b, N).reshape(3, 19)
    assert e[2, 0] > e[2, 1] and (e[2, 3:] == 0).all() and e[2, 2] == 1.0


def test_base_is_the_independence_product():
    """N^-base[d] is the product of the per-dimension histogram selectivities (section
    2.1's independence assumption), until it reaches the floor 1/N."""
    s = np.arange(1600, dtype=np.float64)
    b = np.stack([er.boundaries(s)] * 4)
    N = 10**7
    q = (np.array([0, 2, 3]), np.array([0.0, 100.0, 800.0]), np.array([400.0, 900.0, 1200.0]))
    base = er.base(q, b, N)
    per = [400 / 1600, 800 / 1600, 400 / 1600]  # exact on this grid of boundaries
    assert np.allclose(er.selectivity_from_output(base[[0, 2, 3]], N), per, rtol=1e-12)
    assert base[1] == 0
    assert abs(er.selectivity_from_output(base[4:], N)[0] - np.prod(per)) < 1e-15
    tiny = (np.array([0, 1, 2]), np.array([0.0] * 3), np.array([1.0] * 3))
    assert er.base(tiny, b, N)[4] == 1.0  # (1/1600)^3 < 1/N: clamped
    # the base shifts the network output one to one
    rng = np.random.default_rng(2)
    p = _params(rng, K=4 * 19, O=5)
    X = rng.uniform(-1, 1, (3, 4 * 19))
    Y0, _ = er.forward(p, X, rounding=False)
    Y1, _ = er.forward(p, X, np.stack([base] * 3), rounding=False)
    assert np.allclose(Y1 - Y0, base, atol=1e-15)


def test_targets_and_qerror():
    y, m = er.targets({2: 0.5, 0: 1e-9}, 1e-3, 4, 1000)
    assert m.tolist() == [1, 0, 1, 0, 1]
    assert abs(y[0] - 1.0) < 1e-12            # clamped at 1/N
    assert abs(y[2] - math.log(2) / math.log(1000)) < 1e-12
    assert abs(er.selectivity_from_output(y[4:5], 1000)[0] - 1e-3) < 1e-12
    q = er.qerror([0.1, 0.01, 1e-9], [0.01, 0.1, 1e-12], 1000)
    assert np.allclose(q, [10, 10, 1])


def test_rounded_paths_on_a_hand_computed_network():
    """Where the bfloat16 roundings sit, pinned by a one-unit network worked out by hand.

    Every pre-activation is above 8, where erf(z / sqrt 2) is 1 in float64, so GELU is
    the identity and its derivative 1; the only changes to the numbers are the
    roundings.  bfloat16 keeps 8 significant bits: the spacing is 2^-7 on [1, 2),
    2^-9 on [0.25, 0.5), 2^-4 on [8, 16).

    Forward (operands rounded, biases and base not):
      x  = 1 + 3*2^-9  -> 1 + 2^-7 = 1.0078125        (3/4 of a unit: up)
      W1 = 10.03       -> 10.0                        (0.03 < half of 2^-4)
      z1 = 1.0078125 * 10 + 0.001 = 10.079125 -> h1 = 10.0625
      W2 = 1.5 + 2^-9  -> 1.5
      z2 = 10.0625 * 1.5 + 0.003 = 15.09675  -> h2 = 15.125  (0.03425 > 2^-5: up)
      W3 = 0.2509      -> 0.25
      y  = 15.125 * 0.25 + 0.0007 + 0.5 (base) = 4.28195
    Backward (product operands rounded, bias gradients from the unrounded values):
      dy = 1 + 3*2^-9 -> 1.0078125
      dW3 = 15.125 * 1.0078125 = 15.2431640625;  db3 = 1.005859375
      dz2 = 1.0078125 * 0.25 = 0.251953125 (on the grid)
      dW2 = 10.0625 * 0.251953125 = 2.5352783203125;  db2 = 0.251953125
      dz1 = 0.251953125 * 1.5 = 0.3779296875 = 193.5 units of 2^-9: a tie, to even
            -> 194 * 2^-9 = 0.37890625
      dW1 = 1.0078125 * 0.37890625 = 0.381866455078125;  db1 = 0.3779296875
    """
    p = {"W1": np.array([[10.03]]), "b1": np.array([0.001]),
         "W2": np.array([[1.5 + 2 ** -9]]), "b2": np.array([0.003]),
         "W3": np.array([[0.2509]]), "b3": np.array([0.0007])}
    X = np.array([[1 + 3 * 2 ** -9]])
    Y, cache = er.forward(p, X, np.array([[0.5]]))
    assert cache["X"][0, 0] == 1.0078125 and cache["W1"][0, 0] == 10.0
    assert cache["H1"][0, 0] == 10.0625 and cache["H2"][0, 0] == 15.125
    assert abs(Y[0, 0] - 4.28195) < 1e-12
    g = er.backward(cache, np.array([[1 + 3 * 2 ** -9]]))
    assert g["W3"][0, 0] == 15.2431640625 and g["b3"][0] == 1.005859375
    assert g["W2"][0, 0] == 2.5352783203125 and g["b2"][0] == 0.251953125
    assert g["W1"][0, 0] == 0.381866455078125 and g["b1"][0] == 0.3779296875
    # the unrounded path gives other numbers (so the roundings above are exercised)
    Yu, cu = er.forward(p, X, np.array([[0.5]]), rounding=False)
    assert abs(Yu[0, 0] - 4.28195) > 1e-3
    gu = er.backward(cu, np.array([[1 + 3 * 2 ** -9]]), round_like_gpu=False)
    assert gu["W1"][0, 0] != g["W1"][0, 0]


def test_rounded_paths_equal_unrounded_on_grid_values():
    """Operands that bfloat16 holds exactly (small integers, powers of two), with every
    pre-activation an integer in [12, 256) so that GELU is the identity and keeps
    activations on the grid: the rounded forward and backward equal the unrounded ones
    bit for bit."""
    rng = np.random.default_rng(7)
    K, H, O, n = 3, 4, 2, 5
    p = {"W1": rng.integers(2, 5, (K, H)).astype(np.float64), "b1": np.zeros(H),
         "W2": rng.integers(1, 3, (H, H)).astype(np.float64), "b2": np.zeros(H),
         "W3": 2.0 ** -rng.integers(1, 6, (H, O)), "b3": np.zeros(O)}
    X = rng.integers(2, 5, (n, K)).astype(np.float64)
    Yr, cr = er.forward(p, X)
    Yu, cu = er.forward(p, X, rounding=False)
    assert (cr["H1"] >= 12).all() and (cr["H2"] < 256).all()
    assert np.array_equal(Yr, Yu)
    dY = 2.0 ** -rng.integers(1, 6, (n, O))
    gr = er.backward(cr, dY)
    gu = er.backward(cu, dY, round_like_gpu=False)
    for k in gr:
        assert np.array_equal(gr[k], gu[k]), k

"""CPU reference of the learned selectivity estimator.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product library never uses
it.  Everything is plain numpy in float64; where the GPU path rounds an operand to
bfloat16 before a matrix product, this reference rounds the same operand the same
way (round to nearest, ties to even) and then computes exactly in float64.

Definitions (these are the estimator's, not the paper's: the paper only notes that
ordering dimensions by selectivity needs estimates, section 2.2.4, lists it as future
work, section 8, and defines selectivity and the independence product, section 2.1):

* Equi-depth histogram of a column: from a sorted sample s[0..M), B bins with
  boundaries b_i = s[floor(i*M/B)] for i < B and b_B = s[M-1].
* CDF of the histogram, piecewise linear: H(x) = (i + (x - b_i)/(b_{i+1} - b_i)) / B
  on [b_i, b_{i+1}), 0 below b_0, 1 from b_B on; an empty bin (b_i == b_{i+1})
  contributes a step.
* Log scale: y(s) = -ln(max(s, 1/N)) / ln(N) in [0, 1], so s = N^-y.
* Coverage of bin i: |[lo,hi] & [b_i,b_{i+1}]| / (b_{i+1} - b_i) (an empty bin counts
  as covered iff lo <= b_i <= hi).  Histogram estimate of a predicate: the mean
  coverage over the bins (H(hi) - H(lo) for lo <= hi, without the cancellation).
* Features of a query, per dimension j (B + 3 values): restricted -> H_j(lo), H_j(hi),
  y(histogram estimate) and the B coverages; not restricted (no predicate, or the
  interval [-inf, +inf]) -> (-1, -1, 0) and all bins covered.
* Base estimate (d + 1 values): the histogram estimate of each restricted dimension
  (0 elsewhere) and, last, min(1, their sum) -- the independence product of the
  per-dimension estimates (section 2.1) on the log scale.
* Targets: y(s) for each restricted dimension's own selectivity and for the joint
  selectivity.
* Network: a learned correction of the base estimate.  X -> GELU(X W1 + b1) ->
  GELU(H1 W2 + b2) -> H2 W3 + b3 + base, GELU(z) = z * Phi(z) (erf form).  Loss: mean
  of (y_hat - y)^2 over the targets present.
* Adam (Kingma & Ba 2015) with bias correction.
* q-error: max(s_hat / s, s / s_hat), both clamped to at least 1/N.
"""
from __future__ import annotations

import math

import numpy as np

BINS = 16


# ---------------------------------------------------------------- bfloat16

def bf16_round(x) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(f.shape)


# ---------------------------------------------------------------- histograms, features

def boundaries(sorted_sample: np.ndarray, bins: int = BINS) -> np.ndarray:
    s = np.asarray(sorted_sample, dtype=np.float64)
    m = len(s)
    b = np.array([s[(i * m) // bins] for i in range(bins)] + [s[m - 1]], dtype=np.float64)
    return b


def hist_cdf(b: np.ndarray, x: float) -> float:
    bins = len(b) - 1
    if x < b[0]:
        return 0.0
    if x >= b[bins]:
        return 1.0
    for i in range(bins):
        if b[i] <= x < b[i + 1]:
            return (i + (x - b[i]) / (b[i + 1] - b[i])) / bins
    return 1.0


def coverage(b: np.ndarray, lo: float, hi: float) -> np.ndarray:
    bins = len(b) - 1
    out = np.zeros(bins)
    for i in range(bins):
        a, c = b[i], b[i + 1]
        if c > a:
            out[i] = max(0.0, min(hi, c) - max(lo, a)) / (c - a)
        else:
            out[i] = 1.0 if lo <= a <= hi else 0.0
    return out


def log_scale(s, n_rows: int):
    return -math.log(max(s, 1.0 / n_rows)) / math.log(n_rows)


def _restricted(query):
    for j, lo, hi in zip(*query):
        j, lo, hi = int(j), float(lo), float(hi)
        if lo == -math.inf and hi == math.inf:
            continue  # the partial-match interval restricts nothing (section 2.1)
        yield j, lo, hi


def features(query, bnds: np.ndarray, n_rows: int) -> np.ndarray:
    """bnds: (d, BINS + 1) boundaries; returns d * (BINS + 3) features."""
    d, nb1 = bnds.shape
    bins = nb1 - 1
    f = np.zeros((d, bins + 3))
    f[:, 0] = -1.0
    f[:, 1] = -1.0
    f[:, 2] = 0.0
    f[:, 3:] = 1.0
    for j, lo, hi in _restricted(query):
        f[j, 0] = hist_cdf(bnds[j], lo)
        f[j, 1] = hist_cdf(bnds[j], hi)
        f[j, 3:] = coverage(bnds[j], lo, hi)
        f[j, 2] = log_scale(f[j, 3:].mean(), n_rows)
    return f.reshape(-1)


def base(query, bnds: np.ndarray, n_rows: int) -> np.ndarray:
    """Histogram estimates on the log scale: per restricted dimension, then the
    independence product, min(1, sum)."""
    d = bnds.shape[0]
    out = np.zeros(d + 1)
    for j, lo, hi in _restricted(query):
        out[j] = log_scale(coverage(bnds[j], lo, hi).mean(), n_rows)
    out[d] = min(1.0, out[:d].sum())
    return out


def targets(sel_dims: dict, sel_joint: float, d: int, n_rows: int):
    """(y[d + 1], mask[d + 1]): sel_dims maps queried dim -> its own selectivity."""
    y = np.zeros(d + 1)
    mask = np.zeros(d + 1)
    ln = math.log(n_rows)
    for j, s in sel_dims.items():
        y[j] = -math.log(max(s, 1.0 / n_rows)) / ln
        mask[j] = 1.0
    y[d] = -math.log(max(sel_joint, 1.0 / n_rows)) / ln
    mask[d] = 1.0
    return y, mask


def selectivity_from_output(y: np.ndarray, n_rows: int) -> np.ndarray:
    yc = np.clip(y, 0.0, 1.0)
    return np.exp(-yc * math.log(n_rows))


def qerror(est, true, n_rows: int) -> np.ndarray:
    e = np.maximum(np.asarray(est, dtype=np.float64), 1.0 / n_rows)
    t = np.maximum(np.asarray(true, dtype=np.float64), 1.0 / n_rows)
    return np.maximum(e / t, t / e)


# ---------------------------------------------------------------- network

def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * phi


def _erf(x):
    x = np.asarray(x, dtype=np.float64)
    return np.vectorize(math.erf, otypes=[np.float64])(x)


def forward(params: dict, X: np.ndarray, base_y=None, rounding: bool = True):
    """params: W1 (K x H), b1, W2 (H x H), b2, W3 (H x O), b3 (float32 masters);
    base_y: (n, O) base estimates added to the output (None: zero).
    Matrix operands are rounded to bfloat16 as on the GPU (rounding=False: no rounding,
    for derivative checks); sums are exact (float64).  Returns (Y, cache)."""
    r = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    Xb = r(X)
    W1, W2, W3 = (r(params[k]) for k in ("W1", "W2", "W3"))
    b1, b2, b3 = (np.asarray(params[k], dtype=np.float64) for k in ("b1", "b2", "b3"))
    Z1 = Xb @ W1 + b1
    H1 = r(gelu(Z1).astype(np.float32)) if rounding else gelu(Z1)
    Z2 = H1 @ W2 + b2
    H2 = r(gelu(Z2).astype(np.float32)) if rounding else gelu(Z2)
    Y = H2 @ W3 + b3
    if base_y is not None:
        Y = Y + np.asarray(base_y, dtype=np.float64)
    return Y, {"X": Xb, "W1": W1, "W2": W2, "W3": W3, "Z1": Z1, "H1": H1, "Z2": Z2, "H2": H2}


def loss_and_grad_y(Y: np.ndarray, T: np.ndarray, M: np.ndarray):
    n = M.sum()
    diff = (Y - T) * M
    return float((diff * diff).sum() / n), 2.0 * diff / n


def backward(cache: dict, dY: np.ndarray, round_like_gpu: bool = True):
    """Gradients of the loss with respect to the float32 master parameters, through the
    bfloat16-rounded forward pass (rounding treated as identity, as on the GPU).  With
    round_like_gpu the gradient operands of each product are rounded to bfloat16 the way
    the GPU rounds them."""
    r = bf16_round if round_like_gpu else (lambda a: np.asarray(a, dtype=np.float64))
    X, W1, W2, W3 = cache["X"], cache["W1"], cache["W2"], cache["W3"]
    H1, H2, Z1, Z2 = cache["H1"], cache["H2"], cache["Z1"], cache["Z2"]
    dYr = r(np.asarray(dY, dtype=np.float32))
    g = {}
    g["W3"] = H2.T @ dYr
    g["b3"] = np.asarray(dY, dtype=np.float64).sum(axis=0)
    dH2 = dYr @ W3.T
    dZ2 = dH2 * gelu_grad(Z2)
    dZ2r = r(dZ2.astype(np.float32))
    g["W2"] = H1.T @ dZ2r
    g["b2"] = dZ2.sum(axis=0)
    dH1 = dZ2r @ W2.T
    dZ1 = dH1 * gelu_grad(Z1)
    dZ1r = r(dZ1.astype(np.float32))
    g["W1"] = X.T @ dZ1r
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update of parameter p; returns (p, m, v).  t counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

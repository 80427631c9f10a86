"""Reference computation of the learned clause priority -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP library.

The paper motivates it but does not define it: Section 3.2 measures that a
clause used recently is likely to be used again soon, and Section 3.7 keeps the
GPU's clause store small with MiniSat-style activity (bumped whenever a clause
triggers).  The learned priority turns that observation into a schedule: a small
network scores each clause from its history, and clauses that score low are
tested only on every fourth run.  Everything below is the plain definition of
that extension, in float64:

* features of a clause (12): log1p(length), log1p(LBD), log1p(age in runs),
  source thread / max(1, n_sources - 1), and log1p of its hit count (slots in
  which it was falsified, summed over the words) in each of the last 8 runs
  that tested it, most recent first;
* network: z1 = x W1 + b1, h1 = relu(z1), z2 = h1 W2 + b2, h2 = relu(z2),
  z3 = h2 w3 + b3, p = sigmoid(z3); parameters packed as W1[12][64] (input
  major), b1[64], W2[64][64], b2[64], w3[64], b3 -- 5057 numbers;
* loss: mean binary cross-entropy, written as softplus(z3) - y z3;
* training: Adam (Kingma and Ba, 2015) on minibatches taken in a given order;
* schedule: in run r, a clause whose score is below the threshold is tested
  only when (r + id) mod 4 = 0; every other clause is tested in every run;
* activity (Section 3.7): MiniSat-style, bumped by decay**-r when a clause hits
  in run r; a reduction keeps the most active clauses, the newest among equals.
"""
from __future__ import annotations

import numpy as np

N_FEATURES = 12
HIDDEN = 64
HISTORY = 8
SHAPES = [("W1", (N_FEATURES, HIDDEN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("w3", (HIDDEN,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 5057


def unpack(params: np.ndarray) -> dict:
    """Named float64 views of the packed parameter vector."""
    params = np.asarray(params, dtype=np.float64)
    if params.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters")
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = params[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(params: np.ndarray, x: np.ndarray) -> dict:
    """Every intermediate of the network for a batch x [n][12]."""
    p = unpack(params)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["w3"] + p["b3"][0]
    prob = 1.0 / (1.0 + np.exp(-z3))
    return dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, prob=prob)


def loss(params: np.ndarray, x: np.ndarray, y: np.ndarray) -> float:
    z3 = forward(params, x)["z3"]
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(np.logaddexp(0.0, z3) - y * z3))


def loss_grad(params: np.ndarray, x: np.ndarray, y: np.ndarray):
    """(mean BCE, gradient with respect to the packed parameters), by the chain
    rule through the layers above."""
    f = forward(params, x)
    p = unpack(params)
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    dz3 = (f["prob"] - y) / n                      # d loss / d z3
    g = {"w3": f["h2"].T @ dz3, "b3": np.array([dz3.sum()])}
    dz2 = np.outer(dz3, p["w3"]) * (f["z2"] > 0)   # through w3 and relu
    g["W2"] = f["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * (f["z1"] > 0)        # through W2 and relu
    g["W1"] = f["x"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    value = float(np.mean(np.logaddexp(0.0, f["z3"]) - y * f["z3"]))
    return value, pack(g)


def adam(params, x, y, batches, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam over the given minibatches (a list of index arrays into x, y);
    returns the parameters and the loss of each step."""
    theta = np.asarray(params, dtype=np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = []
    for t, idx in enumerate(batches, start=1):
        value, g = loss_grad(theta, x[idx], y[idx])
        losses.append(value)
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        mhat = m / (1 - beta1 ** t)
        vhat = v / (1 - beta2 ** t)
        theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, np.array(losses)


def features(length, lbd, age, source, n_sources, history) -> np.ndarray:
    """The 12 features of clauses (arrays of one entry per clause; history is
    [n][8] hit counts, most recent first)."""
    history = np.asarray(history, dtype=np.float64)
    x = np.empty((len(history), N_FEATURES))
    x[:, 0] = np.log1p(np.asarray(length, dtype=np.float64))
    x[:, 1] = np.log1p(np.asarray(lbd, dtype=np.float64))
    x[:, 2] = np.log1p(np.asarray(age, dtype=np.float64))
    x[:, 3] = np.asarray(source, dtype=np.float64) / max(1, n_sources - 1)
    x[:, 4:] = np.log1p(history)
    return x


def tested(ids, low, run: int) -> np.ndarray:
    """Which clauses the schedule tests in a run: all but the low-score ones
    whose (run + id) mod 4 is not 0."""
    ids = np.asarray(ids, dtype=np.int64)
    return ~np.asarray(low, dtype=bool) | ((run + ids) % 4 == 0)


def activity(hits_by_run, decay: float) -> np.ndarray:
    """MiniSat-style clause activity after the given runs (Section 3.7: the GPU
    deletes clauses by activity, bumped whenever a clause triggers): in run r
    (0-based) every clause with a hit gains decay**-r, the bump that grows by
    1/decay after each run.  hits_by_run: [runs][n] hit counts (or booleans)."""
    h = np.asarray(hits_by_run) > 0
    bumps = np.power(float(decay), -np.arange(h.shape[0], dtype=np.float64))
    return bumps @ h.astype(np.float64)


def reduce_keep(act, ids, keep: int) -> np.ndarray:
    """The ids a reduction to `keep` clauses keeps: the highest activities, and
    among equal activities the newest (larger id)."""
    act = np.asarray(act, dtype=np.float64)
    ids = np.asarray(ids)
    order = np.lexsort((ids, act))  # ascending activity, then ascending id: removal order
    return np.sort(ids[order[len(ids) - keep:]]) if keep < len(ids) else np.sort(ids)


def hit_counts(dense: np.ndarray) -> np.ndarray:
    """Slots in which each clause was falsified, from dense masks [n][W]."""
    d = np.asarray(dense, dtype=np.uint64)
    return np.array([sum(bin(int(w)).count("1") for w in row) for row in d], dtype=np.int64)

"""Pins of the oracle's nonparametric bootstrap of b (Section 8.4: resample each
row's M draws with replacement).

Independent references: numpy's inverse for b of the draws, numpy's
percentile (inverted CDF) and moments for the per-node summaries, the
multinomial law of the redrawn counts (row sums, means, uniform indices),
degenerate rows, the 1 / sqrt(R) shrinkage of the spread, and the coverage of
the true profile of a known chain."""
import numpy as np
import pytest

import oracle as O


def draws_from_kernel(P, R, seed):
    """next(r, i) drawn from row i of P (columns 0..n-1 transient, n = bottom)."""
    rng = np.random.default_rng(seed)
    n = P.shape[0]
    cum = np.cumsum(P, axis=1)
    cum[:, -1] = 1.0
    u = rng.random((R, n))
    nxt = np.array([np.searchsorted(cum[i], u[:, i], side="right") for i in range(n)]).T
    return np.where(nxt >= n, -1, nxt).astype(np.int32)


def random_kernel(n, seed, leak=0.2):
    rng = np.random.default_rng(seed)
    Q = rng.random((n, n)) * (rng.random((n, n)) < 0.6)
    Q[np.arange(n), rng.integers(0, n, n)] += 0.1
    Q = Q / Q.sum(1, keepdims=True) * (1 - leak)
    return np.hstack([Q, np.full((n, 1), leak)])


def b_of(Q, s):
    mu = s @ np.linalg.inv(np.eye(len(s)) - Q)
    return mu / mu.sum()


def test_b_of_the_draws_and_summaries_match_numpy():
    n, R = 12, 300
    nt = draws_from_kernel(random_kernel(n, 1), R, 2)
    out = O.bootstrap(nt, replicates=40, level=0.9, seed=5)
    C = np.zeros((n, n + 1))
    for i in range(n):
        col = nt[:, i]
        C[i, :n] = np.bincount(col[col >= 0], minlength=n)
        C[i, n] = np.count_nonzero(col < 0)
    Q = C[:, :n] / R
    empty = C[:, n] == 0                                  # floor eta = 0.1 / sqrt(R) on an empty column
    Q[empty] *= 1.0 - 0.1 / np.sqrt(R)
    s = np.full(n, 1.0 / n)
    assert np.allclose(out["b0"], b_of(Q, s), rtol=0, atol=1e-13)
    reps = out["b_rep"]
    assert np.allclose(out["mean"], reps.mean(0), rtol=0, atol=1e-15)
    assert np.allclose(out["sd"], reps.std(0, ddof=1), rtol=1e-12, atol=1e-18)
    assert np.array_equal(out["lo"], np.percentile(reps, 5.0, axis=0, method="inverted_cdf"))
    assert np.array_equal(out["hi"], np.percentile(reps, 95.0, axis=0, method="inverted_cdf"))
    assert np.all(out["lo"] <= out["hi"])


def test_degenerate_rows_give_zero_spread():
    n, R = 6, 50
    nxt = np.array([1, 2, 3, -1, 0, -1], dtype=np.int32)
    nt = np.tile(nxt, (R, 1))
    out = O.bootstrap(nt, replicates=8, seed=1)
    assert np.all(out["sd"] <= 1e-15)                     # the mean's own rounding only
    assert np.array_equal(out["lo"], out["b0"]) and np.array_equal(out["hi"], out["b0"])
    assert np.array_equal(out["b_rep"], np.tile(out["b0"], (8, 1)))


def test_replicate_counts_are_multinomial():
    n, R = 8, 200
    nt = draws_from_kernel(random_kernel(n, 3), R, 4)
    C = np.stack([O.boot_counts(nt, 9, b) for b in range(300)]).astype(np.float64)
    assert np.all(C.sum(2) == R)                          # every row keeps R draws
    C0 = np.zeros((n, n + 1))
    for i in range(n):
        col = nt[:, i]
        C0[i, :n] = np.bincount(col[col >= 0], minlength=n)
        C0[i, n] = np.count_nonzero(col < 0)
    p = C0 / R
    se = np.sqrt(R * p * (1 - p) / C.shape[0]) + 1e-12
    assert np.all(np.abs(C.mean(0) - C0) <= 5 * se)       # E[C*] = C
    assert not np.array_equal(O.boot_counts(nt, 9, 0), O.boot_counts(nt, 9, 1))


def test_redrawn_indices_are_uniform():
    # next(r, i) = r: the counts of row i are the histogram of the redrawn indices
    R = n = 64
    nt = np.tile(np.arange(R, dtype=np.int32)[:, None], (1, n))
    h = sum(O.boot_counts(nt, 2, b)[:, :n].sum(0) for b in range(50)).astype(np.float64)
    expect = h.sum() / R
    chi2 = ((h - expect) ** 2 / expect).sum()
    assert chi2 < R - 1 + 6 * np.sqrt(2 * (R - 1))       # 63 degrees of freedom, far tail


def test_spread_shrinks_with_the_draws_and_covers_the_truth():
    n = 10
    P = random_kernel(n, 6)
    s = np.full(n, 1.0 / n)
    truth = b_of(P[:, :n], s)
    sds = []
    for R in (200, 800):
        nt = draws_from_kernel(P, R, R)
        out = O.bootstrap(nt, replicates=200, level=0.95, eta=0.0, seed=R)
        sds.append(out["sd"])
        covered = np.mean((out["lo"] <= truth) & (truth <= out["hi"]))
        assert covered >= 0.7, covered
    ratio = np.median(sds[0] / sds[1])
    assert 1.5 < ratio < 2.7, ratio                       # about sqrt(4) = 2


def test_arguments():
    nt = np.zeros((4, 3), dtype=np.int32)
    for kw in ({"replicates": 0}, {"level": 1.0}, {"level": 0.0}):
        with pytest.raises(Exception):
            O.bootstrap(nt, **kw)

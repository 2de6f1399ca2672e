"""Pins of the oracle's robust tail: sampled admissible kernels (Section 5.1 and
the robust experiment of Section 9.1), transition reward-AFCs (Section 6.4)
and the first-order sensitivity with its explicit remainder (Section 5.4).

Independent references: the admissible-set constraints themselves, numpy's
inverse for the AFC of a sampled kernel, simulated trajectories of the chain
for the switching and improvement rewards, closed special cases, the quadratic
decay of the first-order error, and the remainder inequality.
"""
import numpy as np
import pytest

import oracle as O


def random_kernel(n, seed, leak=0.2, density=0.5):
    rng = np.random.default_rng(seed)
    Q = rng.random((n, n)) * (rng.random((n, n)) < density)
    Q[np.arange(n), rng.integers(0, n, n)] += 0.1
    return Q / Q.sum(1, keepdims=True) * (1 - leak)


def test_sampled_kernels_are_admissible():
    Q0 = random_kernel(15, 1)
    for k in range(6):
        Q = O.perturbed_kernel(Q0, 9, k, 0.5, 0.05)
        assert np.all(Q >= 0) and np.all(Q <= 1)
        assert np.all(Q.sum(1) <= 1 - 0.05 + 1e-15)
        assert np.all(Q[Q0 == 0] == 0)
        ratio = Q[Q0 > 0] / Q0[Q0 > 0]
        assert ratio.min() >= 0.5 - 1e-15 and ratio.max() <= 1.5 + 1e-15
    assert np.array_equal(O.perturbed_kernel(Q0, 9, 0, 0.0, 0.05), Q0)          # radius 0 keeps Q0
    # the multipliers are uniform on [1 - delta, 1 + delta] (before the row cap)
    Qb = np.full((60, 60), 0.01)
    u = np.concatenate([(O.perturbed_kernel(Qb, 3, k, 0.5, 0.0) / 0.01).ravel() for k in range(4)])
    hist, _ = np.histogram(u, bins=10, range=(0.5, 1.5))
    assert np.abs(hist / len(u) - 0.1).max() < 5 * np.sqrt(0.09 / len(u))


def test_maximisers_and_their_afc():
    Q0 = random_kernel(20, 2)
    s = np.full(20, 0.05)
    r = O.robust(Q0, samples=10, delta=0.5, r_min=0.05, seed=4)
    b0 = s @ np.linalg.inv(np.eye(20) - Q0)
    b0 /= b0.sum()
    assert np.allclose(r["b0"], b0, rtol=0, atol=1e-13)
    assert r["kl_arg"] == int(np.argmax(r["kl"])) and r["tv_arg"] == int(np.argmax(r["tv"]))
    for arg, key in ((r["kl_arg"], "b_kl"), (r["tv_arg"], "b_tv")):
        Q = O.perturbed_kernel(Q0, 4, arg, 0.5, 0.05)
        b = s @ np.linalg.inv(np.eye(20) - Q)
        b /= b.sum()
        assert np.allclose(r[key], b, rtol=0, atol=1e-13)
    kl = r["b_kl"] @ np.log(r["b_kl"] / b0)
    assert r["kl"][r["kl_arg"]] == pytest.approx(kl, rel=1e-10)
    assert r["tv"][r["tv_arg"]] == pytest.approx(0.5 * np.abs(r["b_tv"] - b0).sum(), rel=1e-10)
    z = O.robust(Q0, samples=3, delta=0.0, r_min=0.05, seed=4)
    assert np.all(z["kl"] == 0) and np.all(z["tv"] == 0)


def _simulate_rewards(Q, s, f, episodes, rng):
    n = len(s)
    P = np.hstack([Q, (1 - Q.sum(1))[:, None]])
    cum = np.cumsum(P, axis=1)
    cum[:, -1] = 1.0
    x = rng.choice(n, size=episodes, p=s)
    alive = np.ones(episodes, bool)
    steps = sw = imp = 0.0
    while alive.any():
        idx = np.flatnonzero(alive)
        xs = x[idx]
        nxt = (cum[xs] < rng.random(len(xs))[:, None]).sum(1)
        stay = nxt < n
        steps += len(xs)
        sw += np.count_nonzero(stay & (nxt != xs))
        imp += np.maximum(f[np.minimum(nxt, n - 1)] - f[xs], 0)[stay].sum()
        x[idx[stay]] = nxt[stay]
        alive[idx[~stay]] = False
    return sw / steps, imp / steps


def test_transition_rewards_match_simulation_and_special_cases():
    n = 10
    Q0 = random_kernel(n, 5, leak=0.25)
    f = np.linspace(0.0, 3.0, n)
    r = O.robust(Q0, f=f, samples=0)
    sw, imp = _simulate_rewards(Q0, np.full(n, 0.1), f, 200000, np.random.default_rng(0))
    assert r["b_sw"] == pytest.approx(sw, abs=0.01)
    assert r["b_imp"] == pytest.approx(imp, abs=0.02)
    assert O.robust(Q0, f=np.full(n, 2.0), samples=0)["b_imp"] == 0.0          # constant value: no improvement
    D = np.diag(np.full(n, 0.6))
    assert O.robust(D, f=f, samples=0)["b_sw"] == 0.0                           # the centre never changes


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_first_order_sensitivity_is_second_order_accurate(seed):
    Q0 = random_kernel(18, 10 + seed)
    errs = []
    for delta in (2e-3, 1e-3, 5e-4):
        r = O.robust(Q0, samples=1, delta=delta, r_min=0.05, seed=seed)
        errs.append(np.abs(r["b_lin"] - r["b_kl"]).max())
        assert r["rem_actual"] <= r["rem_bound"] * (1 + 1e-12)
        assert r["norm_N0E"] < 1.0
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0
    big = O.robust(Q0, samples=4, delta=0.5, r_min=0.05, seed=seed)
    if big["norm_N0E"] < 1.0:
        assert big["rem_actual"] <= big["rem_bound"] * (1 + 1e-12)

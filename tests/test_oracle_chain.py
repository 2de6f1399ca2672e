"""Pins of the oracle's chain algebra (Section 4, Section 5, Section 6,
Section 7, Section 8.2 and Appendices A-B of the paper).

Independent references: the Appendix B worked illustration, the closed forms of
the canonical AMC and of constant hazard, numpy's dense inverse, sampled
admissible kernels for the certificate bounds, and the identities the paper
states for rewards, pools and feasibility.
"""
import numpy as np
import pytest

import oracle as O


def test_appendix_b_values(golden):
    ref = golden("appendix_b.json")
    Q0 = np.array(ref["Q0"])
    assert np.allclose(Q0.sum(1) + np.array(ref["r0"]), 1.0)
    ch = O.chain(Q0, np.array(ref["s"]))
    assert np.allclose(ch["mu"], ref["mu"], atol=5e-5)
    assert ch["ET"] == pytest.approx(ref["expected_length"], abs=5e-3)
    mu, N = ch["mu"], ch["N"]
    for pair, val in ref["gaps"].items():
        u, v = (int(x) - 1 for x in pair.split(","))
        g, crude, sharp = O.pair_certificate(N, mu, ref["epsbar"], ref["r_min"], u, v)
        assert g == pytest.approx(val, abs=5e-5)
        assert crude == pytest.approx(ref["crude_threshold"], abs=5e-5)
        assert sharp == pytest.approx(ref["sharp_thresholds"][pair], abs=5e-5)
        assert (g > crude) == ref["crude_certifies"][pair]
        assert (g > sharp) == ref["sharp_certifies"][pair]


def _sample_admissible(rng, Q0, eps, r_low, count):
    """Kernels of the row-wise set U (Section 5.1): entries within eps of Q0,
    clipped to [0, 1], row sums at most 1 - r_low.  Half are box corners."""
    n = Q0.shape[0]
    lo = np.maximum(Q0 - eps, 0.0)
    hi = np.minimum(Q0 + eps, 1.0)
    out = []
    while len(out) < count:
        if len(out) % 2:
            Q = np.where(rng.random(Q0.shape) < 0.5, lo, hi)
        else:
            Q = lo + (hi - lo) * rng.random(Q0.shape)
        if np.all(Q.sum(1) <= 1.0 - r_low):
            out.append(Q)
    return out


def test_certificate_bounds_hold_over_sampled_admissible_kernels(golden):
    ref = golden("appendix_b.json")
    Q0 = np.array(ref["Q0"])
    s = np.array(ref["s"])
    base = O.chain(Q0, s)
    rng = np.random.default_rng(0)
    worst = {}
    for Q in _sample_admissible(rng, Q0, ref["eps_entry"], ref["r_min"], 1000):
        ch = O.chain(Q, s)
        for u in range(3):
            for v in range(3):
                if u == v:
                    continue
                g0, crude, sharp = O.pair_certificate(base["N"], base["mu"], ref["epsbar"], ref["r_min"], u, v)
                dev = abs((ch["mu"][u] - ch["mu"][v]) - g0)
                assert dev <= sharp + 1e-15 and sharp <= crude / 2 + 1e-15
                worst[(u, v)] = max(worst.get((u, v), 0.0), dev / sharp)
    assert max(worst.values()) > 0.3       # the sampled corners get near the bound


@pytest.mark.parametrize("alpha", [0.05, 0.15, 0.5, 1.0])
def test_canonical_amc_closed_form(alpha):
    """Prop. (canonical AMC, Appendix A): Q = (1-alpha) 1 p gives
    N = I + ((1-alpha)/alpha) 1 p and b = alpha s + (1-alpha) p."""
    rng = np.random.default_rng(int(alpha * 100))
    n = 12
    p = rng.dirichlet(np.ones(n))
    s = rng.dirichlet(np.ones(n))
    Q = (1 - alpha) * np.outer(np.ones(n), p)
    ch = O.chain(Q, s)
    assert np.allclose(ch["N"], np.eye(n) + (1 - alpha) / alpha * np.outer(np.ones(n), p), rtol=1e-13, atol=1e-13)
    assert ch["ET"] == pytest.approx(1 / alpha, rel=1e-13)
    assert np.allclose(ch["b"], alpha * s + (1 - alpha) * p, rtol=1e-13, atol=1e-15)


def test_constant_hazard_discounted_occupancy():
    """eq. pm-discounted-occupancy: P_i,bottom = alpha for all i gives
    b = alpha sum_t (1-alpha)^t s M^t, M row-stochastic."""
    rng = np.random.default_rng(2)
    n, alpha = 9, 0.2
    M = rng.dirichlet(np.ones(n), size=n)
    s = rng.dirichlet(np.ones(n))
    ch = O.chain((1 - alpha) * M, s)
    acc, x = np.zeros(n), s.copy()
    for t in range(400):
        acc += alpha * (1 - alpha) ** t * x
        x = x @ M
    assert np.allclose(ch["b"], acc, rtol=1e-12, atol=1e-15)


def _random_kernel(rng, n, r_min):
    Q = rng.random((n, n)) * (rng.random((n, n)) < 0.3)
    r = r_min + (1 - r_min) * rng.random(n) * 0.5
    Q = Q / np.maximum(Q.sum(1, keepdims=True), 1e-300) * (1 - r)[:, None]
    return Q, 1 - Q.sum(1)


def test_fundamental_matches_numpy_and_invariants():
    rng = np.random.default_rng(4)
    for n in (1, 2, 7, 60):
        Q, r = _random_kernel(rng, n, 0.1)
        s = rng.dirichlet(np.ones(n))
        ch = O.chain(Q, s)
        Nref = np.linalg.inv(np.eye(n) - Q)
        assert np.allclose(ch["N"], Nref, rtol=1e-12, atol=1e-13)
        assert np.abs(ch["N"]).sum(1).max() <= 1 / r.min() + 1e-12          # eq. pm-N-bound
        assert ch["b"].sum() == pytest.approx(1.0, abs=1e-14)
        assert ch["ET"] >= 1.0 - 1e-14
        assert np.allclose(ch["N"] @ r, 1.0, atol=1e-12)                    # absorption is certain
        assert np.all(ch["N"] >= -1e-15)


def test_counts_to_kernel_and_floor():
    n, R = 4, 100
    C = np.array([[10, 20, 30, 0, 40], [50, 50, 0, 0, 0], [0, 0, 0, 0, 100], [1, 2, 3, 4, 90]], dtype=np.uint32)
    eta = 0.01
    Q, r = O.counts_to_kernel(C, R, eta)
    assert np.allclose(Q[0], [0.1, 0.2, 0.3, 0.0]) and r[0] == pytest.approx(0.4)
    assert np.allclose(Q[1], [0.495, 0.495, 0, 0]) and r[1] == pytest.approx(eta)    # floored row
    assert np.allclose(Q.sum(1) + r, 1.0, atol=1e-15)                                 # rows stay normalised
    Qraw, _ = O.counts_to_kernel(C, R, 0.0)
    assert np.abs(Q - Qraw).sum(1).max() <= eta + 1e-15                               # Section 8.3: l1 row change <= eta


def test_tail_rewards_pool_feasibility_identities():
    rng = np.random.default_rng(6)
    n, R = 20, 500
    pool = np.array([2, 5, 11, 17])
    C = np.zeros((n, n + 1), np.uint32)
    Cw = np.zeros((n, n + 1), np.uint32)
    for i in range(n):
        C[i] = rng.multinomial(R, rng.dirichlet(np.ones(n + 1) * 0.3))
        pw = np.zeros(n + 1)
        pw[pool] = rng.random(len(pool))
        pw[n] = 1.0
        Cw[i] = rng.multinomial(R, pw / pw.sum())
    f = np.zeros(n)
    f[pool] = rng.uniform(0.5, 2.0, len(pool))
    s_pool = np.zeros(n)
    s_pool[pool] = 1.0 / len(pool)
    for s in (None, s_pool):
        out = O.tail(C, R, s=s, f=f, pool=pool, counts_w=Cw, eps=1e-3, r_lower=0.05, cert_topk=5)
        assert out["b_f"] == pytest.approx(float(out["b"] @ f), rel=1e-14)                 # eq. mr-inner-product
        assert np.allclose(out["xi"], 1 - Cw[:, n] / R)                                     # eq. settopk-xi
        assert out["m_w"] == pytest.approx(out["b_w"][pool].sum(), rel=1e-14)               # eq. settopk-bPsi
        assert out["b_w_f"] == pytest.approx(float(out["b_w"] @ f), rel=1e-14)
        assert out["b_w_bar"][pool].sum() == pytest.approx(1.0, abs=1e-14)
        if s is not None:
            assert out["m_w"] == pytest.approx(1.0, abs=1e-14)     # supp s in W gives m_W = 1 (Section 7.2)
        # certificates against explicit formulas
        top = np.lexsort((np.arange(n), -out["b"]))[:5]
        assert np.array_equal(out["top"], top)
        rest = np.setdiff1d(np.arange(n), top)
        assert np.array_equal(out["cert_v"], rest)
        assert out["epsbar"] == pytest.approx(n * 1e-3)
        assert out["cert_crude"] == pytest.approx(2 * n * 1e-3 / 0.05 ** 2)
        N, mu = out["N"], out["mu"]
        for a, u in enumerate(top):
            for c, v in enumerate(rest):
                assert out["cert_gap"][a, c] == pytest.approx(mu[u] - mu[v], abs=1e-15)
                assert out["cert_sharp"][a, c] == pytest.approx(n * 1e-3 / 0.05 * np.abs(N[:, u] - N[:, v]).max(),
                                                                rel=1e-14)


def test_support_restricted_threshold_without_radius():
    """eps = 0 certifies every strict nominal order; the support-restricted
    threshold uses epsbar_supp = eps * max_i |supp Q_i| in eq. sharp-gap."""
    rng = np.random.default_rng(8)
    n, R = 12, 300
    C = np.stack([rng.multinomial(R, rng.dirichlet(np.ones(n + 1) * 0.5)) for _ in range(n)]).astype(np.uint32)
    out = O.tail(C, R, eps=0.0, r_lower=0.05, cert_topk=3)
    assert np.all(out["cert_sharp"] == 0.0) and np.all(out["cert_sharp_supp"] == 0.0)
    out = O.tail(C, R, eps=2e-3, r_lower=0.05, cert_topk=3)
    Q = out["Q"]
    supp = int((Q > 0).sum(1).max())
    assert out["epsbar_supp"] == pytest.approx(supp * 2e-3)
    N = out["N"]
    for a, u in enumerate(out["top"]):
        for c, v in enumerate(out["cert_v"]):
            assert out["cert_sharp_supp"][a, c] == pytest.approx(supp * 2e-3 / 0.05 * np.abs(N[:, u] - N[:, v]).max(),
                                                                 rel=1e-13)

"""Input generators that carry a definition of the paper: the multi-reward
node values of Section 9.1, solved by hand on small graphs."""
import numpy as np

from paper_2605_14743_amd import workloads as W


def test_multi_reward_path():
    # path 0-1-...-6: degrees 1,2,2,2,2,2,1, so the hubs are 1, 2, 3
    g = W.canonical(7, [(i, i + 1) for i in range(6)])
    f = W.multi_reward(g)
    assert np.allclose(f, [6.0, 10.0, 10.0, 10.0, 6.0, 3.6, 2.16], rtol=1e-15)


def test_multi_reward_star_and_unreachable():
    # star centre 0 with leaves 1..5, vertex 6 isolated: hubs 0, 1, 2
    g = W.canonical(7, [(0, i) for i in range(1, 6)])
    f = W.multi_reward(g)
    assert np.allclose(f, [10.0, 10.0, 10.0, 6.0, 6.0, 6.0, 0.0], rtol=1e-15)


def test_multi_reward_two_components_and_parameters():
    # K4 on 0..3 (degree 3) and the path 4-5-6 (degrees 1, 2, 1): hubs 0, 1, 2
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (4, 5), (5, 6)]
    g = W.canonical(7, pairs)
    f = W.multi_reward(g, R=2.0, beta=0.5)
    assert np.allclose(f, [2.0, 2.0, 2.0, 1.0, 0.0, 0.0, 0.0])
    f1 = W.multi_reward(g, hubs=5, R=2.0, beta=0.5)   # hubs 0..3 (degree 3) and 5 (degree 2)
    assert np.allclose(f1, [2.0, 2.0, 2.0, 2.0, 1.0, 2.0, 1.0])

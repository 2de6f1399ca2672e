"""Pins of the oracle's counter-based generator and its integer event mapping.

The generator is Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  It is
pinned by the published known-answer vectors and by an independent
implementation (the open-source ATen header shipped with PyTorch), compiled
here and driven on the same (counter, key) pairs.
"""
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

KAT = [  # Random123 known-answer vectors for philox4x32 with 10 rounds
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_known_answer_vectors(ctr, key, expect):
    assert tuple(int(x) for x in O.philox4x32_10(ctr, key)) == expect


_ATEN_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    at::Philox4_32 eng(((uint64_t)k1 << 32) | k0, ((uint64_t)c3 << 32) | c2, ((uint64_t)c1 << 32) | c0);
    unsigned a = eng(), b = eng(), c = eng(), d = eng();
    std::printf("%08x %08x %08x %08x\n", a, b, c, d);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def aten_philox(tmp_path_factory):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if shutil.which("g++") is None or not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        pytest.skip("g++ or the ATen Philox header is not available")
    d = tmp_path_factory.mktemp("aten")
    src = d / "p.cpp"
    src.write_text(_ATEN_SRC)
    exe = d / "p"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc, str(src), "-o", str(exe)], check=True)

    def run(rows):
        text = "".join(" ".join("%x" % x for x in r) + "\n" for r in rows)
        out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout
        return np.array([[int(t, 16) for t in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    return run


def test_matches_independent_aten_implementation(aten_philox):
    rng = np.random.default_rng(123)
    rows = rng.integers(0, 2 ** 32, size=(400, 6), dtype=np.uint64)
    rows[:50, 2:4] = 0          # small counters as used by the sweep
    rows[50:60, 2] = 0xFFFFFFFF  # the stop-coin counter word
    ref = aten_philox(rows.tolist())
    mine = np.array([O.philox4x32_10(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    assert np.array_equal(ref, mine)


def test_realization_keying_against_aten(aten_philox):
    """alive(e) = [x0 >= floor(p 2^32)] on counter (r, u, v, 0); weight from x1."""
    from paper_2605_14743_amd import workloads as W
    g = W.er_graph(30, 0.3, 5)
    seed, r, p = 0x1234_5678_9ABC_DEF0, 77, 0.3
    alive, w = O.realize(g.n, g.eu, g.ev, seed, r, p_fail=p, weight="uniform", w_lo=3, w_hi=9)
    rows = [[r, int(u), int(v), 0, seed & 0xFFFFFFFF, seed >> 32] for u, v in zip(g.eu, g.ev)]
    x = aten_philox(rows)
    T = int(Fraction(p) * 2 ** 32)  # exact floor(p * 2^32)
    assert np.array_equal(alive, (x[:, 0] >= T).astype(np.uint8))
    assert np.array_equal(w, (3 + ((x[:, 1].astype(object) * 7) >> 32)).astype(np.uint32))
    # the stop coin uses counter (r, i, 0xFFFFFFFF, 1)
    xs = aten_philox([[r, i, 0xFFFFFFFF, 1, seed & 0xFFFFFFFF, seed >> 32] for i in range(g.n)])
    Ta = int(Fraction(0.15) * 2 ** 32)
    assert [O.stop_coin(seed, r, i, 0.15) for i in range(g.n)] == [bool(v < Ta) for v in xs[:, 0]]


@pytest.mark.parametrize("p", [0.0, 1e-12, 0.05, 0.1, 0.15, 0.2, 0.5, 1 / 3, 0.999999999, 1.0, 1.5, -0.1])
def test_threshold_is_exact_floor(p):
    expect = 0 if p <= 0 else (2 ** 32 if p >= 1 else int(Fraction(p) * 2 ** 32))
    assert O.prob_threshold(p) == expect


def test_uniformity_chi2():
    rng = np.random.default_rng(7)
    ctr = rng.integers(0, 2 ** 32, size=(4000, 4), dtype=np.uint64)
    xs = np.concatenate([O.philox4x32_10(c, (1, 2)) for c in ctr]).astype(np.float64)
    counts, _ = np.histogram(xs / 2 ** 32, bins=32, range=(0, 1))
    e = len(xs) / 32
    chi2 = float(((counts - e) ** 2 / e).sum())
    assert chi2 < 70.0   # 31 dof: P(chi2 > 70) ~ 1e-4


def test_failure_rate_and_weight_range():
    from paper_2605_14743_amd import workloads as W
    g = W.ws_graph(200, 10, 0.1, 3)
    alive_all, w_all = [], []
    for r in range(40):
        a, w = O.realize(g.n, g.eu, g.ev, 9, r, p_fail=0.2, weight="uniform", w_lo=1, w_hi=10)
        alive_all.append(a)
        w_all.append(w)
    a = np.concatenate(alive_all)
    w = np.concatenate(w_all)
    # Hoeffding at delta = 1e-9
    tol = np.sqrt(np.log(2 / 1e-9) / (2 * len(a)))
    assert abs(a.mean() - 0.8) < tol
    assert w.min() == 1 and w.max() == 10
    freq = np.bincount(w, minlength=11)[1:] / len(w)
    assert np.all(np.abs(freq - 0.1) < np.sqrt(np.log(20 / 1e-9) / (2 * len(w))))

"""Model of the shared-step protocol of the trajectory kernel (L2 layout),
run under random interleavings on the CPU.

An owner workgroup publishes a step as a claim word (epoch, |K|, next) after
clearing its completion word; its wavefronts claim sources by atomic adds,
issuing the next claim before a source runs; workgroups that have run out of
episodes claim by an add after checking that sources remain, and an add that
lands in a later step of the same owner is a claim of that step.  The owner
waits until the completion word covers |K| - 1 sources.  Every atomic
operation is one indivisible scheduler step here; everything else may
interleave arbitrarily.  The checks: each step runs exactly the sources
1 .. |K| - 1, once each; every wait ends; the source field never reaches
2^16 (it holds |K| plus at most one lost add per wavefront)."""
import random

import pytest


def simulate(seed, nb, waves, episodes, max_steps=5, kmax=12):
    rng = random.Random(seed)
    claim = [0] * nb
    done = [0] * nb
    ctr = {"next_ep": 0, "ended": 0}
    ran = {}
    steps_of = {e: rng.randint(1, max_steps) for e in range(episodes)}

    def run_source(b, ep, k):
        for _ in range(rng.randint(1, 3)):
            yield
        ran.setdefault((b, ep), []).append(k)

    def owner_wave(b, ep, sz):
        old = claim[b]
        claim[b] += 1
        k = old & 0xFFFF
        yield
        while k < sz:
            old = claim[b]
            claim[b] += 1
            kn = old & 0xFFFF
            yield
            yield from run_source(b, ep, k)
            done[b] += 1
            yield
            k = kn

    def helper(me, w):
        start = (me * 7 + w * 131) % nb
        while ctr["ended"] < episodes:
            yield
            found = next(((start + j) % nb for j in range(nb)
                          if (claim[(start + j) % nb] & 0xFFFF) < ((claim[(start + j) % nb] >> 16) & 0xFFFF)), -1)
            yield
            if found < 0:
                continue
            w_now = claim[found]
            yield
            start = (found + 1) % nb
            if (w_now & 0xFFFF) < ((w_now >> 16) & 0xFFFF):
                yield
                old = claim[found]
                claim[found] += 1
                k, sz, ep = old & 0xFFFF, (old >> 16) & 0xFFFF, old >> 32
                assert k < 0x10000 - 1
                if k < sz:
                    start = found
                    yield
                    yield from run_source(found, ep, k)
                    done[found] += (1 << 32) | 1
            yield

    def workgroup(b):
        epoch = 1
        while True:
            e = ctr["next_ep"]
            ctr["next_ep"] += 1
            yield
            if e >= episodes:
                break
            for _ in range(steps_of[e]):
                sz = rng.randint(1, kmax)
                done[b] = 0
                yield
                claim[b] = (epoch << 32) | (sz << 16) | 1
                yield
                ws = [owner_wave(b, epoch, sz) for _ in range(waves)]
                while ws:
                    w = rng.choice(ws)
                    try:
                        next(w)
                    except StopIteration:
                        ws.remove(w)
                    yield
                polls = 0
                while (done[b] & 0xFFFFFFFF) < sz - 1:
                    polls += 1
                    assert polls < 10 ** 6, "the owner's wait did not end"
                    yield
                assert sorted(ran.get((b, epoch), [])) == list(range(1, sz)), (b, epoch, sz)
                epoch += 1
                yield
            ctr["ended"] += 1
            yield
        hs = [helper(b, w) for w in range(waves)]
        while hs:
            h = rng.choice(hs)
            try:
                next(h)
            except StopIteration:
                hs.remove(h)
            yield

    actors = [workgroup(b) for b in range(nb)]
    turns = 0
    while actors:
        a = rng.choice(actors)
        try:
            next(a)
        except StopIteration:
            actors.remove(a)
        turns += 1
        assert turns < 10 ** 7, "the launch did not end"
    assert ctr["ended"] == episodes
    helped = sum(1 for (b, ep), ks in ran.items())
    return helped


@pytest.mark.parametrize("block", range(4))
def test_shared_steps_under_random_interleavings(block):
    for seed in range(block * 150, (block + 1) * 150):
        simulate(seed, nb=1 + seed % 5, waves=1 + seed % 3, episodes=1 + seed % 11)

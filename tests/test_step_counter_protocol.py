"""The step-counter protocol of the 32-source subdomain solve, run as a model
on the CPU under random schedules (no GPU).

In the kernel the two source halves of a group (each RT product waves) and the
NE expansion waves advance through the block steps without a workgroup
barrier, synchronised by five LDS counters:
  P[h]  product phases of half h done (its reads of the factor block finished),
  E     expansions done (block s + 1 written during step s),
  X[h]  recurrences of half h done (its next operand written).
A product wave of half h at step s waits for E >= NE s and X[h] >= RT s, reads
factor buffer s % 2 and operand buffer (h, s % 2), signals P[h], writes its
part of operand buffer (h, (s + 1) % 2) and signals X[h].  An expansion wave at
step s (s + 1 < nsteps) waits for E >= NE s, P[0] >= RT s and P[1] >= RT s,
writes its part of block s + 1 into factor buffer (s + 1) % 2 and signals E.

The model interleaves the waves' actions at random and checks what the kernel
relies on: every read sees the whole intended block or operand (all parts
written for that step), and no buffer is overwritten while a wave is still
reading it.  Two plausible mistakes -- one shared product counter for both
halves, and expansion waves that do not wait for each other -- must be caught.
"""
import random

import pytest

RT, NE = 5, 6


def run(nsteps, seed, shared_p=False, peer_wait=True):
    """Simulate one workgroup; returns None when every check held, else a message."""
    rng = random.Random(seed)
    P, X, E = [0, 0], [0, 0], [0]
    # factor buffers: part e of buffer b holds the block it was last written with
    M = [[0] * NE, [None] * NE]                       # block 0 expanded before the loop
    Xo = [[[0] * RT, [None] * RT] for _ in range(2)]  # operand of step 0 written before the loop
    readers_M = [set(), set()]                        # waves inside their reads of a factor buffer
    readers_X = [[set(), set()] for _ in range(2)]

    def pcount(h):
        return P[0] + P[1] if shared_p else P[h]

    def ptarget(s):
        return 2 * RT * s if shared_p else RT * s

    def product_wave(h, r):
        for s in range(nsteps):
            yield lambda: E[0] >= NE * s and X[h] >= RT * s
            b = s % 2
            if any(v != s for v in M[b]):
                raise AssertionError(f"half {h} wave {r} step {s}: factor buffer {b} holds {M[b]}")
            if any(v != s for v in Xo[h][b]):
                raise AssertionError(f"half {h} wave {r} step {s}: operand holds {Xo[h][b]}")
            readers_M[b].add((h, r))
            readers_X[h][b].add(r)
            yield None                                # the products take time
            readers_M[b].discard((h, r))
            readers_X[h][b].discard(r)
            P[h] += 1
            yield None
            nb = (s + 1) % 2
            if readers_X[h][nb]:
                raise AssertionError(f"half {h} wave {r} step {s}: operand {nb} overwritten while read")
            Xo[h][nb][r] = s + 1
            X[h] += 1
            yield None

    def expand_wave(e):
        for s in range(nsteps - 1):
            if peer_wait:
                yield lambda: E[0] >= NE * s and pcount(0) >= ptarget(s) and pcount(1) >= ptarget(s)
            else:
                yield lambda: pcount(0) >= ptarget(s) and pcount(1) >= ptarget(s)
            nb = (s + 1) % 2
            if readers_M[nb]:
                raise AssertionError(f"expansion {e} step {s}: factor buffer {nb} overwritten while read")
            M[nb][e] = s + 1
            yield None
            E[0] += 1
            yield None

    waves = [product_wave(h, r) for h in range(2) for r in range(RT)] + [expand_wave(e) for e in range(NE)]
    pending = [next(w, StopIteration) for w in waves]
    while True:
        ready = [i for i, c in enumerate(pending)
                 if c is not StopIteration and (c is None or c())]
        if not ready:
            if all(c is StopIteration for c in pending):
                return None
            return "deadlock"
        i = rng.choice(ready)
        try:
            pending[i] = next(waves[i], StopIteration)
        except AssertionError as err:
            return str(err)


@pytest.mark.parametrize("nsteps", [1, 2, 3, 7, 20])
def test_protocol_holds_under_random_schedules(nsteps):
    for seed in range(300):
        assert run(nsteps, seed) is None, (nsteps, seed, run(nsteps, seed))


def test_one_shared_product_counter_is_caught():
    msgs = [run(12, seed, shared_p=True) for seed in range(400)]
    assert any(m and "overwritten while read" in m for m in msgs), msgs[:3]


def test_expansion_waves_without_peer_wait_are_caught():
    msgs = [run(12, seed, peer_wait=False) for seed in range(400)]
    assert any(m and "factor buffer" in m for m in msgs), msgs[:3]

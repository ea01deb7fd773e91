"""Schedules of the GPU Jacobi eigensolvers, on the CPU.

linalg.hip pairs indices (the one-workgroup solver) and 16-index blocks
(the block solver) by a circle schedule, and the block solver's cross
rounds rotate, at step st, index k of block I with index (k + st) mod 16
of block J.  Restated here, these must give:
  - per round, a perfect matching of the mp indices (so a round's rotations
    commute and run in parallel);
  - over the mp - 1 rounds, every index pair exactly once;
  - over one block-solver sweep (the intra round, which pairs blocks 2P and
    2P + 1 and rotates every index pair inside them, then the circle rounds
    over all block pairs with their cross steps), every off-diagonal index
    pair of the matrix at least once, and twice only the pairs between
    blocks 2P and 2P + 1 that a circle round pairs again.
Test infrastructure; it shares nothing with the oracle or the library.
"""
import itertools

import pytest

KBJ = 16


def pair_of(k, r, mp):
    """Pair k of round r (0 <= r < mp - 1) of the circle schedule over mp
    (even) items: item 0 stays, the others rotate."""
    n1 = mp - 1
    if k == 0:
        return 0, 1 + r
    return 1 + (k + r) % n1, 1 + (r - k) % n1


@pytest.mark.parametrize("mp", [2, 4, 6, 16, 32, 48, 64])
def test_circle_schedule_is_a_round_robin(mp):
    seen = set()
    for r in range(mp - 1):
        pairs = [pair_of(k, r, mp) for k in range(mp // 2)]
        items = sorted(i for p in pairs for i in p)
        assert items == list(range(mp)), (r, pairs)
        for p, q in pairs:
            key = (min(p, q), max(p, q))
            assert key not in seen, (r, key)
            seen.add(key)
    assert len(seen) == mp * (mp - 1) // 2


def cross_steps():
    """Steps of a cross round: rotation k pairs index k of block I with
    index (k + st) mod KBJ of block J."""
    return [[(k, (k + st) % KBJ) for k in range(KBJ)] for st in range(KBJ)]


def test_cross_steps_cover_the_block_pair_once():
    seen = set()
    for step in cross_steps():
        assert sorted(i for i, _ in step) == list(range(KBJ))
        assert sorted(j for _, j in step) == list(range(KBJ))
        for pair in step:
            assert pair not in seen
            seen.add(pair)
    assert seen == set(itertools.product(range(KBJ), range(KBJ)))


@pytest.mark.parametrize("nblk", [2, 4, 8, 16, 48])
def test_block_sweep_rotates_every_pair_once(nblk):
    count = {}

    def hit(a, b):
        key = (min(a, b), max(a, b))
        count[key] = count.get(key, 0) + 1

    # intra round: blocks 2P and 2P + 1, every index pair of the 2 KBJ indices
    for p in range(nblk // 2):
        idx = list(range(2 * p * KBJ, (2 * p + 2) * KBJ))
        for a, b in itertools.combinations(idx, 2):
            hit(a, b)
    # circle rounds over all block pairs, each rotated across only
    for r in range(nblk - 1):
        for k in range(nblk // 2):
            bi, bj = pair_of(k, r, nblk)
            for step in cross_steps():
                for i, j in step:
                    hit(bi * KBJ + i, bj * KBJ + j)
    n = nblk * KBJ
    assert set(count) == {(a, b) for a in range(n) for b in range(a + 1, n)}
    twice = {key for key, c in count.items() if c > 1}
    assert max(count.values()) == 2 or not twice
    # only pairs across an intra pair of blocks (2P, 2P + 1)
    assert all(a // KBJ // 2 == b // KBJ // 2 and a // KBJ != b // KBJ for a, b in twice)
    # and those of every intra pair of blocks: the circle schedule pairs
    # each block with every other once
    assert len(twice) == (nblk // 2) * KBJ * KBJ

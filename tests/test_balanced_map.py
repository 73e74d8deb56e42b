"""The paper's balanced circular pair assignment, checked by enumeration.

Section 4 (algorithm "Proposed algorithm for calculating SPI"): object i
evaluates its partner (i + s) mod N for s = 1 .. (N-1)/2.  For even N (the
paragraph after Proposition 2) every object takes N/2 - 1 such steps and the
objects of the first half take one more, s = N/2.  Propositions 1 and 2 claim
that this evaluates every unordered pair exactly once.

These tests pin the reading of the even-N rule used throughout the library
(extra step s = N/2 for i < N/2) and show that the alternative reading of the
commented-out listing (j = N/2 + 1) is wrong.
"""
import itertools
import json
import os

import pytest


def row_steps(n: int, i: int) -> int:
    """Steps taken by object i: floor((N-1)/2), plus one for i < N/2 when N is even."""
    h = (n - 1) // 2
    return h + (1 if (n % 2 == 0 and i < n // 2) else 0)


def balanced_pairs(n: int):
    for i in range(n):
        for s in range(1, row_steps(n, i) + 1):
            yield i, (i + s) % n


def test_every_pair_exactly_once_small_n():
    for n in range(0, 400):
        seen = {}
        for i, j in balanced_pairs(n):
            key = (min(i, j), max(i, j))
            assert i != j
            seen[key] = seen.get(key, 0) + 1
        assert len(seen) == n * (n - 1) // 2, n
        assert all(v == 1 for v in seen.values()), n


@pytest.mark.parametrize("n", [511, 512, 1023, 1024, 4096, 4097])
def test_every_pair_exactly_once_larger_n(n):
    cnt = [[0] * n for _ in range(n)] if n <= 1024 else None
    if cnt is None:
        # count per unordered pair via a flat bytearray of the upper triangle
        flat = bytearray(n * n)
        for i, j in balanced_pairs(n):
            a, b = (i, j) if i < j else (j, i)
            flat[a * n + b] += 1
        total = sum(flat)
        assert total == n * (n - 1) // 2
        assert max(flat) == 1
        return
    for i, j in balanced_pairs(n):
        a, b = (i, j) if i < j else (j, i)
        cnt[a][b] += 1
    assert sum(map(sum, cnt)) == n * (n - 1) // 2
    assert all(cnt[a][b] == 1 for a, b in itertools.combinations(range(n), 2))


def test_work_per_row_and_depth():
    # Proposition 1 and the work/depth paragraph: depth (N-1)/2 for odd N and
    # N/2 for even N, total work N(N-1)/2.
    for n in range(2, 300):
        steps = [row_steps(n, i) for i in range(n)]
        assert sum(steps) == n * (n - 1) // 2
        assert max(steps) == ((n - 1) // 2 if n % 2 else n // 2)
        assert max(steps) - min(steps) <= 1


def test_proposition2_owner_rule_odd_n():
    # For odd N, i < j: i evaluates the pair iff j - i <= (N-1)/2, else j does.
    for n in range(1, 200, 2):
        owner = {}
        for i, j in balanced_pairs(n):
            owner[(min(i, j), max(i, j))] = i
        for i, j in itertools.combinations(range(n), 2):
            expect = i if (j - i) <= (n - 1) // 2 else j
            assert owner[(i, j)] == expect


def test_figure1_example(golden_dir):
    with open(os.path.join(golden_dir, "fig1_n5.json")) as f:
        g = json.load(f)
    n, b = g["N"], g["bead"]
    pairs = list(balanced_pairs(n))
    reaches = sorted(j for i, j in pairs if i == b)
    reached_by = sorted(i for i, j in pairs if j == b)
    assert reaches == g["reaches"]
    assert reached_by == g["reached_by"]
    # continuing one step past the stop would re-evaluate a pair: at s = 3, bead
    # 3 reaches bead 1 (= 3 + 3 mod 5) after bead 1 reached bead 3 at s = 2
    s = g["first_violation_step"]
    assert s == (n + 1) // 2
    i, j = g["violation_pair"]
    assert (i + s) % n == j
    assert (j, i) in pairs


def test_violation_step_formula():
    # Crossing at s = (N+1)/2 for odd N; meeting at s = N/2 for even N: taking
    # one more step for every object would duplicate a pair.
    for n in range(3, 200):
        h = (n - 1) // 2
        extra = h + 1
        dup = set()
        seen = set()
        for i in range(n):
            for s in range(1, extra + 1):
                p = (min(i, (i + s) % n), max(i, (i + s) % n))
                (dup if p in seen else seen).add(p)
        assert dup, n
        if n % 2:
            assert extra == (n + 1) // 2
        else:
            assert extra == n // 2


def test_commented_listing_reading_is_wrong():
    # The alternative reading (extra partner j = N/2 + 1 for i < N/2) misses pairs.
    n = 6
    seen = set()
    for i in range(n):
        for s in range(1, (n - 1) // 2 + 1):
            seen.add((min(i, (i + s) % n), max(i, (i + s) % n)))
        if i < n // 2:
            j = (i + n // 2 + 1) % n
            seen.add((min(i, j), max(i, j)))
    assert len(seen) == 12 < n * (n - 1) // 2

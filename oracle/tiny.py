"""Second, independent transcription of the phase loop in pure Python.

TEST INFRASTRUCTURE. Written separately from oracle.c (different data
structures: Python sets and dicts, no arrays of flags) so that a slip made
while transcribing the method into C shows up as a disagreement on small
inputs. It is far too slow for anything but n <= ~64.

It follows Section 2.2 of arXiv:2203.03732 with the same readings as the C
oracle: admissible means y(a) + y(b) = cbar(a, b) + eps; the greedy step is
synchronous proposal rounds in which each free b proposes to the first
admissible column, in its scan order, that was untaken when the round began,
and the lowest-index proposer wins; the completion pairs the i-th free b
with the i-th free a.
"""
from __future__ import annotations


def solve(k, T: int, origin: str = "diag"):
    """k: list of lists (rows = B). Returns (mate_b, y_a, y_b, phases, rounds)
    with the completion applied; y are the duals before the completion."""
    n = len(k)
    y_a = [0] * n
    y_b = [1] * n
    mate_of_b: dict[int, int] = {}
    mate_of_a: dict[int, int] = {}
    phases = rounds = 0

    def order(b):
        start = b if origin == "diag" else 0
        return [(start + j) % n for j in range(n)]

    while True:
        free_b = [b for b in range(n) if b not in mate_of_b]
        if len(free_b) <= T:
            break
        phases += 1
        taken: dict[int, int] = {}          # column -> b, the matching M'
        cursor = {b: 0 for b in free_b}      # next scan step of each b
        looking = set(free_b)
        while True:
            offers: dict[int, list[int]] = {}
            for b in sorted(looking):
                cols = order(b)
                hit = None
                for j in range(cursor[b], n):
                    a = cols[j]
                    if a not in taken and k[b][a] + 1 == y_a[a] + y_b[b]:
                        hit = j
                        break
                if hit is None:
                    looking.discard(b)
                else:
                    cursor[b] = hit
                    offers.setdefault(cols[hit], []).append(b)
            if not offers:
                break
            rounds += 1
            for a, bs in offers.items():
                w = min(bs)
                taken[a] = w
                looking.discard(w)
                for b in bs:
                    if b != w:
                        cursor[b] += 1
        matched_now = set(taken.values())
        for a, b in taken.items():
            old = mate_of_a.get(a)
            if old is not None:
                del mate_of_b[old]
            mate_of_a[a] = b
            mate_of_b[b] = a
            y_a[a] -= 1
        for b in free_b:
            if b not in matched_now:
                y_b[b] += 1

    free_b = [b for b in range(n) if b not in mate_of_b]
    free_a = [a for a in range(n) if a not in mate_of_a]
    for b, a in zip(free_b, free_a):
        mate_of_b[b] = a
        mate_of_a[a] = b
    mate_b = [mate_of_b.get(b, -1) for b in range(n)]
    return mate_b, y_a, y_b, phases, rounds


def solve_copies(kp, s, d, T: int, origin: str = "diag"):
    """Section 4 on small inputs: supply point p becomes s[p] unit copies and
    demand point q d[q] copies (in point order); a copy's rounded cost is its
    points' kp[p][q]. Phases as in `solve` on the copies, and after each
    phase every free supply copy takes the largest dual among its point's
    copies. Returns (mate_b, y_a, y_b, phases, rounds) at copy level, with the
    completion applied and the duals from before it."""
    owner_b = [p for p, c in enumerate(s) for _ in range(c)]
    owner_a = [q for q, c in enumerate(d) for _ in range(c)]
    nb, na = len(owner_b), len(owner_a)
    y_a = [0] * na
    y_b = [1] * nb
    mate_of_b: dict[int, int] = {}
    mate_of_a: dict[int, int] = {}
    phases = rounds = 0

    def cost(b, a):
        return kp[owner_b[b]][owner_a[a]]

    def column(b, j):
        return (b + j) % na if origin == "diag" else j

    while True:
        free_b = [b for b in range(nb) if b not in mate_of_b]
        if len(free_b) <= T:
            break
        phases += 1
        taken: dict[int, int] = {}
        cursor = {b: 0 for b in free_b}
        looking = set(free_b)
        while True:
            offers: dict[int, list[int]] = {}
            for b in sorted(looking):
                hit = None
                for j in range(cursor[b], na):
                    a = column(b, j)
                    if a not in taken and cost(b, a) + 1 == y_a[a] + y_b[b]:
                        hit = j
                        break
                if hit is None:
                    looking.discard(b)
                else:
                    cursor[b] = hit
                    offers.setdefault(column(b, hit), []).append(b)
            if not offers:
                break
            rounds += 1
            for a, bs in offers.items():
                w = min(bs)
                taken[a] = w
                looking.discard(w)
                for b in bs:
                    if b != w:
                        cursor[b] += 1
        for a, b in taken.items():
            old = mate_of_a.get(a)
            if old is not None:
                del mate_of_b[old]
            mate_of_a[a] = b
            mate_of_b[b] = a
            y_a[a] -= 1
        winners = set(taken.values())
        for b in free_b:
            if b not in winners:
                y_b[b] += 1
        top: dict[int, int] = {}
        for b in range(nb):
            top[owner_b[b]] = max(top.get(owner_b[b], y_b[b]), y_b[b])
        for b in range(nb):
            if b not in mate_of_b:
                y_b[b] = top[owner_b[b]]

    free_b = [b for b in range(nb) if b not in mate_of_b]
    free_a = [a for a in range(na) if a not in mate_of_a]
    for b, a in zip(free_b, free_a):
        mate_of_b[b] = a
        mate_of_a[a] = b
    mate_b = [mate_of_b.get(b, -1) for b in range(nb)]
    return mate_b, y_a, y_b, phases, rounds

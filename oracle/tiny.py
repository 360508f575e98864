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


def solve_point_rounds_on_copies(kp, s, d, T: int, origin: str = "diag"):
    """Section 4 with the point-level reading of step (I) (the one the
    clustered oracle takes), run on explicit copies: every copy has its own
    dual and mate, and nothing assumes Lemma 4.1. In a phase, each supply
    point b with free copies (which the raise keeps at one dual) proposes, in
    synchronous rounds, to the first point a in its scan order (DIAG: from
    column b mod n_a) that has an untaken copy c with y(c) + y(b) = k + 1,
    for all its looking copies; proposals are served in ascending b, each
    with as many such copies as are left, taken free copies first, then
    matched ones by ascending partner point (then copy index). Then the old
    partners become free, taken copies drop one step, free copies left
    unmatched rise one step, and free copies take their point's largest dual.

    Returns (snapshots, flow, phases, rounds): snapshots[t] = the point-level
    state after phase t + 1 as (Y, F, Z, G, w) with w[b][a][p] = pairs whose
    demand copy's dual has parity p; flow = pairs per point pair after the
    completion (free supply copies in copy order take free demand copies in
    copy order)."""
    n_b, n_a = len(s), len(d)
    owner_b = [p for p, c in enumerate(s) for _ in range(c)]
    owner_a = [q for q, c in enumerate(d) for _ in range(c)]
    copies_of_b = [[x for x in range(len(owner_b)) if owner_b[x] == p] for p in range(n_b)]
    copies_of_a = [[c for c in range(len(owner_a)) if owner_a[c] == q] for q in range(n_a)]
    yb = [1] * len(owner_b)
    ya = [0] * len(owner_a)
    mb: dict[int, int] = {}
    ma: dict[int, int] = {}
    phases = rounds = 0
    snapshots = []

    def point_state():
        Y = [max(yb[x] for x in copies_of_b[p]) if copies_of_b[p] else 1 for p in range(n_b)]
        F = [sum(1 for x in copies_of_b[p] if x not in mb) for p in range(n_b)]
        Z = [max(ya[c] for c in copies_of_a[q]) if copies_of_a[q] else 0 for q in range(n_a)]
        G = [sum(1 for c in copies_of_a[q] if c not in ma) for q in range(n_a)]
        w = [[[0, 0] for _ in range(n_a)] for _ in range(n_b)]
        for c, x in ma.items():
            w[owner_b[x]][owner_a[c]][ya[c] & 1] += 1
        return Y, F, Z, G, w

    while True:
        free = [x for x in range(len(owner_b)) if x not in mb]
        if len(free) <= T:
            break
        phases += 1
        looking = {p: [x for x in copies_of_b[p] if x not in mb] for p in range(n_b)}
        ylev = {}
        for p, xs in looking.items():
            if xs:
                assert len({yb[x] for x in xs}) == 1, "free copies of a point at two duals"
                ylev[p] = yb[xs[0]]
        active = {p for p, xs in looking.items() if xs}
        cursor = {p: 0 for p in active}
        taken: dict[int, int] = {}  # demand copy -> new partner copy

        def col(p, j):
            return (p % n_a + j) % n_a if origin == "diag" else j

        def open_copies(p, q):
            return [c for c in copies_of_a[q]
                    if c not in taken and ya[c] + ylev[p] == kp[p][q] + 1]

        while True:
            offers = {}
            for p in sorted(active):
                hit = None
                for j in range(cursor[p], n_a):
                    if open_copies(p, col(p, j)):
                        hit = j
                        break
                if hit is None:
                    active.discard(p)
                else:
                    cursor[p] = hit
                    offers[p] = col(p, hit)
            if not offers:
                break
            rounds += 1
            for p in sorted(offers):
                q = offers[p]
                cs = open_copies(p, q)
                cs.sort(key=lambda c: (c in ma, owner_b[ma[c]] if c in ma else -1, c))
                for c in cs[:len(looking[p])]:
                    taken[c] = looking[p].pop(0)
                if looking[p]:
                    cursor[p] += 1
                else:
                    active.discard(p)
        for c, x in taken.items():
            old = ma.get(c)
            if old is not None:
                del mb[old]
            ma[c] = x
            mb[x] = c
            ya[c] -= 1
        for x in free:
            if x not in mb:
                yb[x] += 1
        for p in range(n_b):
            if copies_of_b[p]:
                top = max(yb[x] for x in copies_of_b[p])
                for x in copies_of_b[p]:
                    if x not in mb:
                        yb[x] = top
        snapshots.append(point_state())

    flow = [[0] * n_a for _ in range(n_b)]
    for c, x in ma.items():
        flow[owner_b[x]][owner_a[c]] += 1
    free_b = [x for x in range(len(owner_b)) if x not in mb]
    free_a = [c for c in range(len(owner_a)) if c not in ma]
    for x, c in zip(free_b, free_a):
        flow[owner_b[x]][owner_a[c]] += 1
    return snapshots, flow, phases, rounds

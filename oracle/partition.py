"""Multigrid level hierarchies of a locally refined mesh and their parallel
efficiency metrics (oracle; test infrastructure only), Sec. 2 (global
coarsening vs local smoothing; the parallel workload efficiency eta_w and the
vertical communication efficiency eta_v of Tables tab:tc and tab:fpc).

The paper names the metrics and refers to earlier work for their definition.
Readings:
* Cells are (level l, index (i, j, m)) on the (n 2^l)^3 grid of level l;
  the parent of (l, i, j, m) is (l - 1, i // 2, j // 2, m // 2).  Cells are
  ordered along the Morton (z-order) curve of the finest level.
* Partition of P processes: every set of cells that is partitioned on its
  own (the leaves; every global-coarsening level) is cut into P contiguous
  Morton-ordered chunks whose sizes differ by at most one, the first
  (count mod P) chunks one cell larger.
* Global coarsening (GC): level 0 is the leaves; level j + 1 replaces every
  complete family of eight sibling leaves of level j by their parent (the
  library's coarsening); the last level is the uniform base mesh.  Each
  level is partitioned on its own.
* Local smoothing (LS): level l holds every cell of refinement level l of
  the tree (leaves and parents of finer cells), l = 0 .. L.  A leaf keeps
  its owner from the leaf partition; a parent belongs to the owner of its
  first child in Morton order.
* eta_w = sum_l n_l / (P sum_l max_p n_{l,p}): the work of all levels
  against the time of the busiest process on each level.
* eta_v: over all transfers between consecutive levels, the fraction of
  fine cells that have the same owner as the coarse cell they map to (its
  parent, or the cell itself when it is not coarsened).
"""
from __future__ import annotations


def _interleave(i, j, m, bits):
    key = 0
    for b in range(bits):
        key |= ((i >> b) & 1) << (3 * b)
        key |= ((j >> b) & 1) << (3 * b + 1)
        key |= ((m >> b) & 1) << (3 * b + 2)
    return key


def morton(cell, L, n):
    """Morton key of a cell on the finest grid (its lowest corner), level
    first as a tie-breaker so that parents precede their children."""
    lev, i, j, m = cell
    s = L - lev
    bits = max(1, (n << L).bit_length())
    return (_interleave(i << s, j << s, m << s, bits), lev)


def parent(cell):
    lev, i, j, m = cell
    return (lev - 1, i // 2, j // 2, m // 2)


def partition(cells, P, L, n):
    """{cell: owner} by P contiguous Morton chunks."""
    order = sorted(cells, key=lambda c: morton(c, L, n))
    N = len(order)
    base, extra = divmod(N, P)
    owner = {}
    k = 0
    for p in range(P):
        size = base + (1 if p < extra else 0)
        for c in order[k:k + size]:
            owner[c] = p
        k += size
    return owner


def leaves(mesh):
    return [(int(lv), int(a), int(b), int(c)) for lv, (a, b, c) in zip(mesh["level"], mesh["idx"])]


def gc_levels(mesh):
    """Leaf sets, finest first, down to the uniform base mesh."""
    cur = set(leaves(mesh))
    out = [cur]
    while max(c[0] for c in cur) > 0:
        fam = {}
        for c in cur:
            if c[0] > 0:
                fam.setdefault(parent(c), []).append(c)
        nxt = set(cur)
        for par, kids in fam.items():
            if len(kids) == 8:
                for k in kids:
                    nxt.discard(k)
                nxt.add(par)
        if nxt == cur:
            raise ValueError("no complete family to coarsen")
        cur = nxt
        out.append(cur)
    return out


def ls_levels(mesh):
    """Cells of refinement level l of the tree, l = 0 .. L."""
    L = int(mesh["levels"])
    per = [set() for _ in range(L + 1)]
    for c in leaves(mesh):
        per[c[0]].add(c)
        p = c
        while p[0] > 0:
            p = parent(p)
            per[p[0]].add(p)
    return per


def _eta_w(levels, owners, P):
    total = sum(len(lv) for lv in levels)
    crit = 0
    for lv, own in zip(levels, owners):
        counts = [0] * P
        for c in lv:
            counts[own[c]] += 1
        crit += max(counts)
    return total / (P * crit)


def metrics(mesh, P):
    """{"gc": {"eta_w", "eta_v"}, "ls": {...}} for P processes."""
    n, L = int(mesh["n"]), int(mesh["levels"])
    leaf_owner = partition(leaves(mesh), P, L, n)
    # global coarsening
    G = gc_levels(mesh)
    gown = [leaf_owner] + [partition(lv, P, L, n) for lv in G[1:]]
    local = tot = 0
    for j in range(len(G) - 1):
        for c in G[j]:
            target = c if c in G[j + 1] else parent(c)
            tot += 1
            local += gown[j][c] == gown[j + 1][target]
    gc = {"eta_w": _eta_w(G, gown, P), "eta_v": local / tot if tot else 1.0}
    # local smoothing
    S = ls_levels(mesh)
    lown = [dict() for _ in S]
    for lev in range(L, -1, -1):
        for c in S[lev]:
            if c in leaf_owner:
                lown[lev][c] = leaf_owner[c]
        if lev < L:
            kids = {}
            for c in S[lev + 1]:
                kids.setdefault(parent(c), []).append(c)
            for par, ks in kids.items():
                if par not in leaf_owner:
                    first = min(ks, key=lambda c: morton(c, L, n))
                    lown[lev][par] = lown[lev + 1][first]
    local = tot = 0
    for lev in range(L, 0, -1):
        for c in S[lev]:
            tot += 1
            local += lown[lev][c] == lown[lev - 1][parent(c)]
    ls = {"eta_w": _eta_w(S, lown, P), "eta_v": local / tot if tot else 1.0}
    return {"gc": gc, "ls": ls}

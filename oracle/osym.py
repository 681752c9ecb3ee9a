"""O-sym: naive symbolic analysis for the CPU oracle.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything under
``oracle/``. The product path never does, and shares no code with it.

Everything here is written from the definitions in the paper, with plain
Python sets and lists, and recomputes structures from scratch after every
reordering instead of relabelling them:

* column structure glbind(j) = {j} u struct(A_{j+1:n,j}) u the structures of
  the etree children of j minus those children (Section 2.1.2; this is the set
  that makes the containment of eq. (1) hold);
* etree parent p(j) = min(glbind(j) \\ {j}) (Section 2.1.2);
* fundamental supernodes: j and p(j) share a supernode iff
  glbind(j) \\ {j} = glbind(p(j)) and j is p(j)'s only child (Section 2.1.2);
* supernode merging: repeatedly merge the child/parent pair that creates the
  least new fill, stopping before cumulative storage growth exceeds the cap
  (12.5 percent) (Section 3.1);
* within-supernode reordering by partition refinement (Section 1, Fig. 2;
  Section 3.1) -- the paper only cites the algorithm, so the rule below is a
  reading of it (documented in the design notes) that reproduces Fig. 2;
* relind(J, P): each row of J replaced by its distance from the bottom of
  glbind(P) (Section 2.1.2); blocks and relindB (Section 2.2.2, Alg. 5).

Readings where the paper is silent (all mirrored by the product's analysis):
  - ordering: geometric nested dissection on the grid box: if no axis extent
    exceeds 2 emit the nodes lexicographically (x fastest, dofs innermost),
    else cut the longest axis (ties x<y<z) at lo + extent//2 and emit low box,
    high box, then the cut plane lexicographically;
  - postorder: children visited in ascending index, roots in ascending index;
  - merge candidates: (J, p(J)) with last(J) + 1 == first(p(J)); cost
    w_J * (w_J + m_P - m_J); smallest (cost, first(J)) first; stop (not skip)
    at the first merge that would make added/nnz(L_fundamental) > cap;
  - blocks: maximal runs of consecutive global rows below the diagonal block,
    split at supernode boundaries; relindB(J, P) lists the relind of the top
    row of every block of J lying in P or in an ancestor of P.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# orderings


def graph_nested_dissection(n, colptr, rowidx, leaf=8, trace=None):
    """Nested dissection of the adjacency graph of a lower-CSC pattern
    (general sparse input): each vertex set is split into its connected
    components (in the order of their smallest vertex); a component of at
    most `leaf` vertices is emitted ascending; otherwise breadth-first levels
    are grown from a pseudo-peripheral root (start at the component's
    smallest vertex, then move to the least-degree vertex of the last level,
    smallest index on ties, while that gives strictly more levels, at most 8
    moves), each level in ascending order; the separator is the first level m
    with 1 <= m <= depth-1 whose cumulative count reaches half the component
    (else depth-1); the vertices before the separator, then those after it,
    are dissected the same way, and the separator follows, ascending. A
    component with fewer than three levels is emitted ascending.
    When `trace` is a list, every split is appended as (before, after,
    separator) vertex lists. Returns perm[new] = old."""
    adj = [set() for _ in range(n)]
    for j in range(n):
        for e in range(colptr[j], colptr[j + 1]):
            i = int(rowidx[e])
            if i != j:
                adj[i].add(j)
                adj[j].add(i)
    out = []

    def bfs_levels(root, allowed):
        seen = {root}
        levels = [[root]]
        while True:
            nxt = sorted({u for v in levels[-1] for u in adj[v] if u in allowed and u not in seen})
            if not nxt:
                return levels
            seen.update(nxt)
            levels.append(nxt)

    def do_set(vs):
        remaining = set(vs)
        while remaining:
            v = min(remaining)
            comp = set(x for lev in bfs_levels(v, remaining) for x in lev)
            remaining -= comp
            do_component(sorted(comp))

    def do_component(comp):
        if len(comp) <= leaf:
            out.extend(comp)
            return
        cset = set(comp)
        levels = bfs_levels(comp[0], cset)
        for _ in range(8):
            last = levels[-1]
            deg = [len(adj[w] & cset) for w in last]
            u = last[deg.index(min(deg))]
            lu = bfs_levels(u, cset)
            if len(lu) <= len(levels):
                break
            levels = lu
        depth = len(levels) - 1
        if depth < 2:
            out.extend(comp)
            return
        m, cum = depth - 1, 0
        for i in range(depth):
            cum += len(levels[i])
            if i >= 1 and 2 * cum >= len(comp):
                m = i
                break
        before = sorted(x for lev in levels[:m] for x in lev)
        after = sorted(x for lev in levels[m + 1:] for x in lev)
        if trace is not None:
            trace.append((before, after, list(levels[m])))
        do_set(before)
        do_set(after)
        out.extend(levels[m])

    do_set(range(n))
    return np.array(out, np.int64)


def nested_dissection(nx, ny, nz, dofs=1):
    """Geometric nested dissection of an nx*ny*nz grid; returns perm[new] = old."""
    out = []

    def emit(x0, x1, y0, y1, z0, z1):
        for z in range(z0, z1):
            for y in range(y0, y1):
                for x in range(x0, x1):
                    node = x + nx * (y + ny * z)
                    for d in range(dofs):
                        out.append(node * dofs + d)

    def rec(x0, x1, y0, y1, z0, z1):
        ex, ey, ez = x1 - x0, y1 - y0, z1 - z0
        if ex <= 0 or ey <= 0 or ez <= 0:
            return
        big = max(ex, ey, ez)
        if big <= 2:
            emit(x0, x1, y0, y1, z0, z1)
            return
        if ex == big:
            m = x0 + ex // 2
            rec(x0, m, y0, y1, z0, z1)
            rec(m + 1, x1, y0, y1, z0, z1)
            emit(m, m + 1, y0, y1, z0, z1)
        elif ey == big:
            m = y0 + ey // 2
            rec(x0, x1, y0, m, z0, z1)
            rec(x0, x1, m + 1, y1, z0, z1)
            emit(x0, x1, m, m + 1, z0, z1)
        else:
            m = z0 + ez // 2
            rec(x0, x1, y0, y1, z0, m)
            rec(x0, x1, y0, y1, m + 1, z1)
            emit(x0, x1, y0, y1, m, m + 1)

    rec(0, nx, 0, ny, 0, nz)
    return np.array(out, dtype=np.int64)


def permute_lower(n, colptr, rowidx, values, perm):
    """Lower CSC of P A P^T where perm[new] = old (rows ascending per column)."""
    inv = np.empty(n, np.int64)
    inv[np.asarray(perm)] = np.arange(n)
    cols = np.repeat(np.arange(n, dtype=np.int64), np.diff(colptr))
    r = inv[np.asarray(rowidx)]
    c = inv[cols]
    lo = np.minimum(r, c)
    hi = np.maximum(r, c)
    order = np.lexsort((hi, lo))
    hi = hi[order]
    lo = lo[order]
    v = None if values is None else np.asarray(values)[order]
    cp = np.zeros(n + 1, np.int64)
    np.add.at(cp, lo + 1, 1)
    return np.cumsum(cp), hi, v


# ---------------------------------------------------------------------------
# column structures and the elimination tree


def column_structures(n, colptr, rowidx, upto=None):
    """glbind(j) for j < upto (default n) by the set recurrence, and p(j).

    Returns (structs, parent): structs[j] is a sorted int64 array,
    parent[j] = -1 for a root (and for j >= upto, which is not computed).
    """
    upto = n if upto is None else upto
    kids = [[] for _ in range(n)]
    structs = [None] * upto
    parent = np.full(n, -1, np.int64)
    for j in range(upto):
        s = set(int(i) for i in rowidx[colptr[j]:colptr[j + 1]])
        s.add(j)
        for c in kids[j]:
            s.update(int(i) for i in structs[c])
            s.discard(c)
        arr = np.array(sorted(s), dtype=np.int64)
        assert arr[0] == j
        structs[j] = arr
        if arr.size > 1:
            p = int(arr[1])  # min(glbind(j) \ {j})
            parent[j] = p
            kids[p].append(j)
    return structs, parent


def postorder(parent):
    """post[k] = the k-th vertex of a postorder (children ascending, roots ascending)."""
    n = len(parent)
    kids = [[] for _ in range(n)]
    roots = []
    for j in range(n):
        if parent[j] < 0:
            roots.append(j)
        else:
            kids[parent[j]].append(j)
    out = []
    for r in roots:
        stack = [(r, 0)]
        while stack:
            v, k = stack.pop()
            if k < len(kids[v]):
                stack.append((v, k + 1))
                stack.append((kids[v][k], 0))
            else:
                out.append(v)
    return np.array(out, dtype=np.int64)


def fundamental_supernodes(structs, parent):
    """First-column pointers of the fundamental supernode partition."""
    n = len(structs)
    nkids = np.zeros(n, np.int64)
    for j in range(n):
        if parent[j] >= 0:
            nkids[parent[j]] += 1
    ptr = [0]
    for j in range(n - 1):
        p = parent[j]
        same = (p == j + 1 and nkids[p] == 1
                and np.array_equal(structs[j][1:], structs[p]))
        if not same:
            ptr.append(j + 1)
    ptr.append(n)
    return np.array(ptr, dtype=np.int64)


def supernode_of(sn_ptr, n):
    snode = np.empty(n, np.int64)
    for J in range(len(sn_ptr) - 1):
        snode[sn_ptr[J]:sn_ptr[J + 1]] = J
    return snode


def supernodal_parent(sn_ptr, glb):
    """p(J) = supernode holding the first row of glbind(J) below the last column."""
    S = len(sn_ptr) - 1
    n = int(sn_ptr[-1])
    snode = supernode_of(sn_ptr, n)
    par = np.full(S, -1, np.int64)
    for J in range(S):
        last = sn_ptr[J + 1] - 1
        below = glb[J][glb[J] > last]
        if below.size:
            par[J] = snode[below[0]]
    return par


# ---------------------------------------------------------------------------
# supernode merging (Section 3.1)


def merge_supernodes(fund_ptr, structs, cap=0.125, trace=None):
    """Greedy child/parent merging with a cumulative storage-growth cap.

    Returns (sn_ptr, glbind per merged supernode, added entries, base entries).
    When `trace` is a list, every decision is appended to it, in order:
    ("merge", first column of the child, first column of the parent, cost),
    then ("stop", first column of the child, cost) for the merge that would
    pass the cap, or ("exhausted",) when no candidate is left.
    """
    S = len(fund_ptr) - 1
    first = np.array(fund_ptr[:-1], np.int64)
    last = np.array(fund_ptr[1:], np.int64) - 1
    width = last - first + 1
    glb = [structs[int(f)] for f in first]
    m = np.array([g.size for g in glb], np.int64)
    par = supernodal_parent(np.array(fund_ptr), glb)
    base = int(sum(int(m[J]) * int(width[J]) - int(width[J]) * (int(width[J]) - 1) // 2
                   for J in range(S)))
    alive = np.ones(S, bool)
    top = np.arange(S)  # the highest fundamental supernode of a merged chain
    INF = np.iinfo(np.int64).max
    key = np.full(S, INF, np.int64)
    SHIFT = 1 << 24

    def refresh(J):
        P = par[J]
        if alive[J] and P >= 0 and last[J] + 1 == first[P]:
            cost = int(width[J]) * (int(width[J]) + int(m[P]) - int(m[J]))
            key[J] = cost * SHIFT + int(first[J])
        else:
            key[J] = INF

    for J in range(S):
        refresh(J)
    added = 0
    while True:
        J = int(np.argmin(key))
        if key[J] == INF:
            if trace is not None:
                trace.append(("exhausted",))
            break
        cost = int(key[J]) // SHIFT
        if float(added + cost) > cap * float(base):
            if trace is not None:
                trace.append(("stop", int(first[J]), cost))
            break
        P = int(par[J])
        if trace is not None:
            trace.append(("merge", int(first[J]), int(first[P]), cost))
        added += cost
        # J absorbs P: the merged supernode keeps J's slot
        last[J] = last[P]
        width[J] = last[J] - first[J] + 1
        m[J] = int(width[J] - (last[P] - first[P] + 1)) + int(m[P])
        top[J] = top[P]
        alive[P] = False
        key[P] = INF
        par[J] = par[P]
        kids = np.nonzero(alive & (par == P))[0]
        par[kids] = J
        for C in np.nonzero(alive & (par == J))[0]:
            refresh(int(C))
        refresh(J)
    ids = np.nonzero(alive)[0]
    sn_ptr = np.append(first[ids], int(fund_ptr[-1])).astype(np.int64)
    glbm = []
    for J in ids:
        t = top[J]
        g = np.concatenate([np.arange(first[J], first[t], dtype=np.int64), glb[t]])
        assert g.size == m[J]
        glbm.append(g)
    return sn_ptr, glbm, added, base


# ---------------------------------------------------------------------------
# partition refinement inside supernodes (Section 1, Fig. 2; Section 3.1)


def _runs(positions):
    if len(positions) == 0:
        return 0
    p = sorted(positions)
    return 1 + sum(1 for a, b in zip(p, p[1:]) if b != a + 1)


def refine_order(cols, row_sets):
    """Reorder the columns `cols` of one supernode.

    row_sets: for every descendant J touching the supernode, in ascending J,
    the set R_J of its columns among J's rows. Each R_J stably splits every
    current part S into S&R and S-R; S&R goes after S-R when the following
    part meets R, else before. The refined order is kept only if it lowers
    the total number of runs of the R_J.
    """
    parts = [list(cols)]
    for R in row_sets:
        new = []
        for k, S in enumerate(parts):
            inR = [c for c in S if c in R]
            out = [c for c in S if c not in R]
            if not inR or not out:
                new.append(S)
                continue
            nxt = parts[k + 1] if k + 1 < len(parts) else []
            if any(c in R for c in nxt):
                new.extend([out, inR])
            else:
                new.extend([inR, out])
        parts = new
    order = [c for S in parts for c in S]

    def total_runs(seq):
        pos = {c: i for i, c in enumerate(seq)}
        return sum(_runs([pos[c] for c in R]) for R in row_sets)

    if total_runs(order) < total_runs(list(cols)):
        return order
    return list(cols)


def partition_refinement(sn_ptr, glb):
    """New-to-old permutation that reorders columns within every supernode."""
    S = len(sn_ptr) - 1
    n = int(sn_ptr[-1])
    snode = supernode_of(sn_ptr, n)
    touching = [[] for _ in range(S)]  # (J, R_J) in ascending J
    for J in range(S):
        last = sn_ptr[J + 1] - 1
        rows = glb[J][glb[J] > last]
        groups = {}
        for i in rows:
            groups.setdefault(int(snode[i]), set()).add(int(i))
        for P in sorted(groups):
            touching[P].append(groups[P])
    perm = np.arange(n, dtype=np.int64)
    for P in range(S):
        cols = list(range(sn_ptr[P], sn_ptr[P + 1]))
        order = refine_order(cols, touching[P])
        perm[sn_ptr[P]:sn_ptr[P + 1]] = order
    return perm


# ---------------------------------------------------------------------------
# relative indices and blocks (Sections 2.1.2 and 2.2.2)


def relind(rows, glb_P):
    """Distance of every row in `rows` from the bottom of glbind(P)."""
    pos = {int(i): k for k, i in enumerate(glb_P)}
    mP = len(glb_P)
    return np.array([mP - 1 - pos[int(i)] for i in rows], dtype=np.int64)


def blocks_of(rows, snode):
    """Sizes of the blocks: maximal runs of consecutive rows, split at supernodes."""
    sizes = []
    prev = None
    for i in rows:
        i = int(i)
        if prev is not None and i == prev + 1 and snode[i] == snode[prev]:
            sizes[-1] += 1
        else:
            sizes.append(1)
        prev = i
    return sizes


def supernodal_maps(sn_ptr, glb, par):
    """relind(J,p(J)), block sizes and relindB(J,P) for every ancestor P touched."""
    S = len(sn_ptr) - 1
    n = int(sn_ptr[-1])
    snode = supernode_of(sn_ptr, n)
    rel, blks, rb = [], [], []
    for J in range(S):
        last = sn_ptr[J + 1] - 1
        rows = glb[J][glb[J] > last]
        P = par[J]
        rel.append(relind(rows, glb[P]) if P >= 0 else np.zeros(0, np.int64))
        sizes = blocks_of(rows, snode)
        blks.append(np.array(sizes, np.int64))
        tops = []
        k = 0
        for b in sizes:
            tops.append(int(rows[k]))
            k += b
        pairs = []
        A = P
        while A >= 0:
            live = [t for t in tops if t >= sn_ptr[A]]
            if any(snode[t] == A for t in live):
                pairs.append((int(A), relind(live, glb[A])))
            A = par[A]
        rb.append(pairs)
    return rel, blks, rb


# ---------------------------------------------------------------------------
# the whole analysis


def analyze(A, ordering="grid", merge_cap=0.125, reorder=True, user_perm=None):
    """Naive symbolic analysis. A is a lower-CSC SparseSPD-like object.

    Returns a dict with the final permutation, the supernode partition and
    every index map; the exact column structures of the final ordering are
    returned as 'structs' (list of sorted arrays) with the etree 'parent'.
    """
    n = A.n
    if ordering == "grid":
        nx, ny, nz, d = A.grid
        perm0 = nested_dissection(nx, ny, nz, d)
    elif ordering == "natural":
        perm0 = np.arange(n, dtype=np.int64)
    elif ordering == "graph":
        perm0 = graph_nested_dissection(n, A.colptr, A.rowidx)
    elif ordering == "user":
        perm0 = np.asarray(user_perm, np.int64)
    else:
        raise ValueError(ordering)
    assert np.array_equal(np.sort(perm0), np.arange(n))

    # etree of the ordered matrix, then a postorder renumbering
    cp, ri, _ = permute_lower(n, A.colptr, A.rowidx, None, perm0)
    structs, parent = column_structures(n, cp, ri)
    post = postorder(parent)
    perm1 = perm0[post]

    # structures again under the postorder; fundamental supernodes; merging
    cp, ri, _ = permute_lower(n, A.colptr, A.rowidx, None, perm1)
    structs, parent_post = column_structures(n, cp, ri)
    fund_ptr = fundamental_supernodes(structs, parent_post)
    if merge_cap > 0:
        sn_ptr, glbm, added, base = merge_supernodes(fund_ptr, structs, merge_cap)
    else:
        sn_ptr = fund_ptr
        glbm = [structs[int(f)] for f in fund_ptr[:-1]]
        added = 0
        base = sum(len(s) for s in structs)

    # partition refinement inside the merged supernodes
    if reorder:
        pr = partition_refinement(sn_ptr, glbm)
    else:
        pr = np.arange(n, dtype=np.int64)
    perm = perm1[pr]
    inv_pr = np.empty(n, np.int64)
    inv_pr[pr] = np.arange(n)
    glb = [np.sort(inv_pr[g]) for g in glbm]

    # exact structure of the final ordering, from scratch
    cp, ri, _ = permute_lower(n, A.colptr, A.rowidx, None, perm)
    structs, parent = column_structures(n, cp, ri)
    par = supernodal_parent(sn_ptr, glb)
    rel, blks, rb = supernodal_maps(sn_ptr, glb, par)
    return {
        "n": n,
        "perm": perm,
        "perm_nd": perm0,
        "perm_post": perm1,
        "parent_post": parent_post,
        "fund_ptr": fund_ptr,
        "sn_ptr": sn_ptr,
        "sn_parent": par,
        "glbind": glb,
        "relind": rel,
        "blocks": blks,
        "relindB": rb,
        "structs": structs,
        "parent": parent,
        "merge_added": added,
        "merge_base": base,
    }


def exact_nnz(structs):
    return int(sum(len(s) for s in structs))


def exact_flops(structs):
    """Factorization flop count: sum over columns of (column count)^2."""
    return int(sum(len(s) ** 2 for s in structs))

"""Independent checks used to pin the oracle (tests only).

Nothing here is shared with the oracle's C code or the GPU library: each function restates
a definition directly so that a mistake in either implementation shows up as a mismatch.

* ``spec_priority``   numpy restatement of the priority specification.
* ``brute_all``       LocalContraction on every labelled graph of n <= 7 vertices at once,
                      with node neighbourhoods as bitmasks: closed one-hop set N(x) = adj | x,
                      two-hop set N(N(x)) = union of N(y) over y in N(x), label = argmin of the
                      priority over that set (Section 3, "LocalContraction"; Section 2 for N).
* ``two_hop_parents`` the same definition at scale with sparse (A + I)^2 reachability.
* ``union_find``      textbook union-find with path halving and union by size.
* ``canon``           canonical form of a partition (smallest member id per vertex).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

M64 = (1 << 64) - 1


def _sm64_int(x: int) -> int:
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _fmix32_np(h: np.ndarray) -> np.ndarray:
    h = h.astype(np.uint32, copy=True)
    h ^= h >> np.uint32(16)
    h *= np.uint32(0x85EBCA6B)
    h ^= h >> np.uint32(13)
    h *= np.uint32(0xC2B2AE35)
    h ^= h >> np.uint32(16)
    return h


def round_key(seed: int, rnd: int):
    k = _sm64_int((seed & M64) ^ _sm64_int(rnd & 0xFFFFFFFF))
    return np.uint32(k & 0xFFFFFFFF), np.uint32(k >> 32)


def spec_priority(seed: int, rnd: int, names) -> np.ndarray:
    """Priority of node `name` in phase `rnd`: fmix32(fmix32(name ^ k0) ^ k1)."""
    k0, k1 = round_key(seed, rnd)
    x = np.asarray(names, dtype=np.uint32)
    with np.errstate(over="ignore"):
        return _fmix32_np(_fmix32_np(x ^ k0) ^ k1)


def _inv_odd(a: int) -> int:
    x = a
    for _ in range(5):
        x = (x * (2 - a * x)) & 0xFFFFFFFF
    return x


def _unxorshift(h: np.ndarray, s: int) -> np.ndarray:
    out = h.copy()
    t = s
    while t < 32:
        out = h ^ (out >> np.uint32(s))
        t += s
    return out


def spec_priority_inverse(seed: int, rnd: int, prio) -> np.ndarray:
    """Inverse of spec_priority (each step of fmix32 undone in reverse order)."""
    k0, k1 = round_key(seed, rnd)

    def unfmix(h):
        h = _unxorshift(h, 16)
        h = h * np.uint32(_inv_odd(0xC2B2AE35))
        h = _unxorshift(h, 13)
        h = h * np.uint32(_inv_odd(0x85EBCA6B))
        return _unxorshift(h, 16)

    with np.errstate(over="ignore"):
        h = np.asarray(prio, dtype=np.uint32).copy()
        return unfmix(unfmix(h) ^ k1) ^ k0


# --------------------------------------------------------------------------------------
# brute force over all labelled graphs on n <= 7 vertices
# --------------------------------------------------------------------------------------

def all_graph_adjacency(n: int) -> np.ndarray:
    """Adjacency bitmasks [2^C(n,2), n] of every labelled simple graph on n vertices;
    graph g has pair k (in lexicographic order of i < j) iff bit k of g is set."""
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    G = 1 << len(pairs)
    g = np.arange(G, dtype=np.uint32)
    adj = np.zeros((G, n), dtype=np.uint8)
    for k, (i, j) in enumerate(pairs):
        bit = ((g >> np.uint32(k)) & np.uint32(1)).astype(np.uint8)
        adj[:, i] |= bit << np.uint8(j)
        adj[:, j] |= bit << np.uint8(i)
    return adj


def graph_records(adj: np.ndarray):
    """Edge records (src, dst, graph offsets) of every graph of an adjacency stack."""
    G, n = adj.shape
    srcs, dsts, gids = [], [], []
    for i in range(n):
        for j in range(i + 1, n):
            sel = np.nonzero((adj[:, i] >> np.uint8(j)) & np.uint8(1))[0]
            srcs.append(np.full(sel.shape, i, np.uint32))
            dsts.append(np.full(sel.shape, j, np.uint32))
            gids.append(sel)
    if not gids:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(G + 1, np.int64)
    gid = np.concatenate(gids)
    order = np.argsort(gid, kind="stable")
    src = np.concatenate(srcs)[order]
    dst = np.concatenate(dsts)[order]
    counts = np.bincount(gid, minlength=G)
    eoff = np.zeros(G + 1, np.int64)
    np.cumsum(counts, out=eoff[1:])
    return src, dst, eoff


def _argmin_over(mask, prio, n):
    """Per (graph, node): the name of smallest priority among the bits of mask [G, n]."""
    G = mask.shape[0]
    best = np.full((G, n), np.iinfo(np.int64).max, np.int64)
    arg = np.zeros((G, n), np.uint8)
    for y in range(n):
        has_y = ((mask >> np.uint8(y)) & np.uint8(1)).astype(bool)
        better = has_y & (prio[:, y:y + 1] < best)
        best = np.where(better, prio[:, y:y + 1], best)
        arg = np.where(better, np.uint8(y), arg)
    return arg


def brute_all(adj: np.ndarray, prio_of_round, max_rounds: int = 16, variant: str = "local"):
    """Run LocalContraction (or a variant) on a stack of graphs given by adjacency bitmasks
    over names 0..n-1.  prio_of_round(r) -> priorities [n] (or [G, n]) of the names in phase r.

    Labels of a phase, from the definitions (Section 3):
      local    argmin of rho over N(N(x)) (closed two-hop reachability);
      one_hop  argmin of rho over the closed N(x);
      tree     f(x) = argmin of rho over N(x) minus x; walk x, f(x), f(f(x)), ... n steps,
               which ends inside the terminal 2-cycle {y, f(y)} (Lemma "cycle"); the label is
               the member of the cycle with the smaller priority (two nodes share a class iff
               they share the cycle, Lemma "wccs").

    Returns (labels [G, n], rounds [G], parents [max_rounds, G, n] with 255 for names that
    are not nodes of that phase, stats [max_rounds, G, 5])."""
    G, n = adj.shape
    adj = adj.copy()
    labels = np.tile(np.arange(n, dtype=np.uint8), (G, 1))
    rounds = np.zeros(G, np.int32)
    parents = np.full((max_rounds, G, n), 255, np.uint8)
    stats = np.zeros((max_rounds, G, 5), np.int64)
    bit = (np.uint8(1) << np.arange(n, dtype=np.uint8))
    popc = np.array([bin(i).count("1") for i in range(256)], np.int64)
    for r in range(max_rounds):
        in_v = adj != 0                               # nodes of this phase: names with an edge
        running = in_v.any(axis=1)
        if not running.any():
            break
        rounds += running
        prio = np.asarray(prio_of_round(r), dtype=np.int64)
        if prio.ndim == 1:
            prio = np.broadcast_to(prio, (G, n))
        n1 = adj | bit[None, :]                       # closed neighbourhood N(x)
        if variant == "local":
            n2 = n1.copy()                            # N(N(x))
            for y in range(n):
                has_y = ((n1 >> np.uint8(y)) & np.uint8(1)).astype(bool)
                n2 |= np.where(has_y, n1[:, y:y + 1], np.uint8(0))
            arg = _argmin_over(n2, prio, n)
        elif variant == "one_hop":
            arg = _argmin_over(n1, prio, n)
        else:
            f = _argmin_over(adj, prio, n).astype(np.int64)     # open neighbourhood
            y = np.tile(np.arange(n, dtype=np.int64), (G, 1))
            for _ in range(n):
                y = np.take_along_axis(f, y, axis=1)
            fy = np.take_along_axis(f, y, axis=1)
            py = np.take_along_axis(prio, y, axis=1)
            pfy = np.take_along_axis(prio, fy, axis=1)
            arg = np.where(py < pfy, y, fy).astype(np.uint8)
        par = np.where(in_v, arg, np.uint8(255))
        parents[r] = par
        # next graph: the parents of the two endpoints of each edge, loops dropped
        pbit = np.where(in_v, np.uint8(1) << np.where(in_v, arg, 0).astype(np.uint8), np.uint8(0))
        nb = np.zeros((G, n), np.uint8)
        for x in range(n):
            for y in range(n):
                e = ((adj[:, x] >> np.uint8(y)) & np.uint8(1)).astype(bool)
                nb[:, x] |= np.where(e, pbit[:, y], np.uint8(0))
        new_adj = np.zeros((G, n), np.uint8)
        is_label = np.zeros((G, n), bool)
        for x in range(n):
            for t in range(n):
                sel = in_v[:, x] & (arg[:, x] == t)
                new_adj[:, t] |= np.where(sel, nb[:, x], np.uint8(0))
                is_label[:, t] |= sel
        new_adj &= ~bit[None, :]
        # stats: n_active, m_in, m_survive, m_out, n_finalised
        m_in = popc[adj].sum(axis=1) // 2
        surv = np.zeros(G, np.int64)
        for x in range(n):
            for y in range(x + 1, n):
                e = ((adj[:, x] >> np.uint8(y)) & np.uint8(1)).astype(bool)
                surv += e & (arg[:, x] != arg[:, y])
        m_out = popc[new_adj].sum(axis=1) // 2
        n_next = (new_adj != 0).sum(axis=1)
        stats[r, :, 0] = np.where(running, in_v.sum(axis=1), 0)
        stats[r, :, 1] = np.where(running, m_in, 0)
        stats[r, :, 2] = np.where(running, surv, 0)
        stats[r, :, 3] = np.where(running, m_out, 0)
        stats[r, :, 4] = np.where(running, is_label.sum(axis=1) - n_next, 0)
        # compose the labels of the original vertices
        for v in range(n):
            cur = labels[:, v]
            cur_in = np.take_along_axis(in_v, cur[:, None].astype(np.int64), axis=1)[:, 0]
            moved = np.take_along_axis(arg, cur[:, None].astype(np.int64), axis=1)[:, 0]
            labels[:, v] = np.where(cur_in, moved, cur)
        adj = new_adj
    return labels, rounds, parents, stats


# --------------------------------------------------------------------------------------
# definitions at scale
# --------------------------------------------------------------------------------------

def simple_edges(src, dst):
    """Sorted unique loop-free undirected pairs (lo, hi) of a record list."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    keep = src != dst
    lo = np.minimum(src[keep], dst[keep])
    hi = np.maximum(src[keep], dst[keep])
    key = np.unique(lo * (1 << 32) + hi)
    return (key >> 32).astype(np.int64), (key & 0xFFFFFFFF).astype(np.int64)


def two_hop_parents(n: int, lo, hi, prio: np.ndarray):
    """For every node x (a name with an edge): the vertex of smallest priority among the
    vertices at distance <= 2 from x, via the sparse pattern of (A + I)^2."""
    nodes = np.unique(np.concatenate([lo, hi]))
    A = sp.coo_matrix((np.ones(lo.shape[0] * 2, np.int8), (np.concatenate([lo, hi]), np.concatenate([hi, lo]))),
                      shape=(n, n)).tocsr()
    A1 = (A + sp.identity(n, dtype=np.int8, format="csr")).astype(bool).astype(np.int32)
    A2 = (A1 @ A1).tocsr()
    A2.sort_indices()
    out = np.full(n, -1, np.int64)
    ip, ind = A2.indptr, A2.indices
    pr = prio[ind].astype(np.int64)
    for x in nodes:
        seg = slice(ip[x], ip[x + 1])
        out[x] = ind[seg][np.argmin(pr[seg])]
    return nodes, out


def union_find(n: int, src, dst) -> np.ndarray:
    """Textbook union-find (path halving, union by size); returns the root of every vertex."""
    parent = list(range(n))
    size = [1] * n

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            if size[ra] < size[rb]:
                ra, rb = rb, ra
            parent[rb] = ra
            size[ra] += size[rb]
    return np.array([find(x) for x in range(n)], np.int64)


def canon(labels) -> np.ndarray:
    """Canonical partition: every vertex maps to the smallest vertex id with its label."""
    labels = np.asarray(labels, np.int64)
    n = labels.shape[0]
    if n == 0:
        return labels
    uniq, inv = np.unique(labels, return_inverse=True)
    first = np.full(uniq.shape[0], n, np.int64)
    np.minimum.at(first, inv, np.arange(n, dtype=np.int64))
    return first[inv]


def scipy_components(n: int, src, dst) -> np.ndarray:
    from scipy.sparse.csgraph import connected_components
    A = sp.coo_matrix((np.ones(len(src), np.int8), (np.asarray(src, np.int64), np.asarray(dst, np.int64))),
                      shape=(n, n)).tocsr()
    _, lab = connected_components(A, directed=True, connection="weak")
    return lab


def contract_edges(a, b, parent_of):
    """The contraction step (proof of the lemma in Section 3) applied to edges (a[i], b[i])
    by name: the distinct loop-free pairs (parent(a), parent(b)), as sorted uint64 keys
    (smaller name << 32) | larger name.  Loops among (a, b) are dropped first."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    keep = a != b
    pa = np.asarray(parent_of, dtype=np.uint64)[a[keep].astype(np.int64)]
    pb = np.asarray(parent_of, dtype=np.uint64)[b[keep].astype(np.int64)]
    keep = pa != pb
    lo = np.minimum(pa[keep], pb[keep])
    hi = np.maximum(pa[keep], pb[keep])
    return np.unique((lo << np.uint64(32)) | hi)


def split_keys(k):
    """(a, b) name arrays of uint64 keys (a << 32) | b."""
    k = np.asarray(k, dtype=np.uint64)
    return (k >> np.uint64(32)).astype(np.uint32), (k & np.uint64(0xFFFFFFFF)).astype(np.uint32)


# --------------------------------------------------------------------------------------
# MergeToLarge, restated step by step with sets (small graphs only)
# --------------------------------------------------------------------------------------

def merge_to_large_reference(n: int, src, dst, prio_of, alphas, max_rounds: int = 64):
    """LocalContraction phases each followed by the MergeToLarge step (Section 5), written
    with Python sets and dictionaries, independent of the oracle's arrays.

    prio_of(r, v) -> priority of name v in round r (only even rounds are LocalContraction
    steps; their priorities are compared by the smallest).  Phase i is round 2i; its step,
    round 2i + 1, works on the graph the phase left: a node is large when its class had at
    least alpha_i nodes, its priority is the alpha_i-th largest member priority, and every
    node takes the large node of largest priority within distance 2 (itself included) as its
    label, or keeps itself.  Returns (labels, rounds, parents per round as dicts, stats per
    round as tuples (round, n_active, m_in, m_survive, m_out, n_finalised))."""
    src = [int(x) for x in np.asarray(src).tolist()]
    dst = [int(x) for x in np.asarray(dst).tolist()]
    records = [(a, b) for a, b in zip(src, dst) if a != b]
    E = {(min(a, b), max(a, b)) for a, b in records}
    label = list(range(n))
    parents, stats = [], []
    large, mprio = {}, {}
    r = 0
    while E and r < max_rounds:
        V = sorted({x for e in E for x in e})
        nb = {v: {v} for v in V}
        for a, b in E:
            nb[a].add(b)
            nb[b].add(a)
        two = {v: set().union(*(nb[u] for u in nb[v])) for v in V}
        if r % 2 == 0:
            rho = {v: prio_of(r, v) for v in V}
            par = {v: min(two[v], key=lambda u: rho[u]) for v in V}
            members = {}
            for v in V:
                members.setdefault(par[v], []).append(rho[v])
            alpha = alphas[min(r // 2, len(alphas) - 1)]
            large = {y: len(ms) >= alpha for y, ms in members.items()}
            mprio = {y: sorted(ms, reverse=True)[alpha - 1] for y, ms in members.items() if len(ms) >= alpha}
        else:
            par = {}
            for v in V:
                cands = [u for u in two[v] if large.get(u, False)]
                par[v] = max(cands, key=lambda u: mprio[u]) if cands else v
        parents.append(par)
        edges_in = records if r == 0 else sorted(E)
        survive = sum(1 for a, b in edges_in if par[a] != par[b])
        E2 = {(min(par[a], par[b]), max(par[a], par[b])) for a, b in E if par[a] != par[b]}
        keep = {x for e in E2 for x in e}
        fin = len(set(par.values()) - keep)
        stats.append((r, len(V), len(src) if r == 0 else len(E), survive, len(E2), fin))
        label = [par.get(l, l) for l in label]
        E = E2
        r += 1
    return np.array(label, np.int64), r, parents, stats

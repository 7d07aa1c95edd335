"""Multilevel p-way vertex-separator reordering (Sec. 3, Alg. 3).

The paper partitions the graph of |C_{l-1}| + |C_{l-1}^T| at every level
with a p-way vertex separator (ParMETIS) and recurses on the separator's
induced subgraph until the requested number of levels is reached or the
separator is too small to split (Sec. 3.2).  For grid graphs this oracle
uses a geometric separator:

  * per axis with N points and q = p^(1/dim) parts, the cut coordinates are
    c_j = floor(j (N+1) / q), j = 1..q-1 (0-based coordinates);
  * a vertex's class is how many of its coordinates lie on a cut;
  * level l takes B_l = {class == l} and C_l = {class > l}.

Class-0 vertices split into the q^dim boxes with no edge between two boxes;
class-l vertices (faces, then edges ...) split the same way inside the
previous separator, so each level is a valid vertex separator of the
previous level's separator (Sec. 3, definition of a p-way vertex separator).

Stop rule (Sec. 3.2): recursion stops after min(levels, dim) levels, or
earlier when the next separator has fewer than p vertices or no edges.

The diagonal blocks B_l^(i) are the connected components of the level's
vertex set in the graph of |A|+|A^T|, ordered by their smallest original
index; rows keep ascending original index inside a block.  The same rule
gives the block-Jacobi blocks of the last separator C_last (Sec. 4.3).
The global permutation is [B_0 blocks, B_1 blocks, ..., B_{L-1}, C_last]
(the layout of the "global permutation" figure in Sec. 3.2), so every C_l is
the tail of the permuted vector and the per-level permutations P_l compose
into one.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclass
class Partition:
    perm: np.ndarray          # perm[new] = old
    nlevels: int              # L (levels with a Schur complement)
    level_start: np.ndarray   # L+2 entries: start of B_0..B_{L-1}, C_last, n
    blocks: list              # L+1 arrays of global block boundaries

    @property
    def n(self):
        return len(self.perm)


def grid_classes(dims, nparts):
    """Return (class per vertex, q).  Vertex i has coordinates x + N y + ..."""
    dim = len(dims)
    q = int(round(nparts ** (1.0 / dim)))
    if q ** dim != nparts:
        raise ValueError(f"nparts={nparts} is not a {dim}-th power")
    n = int(np.prod(dims))
    cls = np.zeros(n, dtype=np.int64)
    idx = np.arange(n)
    stride = 1
    for N in dims:
        c = (idx // stride) % N
        cuts = [(j * (N + 1)) // q for j in range(1, q)]
        cls += np.isin(c, cuts)
        stride *= N
    return cls, q


def _pattern_graph(n, rowptr, col):
    a = sp.csr_matrix((np.ones(len(col)), col, rowptr), shape=(n, n))
    g = (abs(a) + abs(a.T)).tocsr()
    g.setdiag(0)
    g.eliminate_zeros()
    return g


def _components(g, verts):
    """Connected components of the subgraph induced by `verts` (sorted
    original indices); returned in order of their smallest vertex, each
    sorted ascending."""
    if len(verts) == 0:
        return []
    sub = g[verts][:, verts]
    ncomp, lab = connected_components(sub, directed=False)
    comps = [verts[lab == c] for c in range(ncomp)]
    comps.sort(key=lambda c: c[0])
    return comps


def _has_edges(g, verts):
    if len(verts) == 0:
        return False
    return g[verts][:, verts].nnz > 0


def wirebasket(dims, nparts, levels, rowptr, col):
    """Alg. 3 with the geometric separator; returns a Partition."""
    n = int(np.prod(dims))
    g = _pattern_graph(n, rowptr, col)
    cls, q = grid_classes(dims, nparts)
    dim = len(dims)
    if q == 1:
        L = 1
    else:
        L = min(levels, dim)
        for l in range(L - 1):
            rest = np.nonzero(cls > l)[0]
            if len(rest) < nparts or not _has_edges(g, rest):
                L = l + 1
                break
    groups = [np.nonzero(cls == l)[0] for l in range(L)]
    groups.append(np.nonzero(cls >= L)[0])
    perm, level_start, blocks = [], [0], []
    pos = 0
    for verts in groups:
        comps = _components(g, verts)
        bnd = [pos]
        for c in comps:
            perm.append(c)
            pos += len(c)
            bnd.append(pos)
        blocks.append(np.array(bnd, dtype=np.int64))
        level_start.append(pos)
    perm = np.concatenate(perm) if perm else np.zeros(0, np.int64)
    return Partition(perm.astype(np.int64), L,
                     np.array(level_start, dtype=np.int64), blocks)


# ---------------------------------------------------------------- algebraic
# Partitioner for matrices without grid coordinates (the paper uses
# ParMETIS, Sec. 3.2): nested dissection by breadth-first level structures.
#
#   bisect(P): if the subgraph induced by P is disconnected, its components
#     (largest first, ties by smallest vertex) go to the lighter of two
#     halves (ties to the first), with no separator; otherwise the levels of
#     a breadth-first search from a pseudo-peripheral vertex are computed,
#     m is the level of the vertex at position floor(|P|/2) when P is sorted
#     by (level, index) (the last level is replaced by the one before it),
#     the separator S is the level-m vertices with a neighbour in level m+1,
#     and the halves are {level < m} + (level m minus S) and {level > m}.
#     No edge joins the two halves.
#   pseudo-peripheral vertex: start at the smallest vertex of P; repeatedly
#     move to the smallest vertex of the last level while that increases the
#     eccentricity (at most 10 moves).
#   p-way separator (p = 2^d): d rounds of bisecting every current part; the
#     separator is the union of all bisection separators.
#   levels (Alg. 3): the separator of level l is partitioned again with the
#     same p; class(v) = number of separators v belongs to, and the
#     structure is assembled from the classes exactly as for grids (same
#     stop rule and block order), with at most max(class) levels so that the
#     last separator C_last is never empty.

def _adjacency(n, rowptr, col):
    g = _pattern_graph(n, rowptr, col)
    return [g.indices[g.indptr[i]:g.indptr[i + 1]] for i in range(n)]


def _bfs(adj, inP, r):
    lev = {r: 0}
    frontier = [r]
    d = 0
    while frontier:
        nxt = []
        for u in frontier:
            for w in adj[u]:
                if inP[w] and w not in lev:
                    lev[w] = d + 1
                    nxt.append(w)
        frontier = nxt
        d += 1
    return lev


def _components_list(adj, inP, P):
    seen = set()
    comps = []
    for v in P:
        if v in seen:
            continue
        lev = _bfs(adj, inP, v)
        comp = sorted(lev)
        seen.update(comp)
        comps.append(comp)
    return comps


def _bisect(adj, inP, P):
    if len(P) <= 1:
        return list(P), [], []
    comps = _components_list(adj, inP, P)
    if len(comps) > 1:
        order = sorted(range(len(comps)), key=lambda i: (-len(comps[i]), comps[i][0]))
        A, B, na, nb = [], [], 0, 0
        for i in order:
            if na <= nb:
                A += comps[i]
                na += len(comps[i])
            else:
                B += comps[i]
                nb += len(comps[i])
        return sorted(A), sorted(B), []
    r = P[0]
    lev = _bfs(adj, inP, r)
    ecc = max(lev.values())
    for _ in range(10):
        cand = min(v for v, l in lev.items() if l == ecc)
        lev2 = _bfs(adj, inP, cand)
        ecc2 = max(lev2.values())
        if ecc2 <= ecc:
            break
        r, lev, ecc = cand, lev2, ecc2
    order = sorted(P, key=lambda v: (lev[v], v))
    m = lev[order[len(P) // 2]]
    if m == ecc:
        m = ecc - 1
    S = [v for v in P if lev[v] == m and any(inP[w] and lev[w] == m + 1 for w in adj[v])]
    Sset = set(S)
    A = [v for v in P if lev[v] < m or (lev[v] == m and v not in Sset)]
    B = [v for v in P if lev[v] > m]
    return A, B, S


def _nd_separator(adj, n, verts, d):
    inP = np.zeros(n, dtype=bool)
    parts = [list(verts)]
    seps = []
    for _ in range(d):
        new = []
        for P in parts:
            inP[:] = False
            inP[P] = True
            A, B, S = _bisect(adj, inP, P)
            seps += S
            new += [A, B]
        parts = new
    return np.array(sorted(seps), dtype=np.int64)


def algebraic(n, nparts, levels, rowptr, col):
    """Alg. 3 with the nested-dissection separator above; returns a
    Partition.  nparts must be a power of two."""
    d = int(round(np.log2(nparts))) if nparts >= 1 else -1
    if nparts < 1 or 2 ** d != nparts:
        raise ValueError("nparts must be a power of two")
    adj = _adjacency(n, rowptr, col)
    g = _pattern_graph(n, rowptr, col)
    cls = np.zeros(n, dtype=np.int64)
    active = np.arange(n)
    for l in range(levels):
        if d == 0 or len(active) == 0:
            break
        S = _nd_separator(adj, n, active, d)
        cls[S] = l + 1
        active = S
    if nparts == 1 or cls.max() == 0:
        L = 1
    else:
        # at most as many levels as separator classes, so C_last is never empty
        L = min(levels, int(cls.max()))
        for l in range(L - 1):
            rest = np.nonzero(cls > l)[0]
            if len(rest) < nparts or not _has_edges(g, rest):
                L = l + 1
                break
    groups = [np.nonzero(cls == l)[0] for l in range(L)]
    groups.append(np.nonzero(cls >= L)[0])
    perm, level_start, blocks = [], [0], []
    pos = 0
    for verts in groups:
        comps = _components(g, verts)
        bnd = [pos]
        for c in comps:
            perm.append(c)
            pos += len(c)
            bnd.append(pos)
        blocks.append(np.array(bnd, dtype=np.int64))
        level_start.append(pos)
    perm = np.concatenate(perm) if perm else np.zeros(0, np.int64)
    return Partition(perm.astype(np.int64), L, np.array(level_start, dtype=np.int64), blocks)

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


def from_user(perm, level_start, rowptr, col):
    """Partition from a user permutation and level boundaries; blocks are the
    connected components inside each level segment (in segment order)."""
    perm = np.asarray(perm, dtype=np.int64)
    n = len(perm)
    g = _pattern_graph(n, rowptr, col)
    gp = g[perm][:, perm].tocsr()
    level_start = np.asarray(level_start, dtype=np.int64)
    blocks = []
    for l in range(len(level_start) - 1):
        a, b = level_start[l], level_start[l + 1]
        verts = np.arange(a, b)
        comps = _components(gp, verts)
        if any(np.any(np.diff(c) != 1) for c in comps):
            raise ValueError("user level segment is not ordered by component")
        bnd = [a] + [int(c[-1]) + 1 for c in comps]
        blocks.append(np.array(bnd, dtype=np.int64))
    return Partition(perm, len(level_start) - 2, level_start, blocks)

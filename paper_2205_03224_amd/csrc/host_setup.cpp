// Host stages of the GeMSLR setup: CSR validation, the multilevel geometric
// vertex-separator reordering (Alg. 3), extraction of the level blocks
// A_l = [B_l F_l; E_l C_l] (Sec. 2.4) and incomplete LU of every diagonal
// block (Alg. 1, ILU(0) and Saad's dual-threshold ILUT).
//
// Built with -ffp-contract=off so that every multiply and add rounds on its
// own: the factorisation is then reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>
#include <queue>
#include <thread>
#include <atomic>
#include <mutex>

#include "gs_internal.h"

namespace gs {

void validate_csr(int64_t n, const int64_t* rp, const int32_t* ci,
                  bool need_diag) {
  if (n <= 0) throw Error(GS_EINVAL, "n must be positive");
  if (!rp || !ci) throw Error(GS_EINVAL, "NULL CSR array");
  if (rp[0] != 0) throw Error(GS_EINVAL, "rowptr[0] != 0");
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) throw Error(GS_EINVAL, "rowptr not monotone");
    bool diag = false;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      int64_t c = ci[p];
      if (c < 0 || c >= n)
        throw Error(GS_EINVAL, "column index out of range in row " + std::to_string(i));
      if (p > rp[i] && ci[p - 1] >= c)
        throw Error(GS_EINVAL, "columns not strictly ascending in row " + std::to_string(i));
      if (c == i) diag = true;
    }
    if (need_diag && !diag)
      throw Error(GS_EINVAL, "missing diagonal entry in row " + std::to_string(i));
  }
}

// ---------------------------------------------------------------- partition

namespace {

// Symmetrised adjacency (pattern of |A| + |A^T| without the diagonal).
struct Graph {
  std::vector<int64_t> xadj;
  std::vector<int64_t> adj;
};

Graph sym_graph(int64_t n, const int64_t* rp, const int32_t* ci) {
  std::vector<int64_t> deg(n, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
      if (ci[p] != i) { deg[i]++; deg[ci[p]]++; }
  Graph g;
  g.xadj.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) g.xadj[i + 1] = g.xadj[i] + deg[i];
  g.adj.resize(g.xadj[n]);
  std::vector<int64_t> pos(g.xadj.begin(), g.xadj.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      int64_t j = ci[p];
      if (j != i) { g.adj[pos[i]++] = j; g.adj[pos[j]++] = i; }
    }
  // sort + unique each list
  for (int64_t i = 0; i < n; ++i) {
    auto b = g.adj.begin() + g.xadj[i], e = g.adj.begin() + g.xadj[i + 1];
    std::sort(b, e);
  }
  return g;
}

// Components of the subgraph induced by vertices with in_set[v]; discovered
// by scanning vertices in ascending order, so they come ordered by smallest
// vertex; each is returned sorted.
std::vector<std::vector<int64_t>> components(const Graph& g,
                                             const std::vector<char>& in_set) {
  int64_t n = (int64_t)in_set.size();
  std::vector<char> seen(n, 0);
  std::vector<std::vector<int64_t>> comps;
  std::vector<int64_t> stack;
  for (int64_t v = 0; v < n; ++v) {
    if (!in_set[v] || seen[v]) continue;
    std::vector<int64_t> comp;
    stack.push_back(v);
    seen[v] = 1;
    while (!stack.empty()) {
      int64_t u = stack.back();
      stack.pop_back();
      comp.push_back(u);
      for (int64_t p = g.xadj[u]; p < g.xadj[u + 1]; ++p) {
        int64_t w = g.adj[p];
        if (in_set[w] && !seen[w]) { seen[w] = 1; stack.push_back(w); }
      }
    }
    std::sort(comp.begin(), comp.end());
    comps.push_back(std::move(comp));
  }
  return comps;
}

bool has_edges(const Graph& g, const std::vector<char>& in_set) {
  int64_t n = (int64_t)in_set.size();
  for (int64_t v = 0; v < n; ++v) {
    if (!in_set[v]) continue;
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p)
      if (in_set[g.adj[p]]) return true;
  }
  return false;
}

Partition assemble(const Graph& g, const std::vector<int>& cls, int nparts, int Lmax);

}  // namespace

Partition partition_grid(int ndim, const int32_t* dims, int nparts, int levels,
                         int64_t n, const int64_t* rp, const int32_t* ci) {
  if (ndim < 1 || ndim > 3 || !dims) throw Error(GS_EINVAL, "grid_ndim must be 1..3");
  if (nparts < 1 || levels < 1) throw Error(GS_EINVAL, "nparts and levels must be >= 1");
  int64_t prod = 1;
  for (int a = 0; a < ndim; ++a) {
    if (dims[a] < 1) throw Error(GS_EINVAL, "grid dimension < 1");
    prod *= dims[a];
  }
  if (prod != n) throw Error(GS_EINVAL, "grid dims do not match n");
  int q = 1;
  while (true) {
    int64_t p = 1;
    for (int a = 0; a < ndim; ++a) p *= (q + 1);
    if (p > nparts) break;
    ++q;
  }
  {
    int64_t p = 1;
    for (int a = 0; a < ndim; ++a) p *= q;
    if (p != nparts) throw Error(GS_EINVAL, "nparts is not a dim-th power");
  }
  // cut membership per axis: c_j = floor(j (N+1) / q), j = 1..q-1
  std::vector<std::vector<char>> oncut(ndim);
  for (int a = 0; a < ndim; ++a) {
    oncut[a].assign(dims[a], 0);
    for (int j = 1; j < q; ++j) {
      int64_t c = ((int64_t)j * (dims[a] + 1)) / q;
      if (c < dims[a]) oncut[a][c] = 1;
    }
  }
  std::vector<int> cls(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t r = i;
    int c = 0;
    for (int a = 0; a < ndim; ++a) {
      int64_t x = r % dims[a];
      r /= dims[a];
      c += oncut[a][x];
    }
    cls[i] = c;
  }
  Graph g = sym_graph(n, rp, ci);
  return assemble(g, cls, nparts, q == 1 ? 1 : std::min(levels, ndim));
}

namespace {

// The level structure from vertex classes (B_l = class l, C_l = class > l):
// at most Lmax levels, fewer when the next separator has fewer than nparts
// vertices or no edges (Sec. 3.2); blocks are the connected components in
// order of their smallest vertex, rows ascending inside a block.
Partition assemble(const Graph& g, const std::vector<int>& cls, int nparts, int Lmax) {
  const int64_t n = (int64_t)cls.size();
  int L = std::max(1, Lmax);
  for (int l = 0; l < L - 1; ++l) {
    std::vector<char> rest(n);
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) { rest[i] = cls[i] > l; cnt += rest[i]; }
    if (cnt < nparts || !has_edges(g, rest)) { L = l + 1; break; }
  }
  Partition P;
  P.L = L;
  P.level_start.push_back(0);
  int64_t pos = 0;
  for (int l = 0; l <= L; ++l) {
    std::vector<char> in(n);
    for (int64_t i = 0; i < n; ++i) in[i] = (l < L) ? (cls[i] == l) : (cls[i] >= L);
    auto comps = components(g, in);
    std::vector<int64_t> bnd{pos};
    for (auto& c : comps) {
      P.perm.insert(P.perm.end(), c.begin(), c.end());
      pos += (int64_t)c.size();
      bnd.push_back(pos);
    }
    P.blocks.push_back(std::move(bnd));
    P.level_start.push_back(pos);
  }
  return P;
}

// ---- algebraic separator: nested dissection by breadth-first level
// structures (the rules of the algebraic partitioner, stated in
// include/gemslr.h at gs_partition_graph).  Work arrays are indexed by the
// position of a vertex in the current part P.
struct NdWork {
  std::vector<int64_t> loc;   // vertex -> position in P, -1 outside
  std::vector<int> lev;       // BFS level per position, -1 unreached
  std::vector<int64_t> queue;
  explicit NdWork(int64_t n) : loc(n, -1) {}
};

// BFS levels over P from position r; returns the eccentricity
static int bfs_levels(const Graph& g, const std::vector<int64_t>& P, NdWork& W, int64_t r) {
  W.lev.assign(P.size(), -1);
  W.queue.clear();
  W.queue.push_back(r);
  W.lev[r] = 0;
  int ecc = 0;
  for (size_t h = 0; h < W.queue.size(); ++h) {
    const int64_t u = W.queue[h];
    const int lu = W.lev[u];
    ecc = std::max(ecc, lu);
    for (int64_t p = g.xadj[P[u]]; p < g.xadj[P[u] + 1]; ++p) {
      const int64_t w = W.loc[g.adj[p]];
      if (w >= 0 && W.lev[w] < 0) { W.lev[w] = lu + 1; W.queue.push_back(w); }
    }
  }
  return ecc;
}

// Bisect P (sorted) into A, B and separator S.
static void bisect(const Graph& g, const std::vector<int64_t>& P, NdWork& W,
                   std::vector<int64_t>& A, std::vector<int64_t>& B, std::vector<int64_t>& S) {
  A.clear(); B.clear(); S.clear();
  if (P.size() <= 1) { A = P; return; }
  for (size_t i = 0; i < P.size(); ++i) W.loc[P[i]] = (int64_t)i;
  // connected components of P (each sorted, in order of the smallest vertex)
  std::vector<std::vector<int64_t>> comps;
  {
    std::vector<int> comp(P.size(), -1);
    for (size_t i = 0; i < P.size(); ++i) {
      if (comp[i] >= 0) continue;
      bfs_levels(g, P, W, (int64_t)i);
      std::vector<int64_t> c;
      for (size_t j = 0; j < P.size(); ++j)
        if (W.lev[j] >= 0) { comp[j] = (int)comps.size(); c.push_back(P[j]); }
      comps.push_back(std::move(c));
    }
  }
  if (comps.size() > 1) {
    std::vector<size_t> order(comps.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) {
      if (comps[x].size() != comps[y].size()) return comps[x].size() > comps[y].size();
      return comps[x][0] < comps[y][0];
    });
    size_t na = 0, nb = 0;
    for (size_t i : order) {
      if (na <= nb) { A.insert(A.end(), comps[i].begin(), comps[i].end()); na += comps[i].size(); }
      else { B.insert(B.end(), comps[i].begin(), comps[i].end()); nb += comps[i].size(); }
    }
    std::sort(A.begin(), A.end());
    std::sort(B.begin(), B.end());
  } else {
    // pseudo-peripheral start: smallest vertex, then the smallest vertex of
    // the last level while the eccentricity grows (at most 10 moves)
    int64_t r = 0;
    int ecc = bfs_levels(g, P, W, r);
    for (int it = 0; it < 10; ++it) {
      int64_t cand = -1;
      for (size_t j = 0; j < P.size(); ++j)
        if (W.lev[j] == ecc) { cand = (int64_t)j; break; }  // P sorted: smallest vertex
      std::vector<int> keep = W.lev;
      const int ecc2 = bfs_levels(g, P, W, cand);
      if (ecc2 <= ecc) { W.lev = keep; break; }
      r = cand;
      ecc = ecc2;
    }
    // level of the median vertex in (level, index) order
    std::vector<int64_t> cnt(ecc + 2, 0);
    for (int l : W.lev) ++cnt[l];
    const int64_t half = (int64_t)P.size() / 2;
    int m = 0;
    for (int64_t acc = 0; m <= ecc; ++m) {
      if (acc + cnt[m] > half) break;
      acc += cnt[m];
    }
    if (m == ecc) m = ecc - 1;
    for (size_t j = 0; j < P.size(); ++j) {
      const int lj = W.lev[j];
      if (lj < m) { A.push_back(P[j]); continue; }
      if (lj > m) { B.push_back(P[j]); continue; }
      bool sep = false;
      for (int64_t p = g.xadj[P[j]]; p < g.xadj[P[j] + 1] && !sep; ++p) {
        const int64_t w = W.loc[g.adj[p]];
        sep = w >= 0 && W.lev[w] == m + 1;
      }
      (sep ? S : A).push_back(P[j]);
    }
  }
  for (int64_t v : P) W.loc[v] = -1;
}

}  // namespace

Partition partition_graph(int nparts, int levels, int64_t n, const int64_t* rp,
                          const int32_t* ci) {
  if (nparts < 1 || (nparts & (nparts - 1)) != 0)
    throw Error(GS_EINVAL, "the algebraic partitioner needs nparts = a power of two");
  if (levels < 1) throw Error(GS_EINVAL, "levels must be >= 1");
  int d = 0;
  while ((1 << d) < nparts) ++d;
  Graph g = sym_graph(n, rp, ci);
  std::vector<int> cls(n, 0);
  std::vector<int64_t> active(n);
  for (int64_t i = 0; i < n; ++i) active[i] = i;
  NdWork W(n);
  std::vector<int64_t> A, B, S;
  for (int l = 0; l < levels && d > 0 && !active.empty(); ++l) {
    std::vector<std::vector<int64_t>> parts{active};
    std::vector<int64_t> seps;
    for (int r = 0; r < d; ++r) {
      std::vector<std::vector<int64_t>> next;
      for (auto& Pp : parts) {
        bisect(g, Pp, W, A, B, S);
        seps.insert(seps.end(), S.begin(), S.end());
        next.push_back(A);
        next.push_back(B);
      }
      parts.swap(next);
    }
    std::sort(seps.begin(), seps.end());
    for (int64_t v : seps) cls[v] = l + 1;
    active.swap(seps);
  }
  int maxc = 0;
  for (int c : cls) maxc = std::max(maxc, c);
  return assemble(g, cls, nparts, (nparts == 1 || maxc == 0) ? 1 : std::min(levels, maxc));
}

// ---------------------------------------------------------------- levels

template <class T>
CSR<T> permute(const CSR<T>& A, const std::vector<int64_t>& perm) {
  const int64_t n = A.nrows;
  std::vector<int64_t> inv(n);
  for (int64_t i = 0; i < n; ++i) inv[perm[i]] = i;
  CSR<T> Ap;
  Ap.nrows = Ap.ncols = n;
  Ap.rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t o = perm[i];
    Ap.rp[i + 1] = Ap.rp[i] + (A.rp[o + 1] - A.rp[o]);
  }
  Ap.ci.resize(Ap.nnz());
  Ap.v.resize(Ap.nnz());
  std::vector<std::pair<int64_t, T>> row;
  for (int64_t i = 0; i < n; ++i) {
    int64_t o = perm[i];
    row.clear();
    for (int64_t p = A.rp[o]; p < A.rp[o + 1]; ++p) row.push_back({inv[A.ci[p]], A.v[p]});
    std::sort(row.begin(), row.end(),
              [](const auto& x, const auto& y) { return x.first < y.first; });
    for (size_t t = 0; t < row.size(); ++t) {
      Ap.ci[Ap.rp[i] + t] = (int32_t)row[t].first;
      Ap.v[Ap.rp[i] + t] = row[t].second;
    }
  }
  return Ap;
}

Partition user_partition(int64_t n, const int64_t* rp, const int32_t* ci, const int64_t* perm,
                         const int64_t* level_start, int L, const int64_t* block_ptr,
                         const int64_t* block_count) {
  if (!perm || !level_start) throw Error(GS_EINVAL, "user partition: perm and level_start needed");
  if (L < 0 || L > GS_MAX_LEVELS) throw Error(GS_EINVAL, "user partition: levels out of range");
  Partition p;
  p.L = L;
  p.perm.assign(perm, perm + n);
  {
    std::vector<char> seen((size_t)n, 0);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t o = perm[i];
      if (o < 0 || o >= n || seen[(size_t)o]) throw Error(GS_EINVAL, "user partition: perm is not a permutation");
      seen[(size_t)o] = 1;
    }
  }
  p.level_start.assign(level_start, level_start + L + 2);
  if (p.level_start[0] != 0 || p.level_start[(size_t)L + 1] != n)
    throw Error(GS_EINVAL, "user partition: level_start must run from 0 to n");
  for (int l = 0; l <= L; ++l)
    if (p.level_start[(size_t)l + 1] <= p.level_start[(size_t)l])
      throw Error(GS_EINVAL, "user partition: every segment needs at least one row");
  // new index of every original row
  std::vector<int64_t> inv((size_t)n);
  for (int64_t i = 0; i < n; ++i) inv[(size_t)perm[i]] = i;
  p.blocks.assign((size_t)L + 1, {});
  if (block_ptr) {
    if (!block_count) throw Error(GS_EINVAL, "user partition: block_ptr without block_count");
    int64_t o = 0;
    for (int l = 0; l <= L; ++l) {
      const int64_t nb = block_count[l];
      if (nb < 1) throw Error(GS_EINVAL, "user partition: a segment without blocks");
      std::vector<int64_t>& b = p.blocks[(size_t)l];
      b.assign(block_ptr + o, block_ptr + o + nb + 1);
      o += nb + 1;
      if (b.front() != p.level_start[(size_t)l] || b.back() != p.level_start[(size_t)l + 1])
        throw Error(GS_EINVAL, "user partition: blocks must cover their segment");
      for (int64_t t = 0; t < nb; ++t)
        if (b[(size_t)t + 1] <= b[(size_t)t]) throw Error(GS_EINVAL, "user partition: empty or unordered block");
    }
  } else {
    // connected components of each segment's rows in the symmetrised graph
    // of A (union-find over the entries inside the segment)
    std::vector<int64_t> parent((size_t)n);
    for (int64_t i = 0; i < n; ++i) parent[(size_t)i] = i;
    auto find = [&](int64_t x) {
      while (parent[(size_t)x] != x) {
        parent[(size_t)x] = parent[(size_t)parent[(size_t)x]];
        x = parent[(size_t)x];
      }
      return x;
    };
    auto seg_of = [&](int64_t r) {
      return (int)(std::upper_bound(p.level_start.begin(), p.level_start.end(), r) -
                   p.level_start.begin()) - 1;
    };
    for (int64_t o = 0; o < n; ++o) {
      const int64_t i = inv[(size_t)o];
      const int si = seg_of(i);
      for (int64_t q = rp[o]; q < rp[o + 1]; ++q) {
        const int64_t j = inv[(size_t)ci[q]];
        if (j == i || seg_of(j) != si) continue;
        const int64_t a = find(i), b = find(j);
        if (a != b) parent[(size_t)std::max(a, b)] = std::min(a, b);
      }
    }
    for (int l = 0; l <= L; ++l) {
      const int64_t a = p.level_start[(size_t)l], e = p.level_start[(size_t)l + 1];
      std::vector<int64_t>& b = p.blocks[(size_t)l];
      b.push_back(a);
      std::vector<char> done;  // roots already closed, by offset from a
      done.assign((size_t)(e - a), 0);
      int64_t cur = find(a);
      for (int64_t r = a + 1; r < e; ++r) {
        const int64_t root = find(r);
        if (root == cur) continue;
        done[(size_t)(cur - a)] = 1;
        if (done[(size_t)(root - a)])
          throw Error(GS_EINVAL, "user partition: a connected block of level " + std::to_string(l) +
                                     " is not contiguous in perm");
        b.push_back(r);
        cur = root;
      }
      b.push_back(e);
    }
  }
  // B_l must be block diagonal (the separator property); C_last's blocks
  // are cut on purpose (block-Jacobi)
  for (int l = 0; l < L; ++l) {
    const std::vector<int64_t>& b = p.blocks[(size_t)l];
    const int64_t a = p.level_start[(size_t)l], e = p.level_start[(size_t)l + 1];
    for (int64_t i = a; i < e; ++i) {
      const int64_t bi = std::upper_bound(b.begin(), b.end(), i) - b.begin();
      const int64_t o = perm[i];
      for (int64_t q = rp[o]; q < rp[o + 1]; ++q) {
        const int64_t j = inv[(size_t)ci[q]];
        if (j < a || j >= e) continue;
        if (std::upper_bound(b.begin(), b.end(), j) - b.begin() != bi)
          throw Error(GS_EINVAL, "user partition: two blocks of level " + std::to_string(l) +
                                     " are coupled by an entry of A");
      }
    }
  }
  return p;
}

template <class T>
void extract_levels(const CSR<T>& A, const Partition& part, HostSetup<T>& S) {
  const int64_t n = A.nrows;
  S.n = n;
  S.perm = part.perm;
  S.Ap = permute(A, part.perm);
  const CSR<T>& Ap = S.Ap;
  const int L = part.L;
  S.lv.assign(L + 1, HostLevel<T>());
  for (int l = 0; l <= L; ++l) {
    HostLevel<T>& lv = S.lv[l];
    const int64_t a = part.level_start[l];
    const int64_t b = (l < L) ? part.level_start[l + 1] : n;
    lv.start = a;
    lv.d = b - a;
    lv.s = n - b;
    lv.blocks.clear();
    for (int64_t x : part.blocks[l]) lv.blocks.push_back(x - a);
    // block label for the block-Jacobi cut of the last level
    std::vector<int64_t> lab;
    if (l == L) {
      lab.assign(lv.d, 0);
      for (size_t t = 0; t + 1 < lv.blocks.size(); ++t)
        for (int64_t r = lv.blocks[t]; r < lv.blocks[t + 1]; ++r) lab[r] = (int64_t)t;
    }
    auto& B = lv.L;  // reuse as scratch for B before factorisation
    B = CSR<T>();
    B.nrows = B.ncols = lv.d;
    lv.F = CSR<T>();
    lv.F.nrows = lv.d;
    lv.F.ncols = lv.s;
    for (int64_t i = a; i < b; ++i) {
      for (int64_t p = Ap.rp[i]; p < Ap.rp[i + 1]; ++p) {
        int64_t c = Ap.ci[p];
        if (c >= a && c < b) {
          if (l == L && lab[i - a] != lab[c - a]) continue;
          B.ci.push_back((int32_t)(c - a));
          B.v.push_back(Ap.v[p]);
        } else if (c >= b) {
          lv.F.ci.push_back((int32_t)(c - b));
          lv.F.v.push_back(Ap.v[p]);
        }
      }
      B.rp.push_back((int64_t)B.ci.size());
      lv.F.rp.push_back((int64_t)lv.F.ci.size());
    }
    lv.E = CSR<T>();
    lv.E.nrows = lv.s;
    lv.E.ncols = lv.d;
    for (int64_t i = b; i < n; ++i) {
      for (int64_t p = Ap.rp[i]; p < Ap.rp[i + 1]; ++p) {
        int64_t c = Ap.ci[p];
        if (c >= a && c < b) {
          lv.E.ci.push_back((int32_t)(c - a));
          lv.E.v.push_back(Ap.v[p]);
        }
      }
      lv.E.rp.push_back((int64_t)lv.E.ci.size());
    }
  }
}

// ---------------------------------------------------------------- ILU

template <class T>
void ilu0(const CSR<T>& B, CSR<T>& L, CSR<T>& U) {
  const int64_t n = B.nrows;
  L = CSR<T>();
  U = CSR<T>();
  L.nrows = L.ncols = U.nrows = U.ncols = n;
  std::vector<int64_t> where(n, -1);     // position of column j in the row
  std::vector<T> w;
  std::vector<int64_t> udiag(n);         // position of U(i,i) in U.v
  for (int64_t i = 0; i < n; ++i) {
    const int64_t p0 = B.rp[i], p1 = B.rp[i + 1];
    w.assign(B.v.begin() + p0, B.v.begin() + p1);
    for (int64_t p = p0; p < p1; ++p) where[B.ci[p]] = p - p0;
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t k = B.ci[p];
      if (k >= i) break;
      T& wk = w[p - p0];
      wk = wk / U.v[udiag[k]];
      for (int64_t q = udiag[k] + 1; q < U.rp[k + 1]; ++q) {
        int64_t pos = where[U.ci[q]];
        if (pos >= 0) w[pos] = w[pos] - wk * U.v[q];
      }
    }
    bool hasdiag = false;
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t c = B.ci[p];
      if (c < i) { L.ci.push_back((int32_t)c); L.v.push_back(w[p - p0]); }
      else {
        if (c == i) { hasdiag = true; udiag[i] = (int64_t)U.v.size(); }
        U.ci.push_back((int32_t)c);
        U.v.push_back(w[p - p0]);
      }
      where[c] = -1;
    }
    if (!hasdiag) throw Error(GS_EZEROPIVOT, "missing diagonal in row " + std::to_string(i));
    const T piv = U.v[udiag[i]];
    if (absval(piv) == 0.0 || !finite(piv))
      throw Error(GS_EZEROPIVOT, "zero or non-finite pivot in row " + std::to_string(i));
    L.rp.push_back((int64_t)L.ci.size());
    U.rp.push_back((int64_t)U.ci.size());
  }
}

template <class T>
void ilut(const CSR<T>& B, double tau, int lfil, CSR<T>& L, CSR<T>& U) {
  const int64_t n = B.nrows;
  L = CSR<T>();
  U = CSR<T>();
  L.nrows = L.ncols = U.nrows = U.ncols = n;
  std::vector<T> w(n, T(0));
  std::vector<char> nz(n, 0);
  std::vector<int64_t> cols;             // columns currently nonzero in w
  std::vector<int64_t> udiag(n);
  std::priority_queue<int64_t, std::vector<int64_t>, std::greater<int64_t>> heap;
  std::vector<std::pair<int64_t, T>> lpart, upart;
  for (int64_t i = 0; i < n; ++i) {
    double nrm2 = 0.0;
    cols.clear();
    for (int64_t p = B.rp[i]; p < B.rp[i + 1]; ++p) {
      const int64_t c = B.ci[p];
      const double a = absval(B.v[p]);
      nrm2 = nrm2 + a * a;
      w[c] = B.v[p];
      nz[c] = 1;
      cols.push_back(c);
      if (c < i) heap.push(c);
    }
    const double tau_i = tau * std::sqrt(nrm2);
    while (!heap.empty()) {
      const int64_t k = heap.top();
      heap.pop();
      const T wk = w[k] / U.v[udiag[k]];
      if (absval(wk) < tau_i) {  // multiplier dropped
        w[k] = T(0);
        nz[k] = 0;
        continue;
      }
      w[k] = wk;
      for (int64_t q = U.rp[k]; q < U.rp[k + 1]; ++q) {
        const int64_t j = U.ci[q];
        if (j <= k) continue;
        if (nz[j]) {
          w[j] = w[j] - wk * U.v[q];
        } else {
          w[j] = -(wk * U.v[q]);
          nz[j] = 1;
          cols.push_back(j);
          if (j < i) heap.push(j);
        }
      }
    }
    lpart.clear();
    upart.clear();
    T diag = T(0);
    bool hasdiag = false;
    for (int64_t c : cols) {
      if (!nz[c]) continue;
      if (c == i) { diag = w[c]; hasdiag = true; }
      else if (absval(w[c]) >= tau_i) {
        if (c < i) lpart.push_back({c, w[c]});
        else upart.push_back({c, w[c]});
      }
      w[c] = T(0);
      nz[c] = 0;
    }
    auto keep = [lfil](std::vector<std::pair<int64_t, T>>& part) {
      if ((int64_t)part.size() > lfil) {
        std::sort(part.begin(), part.end(), [](const auto& x, const auto& y) {
          const double ax = absval(x.second), ay = absval(y.second);
          return ax > ay || (ax == ay && x.first < y.first);
        });
        part.resize(lfil);
      }
      std::sort(part.begin(), part.end(),
                [](const auto& x, const auto& y) { return x.first < y.first; });
    };
    keep(lpart);
    keep(upart);
    if (!hasdiag || absval(diag) == 0.0 || !finite(diag))
      throw Error(GS_EZEROPIVOT, "zero or non-finite pivot in row " + std::to_string(i));
    for (auto& e : lpart) { L.ci.push_back((int32_t)e.first); L.v.push_back(e.second); }
    udiag[i] = (int64_t)U.v.size();
    U.ci.push_back((int32_t)i);
    U.v.push_back(diag);
    for (auto& e : upart) { U.ci.push_back((int32_t)e.first); U.v.push_back(e.second); }
    L.rp.push_back((int64_t)L.ci.size());
    U.rp.push_back((int64_t)U.ci.size());
  }
}

// Factor every diagonal block of every level on `nthreads` host threads.
template <class T>
void factor_levels(HostSetup<T>& S, int kind, double tau, int lfil,
                   int nthreads, T shift) {
  struct Job { int l; int64_t b; };
  std::vector<Job> jobs;
  for (int l = 0; l <= S.L(); ++l)
    for (size_t b = 0; b + 1 < S.lv[l].blocks.size(); ++b) jobs.push_back({l, (int64_t)b});
  // largest blocks first for balance
  std::sort(jobs.begin(), jobs.end(), [&](const Job& x, const Job& y) {
    auto sz = [&](const Job& j) { return S.lv[j.l].blocks[j.b + 1] - S.lv[j.l].blocks[j.b]; };
    return sz(x) > sz(y);
  });
  // per-block results
  std::vector<std::vector<CSR<T>>> Lb(S.L() + 1), Ub(S.L() + 1);
  for (int l = 0; l <= S.L(); ++l) {
    Lb[l].resize(S.lv[l].blocks.size() - 1);
    Ub[l].resize(S.lv[l].blocks.size() - 1);
  }
  std::atomic<size_t> next{0};
  std::atomic<int> err_code{0};
  std::string err_msg;
  std::mutex err_mu;
  auto worker = [&]() {
    for (;;) {
      size_t t = next.fetch_add(1);
      if (t >= jobs.size() || err_code.load()) return;
      const Job& jb = jobs[t];
      const HostLevel<T>& lv = S.lv[jb.l];
      const CSR<T>& B = lv.L;  // holds B until factor_levels replaces it
      const int64_t r0 = lv.blocks[jb.b], r1 = lv.blocks[jb.b + 1];
      CSR<T> blk;
      blk.nrows = blk.ncols = r1 - r0;
      for (int64_t i = r0; i < r1; ++i) {
        for (int64_t p = B.rp[i]; p < B.rp[i + 1]; ++p) {
          int64_t c = B.ci[p];
          if (c < r0 || c >= r1) continue;  // cannot happen for components
          blk.ci.push_back((int32_t)(c - r0));
          blk.v.push_back(c == i ? B.v[p] + shift : B.v[p]);
        }
        blk.rp.push_back((int64_t)blk.ci.size());
      }
      try {
        if (kind == GS_ILU0) ilu0(blk, Lb[jb.l][jb.b], Ub[jb.l][jb.b]);
        else ilut(blk, tau, lfil, Lb[jb.l][jb.b], Ub[jb.l][jb.b]);
      } catch (const Error& e) {
        std::lock_guard<std::mutex> g(err_mu);
        if (!err_code.load()) {
          err_msg = "level " + std::to_string(jb.l) + " block " + std::to_string(jb.b) + ": " + e.what();
          err_code.store(e.code);
        }
        return;
      }
    }
  };
  int nt = nthreads > 0 ? nthreads : (int)std::thread::hardware_concurrency();
  nt = std::max(1, std::min<int>(nt, (int)jobs.size()));
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(worker);
  for (auto& x : th) x.join();
  if (err_code.load()) throw Error(err_code.load(), err_msg);
  // stitch blocks back into level-local CSRs
  for (int l = 0; l <= S.L(); ++l) {
    HostLevel<T>& lv = S.lv[l];
    CSR<T> Lf, Uf;
    Lf.nrows = Lf.ncols = Uf.nrows = Uf.ncols = lv.d;
    for (size_t b = 0; b + 1 < lv.blocks.size(); ++b) {
      const int64_t r0 = lv.blocks[b];
      auto app = [r0](CSR<T>& dst, const CSR<T>& src) {
        for (int64_t i = 0; i < src.nrows; ++i) {
          for (int64_t p = src.rp[i]; p < src.rp[i + 1]; ++p) {
            dst.ci.push_back((int32_t)(src.ci[p] + r0));
            dst.v.push_back(src.v[p]);
          }
          dst.rp.push_back((int64_t)dst.ci.size());
        }
      };
      app(Lf, Lb[l][b]);
      app(Uf, Ub[l][b]);
    }
    lv.L = std::move(Lf);
    lv.U = std::move(Uf);
  }
}

void start_vector(uint64_t seed, int64_t n, double* v) {
  const uint64_t gamma = 0x9E3779B97F4A7C15ULL;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t z = seed + (uint64_t)(i + 1) * gamma;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    const double u = (double)(z >> 11) * 0x1.0p-53;
    v[i] = 2.0 * u - 1.0;
  }
}

template CSR<double> permute<double>(const CSR<double>&, const std::vector<int64_t>&);
template CSR<cplx> permute<cplx>(const CSR<cplx>&, const std::vector<int64_t>&);
template void extract_levels<double>(const CSR<double>&, const Partition&, HostSetup<double>&);
template void extract_levels<cplx>(const CSR<cplx>&, const Partition&, HostSetup<cplx>&);
template void factor_levels<double>(HostSetup<double>&, int, double, int, int, double);
template void factor_levels<cplx>(HostSetup<cplx>&, int, double, int, int, cplx);
template void ilu0<double>(const CSR<double>&, CSR<double>&, CSR<double>&);
template void ilu0<cplx>(const CSR<cplx>&, CSR<cplx>&, CSR<cplx>&);
template void ilut<double>(const CSR<double>&, double, int, CSR<double>&, CSR<double>&);
template void ilut<cplx>(const CSR<cplx>&, double, int, CSR<cplx>&, CSR<cplx>&);

}  // namespace gs

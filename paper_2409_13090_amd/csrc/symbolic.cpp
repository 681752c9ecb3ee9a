// Host symbolic phase of RLB supernodal Cholesky.
//
// Steps (each bit-exact with the CPU oracle's naive analysis):
//   1. fill-reducing ordering: geometric nested dissection on the grid box
//      (the paper uses METIS nested dissection, Section 3.1), natural or user;
//   2. elimination tree (parent p(j) = min(glbind(j) \ {j}), Section 2.1.2)
//      by Liu's path-compressed ancestor walk, then a postorder renumbering so
//      supernodes are runs of consecutive columns;
//   3. column counts by row-subtree traversal; fundamental supernodes
//      (j and p(j) together iff glbind(j)\{j} = glbind(p(j)) and j is p(j)'s
//      only child, Section 2.1.2);
//   4. supernode merging in the manner of Section 3.1: greedily merge the
//      child/parent pair that creates the least new fill (a heap), stopping
//      before the cumulative storage growth exceeds the cap (12.5 percent);
//   5. partition-refinement reordering inside every supernode (Section 1,
//      Fig. 2; Section 3.1) so that descendants' rows form fewer blocks;
//   6. glbind(J), relind(J, p(J)) (Section 2.1.2), blocks and relindB(J, P)
//      obtained by composition relindB(J,C) o relind(C,P) (Alg. 5).
#include "symbolic.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>
#include <tuple>

namespace rlb {

namespace {

constexpr int ERR_ARG = -1;
constexpr int ERR_PATTERN = -2;

// --- orderings --------------------------------------------------------------

void nd_emit(int64_t nx, int64_t ny, int64_t dofs, int64_t x0, int64_t x1, int64_t y0,
             int64_t y1, int64_t z0, int64_t z1, std::vector<int64_t>& out) {
  for (int64_t z = z0; z < z1; ++z)
    for (int64_t y = y0; y < y1; ++y)
      for (int64_t x = x0; x < x1; ++x) {
        int64_t node = x + nx * (y + ny * z);
        for (int64_t d = 0; d < dofs; ++d) out.push_back(node * dofs + d);
      }
}

void nd_rec(int64_t nx, int64_t ny, int64_t dofs, int64_t x0, int64_t x1, int64_t y0,
            int64_t y1, int64_t z0, int64_t z1, std::vector<int64_t>& out) {
  int64_t ex = x1 - x0, ey = y1 - y0, ez = z1 - z0;
  if (ex <= 0 || ey <= 0 || ez <= 0) return;
  int64_t big = std::max(ex, std::max(ey, ez));
  if (big <= 2) {
    nd_emit(nx, ny, dofs, x0, x1, y0, y1, z0, z1, out);
    return;
  }
  if (ex == big) {
    int64_t m = x0 + ex / 2;
    nd_rec(nx, ny, dofs, x0, m, y0, y1, z0, z1, out);
    nd_rec(nx, ny, dofs, m + 1, x1, y0, y1, z0, z1, out);
    nd_emit(nx, ny, dofs, m, m + 1, y0, y1, z0, z1, out);
  } else if (ey == big) {
    int64_t m = y0 + ey / 2;
    nd_rec(nx, ny, dofs, x0, x1, y0, m, z0, z1, out);
    nd_rec(nx, ny, dofs, x0, x1, m + 1, y1, z0, z1, out);
    nd_emit(nx, ny, dofs, x0, x1, m, m + 1, z0, z1, out);
  } else {
    int64_t m = z0 + ez / 2;
    nd_rec(nx, ny, dofs, x0, x1, y0, y1, z0, m, out);
    nd_rec(nx, ny, dofs, x0, x1, y0, y1, m + 1, z1, out);
    nd_emit(nx, ny, dofs, x0, x1, y0, y1, m, m + 1, out);
  }
}

// Graph nested dissection of the adjacency graph of A (general sparse
// input; the paper orders with METIS nested dissection, Section 3.1, which is
// not available here). A vertex set is handled one connected component at a
// time, components in the order of their smallest vertex. A component of at
// most GND_LEAF vertices is emitted in ascending order. Otherwise a
// breadth-first level structure is rooted at a pseudo-peripheral vertex
// (start at the smallest vertex; while the last level holds a vertex of
// least degree inside the component -- smallest index on ties -- whose own
// level structure is deeper, move the root there; at most 8 moves); levels
// are visited in ascending vertex order. The separator is the first level m
// (1 <= m <= depth-1) by which the levels hold at least half of the
// component; the levels before it and after it are dissected in turn (in
// that order) and the separator is emitted last, ascending. A component
// whose level structure has fewer than three levels is emitted ascending.
constexpr int64_t GND_LEAF = 8;

struct GraphND {
  const std::vector<int64_t>& ap;
  const std::vector<int32_t>& ai;
  std::vector<int32_t> mark;   // set id of each vertex
  std::vector<int32_t> lvl;    // BFS level scratch
  int32_t next_id = 1;
  std::vector<int64_t>& out;
  GraphND(const std::vector<int64_t>& ap_, const std::vector<int32_t>& ai_, int64_t n,
          std::vector<int64_t>& o)
      : ap(ap_), ai(ai_), mark(n, 0), lvl(n, -1), out(o) {}

  // breadth-first levels from r inside the set `id`; returns the levels
  std::vector<std::vector<int64_t>> levels(int64_t r, int32_t id) {
    std::vector<std::vector<int64_t>> L{{r}};
    lvl[r] = 0;
    std::vector<int64_t> touched{r};
    for (;;) {
      std::vector<int64_t> nxt;
      for (int64_t v : L.back())
        for (int64_t e = ap[v]; e < ap[v + 1]; ++e) {
          const int64_t u = ai[e];
          if (mark[u] == id && lvl[u] < 0) {
            lvl[u] = (int32_t)L.size();
            nxt.push_back(u);
            touched.push_back(u);
          }
        }
      if (nxt.empty()) break;
      std::sort(nxt.begin(), nxt.end());
      L.push_back(std::move(nxt));
    }
    for (int64_t v : touched) lvl[v] = -1;
    return L;
  }
  int64_t degree_in(int64_t v, int32_t id) const {
    int64_t d = 0;
    for (int64_t e = ap[v]; e < ap[v + 1]; ++e) d += mark[ai[e]] == id;
    return d;
  }
  // dissect the vertices of `set` (ascending) one component at a time
  void dissect_set(const std::vector<int64_t>& set) {
    if (set.empty()) return;
    const int32_t id = next_id++;
    for (int64_t v : set) mark[v] = id;
    for (int64_t v : set) {
      if (mark[v] != id) continue;  // already in an earlier component
      std::vector<std::vector<int64_t>> L = levels(v, id);
      std::vector<int64_t> comp;
      for (auto& l : L) comp.insert(comp.end(), l.begin(), l.end());
      std::sort(comp.begin(), comp.end());
      const int32_t cid = next_id++;
      for (int64_t u : comp) mark[u] = cid;
      dissect_component(comp, cid);
    }
  }
  void dissect_component(const std::vector<int64_t>& comp, int32_t id) {
    const int64_t sz = (int64_t)comp.size();
    if (sz <= GND_LEAF) {
      out.insert(out.end(), comp.begin(), comp.end());
      return;
    }
    std::vector<std::vector<int64_t>> L = levels(comp[0], id);
    for (int it = 0; it < 8; ++it) {
      int64_t u = -1, du = 0;
      for (int64_t w : L.back()) {
        const int64_t d = degree_in(w, id);
        if (u < 0 || d < du) {
          u = w;
          du = d;
        }
      }
      std::vector<std::vector<int64_t>> Lu = levels(u, id);
      if (Lu.size() <= L.size()) break;
      L = std::move(Lu);
    }
    const int64_t depth = (int64_t)L.size() - 1;
    if (depth < 2) {
      out.insert(out.end(), comp.begin(), comp.end());
      return;
    }
    int64_t m = depth - 1, cum = 0;
    for (int64_t i = 0; i <= depth - 1; ++i) {
      cum += (int64_t)L[i].size();
      if (i >= 1 && 2 * cum >= sz) {
        m = i;
        break;
      }
    }
    std::vector<int64_t> a, b;
    for (int64_t i = 0; i < m; ++i) a.insert(a.end(), L[i].begin(), L[i].end());
    for (int64_t i = m + 1; i <= depth; ++i) b.insert(b.end(), L[i].begin(), L[i].end());
    std::sort(a.begin(), a.end());
    std::sort(b.begin(), b.end());
    const std::vector<int64_t> sep = L[m];
    dissect_set(a);
    dissect_set(b);
    out.insert(out.end(), sep.begin(), sep.end());
  }
};

// --- graph helpers ------------------------------------------------------------

// Symmetric adjacency (no diagonal) of P A P^T in CSR, rows sorted.
void permuted_adjacency(int64_t n, const std::vector<int64_t>& cp,
                        const std::vector<int64_t>& ri, const std::vector<int64_t>& perm,
                        std::vector<int64_t>& ap, std::vector<int32_t>& ai) {
  std::vector<int64_t> inv(n);
  for (int64_t k = 0; k < n; ++k) inv[perm[k]] = k;
  ap.assign(n + 1, 0);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t e = cp[j]; e < cp[j + 1]; ++e) {
      int64_t i = ri[e];
      if (i == j) continue;
      ap[inv[i] + 1]++;
      ap[inv[j] + 1]++;
    }
  for (int64_t k = 0; k < n; ++k) ap[k + 1] += ap[k];
  ai.assign(ap[n], 0);
  std::vector<int64_t> fill(ap.begin(), ap.end() - 1);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t e = cp[j]; e < cp[j + 1]; ++e) {
      int64_t i = ri[e];
      if (i == j) continue;
      int64_t a = inv[i], b = inv[j];
      ai[fill[a]++] = (int32_t)b;
      ai[fill[b]++] = (int32_t)a;
    }
  for (int64_t k = 0; k < n; ++k) std::sort(ai.begin() + ap[k], ai.begin() + ap[k + 1]);
}

void etree_liu(int64_t n, const std::vector<int64_t>& ap, const std::vector<int32_t>& ai,
               std::vector<int64_t>& parent) {
  parent.assign(n, -1);
  std::vector<int64_t> anc(n, -1);
  for (int64_t j = 0; j < n; ++j) {
    for (int64_t e = ap[j]; e < ap[j + 1]; ++e) {
      int64_t r = ai[e];
      if (r >= j) break;
      while (anc[r] != -1 && anc[r] != j) {
        int64_t t = anc[r];
        anc[r] = j;
        r = t;
      }
      if (anc[r] == -1) {
        anc[r] = j;
        parent[r] = j;
      }
    }
  }
}

void postorder_of(int64_t n, const std::vector<int64_t>& parent, std::vector<int64_t>& post) {
  std::vector<int64_t> head(n, -1), next(n, -1), tail(n, -1);
  std::vector<int64_t> roots;
  for (int64_t j = 0; j < n; ++j) {  // children appended in ascending order
    int64_t p = parent[j];
    if (p < 0) {
      roots.push_back(j);
    } else if (head[p] < 0) {
      head[p] = tail[p] = j;
    } else {
      next[tail[p]] = j;
      tail[p] = j;
    }
  }
  post.clear();
  post.reserve(n);
  std::vector<std::pair<int64_t, int64_t>> stack;
  for (int64_t r : roots) {
    stack.push_back({r, head[r]});
    while (!stack.empty()) {
      auto& top = stack.back();
      if (top.second >= 0) {
        int64_t c = top.second;
        top.second = next[c];
        stack.push_back({c, head[c]});
      } else {
        post.push_back(top.first);
        stack.pop_back();
      }
    }
  }
}

// Column counts |glbind(j)| by traversing every row subtree.
void column_counts(int64_t n, const std::vector<int64_t>& ap, const std::vector<int32_t>& ai,
                   const std::vector<int64_t>& parent, std::vector<int64_t>& cc) {
  cc.assign(n, 1);
  std::vector<int64_t> mark(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    mark[i] = i;
    for (int64_t e = ap[i]; e < ap[i + 1]; ++e) {
      int64_t k = ai[e];
      if (k >= i) break;
      while (mark[k] != i) {
        mark[k] = i;
        cc[k]++;
        k = parent[k];
      }
    }
  }
}

// glbind(J) of a partition by the union rule: J's columns, A's rows below J,
// and the rows of every child supernode below J.
void supernode_structs(int64_t n, const std::vector<int64_t>& ap, const std::vector<int32_t>& ai,
                       const std::vector<int64_t>& sn_ptr, std::vector<int64_t>& gptr,
                       std::vector<int32_t>& gidx, std::vector<int64_t>& spar) {
  int64_t S = (int64_t)sn_ptr.size() - 1;
  std::vector<int64_t> snode(n);
  for (int64_t J = 0; J < S; ++J)
    for (int64_t j = sn_ptr[J]; j < sn_ptr[J + 1]; ++j) snode[j] = J;
  std::vector<std::vector<int64_t>> kids(S);
  std::vector<int64_t> mark(n, -1);
  std::vector<int32_t> buf;
  gptr.assign(S + 1, 0);
  gidx.clear();
  spar.assign(S, -1);
  for (int64_t J = 0; J < S; ++J) {
    int64_t f = sn_ptr[J], l = sn_ptr[J + 1] - 1;
    buf.clear();
    for (int64_t j = f; j <= l; ++j) {
      for (int64_t e = ap[j]; e < ap[j + 1]; ++e) {
        int64_t i = ai[e];
        if (i > l && mark[i] != J) {
          mark[i] = J;
          buf.push_back((int32_t)i);
        }
      }
    }
    for (int64_t C : kids[J]) {
      for (int64_t q = gptr[C]; q < gptr[C + 1]; ++q) {
        int64_t i = gidx[q];
        if (i > l && mark[i] != J) {
          mark[i] = J;
          buf.push_back((int32_t)i);
        }
      }
    }
    std::sort(buf.begin(), buf.end());
    for (int64_t j = f; j <= l; ++j) gidx.push_back((int32_t)j);
    gidx.insert(gidx.end(), buf.begin(), buf.end());
    gptr[J + 1] = (int64_t)gidx.size();
    if (!buf.empty()) {
      spar[J] = snode[buf[0]];
      kids[spar[J]].push_back(J);
    }
  }
}

// --- merging (Section 3.1) ----------------------------------------------------

void merge_supernodes(int64_t n, const std::vector<int64_t>& fund_ptr,
                      const std::vector<int64_t>& fgptr, const std::vector<int64_t>& fpar,
                      double cap, std::vector<int64_t>& sn_ptr, int64_t& added_out,
                      int64_t& base_out) {
  int64_t S = (int64_t)fund_ptr.size() - 1;
  std::vector<int64_t> first(S), last(S), w(S), m(S), par(fpar), into(S), version(S, 0);
  std::vector<char> alive(S, 1);
  std::vector<int64_t> slot_of_last(n, -1);
  int64_t base = 0;
  for (int64_t J = 0; J < S; ++J) {
    first[J] = fund_ptr[J];
    last[J] = fund_ptr[J + 1] - 1;
    w[J] = last[J] - first[J] + 1;
    m[J] = fgptr[J + 1] - fgptr[J];
    into[J] = J;
    slot_of_last[last[J]] = J;
    base += m[J] * w[J] - w[J] * (w[J] - 1) / 2;
  }
  std::function<int64_t(int64_t)> find = [&](int64_t s) {
    int64_t r = s;
    while (into[r] != r) r = into[r];
    while (into[s] != r) {
      int64_t t = into[s];
      into[s] = r;
      s = t;
    }
    return r;
  };
  auto cur_parent = [&](int64_t X) -> int64_t { return par[X] < 0 ? -1 : find(par[X]); };
  typedef std::tuple<int64_t, int64_t, int64_t, int64_t> Ent;  // cost, first, slot, version
  std::priority_queue<Ent, std::vector<Ent>, std::greater<Ent>> heap;
  auto push = [&](int64_t X) {
    version[X]++;
    if (!alive[X]) return;
    int64_t P = cur_parent(X);
    if (P < 0 || last[X] + 1 != first[P]) return;
    int64_t cost = w[X] * (w[X] + m[P] - m[X]);
    heap.push(Ent(cost, first[X], X, version[X]));
  };
  for (int64_t J = 0; J < S; ++J) push(J);
  int64_t added = 0;
  while (!heap.empty()) {
    Ent e = heap.top();
    heap.pop();
    int64_t cost = std::get<0>(e), J = std::get<2>(e);
    if (!alive[J] || std::get<3>(e) != version[J]) continue;
    if ((double)(added + cost) > cap * (double)base) break;
    int64_t P = cur_parent(J);
    added += cost;
    // J absorbs P; the merged supernode keeps J's slot
    int64_t wP = w[P];
    last[J] = last[P];
    w[J] = last[J] - first[J] + 1;
    m[J] = (w[J] - wP) + m[P];
    par[J] = par[P];
    alive[P] = 0;
    version[P]++;
    into[P] = J;
    slot_of_last[last[J]] = J;
    push(J);
    if (first[J] > 0) {
      int64_t C = slot_of_last[first[J] - 1];
      if (C >= 0 && alive[C] && cur_parent(C) == J) push(C);
    }
  }
  sn_ptr.clear();
  for (int64_t J = 0; J < S; ++J)
    if (alive[J]) sn_ptr.push_back(first[J]);
  sn_ptr.push_back(n);
  added_out = added;
  base_out = base;
}

// --- partition refinement inside one supernode (Section 1, Fig. 2) ----------

int64_t count_runs(const std::vector<int32_t>& R, const std::vector<int64_t>& pos,
                   std::vector<int64_t>& tmp) {
  tmp.clear();
  for (int32_t c : R) tmp.push_back(pos[c]);
  std::sort(tmp.begin(), tmp.end());
  int64_t runs = tmp.empty() ? 0 : 1;
  for (size_t k = 1; k < tmp.size(); ++k)
    if (tmp[k] != tmp[k - 1] + 1) runs++;
  return runs;
}

// cols: the supernode's columns in current order (consecutive integers f..l).
// sets: the column sets R_J of the touching descendants, ascending J.
void refine(int64_t f, int64_t w, const std::vector<std::vector<int32_t>>& sets,
            std::vector<int64_t>& order, std::vector<int64_t>& inR_stamp,
            std::vector<int64_t>& pos_scratch) {
  order.resize(w);
  for (int64_t k = 0; k < w; ++k) order[k] = f + k;
  std::vector<int64_t> pstart{0}, pend{w};  // parts as ranges of `order`
  std::vector<int64_t> new_order, ns, ne, a, b;
  int64_t stamp = inR_stamp.empty() ? 0 : 0;
  static int64_t global_stamp = 0;
  for (const auto& R : sets) {
    stamp = ++global_stamp;
    for (int32_t c : R) inR_stamp[c - f] = stamp;
    int64_t np = (int64_t)pstart.size();
    // which parts meet R
    std::vector<char> meets(np, 0);
    for (int64_t p = 0; p < np; ++p)
      for (int64_t q = pstart[p]; q < pend[p]; ++q)
        if (inR_stamp[order[q] - f] == stamp) {
          meets[p] = 1;
          break;
        }
    new_order.clear();
    ns.clear();
    ne.clear();
    for (int64_t p = 0; p < np; ++p) {
      a.clear();
      b.clear();
      for (int64_t q = pstart[p]; q < pend[p]; ++q) {
        if (inR_stamp[order[q] - f] == stamp)
          a.push_back(order[q]);
        else
          b.push_back(order[q]);
      }
      if (a.empty() || b.empty()) {
        ns.push_back((int64_t)new_order.size());
        new_order.insert(new_order.end(), order.begin() + pstart[p], order.begin() + pend[p]);
        ne.push_back((int64_t)new_order.size());
        continue;
      }
      bool after = (p + 1 < np) && meets[p + 1];
      const std::vector<int64_t>& x1 = after ? b : a;
      const std::vector<int64_t>& x2 = after ? a : b;
      ns.push_back((int64_t)new_order.size());
      new_order.insert(new_order.end(), x1.begin(), x1.end());
      ne.push_back((int64_t)new_order.size());
      ns.push_back((int64_t)new_order.size());
      new_order.insert(new_order.end(), x2.begin(), x2.end());
      ne.push_back((int64_t)new_order.size());
    }
    order.swap(new_order);
    pstart.swap(ns);
    pend.swap(ne);
  }
  // keep the refined order only if it lowers the total number of runs
  std::vector<int64_t> pos_old(w), pos_new(w);
  for (int64_t k = 0; k < w; ++k) {
    pos_old[k] = k;
    pos_new[order[k] - f] = k;
  }
  int64_t r_old = 0, r_new = 0;
  std::vector<int32_t> loc;
  for (const auto& R : sets) {
    loc.clear();
    for (int32_t c : R) loc.push_back(c - (int32_t)f);
    r_old += count_runs(loc, pos_old, pos_scratch);
    r_new += count_runs(loc, pos_new, pos_scratch);
  }
  if (!(r_new < r_old))
    for (int64_t k = 0; k < w; ++k) order[k] = f + k;
}

}  // namespace

int analyze(int64_t n, const int64_t* colptr, const int64_t* rowidx, const AnalyzeOptions& opt,
            Symbolic& s, std::string& err) {
  if (n < 0 || (n > 0 && (!colptr || !rowidx))) {
    err = "bad n or null pointer";
    return ERR_ARG;
  }
  if (n > (int64_t)INT32_MAX - 1) {
    err = "n too large for 32-bit row indices";
    return ERR_ARG;
  }
  s = Symbolic();
  s.n = n;
  s.opt = opt;
  if (n == 0) {
    s.sn_ptr = {0};
    s.gl_ptr = {0};
    s.rel_ptr = {0};
    s.blk_ptr = {0};
    s.rbp_ptr = {0};
    s.rbv_ptr = {0};
    s.fund_ptr = {0};
    return 0;
  }
  // validate: lower triangle incl. diagonal, rows strictly ascending
  if (colptr[0] != 0) {
    err = "colptr[0] != 0";
    return ERR_PATTERN;
  }
  for (int64_t j = 0; j < n; ++j) {
    if (colptr[j + 1] < colptr[j]) {
      err = "colptr not monotone";
      return ERR_PATTERN;
    }
    if (colptr[j + 1] == colptr[j] || rowidx[colptr[j]] != j) {
      err = "missing diagonal in column " + std::to_string(j);
      return ERR_PATTERN;
    }
    for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) {
      int64_t i = rowidx[e];
      if (i < j || i >= n) {
        err = "entry outside the lower triangle in column " + std::to_string(j);
        return ERR_PATTERN;
      }
      if (e > colptr[j] && i <= rowidx[e - 1]) {
        err = "rows not strictly ascending (unsorted or duplicate) in column " +
              std::to_string(j);
        return ERR_PATTERN;
      }
    }
  }
  s.nnz_a = colptr[n];
  s.colptr.assign(colptr, colptr + n + 1);
  s.rowidx.assign(rowidx, rowidx + s.nnz_a);

  // 1. ordering
  std::vector<int64_t>& p0 = s.perm_nd;
  if (opt.ordering == 0) {
    p0.resize(n);
    std::iota(p0.begin(), p0.end(), 0);
  } else if (opt.ordering == 1) {
    int64_t nx = opt.grid[0], ny = opt.grid[1], nz = opt.grid[2], d = opt.grid[3];
    if (nx <= 0 || ny <= 0 || nz <= 0 || d <= 0 || nx * ny * nz * d != n) {
      err = "grid dimensions do not match n";
      return ERR_ARG;
    }
    p0.reserve(n);
    nd_rec(nx, ny, d, 0, nx, 0, ny, 0, nz, p0);
  } else if (opt.ordering == 3) {
    std::vector<int64_t> ident(n), ap;
    std::iota(ident.begin(), ident.end(), 0);
    std::vector<int32_t> ai;
    permuted_adjacency(n, s.colptr, s.rowidx, ident, ap, ai);
    p0.reserve(n);
    GraphND g(ap, ai, n, p0);
    g.dissect_set(ident);
  } else if (opt.ordering == 2) {
    if (!opt.user_perm) {
      err = "user ordering without a permutation";
      return ERR_ARG;
    }
    p0.assign(opt.user_perm, opt.user_perm + n);
  } else {
    err = "unknown ordering";
    return ERR_ARG;
  }
  {
    std::vector<char> seen(n, 0);
    for (int64_t k = 0; k < n; ++k) {
      if (p0[k] < 0 || p0[k] >= n || seen[p0[k]]) {
        err = "ordering is not a permutation";
        return ERR_ARG;
      }
      seen[p0[k]] = 1;
    }
  }

  // 2. etree and postorder
  std::vector<int64_t> ap;
  std::vector<int32_t> ai;
  std::vector<int64_t> parent0, post;
  permuted_adjacency(n, s.colptr, s.rowidx, p0, ap, ai);
  etree_liu(n, ap, ai, parent0);
  postorder_of(n, parent0, post);
  s.perm_post.resize(n);
  for (int64_t k = 0; k < n; ++k) s.perm_post[k] = p0[post[k]];
  {
    std::vector<int64_t> ipost(n);
    for (int64_t k = 0; k < n; ++k) ipost[post[k]] = k;
    s.etree_post.resize(n);
    for (int64_t k = 0; k < n; ++k) {
      int64_t p = parent0[post[k]];
      s.etree_post[k] = p < 0 ? -1 : ipost[p];
    }
  }

  // 3. counts and fundamental supernodes (postorder numbering)
  permuted_adjacency(n, s.colptr, s.rowidx, s.perm_post, ap, ai);
  std::vector<int64_t> cc;
  column_counts(n, ap, ai, s.etree_post, cc);
  {
    std::vector<int64_t> nkids(n, 0);
    for (int64_t j = 0; j < n; ++j)
      if (s.etree_post[j] >= 0) nkids[s.etree_post[j]]++;
    s.fund_ptr.assign(1, 0);
    for (int64_t j = 0; j + 1 < n; ++j) {
      bool same = s.etree_post[j] == j + 1 && nkids[j + 1] == 1 && cc[j] == cc[j + 1] + 1;
      if (!same) s.fund_ptr.push_back(j + 1);
    }
    s.fund_ptr.push_back(n);
  }

  // 4. merging
  std::vector<int64_t> gptr, spar;
  std::vector<int32_t> gidx;
  supernode_structs(n, ap, ai, s.fund_ptr, gptr, gidx, spar);
  if (opt.merge_cap > 0) {
    merge_supernodes(n, s.fund_ptr, gptr, spar, opt.merge_cap, s.sn_ptr, s.merge_added,
                     s.merge_base);
  } else {
    s.sn_ptr = s.fund_ptr;
    s.merge_added = 0;
    s.merge_base = 0;
    for (int64_t j = 0; j < n; ++j) s.merge_base += cc[j];
  }
  supernode_structs(n, ap, ai, s.sn_ptr, gptr, gidx, spar);
  int64_t S = (int64_t)s.sn_ptr.size() - 1;
  std::vector<int64_t> snode(n);
  for (int64_t J = 0; J < S; ++J)
    for (int64_t j = s.sn_ptr[J]; j < s.sn_ptr[J + 1]; ++j) snode[j] = J;

  // 5. partition refinement inside every supernode
  std::vector<int64_t> pr(n);
  std::iota(pr.begin(), pr.end(), 0);
  if (opt.reorder) {
    std::vector<std::vector<std::vector<int32_t>>> touch(S);
    for (int64_t J = 0; J < S; ++J) {
      int64_t l = s.sn_ptr[J + 1] - 1;
      int64_t q = gptr[J] + (s.sn_ptr[J + 1] - s.sn_ptr[J]);
      int64_t prevP = -1;
      for (; q < gptr[J + 1]; ++q) {
        int64_t i = gidx[q];
        (void)l;
        int64_t P = snode[i];
        if (P != prevP) {
          touch[P].emplace_back();
          prevP = P;
        }
        touch[P].back().push_back((int32_t)i);
      }
    }
    std::vector<int64_t> order, stamp, scratch;
    for (int64_t P = 0; P < S; ++P) {
      int64_t f = s.sn_ptr[P], w = s.sn_ptr[P + 1] - f;
      if (touch[P].empty() || w < 2) continue;
      stamp.assign(w, 0);
      refine(f, w, touch[P], order, stamp, scratch);
      for (int64_t k = 0; k < w; ++k) pr[f + k] = order[k];
      std::vector<std::vector<int32_t>>().swap(touch[P]);
    }
  }
  s.perm.resize(n);
  std::vector<int64_t> inv_pr(n);
  for (int64_t k = 0; k < n; ++k) {
    s.perm[k] = s.perm_post[pr[k]];
    inv_pr[pr[k]] = k;
  }

  // 6. glbind(J) in the final numbering (the same sets, renumbered)
  s.gl_ptr = gptr;
  s.gl.resize(gidx.size());
  for (int64_t J = 0; J < S; ++J) {
    for (int64_t q = gptr[J]; q < gptr[J + 1]; ++q) s.gl[q] = (int32_t)inv_pr[gidx[q]];
    std::sort(s.gl.begin() + gptr[J], s.gl.begin() + gptr[J + 1]);
  }
  s.sn_parent = spar;

  // exact structure counts of the final ordering
  permuted_adjacency(n, s.colptr, s.rowidx, s.perm, ap, ai);
  etree_liu(n, ap, ai, s.etree);
  column_counts(n, ap, ai, s.etree, s.colcount);
  s.nnz_exact = 0;
  s.flops_exact = 0;
  for (int64_t j = 0; j < n; ++j) {
    s.nnz_exact += s.colcount[j];
    s.flops_exact += (double)s.colcount[j] * (double)s.colcount[j];
  }

  // relind(J, p(J)) and block sizes
  s.rel_ptr.assign(S + 1, 0);
  s.blk_ptr.assign(S + 1, 0);
  s.rel.clear();
  s.blk.clear();
  s.nnz_stored = 0;
  s.flops_padded = 0;
  for (int64_t J = 0; J < S; ++J) {
    int64_t f = s.sn_ptr[J], w = s.sn_ptr[J + 1] - f;
    int64_t m = s.gl_ptr[J + 1] - s.gl_ptr[J];
    s.nnz_stored += m * w - w * (w - 1) / 2;
    for (int64_t t = 0; t < w; ++t) s.flops_padded += (double)(m - t) * (double)(m - t);
    const int32_t* g = s.gl.data() + s.gl_ptr[J];
    int64_t P = s.sn_parent[J];
    if (P >= 0) {
      const int32_t* gp = s.gl.data() + s.gl_ptr[P];
      int64_t mP = s.gl_ptr[P + 1] - s.gl_ptr[P];
      for (int64_t q = w; q < m; ++q) {
        const int32_t* it = std::lower_bound(gp, gp + mP, g[q]);
        s.rel.push_back((int32_t)(mP - 1 - (it - gp)));
      }
    }
    for (int64_t q = w; q < m; ++q) {
      if (q > w && g[q] == g[q - 1] + 1 && snode[g[q]] == snode[g[q - 1]])
        s.blk.back()++;
      else
        s.blk.push_back(1);
    }
    s.rel_ptr[J + 1] = (int64_t)s.rel.size();
    s.blk_ptr[J + 1] = (int64_t)s.blk.size();
  }
  s.n_blocks = (int64_t)s.blk.size();

  // relindB(J, P) for every ancestor P touched, by composition along the
  // ancestor path: relindB(J, P) = relindB(J, C) o relind(C, P)
  s.rbp_ptr.assign(S + 1, 0);
  s.rbp_anc.clear();
  s.rbv_ptr.assign(1, 0);
  s.rbv.clear();
  s.n_calls = 0;
  std::vector<int32_t> cur, nxt;
  std::vector<int64_t> tops;  // global top row of each remaining block
  for (int64_t J = 0; J < S; ++J) {
    int64_t w = s.sn_ptr[J + 1] - s.sn_ptr[J];
    const int32_t* g = s.gl.data() + s.gl_ptr[J];
    int64_t nb = s.blk_ptr[J + 1] - s.blk_ptr[J];
    if (nb == 0) {
      s.rbp_ptr[J + 1] = (int64_t)s.rbp_anc.size();
      continue;
    }
    // extract relindB(J, p(J)) from relind(J, p(J)) (Alg. 5)
    cur.clear();
    tops.clear();
    int64_t q = 0;
    for (int64_t b = 0; b < nb; ++b) {
      cur.push_back(s.rel[s.rel_ptr[J] + q]);
      tops.push_back(g[w + q]);
      q += s.blk[s.blk_ptr[J] + b];
    }
    int64_t P = s.sn_parent[J], C = -1;
    size_t lo = 0;  // first block not yet consumed by an ancestor
    while (lo < tops.size()) {
      if (C >= 0) {
        // compose through relind(C, P)
        int64_t mC = s.gl_ptr[C + 1] - s.gl_ptr[C];
        int64_t wC = s.sn_ptr[C + 1] - s.sn_ptr[C];
        for (size_t b = lo; b < tops.size(); ++b) {
          int64_t posC = mC - 1 - cur[b];
          cur[b] = s.rel[s.rel_ptr[C] + (posC - wC)];
        }
      }
      size_t hi = lo;
      while (hi < tops.size() && snode[tops[hi]] == P) hi++;
      if (hi > lo) {
        s.rbp_anc.push_back((int32_t)P);
        for (size_t b = lo; b < tops.size(); ++b) s.rbv.push_back(cur[b]);
        s.rbv_ptr.push_back((int64_t)s.rbv.size());
        int64_t nbP = (int64_t)(hi - lo), rest = (int64_t)(tops.size() - lo);
        s.n_calls += nbP + (nbP * (2 * rest - nbP - 1)) / 2;  // SYRKs + block pairs below
      }
      lo = hi;
      C = P;
      P = s.sn_parent[P];
      if (P < 0 && lo < tops.size()) {
        err = "internal: rows beyond the root";
        return ERR_ARG;
      }
    }
    s.rbp_ptr[J + 1] = (int64_t)s.rbp_anc.size();
  }
  s.n_pairs = (int64_t)s.rbp_anc.size();
  return 0;
}

}  // namespace rlb

// Nested-dissection ordering of a general sparse pattern (host code).
//
// Sec. 2.2 orders the unknowns by nested dissection: the index set is bisected
// recursively, each bisection removing a separator, so that the sets form a
// tree whose leaves are the last subdomains and whose inner nodes are the
// separators (a node is eliminated after its whole subtree).  The paper takes
// the ordering from George's nested dissection; this is an automatic variant for
// patterns that come without coordinates, built on level structures:
//   - in each connected part, a pseudo-peripheral vertex is found by repeated
//     breadth-first searches (start again from a vertex of least degree in the
//     last level while the number of levels grows);
//   - the level holding the median vertex of that search becomes the
//     separator, minus its vertices with no neighbour in the next level (they
//     join the first half: the rest of the level still separates);
//   - both halves are dissected the same way until a part has at most leaf_max
//     vertices or is too shallow to split (fewer than three levels);
//   - disconnected parts become sibling subtrees (roots of a forest at the top);
//   - a separator (or an unsplittable part) of more than 4096 indices, the
//     largest node the factorization takes, becomes a chain of nodes of at most
//     that size, each the parent of the one before (a different, equally valid
//     elimination order: the ratio test of Sec. 2.2 then runs per chain node).
// Nodes are numbered in postorder (a subtree's nodes are contiguous and precede
// its root), and the indices of a node keep their original relative order.
#include <algorithm>
#include <utility>
#include <vector>

#include "hf_internal.h"

namespace hf {

namespace {

constexpr size_t MAX_NODE = 4096;  // largest node hf_analyse accepts

struct Dissector {
  const int64_t* ip;
  const int32_t* ix;
  int32_t leaf;
  std::vector<int32_t> part;   // per vertex: token of the part it was last put in
  std::vector<int32_t> seen;   // per vertex: token of the last search that reached it
  std::vector<int32_t> level;  // per vertex: level in the last search that reached it
  int32_t tokens = 0;
  std::vector<int32_t> perm, node_ptr, parent;

  int32_t mark(const std::vector<int32_t>& verts) {
    const int32_t t = ++tokens;
    for (int32_t v : verts) part[v] = t;
    return t;
  }

  // breadth-first search from s over the vertices of part p; order receives the
  // vertices in search order; returns the number of levels
  int bfs(int32_t s, int32_t p, std::vector<int32_t>& order) {
    const int32_t t = ++tokens;
    order.clear();
    order.push_back(s);
    seen[s] = t;
    level[s] = 0;
    int depth = 1;
    for (size_t h = 0; h < order.size(); ++h) {
      const int32_t v = order[h];
      for (int64_t e = ip[v]; e < ip[v + 1]; ++e) {
        const int32_t u = ix[e];
        if (part[u] == p && seen[u] != t) {
          seen[u] = t;
          level[u] = level[v] + 1;
          depth = std::max(depth, level[u] + 1);
          order.push_back(u);
        }
      }
    }
    return depth;
  }

  // a node of the given indices; a set above the library's node limit becomes a
  // chain of nodes of at most MAX_NODE indices (each the parent of the one
  // before); returns the first and the last node of the chain
  std::pair<int32_t, int32_t> emit_chain(const std::vector<int32_t>& verts) {
    std::vector<int32_t> s(verts);
    std::sort(s.begin(), s.end());
    const size_t parts = (s.size() + MAX_NODE - 1) / MAX_NODE;
    int32_t first = -1, last = -1;
    for (size_t q = 0; q < parts; ++q) {
      const size_t a = s.size() * q / parts, b = s.size() * (q + 1) / parts;
      perm.insert(perm.end(), s.begin() + a, s.begin() + b);
      node_ptr.push_back((int32_t)perm.size());
      parent.push_back(-1);
      const int32_t j = (int32_t)parent.size() - 1;
      if (last >= 0) parent[last] = j;
      if (first < 0) first = j;
      last = j;
    }
    return {first, last};
  }
  int32_t emit(const std::vector<int32_t>& verts) { return emit_chain(verts).second; }

  // roots of the subtrees covering verts, one per connected part
  std::vector<int32_t> dissect(const std::vector<int32_t>& verts) {
    std::vector<int32_t> roots;
    if (verts.empty()) return roots;
    const int32_t p = mark(verts);
    const int32_t done = ++tokens;  // seen token of vertices already given to a part
    std::vector<std::vector<int32_t>> comps;
    std::vector<int32_t> order;
    for (int32_t v : verts) {
      if (seen[v] == done) continue;
      bfs(v, p, order);
      for (int32_t u : order) seen[u] = done;
      comps.push_back(order);
    }
    for (auto& c : comps) roots.push_back(dissect_connected(c));
    return roots;
  }

  int32_t dissect_connected(const std::vector<int32_t>& comp) {
    const size_t m = comp.size();
    if ((int64_t)m <= leaf) return emit(comp);
    const int32_t p = mark(comp);
    std::vector<int32_t> order, o2;
    int32_t s = comp[0];
    int depth = bfs(s, p, order);
    for (int it = 0; it < 8; ++it) {
      int32_t best = -1;
      int64_t bdeg = INT64_MAX;
      for (int32_t v : order)
        if (level[v] == depth - 1) {
          const int64_t d = ip[v + 1] - ip[v];
          if (d < bdeg || (d == bdeg && v < best)) { bdeg = d; best = v; }
        }
      const int d2 = bfs(best, p, o2);
      if (d2 > depth) {
        depth = d2;
        s = best;
        order.swap(o2);
        continue;
      }
      depth = bfs(s, p, order);  // levels of the deepest search found
      break;
    }
    if (depth < 3) return emit(comp);  // too shallow to split
    // the level of the median vertex, kept off the first and the last level
    const int L = std::min(std::max(level[order[m / 2]], 1), depth - 2);
    const int32_t t = seen[order[0]];  // the search whose levels are current
    std::vector<int32_t> a, b, sep;
    for (int32_t v : order) {
      if (level[v] < L) {
        a.push_back(v);
      } else if (level[v] > L) {
        b.push_back(v);
      } else {
        bool touches_next = false;
        for (int64_t e = ip[v]; e < ip[v + 1] && !touches_next; ++e) {
          const int32_t u = ix[e];
          touches_next = seen[u] == t && level[u] == L + 1;
        }
        (touches_next ? sep : a).push_back(v);
      }
    }
    if (a.empty() || b.empty() || sep.empty()) return emit(comp);
    const std::vector<int32_t> ra = dissect(a);
    const std::vector<int32_t> rb = dissect(b);
    const std::pair<int32_t, int32_t> c = emit_chain(sep);
    for (int32_t r : ra) parent[r] = c.first;
    for (int32_t r : rb) parent[r] = c.first;
    return c.second;
  }
};

}  // namespace

int order_impl(int64_t n, const int64_t* indptr, const int32_t* indices, int32_t leaf_max, int32_t* perm,
               int32_t* n_nodes, int32_t* node_ptr, int32_t* parent) {
  if (n < 0 || leaf_max < 1 || !n_nodes || !node_ptr || (n > 0 && (!indptr || !indices || !perm || !parent)))
    return HF_ERR_ARG;
  if (n == 0) {
    *n_nodes = 0;
    node_ptr[0] = 0;
    return HF_OK;
  }
  if (n >= INT32_MAX) return HF_ERR_NOT_IMPLEMENTED;
  const int rc = validate_csr(n, indptr, indices);
  if (rc) return rc;
  try {
    Dissector d;
    d.ip = indptr;
    d.ix = indices;
    d.leaf = leaf_max;
    d.part.assign((size_t)n, 0);
    d.seen.assign((size_t)n, 0);
    d.level.assign((size_t)n, 0);
    d.node_ptr.push_back(0);
    std::vector<int32_t> all((size_t)n);
    for (int64_t i = 0; i < n; ++i) all[(size_t)i] = (int32_t)i;
    d.dissect(all);
    std::copy(d.perm.begin(), d.perm.end(), perm);
    std::copy(d.node_ptr.begin(), d.node_ptr.end(), node_ptr);
    std::copy(d.parent.begin(), d.parent.end(), parent);
    *n_nodes = (int32_t)d.parent.size();
  } catch (const std::bad_alloc&) {
    return HF_ERR_OOM;
  }
  return HF_OK;
}

}  // namespace hf

extern "C" int hf_order(int64_t n, const int64_t* indptr_host, const int32_t* indices_host, int32_t leaf_max,
                        int32_t* perm_host, int32_t* n_nodes_host, int32_t* node_ptr_host, int32_t* parent_host) {
  return hf::order_impl(n, indptr_host, indices_host, leaf_max, perm_host, n_nodes_host, node_ptr_host,
                        parent_host);
}

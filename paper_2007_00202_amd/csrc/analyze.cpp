// Host-side symbolic analysis (see analyze.hpp).
//
// Nested dissection rule (reading of Sec. 2 / Sec. 6, where the paper uses
// METIS or planar separators): a box [lo, hi) of grid nodes with at most
// leaf_max nodes is a leaf; otherwise the axis of largest extent (ties: x, y,
// z) is cut by the node plane p = lo + ext/2, leaving [lo, p) and [p+1, hi).
// Unknowns are numbered in postorder: left subtree, right subtree, separator.
// A separator is ordered by recursive bisection along its longest in-plane
// extent with ceil(ext/2) planes in the first half (Sec. 5.1, P-hat), down to
// sep_leaf nodes, natural order (x fastest) inside a leaf.
//
// Separator variant (the remark of Sec. 6 on ranks of F12/F21 at high
// frequency): a box at depth d < parallel_levels of the dissection tree is
// cut across the axis of largest extent of the whole grid instead of its
// own (while that extent is at least 3), so the top levels' separators are
// parallel planes and never cross.
#include "analyze.hpp"

#include <algorithm>
#include <functional>

namespace bfmf {

namespace {

struct Box {
  int32_t lo[3], hi[3];
};

int argmax3(const int64_t e[3]) {
  int a = 0;
  for (int d = 1; d < 3; ++d)
    if (e[d] > e[a]) a = d;  // strict: the lower axis wins ties
  return a;
}

struct FrontBuilder {
  Symbolic& s;
  std::vector<std::vector<int32_t>> kids;
  std::vector<std::vector<TreeNode>> trees;
  explicit FrontBuilder(Symbolic& sy) : s(sy) {}

  int32_t add_front(int64_t beg, bool is_leaf, std::vector<int32_t> ch, std::vector<TreeNode> tree) {
    int32_t f = (int32_t)s.sbeg.size();
    s.sbeg.push_back(beg);
    s.send.push_back((int64_t)s.perm.size());
    s.parent.push_back(-1);
    s.leaf.push_back(is_leaf ? 1 : 0);
    for (int32_t c : ch) s.parent[c] = f;
    kids.push_back(std::move(ch));
    trees.push_back(std::move(tree));
    return f;
  }

  void finish() {
    int32_t nf = (int32_t)s.sbeg.size();
    s.child_ptr.assign(nf + 1, 0);
    s.child_list.clear();
    s.sep_ptr.assign(nf + 1, 0);
    s.sep_nodes.clear();
    for (int32_t f = 0; f < nf; ++f) {
      for (int32_t c : kids[f]) s.child_list.push_back(c);
      s.child_ptr[f + 1] = (int32_t)s.child_list.size();
      for (auto& t : trees[f]) s.sep_nodes.push_back(t);
      s.sep_ptr[f + 1] = (int32_t)s.sep_nodes.size();
    }
    s.iperm.assign(s.n, -1);
    for (int64_t i = 0; i < s.n; ++i) s.iperm[s.perm[i]] = i;
  }
};

// Generic recursive bisection of a separator region.  `count` returns the
// number of unknowns of a region, `emit` appends them to perm in natural
// order, `split` halves a region.
template <class R, class C, class E, class S>
int32_t bisect(const R& r, int32_t sep_leaf, C& count, E& emit, S& split, std::vector<TreeNode>& nodes,
               int32_t& base) {
  int32_t me = (int32_t)nodes.size();
  nodes.push_back(TreeNode{base, -1, -1, -1});
  int64_t cnt = count(r);
  if (cnt <= sep_leaf) {
    emit(r);
    base += (int32_t)cnt;
    nodes[me].end = base;
    return me;
  }
  R r1, r2;
  split(r, r1, r2);
  int32_t l = bisect(r1, sep_leaf, count, emit, split, nodes, base);
  int32_t rr = bisect(r2, sep_leaf, count, emit, split, nodes, base);
  nodes[me].end = base;
  nodes[me].left = l;
  nodes[me].right = rr;
  return me;
}

}  // namespace

bool nd_grid(int32_t nx, int32_t ny, int32_t nz, int32_t leaf_max, int32_t sep_leaf, int32_t parallel_levels,
             Symbolic& s, std::string& err) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || leaf_max <= 0 || sep_leaf <= 0) {
    err = "nd_grid: dimensions and leaf sizes must be positive";
    return false;
  }
  if (parallel_levels < 0) {
    err = "nd_grid: parallel_levels must be >= 0";
    return false;
  }
  const int64_t gext[3] = {nx, ny, nz};
  const int fixed_axis = argmax3(gext);
  s = Symbolic();
  s.n = (int64_t)nx * ny * nz;
  s.perm.reserve(s.n);
  FrontBuilder fb(s);

  auto count = [](const Box& b) -> int64_t {
    int64_t v = 1;
    for (int d = 0; d < 3; ++d) v *= std::max<int64_t>(0, (int64_t)b.hi[d] - b.lo[d]);
    return v;
  };
  auto emit = [&](const Box& b) {
    for (int32_t z = b.lo[2]; z < b.hi[2]; ++z)
      for (int32_t y = b.lo[1]; y < b.hi[1]; ++y)
        for (int32_t x = b.lo[0]; x < b.hi[0]; ++x) s.perm.push_back((int64_t)x + (int64_t)nx * (y + (int64_t)ny * z));
  };
  auto split = [](const Box& b, Box& b1, Box& b2) {
    int64_t ext[3] = {b.hi[0] - b.lo[0], b.hi[1] - b.lo[1], b.hi[2] - b.lo[2]};
    int a = argmax3(ext);
    int32_t first = (int32_t)((ext[a] + 1) / 2);
    b1 = b;
    b2 = b;
    b1.hi[a] = b.lo[a] + first;
    b2.lo[a] = b.lo[a] + first;
  };

  std::function<int32_t(const Box&, int32_t)> rec = [&](const Box& b, int32_t depth) -> int32_t {
    int64_t vol = count(b);
    if (vol == 0) return -1;
    if (vol <= leaf_max) {
      int64_t beg = (int64_t)s.perm.size();
      emit(b);
      return fb.add_front(beg, true, {}, {TreeNode{0, (int32_t)vol, -1, -1}});
    }
    int64_t ext[3] = {b.hi[0] - b.lo[0], b.hi[1] - b.lo[1], b.hi[2] - b.lo[2]};
    int a = argmax3(ext);
    if (depth < parallel_levels && ext[fixed_axis] >= 3) a = fixed_axis;
    int32_t p = b.lo[a] + (int32_t)(ext[a] / 2);
    Box left = b, right = b, sep = b;
    left.hi[a] = p;
    right.lo[a] = p + 1;
    sep.lo[a] = p;
    sep.hi[a] = p + 1;
    std::vector<int32_t> ch;
    int32_t c1 = rec(left, depth + 1);
    if (c1 >= 0) ch.push_back(c1);
    int32_t c2 = rec(right, depth + 1);
    if (c2 >= 0) ch.push_back(c2);
    int64_t beg = (int64_t)s.perm.size();
    std::vector<TreeNode> nodes;
    int32_t base = 0;
    bisect(sep, sep_leaf, count, emit, split, nodes, base);
    return fb.add_front(beg, false, ch, nodes);
  };
  rec(Box{{0, 0, 0}, {nx, ny, nz}}, 0);
  fb.finish();
  return true;
}

bool nd_yee(int32_t ncell, int64_t n, const int32_t* coords, int32_t leaf_max, int32_t sep_leaf,
            Symbolic& s, std::string& err) {
  if (ncell <= 1 || n <= 0 || !coords || leaf_max <= 0 || sep_leaf <= 0) {
    err = "nd_yee: bad arguments";
    return false;
  }
  const int64_t m = 2 * (int64_t)ncell + 1;
  std::vector<int64_t> lookup((size_t)(m * m * m), -1);
  for (int64_t e = 0; e < n; ++e) {
    int64_t x = coords[3 * e], y = coords[3 * e + 1], z = coords[3 * e + 2];
    if (x < 0 || y < 0 || z < 0 || x >= m || y >= m || z >= m || ((x & 1) + (y & 1) + (z & 1)) != 1) {
      err = "nd_yee: edge coordinate out of range or not an edge";
      return false;
    }
    int64_t& slot = lookup[(z * m + y) * m + x];
    if (slot >= 0) {
      err = "nd_yee: duplicate edge coordinate";
      return false;
    }
    slot = e;
  }
  s = Symbolic();
  s.n = n;
  s.perm.reserve(n);
  FrontBuilder fb(s);
  // region in doubled coordinates, inclusive [lo, hi]
  auto count = [&](const Box& b) -> int64_t {
    int64_t c = 0;
    for (int32_t z = b.lo[2]; z <= b.hi[2]; ++z)
      for (int32_t y = b.lo[1]; y <= b.hi[1]; ++y)
        for (int32_t x = b.lo[0]; x <= b.hi[0]; ++x)
          if (lookup[((int64_t)z * m + y) * m + x] >= 0) ++c;
    return c;
  };
  auto emit = [&](const Box& b) {
    for (int32_t z = b.lo[2]; z <= b.hi[2]; ++z)
      for (int32_t y = b.lo[1]; y <= b.hi[1]; ++y)
        for (int32_t x = b.lo[0]; x <= b.hi[0]; ++x) {
          int64_t e = lookup[((int64_t)z * m + y) * m + x];
          if (e >= 0) s.perm.push_back(e);
        }
  };
  auto split = [](const Box& b, Box& b1, Box& b2) {
    int64_t ext[3] = {b.hi[0] - b.lo[0], b.hi[1] - b.lo[1], b.hi[2] - b.lo[2]};
    int a = argmax3(ext);
    int32_t cnt = (int32_t)ext[a] + 1;
    int32_t first = (cnt + 1) / 2;
    b1 = b;
    b2 = b;
    b1.hi[a] = b.lo[a] + first - 1;
    b2.lo[a] = b.lo[a] + first;
  };
  // cells [lo, hi): interior edges have doubled coordinates in [2 lo + 1, 2 hi - 1]
  auto interior = [](const Box& c) {
    Box d;
    for (int k = 0; k < 3; ++k) {
      d.lo[k] = 2 * c.lo[k] + 1;
      d.hi[k] = 2 * c.hi[k] - 1;
    }
    return d;
  };
  std::function<int32_t(const Box&)> rec = [&](const Box& c) -> int32_t {
    Box d = interior(c);
    int64_t vol = count(d);
    if (vol == 0) return -1;
    if (vol <= leaf_max) {
      int64_t beg = (int64_t)s.perm.size();
      emit(d);
      return fb.add_front(beg, true, {}, {TreeNode{0, (int32_t)vol, -1, -1}});
    }
    int64_t ext[3] = {c.hi[0] - c.lo[0], c.hi[1] - c.lo[1], c.hi[2] - c.lo[2]};
    int a = argmax3(ext);
    int32_t p = c.lo[a] + (int32_t)(ext[a] / 2);
    Box left = c, right = c;
    left.hi[a] = p;
    right.lo[a] = p;
    std::vector<int32_t> ch;
    int32_t c1 = rec(left);
    if (c1 >= 0) ch.push_back(c1);
    int32_t c2 = rec(right);
    if (c2 >= 0) ch.push_back(c2);
    Box sep = d;
    sep.lo[a] = 2 * p;
    sep.hi[a] = 2 * p;
    int64_t beg = (int64_t)s.perm.size();
    std::vector<TreeNode> nodes;
    int32_t base = 0;
    bisect(sep, sep_leaf, count, emit, split, nodes, base);
    return fb.add_front(beg, false, ch, nodes);
  };
  rec(Box{{0, 0, 0}, {ncell, ncell, ncell}});
  if ((int64_t)s.perm.size() != n) {
    err = "nd_yee: some unknowns are not interior edges of the grid";
    return false;
  }
  fb.finish();
  return true;
}

bool nd_user(int64_t n, const int64_t* perm, int32_t nfronts, const int64_t* front_ptr, const int32_t* front_parent,
             int32_t sep_leaf, Symbolic& s, std::string& err) {
  if (n <= 0 || !perm || nfronts <= 0 || !front_ptr || !front_parent || sep_leaf <= 0) {
    err = "user ordering: null array or non-positive size";
    return false;
  }
  std::vector<uint8_t> seen(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (perm[i] < 0 || perm[i] >= n || seen[perm[i]]) {
      err = "user ordering: perm is not a permutation of 0..n-1";
      return false;
    }
    seen[perm[i]] = 1;
  }
  if (front_ptr[0] != 0 || front_ptr[nfronts] != n) {
    err = "user ordering: front_ptr must start at 0 and end at n";
    return false;
  }
  for (int32_t f = 0; f < nfronts; ++f)
    if (front_ptr[f + 1] <= front_ptr[f]) {
      err = "user ordering: every front needs at least one separator unknown (front_ptr increasing)";
      return false;
    }
  // postorder: parent after child, one root (the last front), and the subtree of every front is the
  // contiguous run of fronts [first[f], f]: children in increasing order, each starting right after
  // the previous one's subtree
  if (front_parent[nfronts - 1] != -1) {
    err = "user ordering: the last front must be the root";
    return false;
  }
  std::vector<std::vector<int32_t>> kids(nfronts);
  for (int32_t f = 0; f + 1 < nfronts; ++f) {
    const int32_t p = front_parent[f];
    if (p <= f || p >= nfronts) {
      err = "user ordering: front tree not in postorder (parent must follow its child; one root)";
      return false;
    }
    kids[p].push_back(f);
  }
  std::vector<int32_t> first(nfronts);
  for (int32_t f = 0; f < nfronts; ++f) {
    int32_t next = -1;
    for (int32_t c : kids[f]) {
      if (next >= 0 && first[c] != next) {
        err = "user ordering: front tree not in postorder (subtrees interleave)";
        return false;
      }
      if (next < 0) first[f] = first[c];
      next = c + 1;
    }
    if (kids[f].empty()) first[f] = f;
    else if (next != f) {
      err = "user ordering: front tree not in postorder (a subtree does not end right before its root)";
      return false;
    }
  }
  s = Symbolic();
  s.n = n;
  s.perm.assign(perm, perm + n);
  FrontBuilder fb(s);
  for (int32_t f = 0; f < nfronts; ++f) {
    // fb.add_front takes the separator as [beg, perm.size()): perm is already whole, so set the
    // range directly afterwards
    const int32_t ns = (int32_t)(front_ptr[f + 1] - front_ptr[f]);
    fb.add_front(front_ptr[f], kids[f].empty(), kids[f], balanced_tree(ns, sep_leaf));
    s.send[f] = front_ptr[f + 1];
  }
  fb.finish();
  return true;
}

bool separator_property(const Symbolic& s, std::string& err) {
  // every index of I^u_f lies in the separator of an ancestor of f (no edge of A, and no fill,
  // between two subtrees that are not nested); in postorder g is an ancestor of f iff
  // first[g] <= f < g, first[g] being the first front of g's subtree
  const int32_t nf = s.nfronts();
  std::vector<int32_t> owner(s.n), first(nf);
  for (int32_t f = 0; f < nf; ++f) {
    for (int64_t i = s.sbeg[f]; i < s.send[f]; ++i) owner[i] = f;
    first[f] = s.child_ptr[f + 1] > s.child_ptr[f] ? first[s.child_list[s.child_ptr[f]]] : f;
  }
  for (int32_t f = 0; f < nf; ++f)
    for (int64_t t = s.iu_ptr[f]; t < s.iu_ptr[f + 1]; ++t) {
      const int32_t g = owner[s.iu[t]];
      if (!(first[g] <= f && f < g)) {
        err = "ordering: the separator property fails (front " + std::to_string(f) + " couples to front " +
              std::to_string(g) + ", which is not one of its ancestors)";
        return false;
      }
    }
  return true;
}

bool symbolic_phase(int64_t n, const int64_t* rowptr, const int32_t* colind, Symbolic& s, std::string& err) {
  if (n != s.n) {
    err = "symbolic: matrix size does not match the ordering";
    return false;
  }
  // pattern of P (A + A^T) P^T as adjacency lists in the new numbering
  std::vector<int64_t> deg(n + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
      int64_t j = colind[t];
      if (j == i) continue;
      deg[s.iperm[i] + 1]++;
      deg[s.iperm[j] + 1]++;
    }
  for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
  std::vector<int64_t> adj(deg[n]);
  std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
      int64_t j = colind[t];
      if (j == i) continue;
      int64_t a = s.iperm[i], b = s.iperm[j];
      adj[fill[a]++] = b;
      adj[fill[b]++] = a;
    }
  int32_t nf = s.nfronts();
  std::vector<int32_t> stamp(n, -1);
  s.iu_ptr.assign(nf + 1, 0);
  s.iu.clear();
  std::vector<int64_t> cand;
  for (int32_t f = 0; f < nf; ++f) {
    cand.clear();
    const int64_t e = s.send[f];
    auto take = [&](int64_t j) {
      if (j >= e && stamp[j] != f) {
        stamp[j] = f;
        cand.push_back(j);
      }
    };
    for (int64_t i = s.sbeg[f]; i < e; ++i)
      for (int64_t t = deg[i]; t < deg[i + 1]; ++t) take(adj[t]);
    for (int32_t k = s.child_ptr[f]; k < s.child_ptr[f + 1]; ++k) {
      int32_t c = s.child_list[k];
      for (int64_t t = s.iu_ptr[c]; t < s.iu_ptr[c + 1]; ++t) take(s.iu[t]);
    }
    std::sort(cand.begin(), cand.end());
    s.iu.insert(s.iu.end(), cand.begin(), cand.end());
    s.iu_ptr[f + 1] = (int64_t)s.iu.size();
  }
  if (!separator_property(s, err)) return false;
  s.map.assign(s.iu.size(), 0);
  for (int32_t f = 0; f < nf; ++f) {
    int32_t p = s.parent[f];
    if (p < 0) {
      if (s.nu(f) != 0) {
        err = "symbolic: root front has a non-empty update set (disconnected ordering?)";
        return false;
      }
      continue;
    }
    const int64_t* pu = s.iu.data() + s.iu_ptr[p];
    const int64_t pn = s.nu(p), pns = s.ns(p);
    for (int64_t t = s.iu_ptr[f]; t < s.iu_ptr[f + 1]; ++t) {
      int64_t j = s.iu[t];
      if (j >= s.sbeg[p] && j < s.send[p]) {
        s.map[t] = (int32_t)(j - s.sbeg[p]);
      } else {
        const int64_t* it = std::lower_bound(pu, pu + pn, j);
        if (it == pu + pn || *it != j) {
          err = "symbolic: child update index missing from the parent front";
          return false;
        }
        s.map[t] = (int32_t)(pns + (it - pu));
      }
    }
  }
  s.level.assign(nf, 0);
  s.nlevels = 0;
  for (int32_t f = nf - 1; f >= 0; --f) {
    int32_t p = s.parent[f];
    s.level[f] = p < 0 ? 0 : s.level[p] + 1;
    s.nlevels = std::max(s.nlevels, s.level[f] + 1);
  }
  return true;
}

std::vector<TreeNode> balanced_tree(int32_t count, int32_t leaf) {
  std::vector<TreeNode> nodes;
  if (count <= 0) return nodes;
  std::function<int32_t(int32_t, int32_t)> rec = [&](int32_t b, int32_t e) -> int32_t {
    int32_t me = (int32_t)nodes.size();
    nodes.push_back(TreeNode{b, e, -1, -1});
    if (e - b <= leaf) return me;
    int32_t mid = b + (e - b + 1) / 2;
    int32_t l = rec(b, mid);
    int32_t r = rec(mid, e);
    nodes[me].left = l;
    nodes[me].right = r;
    return me;
  };
  rec(0, count);
  return nodes;
}

}  // namespace bfmf

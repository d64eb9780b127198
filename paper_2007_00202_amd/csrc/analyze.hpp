// Host-side symbolic analysis: nested dissection, separator bisection,
// assembly tree, update index sets and extend-add maps.
//
// Paper Sec. 2 (multifrontal method, index sets I^s / I^u, extend-add),
// Sec. 5.1 (recursive separator bisection defining P-hat and the HOD-BF tree
// of F11; balanced tree on I^u), Sec. 6 (planar separators on regular grids).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace bfmf {

struct TreeNode {  // bisection tree node, preorder; beg/end relative to the front
  int32_t beg, end, left, right;
};

struct Symbolic {
  int64_t n = 0;
  std::vector<int64_t> perm, iperm;          // new -> old, old -> new
  std::vector<int64_t> sbeg, send;           // I^s range per front (postorder)
  std::vector<int32_t> parent, level;
  std::vector<int32_t> child_ptr, child_list;
  std::vector<uint8_t> leaf;
  std::vector<int32_t> sep_ptr;              // per front, into sep_nodes (TreeNode units)
  std::vector<TreeNode> sep_nodes;
  std::vector<int64_t> iu_ptr, iu;           // sorted I^u per front
  std::vector<int32_t> map;                  // at iu_ptr[f]: position in parent front
  int32_t nlevels = 0;

  int32_t nfronts() const { return (int32_t)sbeg.size(); }
  int64_t ns(int32_t f) const { return send[f] - sbeg[f]; }
  int64_t nu(int32_t f) const { return iu_ptr[f + 1] - iu_ptr[f]; }
  int64_t nfront(int32_t f) const { return ns(f) + nu(f); }
};

// Geometric nested dissection of an nx*ny*nz node grid (natural index
// x + nx*(y + ny*z)).  The boxes at the top `parallel_levels` levels of the
// tree are all cut across the grid's longest axis, so their separators are
// parallel planes (the separator variant of the Sec. 6 remark on high
// frequencies).  Returns false with a message on bad arguments.
bool nd_grid(int32_t nx, int32_t ny, int32_t nz, int32_t leaf_max, int32_t sep_leaf, int32_t parallel_levels,
             Symbolic& s, std::string& err);

// Nested dissection of the interior edges of an ncell^3 Yee grid given the
// doubled coordinates of every unknown (n rows of 3 int32).
bool nd_yee(int32_t ncell, int64_t n, const int32_t* coords, int32_t leaf_max,
            int32_t sep_leaf, Symbolic& s, std::string& err);

// Caller-supplied ordering: perm (new -> old), the separator of front f is
// [front_ptr[f], front_ptr[f+1]) of the new numbering, front_parent[f] its
// parent (-1 at the root).  The tree must be in postorder with the root last;
// each separator is bisected by halving its index range (first half ceil)
// down to sep_leaf.  Returns false with a message on a malformed ordering.
bool nd_user(int64_t n, const int64_t* perm, int32_t nfronts, const int64_t* front_ptr, const int32_t* front_parent,
             int32_t sep_leaf, Symbolic& s, std::string& err);

// Every update index of a front belongs to an ancestor's separator (the
// property nested dissection guarantees); checked by symbolic_phase once the
// update sets are known.
bool separator_property(const Symbolic& s, std::string& err);

// I^u, extend-add maps and levels from the pattern of A + A^T.
bool symbolic_phase(int64_t n, const int64_t* rowptr, const int32_t* colind, Symbolic& s,
                    std::string& err);

// Balanced bisection tree of `count` sorted indices (first half ceil), down to
// at most `leaf` per node; preorder.
std::vector<TreeNode> balanced_tree(int32_t count, int32_t leaf);

}  // namespace bfmf

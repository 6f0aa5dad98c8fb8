// Test driver: builds the BVH with the library's host builder and checks the structure the
// device traversal relies on. Compiled with g++ by tests/test_bvh_builder.py; not part of the
// product library.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../paper_2608_24109_amd/csrc/exm_internal.h"

using namespace exm;

// stats: binary nodes, binary depth, largest leaf, builder's depth, wide nodes, wide depth
extern "C" int bvh_check(const float* pos, int nV, const int* tri, int nF, int* stats) {
  HostBvh b{};
  std::string err;
  if (!build_bvh_host(pos, nV, tri, nF, &b, &err)) return 1;
  int rc = 0;
  std::vector<int> seen_node(b.n_nodes, 0), seen_tri(nF, 0);
  int max_depth = 0, max_leaf = 0;
  const int32_t kEmpty = (int32_t)0x80000000;
  struct Item {
    int32_t ref;
    int depth;
    float lo[3], hi[3];
  };
  std::vector<Item> st;
  auto push = [&](int32_t ref, int depth, const float* lo, const float* hi) {
    Item it{ref, depth, {lo[0], lo[1], lo[2]}, {hi[0], hi[1], hi[2]}};
    st.push_back(it);
  };
  const float inf[3] = {INFINITY, INFINITY, INFINITY}, ninf[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (b.root_is_leaf) {
    push(b.nodes[0].c0, 0, b.nodes[0].lo0, b.nodes[0].hi0);
    if (b.nodes[0].c1 != kEmpty) rc = rc ? rc : 2;
  } else {
    push(0, 0, ninf, inf);
  }
  while (!st.empty() && !rc) {
    Item it = st.back();
    st.pop_back();
    if (it.ref == kEmpty) continue;
    max_depth = std::max(max_depth, it.depth);
    if (it.ref >= 0) {
      if (it.ref >= b.n_nodes || seen_node[it.ref]++) { rc = 3; break; }  // out of range or revisit
      const BvhNode& n = b.nodes[it.ref];
      for (int a = 0; a < 3; ++a)  // children inside the parent's box
        if (n.lo0[a] < it.lo[a] || n.hi0[a] > it.hi[a] || n.lo1[a] < it.lo[a] || n.hi1[a] > it.hi[a]) rc = 4;
      push(n.c0, it.depth + 1, n.lo0, n.hi0);
      push(n.c1, it.depth + 1, n.lo1, n.hi1);
    } else {
      const uint32_t v = ~(uint32_t)it.ref;
      const int first = (int)(v >> 4), cnt = (int)(v & 15u);
      if (cnt < 1 || first + cnt > nF) { rc = 5; break; }
      max_leaf = std::max(max_leaf, cnt);
      for (int i = first; i < first + cnt; ++i) {
        const BvhTri& t = b.tris[i];
        if (t.id < 0 || t.id >= nF || seen_tri[t.id]++) { rc = 6; break; }
        const float* vs[3] = {t.v0, t.v1, t.v2};
        for (int k = 0; k < 3; ++k) {
          if (std::memcmp(vs[k], pos + 3 * (size_t)tri[3 * t.id + k], 12) != 0) rc = 7;
          for (int a = 0; a < 3; ++a)
            if (vs[k][a] < it.lo[a] || vs[k][a] > it.hi[a]) rc = 8;
        }
      }
    }
  }
  for (int f = 0; f < nF && !rc; ++f)
    if (seen_tri[f] != 1) rc = 9;
  for (int i = 0; i < b.n_nodes && !rc; ++i)
    if (!b.root_is_leaf && seen_node[i] != 1) rc = 10;
  if (!rc && max_depth > kMaxDepth) rc = 11;
  // the 4-wide tree: every wide node reached once from the root, each used slot's box inside the
  // box it hangs from and around its triangles, every triangle in exactly one leaf slot, empty
  // slots marked, depth <= kMaxDepth4
  std::vector<int> seen4(b.n_nodes4, 0), seen_tri4(nF, 0);
  int max_depth4 = 0;
  std::vector<Item> st4;
  if (!rc) st4.push_back(Item{0, 1, {-INFINITY, -INFINITY, -INFINITY}, {INFINITY, INFINITY, INFINITY}});
  while (!st4.empty() && !rc) {
    Item it = st4.back();
    st4.pop_back();
    if (it.ref >= 0) {
      if (it.ref >= b.n_nodes4 || seen4[it.ref]++) { rc = 12; break; }
      max_depth4 = std::max(max_depth4, it.depth);
      const BvhNode4& w = b.nodes4[it.ref];
      for (int k = 0; k < 4; ++k) {
        const float lo[3] = {w.lo_x[k], w.lo_y[k], w.lo_z[k]}, hi[3] = {w.hi_x[k], w.hi_y[k], w.hi_z[k]};
        if (w.child[k] == kEmpty) continue;
        for (int a = 0; a < 3; ++a)
          if (lo[a] < it.lo[a] || hi[a] > it.hi[a]) rc = 13;
        Item c{w.child[k], it.depth + 1, {lo[0], lo[1], lo[2]}, {hi[0], hi[1], hi[2]}};
        st4.push_back(c);
      }
    } else {
      const uint32_t v = ~(uint32_t)it.ref;
      const int first = (int)(v >> 4), cnt = (int)(v & 15u);
      if (cnt < 1 || first + cnt > nF) { rc = 14; break; }
      for (int i = first; i < first + cnt; ++i) {
        const BvhTri& t = b.tris[i];
        if (t.id < 0 || t.id >= nF || seen_tri4[t.id]++) { rc = 15; break; }
        const float* vs[3] = {t.v0, t.v1, t.v2};
        for (int k = 0; k < 3; ++k)
          for (int a = 0; a < 3; ++a)
            if (vs[k][a] < it.lo[a] || vs[k][a] > it.hi[a]) rc = 16;
      }
    }
  }
  for (int f = 0; f < nF && !rc; ++f)
    if (seen_tri4[f] != 1) rc = 17;
  for (int i = 0; i < b.n_nodes4 && !rc; ++i)
    if (seen4[i] != 1) rc = 18;
  if (!rc && (max_depth4 > kMaxDepth4 || max_depth4 != b.depth4)) rc = 19;
  stats[0] = b.n_nodes;
  stats[1] = max_depth;
  stats[2] = max_leaf;
  stats[3] = b.depth;
  stats[4] = b.n_nodes4;
  stats[5] = max_depth4;
  free_bvh_host(&b);
  return rc;
}

// Host builder of the ray-query acceleration structure: a BVH2 over the fixed triangles with
// binned SAH splits (32 bins per axis), leaves of 2 to 8 triangles, and a depth bound; then the
// 4-wide tree the traversal reads, collapsed from it two levels at a time.
//
// Depth bound: with need(N) = smallest k such that 2 * 2^k >= N, every node at depth d holds
// d + need(N) <= kMaxDepth. A node at the bound is split at the object median of its longest
// centroid axis (each child gets at most ceil(N/2) triangles, so need drops by one); leaves
// therefore sit at depth <= kMaxDepth = 24, the wide tree is at most kMaxDepth4 = 12 levels deep,
// and the traversal, which defers at most three children per wide level, never holds more than
// kStack = 37 references (with the bottom sentinel).
// Subtrees above a size threshold are built on separate threads; node slots come from an
// atomic counter and each thread partitions its own index range, so the result is
// deterministic up to node numbering, which does not change any ray query's answer.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <future>
#include <new>
#include <vector>

#include "exm_internal.h"

namespace exm {
namespace {

struct AABB {
  float lo[3], hi[3];
  void reset() {
    for (int a = 0; a < 3; ++a) {
      lo[a] = INFINITY;
      hi[a] = -INFINITY;
    }
  }
  void grow(const AABB& b) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], b.lo[a]);
      hi[a] = std::max(hi[a], b.hi[a]);
    }
  }
  void grow(const float* p) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], p[a]);
      hi[a] = std::max(hi[a], p[a]);
    }
  }
  float area() const {
    const float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    if (!(dx >= 0.f)) return 0.f;
    return 2.0f * (dx * dy + dy * dz + dz * dx);
  }
};

constexpr int kBins = 32;
constexpr int kLeafMin = 2;
constexpr int kLeafMax = 8;
constexpr int32_t kEmptyRef = (int32_t)0x80000000;

int need(int64_t n) {
  int k = 0;
  while ((int64_t)kLeafMin << k < n) ++k;
  return k;
}

struct Builder {
  const float* pos;
  const int32_t* tri;
  std::vector<AABB> box;
  std::vector<float> cen;  // [nF,3]
  std::vector<int32_t> idx;
  BvhNode* nodes = nullptr;
  std::atomic<int32_t> n_nodes{0};
  std::atomic<int32_t> max_depth{0};

  int32_t leaf_ref(int32_t first, int32_t count) { return (int32_t) ~(uint32_t)(((uint32_t)first << 4) | (uint32_t)count); }

  // returns the reference of the subtree over idx[first, first+count); fills its bounds
  int32_t build(int32_t first, int32_t count, int depth, AABB* out_box) {
    AABB bb, cb;
    bb.reset();
    cb.reset();
    for (int32_t i = first; i < first + count; ++i) {
      bb.grow(box[idx[i]]);
      cb.grow(&cen[3 * (size_t)idx[i]]);
    }
    *out_box = bb;
    int d = max_depth.load();
    while (depth > d && !max_depth.compare_exchange_weak(d, depth)) {
    }
    if (count <= kLeafMin) return leaf_ref(first, count);

    int axis = -1, split_bin = -1;
    float best_cost = INFINITY;
    const bool forced = depth + need(count) >= kMaxDepth;
    float ext[3];
    for (int a = 0; a < 3; ++a) ext[a] = cb.hi[a] - cb.lo[a];
    if (!forced) {
      for (int a = 0; a < 3; ++a) {
        if (!(ext[a] > 0.f)) continue;
        AABB bins[kBins];
        int32_t cnt[kBins] = {0};
        for (int b = 0; b < kBins; ++b) bins[b].reset();
        const float scale = kBins / ext[a];
        for (int32_t i = first; i < first + count; ++i) {
          const int32_t t = idx[i];
          int b = (int)((cen[3 * (size_t)t + a] - cb.lo[a]) * scale);
          b = std::min(kBins - 1, std::max(0, b));
          cnt[b]++;
          bins[b].grow(box[t]);
        }
        float la[kBins], ra[kBins];
        int32_t lc[kBins], rc[kBins];
        AABB acc;
        acc.reset();
        int32_t c = 0;
        for (int b = 0; b < kBins; ++b) {
          acc.grow(bins[b]);
          c += cnt[b];
          la[b] = acc.area();
          lc[b] = c;
        }
        acc.reset();
        c = 0;
        for (int b = kBins - 1; b >= 0; --b) {
          acc.grow(bins[b]);
          c += cnt[b];
          ra[b] = acc.area();
          rc[b] = c;
        }
        for (int b = 0; b < kBins - 1; ++b) {
          if (lc[b] == 0 || rc[b + 1] == 0) continue;
          const float cost = la[b] * lc[b] + ra[b + 1] * rc[b + 1];
          if (cost < best_cost) {
            best_cost = cost;
            axis = a;
            split_bin = b;
          }
        }
      }
      const float leaf_cost = bb.area() * count;
      // a wide node visit costs about two triangle tests (the any-hit leaf phase tests triangles
      // across the whole wave); swept at 1, 2 and 4 with leaves of at least 2 or 4 triangles: 2
      // took the tori's any-hit traversal 18.7 -> 18.2 ms (closest hit 2.53 -> 2.64 ms), 4 made
      // it slower (19.1 ms, 16 triangle tests per ray)
      const float trav = 2.0f * bb.area();
      if (count <= kLeafMax && (axis < 0 || leaf_cost <= trav + best_cost)) return leaf_ref(first, count);
    }
    int32_t mid;
    if (axis >= 0) {
      const float scale = kBins / ext[axis];
      const float lo = cb.lo[axis];
      int32_t* beg = idx.data() + first;
      int32_t* p = std::partition(beg, beg + count, [&](int32_t t) {
        int b = (int)((cen[3 * (size_t)t + axis] - lo) * scale);
        b = std::min(kBins - 1, std::max(0, b));
        return b <= split_bin;
      });
      mid = (int32_t)(p - idx.data());
    } else {
      // object median on the longest centroid axis (degenerate centroids: by index)
      int a = 0;
      for (int k = 1; k < 3; ++k)
        if (ext[k] > ext[a]) a = k;
      mid = first + count / 2;
      int32_t* beg = idx.data() + first;
      std::nth_element(beg, idx.data() + mid, beg + count, [&](int32_t x, int32_t y) {
        const float cx = cen[3 * (size_t)x + a], cy = cen[3 * (size_t)y + a];
        return cx < cy || (cx == cy && x < y);
      });
    }
    if (mid == first || mid == first + count) mid = first + count / 2;

    const int32_t me = n_nodes.fetch_add(1);
    AABB lb, rb;
    int32_t lref, rref;
    if (count > 200000 && depth < 4) {
      auto fut = std::async(std::launch::async, [&] { return build(first, mid - first, depth + 1, &lb); });
      rref = build(mid, first + count - mid, depth + 1, &rb);
      lref = fut.get();
    } else {
      lref = build(first, mid - first, depth + 1, &lb);
      rref = build(mid, first + count - mid, depth + 1, &rb);
    }
    BvhNode& n = nodes[me];
    std::memset(&n, 0, sizeof(n));
    for (int a = 0; a < 3; ++a) {
      n.lo0[a] = lb.lo[a];
      n.hi0[a] = lb.hi[a];
      n.lo1[a] = rb.lo[a];
      n.hi1[a] = rb.hi[a];
    }
    n.c0 = lref;
    n.c1 = rref;
    return me;
  }
};

// The 4-wide tree: each wide node holds the children of a binary node's children (a child that is
// a leaf stays one slot), so wide nodes are the binary nodes at even depths. Nodes are numbered in
// depth-first pre-order. Returns the wide depth below `n2` (1 for a node whose slots are all leaves).
struct Collapser {
  const BvhNode* n2;
  std::vector<BvhNode4> out;
  int32_t emit(int32_t b, int32_t* depth) {
    const int32_t me = (int32_t)out.size();
    out.emplace_back();
    int32_t ref[4];
    float lo[4][3], hi[4][3];
    int n = 0;
    const BvhNode& N = n2[b];
    for (int c = 0; c < 2; ++c) {
      const int32_t ci = c == 0 ? N.c0 : N.c1;
      const float* clo = c == 0 ? N.lo0 : N.lo1;
      const float* chi = c == 0 ? N.hi0 : N.hi1;
      if (ci >= 0) {
        const BvhNode& C = n2[ci];
        ref[n] = C.c0;
        std::memcpy(lo[n], C.lo0, 12);
        std::memcpy(hi[n], C.hi0, 12);
        ++n;
        ref[n] = C.c1;
        std::memcpy(lo[n], C.lo1, 12);
        std::memcpy(hi[n], C.hi1, 12);
        ++n;
      } else if (ci != kEmptyChild) {
        ref[n] = ci;
        std::memcpy(lo[n], clo, 12);
        std::memcpy(hi[n], chi, 12);
        ++n;
      }
    }
    int32_t sub = 0;
    for (int k = 0; k < n; ++k)
      if (ref[k] >= 0) {
        int32_t d = 0;
        ref[k] = emit(ref[k], &d);
        sub = std::max(sub, d);
      }
    *depth = sub + 1;
    BvhNode4& W = out[me];  // after the recursion: `out` may have grown
    std::memset(&W, 0, sizeof(W));
    for (int k = 0; k < 4; ++k) {
      const bool used = k < n;
      W.lo_x[k] = used ? lo[k][0] : INFINITY;
      W.lo_y[k] = used ? lo[k][1] : INFINITY;
      W.lo_z[k] = used ? lo[k][2] : INFINITY;
      W.hi_x[k] = used ? hi[k][0] : -INFINITY;
      W.hi_y[k] = used ? hi[k][1] : -INFINITY;
      W.hi_z[k] = used ? hi[k][2] : -INFINITY;
      W.child[k] = used ? ref[k] : kEmptyChild;
    }
    return me;
  }
};

}  // namespace

bool build_bvh_host(const float* pos, int32_t nV, const int32_t* tri, int32_t nF, HostBvh* out, std::string* err) {
  (void)nV;
  Builder B;
  B.pos = pos;
  B.tri = tri;
  B.box.resize(nF);
  B.cen.resize(3 * (size_t)nF);
  B.idx.resize(nF);
  for (int32_t f = 0; f < nF; ++f) {
    AABB b;
    b.reset();
    for (int k = 0; k < 3; ++k) b.grow(pos + 3 * (size_t)tri[3 * f + k]);
    B.box[f] = b;
    for (int a = 0; a < 3; ++a) B.cen[3 * (size_t)f + a] = 0.5f * (b.lo[a] + b.hi[a]);
    B.idx[f] = f;
  }
  const int32_t cap = std::max<int32_t>(1, nF);
  B.nodes = static_cast<BvhNode*>(::operator new[](sizeof(BvhNode) * (size_t)cap, std::align_val_t(64), std::nothrow));
  if (!B.nodes) {
    *err = "host allocation of BVH nodes failed";
    return false;
  }
  out->root_is_leaf = 0;
  AABB root_box;
  int32_t root;
  if (nF == 0) {
    root = kEmptyRef;
  } else {
    root = B.build(0, nF, 0, &root_box);
  }
  if (root < 0) {  // whole mesh in one leaf (or empty): a root node whose first child is it
    const int32_t me = B.n_nodes.fetch_add(1);
    BvhNode& n = B.nodes[me];
    std::memset(&n, 0, sizeof(n));
    if (nF > 0)
      for (int a = 0; a < 3; ++a) {
        n.lo0[a] = root_box.lo[a];
        n.hi0[a] = root_box.hi[a];
      }
    n.c0 = root;
    n.c1 = kEmptyRef;
    out->root_is_leaf = 1;
  } else if (root != 0) {
    *err = "internal: BVH root is not node 0";
    ::operator delete[](B.nodes, std::align_val_t(64));
    return false;
  }
  BvhTri* tris = static_cast<BvhTri*>(::operator new[](sizeof(BvhTri) * (size_t)std::max(1, nF), std::align_val_t(64), std::nothrow));
  if (!tris) {
    *err = "host allocation of BVH triangles failed";
    ::operator delete[](B.nodes, std::align_val_t(64));
    return false;
  }
  for (int32_t i = 0; i < nF; ++i) {
    const int32_t f = B.idx[i];
    BvhTri& t = tris[i];
    std::memset(&t, 0, sizeof(t));
    std::memcpy(t.v0, pos + 3 * (size_t)tri[3 * f], 12);
    std::memcpy(t.v1, pos + 3 * (size_t)tri[3 * f + 1], 12);
    std::memcpy(t.v2, pos + 3 * (size_t)tri[3 * f + 2], 12);
    t.id = f;
  }
  out->nodes = B.nodes;
  out->tris = tris;
  out->n_nodes = B.n_nodes.load();
  out->n_tris = nF;
  out->depth = B.max_depth.load();
  Collapser W{B.nodes, {}};
  W.out.reserve((size_t)out->n_nodes / 2 + 1);
  int32_t d4 = 0;
  W.emit(0, &d4);
  out->nodes4 = static_cast<BvhNode4*>(::operator new[](sizeof(BvhNode4) * W.out.size(), std::align_val_t(128), std::nothrow));
  if (!out->nodes4) {
    *err = "host allocation of the wide BVH nodes failed";
    ::operator delete[](B.nodes, std::align_val_t(64));
    ::operator delete[](tris, std::align_val_t(64));
    out->nodes = nullptr;
    out->tris = nullptr;
    return false;
  }
  std::memcpy(out->nodes4, W.out.data(), sizeof(BvhNode4) * W.out.size());
  out->n_nodes4 = (int32_t)W.out.size();
  out->depth4 = d4;
  return true;
}

void free_bvh_host(HostBvh* b) {
  if (b->nodes) ::operator delete[](b->nodes, std::align_val_t(64));
  if (b->nodes4) ::operator delete[](b->nodes4, std::align_val_t(128));
  if (b->tris) ::operator delete[](b->tris, std::align_val_t(64));
  b->nodes = nullptr;
  b->nodes4 = nullptr;
  b->tris = nullptr;
}

}  // namespace exm

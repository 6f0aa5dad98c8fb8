// Stage-I topology operations on the device (Vertex Splitting, Vertex Merging, UV Maintenance;
// Eq. 1-6): the per-vertex gradient EMA, face scores, and one round of concurrent splits and
// edge collapses with UV updates and index compaction.
//
// A round evaluates every criterion on the mesh as it stands at the start of the round. The
// paper skips an operation when a face it would modify was already modified in the round; with
// the operations ranked (splits by descending S_f, then merges by ascending D_f) that is the
// greedy independent set of the ranked operations under "shares a face". It is computed in
// parallel passes: every undecided operation claims its faces with atomicMin of its rank; an
// operation that holds all its faces and touches no face of an accepted one is accepted, one that
// touches such a face is rejected; repeat until none is undecided. Every pass decides at least the
// lowest-ranked undecided operation, and the result is the sequential one exactly.
//
// Readings (the same as the FP64 reference): normals, areas, lengths, projections and UV
// interpolation in FP64 from the float inputs, without contraction (this file is compiled with
// -ffp-contract=off), so that the decisions and the new coordinates match the reference bit for
// bit; "relatively large / small" faces against the mean face area; K splits with
// K = min(floor(split_fraction nF), floor((max_faces - nF) / 2)); ties to the lower face index or
// the first edge; mu = mean projection of the opposite vertices onto the edge, kept within
// [0.25, 0.75]; new faces keep the orientation of the face they replace; a merge removes the
// lower-degree endpoint (the larger index on equal degrees), keeps every corner's UV index, and
// modifies all faces around the removed vertex; unreferenced vertices and UVs are dropped.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "exm_internal.h"

namespace exm {
namespace {

constexpr int kThreads = 256;
constexpr uint64_t kEmpty = ~0ull;

enum : int32_t { kUndecided = 0, kAcceptNew = 1, kAccepted = 2, kConflict = 3, kInvalid = 4 };

// stats slots in the device counter array
enum : int32_t {
  kSplitCand = 0, kMergeCand = 1, kUndecidedLeft = 2, kSplitInvalid = 3, kSplitConflict = 4, kSplitAccepted = 5,
  kMergeConflict = 6, kMergeAccepted = 7, kFacesDeleted = 8, kNumCounters = 16
};

unsigned nblk(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

struct D3 {
  double x, y, z;
};
__device__ __forceinline__ D3 ld3(const float* p, int32_t v) {
  return D3{(double)p[3 * v], (double)p[3 * v + 1], (double)p[3 * v + 2]};
}
__device__ __forceinline__ D3 sub(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dot(D3 a, D3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }

__device__ __forceinline__ uint64_t mix64(uint64_t k) {  // splitmix64 finaliser
  k ^= k >> 30;
  k *= 0xbf58476d1ce4e5b9ull;
  k ^= k >> 27;
  k *= 0x94d049bb133111ebull;
  k ^= k >> 31;
  return k;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---- Eq. 1 and the render counts -------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_grad_ema(float* __restrict__ G, const float* __restrict__ grad,
                                                       int32_t nV, double beta) {
  const int32_t v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= nV) return;
  const double gx = grad[3 * v], gy = grad[3 * v + 1], gz = grad[3 * v + 2];
  const double nrm = sqrt((gx * gx + gy * gy) + gz * gz);
  G[v] = (float)(beta * (double)G[v] + (1.0 - beta) * nrm);
}

__global__ __launch_bounds__(kThreads) void k_face_counts(const int32_t* __restrict__ tri_id, int64_t n_px,
                                                          int32_t nF, int32_t* __restrict__ counts) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= n_px) return;
  const int32_t f = tri_id[p];
  if (f >= 0 && f < nF) atomicAdd(&counts[f], 1);
}

// ---- adjacency -------------------------------------------------------------------------------

// every face and corner index inside the current counts (flag set otherwise)
__global__ __launch_bounds__(kThreads) void k_check_indices(const int32_t* __restrict__ tri,
                                                            const int32_t* __restrict__ tri_uv, int32_t nF, int32_t nV,
                                                            int32_t nUV, int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= 3 * (int64_t)nF) return;
  const int32_t v = tri[i], u = tri_uv[i];
  if (v < 0 || v >= nV || u < 0 || u >= nUV) atomicOr(flag, 1);
}

// Edge table: open addressing over (min, max) vertex pairs; per slot up to two faces and the face
// count; the first insertion of an edge counts it in both endpoint degrees.
__global__ __launch_bounds__(kThreads) void k_edge_insert(const int32_t* __restrict__ tri, int32_t nF, uint32_t mask,
                                                          uint64_t* __restrict__ keys, int32_t* __restrict__ hface,
                                                          int32_t* __restrict__ hcnt, int32_t* __restrict__ deg,
                                                          int32_t* __restrict__ edge_slot) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= 3 * (int64_t)nF) return;
  const int32_t f = (int32_t)(i / 3), k = (int32_t)(i % 3);
  const int32_t a = tri[3 * f + k], b = tri[3 * f + (k + 1) % 3];
  const uint32_t lo = (uint32_t)min(a, b), hi = (uint32_t)max(a, b);
  const uint64_t key = ((uint64_t)lo << 32) | hi;
  uint32_t h = (uint32_t)mix64(key) & mask;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const uint64_t prev = atomicCAS((unsigned long long*)&keys[h], (unsigned long long)kEmpty,
                                    (unsigned long long)key);
    if (prev == kEmpty) {
      atomicAdd(&deg[lo], 1);
      atomicAdd(&deg[hi], 1);
      break;
    }
    if (prev == key) break;
    h = (h + 1) & mask;
  }
  const int32_t c = atomicAdd(&hcnt[h], 1);
  if (c < 2) hface[2 * h + c] = f;
  edge_slot[i] = (int32_t)h;
}

__global__ __launch_bounds__(kThreads) void k_vf_count(const int32_t* __restrict__ tri, int32_t nF,
                                                       int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < 3 * (int64_t)nF) atomicAdd(&cnt[tri[i]], 1);
}

__global__ __launch_bounds__(kThreads) void k_vf_fill(const int32_t* __restrict__ tri, int32_t nF,
                                                      const int32_t* __restrict__ off, int32_t* __restrict__ cursor,
                                                      int32_t* __restrict__ list) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= 3 * (int64_t)nF) return;
  const int32_t v = tri[i];
  list[off[v] + atomicAdd(&cursor[v], 1)] = (int32_t)(i / 3);
}

// ---- face geometry and scores (Eq. 2-4) ------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_face_geom(const float* __restrict__ pos, const int32_t* __restrict__ tri,
                                                        int32_t nF, double* __restrict__ fn, double* __restrict__ area,
                                                        double* __restrict__ ell, double* __restrict__ Dg,
                                                        double* __restrict__ part) {
  __shared__ double red[kThreads];
  const int32_t f = blockIdx.x * kThreads + threadIdx.x;
  double ar = 0.0;
  if (f < nF) {
    D3 p[3];
    for (int k = 0; k < 3; ++k) p[k] = ld3(pos, tri[3 * f + k]);
    const D3 e1 = sub(p[1], p[0]), e2 = sub(p[2], p[0]);
    const D3 c{e1.y * e2.z - e1.z * e2.y, e1.z * e2.x - e1.x * e2.z, e1.x * e2.y - e1.y * e2.x};
    const double ln = sqrt(dot(c, c));
    ar = 0.5 * ln;
    area[f] = ar;
    fn[3 * f] = ln > 0.0 ? c.x / ln : 0.0;
    fn[3 * f + 1] = ln > 0.0 ? c.y / ln : 0.0;
    fn[3 * f + 2] = ln > 0.0 ? c.z / ln : 0.0;
    double lmax = 0.0;
    for (int k = 0; k < 3; ++k) {
      const D3 d = sub(p[(k + 1) % 3], p[k]);
      const double l = sqrt(dot(d, d));
      ell[3 * f + k] = l;
      lmax = k == 0 ? l : fmax(lmax, l);
    }
    Dg[f] = lmax > 0.0 ? ar / (lmax * lmax) : 0.0;
  }
  red[threadIdx.x] = ar;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// mean face area from the per-block partial sums (one block, fixed order)
__global__ __launch_bounds__(kThreads) void k_area_mean(const double* __restrict__ part, int32_t n_part, int32_t nF,
                                                        double* __restrict__ mean) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int32_t i = threadIdx.x; i < n_part; i += kThreads) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int t = kThreads / 2; t > 0; t >>= 1) {
    if (threadIdx.x < t) red[threadIdx.x] += red[threadIdx.x + t];
    __syncthreads();
  }
  if (threadIdx.x == 0) *mean = nF > 0 ? red[0] / (double)nF : 0.0;
}

struct ScoreArgs {
  double w_g, w_k, tau_degen;
};

__global__ __launch_bounds__(kThreads) void k_face_scores(
    const int32_t* __restrict__ tri, const float* __restrict__ G, int32_t nF, const int32_t* __restrict__ edge_slot,
    const int32_t* __restrict__ hface, const int32_t* __restrict__ hcnt, const double* __restrict__ fn,
    const double* __restrict__ area, const double* __restrict__ Dg, const int32_t* __restrict__ c_rend,
    const double* __restrict__ mean, ScoreArgs sa, double* __restrict__ S, double* __restrict__ Kf,
    uint64_t* __restrict__ skey, int32_t* __restrict__ sval, uint64_t* __restrict__ mkey,
    int32_t* __restrict__ mval, int32_t* __restrict__ counters) {
  const int32_t f = blockIdx.x * kThreads + threadIdx.x;
  if (f >= nF) return;
  double s = 0.0;
  int32_t cnt = 0;
  const D3 nf{fn[3 * f], fn[3 * f + 1], fn[3 * f + 2]};
  for (int k = 0; k < 3; ++k) {
    const int32_t h = edge_slot[3 * f + k];
    if (hcnt[h] != 2) continue;
    const int32_t g = hface[2 * h] == f ? hface[2 * h + 1] : hface[2 * h];
    const double d = dot(nf, D3{fn[3 * g], fn[3 * g + 1], fn[3 * g + 2]});
    s += acos(fmin(1.0, fmax(-1.0, d)));
    ++cnt;
  }
  const double K = cnt ? s / (double)cnt : 0.0;
  const double Gf = (((double)G[tri[3 * f]] + (double)G[tri[3 * f + 1]]) + (double)G[tri[3 * f + 2]]) / 3.0;
  const double Sf = sa.w_g * Gf + sa.w_k * K;
  Kf[f] = K;
  S[f] = Sf;
  if (skey) {
    const double m = *mean;
    const bool sc = area[f] >= m;
    const bool mc = area[f] < m && ((c_rend ? c_rend[f] : 1) == 0 || Dg[f] < sa.tau_degen);
    // split candidates first in a descending sort (key = bits(S) + 1 > 0, S >= 0), merge
    // candidates first in an ascending one (key = bits(D) < ~0)
    skey[f] = sc ? (uint64_t)__double_as_longlong(Sf) + 1ull : 0ull;
    sval[f] = f;
    mkey[f] = mc ? (uint64_t)__double_as_longlong(Dg[f]) : ~0ull;
    mval[f] = f;
    if (sc) atomicAdd(&counters[kSplitCand], 1);
    if (mc) atomicAdd(&counters[kMergeCand], 1);
  }
}

// ---- the operations ----------------------------------------------------------------------------

struct SplitOp {
  int32_t f, g, a, b, c, d;
  int32_t ua, ub, uc, ua2, ub2, ud2;
  int32_t flip, n_uv;  // n_uv: 1 (shared or boundary) or 2 (seam)
  float px, py, pz, Gs;
  float u1x, u1y, u2x, u2y;
};

struct MergeOp {
  int32_t r, s;
};

struct SplitArgs {
  double tau_uv;
};

__device__ __forceinline__ int32_t edge_start(const int32_t* t, int32_t x, int32_t y) {
  for (int j = 0; j < 3; ++j)
    if (t[j] == x && t[(j + 1) % 3] == y) return j;
  return -1;
}

__global__ __launch_bounds__(kThreads) void k_split_prepare(
    const float* __restrict__ pos, const float* __restrict__ G, const float* __restrict__ uv,
    const int32_t* __restrict__ tri, const int32_t* __restrict__ tri_uv, const int32_t* __restrict__ deg,
    const int32_t* __restrict__ edge_slot, const int32_t* __restrict__ hface, const int32_t* __restrict__ hcnt,
    const double* __restrict__ ell, const int32_t* __restrict__ order, int32_t K, SplitArgs sa,
    SplitOp* __restrict__ ops, int32_t* __restrict__ op_faces, int32_t* __restrict__ op_off,
    int32_t* __restrict__ op_len, int32_t* __restrict__ state) {
  const int32_t r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= K) return;
  const int32_t f = order[r];
  int32_t k = 0;
  double best = -1.0;
  for (int kk = 0; kk < 3; ++kk) {
    const int32_t a = tri[3 * f + kk], b = tri[3 * f + (kk + 1) % 3];
    const double se = ell[3 * f + kk] / ((double)(deg[a] + deg[b]) / 2.0);
    if (se > best) {
      best = se;
      k = kk;
    }
  }
  SplitOp op;
  op.f = f;
  op.a = tri[3 * f + k];
  op.b = tri[3 * f + (k + 1) % 3];
  op.c = tri[3 * f + (k + 2) % 3];
  op.ua = tri_uv[3 * f + k];
  op.ub = tri_uv[3 * f + (k + 1) % 3];
  op.uc = tri_uv[3 * f + (k + 2) % 3];
  op.g = -1;
  op.d = op.ua2 = op.ub2 = op.ud2 = -1;
  op.flip = 0;
  op_off[r] = 2 * r;
  op_faces[2 * r] = f;
  op_faces[2 * r + 1] = -1;
  const int32_t h = edge_slot[3 * f + k];
  const int32_t cnt = hcnt[h];
  const D3 pa = ld3(pos, op.a), pb = ld3(pos, op.b);
  const D3 e = sub(pb, pa);
  double mu = 0.5;
  if (cnt > 2) {  // non-manifold edge: discarded
    op_len[r] = 1;
    state[r] = kInvalid;
    ops[r] = op;
    return;
  }
  if (cnt == 2) {
    const int32_t g = hface[2 * h] == f ? hface[2 * h + 1] : hface[2 * h];
    const int32_t* tg = tri + 3 * g;
    int32_t j = edge_start(tg, op.b, op.a);
    op.flip = j < 0;
    if (j < 0) j = edge_start(tg, op.a, op.b);
    if (j < 0) {  // the neighbour repeats a vertex: discarded
      op_len[r] = 1;
      state[r] = kInvalid;
      ops[r] = op;
      return;
    }
    op.g = g;
    op.d = tg[(j + 2) % 3];
    if (!op.flip) {
      op.ub2 = tri_uv[3 * g + j];
      op.ua2 = tri_uv[3 * g + (j + 1) % 3];
    } else {
      op.ua2 = tri_uv[3 * g + j];
      op.ub2 = tri_uv[3 * g + (j + 1) % 3];
    }
    op.ud2 = tri_uv[3 * g + (j + 2) % 3];
    const double ee = dot(e, e);
    const double lc = dot(sub(ld3(pos, op.c), pa), e) / ee;
    const double ld = dot(sub(ld3(pos, op.d), pa), e) / ee;
    mu = (lc + ld) * 0.5;
    op_faces[2 * r + 1] = g;
  }
  op_len[r] = cnt == 2 ? 2 : 1;
  const bool valid = mu >= 0.25 && mu <= 0.75;
  state[r] = valid ? kUndecided : kInvalid;
  op.px = (float)(pa.x + mu * e.x);
  op.py = (float)(pa.y + mu * e.y);
  op.pz = (float)(pa.z + mu * e.z);
  op.Gs = (float)((1.0 - mu) * (double)G[op.a] + mu * (double)G[op.b]);
  const double u1x = (1.0 - mu) * (double)uv[2 * op.ua] + mu * (double)uv[2 * op.ub];
  const double u1y = (1.0 - mu) * (double)uv[2 * op.ua + 1] + mu * (double)uv[2 * op.ub + 1];
  op.n_uv = 1;
  op.u1x = (float)u1x;
  op.u1y = (float)u1y;
  op.u2x = op.u1x;
  op.u2y = op.u1y;
  if (op.g >= 0) {
    const double u2x = (1.0 - mu) * (double)uv[2 * op.ua2] + mu * (double)uv[2 * op.ub2];
    const double u2y = (1.0 - mu) * (double)uv[2 * op.ua2 + 1] + mu * (double)uv[2 * op.ub2 + 1];
    const double dx = u1x - u2x, dy = u1y - u2y;
    if (sqrt(dx * dx + dy * dy) < sa.tau_uv) {
      op.u1x = op.u2x = (float)((u1x + u2x) * 0.5);
      op.u1y = op.u2y = (float)((u1y + u2y) * 0.5);
    } else {
      op.n_uv = 2;
      op.u2x = (float)u2x;
      op.u2y = (float)u2y;
    }
  }
  ops[r] = op;
}

__global__ __launch_bounds__(kThreads) void k_merge_prepare(
    const int32_t* __restrict__ tri, const int32_t* __restrict__ deg, const int32_t* __restrict__ edge_slot,
    const int32_t* __restrict__ hcnt, const double* __restrict__ ell, const int32_t* __restrict__ order, int32_t M,
    const int32_t* __restrict__ vf_off, const int32_t* __restrict__ vf_cnt, MergeOp* __restrict__ ops,
    int32_t* __restrict__ op_off, int32_t* __restrict__ op_len, int32_t* __restrict__ state) {
  const int32_t r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= M) return;
  const int32_t f = order[r];
  bool bnd[3];
  bool any = false;
  for (int k = 0; k < 3; ++k) {
    bnd[k] = hcnt[edge_slot[3 * f + k]] == 1;
    any |= bnd[k];
  }
  int32_t k = -1;
  for (int kk = 0; kk < 3; ++kk) {
    if (any && !bnd[kk]) continue;
    if (k < 0 || ell[3 * f + kk] < ell[3 * f + k]) k = kk;
  }
  const int32_t i = tri[3 * f + k], j = tri[3 * f + (k + 1) % 3];
  MergeOp op;
  if (deg[i] < deg[j] || (deg[i] == deg[j] && i > j)) {
    op.r = i;
    op.s = j;
  } else {
    op.r = j;
    op.s = i;
  }
  ops[r] = op;
  op_off[r] = vf_off[op.r];
  op_len[r] = vf_cnt[op.r];
  state[r] = kUndecided;
}

// ---- greedy independent set of ranked operations ---------------------------------------------

__global__ __launch_bounds__(kThreads) void k_mis_claim(int32_t n, const int32_t* __restrict__ off,
                                                        const int32_t* __restrict__ len, const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ state, int32_t* __restrict__ best) {
  const int32_t r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= n || state[r] != kUndecided) return;
  for (int32_t q = 0; q < len[r]; ++q) atomicMin(&best[list[off[r] + q]], r);
}

__global__ __launch_bounds__(kThreads) void k_mis_decide(int32_t n, const int32_t* __restrict__ off,
                                                         const int32_t* __restrict__ len,
                                                         const int32_t* __restrict__ list,
                                                         int32_t* __restrict__ state, const int32_t* __restrict__ best,
                                                         const int32_t* __restrict__ taken,
                                                         int32_t* __restrict__ counters, int32_t conflict_slot) {
  const int32_t r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= n || state[r] != kUndecided) return;
  bool owner = true, hit = false;
  for (int32_t q = 0; q < len[r]; ++q) {
    const int32_t g = list[off[r] + q];
    hit |= taken[g] != 0;
    owner &= best[g] == r;
  }
  if (hit) {
    state[r] = kConflict;
    atomicAdd(&counters[conflict_slot], 1);
  } else if (owner) {
    state[r] = kAcceptNew;
  } else {
    atomicAdd(&counters[kUndecidedLeft], 1);
  }
}

__global__ __launch_bounds__(kThreads) void k_mis_mark(int32_t n, const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ len, const int32_t* __restrict__ list,
                                                       int32_t* __restrict__ state, int32_t* __restrict__ best,
                                                       int32_t* __restrict__ taken, int32_t* __restrict__ counters,
                                                       int32_t accept_slot) {
  const int32_t r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= n) return;
  const int32_t st = state[r];
  if (st == kInvalid) return;
  const bool acc = st == kAcceptNew;
  for (int32_t q = 0; q < len[r]; ++q) {
    const int32_t g = list[off[r] + q];
    best[g] = INT_MAX;
    if (acc) taken[g] = 1;
  }
  if (acc) {
    state[r] = kAccepted;
    atomicAdd(&counters[accept_slot], 1);
  }
}

// ---- applying the accepted operations ----------------------------------------------------------

// per accepted split: 1 vertex, 1 or 2 faces, 1 or 2 UVs (three arrays of K, one scan each)
__global__ __launch_bounds__(kThreads) void k_split_counts(int32_t K, const SplitOp* __restrict__ ops,
                                                           const int32_t* __restrict__ state, int32_t* __restrict__ add) {
  const int32_t r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= K) return;
  const bool acc = state[r] == kAccepted;
  add[r] = acc ? 1 : 0;
  add[K + r] = acc ? (ops[r].g >= 0 ? 2 : 1) : 0;
  add[2 * K + r] = acc ? ops[r].n_uv : 0;
}

__global__ __launch_bounds__(kThreads) void k_split_apply(int32_t K, const SplitOp* __restrict__ ops,
                                                          const int32_t* __restrict__ state,
                                                          const int32_t* __restrict__ off, int32_t nV, int32_t nF,
                                                          int32_t nUV, float* __restrict__ pos, float* __restrict__ G,
                                                          float* __restrict__ uv, int32_t* __restrict__ tri,
                                                          int32_t* __restrict__ tri_uv) {
  const int32_t r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= K || state[r] != kAccepted) return;
  const SplitOp op = ops[r];
  const int32_t s = nV + off[r], fn = nF + off[K + r], us1 = nUV + off[2 * K + r];
  const int32_t us2 = op.n_uv == 2 ? us1 + 1 : us1;
  pos[3 * s] = op.px;
  pos[3 * s + 1] = op.py;
  pos[3 * s + 2] = op.pz;
  G[s] = op.Gs;
  uv[2 * us1] = op.u1x;
  uv[2 * us1 + 1] = op.u1y;
  if (op.n_uv == 2) {
    uv[2 * us2] = op.u2x;
    uv[2 * us2 + 1] = op.u2y;
  }
  auto put = [&](int32_t slot, int32_t x, int32_t y, int32_t z, int32_t ux, int32_t uy, int32_t uz) {
    tri[3 * slot] = x;
    tri[3 * slot + 1] = y;
    tri[3 * slot + 2] = z;
    tri_uv[3 * slot] = ux;
    tri_uv[3 * slot + 1] = uy;
    tri_uv[3 * slot + 2] = uz;
  };
  put(op.f, op.a, s, op.c, op.ua, us1, op.uc);
  put(fn, s, op.b, op.c, us1, op.ub, op.uc);
  if (op.g >= 0) {
    if (!op.flip) {
      put(op.g, op.b, s, op.d, op.ub2, us2, op.ud2);
      put(fn + 1, s, op.a, op.d, us2, op.ua2, op.ud2);
    } else {
      put(op.g, op.a, s, op.d, op.ua2, us2, op.ud2);
      put(fn + 1, s, op.b, op.d, us2, op.ub2, op.ud2);
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_merge_apply(int32_t M, const MergeOp* __restrict__ ops,
                                                          const int32_t* __restrict__ state,
                                                          const int32_t* __restrict__ vf_off,
                                                          const int32_t* __restrict__ vf_cnt,
                                                          const int32_t* __restrict__ vf_list,
                                                          int32_t* __restrict__ tri, int32_t* __restrict__ deleted,
                                                          int32_t* __restrict__ counters) {
  const int32_t r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= M || state[r] != kAccepted) return;
  const MergeOp op = ops[r];
  for (int32_t q = 0; q < vf_cnt[op.r]; ++q) {
    const int32_t g = vf_list[vf_off[op.r] + q];
    int32_t* t = tri + 3 * g;
    if (t[0] == op.s || t[1] == op.s || t[2] == op.s) {
      deleted[g] = 1;
      atomicAdd(&counters[kFacesDeleted], 1);
    } else {
      for (int k = 0; k < 3; ++k)
        if (t[k] == op.r) t[k] = op.s;
    }
  }
}

// ---- compaction -------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_mark_refs(int32_t F1, const int32_t* __restrict__ tri,
                                                        const int32_t* __restrict__ tri_uv,
                                                        const int32_t* __restrict__ deleted, int32_t* __restrict__ alive,
                                                        int32_t* __restrict__ vref, int32_t* __restrict__ uref) {
  const int32_t g = blockIdx.x * kThreads + threadIdx.x;
  if (g >= F1) return;
  const bool a = deleted[g] == 0;
  alive[g] = a;
  if (!a) return;
  for (int k = 0; k < 3; ++k) {
    vref[tri[3 * g + k]] = 1;
    uref[tri_uv[3 * g + k]] = 1;
  }
}

__global__ __launch_bounds__(kThreads) void k_compact_rows(int32_t n, int32_t width, const int32_t* __restrict__ keep,
                                                           const int32_t* __restrict__ map,
                                                           const float* __restrict__ src, float* __restrict__ dst) {
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n || !keep[i]) return;
  for (int c = 0; c < width; ++c) dst[(int64_t)map[i] * width + c] = src[(int64_t)i * width + c];
}

__global__ __launch_bounds__(kThreads) void k_compact_faces(int32_t F1, const int32_t* __restrict__ alive,
                                                            const int32_t* __restrict__ fmap,
                                                            const int32_t* __restrict__ vmap,
                                                            const int32_t* __restrict__ umap,
                                                            const int32_t* __restrict__ tri,
                                                            const int32_t* __restrict__ tri_uv,
                                                            int32_t* __restrict__ tri2, int32_t* __restrict__ tri_uv2) {
  const int32_t g = blockIdx.x * kThreads + threadIdx.x;
  if (g >= F1 || !alive[g]) return;
  const int32_t o = fmap[g];
  for (int k = 0; k < 3; ++k) {
    tri2[3 * o + k] = vmap[tri[3 * g + k]];
    tri_uv2[3 * o + k] = umap[tri_uv[3 * g + k]];
  }
}

// ---- sort and scan -----------------------------------------------------------------------------

// One compare-exchange step of a bitonic sort of n2 (a power of two) (key, value) pairs in
// ascending lexicographic order; the pairs are unique (values are face indices), so the result
// does not depend on how equal keys would be ordered.
__global__ __launch_bounds__(kThreads) void k_bitonic_step(uint64_t* __restrict__ key, int32_t* __restrict__ val,
                                                           uint32_t n2, uint32_t j, uint32_t k) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n2) return;
  const uint32_t l = i ^ j;
  if (l <= i) return;
  const uint64_t ki = key[i], kl = key[l];
  const int32_t vi = val[i], vl = val[l];
  const bool gt = ki > kl || (ki == kl && vi > vl);
  const bool up = (i & k) == 0;
  if (up == gt) {
    key[i] = kl;
    key[l] = ki;
    val[i] = vl;
    val[l] = vi;
  }
}

// keys for the sort: the ascending order of `out` is the descending order of `in` when `desc`;
// the padding sorts last
__global__ __launch_bounds__(kThreads) void k_sort_keys(const uint64_t* __restrict__ in, int32_t n, uint32_t n2,
                                                        bool desc, uint64_t* __restrict__ out,
                                                        int32_t* __restrict__ val) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n2) return;
  if ((int32_t)i < n) {
    out[i] = desc ? ~in[i] : in[i];
    val[i] = (int32_t)i;
  } else {
    out[i] = ~0ull;
    val[i] = INT_MAX;
  }
}

template <typename T>
struct ScanOps;
template <>
struct ScanOps<int32_t> {
  __device__ static int32_t zero() { return 0; }
  __device__ static int32_t add(int32_t a, int32_t b) { return a + b; }
};

// Exclusive scan in three passes: per block (256 elements) in LDS with the block total kept,
// the block totals by one block in order, and the block offsets added. Deterministic.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_block(const T* __restrict__ in, int32_t n, T* __restrict__ out,
                                                         T* __restrict__ sums) {
  __shared__ T buf[kThreads];
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  const T x = i < n ? in[i] : ScanOps<T>::zero();
  buf[threadIdx.x] = x;
  __syncthreads();
  for (int d = 1; d < kThreads; d <<= 1) {
    const T y = threadIdx.x >= d ? buf[threadIdx.x - d] : ScanOps<T>::zero();
    __syncthreads();
    buf[threadIdx.x] = ScanOps<T>::add(buf[threadIdx.x], y);
    __syncthreads();
  }
  if (i < n) out[i] = ScanOps<T>::add(buf[threadIdx.x], ScanOps<T>::zero()) - x;
  if (threadIdx.x == kThreads - 1) sums[blockIdx.x] = buf[kThreads - 1];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_sums(T* __restrict__ sums, int32_t nb) {
  __shared__ T buf[kThreads];
  T carry = ScanOps<T>::zero();
  for (int32_t base = 0; base < nb; base += kThreads) {
    const int32_t i = base + threadIdx.x;
    const T x = i < nb ? sums[i] : ScanOps<T>::zero();
    buf[threadIdx.x] = x;
    __syncthreads();
    for (int d = 1; d < kThreads; d <<= 1) {
      const T y = threadIdx.x >= d ? buf[threadIdx.x - d] : ScanOps<T>::zero();
      __syncthreads();
      buf[threadIdx.x] = ScanOps<T>::add(buf[threadIdx.x], y);
      __syncthreads();
    }
    if (i < nb) sums[i] = ScanOps<T>::add(carry, buf[threadIdx.x] - x);
    const T tot = buf[kThreads - 1];
    __syncthreads();
    carry = ScanOps<T>::add(carry, tot);
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_add(T* __restrict__ out, int32_t n, const T* __restrict__ sums) {
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i < n) out[i] = ScanOps<T>::add(out[i], sums[blockIdx.x]);
}

// ---- host side ---------------------------------------------------------------------------------

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

uint32_t table_size(int32_t nF) {
  uint64_t need = std::max<uint64_t>(64, 6ull * (uint64_t)std::max(nF, 1));
  uint64_t c = 64;
  while (c < need) c <<= 1;
  return (uint32_t)c;
}

// A bump allocator over the caller's workspace; `size_only` walks the same layout to size it.
struct Arena {
  char* base;
  size_t used = 0;
  template <typename T>
  T* take(size_t n) {
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += align256(std::max<size_t>(n, 1) * sizeof(T));
    return p;
  }
};

uint32_t pow2_at_least(int32_t n) {
  uint32_t c = 1;
  while ((int64_t)c < n) c <<= 1;
  return c;
}

struct Layout {
  // adjacency and scores
  uint64_t* hkeys;
  int32_t *hface, *hcnt, *edge_slot, *deg;
  double *fn, *area, *ell, *Dg, *S, *Kf, *part, *mean;
  uint64_t *skey, *mkey, *sort_key;
  int32_t *sval, *mval, *sval2, *mval2;
  int32_t* counters;
  // vertex -> faces
  int32_t *vf_cnt, *vf_off, *vf_cur, *vf_list;
  // operations
  SplitOp* sops;
  int32_t *s_faces, *s_off, *s_len, *s_state;
  MergeOp* mops;
  int32_t *m_off, *m_len, *m_state;
  int32_t *best, *taken, *deleted;
  int32_t *add, *add_off;
  // compaction
  int32_t *alive, *fmap, *vref, *vmap, *uref, *umap;
  float *pos2, *G2, *uv2;
  int32_t *tri2, *tri_uv2;
  int32_t* scan_sums;
  int32_t* host_words;  // device words read back at once
  size_t total;
};

Layout make_layout(char* base, int32_t nV, int32_t nF, int32_t nUV, int32_t K) {
  Arena a{base};
  Layout L;
  const uint32_t cap = table_size(nF);
  const int32_t V1 = nV + K, F1 = nF + 2 * K, U1 = nUV + 2 * K;
  L.hkeys = a.take<uint64_t>(cap);
  L.hface = a.take<int32_t>(2 * (size_t)cap);
  L.hcnt = a.take<int32_t>(cap);
  L.edge_slot = a.take<int32_t>(3 * (size_t)nF);
  L.deg = a.take<int32_t>(nV);
  L.fn = a.take<double>(3 * (size_t)nF);
  L.area = a.take<double>(nF);
  L.ell = a.take<double>(3 * (size_t)nF);
  L.Dg = a.take<double>(nF);
  L.S = a.take<double>(nF);
  L.Kf = a.take<double>(nF);
  L.part = a.take<double>(nblk(nF));
  L.mean = a.take<double>(1);
  const uint32_t n2 = pow2_at_least(nF);
  L.skey = a.take<uint64_t>(nF);
  L.mkey = a.take<uint64_t>(nF);
  L.sort_key = a.take<uint64_t>(n2);
  L.sval = a.take<int32_t>(nF);
  L.mval = a.take<int32_t>(nF);
  L.sval2 = a.take<int32_t>(n2);
  L.mval2 = a.take<int32_t>(n2);
  L.counters = a.take<int32_t>(kNumCounters);
  L.vf_cnt = a.take<int32_t>(nV);
  L.vf_off = a.take<int32_t>(nV);
  L.vf_cur = a.take<int32_t>(nV);
  L.vf_list = a.take<int32_t>(3 * (size_t)nF);
  L.sops = a.take<SplitOp>(K);
  L.s_faces = a.take<int32_t>(2 * (size_t)K);
  L.s_off = a.take<int32_t>(K);
  L.s_len = a.take<int32_t>(K);
  L.s_state = a.take<int32_t>(K);
  L.mops = a.take<MergeOp>(nF);
  L.m_off = a.take<int32_t>(nF);
  L.m_len = a.take<int32_t>(nF);
  L.m_state = a.take<int32_t>(nF);
  L.best = a.take<int32_t>(nF);
  L.taken = a.take<int32_t>(nF);
  L.deleted = a.take<int32_t>(F1);
  L.add = a.take<int32_t>(3 * (size_t)K);
  L.add_off = a.take<int32_t>(3 * (size_t)K);
  L.alive = a.take<int32_t>(F1);
  L.fmap = a.take<int32_t>(F1);
  L.vref = a.take<int32_t>(V1);
  L.vmap = a.take<int32_t>(V1);
  L.uref = a.take<int32_t>(U1);
  L.umap = a.take<int32_t>(U1);
  L.pos2 = a.take<float>(3 * (size_t)V1);
  L.G2 = a.take<float>(V1);
  L.uv2 = a.take<float>(2 * (size_t)U1);
  L.tri2 = a.take<int32_t>(3 * (size_t)F1);
  L.tri_uv2 = a.take<int32_t>(3 * (size_t)F1);
  L.scan_sums = a.take<int32_t>(nblk(std::max({F1, V1, U1, 3 * K, nV})));
  L.host_words = a.take<int32_t>(16);
  L.total = a.used;
  return L;
}

#define HIP_TRY(x)                      \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n > 0) k_fill_i32<<<nblk(n), kThreads, 0, s>>>(p, n, v);
  return hipGetLastError();
}

// exclusive scan of n ints (in and out may not alias)
hipError_t scan(const Layout& L, const int32_t* in, int32_t* out, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int32_t nb = (int32_t)nblk(n);
  k_scan_block<int32_t><<<nb, kThreads, 0, s>>>(in, n, out, L.scan_sums);
  k_scan_sums<int32_t><<<1, kThreads, 0, s>>>(L.scan_sums, nb);
  k_scan_add<int32_t><<<nb, kThreads, 0, s>>>(out, n, L.scan_sums);
  return hipGetLastError();
}

// the values (face indices) of n keys in ascending (key, index) order, into val[0, n)
hipError_t sort_faces(const Layout& L, const uint64_t* keys, int32_t n, bool desc, int32_t* val, hipStream_t s) {
  const uint32_t n2 = pow2_at_least(n);
  k_sort_keys<<<nblk(n2), kThreads, 0, s>>>(keys, n, n2, desc, L.sort_key, val);
  for (uint32_t k = 2; k <= n2; k <<= 1)
    for (uint32_t j = k >> 1; j > 0; j >>= 1) k_bitonic_step<<<nblk(n2), kThreads, 0, s>>>(L.sort_key, val, n2, j, k);
  return hipGetLastError();
}

hipError_t read_words(const int32_t* dev, int32_t* host, int n, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(host, dev, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  return hipStreamSynchronize(s);
}

// adjacency, geometry and scores of the current mesh
hipError_t scores_pass(const Layout& L, const exm_topo_mesh* m, const int32_t* c_rend, const exm_topo_params* p,
                       bool keys, hipStream_t s) {
  const int32_t nV = m->nV, nF = m->nF;
  const uint32_t cap = table_size(nF);
  k_fill_u64<<<nblk(cap), kThreads, 0, s>>>(L.hkeys, cap, kEmpty);
  HIP_TRY(fill_i32(L.hcnt, cap, 0, s));
  HIP_TRY(fill_i32(L.deg, nV, 0, s));
  HIP_TRY(fill_i32(L.counters, kNumCounters, 0, s));
  if (nF == 0) return hipGetLastError();
  k_edge_insert<<<nblk(3 * (int64_t)nF), kThreads, 0, s>>>(m->tri, nF, cap - 1, L.hkeys, L.hface, L.hcnt, L.deg,
                                                           L.edge_slot);
  k_face_geom<<<nblk(nF), kThreads, 0, s>>>(m->pos, m->tri, nF, L.fn, L.area, L.ell, L.Dg, L.part);
  k_area_mean<<<1, kThreads, 0, s>>>(L.part, (int32_t)nblk(nF), nF, L.mean);
  ScoreArgs sa{p->w_g, p->w_k, p->tau_degen};
  k_face_scores<<<nblk(nF), kThreads, 0, s>>>(m->tri, m->G, nF, L.edge_slot, L.hface, L.hcnt, L.fn, L.area, L.Dg,
                                              c_rend, L.mean, sa, L.S, L.Kf, keys ? L.skey : nullptr, L.sval, L.mkey,
                                              L.mval, L.counters);
  return hipGetLastError();
}

// Greedy independent set of n ranked operations over faces; `taken` carries over between calls.
hipError_t mis(const Layout& L, int32_t n, const int32_t* off, const int32_t* len, const int32_t* list,
               int32_t* state, int32_t conflict_slot, int32_t accept_slot, int32_t* host, int32_t* iters,
               hipStream_t s) {
  for (int32_t it = 0; it <= n && n > 0; ++it) {
    ++*iters;
    HIP_TRY(fill_i32(L.counters + kUndecidedLeft, 1, 0, s));
    k_mis_claim<<<nblk(n), kThreads, 0, s>>>(n, off, len, list, state, L.best);
    k_mis_decide<<<nblk(n), kThreads, 0, s>>>(n, off, len, list, state, L.best, L.taken, L.counters, conflict_slot);
    k_mis_mark<<<nblk(n), kThreads, 0, s>>>(n, off, len, list, state, L.best, L.taken, L.counters, accept_slot);
    HIP_TRY(hipGetLastError());
    HIP_TRY(read_words(L.counters + kUndecidedLeft, host, 1, s));
    if (host[0] == 0) return hipSuccess;
  }
  return hipSuccess;
}

template <typename T>
hipError_t copy_back(T* dst, const T* src, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, s);
}

}  // namespace

int32_t topology_split_count(int32_t nF, const exm_topo_params* p) {
  if (p->flags & EXM_TOPO_NO_SPLIT) return 0;
  const int64_t by_frac = (int64_t)std::floor(p->split_fraction * (double)nF);
  const int64_t room = (int64_t)p->max_faces - nF;
  const int64_t by_budget = room > 0 ? room / 2 : 0;
  return (int32_t)std::max<int64_t>(0, std::min(by_frac, by_budget));
}

size_t topology_ws_bytes(int32_t nV, int32_t nF, int32_t nUV, const exm_topo_params* p) {
  return make_layout(nullptr, nV, nF, nUV, topology_split_count(nF, p)).total;
}

hipError_t topology_check_indices(const exm_topo_mesh* m, void* ws, bool* ok, hipStream_t s) {
  *ok = true;
  if (m->nF == 0) return hipSuccess;
  int32_t* flag = static_cast<int32_t*>(ws);  // the first word of the workspace, before a pass uses it
  HIP_TRY(fill_i32(flag, 1, 0, s));
  k_check_indices<<<nblk(3 * (int64_t)m->nF), kThreads, 0, s>>>(m->tri, m->tri_uv, m->nF, m->nV, m->nUV, flag);
  HIP_TRY(hipGetLastError());
  int32_t h = 0;
  HIP_TRY(read_words(flag, &h, 1, s));
  *ok = h == 0;
  return hipSuccess;
}

hipError_t launch_grad_ema(float* G, const float* grad, int32_t nV, double beta, hipStream_t s) {
  EXM_TIMED("grad_ema", s);
  k_grad_ema<<<nblk(nV), kThreads, 0, s>>>(G, grad, nV, beta);
  return hipGetLastError();
}

hipError_t launch_face_counts(const int32_t* tri_id, int64_t n_px, int32_t nF, int32_t* counts, hipStream_t s) {
  EXM_TIMED("face_counts", s);
  k_face_counts<<<nblk(n_px), kThreads, 0, s>>>(tri_id, n_px, nF, counts);
  return hipGetLastError();
}

hipError_t launch_topology_scores(const exm_topo_mesh* m, const exm_topo_params* p, double* S, double* K, double* D,
                                  double* area, void* ws, hipStream_t s) {
  Layout L = make_layout(static_cast<char*>(ws), m->nV, m->nF, m->nUV, topology_split_count(m->nF, p));
  EXM_TIMED("topology_scores", s);
  HIP_TRY(scores_pass(L, m, nullptr, p, false, s));
  const size_t n = (size_t)m->nF * sizeof(double);
  if (n) {
    HIP_TRY(hipMemcpyAsync(S, L.S, n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(K, L.Kf, n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(D, L.Dg, n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(area, L.area, n, hipMemcpyDeviceToDevice, s));
  }
  return hipGetLastError();
}

hipError_t launch_topology_round(exm_topo_mesh* m, const int32_t* c_rend, const exm_topo_params* p, void* ws,
                                 exm_topo_stats* st, hipStream_t s) {
  const int32_t nV = m->nV, nF = m->nF, nUV = m->nUV;
  const int32_t K0 = topology_split_count(nF, p);
  Layout L = make_layout(static_cast<char*>(ws), nV, nF, nUV, K0);
  int32_t* host = nullptr;
  std::vector<int32_t> hbuf(16, 0);
  host = hbuf.data();
  std::memset(st, 0, sizeof(*st));
  if (nF == 0) return hipSuccess;
  EXM_TIMED("topology_round", s);
  HIP_TRY(scores_pass(L, m, c_rend, p, true, s));
  // vertex -> faces of the round-start mesh
  HIP_TRY(fill_i32(L.vf_cnt, nV, 0, s));
  HIP_TRY(fill_i32(L.vf_cur, nV, 0, s));
  k_vf_count<<<nblk(3 * (int64_t)nF), kThreads, 0, s>>>(m->tri, nF, L.vf_cnt);
  HIP_TRY(scan(L, L.vf_cnt, L.vf_off, nV, s));
  k_vf_fill<<<nblk(3 * (int64_t)nF), kThreads, 0, s>>>(m->tri, nF, L.vf_off, L.vf_cur, L.vf_list);
  HIP_TRY(hipGetLastError());
  HIP_TRY(read_words(L.counters, host, 2, s));
  const int32_t K = (p->flags & EXM_TOPO_NO_SPLIT) ? 0 : std::min(K0, host[kSplitCand]);
  const int32_t M = (p->flags & EXM_TOPO_NO_MERGE) ? 0 : host[kMergeCand];
  st->split_selected = K;
  st->merge_candidates = M;
  // rank the candidates: splits by descending S_f, merges by ascending D_f (stable: ties keep
  // the face order)
  if (K > 0) HIP_TRY(sort_faces(L, L.skey, nF, true, L.sval2, s));
  if (M > 0) HIP_TRY(sort_faces(L, L.mkey, nF, false, L.mval2, s));
  SplitArgs sa{p->tau_uv};
  if (K > 0)
    k_split_prepare<<<nblk(K), kThreads, 0, s>>>(m->pos, m->G, m->uv, m->tri, m->tri_uv, L.deg, L.edge_slot, L.hface,
                                                 L.hcnt, L.ell, L.sval2, K, sa, L.sops, L.s_faces, L.s_off, L.s_len,
                                                 L.s_state);
  if (M > 0)
    k_merge_prepare<<<nblk(M), kThreads, 0, s>>>(m->tri, L.deg, L.edge_slot, L.hcnt, L.ell, L.mval2, M, L.vf_off,
                                                 L.vf_cnt, L.mops, L.m_off, L.m_len, L.m_state);
  HIP_TRY(hipGetLastError());
  // conflicts: splits first, then merges against the faces the splits took
  HIP_TRY(fill_i32(L.best, nF, INT_MAX, s));
  HIP_TRY(fill_i32(L.taken, nF, 0, s));
  int32_t iters = 0;
  HIP_TRY(mis(L, K, L.s_off, L.s_len, L.s_faces, L.s_state, kSplitConflict, kSplitAccepted, host, &iters, s));
  HIP_TRY(mis(L, M, L.m_off, L.m_len, L.vf_list, L.m_state, kMergeConflict, kMergeAccepted, host, &iters, s));
  st->mis_iterations = iters;
  // new vertices, faces and UVs of the accepted splits, numbered in rank order
  int32_t tot[3] = {0, 0, 0};
  if (K > 0) {
    k_split_counts<<<nblk(K), kThreads, 0, s>>>(K, L.sops, L.s_state, L.add);
    for (int q = 0; q < 3; ++q) HIP_TRY(scan(L, L.add + (size_t)q * K, L.add_off + (size_t)q * K, K, s));
    int32_t last[6];
    for (int q = 0; q < 3; ++q) {
      HIP_TRY(hipMemcpyAsync(&last[2 * q], L.add_off + (size_t)q * K + K - 1, 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(&last[2 * q + 1], L.add + (size_t)q * K + K - 1, 4, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    for (int q = 0; q < 3; ++q) tot[q] = last[2 * q] + last[2 * q + 1];
  }
  const int32_t V1 = nV + tot[0], F1 = nF + tot[1], U1 = nUV + tot[2];
  HIP_TRY(fill_i32(L.deleted, F1, 0, s));
  if (K > 0)
    k_split_apply<<<nblk(K), kThreads, 0, s>>>(K, L.sops, L.s_state, L.add_off, nV, nF, nUV, m->pos, m->G, m->uv,
                                               m->tri, m->tri_uv);
  if (M > 0)
    k_merge_apply<<<nblk(M), kThreads, 0, s>>>(M, L.mops, L.m_state, L.vf_off, L.vf_cnt, L.vf_list, m->tri, L.deleted,
                                               L.counters);
  // compaction: unreferenced vertices and UVs dropped, order kept
  HIP_TRY(fill_i32(L.vref, V1, 0, s));
  HIP_TRY(fill_i32(L.uref, U1, 0, s));
  k_mark_refs<<<nblk(F1), kThreads, 0, s>>>(F1, m->tri, m->tri_uv, L.deleted, L.alive, L.vref, L.uref);
  HIP_TRY(hipGetLastError());
  int32_t* totals = L.host_words;  // [fmap_last, vmap_last, umap_last]
  HIP_TRY(scan(L, L.alive, L.fmap, F1, s));
  HIP_TRY(scan(L, L.vref, L.vmap, V1, s));
  HIP_TRY(scan(L, L.uref, L.umap, U1, s));
  HIP_TRY(hipMemcpyAsync(totals + 0, L.fmap + (F1 - 1), 4, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(totals + 1, L.alive + (F1 - 1), 4, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(totals + 2, L.vmap + (V1 - 1), 4, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(totals + 3, L.vref + (V1 - 1), 4, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(totals + 4, L.umap + (U1 - 1), 4, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(totals + 5, L.uref + (U1 - 1), 4, hipMemcpyDeviceToDevice, s));
  k_compact_rows<<<nblk(V1), kThreads, 0, s>>>(V1, 3, L.vref, L.vmap, m->pos, L.pos2);
  k_compact_rows<<<nblk(V1), kThreads, 0, s>>>(V1, 1, L.vref, L.vmap, m->G, L.G2);
  k_compact_rows<<<nblk(U1), kThreads, 0, s>>>(U1, 2, L.uref, L.umap, m->uv, L.uv2);
  k_compact_faces<<<nblk(F1), kThreads, 0, s>>>(F1, L.alive, L.fmap, L.vmap, L.umap, m->tri, m->tri_uv, L.tri2,
                                                L.tri_uv2);
  HIP_TRY(hipGetLastError());
  HIP_TRY(read_words(totals, host, 6, s));
  const int32_t F2 = host[0] + host[1], V2 = host[2] + host[3], U2 = host[4] + host[5];
  HIP_TRY(copy_back(m->pos, L.pos2, 3 * (size_t)V2, s));
  HIP_TRY(copy_back(m->G, L.G2, (size_t)V2, s));
  HIP_TRY(copy_back(m->uv, L.uv2, 2 * (size_t)U2, s));
  HIP_TRY(copy_back(m->tri, L.tri2, 3 * (size_t)F2, s));
  HIP_TRY(copy_back(m->tri_uv, L.tri_uv2, 3 * (size_t)F2, s));
  HIP_TRY(read_words(L.counters, host, kNumCounters, s));
  st->split_invalid = 0;
  st->split_conflict = host[kSplitConflict];
  st->splits = host[kSplitAccepted];
  st->merge_conflict = host[kMergeConflict];
  st->merges = host[kMergeAccepted];
  st->faces_deleted = host[kFacesDeleted];
  st->split_invalid = K - st->splits - st->split_conflict;
  m->nV = V2;
  m->nF = F2;
  m->nUV = U2;
  return hipSuccess;
}

}  // namespace exm

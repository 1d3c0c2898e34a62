// LBVH construction and refit on the GPU.
//
// Build: centroid bounds -> 30-bit Morton codes -> stable LSD radix sort
// (four 8-bit passes; ranks from wave ballots, so equal keys keep their
// order) -> binary radix tree over the sorted codes (Karras, HPG 2012, with
// the index as tie-break for equal codes) -> bottom-up boxes.
// Refit: the bottom-up box pass alone, over the last built topology.
// Alternative build (FR_REBUILD_SAH): a binned surface-area-heuristic tree
// built on the host, numbered like a binary radix tree so that the same
// refit, collapse and traversal apply.
//
// A boundary-to-root walk per leaf gives the depth; the traversal stack is 64
// entries, so trees deeper than that are rejected by the host.
#include <algorithm>
#include <cstring>
#include <vector>

#include "fr_kernels.h"

namespace fr {

// ---------------------------------------------------------------------------
// Centroid bounds (two-level min/max reduction) and Morton codes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ V3 centroid(const float* __restrict__ v, const int32_t* __restrict__ tris, int f) {
  const V3 a = ld3(v, tris[3 * f]), b = ld3(v, tris[3 * f + 1]), c = ld3(v, tris[3 * f + 2]);
  return {(a.x + b.x + c.x) * (1.0f / 3.0f), (a.y + b.y + c.y) * (1.0f / 3.0f), (a.z + b.z + c.z) * (1.0f / 3.0f)};
}

__global__ __launch_bounds__(256) void k_centroid_bounds(const float* __restrict__ v, const int32_t* __restrict__ tris,
                                                         int F, float* __restrict__ partial) {
  __shared__ float red[6][256];
  float mn[3] = {3.4e38f, 3.4e38f, 3.4e38f}, mx[3] = {-3.4e38f, -3.4e38f, -3.4e38f};
  for (int f = blockIdx.x * 256 + threadIdx.x; f < F; f += gridDim.x * 256) {
    const V3 c = centroid(v, tris, f);
    mn[0] = fminf(mn[0], c.x); mn[1] = fminf(mn[1], c.y); mn[2] = fminf(mn[2], c.z);
    mx[0] = fmaxf(mx[0], c.x); mx[1] = fmaxf(mx[1], c.y); mx[2] = fmaxf(mx[2], c.z);
  }
  for (int k = 0; k < 3; ++k) { red[k][threadIdx.x] = mn[k]; red[3 + k][threadIdx.x] = mx[k]; }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fminf(red[k][threadIdx.x], red[k][threadIdx.x + s]);
        red[3 + k][threadIdx.x] = fmaxf(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// Spread the low 10 bits of x so that bit i lands at bit 3i.
__device__ __forceinline__ uint32_t spread3(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ v, const int32_t* __restrict__ tris, int F,
                                                const float* __restrict__ partial, int nparts,
                                                uint32_t* __restrict__ keys, int32_t* __restrict__ vals,
                                                float* __restrict__ scene_box) {
  float mn[3] = {3.4e38f, 3.4e38f, 3.4e38f}, mx[3] = {-3.4e38f, -3.4e38f, -3.4e38f};
  for (int p = 0; p < nparts; ++p)
    for (int k = 0; k < 3; ++k) { mn[k] = fminf(mn[k], partial[6 * p + k]); mx[k] = fmaxf(mx[k], partial[6 * p + 3 + k]); }
  const int f = blockIdx.x * 256 + threadIdx.x;
  if (f == 0)
    for (int k = 0; k < 3; ++k) { scene_box[k] = mn[k]; scene_box[3 + k] = mx[k]; }
  if (f >= F) return;
  const V3 c = centroid(v, tris, f);
  const float cc[3] = {c.x, c.y, c.z};
  uint32_t q[3];
  for (int k = 0; k < 3; ++k) {
    const float ext = mx[k] - mn[k];
    const float u = ext > 0.0f ? (cc[k] - mn[k]) / ext : 0.5f;
    q[k] = (uint32_t)fminf(fmaxf(u * 1024.0f, 0.0f), 1023.0f);
  }
  keys[f] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
  vals[f] = f;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits, tiles of 1024 keys per 256-thread block.
// ---------------------------------------------------------------------------
constexpr int kSortTile = 1024;

__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ keys, int n, int shift,
                                                    uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortTile;
  for (int i = threadIdx.x; i < kSortTile; i += 256) {
    const int k = base + i;
    if (k < n) atomicAdd(&cnt[(keys[k] >> shift) & 0xffu], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];   // digit-major
}

// Exclusive scan of hist[256 * nblocks] in place (single block of 1024).
__global__ __launch_bounds__(1024) void k_radix_scan(uint32_t* __restrict__ hist, int total) {
  __shared__ uint32_t part[1024];
  const int per = (total + 1023) / 1024;
  const int b = threadIdx.x * per;
  uint32_t s = 0;
  for (int i = 0; i < per; ++i) if (b + i < total) s += hist[b + i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t x = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int i = 0; i < per; ++i)
    if (b + i < total) { const uint32_t h = hist[b + i]; hist[b + i] = run; run += h; }
}

__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                                       int n, int shift, const uint32_t* __restrict__ offs, int nblocks,
                                                       uint32_t* __restrict__ kout, int32_t* __restrict__ vout) {
  __shared__ uint32_t run[256];        // keys of each digit already placed by this block
  __shared__ uint32_t wcnt[4][256];    // per-wave digit counts of the current round
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  run[threadIdx.x] = 0;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int round = 0; round < kSortTile / 256; ++round) {
    for (int w = 0; w < 4; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const int k = blockIdx.x * kSortTile + round * 256 + threadIdx.x;
    const bool ok = k < n;
    const uint32_t key = ok ? kin[k] : 0u;
    const uint32_t dig = (key >> shift) & 0xffu;
    uint64_t peers = ballot(ok);
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (dig >> bit) & 1u;
      const uint64_t m = ballot(on);
      peers &= on ? m : ~m;
    }
    const uint32_t rank_w = (uint32_t)__popcll(peers & lt);
    if (ok && (peers >> lane) == 1ull) wcnt[wave][dig] = rank_w + 1;   // highest lane of the group
    __syncthreads();
    if (ok) {
      uint32_t before = run[dig];
      for (int w = 0; w < wave; ++w) before += wcnt[w][dig];
      const uint32_t pos = offs[dig * nblocks + blockIdx.x] + before + rank_w;
      kout[pos] = key;
      vout[pos] = vin[k];
    }
    __syncthreads();
    run[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] + wcnt[2][threadIdx.x] + wcnt[3][threadIdx.x];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Binary radix tree (Karras 2012).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int common_prefix(const uint32_t* __restrict__ k, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  const uint32_t a = k[i], b = k[j];
  if (a != b) return __clz(a ^ b);
  return 32 + __clz((uint32_t)i ^ (uint32_t)j);
}

__global__ __launch_bounds__(256) void k_karras(const uint32_t* __restrict__ k, int n, BvhNode* __restrict__ nodes,
                                                int32_t* __restrict__ node_parent, int32_t* __restrict__ leaf_parent) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n - 1) return;
  const int d = common_prefix(k, n, i, i + 1) - common_prefix(k, n, i, i - 1) > 0 ? 1 : -1;
  const int dmin = common_prefix(k, n, i, i - d);
  int lmax = 2;
  while (common_prefix(k, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int l = 0;
  for (int t = lmax >> 1; t >= 1; t >>= 1)
    if (common_prefix(k, n, i, i + (l + t) * d) > dmin) l += t;
  const int j = i + l * d;
  const int dnode = common_prefix(k, n, i, j);
  int s = 0;
  int t = l;
  do {
    t = (t + 1) >> 1;
    if (common_prefix(k, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  const int split = i + s * d + (d < 0 ? -1 : 0);
  const int lo = min(i, j), hi = max(i, j);
  const int c0 = (lo == split) ? ~split : split;
  const int c1 = (hi == split + 1) ? ~(split + 1) : split + 1;
  nodes[i].c0 = c0;
  nodes[i].c1 = c1;
  nodes[i].lo = lo;       // sorted leaf range of the node (tile-local refit)
  nodes[i].hi = hi;
  if (c0 < 0) leaf_parent[~c0] = i; else node_parent[c0] = i;
  if (c1 < 0) leaf_parent[~c1] = i; else node_parent[c1] = i;
  if (i == 0) node_parent[0] = -1;
}

// Single-triangle mesh: one node whose second child box is empty.
__global__ void k_single_leaf(BvhNode* __restrict__ nodes, int32_t* __restrict__ leaf_parent) {
  nodes[0].c0 = ~0;
  nodes[0].c1 = ~0;
  nodes[0].lo = 0;
  nodes[0].hi = 0;
  for (int k = 0; k < 3; ++k) { nodes[0].b1[k] = 3.4e38f; nodes[0].b1[3 + k] = -3.4e38f; }
  leaf_parent[0] = 0;
}

// ---------------------------------------------------------------------------
// Refit: leaf records + bottom-up boxes, in two phases over the fixed
// topology.  (1) One workgroup per tile of kRefitTile consecutive sorted
// leaves: every leaf's thread climbs while the parent's leaf range lies in the
// tile; the second child to arrive at a node (LDS counter) merges both child
// boxes (kept in LDS) and climbs on.  A climb that reaches a node spanning
// several tiles stores its box in that node and stops.  (2) One workgroup
// finishes the spanning ("top") nodes level by level, children before
// parents (the order is computed on the host at build time).  No device-scope
// synchronisation.
// ---------------------------------------------------------------------------
constexpr int kRefitTile = 256;

__device__ __forceinline__ void store_child_box(BvhNode* nodes, int p, int child, const float box[6]) {
  float* dst = nodes[p].c0 == child ? nodes[p].b0 : nodes[p].b1;
  for (int k = 0; k < 6; ++k) dst[k] = box[k];
}

__device__ __forceinline__ void refit_local_block(const float* __restrict__ v, const int32_t* __restrict__ tris,
                                                  const int32_t* __restrict__ order, int F, BvhNode* nodes,
                                                  const int32_t* __restrict__ node_parent,
                                                  const int32_t* __restrict__ leaf_parent, TriRec* __restrict__ recs,
                                                  float pad, int bid) {
  __shared__ uint32_t flag[kRefitTile];
  __shared__ float sbox[kRefitTile][2][6];
  flag[threadIdx.x] = 0u;
  __syncthreads();
  const int t0 = bid * kRefitTile, t1 = min(F, t0 + kRefitTile) - 1;
  const int slot = t0 + threadIdx.x;
  if (slot >= F) return;
  const int f = order[slot];
  const V3 a = ld3(v, tris[3 * f]), b = ld3(v, tris[3 * f + 1]), c = ld3(v, tris[3 * f + 2]);
  TriRec r;
  r.v[0] = a.x; r.v[1] = a.y; r.v[2] = a.z; r.v[3] = b.x; r.v[4] = b.y; r.v[5] = b.z;
  r.v[6] = c.x; r.v[7] = c.y; r.v[8] = c.z;
  r.id = f; r.pad0 = 0; r.pad1 = 0;
  recs[slot] = r;
  float box[6] = {fminf(a.x, fminf(b.x, c.x)) - pad, fminf(a.y, fminf(b.y, c.y)) - pad,
                  fminf(a.z, fminf(b.z, c.z)) - pad, fmaxf(a.x, fmaxf(b.x, c.x)) + pad,
                  fmaxf(a.y, fmaxf(b.y, c.y)) + pad, fmaxf(a.z, fmaxf(b.z, c.z)) + pad};
  int child = ~slot;
  int p = leaf_parent[slot];
  while (p >= 0) {
    store_child_box(nodes, p, child, box);
    if (F == 1) return;
    const int lo = nodes[p].lo, hi = nodes[p].hi;
    if (lo < t0 || hi > t1) return;          // spanning node: finished by the top pass
    const int q = p - t0;                    // a node's index is one end of its range
    const int side = nodes[p].c0 == child ? 0 : 1;
    for (int k = 0; k < 6; ++k) sbox[q][side][k] = box[k];
    __threadfence_block();
    if (atomicAdd(&flag[q], 1u) == 0u) return;   // the sibling finishes this node
    __threadfence_block();
    for (int k = 0; k < 3; ++k) {
      box[k] = fminf(sbox[q][0][k], sbox[q][1][k]);
      box[3 + k] = fmaxf(sbox[q][0][3 + k], sbox[q][1][3 + k]);
    }
    child = p;
    p = node_parent[p];
  }
}

__global__ __launch_bounds__(kRefitTile) void k_refit_local(const float* __restrict__ v,
                                                            const int32_t* __restrict__ tris,
                                                            const int32_t* __restrict__ order, int F, BvhNode* nodes,
                                                            const int32_t* __restrict__ node_parent,
                                                            const int32_t* __restrict__ leaf_parent,
                                                            TriRec* __restrict__ recs, float pad) {
  refit_local_block(v, tris, order, F, nodes, node_parent, leaf_parent, recs, pad, blockIdx.x);
}

// top[]: spanning nodes, children before parents; level_off[l]..level_off[l+1]
// is level l (nodes of a level are independent).
__device__ __forceinline__ void refit_top_block(BvhNode* nodes, const int32_t* __restrict__ node_parent,
                                                const int32_t* __restrict__ top, const int32_t* __restrict__ level_off,
                                                int n_levels) {
  for (int l = 0; l < n_levels; ++l) {
    for (int i = level_off[l] + threadIdx.x; i < level_off[l + 1]; i += blockDim.x) {
      const int p = top[i];
      const int g = node_parent[p];
      if (g < 0) continue;
      float box[6];
      for (int k = 0; k < 3; ++k) {
        box[k] = fminf(nodes[p].b0[k], nodes[p].b1[k]);
        box[3 + k] = fmaxf(nodes[p].b0[3 + k], nodes[p].b1[3 + k]);
      }
      store_child_box(nodes, g, p, box);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void k_refit_top(BvhNode* nodes, const int32_t* __restrict__ node_parent,
                                                    const int32_t* __restrict__ top,
                                                    const int32_t* __restrict__ level_off, int n_levels) {
  refit_top_block(nodes, node_parent, top, level_off, n_levels);
}

// Structural check of a freshly built tree: sorted keys, child and parent
// indices in range, and every node the child of exactly one parent (so the
// topology is a tree and traversal terminates).  Counts violations.
__global__ __launch_bounds__(256) void k_validate(const uint32_t* __restrict__ keys, int F,
                                                  const BvhNode* __restrict__ nodes,
                                                  const int32_t* __restrict__ node_parent,
                                                  const int32_t* __restrict__ leaf_parent, uint32_t* __restrict__ bad) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= F) return;
  uint32_t err = 0;
  if (i + 1 < F && keys[i] > keys[i + 1]) ++err;
  const int lp = leaf_parent[i];
  if (lp < 0 || lp >= max(F - 1, 1)) ++err;
  else if (nodes[lp].c0 != ~i && nodes[lp].c1 != ~i) ++err;
  if (i < F - 1) {
    const int c[2] = {nodes[i].c0, nodes[i].c1};
    for (int k = 0; k < 2; ++k) {
      if (c[k] >= 0) {
        if (c[k] >= F - 1 || c[k] == 0) ++err;
        else if (node_parent[c[k]] != i) ++err;
      } else if (~c[k] >= F || leaf_parent[~c[k]] != i) {
        ++err;
      }
    }
    if (i > 0) {
      const int p = node_parent[i];
      if (p < 0 || p >= F - 1) ++err;
      else if (nodes[p].c0 != i && nodes[p].c1 != i) ++err;
    }
  }
  if (err) atomicAdd(bad, err);
}

__global__ __launch_bounds__(256) void k_leaf_depth(const int32_t* __restrict__ node_parent,
                                                    const int32_t* __restrict__ leaf_parent, int F,
                                                    int32_t* __restrict__ max_depth) {
  const int slot = blockIdx.x * 256 + threadIdx.x;
  if (slot >= F) return;
  int d = 1;
  int p = leaf_parent[slot];
  while (p > 0 && p < F - 1 && d < 4096) { p = node_parent[p]; ++d; }
  // a leaf whose parent chain does not end at the root makes the tree invalid
  atomicMax(max_depth, p == 0 ? d : 1 << 20);
}

// Child boxes of the 4-wide nodes, copied from the binary tree after a refit:
// one thread per (node, slot).
__device__ __forceinline__ void gather4_block(const BvhNode* __restrict__ nodes, const int32_t* __restrict__ src,
                                              int n4, Bvh4Node* __restrict__ out, int bid) {
  const int t = bid * 256 + threadIdx.x;
  if (t >= 4 * n4) return;
  const int i = t >> 2, k = t & 3;
  const int sref = src[t];
  float b[6] = {3.4e38f, 3.4e38f, 3.4e38f, -3.4e38f, -3.4e38f, -3.4e38f};
  if (sref >= 0) {
    const float* bb = (sref & 1) ? nodes[sref >> 1].b1 : nodes[sref >> 1].b0;
    for (int q = 0; q < 6; ++q) b[q] = bb[q];
  }
  for (int a = 0; a < 3; ++a) {
    out[i].lo[a][k] = b[a];
    out[i].hi[a][k] = b[3 + a];
  }
}

__global__ __launch_bounds__(256) void k_gather4(const BvhNode* __restrict__ nodes, const int32_t* __restrict__ src,
                                                 int n4, Bvh4Node* __restrict__ out) {
  gather4_block(nodes, src, n4, out, blockIdx.x);
}

__device__ __forceinline__ void zero_u32_block(uint32_t* p, int n, int bid) {
  const int i = bid * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  zero_u32_block(p, n, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Host drivers
// ---------------------------------------------------------------------------

void bvh_refit(MeshDev& m, const float* d_verts, hipStream_t st) {
  const int F = m.F;
  hipLaunchKernelGGL(k_refit_local, dim3(cdiv(F, kRefitTile)), dim3(kRefitTile), 0, st, d_verts, m.tris, m.order, F,
                     m.nodes, m.node_parent, m.leaf_parent, m.recs, kBoxPad);
  if (m.n_top_levels > 0)
    hipLaunchKernelGGL(k_refit_top, dim3(1), dim3(1024), 0, st, m.nodes, m.node_parent, m.top_nodes,
                       m.top_level_off, m.n_top_levels);
  if (m.n4 > 0)
    hipLaunchKernelGGL(k_gather4, dim3(cdiv(4 * m.n4, 256)), dim3(256), 0, st, m.nodes, m.n4_src, m.n4, m.nodes4);
}

static int download_nodes(const MeshDev& m, std::vector<BvhNode>& bn, hipStream_t st) {
  bn.resize((size_t)m.F - 1);
  if (hipMemcpyAsync(bn.data(), m.nodes, sizeof(BvhNode) * (m.F - 1), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return FR_ERR_DEVICE;
  return FR_OK;
}

// Refit schedule of a binary tree (host side, once per build): the nodes
// whose leaf range spans several refit tiles, grouped by height (children
// first), for the one-workgroup top pass.
static int bvh_refit_schedule(MeshDev& m, const std::vector<BvhNode>& bn, hipStream_t st) {
  const int F = m.F;
  auto child = [&](int b, int s) { return s ? bn[b].c1 : bn[b].c0; };
  std::vector<int> height((size_t)F - 1, 0);   // longest path to a leaf, by a post-order walk
  std::vector<int> post;
  post.reserve((size_t)F - 1);
  std::vector<std::pair<int, int>> st2 = {{0, 0}};
  while (!st2.empty()) {
    auto& top = st2.back();
    const int b = top.first;
    if (top.second < 2) {
      const int c = child(b, top.second++);
      if (c >= 0) st2.push_back({c, 0});
    } else {
      int h = 0;
      for (int q = 0; q < 2; ++q) { const int c = child(b, q); if (c >= 0) h = std::max(h, height[c] + 1); }
      height[b] = h;
      post.push_back(b);
      st2.pop_back();
    }
  }
  std::vector<std::vector<int>> levels;
  for (int b : post) {
    if (bn[b].lo / kRefitTile == bn[b].hi / kRefitTile) continue;   // tile-local
    const int h = height[b];   // a spanning child has a smaller height: an earlier level
    if ((int)levels.size() <= h) levels.resize(h + 1);
    levels[h].push_back(b);
  }
  std::vector<int32_t> top, off = {0};
  for (auto& lv : levels) {
    if (lv.empty()) continue;
    top.insert(top.end(), lv.begin(), lv.end());
    off.push_back((int32_t)top.size());
  }
  const int nt = (int)top.size();
  if (nt > m.top_cap) {
    if (m.top_nodes) (void)hipFree(m.top_nodes);
    if (m.top_level_off) (void)hipFree(m.top_level_off);
    m.top_nodes = nullptr; m.top_level_off = nullptr; m.top_cap = 0;
    if (hipMalloc(&m.top_nodes, sizeof(int32_t) * std::max(nt, 1)) != hipSuccess) return FR_ERR_OOM;
    if (hipMalloc(&m.top_level_off, sizeof(int32_t) * (std::max(nt, 1) + 1)) != hipSuccess) return FR_ERR_OOM;
    m.top_cap = nt;
  }
  if (nt > 0 &&
      (hipMemcpyAsync(m.top_nodes, top.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(m.top_level_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, st) !=
           hipSuccess ||
       hipStreamSynchronize(st) != hipSuccess))
    return FR_ERR_DEVICE;
  m.n_top = nt;
  m.n_top_levels = (int)off.size() - 1;
  return FR_OK;
}

// Collapse the binary tree (with its boxes from a first refit) into the
// 4-wide traversal tree, host side, once per build.  Each 4-wide node starts
// from the two children of a binary node and repeatedly opens the internal
// child of largest surface area (the one a random ray is likeliest to enter)
// until it holds four children or only leaves; nodes are numbered in
// depth-first order.  Boxes are filled by k_gather4 at every refit, each
// slot from the binary box it was made of (parent node, side).
static int bvh_collapse(MeshDev& m, const std::vector<BvhNode>& bn, hipStream_t st) {
  const int F = m.F;
  auto child = [&](int b, int s) { return s ? bn[b].c1 : bn[b].c0; };
  // parent and side of every internal node and leaf
  std::vector<int> par_i((size_t)F - 1, -1), par_l((size_t)F, -1);
  for (int b = 0; b < F - 1; ++b)
    for (int sd = 0; sd < 2; ++sd) {
      const int c = child(b, sd);
      if (c >= 0) par_i[c] = 2 * b + sd;
      else par_l[~c] = 2 * b + sd;
    }
  auto src_of = [&](int ref) { return ref >= 0 ? par_i[ref] : par_l[~ref]; };
  auto area_of = [&](int ref) {
    const int ps = src_of(ref);
    const float* b = (ps & 1) ? bn[ps >> 1].b1 : bn[ps >> 1].b0;
    const float dx = std::max(b[3] - b[0], 0.0f), dy = std::max(b[4] - b[1], 0.0f), dz = std::max(b[5] - b[2], 0.0f);
    return dx * dy + dy * dz + dz * dx;
  };
  // children of the 4-wide node made from binary node b
  auto slots = [&](int b, int ref[4]) {
    int n = 2;
    ref[0] = child(b, 0);
    ref[1] = child(b, 1);
    while (n < 4) {
      int best = -1;
      float ba = -1.0f;
      for (int k = 0; k < n; ++k)
        if (ref[k] >= 0) {
          const float a = area_of(ref[k]);
          if (a > ba) { ba = a; best = k; }
        }
      if (best < 0) break;
      const int c = ref[best];
      for (int k = n; k > best + 1; --k) ref[k] = ref[k - 1];
      ref[best] = child(c, 0);
      ref[best + 1] = child(c, 1);
      ++n;
    }
    for (int k = n; k < 4; ++k) ref[k] = kEmpty;
    return n;
  };
  // depth-first numbering
  m.depth4 = 0;
  std::vector<int> id((size_t)F - 1, -1), order;
  std::vector<int> todo = {0}, tdepth = {1};
  while (!todo.empty()) {
    const int b = todo.back(), d = tdepth.back();
    todo.pop_back(); tdepth.pop_back();
    id[b] = (int)order.size();
    order.push_back(b);
    m.depth4 = std::max(m.depth4, d);
    int ref[4];
    const int n = slots(b, ref);
    for (int k = n - 1; k >= 0; --k)
      if (ref[k] >= 0) { todo.push_back(ref[k]); tdepth.push_back(d + 1); }
  }
  const int n4 = (int)order.size();
  std::vector<Bvh4Node> h4((size_t)n4);
  std::vector<int32_t> hsrc((size_t)4 * n4);
  for (int i = 0; i < n4; ++i) {
    int ref[4];
    slots(order[i], ref);
    Bvh4Node& nd = h4[i];
    std::memset(&nd, 0, sizeof(nd));
    for (int k = 0; k < 4; ++k) {
      nd.c[k] = ref[k] == kEmpty ? kEmpty : (ref[k] >= 0 ? id[ref[k]] : ref[k]);
      int sub = 0;
      if (ref[k] >= 0 && ref[k] != kEmpty) { int r2[4]; sub = slots(ref[k], r2); }
      nd.nsub[k] = sub;
      hsrc[(size_t)4 * i + k] = ref[k] == kEmpty ? -1 : src_of(ref[k]);
    }
  }
  if (n4 > m.n4_cap) {
    if (m.nodes4) (void)hipFree(m.nodes4);
    if (m.n4_src) (void)hipFree(m.n4_src);
    m.nodes4 = nullptr; m.n4_src = nullptr; m.n4_cap = 0;
    if (hipMalloc(&m.nodes4, sizeof(Bvh4Node) * n4) != hipSuccess) return FR_ERR_OOM;
    if (hipMalloc(&m.n4_src, sizeof(int32_t) * 4 * n4) != hipSuccess) return FR_ERR_OOM;
    m.n4_cap = n4;
  }
  if (hipMemcpyAsync(m.nodes4, h4.data(), sizeof(Bvh4Node) * n4, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(m.n4_src, hsrc.data(), sizeof(int32_t) * 4 * n4, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return FR_ERR_DEVICE;
  m.n4 = n4;
  return FR_OK;
}

// Binned SAH build on the host (Wald, "On fast construction of SAH-based
// bounding volume hierarchies", 2007): at each node, 32 centroid bins per
// axis, the split between bins that minimises A(left) N(left) + A(right)
// N(right) (A the box surface area), a median split by index when all
// centroids coincide.  Each node covers a contiguous range [lo, hi] of the
// leaf order; numbering as in a binary radix tree: the root is 0, the child
// ranges [lo, s] and [s + 1, hi] of a split after slot s get the indices s
// and s + 1 (a one-leaf range is the leaf ~slot).  Every internal index is
// then one end of its node's range and the F - 1 internal nodes take the
// indices 0 .. F - 2 exactly once, which the refit relies on.
static int bvh_build_sah_host(MeshDev& m, const float* d_verts, hipStream_t st) {
  const int F = m.F, N = m.N;
  std::vector<float> v((size_t)3 * N);
  std::vector<int32_t> t((size_t)3 * F);
  if (hipMemcpyAsync(v.data(), d_verts, sizeof(float) * 3 * N, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(t.data(), m.tris, sizeof(int32_t) * 3 * F, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return FR_ERR_DEVICE;
  std::vector<float> pb((size_t)6 * F), pc((size_t)3 * F);
  for (int f = 0; f < F; ++f) {
    for (int a = 0; a < 3; ++a) {
      const float x0 = v[3 * t[3 * f] + a], x1 = v[3 * t[3 * f + 1] + a], x2 = v[3 * t[3 * f + 2] + a];
      pb[6 * f + a] = std::min(x0, std::min(x1, x2));
      pb[6 * f + 3 + a] = std::max(x0, std::max(x1, x2));
      pc[3 * f + a] = (x0 + x1 + x2) * (1.0f / 3.0f);
    }
  }
  std::vector<int32_t> idx((size_t)F), npar((size_t)F - 1, -1), lpar((size_t)F, -1);
  for (int f = 0; f < F; ++f) idx[f] = f;
  std::vector<BvhNode> nodes((size_t)F - 1);
  std::memset(nodes.data(), 0, sizeof(BvhNode) * nodes.size());
  constexpr int B = 32;
  struct Task { int lo, hi, id, parent; };
  std::vector<Task> todo = {{0, F - 1, 0, -1}};
  auto area = [](const float* b) {
    const float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return dx * dy + dy * dz + dz * dx;
  };
  auto grow = [](float* b, const float* c) {
    for (int a = 0; a < 3; ++a) { b[a] = std::min(b[a], c[a]); b[3 + a] = std::max(b[3 + a], c[3 + a]); }
  };
  while (!todo.empty()) {
    const Task tk = todo.back();
    todo.pop_back();
    const int lo = tk.lo, hi = tk.hi, n = hi - lo + 1;
    float cmin[3] = {3.4e38f, 3.4e38f, 3.4e38f}, cmax[3] = {-3.4e38f, -3.4e38f, -3.4e38f};
    for (int i = lo; i <= hi; ++i)
      for (int a = 0; a < 3; ++a) {
        cmin[a] = std::min(cmin[a], pc[3 * idx[i] + a]);
        cmax[a] = std::max(cmax[a], pc[3 * idx[i] + a]);
      }
    double best = 1e300;
    int bax = -1, bbin = -1;
    for (int a = 0; a < 3; ++a) {
      const float ext = cmax[a] - cmin[a];
      if (!(ext > 0.0f)) continue;
      const float sc = (float)B / ext;
      int cnt[B] = {};
      float bb[B][6];
      for (int k = 0; k < B; ++k) { bb[k][0] = bb[k][1] = bb[k][2] = 3.4e38f; bb[k][3] = bb[k][4] = bb[k][5] = -3.4e38f; }
      for (int i = lo; i <= hi; ++i) {
        const int f = idx[i];
        const int k = std::min(B - 1, (int)((pc[3 * f + a] - cmin[a]) * sc));
        ++cnt[k];
        grow(bb[k], &pb[6 * f]);
      }
      double la[B], ra[B];
      int ln[B], rn[B];
      float acc[6] = {3.4e38f, 3.4e38f, 3.4e38f, -3.4e38f, -3.4e38f, -3.4e38f};
      int c = 0;
      for (int k = 0; k < B - 1; ++k) {
        if (cnt[k]) grow(acc, bb[k]);
        c += cnt[k];
        ln[k] = c;
        la[k] = c ? area(acc) : 0.0;
      }
      float acc2[6] = {3.4e38f, 3.4e38f, 3.4e38f, -3.4e38f, -3.4e38f, -3.4e38f};
      c = 0;
      for (int k = B - 1; k > 0; --k) {
        if (cnt[k]) grow(acc2, bb[k]);
        c += cnt[k];
        rn[k - 1] = c;
        ra[k - 1] = c ? area(acc2) : 0.0;
      }
      for (int k = 0; k < B - 1; ++k) {
        if (ln[k] == 0 || rn[k] == 0) continue;
        const double cost = la[k] * ln[k] + ra[k] * rn[k];
        if (cost < best) { best = cost; bax = a; bbin = k; }
      }
    }
    int mid;   // left = [lo, mid], right = [mid + 1, hi]
    if (bax < 0) {
      mid = lo + n / 2 - 1;
    } else {
      const float sc = (float)B / (cmax[bax] - cmin[bax]);
      const float c0 = cmin[bax];
      auto it = std::partition(idx.begin() + lo, idx.begin() + hi + 1, [&](int f) {
        return std::min(B - 1, (int)((pc[3 * f + bax] - c0) * sc)) <= bbin;
      });
      mid = (int)(it - idx.begin()) - 1;
    }
    BvhNode& nd = nodes[tk.id];
    nd.lo = lo;
    nd.hi = hi;
    nd.c0 = mid == lo ? ~lo : mid;
    nd.c1 = mid + 1 == hi ? ~hi : mid + 1;
    npar[tk.id] = tk.parent;
    if (nd.c0 < 0) lpar[lo] = tk.id; else todo.push_back({lo, mid, mid, tk.id});
    if (nd.c1 < 0) lpar[hi] = tk.id; else todo.push_back({mid + 1, hi, mid + 1, tk.id});
  }
  // structural check: every internal index and leaf slot has exactly one parent
  for (int i = 1; i < F - 1; ++i)
    if (npar[i] < 0) return FR_ERR_LIMIT;
  for (int i = 0; i < F; ++i)
    if (lpar[i] < 0) return FR_ERR_LIMIT;
  if (hipMemcpyAsync(m.nodes, nodes.data(), sizeof(BvhNode) * (F - 1), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(m.order, idx.data(), sizeof(int32_t) * F, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(m.node_parent, npar.data(), sizeof(int32_t) * (F - 1), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(m.leaf_parent, lpar.data(), sizeof(int32_t) * F, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return FR_ERR_DEVICE;
  return FR_OK;
}

static int bvh_finish(MeshDev& m, const float* d_verts, hipStream_t st, int* depth_out);

int bvh_build(MeshDev& m, const float* d_verts, hipStream_t st, bool sah, int* depth_out) {
  const int F = m.F;
  if (sah && F > 1) {
    const int rc = bvh_build_sah_host(m, d_verts, st);
    if (rc != FR_OK) return rc;
    return bvh_finish(m, d_verts, st, depth_out);
  }
  const int nparts = 64;
  hipLaunchKernelGGL(k_centroid_bounds, dim3(nparts), dim3(256), 0, st, d_verts, m.tris, F, m.partial);
  hipLaunchKernelGGL(k_morton, dim3(cdiv(F, 256)), dim3(256), 0, st, d_verts, m.tris, F, m.partial, nparts,
                     m.keys[0], m.vals[0], m.scene_box);
  const int nb = cdiv(F, kSortTile);
  int cur = 0;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(256), 0, st, m.keys[cur], F, shift, m.hist, nb);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, st, m.hist, 256 * nb);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(256), 0, st, m.keys[cur], m.vals[cur], F, shift, m.hist, nb,
                       m.keys[cur ^ 1], m.vals[cur ^ 1]);
    cur ^= 1;
  }
  // after an even number of passes the sorted data is back in buffer 0
  if (hipMemcpyAsync(m.order, m.vals[cur], sizeof(int32_t) * F, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return FR_ERR_DEVICE;
  if (F > 1) {
    hipLaunchKernelGGL(k_karras, dim3(cdiv(F - 1, 256)), dim3(256), 0, st, m.keys[cur], F, m.nodes, m.node_parent,
                       m.leaf_parent);
  } else {
    hipLaunchKernelGGL(k_single_leaf, dim3(1), dim3(1), 0, st, m.nodes, m.leaf_parent);
  }
  // validate the topology before anything walks it
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t*>(m.depth), 2);
  hipLaunchKernelGGL(k_validate, dim3(cdiv(F, 256)), dim3(256), 0, st, m.keys[cur], F, m.nodes, m.node_parent,
                     m.leaf_parent, reinterpret_cast<uint32_t*>(m.depth) + 1);
  int32_t chk[2] = {0, 0};
  if (hipMemcpyAsync(chk, m.depth, sizeof(chk), hipMemcpyDeviceToHost, st) != hipSuccess) return FR_ERR_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return FR_ERR_DEVICE;
  if (chk[1] != 0) return FR_ERR_LIMIT;
  return bvh_finish(m, d_verts, st, depth_out);
}

// After either build: refit schedule, binary boxes, 4-wide collapse, 4-wide
// boxes, depth.
static int bvh_finish(MeshDev& m, const float* d_verts, hipStream_t st, int* depth_out) {
  const int F = m.F;
  m.n4 = 0;
  m.depth4 = 0;
  m.n_top = 0;
  m.n_top_levels = 0;
  if (F > 1) {
    // topology -> refit schedule -> binary boxes -> 4-wide collapse -> 4-wide boxes
    std::vector<BvhNode> bn;
    int rc = download_nodes(m, bn, st);
    if (rc == FR_OK) rc = bvh_refit_schedule(m, bn, st);
    if (rc != FR_OK) return rc;
    bvh_refit(m, d_verts, st);
    if ((rc = download_nodes(m, bn, st)) != FR_OK || (rc = bvh_collapse(m, bn, st)) != FR_OK) return rc;
  }
  bvh_refit(m, d_verts, st);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t*>(m.depth), 1);
  hipLaunchKernelGGL(k_leaf_depth, dim3(cdiv(F, 256)), dim3(256), 0, st, m.node_parent, m.leaf_parent, F, m.depth);
  int32_t depth = 0;
  if (hipMemcpyAsync(&depth, m.depth, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess) return FR_ERR_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return FR_ERR_DEVICE;
  *depth_out = depth;
  return FR_OK;
}

}  // namespace fr

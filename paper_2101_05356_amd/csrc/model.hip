// Morphable blend (Sec. 3.1, 3.2), rigid pose, vertex normals, Adam
// (Sec. 5), light records, and their adjoints.
#include "fr_kernels.h"

namespace fr {


// ---------------------------------------------------------------------------
// Vertex normals: n_i = N_i / |N_i|, N_i = sum over incident faces of
// (v1 - v0) x (v2 - v0), gathered per vertex through the vertex->face CSR
// (no atomics).  FP64: the edge vectors of a fine mesh are short differences
// of O(1) coordinates, and the normal adjoint sums one-ring terms that largely
// cancel, so FP32 would lose ~1e-5 relative there.
//
// Eight lanes per vertex: lane s of the group takes the incident faces
// s, s + 8, ... (all of them for valence <= 8, so one round of the dependent
// CSR -> face -> vertex loads), and the group sums its partials with a fixed
// xor butterfly, which leaves the same bits in all eight lanes.  A face-scale
// mesh then fills the chip instead of giving each SIMD less than one wave.
// ---------------------------------------------------------------------------
constexpr int kVtxLanes = 8;

__device__ __forceinline__ D3 d3(const float* __restrict__ p, int i) {
  return {(double)p[3 * i], (double)p[3 * i + 1], (double)p[3 * i + 2]};
}
// Sum over the eight lanes of a group; every lane of the wave must call it.
__device__ __forceinline__ D3 group8_sum(D3 a) {
#pragma unroll
  for (int m = 1; m < kVtxLanes; m <<= 1)
    a = a + D3{__shfl_xor(a.x, m, kVtxLanes), __shfl_xor(a.y, m, kVtxLanes), __shfl_xor(a.z, m, kVtxLanes)};
  return a;
}
// Vertex of this lane's group, and the lane's index in the group.
__device__ __forceinline__ int group_vertex(int bid, int& sub) {
  const int t = bid * (int)blockDim.x + (int)threadIdx.x;
  sub = t & (kVtxLanes - 1);
  return t / kVtxLanes;
}
// This lane's share of N_i (zero for lanes past the last vertex).
__device__ __forceinline__ D3 face_normal_part(const float* __restrict__ v, const int32_t* __restrict__ tris,
                                               const int32_t* __restrict__ off, const int32_t* __restrict__ idx,
                                               int N, int i, int sub) {
  D3 acc = {0.0, 0.0, 0.0};
  if (i >= N) return acc;
  const int k1 = off[i + 1];
  for (int k = off[i] + sub; k < k1; k += kVtxLanes) {
    const int f = idx[k];
    const D3 a = d3(v, tris[3 * f]);
    acc = acc + crossd(d3(v, tris[3 * f + 1]) - a, d3(v, tris[3 * f + 2]) - a);
  }
  return acc;
}

__device__ __forceinline__ void normals_block(const float* __restrict__ v, const int32_t* __restrict__ tris,
                                                 const int32_t* __restrict__ off, const int32_t* __restrict__ idx, int N,
                                                 float* __restrict__ n, float* __restrict__ nlen, int bid) {
  int sub;
  const int i = group_vertex(bid, sub);
  const D3 acc = group8_sum(face_normal_part(v, tris, off, idx, N, i, sub));
  if (i >= N || sub != 0) return;
  const double len = sqrt(acc.x * acc.x + acc.y * acc.y + acc.z * acc.z);
  n[3 * i] = (float)(acc.x / len); n[3 * i + 1] = (float)(acc.y / len); n[3 * i + 2] = (float)(acc.z / len);
  nlen[i] = (float)len;
}

__global__ __launch_bounds__(256) void k_normals(const float* __restrict__ v, const int32_t* __restrict__ tris,
                                                 const int32_t* __restrict__ off, const int32_t* __restrict__ idx, int N,
                                                 float* __restrict__ n, float* __restrict__ nlen) {
  normals_block(v, tris, off, idx, N, n, nlen, blockIdx.x);
}

// g_N_i = (I - n n^T) g_n_i / |N_i|, written in place over g_n.  n and |N| are
// recomputed in FP64 from the vertices, by the same group sum as above.
__device__ __forceinline__ void normals_bwd_project_block(const float* __restrict__ v,
                                                             const int32_t* __restrict__ tris,
                                                             const int32_t* __restrict__ off,
                                                             const int32_t* __restrict__ idx, int N,
                                                             const fix_t* __restrict__ gacc,
                                                             float* __restrict__ g, int bid) {
  int sub;
  const int i = group_vertex(bid, sub);
  const D3 acc = group8_sum(face_normal_part(v, tris, off, idx, N, i, sub));
  if (i >= N || sub != 0) return;
  const double len = sqrt(acc.x * acc.x + acc.y * acc.y + acc.z * acc.z);
  const D3 nn = {acc.x / len, acc.y / len, acc.z / len};
  const D3 gg = {from_fix(gacc[3 * i]), from_fix(gacc[3 * i + 1]), from_fix(gacc[3 * i + 2])};
  const double d = nn.x * gg.x + nn.y * gg.y + nn.z * gg.z;
  g[3 * i] = (float)((gg.x - nn.x * d) / len);
  g[3 * i + 1] = (float)((gg.y - nn.y * d) / len);
  g[3 * i + 2] = (float)((gg.z - nn.z * d) / len);
}

__global__ __launch_bounds__(256) void k_normals_bwd_project(const float* __restrict__ v,
                                                             const int32_t* __restrict__ tris,
                                                             const int32_t* __restrict__ off,
                                                             const int32_t* __restrict__ idx, int N,
                                                             const fix_t* __restrict__ gacc,
                                                             float* __restrict__ g) {
  normals_bwd_project_block(v, tris, off, idx, N, gacc, g, blockIdx.x);
}

// For face f with N_f = a x b (a = v1 - v0, b = v2 - v0) and gN = sum of the
// projected gradients of its three vertices: g_a = b x gN, g_b = gN x a;
// vertex 1 gets g_a, vertex 2 gets g_b, vertex 0 gets -(g_a + g_b).
__device__ __forceinline__ void normals_bwd_gather_block(const float* __restrict__ v, const int32_t* __restrict__ tris,
                                                            const int32_t* __restrict__ off,
                                                            const int32_t* __restrict__ idx, int N,
                                                            const float* __restrict__ gN, fix_t* __restrict__ gv,
                                                            int bid) {
  int sub;
  const int i = group_vertex(bid, sub);
  D3 acc = {0.0, 0.0, 0.0};
  if (i < N) {
    const int k1 = off[i + 1];
    for (int k = off[i] + sub; k < k1; k += kVtxLanes) {
      const int f = idx[k];
      const int i0 = tris[3 * f], i1 = tris[3 * f + 1], i2 = tris[3 * f + 2];
      const D3 g = d3(gN, i0) + d3(gN, i1) + d3(gN, i2);
      const D3 p0 = d3(v, i0);
      const D3 a = d3(v, i1) - p0, b = d3(v, i2) - p0;
      const D3 ga = crossd(b, g), gb = crossd(g, a);
      if (i == i0) acc = acc - (ga + gb);
      else if (i == i1) acc = acc + ga;
      else acc = acc + gb;
    }
  }
  acc = group8_sum(acc);
  if (i >= N || sub != 0) return;
  // one lane owns vertex i; atomic all the same: the primary-edge and
  // shadow-edge terms may be adding into the same accumulators concurrently
  atomicAdd(gv + 3 * i, to_fix_d(acc.x)); atomicAdd(gv + 3 * i + 1, to_fix_d(acc.y));
  atomicAdd(gv + 3 * i + 2, to_fix_d(acc.z));
}

__global__ __launch_bounds__(256) void k_normals_bwd_gather(const float* __restrict__ v, const int32_t* __restrict__ tris,
                                                            const int32_t* __restrict__ off,
                                                            const int32_t* __restrict__ idx, int N,
                                                            const float* __restrict__ gN, fix_t* __restrict__ gv) {
  normals_bwd_gather_block(v, tris, off, idx, N, gN, gv, blockIdx.x);
}

int normals_blocks(int N) { return cdiv(N, 256 / kVtxLanes); }

void launch_normals(MeshDev& m, const float* d_verts, hipStream_t st) {
  hipLaunchKernelGGL(k_normals, dim3(normals_blocks(m.N)), dim3(256), 0, st, d_verts, m.tris, m.vf_off, m.vf_idx,
                     m.N, m.normals, m.nlen);
}

void launch_normals_backward(MeshDev& m, const float* d_verts, const fix_t* acc_n, float* gn_tmp, fix_t* acc_v,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_normals_bwd_project, dim3(normals_blocks(m.N)), dim3(256), 0, st, d_verts, m.tris, m.vf_off,
                     m.vf_idx, m.N, acc_n, gn_tmp);
  hipLaunchKernelGGL(k_normals_bwd_gather, dim3(normals_blocks(m.N)), dim3(256), 0, st, d_verts, m.tris, m.vf_off,
                     m.vf_idx, m.N, gn_tmp, acc_v);
}

__device__ __forceinline__ void fix_to_float_block(const fix_t* __restrict__ acc, float* __restrict__ out, int n,
                                                   int bid, const uint32_t* gmax = nullptr) {
  const int i = bid * 256 + threadIdx.x;
  if (i < n) out[i] += (float)(from_fix(acc[i]) / (double)grad_scale(gmax));
}

__global__ __launch_bounds__(256) void k_fix_to_float(const fix_t* __restrict__ acc, float* __restrict__ out, int n,
                                                      const uint32_t* gmax) {
  fix_to_float_block(acc, out, n, blockIdx.x, gmax);
}

void launch_fix_to_float(const fix_t* acc, float* out, int n, hipStream_t st, const uint32_t* gmax) {
  if (n > 0) hipLaunchKernelGGL(k_fix_to_float, dim3(cdiv(n, 256)), dim3(256), 0, st, acc, out, n, gmax);
}

// Maximum of |x| / spp as float bits (non-negative floats order like their
// bits; spp a power of two, so the division is exact): a grid-stride pass,
// the block's maximum through LDS, one atomic per block.
__global__ __launch_bounds__(256) void k_abs_max(const float* __restrict__ x, int n, float inv_spp,
                                                 uint32_t* __restrict__ gmax) {
  __shared__ uint32_t wmax[4];
  uint32_t m = 0u;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float v = fabsf(x[i]);
    if (v == v) m = max(m, __float_as_uint(v));   // NaN left out
  }
  for (int off = 32; off >= 1; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
    const uint32_t q = __float_as_uint(__uint_as_float(m) * inv_spp);
    if (q != 0u) atomicMax(gmax, q);
  }
}

void launch_abs_max(const float* x, int n, int spp, uint32_t* gmax, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_abs_max, dim3(std::min(cdiv(n, 256 * 8), 256)), dim3(256), 0, st, x, n,
                       1.0f / (float)spp, gmax);
}

__global__ __launch_bounds__(256) void k_zero_fix(fix_t* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

void launch_zero_fix(fix_t* p, size_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_zero_fix, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
}

// ---------------------------------------------------------------------------
// Morphable blend: out = mean + sum_k coef_k basis_k (component-major basis).
// HBM-bound GEMV: consecutive threads own consecutive outputs, so every basis
// row is streamed with fully coalesced loads; coefficients are wave-uniform
// scalar loads.  Accumulation order k = 0..K-1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void blend_block(const float* __restrict__ mean, const float* __restrict__ basis,
                                               const float* __restrict__ coef, int K, int M, float* __restrict__ out, int bid) {
  const int m = bid * 256 + threadIdx.x;
  if (m >= M) return;
  float acc = mean[m];
  // loads issued 16 components ahead of the (ordered) accumulation
#pragma unroll 16
  for (int k = 0; k < K; ++k) acc = fmaf(coef[k], __builtin_nontemporal_load(basis + (size_t)k * M + m), acc);
  out[m] = acc;
}

__global__ __launch_bounds__(256) void k_blend(const float* __restrict__ mean, const float* __restrict__ basis,
                                               const float* __restrict__ coef, int K, int M, float* __restrict__ out) {
  blend_block(mean, basis, coef, K, M, out, blockIdx.x);
}

// gcoef[k] += sum_m basis[k][m] gout[m]: one block per component, fixed-order
// tree reduction (deterministic).
__device__ __forceinline__ void blend_bwd_block(const float* __restrict__ basis, const float* __restrict__ gout,
                                                    int M, float* __restrict__ gcoef, int bid) {
  __shared__ float red[1024];
  const int k = bid;
  const float* row = basis + (size_t)k * M;
  float acc = 0.0f;
#pragma unroll 8
  for (int m = threadIdx.x; m < M; m += 1024) acc = fmaf(row[m], gout[m], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) gcoef[k] += red[0];
}

__global__ __launch_bounds__(1024) void k_blend_bwd(const float* __restrict__ basis, const float* __restrict__ gout,
                                                    int M, float* __restrict__ gcoef) {
  blend_bwd_block(basis, gout, M, gcoef, blockIdx.x);
}

void launch_blend(const float* mean, const float* basis, const float* coef, int K, int M, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_blend, dim3(cdiv(M, 256)), dim3(256), 0, st, mean, basis, coef, K, M, out);
}

void launch_blend_backward(const float* basis, const float* gout, int K, int M, float* gcoef, hipStream_t st) {
  hipLaunchKernelGGL(k_blend_bwd, dim3(K), dim3(1024), 0, st, basis, gout, M, gcoef);
}

// ---------------------------------------------------------------------------
// Rigid pose: R = Rz(rz) Ry(ry) Rx(rx), vw = R v + t.
// ---------------------------------------------------------------------------
struct Rot { float m[9]; };

__device__ __forceinline__ void elem_rot(int axis, float ang, bool deriv, float out[9]) {
  const float c = cosf(ang), s = sinf(ang);
  for (int i = 0; i < 9; ++i) out[i] = 0.0f;
  // rotation about `axis` (or its derivative w.r.t. the angle)
  const int a = (axis + 1) % 3, b = (axis + 2) % 3;
  if (!deriv) {
    out[axis * 3 + axis] = 1.0f;
    out[a * 3 + a] = c; out[a * 3 + b] = -s;
    out[b * 3 + a] = s; out[b * 3 + b] = c;
  } else {
    out[a * 3 + a] = -s; out[a * 3 + b] = -c;
    out[b * 3 + a] = c; out[b * 3 + b] = -s;
  }
}

__device__ __forceinline__ void mat3_mul(const float A[9], const float B[9], float C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// R and optionally the three dR/d(angle).
__device__ void pose_matrices(const float* p, float R[9], float dR[3][9], bool want_d) {
  float X[9], Y[9], Z[9], T[9];
  elem_rot(0, p[0], false, X);
  elem_rot(1, p[1], false, Y);
  elem_rot(2, p[2], false, Z);
  mat3_mul(Z, Y, T);
  mat3_mul(T, X, R);
  if (want_d) {
    float D[9], U[9];
    elem_rot(0, p[0], true, D);  mat3_mul(T, D, dR[0]);                    // Rz Ry dRx
    elem_rot(1, p[1], true, D);  mat3_mul(Z, D, U); mat3_mul(U, X, dR[1]);  // Rz dRy Rx
    elem_rot(2, p[2], true, D);  mat3_mul(D, Y, U); mat3_mul(U, X, dR[2]);  // dRz Ry Rx
  }
}

__device__ __forceinline__ void pose_block(const float* __restrict__ v, int N, const float* __restrict__ pose,
                                              float* __restrict__ vw, int bid) {
  const int i = bid * 256 + threadIdx.x;
  if (i >= N) return;
  float R[9], dR[3][9];
  pose_matrices(pose, R, dR, false);
  const V3 p = ld3(v, i);
  vw[3 * i] = R[0] * p.x + R[1] * p.y + R[2] * p.z + pose[3];
  vw[3 * i + 1] = R[3] * p.x + R[4] * p.y + R[5] * p.z + pose[4];
  vw[3 * i + 2] = R[6] * p.x + R[7] * p.y + R[8] * p.z + pose[5];
}

__global__ __launch_bounds__(256) void k_pose(const float* __restrict__ v, int N, const float* __restrict__ pose,
                                              float* __restrict__ vw) {
  pose_block(v, N, pose, vw, blockIdx.x);
}

__device__ __forceinline__ void pose_bwd_v_block(int N, const float* __restrict__ pose, const float* __restrict__ gw,
                                                    float* __restrict__ gv, int bid) {
  const int i = bid * 256 + threadIdx.x;
  if (i >= N) return;
  float R[9], dR[3][9];
  pose_matrices(pose, R, dR, false);
  const V3 g = ld3(gw, i);
  gv[3 * i] += R[0] * g.x + R[3] * g.y + R[6] * g.z;
  gv[3 * i + 1] += R[1] * g.x + R[4] * g.y + R[7] * g.z;
  gv[3 * i + 2] += R[2] * g.x + R[5] * g.y + R[8] * g.z;
}

__global__ __launch_bounds__(256) void k_pose_bwd_v(int N, const float* __restrict__ pose, const float* __restrict__ gw,
                                                    float* __restrict__ gv) {
  pose_bwd_v_block(N, pose, gw, gv, blockIdx.x);
}

// One block: gR = sum_i gw_i v_i^T, gt = sum_i gw_i, then the chain rule
// through the Euler angles.
__device__ __forceinline__ void pose_bwd_p_block(const float* __restrict__ v, int N, const float* __restrict__ pose,
                                                     const float* __restrict__ gw, float* __restrict__ gpose, int bid) {
  __shared__ float red[12][1024];
  float acc[12];
  for (int k = 0; k < 12; ++k) acc[k] = 0.0f;
  for (int i = threadIdx.x; i < N; i += 1024) {
    const V3 g = ld3(gw, i), p = ld3(v, i);
    acc[0] += g.x * p.x; acc[1] += g.x * p.y; acc[2] += g.x * p.z;
    acc[3] += g.y * p.x; acc[4] += g.y * p.y; acc[5] += g.y * p.z;
    acc[6] += g.z * p.x; acc[7] += g.z * p.y; acc[8] += g.z * p.z;
    acc[9] += g.x; acc[10] += g.y; acc[11] += g.z;
  }
  for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 12; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    float R[9], dR[3][9];
    pose_matrices(pose, R, dR, true);
    for (int a = 0; a < 3; ++a) {
      float s = 0.0f;
      for (int k = 0; k < 9; ++k) s += red[k][0] * dR[a][k];
      gpose[a] += s;
    }
    gpose[3] += red[9][0]; gpose[4] += red[10][0]; gpose[5] += red[11][0];
  }
}

__global__ __launch_bounds__(1024) void k_pose_bwd_p(const float* __restrict__ v, int N, const float* __restrict__ pose,
                                                     const float* __restrict__ gw, float* __restrict__ gpose) {
  pose_bwd_p_block(v, N, pose, gw, gpose, blockIdx.x);
}

void launch_pose(const float* v, int N, const float* pose, float* vw, hipStream_t st) {
  hipLaunchKernelGGL(k_pose, dim3(cdiv(N, 256)), dim3(256), 0, st, v, N, pose, vw);
}

void launch_pose_backward(const float* v, int N, const float* pose, const float* gw, float* gv, float* gpose,
                          hipStream_t st) {
  if (gv) hipLaunchKernelGGL(k_pose_bwd_v, dim3(cdiv(N, 256)), dim3(256), 0, st, N, pose, gw, gv);
  if (gpose) hipLaunchKernelGGL(k_pose_bwd_p, dim3(1), dim3(1024), 0, st, v, N, pose, gw, gpose);
}

// ---------------------------------------------------------------------------
// Adam
// ---------------------------------------------------------------------------
__device__ __forceinline__ void adam_block(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ lr, int n, float b1,
                                              float b2, float eps, float c1, float c2, int bid) {
  const int i = bid * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr[i] * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ lr, int n, float b1,
                                              float b2, float eps, float c1, float c2) {
  adam_block(p, g, m, v, lr, n, b1, b2, eps, c1, c2, blockIdx.x);
}

void launch_adam(float* p, const float* g, float* m, float* v, const float* lr, int n, int t, float b1, float b2,
                 float eps, hipStream_t st) {
  const float c1 = adam_bias(b1, t), c2 = adam_bias(b2, t);
  hipLaunchKernelGGL(k_adam, dim3(cdiv(n, 256)), dim3(256), 0, st, p, g, m, v, lr, n, b1, b2, eps, c1, c2);
}

// ---------------------------------------------------------------------------
// Light records: na = -kappa (e1 x e2), kappa = 1 or 1/2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void light_setup_block(const float* __restrict__ p0, const float* __restrict__ e1, const float* __restrict__ e2,
                              const float* __restrict__ rad, const int32_t* __restrict__ shape, int L,
                              LightRec* __restrict__ out, int bid) {
  const int j = bid * blockDim.x + threadIdx.x;
  if (j >= L) return;
  LightRec r;
  for (int k = 0; k < 3; ++k) r.rad[k] = rad[3 * j + k];
  r.shape = shape[j];
  if (r.shape == FR_LIGHT_DIRECTIONAL) {
    const V3 d = ld3(p0, j);
    const float il = 1.0f / sqrtf(dot(d, d));
    r.p0[0] = d.x * il; r.p0[1] = d.y * il; r.p0[2] = d.z * il;
    for (int k = 0; k < 3; ++k) { r.e1[k] = 0.0f; r.e2[k] = 0.0f; r.na[k] = 0.0f; }
    r.e1[0] = il;
  } else {
    const V3 a = ld3(e1, j), b = ld3(e2, j);
    const V3 n = cross(a, b);
    const float kappa = r.shape == FR_LIGHT_TRIANGLE ? 0.5f : 1.0f;
    for (int k = 0; k < 3; ++k) { r.p0[k] = p0[3 * j + k]; r.e1[k] = e1[3 * j + k]; r.e2[k] = e2[3 * j + k]; }
    r.na[0] = -kappa * n.x; r.na[1] = -kappa * n.y; r.na[2] = -kappa * n.z;
  }
  out[j] = r;
}

__global__ void k_light_setup(const float* __restrict__ p0, const float* __restrict__ e1, const float* __restrict__ e2,
                              const float* __restrict__ rad, const int32_t* __restrict__ shape, int L,
                              LightRec* __restrict__ out) {
  light_setup_block(p0, e1, e2, rad, shape, L, out, blockIdx.x);
}

void launch_light_setup(const fr_scene& sc, LightRec* out, hipStream_t st) {
  hipLaunchKernelGGL(k_light_setup, dim3(cdiv(sc.n_lights, 64)), dim3(64), 0, st, sc.light_p0, sc.light_e1,
                     sc.light_e2, sc.light_rad, sc.light_shape, sc.n_lights, out);
}

__device__ __forceinline__ void zero_f32_block(float* __restrict__ p, int n, int bid) {
  const int i = bid * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

__global__ void k_zero_f32(float* __restrict__ p, int n) {
  zero_f32_block(p, n, blockIdx.x);
}

// dst += a s[0] src (s nullable: 1): the sums of loss terms and gradient
// contributions that the optimisation steps compose.
__global__ void k_axpy(float* __restrict__ dst, const float* __restrict__ src, float a, const float* __restrict__ s,
                       int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] += (s ? a * s[0] : a) * src[i];
}

void launch_zero(float* p, int n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_zero_f32, dim3(cdiv(n, 256)), dim3(256), 0, st, p, n);
}

void launch_axpy(float* dst, const float* src, float a, const float* s, int n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_axpy, dim3(cdiv(n, 256)), dim3(256), 0, st, dst, src, a, s, n);
}

// ---------------------------------------------------------------------------
// Per-vertex attribute baked into an M x M texture map (the Stage II maps
// start from the Stage I statistical albedo, Sec. 4 "Stage II"): one thread per
// face tests the texel centres ((i + 1/2)/M, (j + 1/2)/M) of its texture
// triangle's bounding box; a centre is the face's when every edge function
// (counter-clockwise) is positive, or zero on a left or top edge, each edge
// evaluated from its lexicographically lower end so that the two faces of an
// edge get exactly opposite values.  Every texel has at most one owner, so the
// writes never collide.  FP64 throughout.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bake_map(const int32_t* __restrict__ tris, const float* __restrict__ uv, int F,
                                                  const float* __restrict__ attr, int C, int M,
                                                  float* __restrict__ map) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  if (f >= F) return;
  double px[3], py[3];
  int vid[3];
  for (int k = 0; k < 3; ++k) {
    px[k] = uv[6 * f + 2 * k];
    py[k] = uv[6 * f + 2 * k + 1];
    vid[k] = tris[3 * f + k];
  }
  double area = (px[1] - px[0]) * (py[2] - py[0]) - (py[1] - py[0]) * (px[2] - px[0]);
  if (area == 0.0) return;
  if (area < 0.0) {
    double t = px[1]; px[1] = px[2]; px[2] = t;
    t = py[1]; py[1] = py[2]; py[2] = t;
    const int v = vid[1]; vid[1] = vid[2]; vid[2] = v;
    area = -area;
  }
  const double Md = (double)M;
  const int i0 = max(0, (int)floor(fmin(px[0], fmin(px[1], px[2])) * Md - 0.5));
  const int i1 = min(M - 1, (int)ceil(fmax(px[0], fmax(px[1], px[2])) * Md - 0.5));
  const int j0 = max(0, (int)floor(fmin(py[0], fmin(py[1], py[2])) * Md - 0.5));
  const int j1 = min(M - 1, (int)ceil(fmax(py[0], fmax(py[1], py[2])) * Md - 0.5));
  for (int j = j0; j <= j1; ++j) {
    const double cv = ((double)j + 0.5) / Md;
    for (int i = i0; i <= i1; ++i) {
      const double cu = ((double)i + 0.5) / Md;
      double w[3];
      bool in = true;
      for (int k = 0; k < 3; ++k) {
        const int k1 = k == 2 ? 0 : k + 1;
        const double ax = px[k], ay = py[k], bx = px[k1], by = py[k1];
        const bool flip = bx < ax || (bx == ax && by < ay);
        const double lx = flip ? bx : ax, ly = flip ? by : ay, hx = flip ? ax : bx, hy = flip ? ay : by;
        double e = (hx - lx) * (cv - ly) - (hy - ly) * (cu - lx);
        if (flip) e = -e;
        const double dx = bx - ax, dy = by - ay;
        const bool top_left = dy < 0.0 || (dy == 0.0 && dx < 0.0);
        in = in && (e > 0.0 || (e == 0.0 && top_left));
        w[k] = e;
      }
      if (!in) continue;
      // edge k's function weighs the opposite corner (k + 2) % 3
      const double b0 = w[1] / area, b1 = w[2] / area, b2 = w[0] / area;
      for (int c = 0; c < C; ++c)
        map[((size_t)j * M + i) * C + c] = (float)(b0 * (double)attr[(size_t)vid[0] * C + c] +
                                                   b1 * (double)attr[(size_t)vid[1] * C + c] +
                                                   b2 * (double)attr[(size_t)vid[2] * C + c]);
    }
  }
}

void launch_bake_map(const int32_t* tris, const float* uv, int F, const float* attr, int C, int M, float* map,
                     hipStream_t st) {
  if (F > 0) hipLaunchKernelGGL(k_bake_map, dim3(cdiv(F, 256)), dim3(256), 0, st, tris, uv, F, attr, C, M, map);
}

// ---------------------------------------------------------------------------
// Virtual light stage (Sec. 3.3, Eq. lightIntensity): light j on face
// (V0, V1, V2) with (d, a, p1, p2, i).  With C the face's centroid,
// scale = d / |C|, B = V0 + p1 (V1 - V0) + p2 (V2 - V0) and
// s = sqrt(a) scale:  p0 = scale B + s (V0 - C),  e1 = s (V2 - V0),
// e2 = s (V1 - V0) (vertex order reversed: e1 x e2 points at the origin),
// rad = d^2 / a * i.  One thread per light.
// ---------------------------------------------------------------------------
struct StageFace { V3 V0, V1, V2, C, B; float h; };
__device__ __forceinline__ StageFace stage_face(const float* __restrict__ faces, const float* __restrict__ P, int j) {
  StageFace f;
  f.V0 = ld3(faces, 3 * j); f.V1 = ld3(faces, 3 * j + 1); f.V2 = ld3(faces, 3 * j + 2);
  f.C = (f.V0 + f.V1 + f.V2) * (1.0f / 3.0f);
  f.h = sqrtf(dot(f.C, f.C));
  f.B = f.V0 + (f.V1 - f.V0) * P[7 * j + 2] + (f.V2 - f.V0) * P[7 * j + 3];
  return f;
}

__global__ __launch_bounds__(64) void k_light_stage(const float* __restrict__ faces, const float* __restrict__ P, int J,
                                                    float* __restrict__ p0, float* __restrict__ e1,
                                                    float* __restrict__ e2, float* __restrict__ rad,
                                                    int32_t* __restrict__ shape) {
  const int j = blockIdx.x * 64 + threadIdx.x;
  if (j >= J) return;
  const StageFace f = stage_face(faces, P, j);
  const float d = P[7 * j], a = P[7 * j + 1];
  const float scale = d / f.h, s = sqrtf(a) * scale;
  const V3 q0 = f.B * scale + (f.V0 - f.C) * s, u = (f.V2 - f.V0) * s, w = (f.V1 - f.V0) * s;
  const float I = d * d / a;
  if (p0) { p0[3 * j] = q0.x; p0[3 * j + 1] = q0.y; p0[3 * j + 2] = q0.z; }
  if (e1) { e1[3 * j] = u.x; e1[3 * j + 1] = u.y; e1[3 * j + 2] = u.z; }
  if (e2) { e2[3 * j] = w.x; e2[3 * j + 1] = w.y; e2[3 * j + 2] = w.z; }
  if (rad) for (int k = 0; k < 3; ++k) rad[3 * j + k] = I * P[7 * j + 4 + k];
  if (shape) shape[j] = FR_LIGHT_TRIANGLE;
}

__global__ __launch_bounds__(64) void k_light_stage_bwd(const float* __restrict__ faces, const float* __restrict__ P,
                                                        int J, const float* __restrict__ gg,
                                                        const float* __restrict__ gr, float* __restrict__ gP) {
  const int j = blockIdx.x * 64 + threadIdx.x;
  if (j >= J) return;
  const StageFace f = stage_face(faces, P, j);
  const float d = P[7 * j], a = P[7 * j + 1];
  const float ra = sqrtf(a), scale = d / f.h;
  const V3 z = {0.0f, 0.0f, 0.0f};
  const V3 g0 = gg ? ld3(gg, 3 * j) : z, g1 = gg ? ld3(gg, 3 * j + 1) : z, g2 = gg ? ld3(gg, 3 * j + 2) : z;
  // the parts that scale with s = sqrt(a) d / h
  const float gs = dot(g0, f.V0 - f.C) + dot(g1, f.V2 - f.V0) + dot(g2, f.V1 - f.V0);
  float gd = dot(g0, f.B) / f.h + gs * ra / f.h;
  float ga = gs * scale * 0.5f / ra;
  const float gp1 = dot(g0, f.V1 - f.V0) * scale, gp2 = dot(g0, f.V2 - f.V0) * scale;
  float gi[3] = {0.0f, 0.0f, 0.0f};
  if (gr) {
    const float I = d * d / a;
    for (int k = 0; k < 3; ++k) {
      const float g = gr[3 * j + k], i = P[7 * j + 4 + k];
      gd += g * 2.0f * d / a * i;
      ga -= g * I / a * i;
      gi[k] = g * I;
    }
  }
  gP[7 * j] += gd; gP[7 * j + 1] += ga; gP[7 * j + 2] += gp1; gP[7 * j + 3] += gp2;
  for (int k = 0; k < 3; ++k) gP[7 * j + 4 + k] += gi[k];
}

void launch_light_stage(const float* faces, const float* P, int J, float* p0, float* e1, float* e2, float* rad,
                        int32_t* shape, hipStream_t st) {
  hipLaunchKernelGGL(k_light_stage, dim3(cdiv(J, 64)), dim3(64), 0, st, faces, P, J, p0, e1, e2, rad, shape);
}

void launch_light_stage_backward(const float* faces, const float* P, int J, const float* gg, const float* gr,
                                 float* gP, hipStream_t st) {
  hipLaunchKernelGGL(k_light_stage_bwd, dim3(cdiv(J, 64)), dim3(64), 0, st, faces, P, J, gg, gr, gP);
}

}  // namespace fr

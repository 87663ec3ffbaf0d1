// tpmc_bvh.hip -- linear BVH over the triangle mesh, built on the device.
//
// Closest-hit tracing on a triangulation (Sec. II.A) needs an acceleration
// structure; this is an LBVH: 30-bit Morton codes of triangle centroids, a
// stable LSD radix sort (4-bit digits, wave-ballot ranking), the binary radix
// tree of Karras (HPG 2012) and a bottom-up box refit with atomic flags.
// Triangles are then packed in Morton order for locality.
#include <hip/hip_runtime.h>

#include "tpmc_device.hpp"
#include "tpmc_launch.h"

namespace tpmc {

namespace {

constexpr int kSortItems = 4;
constexpr int kSortTile = kBlock * kSortItems;

__device__ __forceinline__ uint32_t spread_bits10(uint32_t v) {
  v = (v * 0x00010001u) & 0xFF0000FFu;
  v = (v * 0x00000101u) & 0x0F00F00Fu;
  v = (v * 0x00000011u) & 0xC30C30C3u;
  v = (v * 0x00000005u) & 0x49249249u;
  return v;
}

__global__ void morton_kernel(const float* __restrict__ xyz, const uint32_t* __restrict__ tri, uint32_t nt, float lox,
                              float loy, float loz, float sx, float sy, float sz, uint32_t* __restrict__ keys,
                              uint32_t* __restrict__ vals) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const uint32_t a = tri[3 * i], b = tri[3 * i + 1], c = tri[3 * i + 2];
  const float cx = (xyz[3 * a] + xyz[3 * b] + xyz[3 * c]) * (1.0f / 3.0f);
  const float cy = (xyz[3 * a + 1] + xyz[3 * b + 1] + xyz[3 * c + 1]) * (1.0f / 3.0f);
  const float cz = (xyz[3 * a + 2] + xyz[3 * b + 2] + xyz[3 * c + 2]) * (1.0f / 3.0f);
  const uint32_t qx = (uint32_t)fminf(fmaxf((cx - lox) * sx, 0.0f), 1023.0f);
  const uint32_t qy = (uint32_t)fminf(fmaxf((cy - loy) * sy, 0.0f), 1023.0f);
  const uint32_t qz = (uint32_t)fminf(fmaxf((cz - loz) * sz, 0.0f), 1023.0f);
  keys[i] = (spread_bits10(qx) << 2) | (spread_bits10(qy) << 1) | spread_bits10(qz);
  vals[i] = i;
}

// ---- stable LSD radix sort, 4-bit digits ----

__global__ void radix_count_kernel(const uint32_t* __restrict__ keys, uint32_t n, int shift,
                                   uint32_t* __restrict__ counts, uint32_t nblocks) {
  __shared__ uint32_t h[16];
  if (threadIdx.x < 16) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kSortTile;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint32_t idx = base + j * kBlock + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 15u], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 16) counts[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of m entries by one workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) scan_kernel(uint32_t* __restrict__ a, uint32_t m) {
  __shared__ uint32_t s[1024];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < m; base += 1024) {
    const uint32_t idx = base + threadIdx.x;
    const uint32_t v = idx < m ? a[idx] : 0u;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const uint32_t add = threadIdx.x >= (uint32_t)o ? s[threadIdx.x - o] : 0u;
      __syncthreads();
      s[threadIdx.x] += add;
      __syncthreads();
    }
    const uint32_t incl = s[threadIdx.x];
    if (idx < m) a[idx] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += incl;
    __syncthreads();
  }
}

__global__ void radix_scatter_kernel(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                     uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, uint32_t n, int shift,
                                     const uint32_t* __restrict__ offsets, uint32_t nblocks) {
  __shared__ uint32_t run[16];
  __shared__ uint32_t wc[kBlock / 64][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < 16) run[threadIdx.x] = offsets[threadIdx.x * nblocks + blockIdx.x];
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  const uint32_t base = blockIdx.x * kSortTile;
  for (int j = 0; j < kSortItems; ++j) {
    if (threadIdx.x < kBlock / 64 * 16) wc[threadIdx.x >> 4][threadIdx.x & 15] = 0;
    __syncthreads();
    const uint32_t idx = base + j * kBlock + threadIdx.x;
    const bool valid = idx < n;
    const uint32_t key = valid ? kin[idx] : 0u;
    const uint32_t d = (key >> shift) & 15u;
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint64_t bal = __ballot(valid && ((d >> b) & 1u));
      same &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t rank = __popcll(same & lt_mask);
    if (valid && rank == 0) wc[wave][d] = __popcll(same);
    __syncthreads();
    if (threadIdx.x < 16) {
      uint32_t r = run[threadIdx.x];
      for (int w = 0; w < kBlock / 64; ++w) {
        const uint32_t c = wc[w][threadIdx.x];
        wc[w][threadIdx.x] = r;
        r += c;
      }
      run[threadIdx.x] = r;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = wc[wave][d] + rank;
      kout[pos] = key;
      vout[pos] = vin[idx];
    }
    __syncthreads();
  }
}

// ---- Karras (2012) binary radix tree over sorted unique keys ----

__device__ __forceinline__ int common_prefix(const uint32_t* __restrict__ k, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  const uint32_t a = k[i], b = k[j];
  if (a == b) return 32 + __clz((uint32_t)(i ^ j));
  return __clz(a ^ b);
}

__global__ void karras_kernel(const uint32_t* __restrict__ keys, int n, Node* __restrict__ nodes,
                              int32_t* __restrict__ leaf_parent) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  const int d = (common_prefix(keys, n, i, i + 1) - common_prefix(keys, n, i, i - 1)) >= 0 ? 1 : -1;
  const int dmin = common_prefix(keys, n, i, i - d);
  int lmax = 2;
  while (common_prefix(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int l = 0;
  for (int t = lmax >> 1; t >= 1; t >>= 1)
    if (common_prefix(keys, n, i, i + (l + t) * d) > dmin) l += t;
  const int j = i + l * d;
  const int dnode = common_prefix(keys, n, i, j);
  int s = 0;
  int div = 2;
  int t;
  do {
    t = (l + div - 1) / div;
    if (common_prefix(keys, n, i, i + (s + t) * d) > dnode) s += t;
    div <<= 1;
  } while (t > 1);
  const int split = i + s * d + (d < 0 ? -1 : 0);
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  int c0, c1;
  if (lo == split) {
    c0 = ~split;
    leaf_parent[split] = i;
  } else {
    c0 = split;
    nodes[split].parent = i;
  }
  if (hi == split + 1) {
    c1 = ~(split + 1);
    leaf_parent[split + 1] = i;
  } else {
    c1 = split + 1;
    nodes[split + 1].parent = i;
  }
  nodes[i].c0 = c0;
  nodes[i].c1 = c1;
  if (i == 0) nodes[0].parent = -1;
}

// Pack triangles in Morton order with their unit normals (computed in FP64).
__global__ void pack_tris_kernel(const float* __restrict__ xyz, const uint32_t* __restrict__ tri,
                                 const uint32_t* __restrict__ order, uint32_t nt, TriRec* __restrict__ recs,
                                 uint32_t* __restrict__ orig) {
  // Products evaluated without contraction: a component that is exactly zero
  // (e.g. a vertical face) stays zero instead of becoming an FMA residue whose
  // sign would choose a different tangent basis at re-emission.
#pragma clang fp contract(off)
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nt) return;
  const uint32_t id = order[k];
  const uint32_t a = tri[3 * id], b = tri[3 * id + 1], c = tri[3 * id + 2];
  TriRec r;
  r.v0x = xyz[3 * a]; r.v0y = xyz[3 * a + 1]; r.v0z = xyz[3 * a + 2];
  r.v1x = xyz[3 * b]; r.v1y = xyz[3 * b + 1]; r.v1z = xyz[3 * b + 2];
  r.v2x = xyz[3 * c]; r.v2y = xyz[3 * c + 1]; r.v2z = xyz[3 * c + 2];
  const double e1x = (double)r.v1x - r.v0x, e1y = (double)r.v1y - r.v0y, e1z = (double)r.v1z - r.v0z;
  const double e2x = (double)r.v2x - r.v0x, e2y = (double)r.v2y - r.v0y, e2z = (double)r.v2z - r.v0z;
  double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const double len = sqrt(nx * nx + ny * ny + nz * nz);
  const double inv = len > 0.0 ? 1.0 / len : 0.0;
  r.nx = (float)(nx * inv);
  r.ny = (float)(ny * inv);
  r.nz = (float)(nz * inv);
  recs[k] = r;
  orig[k] = id;
}

// Supporting-plane flags, used to resolve the segment that leaves a hit
// without tracing it.  For triangle k (Morton order) with exact plane
// through v0 and normal n = (v1 - v0) x (v2 - v0) / |...|: bit 30 of orig[k]
// when no mesh vertex lies above the plane by more than tol, bit 31 when none
// lies below it by more than tol, tol = 2^-22 max|coordinate of triangle k|.
// A particle re-emitted from k leaves from a point 8 ulps of that scale (at
// least 5 once the rounding of the hit point is counted) above the plane on
// its emission side and moves away from the plane (or parallel to it), so
// when the mesh lies within tol of the other side, the outgoing ray cannot hit
// anything: every mesh point is below its starting height.  FP64 distances
// over all vertices, tiled through LDS.
__global__ __launch_bounds__(kBlock) void support_kernel(const float* __restrict__ xyz, uint32_t nv,
                                                         const TriRec* __restrict__ tris, uint32_t nt,
                                                         uint32_t* __restrict__ orig) {
  __shared__ float vx[kBlock], vy[kBlock], vz[kBlock];
  const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
  const TriRec t = tris[k < nt ? k : nt - 1];
  const double ox = t.v0x, oy = t.v0y, oz = t.v0z;
  const double e1x = (double)t.v1x - ox, e1y = (double)t.v1y - oy, e1z = (double)t.v1z - oz;
  const double e2x = (double)t.v2x - ox, e2y = (double)t.v2y - oy, e2z = (double)t.v2z - oz;
  double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const double len = sqrt(nx * nx + ny * ny + nz * nz);
  const double inv = len > 0.0 ? 1.0 / len : 0.0;
  nx *= inv;
  ny *= inv;
  nz *= inv;
  double hi = -__builtin_inf(), lo = __builtin_inf();
  for (uint32_t base = 0; base < nv; base += kBlock) {
    const uint32_t i = base + threadIdx.x;
    __syncthreads();
    if (i < nv) {
      vx[threadIdx.x] = xyz[3ull * i];
      vy[threadIdx.x] = xyz[3ull * i + 1];
      vz[threadIdx.x] = xyz[3ull * i + 2];
    }
    __syncthreads();
    const uint32_t m = nv - base < (uint32_t)kBlock ? nv - base : (uint32_t)kBlock;
    for (uint32_t j = 0; j < m; ++j) {
      const double d = nx * ((double)vx[j] - ox) + ny * ((double)vy[j] - oy) + nz * ((double)vz[j] - oz);
      hi = fmax(hi, d);
      lo = fmin(lo, d);
    }
  }
  if (k >= nt || len == 0.0) return;  // zero-area triangles are never hit
  const float sc = fmaxf(fmaxf(fmaxf(fabsf(t.v0x), fabsf(t.v0y)), fmaxf(fabsf(t.v0z), fabsf(t.v1x))),
                         fmaxf(fmaxf(fabsf(t.v1y), fabsf(t.v1z)), fmaxf(fmaxf(fabsf(t.v2x), fabsf(t.v2y)), fabsf(t.v2z))));
  const double tol = ldexp((double)sc, -22);
  uint32_t w = orig[k];
  if (hi <= tol) w |= 1u << 30;
  if (lo >= -tol) w |= 1u << 31;
  orig[k] = w;
}

__device__ __forceinline__ float ld_relaxed(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void child_box(const Node* nodes, const float* nbox, const TriRec* tris, int c, float b[6]) {
  if (c < 0) {
    const TriRec& t = tris[~c];
    b[0] = fminf(fminf(t.v0x, t.v1x), t.v2x);
    b[1] = fminf(fminf(t.v0y, t.v1y), t.v2y);
    b[2] = fminf(fminf(t.v0z, t.v1z), t.v2z);
    b[3] = fmaxf(fmaxf(t.v0x, t.v1x), t.v2x);
    b[4] = fmaxf(fmaxf(t.v0y, t.v1y), t.v2y);
    b[5] = fmaxf(fmaxf(t.v0z, t.v1z), t.v2z);
  } else {
    for (int k = 0; k < 6; ++k) b[k] = ld_relaxed(nbox + 6 * c + k);
  }
}

// Bottom-up refit: one thread per leaf climbs; the second thread to reach a
// node writes its children's boxes and continues upward.
__global__ void refit_kernel(Node* __restrict__ nodes, const int32_t* __restrict__ leaf_parent,
                             const TriRec* __restrict__ tris, uint32_t nt, uint32_t* __restrict__ flags,
                             float* __restrict__ nbox) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nt) return;
  int p = leaf_parent[k];
  for (int level = 0; p >= 0 && level < 4096; ++level) {  // bounded climb
    __threadfence();
    if (atomicAdd(&flags[p], 1u) == 0u) return;
    __threadfence();
    const int c0 = __hip_atomic_load(&nodes[p].c0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int c1 = __hip_atomic_load(&nodes[p].c1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    float b0[6], b1[6];
    child_box(nodes, nbox, tris, c0, b0);
    child_box(nodes, nbox, tris, c1, b1);
    Node& nd = nodes[p];
    nd.lo0x = b0[0]; nd.lo0y = b0[1]; nd.lo0z = b0[2]; nd.hi0x = b0[3]; nd.hi0y = b0[4]; nd.hi0z = b0[5];
    nd.lo1x = b1[0]; nd.lo1y = b1[1]; nd.lo1z = b1[2]; nd.hi1x = b1[3]; nd.hi1y = b1[4]; nd.hi1z = b1[5];
    for (int q = 0; q < 3; ++q) {
      __hip_atomic_store(nbox + 6 * p + q, fminf(b0[q], b1[q]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(nbox + 6 * p + 3 + q, fmaxf(b0[3 + q], b1[3 + q]), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    p = __hip_atomic_load(&nodes[p].parent, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Depth of every leaf (root = depth 0), maximum kept.
__global__ void depth_kernel(const Node* __restrict__ nodes, const int32_t* __restrict__ leaf_parent, uint32_t nt,
                             uint32_t* __restrict__ max_depth) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nt) return;
  uint32_t dpt = 0;
  int p = leaf_parent[k];
  while (p >= 0 && dpt < 4096) {  // bounded climb
    ++dpt;
    p = nodes[p].parent;
  }
  atomicMax(max_depth, dpt);
}

// One-triangle mesh: a single node whose two links both name leaf 0.
__global__ void single_node_kernel(Node* nodes, const TriRec* tris) {
  const TriRec& t = tris[0];
  Node nd;
  nd.lo0x = nd.lo1x = fminf(fminf(t.v0x, t.v1x), t.v2x);
  nd.lo0y = nd.lo1y = fminf(fminf(t.v0y, t.v1y), t.v2y);
  nd.lo0z = nd.lo1z = fminf(fminf(t.v0z, t.v1z), t.v2z);
  nd.hi0x = nd.hi1x = fmaxf(fmaxf(t.v0x, t.v1x), t.v2x);
  nd.hi0y = nd.hi1y = fmaxf(fmaxf(t.v0y, t.v1y), t.v2y);
  nd.hi0z = nd.hi1z = fmaxf(fmaxf(t.v0z, t.v1z), t.v2z);
  nd.c0 = ~0;
  nd.c1 = ~0;
  nd.parent = -1;
  nd.pad = 0;
  nodes[0] = nd;
}


// ---- top-down binned SAH build ----
//
// Alternative to the Morton/Karras hierarchy, same node and leaf format.  A
// node's triangles (a contiguous range of an index array) are split where the
// surface-area heuristic (cost of a child = its box area x its triangle count)
// is lowest among kSahBins - 1 planes per axis, planes equally spaced over the
// range of the triangle box centres; the range is then partitioned stably into
// the other index array.  One workgroup per node, all nodes of one tree level
// per launch.  Internal node ids follow Karras's rule, valid for any binary
// tree over ordered leaves: the root is 0, an internal left child takes the
// position of its last triangle and an internal right child that of its first,
// so ids are known before the children are processed and the build is
// deterministic.  Below level kSahMaxLevel (or when every centre coincides)
// ranges are halved by position, so no leaf lies deeper than
// kSahMaxLevel + 30 <= 64 for nt < 2^30.
constexpr int kSahBins = 32;
constexpr uint32_t kSahMaxLevel = 32;

struct SahTask {
  uint32_t a, b, id;  // triangle positions [a, b] (b > a), node id
  int32_t parent;
};

// Order-preserving map of finite floats to int32 (for LDS integer min / max).
__device__ __forceinline__ int f2o(float f) {
  const int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float o2f(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7FFFFFFF); }

__device__ __forceinline__ int sah_bin(float c, float cmin, float scale) {
  return min(kSahBins - 1, (int)((c - cmin) * scale));
}

__device__ __forceinline__ float box_area(float lx, float ly, float lz, float hx, float hy, float hz) {
  const float ex = hx - lx, ey = hy - ly, ez = hz - lz;
  return ex * ey + ey * ez + ez * ex;
}

// Triangle boxes (exact min / max of the FP32 vertices); the box centre is the
// binning key.
__global__ void prim_box_kernel(const float* __restrict__ xyz, const uint32_t* __restrict__ tri, uint32_t nt,
                                float4* __restrict__ plo, float4* __restrict__ phi, uint32_t* __restrict__ idx) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const uint32_t a = tri[3 * i], b = tri[3 * i + 1], c = tri[3 * i + 2];
  float lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float x = xyz[3 * a + k], y = xyz[3 * b + k], z = xyz[3 * c + k];
    lo[k] = fminf(fminf(x, y), z);
    hi[k] = fmaxf(fmaxf(x, y), z);
  }
  plo[i] = make_float4(lo[0], lo[1], lo[2], 0.0f);
  phi[i] = make_float4(hi[0], hi[1], hi[2], 0.0f);
  idx[i] = i;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

__global__ __launch_bounds__(kBlock) void sah_level_kernel(const float4* __restrict__ plo,
                                                          const float4* __restrict__ phi,
                                                          const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                          uint32_t* __restrict__ order, const SahTask* __restrict__ tasks,
                                                          uint32_t ntasks, SahTask* __restrict__ next,
                                                          uint32_t* __restrict__ nnext, Node* __restrict__ nodes,
                                                          uint32_t level, uint32_t* __restrict__ err) {
  __shared__ int s_cb[6];  // centre bounds: lo xyz, hi xyz (ordered ints)
  __shared__ uint32_t s_cnt[3][kSahBins];
  __shared__ int s_lo[3][kSahBins][3], s_hi[3][kSahBins][3];
  __shared__ unsigned long long s_best;
  __shared__ int s_box[2][6];  // child boxes: lo xyz, hi xyz
  __shared__ uint32_t s_wl[kBlock / 64], s_wv[kBlock / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  constexpr float kInf = __builtin_inff();

  for (uint32_t ti = blockIdx.x; ti < ntasks; ti += gridDim.x) {
    const SahTask T = tasks[ti];
    const uint32_t a = T.a, b = T.b, m = b - a + 1;

    // 1. bounds of the box centres
    if (tid < 6) s_cb[tid] = tid < 3 ? f2o(kInf) : f2o(-kInf);
    if (tid < 12) s_box[tid / 6][tid % 6] = tid % 6 < 3 ? f2o(kInf) : f2o(-kInf);
    for (int e = tid; e < 3 * kSahBins; e += kBlock) {
      (&s_cnt[0][0])[e] = 0u;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        (&s_lo[0][0][0])[3 * e + q] = f2o(kInf);
        (&s_hi[0][0][0])[3 * e + q] = f2o(-kInf);
      }
    }
    if (tid == 0) s_best = ~0ull;
    float cl[3] = {kInf, kInf, kInf}, ch[3] = {-kInf, -kInf, -kInf};
    for (uint32_t i = a + tid; i <= b; i += kBlock) {
      const uint32_t p = src[i];
      const float4 lo = plo[p], hi = phi[p];
      const float c[3] = {0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z)};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        cl[k] = fminf(cl[k], c[k]);
        ch[k] = fmaxf(ch[k], c[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cl[k] = wave_min(cl[k]);
      ch[k] = wave_max(ch[k]);
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        atomicMin(&s_cb[k], f2o(cl[k]));
        atomicMax(&s_cb[3 + k], f2o(ch[k]));
      }
    }
    __syncthreads();
    float cmin[3], scale[3];
    bool use[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cmin[k] = o2f(s_cb[k]);
      const float ext = o2f(s_cb[3 + k]) - cmin[k];
      scale[k] = (float)kSahBins / ext;
      use[k] = level < kSahMaxLevel && ext > 0.0f && scale[k] < kInf;
    }

    // 2. bins of every usable axis: count and box union
    if (use[0] || use[1] || use[2]) {
      for (uint32_t i = a + tid; i <= b; i += kBlock) {
        const uint32_t p = src[i];
        const float4 lo = plo[p], hi = phi[p];
        const float c[3] = {0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z)};
        const int ilo[3] = {f2o(lo.x), f2o(lo.y), f2o(lo.z)}, ihi[3] = {f2o(hi.x), f2o(hi.y), f2o(hi.z)};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if (!use[k]) continue;
          const int bin = sah_bin(c[k], cmin[k], scale[k]);
          atomicAdd(&s_cnt[k][bin], 1u);
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            atomicMin(&s_lo[k][bin][q], ilo[q]);
            atomicMax(&s_hi[k][bin][q], ihi[q]);
          }
        }
      }
      __syncthreads();
      // 3. cost of every plane (axis k, left = bins below s); lowest (cost, k, s) wins
      if (tid < 3 * kSahBins) {
        const int k = tid / kSahBins, s = tid % kSahBins;
        if (s > 0 && use[k]) {
          uint32_t nl = 0, nr = 0;
          int L[6] = {f2o(kInf), f2o(kInf), f2o(kInf), f2o(-kInf), f2o(-kInf), f2o(-kInf)};
          int R[6] = {L[0], L[1], L[2], L[3], L[4], L[5]};
          for (int j = 0; j < s; ++j) {
            nl += s_cnt[k][j];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              L[q] = min(L[q], s_lo[k][j][q]);
              L[3 + q] = max(L[3 + q], s_hi[k][j][q]);
            }
          }
          for (int j = s; j < kSahBins; ++j) {
            nr += s_cnt[k][j];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              R[q] = min(R[q], s_lo[k][j][q]);
              R[3 + q] = max(R[3 + q], s_hi[k][j][q]);
            }
          }
          if (nl > 0 && nr > 0) {
            const float cost =
                box_area(o2f(L[0]), o2f(L[1]), o2f(L[2]), o2f(L[3]), o2f(L[4]), o2f(L[5])) * (float)nl +
                box_area(o2f(R[0]), o2f(R[1]), o2f(R[2]), o2f(R[3]), o2f(R[4]), o2f(R[5])) * (float)nr;
            atomicMin(&s_best, ((unsigned long long)__float_as_uint(cost) << 32) | (unsigned)tid);
          }
        }
      }
    }
    __syncthreads();
    const unsigned long long best = s_best;
    const bool halve = best == ~0ull;
    int ax = 0, split = 0;
    uint32_t nl = m / 2;
    if (!halve) {
      const int t = (int)(best & 0xFFFFFFFFull);
      ax = t / kSahBins;
      split = t % kSahBins;
      nl = 0;
      for (int j = 0; j < split; ++j) nl += s_cnt[ax][j];
    }

    // 4. stable partition into dst[a..b]: left part first; child boxes
    float bl[2][3] = {{kInf, kInf, kInf}, {kInf, kInf, kInf}};
    float bh[2][3] = {{-kInf, -kInf, -kInf}, {-kInf, -kInf, -kInf}};
    uint32_t baseL = 0, baseR = 0;
    for (uint32_t c0 = a; c0 <= b; c0 += kBlock) {
      const uint32_t i = c0 + tid;
      const bool valid = i <= b;
      uint32_t p = 0;
      bool left = false;
      if (valid) {
        p = src[i];
        const float4 lo = plo[p], hi = phi[p];
        if (halve) {
          left = i - a < nl;
        } else {
          const float c = ax == 0 ? 0.5f * (lo.x + hi.x) : ax == 1 ? 0.5f * (lo.y + hi.y) : 0.5f * (lo.z + hi.z);
          left = sah_bin(c, cmin[ax], scale[ax]) < split;
        }
        const int side = left ? 0 : 1;
        bl[side][0] = fminf(bl[side][0], lo.x); bl[side][1] = fminf(bl[side][1], lo.y);
        bl[side][2] = fminf(bl[side][2], lo.z);
        bh[side][0] = fmaxf(bh[side][0], hi.x); bh[side][1] = fmaxf(bh[side][1], hi.y);
        bh[side][2] = fmaxf(bh[side][2], hi.z);
      }
      const unsigned long long wl = __ballot(left), wv = __ballot(valid);
      if (lane == 0) {
        s_wl[wave] = (uint32_t)__popcll(wl);
        s_wv[wave] = (uint32_t)__popcll(wv);
      }
      __syncthreads();
      uint32_t offL = 0, offV = 0, totL = 0, totV = 0;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wave) {
          offL += s_wl[w];
          offV += s_wv[w];
        }
        totL += s_wl[w];
        totV += s_wv[w];
      }
      if (valid) {
        const uint32_t pl = (uint32_t)__popcll(wl & lt_mask), pv = (uint32_t)__popcll(wv & lt_mask);
        const uint32_t pos = left ? a + baseL + offL + pl : a + nl + baseR + (offV - offL) + (pv - pl);
        if (pos >= a && pos <= b) {
          dst[pos] = p;
          if (left ? nl == 1 : m - nl == 1) order[pos] = p;  // a one-triangle child is a leaf
        }
      }
      baseL += totL;
      baseR += totV - totL;
      __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        bl[s][q] = wave_min(bl[s][q]);
        bh[s][q] = wave_max(bh[s][q]);
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          atomicMin(&s_box[s][q], f2o(bl[s][q]));
          atomicMax(&s_box[s][3 + q], f2o(bh[s][q]));
        }
      }
    }
    __syncthreads();

    // 5. the node, its internal children as tasks of the next level
    if (tid == 0) {
      if (baseL != nl) atomicOr(err, 1u);  // partition disagrees with the bin counts
      const uint32_t nr = m - nl;
      const int c0 = nl == 1 ? ~(int)a : (int)(a + nl - 1);
      const int c1 = nr == 1 ? ~(int)b : (int)(a + nl);
      Node nd;
      nd.lo0x = o2f(s_box[0][0]); nd.lo0y = o2f(s_box[0][1]); nd.lo0z = o2f(s_box[0][2]);
      nd.hi0x = o2f(s_box[0][3]); nd.hi0y = o2f(s_box[0][4]); nd.hi0z = o2f(s_box[0][5]);
      nd.lo1x = o2f(s_box[1][0]); nd.lo1y = o2f(s_box[1][1]); nd.lo1z = o2f(s_box[1][2]);
      nd.hi1x = o2f(s_box[1][3]); nd.hi1y = o2f(s_box[1][4]); nd.hi1z = o2f(s_box[1][5]);
      nd.c0 = c0;
      nd.c1 = c1;
      nd.parent = T.parent;
      nd.pad = 0;
      nodes[T.id] = nd;
      const uint32_t k = (nl > 1 ? 1u : 0u) + (nr > 1 ? 1u : 0u);
      if (k) {
        uint32_t slot = atomicAdd(nnext, k);
        if (nl > 1) next[slot++] = SahTask{a, a + nl - 1, a + nl - 1, (int32_t)T.id};
        if (nr > 1) next[slot] = SahTask{a + nl, b, a + nl, (int32_t)T.id};
      }
    }
    __syncthreads();  // LDS is reused by the next task
  }
}

__global__ void sah_root_kernel(SahTask* tasks, uint32_t nt) { tasks[0] = SahTask{0u, nt - 1u, 0u, -1}; }

}  // namespace

void mark_support(const float* d_xyz, uint64_t nv, const TriRec* d_tris, uint64_t nt, uint32_t* d_orig,
                  hipStream_t st) {
  support_kernel<<<(unsigned)((nt + kBlock - 1) / kBlock), kBlock, 0, st>>>(d_xyz, (uint32_t)nv, d_tris,
                                                                           (uint32_t)nt, d_orig);
}

size_t bvh_scratch_bytes(uint64_t nt) {
  const uint64_t nblocks = (nt + kSortTile - 1) / kSortTile;
  // xyz/tri copies are separate; here: keys x2, vals x2, counts, leaf_parent, flags, nbox, depth
  return (4 * nt + 16 * nblocks + 2 * nt + 6 * nt + 64) * sizeof(uint32_t) + 4096;
}

hipError_t build_bvh(const float* d_xyz, const uint32_t* d_tri, uint64_t nt64, const float box_lo[3],
                     const float box_hi[3], void* scratch, Node* d_nodes, TriRec* d_tris, uint32_t* d_orig,
                     uint32_t* h_depth, hipStream_t st) {
  const uint32_t nt = (uint32_t)nt64;
  const uint32_t nblocks = (nt + kSortTile - 1) / kSortTile;
  uint32_t* k0 = static_cast<uint32_t*>(scratch);
  uint32_t* v0 = k0 + nt;
  uint32_t* k1 = v0 + nt;
  uint32_t* v1 = k1 + nt;
  uint32_t* counts = v1 + nt;
  int32_t* leaf_parent = reinterpret_cast<int32_t*>(counts + 16 * nblocks);
  uint32_t* flags = reinterpret_cast<uint32_t*>(leaf_parent + nt);
  float* nbox = reinterpret_cast<float*>(flags + nt);
  uint32_t* depth = reinterpret_cast<uint32_t*>(nbox + 6 * nt);

  float ext[3], sc[3];
  for (int k = 0; k < 3; ++k) {
    ext[k] = box_hi[k] - box_lo[k];
    sc[k] = ext[k] > 0.0f ? 1024.0f / ext[k] : 0.0f;
  }
  const uint32_t g = (nt + kBlock - 1) / kBlock;
  morton_kernel<<<g, kBlock, 0, st>>>(d_xyz, d_tri, nt, box_lo[0], box_lo[1], box_lo[2], sc[0], sc[1], sc[2], k0, v0);
  for (int shift = 0; shift < 30; shift += 4) {
    radix_count_kernel<<<nblocks, kBlock, 0, st>>>(k0, nt, shift, counts, nblocks);
    scan_kernel<<<1, 1024, 0, st>>>(counts, 16 * nblocks);
    radix_scatter_kernel<<<nblocks, kBlock, 0, st>>>(k0, v0, k1, v1, nt, shift, counts, nblocks);
    uint32_t* t = k0; k0 = k1; k1 = t;
    t = v0; v0 = v1; v1 = t;
  }
  pack_tris_kernel<<<g, kBlock, 0, st>>>(d_xyz, d_tri, v0, nt, d_tris, d_orig);
  hipError_t e;
  if (nt == 1) {
    single_node_kernel<<<1, 1, 0, st>>>(d_nodes, d_tris);
    *h_depth = 1;
    e = hipStreamSynchronize(st);
    return e != hipSuccess ? e : hipGetLastError();
  }
  zero_u32(flags, nt, st);
  zero_u32(depth, 1, st);
  e = hipMemsetAsync(leaf_parent, 0xFF, nt * sizeof(int32_t), st);  // -1: no parent yet
  if (e != hipSuccess) return e;
  const uint32_t gi = (nt - 1 + kBlock - 1) / kBlock;
  karras_kernel<<<gi, kBlock, 0, st>>>(k0, (int)nt, d_nodes, leaf_parent);
  refit_kernel<<<g, kBlock, 0, st>>>(d_nodes, leaf_parent, d_tris, nt, flags, nbox);
  depth_kernel<<<g, kBlock, 0, st>>>(d_nodes, leaf_parent, nt, depth);
  e = hipMemcpyAsync(h_depth, depth, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  return e != hipSuccess ? e : hipGetLastError();
}

size_t sah_scratch_bytes(uint64_t nt) {
  // prim boxes (2 x 16 B), two index arrays and the leaf order (3 x 4 B), two
  // task lists of at most nt / 2 + 1 entries (16 B), two counters
  return nt * (2 * sizeof(float4) + 3 * sizeof(uint32_t)) + 2 * (nt / 2 + 1) * sizeof(SahTask) + 4096;
}

hipError_t build_bvh_sah(const float* d_xyz, const uint32_t* d_tri, uint64_t nt64, void* scratch, Node* d_nodes,
                         TriRec* d_tris, uint32_t* d_orig, uint32_t* h_depth, hipStream_t st) {
  const uint32_t nt = (uint32_t)nt64;
  char* p = static_cast<char*>(scratch);
  auto take = [&p](size_t bytes) {
    char* q = p;
    p += (bytes + 255) & ~size_t(255);
    return q;
  };
  float4* plo = reinterpret_cast<float4*>(take(nt * sizeof(float4)));
  float4* phi = reinterpret_cast<float4*>(take(nt * sizeof(float4)));
  uint32_t* idx[2] = {reinterpret_cast<uint32_t*>(take(nt * sizeof(uint32_t))),
                      reinterpret_cast<uint32_t*>(take(nt * sizeof(uint32_t)))};
  uint32_t* order = reinterpret_cast<uint32_t*>(take(nt * sizeof(uint32_t)));
  const size_t ntask = nt / 2 + 1;
  SahTask* tasks[2] = {reinterpret_cast<SahTask*>(take(ntask * sizeof(SahTask))),
                       reinterpret_cast<SahTask*>(take(ntask * sizeof(SahTask)))};
  uint32_t* cnt = reinterpret_cast<uint32_t*>(take(2 * sizeof(uint32_t)));  // next-level tasks, error flag
  const uint32_t g = (nt + kBlock - 1) / kBlock;
  hipError_t e;
  prim_box_kernel<<<g, kBlock, 0, st>>>(d_xyz, d_tri, nt, plo, phi, idx[0]);
  if (nt == 1) {
    pack_tris_kernel<<<1, kBlock, 0, st>>>(d_xyz, d_tri, idx[0], 1u, d_tris, d_orig);
    single_node_kernel<<<1, 1, 0, st>>>(d_nodes, d_tris);
    *h_depth = 1;
    e = hipStreamSynchronize(st);
    return e != hipSuccess ? e : hipGetLastError();
  }
  zero_u32(cnt, 2, st);
  sah_root_kernel<<<1, 1, 0, st>>>(tasks[0], nt);
  uint32_t ntasks = 1, level = 0, h_cnt[2] = {0u, 0u};
  while (ntasks > 0) {
    if (level >= 64) return hipErrorUnknown;  // cannot happen: see kSahMaxLevel
    zero_u32(cnt, 1, st);
    const uint32_t grid = ntasks < 2048u ? ntasks : 2048u;
    sah_level_kernel<<<grid, kBlock, 0, st>>>(plo, phi, idx[level & 1], idx[(level + 1) & 1], order, tasks[level & 1],
                                              ntasks, tasks[(level + 1) & 1], cnt, d_nodes, level, cnt + 1);
    e = hipMemcpyAsync(h_cnt, cnt, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (h_cnt[1] != 0u) return hipErrorUnknown;  // partition inconsistent with the bin counts
    ntasks = h_cnt[0];
    ++level;
  }
  *h_depth = level;  // internal nodes on the longest root-to-leaf path
  pack_tris_kernel<<<g, kBlock, 0, st>>>(d_xyz, d_tri, order, nt, d_tris, d_orig);
  e = hipStreamSynchronize(st);
  return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace tpmc

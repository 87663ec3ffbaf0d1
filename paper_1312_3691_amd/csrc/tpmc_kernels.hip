// tpmc_kernels.hip -- the per-query hot path on gfx950:
//   seed_kernel     a2-a4  Philox streams, FP64 boundary seeding -> FP32 SoA
//   trace_kernel    a6-a9  BVH traversal, watertight hit, re-emission, tallies, bounce loop
//   batch_kernel    a11    persistent (query, tile) work queue; seeding fused on chip
//   reduce/finalize a10    exact integer reduction, force / moment / C_D in FP64
#include <hip/hip_runtime.h>

#include "tpmc_device.hpp"
#include "tpmc_launch.h"

namespace tpmc {

namespace {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
__global__ void zero_i64_kernel(long long* __restrict__ p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void zero_u32_kernel(uint32_t* __restrict__ p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

int grid_for(uint64_t n, int cap) {
  const uint64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < (uint64_t)cap ? (g > 0 ? g : 1) : cap);
}

// ---------------------------------------------------------------------------
// a2-a4: seeding
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void seed_kernel(const QueryDev* __restrict__ qp, uint64_t n,
                                                      float* __restrict__ x0, float* __restrict__ x1,
                                                      float* __restrict__ x2, float* __restrict__ w0,
                                                      float* __restrict__ w1, float* __restrict__ w2) {
  const QueryDev& q = *qp;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    double x[3], w[3];
    seed_particle(q, i, x, w);
    x0[i] = (float)x[0];
    x1[i] = (float)x[1];
    x2[i] = (float)x[2];
    w0[i] = (float)w[0];
    w1[i] = (float)w[1];
    w2[i] = (float)w[2];
  }
}

// ---------------------------------------------------------------------------
// a6: closest hit.  Nearest-child-first traversal of the binary BVH with the
// far child on a per-lane stack in LDS (stack[slot][lane], conflict free);
// leaves are tested as soon as their box is hit.  Returns the Morton-order
// triangle position or -1; equal t keeps the lower original index.
// ---------------------------------------------------------------------------
template <int STACK, bool COUNT>
__device__ __forceinline__ int closest_hit(const Node* __restrict__ nodes, const TriRec* __restrict__ tris,
                                           const uint32_t* __restrict__ orig, const Ray& r, int prev,
                                           int (*stk)[kBlock], float& t_best, float& b0, float& b1, float& b2,
                                           uint32_t& n_nodes, uint32_t& n_tests) {
  const int lane = threadIdx.x;
  int best = -1;
  t_best = __builtin_inff();
  int sp = 0;
  int node = 0;
  // Each node is entered at most once per ray; the bound only guarantees that a
  // damaged tree cannot keep a wave spinning.
  for (uint32_t guard = 0; guard < (1u << 24); ++guard) {
    const float4* np = reinterpret_cast<const float4*>(nodes + node);
    const float4 A = np[0], B = np[1], C = np[2];
    const int4 L = reinterpret_cast<const int4*>(nodes + node)[3];
    if (COUNT) ++n_nodes;
    float tn0, tn1;
    bool h0 = slab(r, A.x, A.y, A.z, A.w, B.x, B.y, t_best, tn0);
    bool h1 = slab(r, B.z, B.w, C.x, C.y, C.z, C.w, t_best, tn1);
    if (h0 && L.x < 0) {
      const int k = ~L.x;
      float t, u0, u1, u2;
      if (COUNT && k != prev) ++n_tests;
      if (k != prev && intersect_tri(r, tris[k], t_best, t, u0, u1, u2) &&
          (t < t_best || (best >= 0 && orig[k] < orig[best]))) {
        best = k; t_best = t; b0 = u0; b1 = u1; b2 = u2;
      }
      h0 = false;
    }
    if (h1 && L.y < 0) {
      const int k = ~L.y;
      float t, u0, u1, u2;
      if (COUNT && k != prev) ++n_tests;
      if (k != prev && intersect_tri(r, tris[k], t_best, t, u0, u1, u2) &&
          (t < t_best || (best >= 0 && orig[k] < orig[best]))) {
        best = k; t_best = t; b0 = u0; b1 = u1; b2 = u2;
      }
      h1 = false;
    }
    if (h0 && h1 && sp < STACK) {
      const bool first0 = tn0 <= tn1;
      stk[sp][lane] = first0 ? L.y : L.x;
      ++sp;
      node = first0 ? L.x : L.y;
    } else if (h0) {
      node = L.x;
    } else if (h1) {
      node = L.y;
    } else {
      if (sp == 0) break;
      --sp;
      node = stk[sp][lane];
    }
  }
  return best;
}

// One lane's particle in flight.
struct Lane {
  float ox, oy, oz, wx, wy, wz;
  float D;        // momentum given along U so far (this particle)
  int prev;       // Morton position of the triangle just left
  uint32_t hits;
  uint64_t pid;   // particle index within its query
  bool live;
};

// Momentum and moment of one hit, ready for the tallies.
struct Hit {
  bool valid;
  uint32_t id;    // original triangle index
  float dx, dy, dz, lx, ly, lz;
};

// Per-lane exact integer accumulators.
struct Acc {
  long long sD, sD2, tot[7];
  long long tri2[2 * 7];  // per-triangle sums of a mesh of at most two triangles
  uint32_t rays, hits, segs, missed, escaped, capped;
  uint32_t nodes, tests;  // traversal work (counting kernels only)
};

__device__ __forceinline__ void acc_zero(Acc& A) {
  A.sD = A.sD2 = 0;
#pragma unroll
  for (int c = 0; c < 7; ++c) A.tot[c] = 0;
#pragma unroll
  for (int c = 0; c < 14; ++c) A.tri2[c] = 0;
  A.rays = A.hits = A.segs = A.missed = A.escaped = A.capped = 0;
  A.nodes = A.tests = 0;
}

// a6-a9 for one lane: one ray segment, then re-emission and the per-particle
// bookkeeping.  Returns true when the particle retires.
template <int STACK, bool COUNT>
__device__ __forceinline__ bool segment(const Node* __restrict__ nodes, const TriRec* __restrict__ tris,
                                        const uint32_t* __restrict__ orig, const QueryDev& q, Lane& L, Acc& A,
                                        Hit& h, int (*stk)[kBlock], int32_t& first_id) {
  Ray r;
  make_ray(r, L.ox, L.oy, L.oz, L.wx, L.wy, L.wz);
  float t, b0 = 0.f, b1 = 0.f, b2 = 0.f;
  const int k = closest_hit<STACK, COUNT>(nodes, tris, orig, r, L.prev, stk, t, b0, b1, b2, A.nodes, A.tests);
  ++A.segs;
  first_id = -2;  // not the first segment's outcome
  if (k < 0) {
    if (L.hits == 0) {
      ++A.missed;
      first_id = -1;
    } else {
      ++A.escaped;
    }
    return true;
  }
  const TriRec tr = tris[k];
  const uint32_t id = orig[k];
  const float px = b0 * tr.v0x + b1 * tr.v1x + b2 * tr.v2x;
  const float py = b0 * tr.v0y + b1 * tr.v1y + b2 * tr.v2y;
  const float pz = b0 * tr.v0z + b1 * tr.v1z + b2 * tr.v2z;
  float nwx = L.wx, nwy = L.wy, nwz = L.wz;
  reemit(q, L.pid, L.hits, tr.nx, tr.ny, tr.nz, nwx, nwy, nwz);
  const float dx = L.wx - nwx, dy = L.wy - nwy, dz = L.wz - nwz;
  const float rx = px - q.c0f[0], ry = py - q.c0f[1], rz = pz - q.c0f[2];
  h.valid = true;
  h.id = id;
  h.dx = dx; h.dy = dy; h.dz = dz;
  h.lx = ry * dz - rz * dy;
  h.ly = rz * dx - rx * dz;
  h.lz = rx * dy - ry * dx;
  L.D += dx * q.Uf[0] + dy * q.Uf[1] + dz * q.Uf[2];
  if (L.hits == 0) first_id = (int32_t)id;
  ++L.hits;
  ++A.hits;
  // The next ray starts at the hit point moved to the side the particle leaves
  // from by 8 FP32 ulps of the triangle's coordinate scale: the rounded
  // barycentric point can lie a few ulps behind the surface, and a ray started
  // there would cross a coplanar or adjacent triangle from the wrong side.
  const float scale = fmaxf(fmaxf(fmaxf(fabsf(tr.v0x), fabsf(tr.v0y)), fmaxf(fabsf(tr.v0z), fabsf(tr.v1x))),
                            fmaxf(fmaxf(fabsf(tr.v1y), fabsf(tr.v1z)),
                                  fmaxf(fmaxf(fabsf(tr.v2x), fabsf(tr.v2y)), fabsf(tr.v2z))));
  const float side = (L.wx * tr.nx + L.wy * tr.ny + L.wz * tr.nz) < 0.0f ? 1.0f : -1.0f;
  const float eps = side * scale * 0x1p-20f;
  L.ox = px + eps * tr.nx; L.oy = py + eps * tr.ny; L.oz = pz + eps * tr.nz;
  L.wx = nwx; L.wy = nwy; L.wz = nwz;
  L.prev = k;
  if (L.hits >= q.rmax) {
    ++A.capped;
    return true;
  }
  return false;
}

__device__ __forceinline__ void retire(const QueryDev& q, const Lane& L, Acc& A) {
  A.sD += fx(L.D, q.scaleD);
  A.sD2 += fx(L.D * L.D, q.scaleD2);
  ++A.rays;
}

// Tally of one hit per lane.  Called by every lane of the wave (convergent).
template <int MODE>
__device__ __forceinline__ void tally(const QueryDev& q, const Hit& h, long long* __restrict__ g,
                                      unsigned long long* lds, uint32_t nt, Acc& A) {
  long long v[7];
  v[0] = fx(h.dx, q.scaleF); v[1] = fx(h.dy, q.scaleF); v[2] = fx(h.dz, q.scaleF);
  v[3] = fx(h.lx, q.scaleL); v[4] = fx(h.ly, q.scaleL); v[5] = fx(h.lz, q.scaleL);
  v[6] = 1;
  if (MODE == kTallyTotals || (MODE == kTallyAuto && !q.per_tri)) {
    if (h.valid) {
#pragma unroll
      for (int c = 0; c < 7; ++c) A.tot[c] += v[c];
    }
  } else if (MODE == kTallyGlobal || MODE == kTallyAuto) {
    if (h.valid) {
#pragma unroll
      for (int c = 0; c < 7; ++c) atomic_add_i64(g + 7ull * h.id + c, v[c]);
    }
  } else if (MODE == kTallyLds) {
    if (h.valid) {
#pragma unroll
      for (int c = 0; c < 7; ++c) atomicAdd(lds + 7u * h.id + c, (unsigned long long)v[c]);
    }
  } else {  // kTallyRegs: per-lane registers, flushed once (meshes of <= 2 triangles)
    if (h.valid) {
#pragma unroll
      for (int c = 0; c < 7; ++c) {
        A.tri2[c] += h.id == 0 ? v[c] : 0ll;
        A.tri2[7 + c] += h.id == 1 ? v[c] : 0ll;
      }
    }
  }
}

// Flush of the register tallies of a <= 2-triangle mesh (convergent).
__device__ __forceinline__ void flush_tri2(const Acc& A, long long* __restrict__ g, uint32_t nt) {
#pragma unroll
  for (int c = 0; c < 14; ++c) {
    const long long s = wave_sum(A.tri2[c]);
    if ((threadIdx.x & 63) == 0 && s != 0 && c < (int)nt * 7) atomic_add_i64(g + c, s);
  }
}

// Wave-reduce the per-lane accumulators into a query's scalar block.
__device__ __forceinline__ void flush_acc(const Acc& A, long long* __restrict__ scal, bool TOTALS) {
  long long s[8 + 7];
  s[0] = wave_sum(A.sD);
  s[1] = wave_sum(A.sD2);
  s[2] = wave_sum((long long)A.rays);
  s[3] = wave_sum((long long)A.hits);
  s[4] = wave_sum((long long)A.segs);
  s[5] = wave_sum((long long)A.missed);
  s[6] = wave_sum((long long)A.escaped);
  s[7] = wave_sum((long long)A.capped);
  if (TOTALS) {
#pragma unroll
    for (int c = 0; c < 7; ++c) s[8 + c] = wave_sum(A.tot[c]);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (s[c]) atomic_add_i64(scal + c, s[c]);
    if (TOTALS) {
#pragma unroll
      for (int c = 0; c < 7; ++c)
        if (s[8 + c]) atomic_add_i64(scal + kFx + c, s[8 + c]);
    }
  }
}

// ---------------------------------------------------------------------------
// a6-a9, plain path: one query per launch, particles read from the SoA.  The
// loop is wave-uniform; a lane whose particle retires loads the next one
// (grid stride) at once, so lanes stay busy while particles have different
// numbers of bounces.
// ---------------------------------------------------------------------------
template <int STACK, int MODE, bool COUNT>
__global__ __launch_bounds__(kBlock) void trace_kernel(TraceArgs a) {
  __shared__ int stk[STACK][kBlock];
  __shared__ unsigned long long lt[MODE == kTallyLds ? kLdsTallyMaxTris * 7 : 1];
  const QueryDev& q = *a.q;
  if (MODE == kTallyLds) {
    for (uint32_t i = threadIdx.x; i < a.nt * 7u; i += kBlock) lt[i] = 0ull;
    __syncthreads();
  }
  Acc A;
  acc_zero(A);
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  Lane L;
  L.pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  L.live = L.pid < a.n;
  auto load = [&](Lane& l) {
    l.ox = a.x[0][l.pid]; l.oy = a.x[1][l.pid]; l.oz = a.x[2][l.pid];
    l.wx = a.w[0][l.pid]; l.wy = a.w[1][l.pid]; l.wz = a.w[2][l.pid];
    l.D = 0.0f;
    l.prev = -1;
    l.hits = 0;
  };
  if (L.live) load(L);
  while (__ballot(L.live) != 0ull) {
    Hit h;
    h.valid = false;
    bool done = false;
    int32_t fid = -2;
    if (L.live) done = segment<STACK, COUNT>(a.nodes, a.tris, a.orig, q, L, A, h, stk, fid);
    tally<MODE>(q, h, a.tally, lt, a.nt, A);
    if (L.live) {
      if (a.first_tri && fid != -2) a.first_tri[L.pid] = fid;
      if (done) {
        retire(q, L, A);
        L.pid += stride;
        L.live = L.pid < a.n;
        if (L.live) load(L);
      }
    }
  }
  flush_acc(A, a.scal, MODE == kTallyTotals);
  if (MODE == kTallyRegs) flush_tri2(A, a.tally, a.nt);
  if (COUNT) {
    const long long nn = wave_sum((long long)A.nodes), nt2 = wave_sum((long long)A.tests);
    if ((threadIdx.x & 63) == 0) {
      atomic_add_i64(reinterpret_cast<long long*>(a.counters), nn);
      atomic_add_i64(reinterpret_cast<long long*>(a.counters) + 1, nt2);
    }
  }
  if (MODE == kTallyLds) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < a.nt * 7u; i += kBlock)
      if (lt[i]) atomic_add_i64(a.tally + i, (long long)lt[i]);
  }
}

// ---------------------------------------------------------------------------
// a11: persistent batched kernel.  A workgroup claims tiles of one work entry
// (a query, or a range of its tiles) from that entry's counter until the entry
// is exhausted, then moves to the next entry with work left; its four waves
// share each tile, claiming 64 particles at a time from a workgroup counter in
// LDS.  A wave seeds its 64 particles with every lane active (the FP64 seeding
// is the costliest per-particle step) into a wave-private LDS queue, and lanes
// whose particle retires refill from that queue; particle states never leave
// the chip.  Partial sums -- per-lane scalars, per-lane register tallies of
// tiny meshes, the workgroup's LDS tally of meshes up to kLdsTallyMaxTris
// triangles -- stay on chip while the workgroup stays on one query and are
// flushed to HBM with atomics only when it changes query or finishes.
// Per-particle arithmetic is the plain path's, so results match it bit for bit.
// ---------------------------------------------------------------------------

template <int STACK, int MODE>
__global__ __launch_bounds__(kBlock) void batch_kernel(BatchArgs a) {
  constexpr bool kMayLds = MODE == kTallyLds || MODE == kTallyAuto;
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  __shared__ int stk[STACK][kBlock];
  __shared__ float qbuf[kBlock / 64][6][64];
  __shared__ unsigned long long lt[kMayLds ? kLdsTallyMaxTris * 7 : 1];
  __shared__ unsigned long long tile_sh, next_sh;
  __shared__ uint32_t entry_sh;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  uint32_t scan = blockIdx.x % a.n_entries;  // thread 0's position in the entry list
  uint32_t held = kNone;                     // entry whose partial sums the workgroup holds
  Acc A;
  acc_zero(A);
  for (;;) {
    if (threadIdx.x == 0) {
      // claim a tile: current entry first, then the following ones (bounded scan)
      uint32_t found = kNone;
      unsigned long long t = 0;
      for (uint32_t k = 0; k < a.n_entries; ++k) {
        const uint64_t cap = a.entry_tiles[scan];
        if (__hip_atomic_load(&a.entry_next[scan], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < cap) {
          t = atomicAdd(&a.entry_next[scan], 1ull);
          if (t < cap) {
            found = scan;
            break;
          }
        }
        scan = scan + 1 == a.n_entries ? 0u : scan + 1;
      }
      entry_sh = found;
      tile_sh = t;
    }
    __syncthreads();
    const uint32_t j = entry_sh;  // uniform over the workgroup
    const uint64_t tile = tile_sh;
    if (j != held && held != kNone) {
      // leaving the held query: flush its partial sums
      const QueryDev& qh = a.qs[a.entry_query ? a.entry_query[held] : held];
      long long* htally = qh.per_tri ? a.tally_base + qh.tally_offset : nullptr;
      flush_acc(A, a.scal_base + qh.scalar_offset, MODE == kTallyTotals || (MODE == kTallyAuto && !qh.per_tri));
      if (MODE == kTallyRegs) flush_tri2(A, htally, qh.nt);
      acc_zero(A);
      if (kMayLds && qh.per_tri && qh.nt <= (uint32_t)kLdsTallyMaxTris)
        for (uint32_t i = threadIdx.x; i < qh.nt * 7u; i += kBlock)
          if (lt[i]) atomic_add_i64(htally + i, (long long)lt[i]);
    }
    if (j == kNone) break;  // uniform
    const QueryDev& q = a.qs[a.entry_query ? a.entry_query[j] : j];
    const bool use_lds = kMayLds && q.per_tri && q.nt <= (uint32_t)kLdsTallyMaxTris;
    if (j != held) {
      __syncthreads();  // the flush above has read lt
      if (use_lds)
        for (uint32_t i = threadIdx.x; i < q.nt * 7u; i += kBlock) lt[i] = 0ull;
      held = j;
    }
    const uint64_t tile_in_q = (a.entry_tile0 ? a.entry_tile0[j] : 0ull) + tile;
    const uint64_t p_begin = tile_in_q * kBatchTile;
    const uint64_t p_end = p_begin + kBatchTile < q.N ? p_begin + kBatchTile : q.N;
    long long* qtally = q.per_tri ? a.tally_base + q.tally_offset : nullptr;
    if (threadIdx.x == 0) next_sh = p_begin;
    __syncthreads();

    Lane L;
    L.live = false;
    bool exhausted = false;            // wave-uniform: the tile has no particles left to claim
    uint32_t q_head = 0, q_count = 0;  // wave-uniform queue state
    uint64_t q_pid0 = 0;               // particle id of queue slot 0
    for (;;) {
      const uint64_t dead = __ballot(!L.live);
      const uint32_t ndead = __popcll(dead);
      if (q_count == 0 && !exhausted && ndead >= 16) {
        // claim and seed the next (up to) 64 particles, one per lane
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&next_sh, 64ull);
        base = (unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)base) |
               ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32);
        if (base >= p_end) {
          exhausted = true;
        } else {
          const uint64_t pid = base + lane;
          if (pid < p_end) {
            double x[3], w[3];
            seed_particle(q, pid, x, w);
            qbuf[wave][0][lane] = (float)x[0];
            qbuf[wave][1][lane] = (float)x[1];
            qbuf[wave][2][lane] = (float)x[2];
            qbuf[wave][3][lane] = (float)w[0];
            qbuf[wave][4][lane] = (float)w[1];
            qbuf[wave][5][lane] = (float)w[2];
          }
          const uint64_t left = p_end - base;
          q_count = left < 64 ? (uint32_t)left : 64u;
          q_head = 0;
          q_pid0 = base;
          __builtin_amdgcn_wave_barrier();
        }
      }
      if (q_count > 0 && dead != 0ull) {
        // dead lanes take queue entries in lane order
        const uint32_t rank = __popcll(dead & lt_mask);
        if (!L.live && rank < q_count) {
          const uint32_t slot = q_head + rank;
          L.ox = qbuf[wave][0][slot]; L.oy = qbuf[wave][1][slot]; L.oz = qbuf[wave][2][slot];
          L.wx = qbuf[wave][3][slot]; L.wy = qbuf[wave][4][slot]; L.wz = qbuf[wave][5][slot];
          L.pid = q_pid0 + slot;
          L.D = 0.0f;
          L.prev = -1;
          L.hits = 0;
          L.live = true;
        }
        const uint32_t took = ndead < q_count ? ndead : q_count;
        q_head += took;
        q_count -= took;
        __builtin_amdgcn_wave_barrier();
      }
      if (__ballot(L.live) == 0ull) {
        if (exhausted && q_count == 0) break;
        continue;  // nothing in flight: claim more next round
      }
      Hit h;
      h.valid = false;
      bool done = false;
      int32_t fid;
      if (L.live) done = segment<STACK, false>(q.nodes, q.tris, q.orig, q, L, A, h, stk, fid);
      if (use_lds) tally<kTallyLds>(q, h, qtally, lt, q.nt, A);
      else tally<MODE>(q, h, qtally, nullptr, q.nt, A);
      if (L.live && done) {
        retire(q, L, A);
        L.live = false;
      }
    }
    __syncthreads();  // every wave is done with the tile; tile_sh / entry_sh / next_sh may be reused
  }
}

// ---------------------------------------------------------------------------
// a10: reduction and finalisation
// ---------------------------------------------------------------------------
constexpr int kReduceChunk = 4096;  // triangles per workgroup

__device__ __forceinline__ void reduce_one(const long long* __restrict__ tally, uint32_t nt, long long* __restrict__ scal,
                                           uint32_t chunk) {
  __shared__ long long part[kBlock / 64][7];
  long long s[7] = {0, 0, 0, 0, 0, 0, 0};
  const uint32_t t0 = chunk * kReduceChunk;
  const uint32_t t1 = t0 + kReduceChunk < nt ? t0 + kReduceChunk : nt;
  for (uint32_t t = t0 + threadIdx.x; t < t1; t += kBlock)
#pragma unroll
    for (int c = 0; c < 7; ++c) s[c] += tally[7ull * t + c];
#pragma unroll
  for (int c = 0; c < 7; ++c) s[c] = wave_sum(s[c]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < 7; ++c) part[threadIdx.x >> 6][c] = s[c];
  __syncthreads();
  if (threadIdx.x < 7) {
    long long v = 0;
    for (int w = 0; w < kBlock / 64; ++w) v += part[w][threadIdx.x];
    if (v) atomic_add_i64(scal + kFx + threadIdx.x, v);
  }
}

__global__ __launch_bounds__(kBlock) void reduce_kernel(const long long* __restrict__ tally, uint32_t nt,
                                                        long long* __restrict__ scal) {
  reduce_one(tally, nt, scal, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void reduce_batch_kernel(const QueryDev* __restrict__ qs,
                                                              long long* __restrict__ tally_base,
                                                              long long* __restrict__ scal_base) {
  const QueryDev& q = qs[blockIdx.y];
  if (!q.per_tri || blockIdx.x * (uint32_t)kReduceChunk >= q.nt) return;
  reduce_one(tally_base + q.tally_offset, q.nt, scal_base + q.scalar_offset, blockIdx.x);
}

// F/q = K sum(w - w'), K = 2 Gamma_hat / (N S^2) (eq. drag with the effective
// mass of Sec. II.A); moment about x_ref from the moment about the CV centre.
__global__ void finalize_kernel(const QueryDev* __restrict__ qs, const uint32_t* __restrict__ idx,
                                const long long* __restrict__ scal_base, uint32_t nq, double xr, double yr, double zr,
                                double A_ref, ResultDev* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const QueryDev& q = qs[idx ? idx[i] : i];
  const long long* s = scal_base + q.scalar_offset;
  const double N = (double)q.N;
  double F[3], Lc[3];
  for (int k = 0; k < 3; ++k) {
    F[k] = (double)s[kFx + k] * q.inv_scaleF;
    Lc[k] = (double)s[kLx + k] * q.inv_scaleL;
  }
  const double cx = q.c0[0] - xr, cy = q.c0[1] - yr, cz = q.c0[2] - zr;
  const double M[3] = {Lc[0] + (cy * F[2] - cz * F[1]), Lc[1] + (cz * F[0] - cx * F[2]), Lc[2] + (cx * F[1] - cy * F[0])};
  const double nan = __builtin_nan("");
  const double K = q.s_zero ? nan : 2.0 * q.Gamma_hat / (N * q.S * q.S);
  ResultDev r;
  for (int k = 0; k < 3; ++k) {
    r.F_over_q[k] = K * F[k];
    r.M_over_q[k] = K * M[k];
    r.Fhat[k] = q.Gamma_hat / N * F[k];
  }
  r.CD = (r.F_over_q[0] * q.U[0] + r.F_over_q[1] * q.U[1] + r.F_over_q[2] * q.U[2]) / A_ref;
  const double meanD = (double)s[kSD] * q.inv_scaleD / N;
  double varD = (double)s[kSD2] * q.inv_scaleD2 / N - meanD * meanD;
  if (varD < 0.0) varD = 0.0;
  r.CD_sigma = q.s_zero ? nan : 2.0 * q.Gamma_hat / (q.S * q.S * A_ref) * sqrt(varD / N);
  r.Gamma_hat = q.Gamma_hat;
  r.rays = (uint64_t)s[kRays];
  r.hits = (uint64_t)s[kHits];
  r.segments = (uint64_t)s[kSegments];
  r.missed = (uint64_t)s[kMissed];
  r.escaped = (uint64_t)s[kEscaped];
  r.capped = (uint64_t)s[kCapped];
  out[i] = r;
}

template <int STACK, bool COUNT>
void launch_trace_mode(const TraceArgs& a, TallyMode mode, int grid, hipStream_t st) {
  switch (mode) {
    case kTallyGlobal: trace_kernel<STACK, kTallyGlobal, COUNT><<<grid, kBlock, 0, st>>>(a); break;
    case kTallyLds: trace_kernel<STACK, kTallyLds, COUNT><<<grid, kBlock, 0, st>>>(a); break;
    case kTallyRegs: trace_kernel<STACK, kTallyRegs, COUNT><<<grid, kBlock, 0, st>>>(a); break;
    default: trace_kernel<STACK, kTallyTotals, COUNT><<<grid, kBlock, 0, st>>>(a); break;
  }
}

template <int STACK>
void launch_trace_stack(const TraceArgs& a, TallyMode mode, int grid, hipStream_t st) {
  if (a.counters) launch_trace_mode<STACK, true>(a, mode, grid, st);
  else launch_trace_mode<STACK, false>(a, mode, grid, st);
}

template <int STACK>
void launch_batch_mode(const BatchArgs& a, TallyMode mode, int grid, hipStream_t st) {
  switch (mode) {
    case kTallyRegs: batch_kernel<STACK, kTallyRegs><<<grid, kBlock, 0, st>>>(a); break;
    case kTallyLds: batch_kernel<STACK, kTallyLds><<<grid, kBlock, 0, st>>>(a); break;
    case kTallyTotals: batch_kernel<STACK, kTallyTotals><<<grid, kBlock, 0, st>>>(a); break;
    case kTallyAuto: batch_kernel<STACK, kTallyAuto><<<grid, kBlock, 0, st>>>(a); break;
    default: batch_kernel<STACK, kTallyGlobal><<<grid, kBlock, 0, st>>>(a); break;
  }
}

}  // namespace

void zero_i64(long long* p, uint64_t n, hipStream_t st) {
  if (n) zero_i64_kernel<<<grid_for(n, 4096), kBlock, 0, st>>>(p, n);
}

void zero_u32(uint32_t* p, uint64_t n, hipStream_t st) {
  if (n) zero_u32_kernel<<<grid_for(n, 4096), kBlock, 0, st>>>(p, n);
}

int stack_slots_for_depth(uint32_t depth) {
  if (depth <= 8) return 8;
  if (depth <= 16) return 16;
  if (depth <= 32) return 32;
  if (depth <= 64) return 64;
  return 0;
}

void launch_seed(const QueryDev* d_q, uint64_t n, float* const x[3], float* const w[3], int grid, hipStream_t st) {
  seed_kernel<<<grid, kBlock, 0, st>>>(d_q, n, x[0], x[1], x[2], w[0], w[1], w[2]);
}

void launch_trace(const TraceArgs& a, int stack_slots, TallyMode mode, int grid, hipStream_t st) {
  switch (stack_slots) {
    case 8: launch_trace_stack<8>(a, mode, grid, st); break;
    case 16: launch_trace_stack<16>(a, mode, grid, st); break;
    case 32: launch_trace_stack<32>(a, mode, grid, st); break;
    default: launch_trace_stack<64>(a, mode, grid, st); break;
  }
}

void launch_batch(const BatchArgs& a, int stack_slots, TallyMode mode, int grid, hipStream_t st) {
  switch (stack_slots) {
    case 8: launch_batch_mode<8>(a, mode, grid, st); break;
    case 16: launch_batch_mode<16>(a, mode, grid, st); break;
    case 32: launch_batch_mode<32>(a, mode, grid, st); break;
    default: launch_batch_mode<64>(a, mode, grid, st); break;
  }
}

void launch_reduce(const long long* tally, uint32_t nt, long long* scal, hipStream_t st) {
  const int g = (int)((nt + kReduceChunk - 1) / kReduceChunk);
  reduce_kernel<<<g, kBlock, 0, st>>>(tally, nt, scal);
}

void launch_reduce_batch(const QueryDev* d_qs, uint32_t nq, long long* tally_base, long long* scal_base,
                         uint32_t max_nt, hipStream_t st) {
  dim3 g((max_nt + kReduceChunk - 1) / kReduceChunk, nq);
  reduce_batch_kernel<<<g, kBlock, 0, st>>>(d_qs, tally_base, scal_base);
}

void launch_finalize(const QueryDev* d_qs, const uint32_t* d_idx, const long long* scal_base, uint32_t nq, double xr,
                     double yr, double zr, double A_ref, ResultDev* out, hipStream_t st) {
  finalize_kernel<<<(nq + 63) / 64, 64, 0, st>>>(d_qs, d_idx, scal_base, nq, xr, yr, zr, A_ref, out);
}

// Per-triangle reduction of a list of slots (serving): entry y reduces slot idx[y].
__global__ __launch_bounds__(kBlock) void reduce_slots_kernel(const QueryDev* __restrict__ qs,
                                                              const uint32_t* __restrict__ idx,
                                                              long long* __restrict__ tally_base,
                                                              long long* __restrict__ scal_base) {
  const QueryDev& q = qs[idx[blockIdx.y]];
  if (!q.per_tri || blockIdx.x * (uint32_t)kReduceChunk >= q.nt) return;
  reduce_one(tally_base + q.tally_offset, q.nt, scal_base + q.scalar_offset, blockIdx.x);
}

// Clears slots kFx..kCount of the listed per-triangle queries before a reduction.
__global__ void clear_totals_kernel(const QueryDev* __restrict__ qs, const uint32_t* __restrict__ idx,
                                    long long* __restrict__ scal_base, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * 7u) return;
  const QueryDev& q = qs[idx ? idx[i / 7u] : i / 7u];
  if (q.per_tri) scal_base[q.scalar_offset + kFx + i % 7u] = 0;
}

void launch_reduce_slots(const QueryDev* d_qs, const uint32_t* d_idx, uint32_t n, long long* tally_base,
                         long long* scal_base, uint32_t max_nt, hipStream_t st) {
  clear_totals_kernel<<<(n * 7 + 255) / 256, 256, 0, st>>>(d_qs, d_idx, scal_base, n);
  dim3 g((max_nt + kReduceChunk - 1) / kReduceChunk, n);
  reduce_slots_kernel<<<g, kBlock, 0, st>>>(d_qs, d_idx, tally_base, scal_base);
}

}  // namespace tpmc

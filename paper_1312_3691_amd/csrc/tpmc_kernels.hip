// tpmc_kernels.hip -- the per-query hot path on gfx950:
//   seed_kernel     a2-a4  Philox streams, FP64 boundary seeding -> FP32 SoA
//   trace_kernel    a6-a9  BVH traversal, watertight hit, re-emission, tallies, bounce loop
//   batch_kernel    a11    persistent (query, tile) work queue; seeding fused on chip
//   reduce/finalize a10    exact integer reduction, force / moment / C_D in FP64
#include <hip/hip_runtime.h>

#include "tpmc_device.hpp"
#include "tpmc_launch.h"

#ifndef TPMC_PHASE_PROBE
#define TPMC_PHASE_PROBE 0
#endif

namespace tpmc {

#if TPMC_PHASE_PROBE
__device__ unsigned long long g_probe[kProbeSlots];  // ProbeSlot sums of the batched launches
#endif

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
// Starting points of the latitude and normal-speed solves (latitude_start,
// normal_speed_start); part of the code object, filled once per device.
__device__ float g_lat_start[kLatNS * kLatNT];
__device__ float g_lat_fine[kLatFNS * kLatFNT];  // the seeding estimate's latitude table
__device__ float g_vn_start[kVnNS * kVnNT];
// sin and cos of 2 pi j / 256, j = 0..255 (sincos_2pi_draw)
__device__ double g_sc_tab[512];
// exp(-y_j^2) and erfc(y_j) at y_j = j / 256 (exp_erfc_grid)
__device__ double g_ee_tab[2 * kExpErfcN];

__global__ void ee_table_kernel(double* __restrict__ tab) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kExpErfcN) return;
  const double y = (double)j * 0x1p-8;  // y and y^2 are exact
  tab[2 * j] = exp(-(y * y));
  tab[2 * j + 1] = erfc(y);
}

__global__ void sc_table_kernel(double* __restrict__ tab) {
  const int j = threadIdx.x;
  if (j >= 256) return;
  double s, c;
  sincospi((double)j / 128.0, &s, &c);
  tab[2 * j] = s;
  tab[2 * j + 1] = c;
}

__global__ void lat_table_kernel(float* __restrict__ tab, const double* __restrict__ ee) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kLatNS * kLatNT) return;
  QueryDev q{};
  q.S = (double)kLatS0 * exp((double)(i / kLatNT) * (double)kLatDL);
  q.erfS = erf(q.S);
  q.erfcS = erfc(q.S);
  q.expmS2 = exp(-q.S * q.S);
  q.lat_k = kSqrtPi / (4.0 * q.S);
  const double t = (double)kLatT0 + (double)(i % kLatNT) * (double)kLatDT;
  const double u = 1.0 / (1.0 + exp(-t));
  double Z, G, dG, d2G, e, ta;
  latitude_G(q, ee, 1.0, Z, dG, d2G, e, ta);
  const double target = u * Z;
  double lo = -1.0, hi = 1.0;
  for (int it = 0; it < 60; ++it) {
    const double m = 0.5 * (lo + hi);
    latitude_G(q, ee, m, G, dG, d2G, e, ta);
    if (G < target) lo = m;
    else hi = m;
  }
  tab[i] = (float)(0.5 * (lo + hi));
}

// The seeding estimate's fine latitude table: the same root by the same
// FP64 bisection, at the fine table's nodes.
__global__ void lat_fine_kernel(float* __restrict__ tab, const double* __restrict__ ee) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kLatFNS * kLatFNT) return;
  QueryDev q{};
  q.S = exp(kLatFL0 + (double)(i / kLatFNT) * kLatFDL);
  q.erfS = erf(q.S);
  q.erfcS = erfc(q.S);
  q.expmS2 = exp(-q.S * q.S);
  q.lat_k = kSqrtPi / (4.0 * q.S);
  const double t = (double)kLatFT0 + (double)(i % kLatFNT) * (double)kLatFDT;
  const double u = 1.0 / (1.0 + exp(-t));
  double Z, G, dG, d2G, e, ta;
  latitude_G(q, ee, 1.0, Z, dG, d2G, e, ta);
  const double target = u * Z;
  double lo = -1.0, hi = 1.0;
  for (int it = 0; it < 60; ++it) {
    const double m = 0.5 * (lo + hi);
    latitude_G(q, ee, m, G, dG, d2G, e, ta);
    if (G < target) lo = m;
    else hi = m;
  }
  tab[i] = (float)(0.5 * (lo + hi));
}

__global__ void vn_table_kernel(float* __restrict__ tab, const double* __restrict__ ee) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kVnNS * kVnNT) return;
  const double s = (double)kVnS0 + (double)(i / kVnNT) * (double)kVnDS;
  const double t = (double)kVnT0 + (double)(i % kVnNT) * (double)kVnDT;
  const double u = 1.0 / (1.0 + exp(-t));
  const NormalSpeedConsts k = normal_speed_consts(ee, s);
  const double target = u * k.chi;
  double lo = 0.0, hi = (s > 0.0 ? s : 0.0) + 8.0;
  for (int it = 0; it < 80; ++it) {
    const double m = 0.5 * (lo + hi);
    double F, dF, d2F;
    normal_speed_F(ee, k, m, F, dF, d2F);
    if (F < target) lo = m;
    else hi = m;
  }
  tab[i] = (float)(0.5 * (lo + hi));
}

__global__ __launch_bounds__(kBlock) void seed_kernel(const QueryDev* __restrict__ qp, uint64_t n,
                                                      float* __restrict__ x0, float* __restrict__ x1,
                                                      float* __restrict__ x2, float* __restrict__ w0,
                                                      float* __restrict__ w1, float* __restrict__ w2) {
  const QueryDev& q = *qp;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    double x[3], w[3];
    seed_particle(q, g_lat_start, g_lat_fine, g_vn_start, g_sc_tab, g_ee_tab, i, x, w);
    x0[i] = (float)x[0];
    x1[i] = (float)x[1];
    x2[i] = (float)x[2];
    w0[i] = (float)w[0];
    w1[i] = (float)w[1];
    w2[i] = (float)w[2];
  }
}

// ---------------------------------------------------------------------------
// Loads through the global address space.  The mesh pointers reach the
// kernels inside the query record, so the compiler cannot prove that they
// address global memory and would emit flat loads, which also count against
// the LDS counter and so delay every LDS access behind them.
// ---------------------------------------------------------------------------
template <class T>
using gptr = const T __attribute__((address_space(1)))*;
typedef float vf4 __attribute__((ext_vector_type(4)));  // native vectors: HIP's float4 cannot
typedef int vi4 __attribute__((ext_vector_type(4)));    // be copied from an address-space reference

__device__ __forceinline__ TriRec load_tri(const TriRec* p, int k) {
  const gptr<vf4> g = (gptr<vf4>)(p + k);
  const vf4 a = g[0], b = g[1], c = g[2];
  return TriRec{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
}

// orig[] word of a triangle: original index in bits 0..29, supporting-plane
// flags in bits 30 (nothing above the plane) and 31 (nothing below).
__device__ __forceinline__ uint32_t load_orig_word(const uint32_t* p, int k) { return ((gptr<uint32_t>)p)[k]; }
__device__ __forceinline__ uint32_t load_orig(const uint32_t* p, int k) { return load_orig_word(p, k) & kOrigIdMask; }

// Mask of the lanes where p holds.  The builtin takes the comparison's lane
// mask as it is; __ballot(int) first turns it into 0/1 values and compares
// them again.
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// A pointer every lane holds the same value of, moved to scalar registers.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(lo | (hi << 32));
}

// One lane's particle in flight.
struct Lane {
  float ox = 0.0f, oy = 0.0f, oz = 0.0f, wx = 0.0f, wy = 0.0f, wz = 0.0f;
  float D;        // momentum given along U so far (this particle)
  float E;        // energy given to the body so far, sum of |w|^2 - |w'|^2
  int prev;       // Morton position of the triangle just left
  uint32_t hits;
  uint64_t pid;   // particle index within its query
  bool live;
};

// ---------------------------------------------------------------------------
// a6: closest hit, one BVH node per step.  Nearest-child-first traversal of
// the binary BVH with the far child on a per-lane stack in LDS
// (stack[slot][lane], conflict free); leaves are tested as soon as their box
// is hit.  The traversal state lives in registers between steps, so a lane
// whose segment has ended can be given its next segment while the other
// lanes of the wave are still traversing.  The closest hit does not depend
// on the visiting order: every triangle whose t is at most the final t_best
// lies in boxes that are never culled (conservative far bound), and equal t
// keeps the lower original index.  The ray's derived constants (Ray) are
// recomputed from the lane's origin and direction after every service pass,
// so they are not held in registers across the seeding code.
// ---------------------------------------------------------------------------
constexpr int kDone = -0x7FFFFFFF - 1;  // Seg::cur once the traversal has ended

struct Seg {
  int cur;     // next node to visit, or kDone
  int sp;      // stack depth
  int best;    // closest triangle so far (Morton position), -1 if none
  int p0, p1;  // leaves whose boxes were hit, waiting for a leaf phase (-1: none)
  float t_best, b0, b1, b2;
};

__device__ __forceinline__ void seg_begin(Seg& s) {
  s.cur = 0;
  s.sp = 0;
  s.best = -1;
  s.p0 = s.p1 = -1;
  s.t_best = __builtin_inff();
}

// Lane states: traversing (next node known, no leaf waiting), waiting for a
// leaf phase, or finished (segment ready for its service pass).
__device__ __forceinline__ bool seg_traversing(const Seg& s) { return s.cur != kDone && s.p0 < 0; }
__device__ __forceinline__ bool seg_finished(const Seg& s) { return s.cur == kDone && s.p0 < 0; }

// Candidate leaf k: two-sided test, the triangle just left excluded.
template <bool COUNT>
__device__ __forceinline__ void test_leaf(const TriRec* tris, const uint32_t* orig, const Ray& r, int k, int prev,
                                          Seg& s, uint32_t& n_tests) {
  if (COUNT && k != prev) ++n_tests;
  float t, u0, u1, u2;
  if (intersect_tri(r, load_tri(tris, k), s.t_best, t, u0, u1, u2) && k != prev) {
    // t <= t_best here; an exact tie keeps the lower original index
    const bool take = t < s.t_best || (s.best >= 0 && load_orig(orig, k) < load_orig(orig, s.best));
    if (take) {
      s.best = k;
      s.t_best = t;
      s.b0 = u0;
      s.b1 = u1;
      s.b2 = u2;
    }
  }
}

// One traversal step of a traversing lane.  Hit leaves are not tested here
// but recorded in p0 / p1 (a node has two children), and the lane then waits
// for a leaf phase: the costly triangle test runs for many lanes at once
// instead of for the few lanes that happen to reach a leaf in a given step.
// Each node is entered at most once per ray, so a segment takes at most nt - 1
// steps and nt leaf tests.  Trees of depth <= 4 (a 4-slot stack: meshes of a
// few triangles, where nearly every step ends at leaves) test them in place.
template <int STACK, bool COUNT>
__device__ __forceinline__ void trav_step(const Node* nodes, const TriRec* tris, const uint32_t* orig, const Ray& r,
                                          int prev, Seg& s, int (*stk)[kBlock], uint32_t& n_nodes,
                                          uint32_t& n_tests) {
  const int lane = threadIdx.x;
  // 32-bit byte offset from the (scalar) base: one shift, no 64-bit address math
  const gptr<char> base = (gptr<char>)nodes;
  const uint32_t off = (uint32_t)s.cur * (uint32_t)sizeof(Node);
  const gptr<vf4> np = (gptr<vf4>)(base + off);
  const vf4 A = np[0], B = np[1], C = np[2];
  const vi4 L = ((gptr<vi4>)(base + off))[3];
  if (COUNT) ++n_nodes;
  float tn0, tn1;
  bool h0 = slab(r, A.x, A.y, A.z, A.w, B.x, B.y, s.t_best, tn0);
  bool h1 = slab(r, B.z, B.w, C.x, C.y, C.z, C.w, s.t_best, tn1);
  const bool leaf0 = h0 && L.x < 0, leaf1 = h1 && L.y < 0;
  if (STACK <= 4) {
    if (leaf0) test_leaf<COUNT>(tris, orig, r, ~L.x, prev, s, n_tests);
    if (leaf1) test_leaf<COUNT>(tris, orig, r, ~L.y, prev, s, n_tests);
  } else {
    if (leaf0) s.p0 = ~L.x;
    if (leaf1) {
      if (leaf0) s.p1 = ~L.y;
      else s.p0 = ~L.y;
    }
  }
  h0 = h0 && !leaf0;
  h1 = h1 && !leaf1;
  if (h0 && h1 && s.sp < STACK) {
    const bool first0 = tn0 <= tn1;
    stk[s.sp][lane] = first0 ? L.y : L.x;
    ++s.sp;
    s.cur = first0 ? L.x : L.y;
  } else if (h0) {
    s.cur = L.x;
  } else if (h1) {
    s.cur = L.y;
  } else {
    s.cur = s.sp == 0 ? kDone : stk[--s.sp][lane];
  }
}

// Leaf phase (convergent): every waiting lane tests its first pending leaf;
// a second one moves up and waits for the next phase.
template <bool COUNT>
__device__ __forceinline__ void leaf_phase(const TriRec* tris, const uint32_t* orig, const Ray& r, int prev, Seg& s,
                                           uint32_t& n_tests) {
  if (s.p0 >= 0) {
    test_leaf<COUNT>(tris, orig, r, s.p0, prev, s, n_tests);
    s.p0 = s.p1;
    s.p1 = -1;
  }
}

// Whether a ray from (o, w) passes the slab test of either box of the root
// node with no distance bound, i.e. whether its first traversal step can find
// anything.  Same reciprocals and test as the traversal.
__device__ __forceinline__ bool ray_enters_root(const Node* nodes, const float o[3], const float w[3]) {
  Ray r;
  r.ox = o[0]; r.oy = o[1]; r.oz = o[2];
  r.idx = __builtin_amdgcn_rcpf(w[0]);
  r.idy = __builtin_amdgcn_rcpf(w[1]);
  r.idz = __builtin_amdgcn_rcpf(w[2]);
  const gptr<vf4> np = (gptr<vf4>)nodes;
  const vf4 A = np[0], B = np[1], C = np[2];
  float tn;
  const float inf = __builtin_inff();
  return slab(r, A.x, A.y, A.z, A.w, B.x, B.y, inf, tn) || slab(r, B.z, B.w, C.x, C.y, C.z, C.w, inf, tn);
}

// Momentum and moment of one hit, ready for the tallies.
struct Hit {
  bool valid;
  uint32_t id;    // original triangle index
  float dx, dy, dz, lx, ly, lz;
};

// Exact integer accumulators: per lane the quantised per-particle sums, per
// wave (scalar registers, from ballots at convergent points) the event
// counts.  Rays and segments are not kept: a particle retires by missing,
// escaping or reaching the hit cap, and every segment ends in a hit, an
// escape or a miss, so rays = missed + escaped + capped and segments = hits +
// missed + escaped (an escape through a supporting plane is one untraced
// segment after the hit).
struct Acc {
  long long sD, sD2, sE, sE2, tot[7];
  uint32_t nodes, tests;  // traversal work (counting kernels only)
  // wave-uniform
  uint64_t hits, missed, escaped, capped;
  uint64_t tr_capped;  // re-emissions whose temperature the kernel's bound limited
  uint64_t guard;      // segments ended by the traversal step bound
};

__device__ __forceinline__ void acc_zero(Acc& A) {
  A.sD = A.sD2 = A.sE = A.sE2 = 0;
#pragma unroll
  for (int c = 0; c < 7; ++c) A.tot[c] = 0;
  A.hits = A.missed = A.escaped = A.capped = 0;
  A.tr_capped = A.guard = 0;
  A.nodes = A.tests = 0;
}

__device__ __forceinline__ uint64_t lanes(bool p) { return (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(p)); }

// Set bits of a wave mask below the calling lane (v_mbcnt; no per-lane mask kept live).
__device__ __forceinline__ uint32_t below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Phase probe of batch_kernel, in libraries built with TPMC_PHASE_PROBE=1
// (elsewhere PROBE(...) expands to nothing): each wave reads the shader clock
// around its phases and sums cycles, passes and active lanes, all
// wave-uniform, into one VGPR whose lane k holds ProbeSlot k (32 bits: a wave
// of one launch stays far below 2^32 cycles and passes); lanes kPrTs, kPrTc
// and kPrTp hold the clock at the wave's start, at the current tile claim and
// at the current phase's start.  Lanes are written with v_writelane and read
// with v_readlane (no lane masks, no long-lived scalar registers), so the
// instrumented kernel needs at most a register or two more than the ordinary
// one; the instances that run four waves per SIMD are held to that occupancy
// (amdgpu_waves_per_eu, at the cost of a few spilled dwords), so that the
// probe measures the kernel at its own occupancy.  At exit lane k adds its
// slot to g_probe.
#if TPMC_PHASE_PROBE
#define PROBE(...) __VA_ARGS__
constexpr int kPrTp = 29, kPrTs = 30, kPrTc = 31;
static_assert(kProbeSlots <= kPrTp, "probe lanes");
__device__ __forceinline__ uint32_t probe_now() { return (uint32_t)__builtin_amdgcn_s_memtime(); }
__device__ __forceinline__ uint32_t probe_get(uint32_t v, int k) { return __builtin_amdgcn_readlane(v, k); }
template <int K>
__device__ __forceinline__ void probe_set(uint32_t& v, uint32_t x) {
  // the trailing wait states keep a v_readlane of the written VGPR right after it exact
  asm("v_writelane_b32 %0, %1, %2\n\ts_nop 1" : "+v"(v) : "s"(x), "i"(K));
}
template <int K>
__device__ __forceinline__ void probe_add(uint32_t& v, uint32_t x) { probe_set<K>(v, probe_get(v, K) + x); }
template <int K>
__device__ __forceinline__ void probe_since(uint32_t& v, int t) { probe_add<K>(v, probe_now() - probe_get(v, t)); }
#else
#define PROBE(...)
#endif

// Outcome of a finished segment.  kOutHitLeft: a hit whose outgoing segment
// cannot hit anything (the mesh lies on the other side of the triangle's
// plane), so that segment is counted and the particle escapes untraced.
// (names distinct from the scalar-slot indices kMissed, kEscaped, kCapped)
enum Outcome : int { kOutGoOn = 0, kOutMissed = 1, kOutEscaped = 2, kOutCapped = 3, kOutHitLeft = 4 };

// a7-a9 for a lane whose traversal has ended: re-emission and bookkeeping of
// the hit, or the particle's exit.  The particle retires unless kOutGoOn.
__device__ __forceinline__ int finish_segment(const TriRec* tris, const uint32_t* orig, const QueryDev& q, Lane& L,
                                              const Seg& s, Hit& h, int32_t& first_id, bool& tr_limited) {
  const int k = s.best;
  first_id = -2;  // not the first segment's outcome
  if (k < 0) {
    if (L.hits == 0) {
      first_id = -1;
      return kOutMissed;
    }
    return kOutEscaped;
  }
  const TriRec tr = load_tri(tris, k);
  const uint32_t ow = load_orig_word(orig, k);
  const uint32_t id = ow & kOrigIdMask;
  const float px = s.b0 * tr.v0x + s.b1 * tr.v1x + s.b2 * tr.v2x;
  const float py = s.b0 * tr.v0y + s.b1 * tr.v1y + s.b2 * tr.v2y;
  const float pz = s.b0 * tr.v0z + s.b1 * tr.v1z + s.b2 * tr.v2z;
  float nwx = L.wx, nwy = L.wy, nwz = L.wz;
  tr_limited = reemit(q, L.pid, L.hits, tr.nx, tr.ny, tr.nz, nwx, nwy, nwz);
  L.E += (L.wx * L.wx + L.wy * L.wy + L.wz * L.wz) - (nwx * nwx + nwy * nwy + nwz * nwz);
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
  if (L.hits >= q.rmax) return kOutCapped;
  // the emission side is empty of mesh points (see support_kernel)
  const bool clear = side > 0.0f ? (ow >> 30) & 1u : (ow >> 31) & 1u;
  return clear ? kOutHitLeft : kOutGoOn;
}

// Event counts of a service pass (convergent): lanes with fin set ended a
// segment with outcome out (hit: with a hit; limited: whose re-emission the
// temperature bound limited).
__device__ __forceinline__ void count_pass(Acc& A, bool fin, int out, bool hit, bool limited) {
  A.hits += lanes(fin && hit);
  A.missed += lanes(fin && out == kOutMissed);
  A.escaped += lanes(fin && (out == kOutEscaped || out == kOutHitLeft));
  A.capped += lanes(fin && out == kOutCapped);
  A.tr_capped += lanes(fin && limited);
}

__device__ __forceinline__ void retire(const QueryDev& q, const Lane& L, Acc& A) {
  A.sD += fx(L.D, q.scaleD);
  A.sD2 += fx(L.D * L.D, q.scaleD2);
  A.sE += fx(L.E, q.scaleE);
  A.sE2 += fx(L.E * L.E, q.scaleE2);
}

// Tally of one hit per lane.  Called by every lane of the wave (convergent).
// Totals-only sums go to the wave's LDS slots lds[c][wave] (LDS atomics; the
// few lanes of a pass with a hit share them) when TOT_LDS (the persistent
// kernel, short of registers), else to the lane's registers.
template <int MODE, bool TOT_LDS = true>
__device__ __forceinline__ void tally(const QueryDev& q, const Hit& h, long long* __restrict__ g,
                                      unsigned long long* lds, uint32_t nt, Acc& A) {
  long long v[7];
  // one hit's values are below 2^30 in magnitude after scaling (scale choice)
  v[0] = fx32(h.dx, q.scaleF); v[1] = fx32(h.dy, q.scaleF); v[2] = fx32(h.dz, q.scaleF);
  v[3] = fx32(h.lx, q.scaleL); v[4] = fx32(h.ly, q.scaleL); v[5] = fx32(h.lz, q.scaleL);
  v[6] = 1;
  if ((MODE == kTallyTotals || (MODE == kTallyAuto && !q.per_tri)) && TOT_LDS) {  // the wave's LDS slots [c][wave]
    if (h.valid) {
#pragma unroll
      for (int c = 0; c < 7; ++c) atomicAdd(lds + c * kWaves + (threadIdx.x >> 6), (unsigned long long)v[c]);
    }
  } else if (MODE == kTallyTotals || (MODE == kTallyAuto && !q.per_tri)) {
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
  } else {  // kTallyLane: the lane's own LDS slots [7 * id + c][lane] (meshes of <= 2 triangles)
    if (h.valid) {
#pragma unroll
      for (int c = 0; c < 7; ++c) atomicAdd(lds + (7u * h.id + c) * kBlock + threadIdx.x, (unsigned long long)v[c]);
    }
  }
}

// Flush (and clear) the calling lane's per-lane tallies of a <= 2-triangle
// mesh: one wave sum per slot, one atomic per wave (convergent).
__device__ __forceinline__ void flush_lane_tally(unsigned long long* lds, long long* __restrict__ g, uint32_t nt) {
#pragma unroll
  for (int c = 0; c < 2 * 7; ++c) {
    const long long s = wave_sum((long long)lds[c * kBlock + threadIdx.x]);
    lds[c * kBlock + threadIdx.x] = 0ull;
    if ((threadIdx.x & 63) == 0 && s != 0 && c < (int)nt * 7) atomic_add_i64(g + c, s);
  }
}

// Wave-reduce the per-lane accumulators into a query's scalar block.  With
// TOTALS the query's force and moment totals come from the lanes' registers,
// or, with TOT_LDS, from (and clearing) the wave's LDS slots wave_tot[c][wave]
// (a compile-time choice, so that the register totals are not kept live
// across the trace loop of a kernel that never uses them).
template <bool TOT_LDS = false>
__device__ __forceinline__ void flush_acc(Acc& A, long long* __restrict__ scal, bool TOTALS,
                                          unsigned long long* wave_tot = nullptr) {
  // one value at a time, each total moved to scalar registers, so that the
  // flush adds little to the kernel's vector-register peak
  const bool lead = (threadIdx.x & 63) == 0;
  auto put = [&](long long total, int slot) {
    if (lead && total) atomic_add_i64(scal + slot, total);
  };
  put(wave_sum_uniform(A.sD), kSD);
  put(wave_sum_uniform(A.sD2), kSD2);
  put((long long)A.hits, kHits);
  put((long long)A.missed, kMissed);
  put((long long)A.escaped, kEscaped);
  put((long long)A.capped, kCapped);
  put((long long)(A.missed + A.escaped + A.capped), kRays);
  put((long long)(A.hits + A.missed + A.escaped), kSegments);
  put(wave_sum_uniform(A.sE), kSE);
  put(wave_sum_uniform(A.sE2), kSE2);
  put((long long)A.tr_capped, kTrCap);
  put((long long)A.guard, kGuard);
  if (TOTALS && TOT_LDS) {
    long long t[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) t[c] = (long long)wave_tot[c * kWaves + (threadIdx.x >> 6)];
#pragma unroll
    for (int c = 0; c < 7; ++c) put(t[c], kFx + c);
    if (lead)  // after every lane of the wave has read them (one wave: LDS in program order)
#pragma unroll
      for (int c = 0; c < 7; ++c) wave_tot[c * kWaves + (threadIdx.x >> 6)] = 0ull;
  } else if (TOTALS) {
#pragma unroll
    for (int c = 0; c < 7; ++c) put(wave_sum_uniform(A.tot[c]), kFx + c);
  }
}

// ---------------------------------------------------------------------------
// a6-a9, plain path: one query per launch, particles read from the SoA.  Each
// loop iteration advances every traversing lane by one BVH step.  Lanes whose
// segment has ended wait until fewer than a.refill lanes are still
// traversing; then all of them are served at once (re-emission, tallies, the
// next segment, or the next particle by grid stride), so the costly per-hit
// work runs with many lanes active and no lane idles for the rest of a
// segment's traversal.
// ---------------------------------------------------------------------------
template <int STACK, int MODE, bool COUNT>
__global__ __launch_bounds__(kBlock) void trace_kernel(TraceArgs a) {
  __shared__ int stk[STACK][kBlock];
  extern __shared__ unsigned long long lt[];  // tallies in LDS, sized at launch (tally_lds_bytes)
  const QueryDev& q = *a.q;
  if (MODE == kTallyLds) {
    for (uint32_t i = threadIdx.x; i < a.nt * 7u; i += kBlock) lt[i] = 0ull;
    __syncthreads();
  }
  if (MODE == kTallyLane)
    for (int c = 0; c < 2 * 7; ++c) lt[c * kBlock + threadIdx.x] = 0ull;
  Acc A;
  acc_zero(A);
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const uint32_t max_steps = 2u * a.nt + 64u;
  Lane L;
  Seg s;
  Ray r;
  seg_begin(s);
  auto load = [&](Lane& l) {
    l.ox = a.x[0][l.pid]; l.oy = a.x[1][l.pid]; l.oz = a.x[2][l.pid];
    l.wx = a.w[0][l.pid]; l.wy = a.w[1][l.pid]; l.wz = a.w[2][l.pid];
    l.D = 0.0f;
    l.E = 0.0f;
    l.prev = -1;
    l.hits = 0;
  };
  L.pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  L.live = L.pid < a.n;
  s.cur = kDone;
  if (L.live) {
    load(L);
    seg_begin(s);
  }
  make_ray(r, L.ox, L.oy, L.oz, L.wx, L.wy, L.wz);
  uint32_t guard = 0;  // steps since the last service pass (wave-uniform)
  while (ballot(L.live) != 0ull) {
    uint32_t ntrav = (uint32_t)__popcll(ballot(L.live && seg_traversing(s)));
    if (ntrav < a.refill && ballot(L.live && s.p0 >= 0) != 0ull) {
      leaf_phase<COUNT>(a.tris, a.orig, r, L.prev, s, A.tests);
      ntrav = (uint32_t)__popcll(ballot(L.live && seg_traversing(s)));
    }
    if (ntrav < a.refill) {
      const bool fin = L.live && seg_finished(s);
      if (ballot(fin) != 0ull) {
        Hit h;
        h.valid = false;
        int out = kOutGoOn;
        int32_t fid = -2;
        bool limited = false;
        if (fin) out = finish_segment(a.tris, a.orig, q, L, s, h, fid, limited);
        count_pass(A, fin, out, h.valid, limited);
        tally<MODE, false>(q, h, a.tally, lt, a.nt, A);
        if (fin) {
          if (a.first_tri && fid != -2) a.first_tri[L.pid] = fid;
          if (out != kOutGoOn) {
            retire(q, L, A);
            L.pid += stride;
            L.live = L.pid < a.n;
            if (L.live) load(L);
          }
          if (L.live) seg_begin(s);
        }
      }
      make_ray(r, L.ox, L.oy, L.oz, L.wx, L.wy, L.wz);
      guard = 0;
    }
    // Between service passes every traversing lane ends its segment within
    // nt - 1 steps and nt leaf phases; the bound only keeps a damaged tree
    // from spinning a wave, and every segment it ends is counted.
    if (++guard > max_steps) {
      A.guard += lanes(L.live && s.cur != kDone);
      s.cur = kDone;
    }
    if (L.live && seg_traversing(s))
      trav_step<STACK, COUNT>(a.nodes, a.tris, a.orig, r, L.prev, s, stk, A.nodes, A.tests);
  }
  flush_acc(A, a.scal, MODE == kTallyTotals);
  if (MODE == kTallyLane) flush_lane_tally(lt, a.tally, a.nt);
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
// is the costliest per-particle step) into a wave-private LDS queue; the
// traversal advances one BVH step per iteration as in the plain path, and when
// fewer than a.refill lanes are still traversing, the lanes whose segment has
// ended are served together and lanes whose particle retired take the next
// queued particle.  Particle states never leave the chip.  Partial sums --
// per-lane scalars, per-lane LDS tallies of tiny meshes, the workgroup's
// LDS tally of meshes up to kLdsTallyMaxTris triangles -- stay on chip while
// the workgroup stays on one query and are flushed to HBM with atomics only
// when it changes query or finishes.  Per-particle arithmetic is the plain
// path's, so results match it bit for bit.
// ---------------------------------------------------------------------------

// Seeding in two stages (precull_may_enter) in every instance whose LDS
// leaves room for the survivor rings (not the 64-slot stack).
template <int STACK, int MODE>
constexpr bool kPrecullInstance = STACK <= 32;

// Work is claimed per wave in units of a quarter tile (a whole tile when the
// tile is not a multiple of 256 particles): a wave's lanes draw particles
// from its own unit, and when the unit runs out while lanes are still busy
// the wave goes on with another unit of the same entry instead of draining
// (lanes in flight keep their absolute particle ids), so waves drain only
// when their entry is used up.  Where no tally state is shared by the
// workgroup's waves (global atomics, per-lane LDS tallies, the waves' own
// totals) each wave also chooses its entries alone and never waits for the
// others; with workgroup LDS tallies the workgroup chooses the entry together
// and its waves meet at a barrier only when they leave it (the tallies are
// flushed then).
template <int MODE>
constexpr bool kWaveEntries = MODE == kTallyGlobal || MODE == kTallyLane || MODE == kTallyTotals;

// Claim the next tile (or quarter tile) of the entry list from `scan` on:
// the current entry first, then the following ones (bounded scan).  Returns
// the entry, or kNoEntry when every entry is used up; t gets the unit's index.
constexpr uint32_t kNoEntry = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t claim_unit(const BatchArgs& a, uint32_t& scan, uint32_t units_per_tile,
                                               unsigned long long& t) {
  for (uint32_t k = 0; k < a.n_entries; ++k) {
    const uint64_t cap = a.entry_tiles[scan] * units_per_tile;
    if (__hip_atomic_load(&a.entry_next[scan], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < cap) {
      t = atomicAdd(&a.entry_next[scan], 1ull);
      if (t < cap) return scan;
    }
    scan = scan + 1 == a.n_entries ? 0u : scan + 1;
  }
  return kNoEntry;
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  return (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v) |
         ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32);
}

template <int STACK, int MODE>
__global__ __launch_bounds__(kBlock) PROBE(__attribute__((amdgpu_waves_per_eu(STACK <= 32 && MODE != kTallyAuto ? 4 : 1)))) void batch_kernel(BatchArgs a) {
  constexpr bool kMayLds = MODE == kTallyLds || MODE == kTallyAuto;
  constexpr bool kPre = kPrecullInstance<STACK, MODE>;
  constexpr bool kWave = kWaveEntries<MODE>;
  constexpr uint32_t kSteps = STACK >= 32 ? 2u : 1u;  // traversal steps per round of the trace loop
  constexpr uint32_t kNone = kNoEntry;
  constexpr uint32_t kRing = 128;  // survivors of the estimate awaiting exact seeding (< 64 + 64)
  __shared__ int stk[STACK][kBlock];
  __shared__ float qbuf[kBlock / 64][6][64];
  // queue slot -> particle: its offset in its seeding batch, or (two-stage
  // seeding) in the wave's unit
  __shared__ uint8_t qlane[kPre ? 1 : kBlock / 64][64];
  __shared__ uint16_t qoff[kPre ? kBlock / 64 : 1][64];
  __shared__ uint16_t ring[kPre ? kBlock / 64 : 1][kPre ? kRing : 1];  // survivor offsets in the unit
  extern __shared__ unsigned long long lt[];  // tallies in LDS, sized at launch (tally_lds_bytes)
  // per-wave totals [c][wave]: the start of lt, or after the per-triangle area in the mixed mode
  unsigned long long* const wave_tot = MODE == kTallyAuto ? lt + 7u * a.lds_tris : lt;
  __shared__ unsigned long long tile_sh;
  __shared__ unsigned long long w_next_sh[kWaves];  // each wave's next unclaimed particle
  __shared__ uint32_t entry_sh;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t scan;  // the claiming thread's position in the entry list (thread 0, or each wave's lane 0)
  {
    const uint32_t x = blockIdx.x & 7u, lo = a.xcd_start[x], hi = a.xcd_start[x + 1];
    scan = a.xcd_start[8] == 0u ? blockIdx.x % a.n_entries : (hi > lo ? lo + (blockIdx.x >> 3) % (hi - lo) : lo);
  }
  uint32_t held = kNone;                     // entry whose partial sums the wave (and workgroup) holds
  Acc A;
  acc_zero(A);
  PROBE(uint32_t pr = 0u; probe_set<kPrTs>(pr, probe_now()); probe_set<kPrTc>(pr, probe_get(pr, kPrTs));)
  // two-stage seeding, wave-uniform: particles the estimate removed (for the
  // held query), and the estimate's yield so far on it.  A wave that finds
  // more than 60 % of a query's particles surviving the estimate switches it
  // off for the query (its kPrecullOff slot, read whenever a wave takes up the query), since the
  // estimate then costs more than it saves.
  uint64_t pre = 0;
  uint32_t pc_seen = 0, pc_kept = 0;
  if (MODE == kTallyLane)
    for (int c = 0; c < 2 * 7; ++c) lt[c * kBlock + threadIdx.x] = 0ull;
  if (MODE == kTallyTotals || (MODE == kTallyAuto && a.wave_totals)) {
    if (kWave) {  // each wave its own slots (no barrier before its first tally)
      if (lane < 7) wave_tot[lane * kWaves + wave] = 0ull;
    } else if (threadIdx.x < 7u * kWaves) {
      wave_tot[threadIdx.x] = 0ull;
    }
  }
  // claim units per tile (quarter tiles when they stay multiples of 64 particles)
  const uint32_t units = (a.tile & 255u) == 0u ? 4u : 1u;
  for (;;) {
    uint32_t j;
    uint64_t tile;  // claim unit within the entry
    if (kWave) {
      uint32_t found = kNone;
      unsigned long long t = 0;
      if (lane == 0) found = claim_unit(a, scan, units, t);
      j = __builtin_amdgcn_readfirstlane(found);  // uniform over the wave
      tile = uniform_u64(t);
    } else {
      if (threadIdx.x == 0) {  // the workgroup's entry, and wave 0's first unit of it
        unsigned long long t = 0;
        entry_sh = claim_unit(a, scan, units, t);
        tile_sh = t;
      }
      __syncthreads();
      j = __builtin_amdgcn_readfirstlane(entry_sh);  // uniform over the workgroup
      tile = uniform_u64(tile_sh);
    }
    if (j != held && held != kNone) {
      // leaving the held query: flush its partial sums
      const QueryDev& qh = a.qs[a.entry_query ? a.entry_query[held] : held];
      long long* htally = qh.per_tri ? a.tally_base + qh.tally_offset : nullptr;
      flush_acc<MODE == kTallyTotals || MODE == kTallyAuto>(
          A, a.scal_base + qh.scalar_offset, MODE == kTallyTotals || (MODE == kTallyAuto && !qh.per_tri), wave_tot);
      if (MODE == kTallyLane) flush_lane_tally(lt, htally, qh.nt);
      acc_zero(A);
      if (kPre) {
        if (lane == 0 && pre != 0) atomic_add_i64(a.scal_base + qh.scalar_offset + kPreculled, (long long)pre);
        pre = 0;
        pc_seen = pc_kept = 0;
      }
      if (kMayLds && qh.per_tri && qh.nt <= (uint32_t)kLdsTallyMaxTris)
        for (uint32_t i = threadIdx.x; i < qh.nt * 7u; i += kBlock)
          if (lt[i]) atomic_add_i64(htally + i, (long long)lt[i]);
    }
    if (j == kNone) break;  // uniform (the last claim's cycles are not in the claim slot)
    const QueryDev& q = a.qs[a.entry_query ? a.entry_query[j] : j];
    const bool use_lds = kMayLds && q.per_tri && q.nt <= (uint32_t)kLdsTallyMaxTris;
    if (j != held) {
      if (!kWave) __syncthreads();  // the flush above has read lt
      if (use_lds) {
        for (uint32_t i = threadIdx.x; i < q.nt * 7u; i += kBlock) lt[i] = 0ull;
        __syncthreads();  // cleared before any wave tallies into it
      }
      held = j;
    }
    // particles [p_begin, p_end) of claim unit u of the entry (of its tile u / units);
    // everything is read again at each claim, so nothing of it stays live across the trace loop
    auto unit_range = [&](uint64_t u, uint64_t& b, uint64_t& e) {
      const uint32_t sh = (a.tile & 255u) == 0u ? 2u : 0u;
      const uint64_t tb = ((a.entry_tile0 ? a.entry_tile0[j] : 0ull) + (u >> sh)) * a.tile;
      b = tb + (u & ((1u << sh) - 1u)) * (a.tile >> sh);
      e = b + (a.tile >> sh);
      if (e > tb + a.tile) e = tb + a.tile;
      if (e > q.N) e = q.N;
    };
    bool have = true;  // the wave holds a unit of entry j
    // the other waves claim their own first unit of the workgroup's entry (wave number
    // read into a scalar register, so that the branch and what it sets stay wave-uniform)
    if (!kWave && __builtin_amdgcn_readfirstlane(wave) != 0) {
      unsigned long long t = 0;
      if (lane == 0) t = atomicAdd(&a.entry_next[j], 1ull);
      tile = uniform_u64(t);
      have = tile < a.entry_tiles[j] * units;
    }
    uint64_t p_begin = 0, p_end = 0;
    if (have) unit_range(tile, p_begin, p_end);
    if (lane == 0) w_next_sh[wave] = p_begin;  // the next unclaimed particle of the wave's unit
    long long* qtally = q.per_tri ? a.tally_base + q.tally_offset : nullptr;
    const Node* nodes = uniform_ptr(q.nodes);
    const TriRec* tris = uniform_ptr(q.tris);
    const uint32_t* orig = uniform_ptr(q.orig);
    PROBE(probe_since<kPrClaimCyc>(pr, kPrTc); probe_add<kPrClaims>(pr, 1u);)
    // next 64 particle ids of the wave's unit
    auto claim64 = [&]() -> uint64_t {
      const uint64_t b = uniform_u64(w_next_sh[wave]);
      if (lane == 0) w_next_sh[wave] = b + 64u;
      return b;
    };

    Lane L;
    Seg s;
    Ray r;
    L.live = false;
    seg_begin(s);
    s.cur = kDone;
    const uint32_t max_steps = __builtin_amdgcn_readfirstlane(2u * q.nt + 64u);
    uint32_t guard = 0;                // steps since the last service pass (wave-uniform)
    bool exhausted = !have;            // wave-uniform: the unit has no particles left to claim
    bool dry = !have;                  // wave-uniform: the entry has no units left
    uint32_t q_head = 0, q_count = 0;  // wave-uniform queue state
    uint64_t q_pid0 = 0;               // particle id of queue slot 0
    uint32_t s_head = 0, s_count = 0;  // wave-uniform survivor ring state (two-stage seeding)
    bool pc_on = true, pc_off_now = false;  // wave-uniform
    if (kPre)
      pc_on = __builtin_amdgcn_readfirstlane((uint32_t)__hip_atomic_load(
                  a.scal_base + q.scalar_offset + kPrecullOff, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0u;
    for (;;) {
      uint32_t ntrav = (uint32_t)__popcll(ballot(L.live && seg_traversing(s)));
      if (ntrav < a.refill && ballot(L.live && s.p0 >= 0) != 0ull) {
        PROBE(probe_set<kPrTp>(pr, probe_now()); probe_add<kPrLeafPasses>(pr, 1u);
              probe_add<kPrLeafLanes>(pr, (uint32_t)lanes(L.live && s.p0 >= 0));)
        uint32_t n1 = 0;
        leaf_phase<false>(tris, orig, r, L.prev, s, n1);
        ntrav = (uint32_t)__popcll(ballot(L.live && seg_traversing(s)));
        PROBE(probe_since<kPrLeafCyc>(pr, kPrTp);)
      }
      if (ntrav < a.refill) {
        // serve every lane whose segment has ended
        const bool fin = L.live && seg_finished(s);
        if (ballot(fin) != 0ull) {
          PROBE(probe_set<kPrTp>(pr, probe_now()); probe_add<kPrServes>(pr, 1u);
                probe_add<kPrServeLanes>(pr, (uint32_t)lanes(fin));)
          Hit h;
          h.valid = false;
          int out = kOutGoOn;
          int32_t fid;
          bool limited = false;
          if (fin) out = finish_segment(tris, orig, q, L, s, h, fid, limited);
          count_pass(A, fin, out, h.valid, limited);
          if (use_lds) tally<kTallyLds>(q, h, qtally, lt, q.nt, A);
          else tally<MODE>(q, h, qtally, wave_tot, q.nt, A);
          if (fin) {
            if (out != kOutGoOn) {
              retire(q, L, A);
              L.live = false;
            } else {
              seg_begin(s);
            }
          }
          PROBE(probe_since<kPrServeCyc>(pr, kPrTp);)
        }
        const uint64_t dead = ballot(!L.live);
        if (dead != 0ull && exhausted && !dry && q_count == 0 && s_count == 0) {
          // the unit is used up (survivor ring and queue empty, so no offset refers to it):
          // go on with the entry's next unit while the other lanes are still busy
          unsigned long long t = 0;
          if (lane == 0) t = atomicAdd(&a.entry_next[j], 1ull);
          t = uniform_u64(t);
          if (t < a.entry_tiles[j] * units) {
            unit_range(t, p_begin, p_end);
            if (lane == 0) w_next_sh[wave] = p_begin;
            exhausted = false;
            PROBE(probe_add<kPrClaims>(pr, 1u);)
          } else {
            dry = true;
          }
        }
        if (kPre && dead != 0ull) {
          while (q_count == 0 && !(exhausted && s_count == 0)) {  // wave-uniform
            if (s_count < 64 && !exhausted) {
              // stage 1: claim 64 particles, keep those the estimate cannot rule out
              PROBE(probe_set<kPrTp>(pr, probe_now());)
              const uint64_t base = claim64();
              if (base >= p_end) {
                exhausted = true;
              } else {
                const uint64_t pid = base + lane;
                const bool valid = pid < p_end;
                bool maybe = valid;
                if (valid && pc_on) maybe = precull_may_enter(q, g_lat_fine, g_vn_start, nodes, pid);
                const uint64_t mb = ballot(maybe);
                if (maybe) ring[wave][(s_head + s_count + below(mb)) & (kRing - 1)] =
                    (uint16_t)(pid - p_begin);
                const uint32_t nvalid = (uint32_t)__popcll(ballot(valid)), nmaybe = (uint32_t)__popcll(mb);
                s_count += nmaybe;
                pre += nvalid - nmaybe;
                A.missed += nvalid - nmaybe;
                pc_seen += nvalid;
                pc_kept += nmaybe;
                if (pc_on && pc_seen >= 256u && 5u * pc_kept > 3u * pc_seen) {
                  pc_on = false;
                  pc_off_now = true;
                }
                PROBE(probe_add<kPrEstBatches>(pr, 1u); probe_add<kPrEstLanes>(pr, nvalid);
                      probe_add<kPrEstKept>(pr, nmaybe);)
                __builtin_amdgcn_wave_barrier();
              }
              PROBE(probe_since<kPrEstCyc>(pr, kPrTp);)
            } else {
            // stage 2: exact seeding of up to 64 survivors, one per lane; the
            // exact root test as in the one-stage seeding below
            const uint32_t n = s_count < 64u ? s_count : 64u;
            PROBE(probe_set<kPrTp>(pr, probe_now());)
            bool keep = false;
            float xs[3], ws[3];
            if ((uint32_t)lane < n) {
              double x[3], w[3];
              seed_particle(q, g_lat_start, g_lat_fine, g_vn_start, g_sc_tab, g_ee_tab,
                            p_begin + ring[wave][(s_head + lane) & (kRing - 1)], x, w);
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                xs[c] = (float)x[c];
                ws[c] = (float)w[c];
              }
              keep = STACK <= 4 || ray_enters_root(nodes, xs, ws);
            }
            A.missed += lanes((uint32_t)lane < n && !keep);
            const uint64_t kb = ballot(keep);
            if (keep) {
              const uint32_t slot = below(kb);
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                qbuf[wave][c][slot] = xs[c];
                qbuf[wave][3 + c][slot] = ws[c];
              }
              qoff[wave][slot] = ring[wave][(s_head + lane) & (kRing - 1)];  // read again: not held across the seeding
            }
            s_head += n;
            s_count -= n;
            q_count = (uint32_t)__popcll(kb);
            q_head = 0;
            PROBE(probe_since<kPrSeedCyc>(pr, kPrTp); probe_add<kPrSeedBatches>(pr, 1u);
                  probe_add<kPrSeedLanes>(pr, n); probe_add<kPrSeedKept>(pr, q_count);)
            __builtin_amdgcn_wave_barrier();
            }
          }
        }
        if (!kPre && dead != 0ull) {
          while (q_count == 0 && !exhausted) {  // wave-uniform
            // claim and seed the next (up to) 64 particles, one per lane
            PROBE(probe_set<kPrTp>(pr, probe_now());)
            const uint64_t base = claim64();
            if (base >= p_end) {
              exhausted = true;
            } else {
              // Seed; a particle whose first ray misses both boxes of the root
              // node would end its first traversal step with no hit, so it is
              // counted as missed here and only the others are queued (trees
              // deeper than a 4-slot stack: there it spares the lane its idle
              // wait for the next service pass; in tiny trees every step ends
              // at leaves and the test would only add work).
              const uint64_t pid = base + lane;
              bool keep = false;
              float xs[3], ws[3];
              if (pid < p_end) {
                double x[3], w[3];
                seed_particle(q, g_lat_start, g_lat_fine, g_vn_start, g_sc_tab, g_ee_tab, pid, x, w);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                  xs[c] = (float)x[c];
                  ws[c] = (float)w[c];
                }
                keep = STACK <= 4 || ray_enters_root(nodes, xs, ws);
              }
              A.missed += lanes(pid < p_end && !keep);
              const uint64_t kb = ballot(keep);
              if (keep) {
                const uint32_t slot = below(kb);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                  qbuf[wave][c][slot] = xs[c];
                  qbuf[wave][3 + c][slot] = ws[c];
                }
                qlane[wave][slot] = (uint8_t)lane;
              }
              q_count = (uint32_t)__popcll(kb);
              q_head = 0;
              q_pid0 = base;
              PROBE(probe_add<kPrSeedBatches>(pr, 1u); probe_add<kPrSeedLanes>(pr, (uint32_t)lanes(pid < p_end));
                    probe_add<kPrSeedKept>(pr, q_count);)
              __builtin_amdgcn_wave_barrier();
            }
            PROBE(probe_since<kPrSeedCyc>(pr, kPrTp);)
          }
        }
        if (dead != 0ull) {
          if (q_count > 0) {
            // dead lanes take queue entries in lane order
            PROBE(probe_set<kPrTp>(pr, probe_now());)
            const uint32_t rank = below(dead);
            if (!L.live && rank < q_count) {
              const uint32_t slot = q_head + rank;
              L.ox = qbuf[wave][0][slot]; L.oy = qbuf[wave][1][slot]; L.oz = qbuf[wave][2][slot];
              L.wx = qbuf[wave][3][slot]; L.wy = qbuf[wave][4][slot]; L.wz = qbuf[wave][5][slot];
              L.pid = kPre ? p_begin + qoff[wave][slot] : q_pid0 + qlane[wave][slot];
              L.D = 0.0f;
              L.E = 0.0f;
              L.prev = -1;
              L.hits = 0;
              L.live = true;
              seg_begin(s);
            }
            const uint32_t ndead = __popcll(dead);
            const uint32_t took = ndead < q_count ? ndead : q_count;
            q_head += took;
            q_count -= took;
            PROBE(probe_since<kPrAssignCyc>(pr, kPrTp); probe_add<kPrAssigns>(pr, 1u);
                  probe_add<kPrAssignLanes>(pr, took);)
            __builtin_amdgcn_wave_barrier();
          }
        }
        // nothing in flight and nothing left: the wave is done with the entry
        // (with no lane live but particles left, the next iteration claims more)
        if (ballot(L.live) == 0ull && exhausted && q_count == 0 && s_count == 0) break;
        make_ray(r, L.ox, L.oy, L.oz, L.wx, L.wy, L.wz);
        guard = 0;
      }
      // as in the plain path: a bound only against a damaged tree, counted
      if ((guard += kSteps) > kSteps * max_steps) {
        A.guard += lanes(L.live && s.cur != kDone);
        s.cur = kDone;
      }
      PROBE(const uint32_t nl = (uint32_t)lanes(L.live && seg_traversing(s)); probe_add<kPrTravLanes>(pr, nl);
            probe_add<kPrTravSteps>(pr, nl != 0u ? 1u : 0u); probe_set<kPrTp>(pr, probe_now());)
      if (L.live && seg_traversing(s)) {
        uint32_t n0 = 0, n1 = 0;
        trav_step<STACK, false>(nodes, tris, orig, r, L.prev, s, stk, n0, n1);
      }
      // deep trees (32-slot stacks): a second step before the next round of checks
      // (refill, leaf phase, guard), whose cost there is worth sparing for every
      // other step (attitude sweep -2.4 %, satellite -1.2 %; neutral on shallow trees)
      PROBE(if (kSteps == 2) {
        const uint32_t nl2 = (uint32_t)lanes(L.live && seg_traversing(s));
        probe_add<kPrTravLanes>(pr, nl2);
        probe_add<kPrTravSteps>(pr, nl2 != 0u ? 1u : 0u);
      })
      if (kSteps == 2 && L.live && seg_traversing(s)) {
        uint32_t n0 = 0, n1 = 0;
        trav_step<STACK, false>(nodes, tris, orig, r, L.prev, s, stk, n0, n1);
      }
      PROBE(probe_since<kPrTravCyc>(pr, kPrTp);)
    }
    PROBE(probe_set<kPrTc>(pr, probe_now());)
    if (kPre && pc_off_now && lane == 0)  // published when the wave leaves the entry, outside the trace loop
      __hip_atomic_store(a.scal_base + q.scalar_offset + kPrecullOff, 1ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!kWave) __syncthreads();  // every wave is done with the entry; entry_sh / tile_sh may be reused
  }
  PROBE(probe_set<kPrWaves>(pr, 1u); probe_set<kPrCycles>(pr, probe_now() - probe_get(pr, kPrTs));
        if (lane < kProbeSlots) atomicAdd(&g_probe[lane], (unsigned long long)pr);)
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
    r.Mhat[k] = q.Gamma_hat / N * M[k];  // M / (rho c_mp^2), finite at S = 0
  }
  r.CD = (r.F_over_q[0] * q.U[0] + r.F_over_q[1] * q.U[1] + r.F_over_q[2] * q.U[2]) / A_ref;
  const double meanD = (double)s[kSD] * q.inv_scaleD / N;
  double varD = (double)s[kSD2] * q.inv_scaleD2 / N - meanD * meanD;
  if (varD < 0.0) varD = 0.0;
  r.CD_sigma = q.s_zero ? nan : 2.0 * q.Gamma_hat / (q.S * q.S * A_ref) * sqrt(varD / N);
  r.Gamma_hat = q.Gamma_hat;
  // energy: power Q = n c_mp (m c_mp^2 / 2) (Gamma_hat / N) sum E, and
  // C_H = Q / (rho U^3 A_ref / 2) = Gamma_hat sum E / (N S^3 A_ref)
  const double meanE = (double)s[kSE] * q.inv_scaleE / N;
  double varE = (double)s[kSE2] * q.inv_scaleE2 / N - meanE * meanE;
  if (varE < 0.0) varE = 0.0;
  const double S3 = q.S * q.S * q.S;
  r.Qhat = q.Gamma_hat * meanE;
  r.CH = q.s_zero ? nan : q.Gamma_hat * meanE / (S3 * A_ref);
  r.CH_sigma = q.s_zero ? nan : q.Gamma_hat / (S3 * A_ref) * sqrt(varE / N);
  r.rays = (uint64_t)s[kRays];
  r.hits = (uint64_t)s[kHits];
  r.segments = (uint64_t)s[kSegments];
  r.missed = (uint64_t)s[kMissed];
  r.escaped = (uint64_t)s[kEscaped];
  r.capped = (uint64_t)s[kCapped];
  r.tr_capped = (uint64_t)s[kTrCap];
  r.guard_trips = (uint64_t)s[kGuard];
  r.preculled = (uint64_t)s[kPreculled];
  out[i] = r;
}

// Dynamic LDS of the tallies: the workgroup tally of lds_tris triangles, the
// per-lane slots of <= 2-triangle meshes, or per-wave totals (persistent
// kernel only; the plain kernel keeps totals in registers); the mixed mode
// of serving steps holds both a workgroup tally and per-wave totals.
size_t tally_lds_bytes(TallyMode mode, uint32_t lds_tris, bool persistent, bool wave_totals = false) {
  switch (mode) {
    case kTallyLds: return (size_t)lds_tris * 7 * sizeof(unsigned long long);
    case kTallyAuto:  // per-triangle area, then (persistent, if any entry keeps totals only) the per-wave totals
      return ((size_t)lds_tris * 7 + (persistent && wave_totals ? (size_t)7 * kWaves : 0)) * sizeof(unsigned long long);
    case kTallyLane: return (size_t)2 * 7 * kBlock * sizeof(unsigned long long);
    case kTallyTotals: return persistent ? (size_t)7 * kWaves * sizeof(unsigned long long) : 0;
    default: return 0;
  }
}

template <int STACK, bool COUNT>
void launch_trace_mode(const TraceArgs& a, TallyMode mode, int grid, hipStream_t st) {
  const size_t lds = tally_lds_bytes(mode, a.nt, false);
  switch (mode) {
    case kTallyGlobal: trace_kernel<STACK, kTallyGlobal, COUNT><<<grid, kBlock, lds, st>>>(a); break;
    case kTallyLds: trace_kernel<STACK, kTallyLds, COUNT><<<grid, kBlock, lds, st>>>(a); break;
    case kTallyLane: trace_kernel<STACK, kTallyLane, COUNT><<<grid, kBlock, lds, st>>>(a); break;
    default: trace_kernel<STACK, kTallyTotals, COUNT><<<grid, kBlock, lds, st>>>(a); break;
  }
}

template <int STACK>
void launch_trace_stack(const TraceArgs& a, TallyMode mode, int grid, hipStream_t st) {
  if (a.counters) launch_trace_mode<STACK, true>(a, mode, grid, st);
  else launch_trace_mode<STACK, false>(a, mode, grid, st);
}

template <int STACK>
void launch_batch_mode(const BatchArgs& a, TallyMode mode, int grid, hipStream_t st) {
  const size_t lds = tally_lds_bytes(mode, a.lds_tris, true, a.wave_totals != 0u);
  switch (mode) {
    case kTallyLane: batch_kernel<STACK, kTallyLane><<<grid, kBlock, lds, st>>>(a); break;
    case kTallyLds: batch_kernel<STACK, kTallyLds><<<grid, kBlock, lds, st>>>(a); break;
    case kTallyTotals: batch_kernel<STACK, kTallyTotals><<<grid, kBlock, lds, st>>>(a); break;
    case kTallyAuto: batch_kernel<STACK, kTallyAuto><<<grid, kBlock, lds, st>>>(a); break;
    default: batch_kernel<STACK, kTallyGlobal><<<grid, kBlock, lds, st>>>(a); break;
  }
}

static_assert(sizeof(QueryDev) % 8 == 0 && kScalarSlots <= kBlock, "admission copies 8-byte words");

// Serving admission, entry blockIdx.y: the slot's constants and cleared
// scalar block (first workgroup), its per-triangle tally words (all).
__global__ __launch_bounds__(kBlock) void admit_kernel(const AdmitRec* __restrict__ rec, QueryDev* __restrict__ qs,
                                                       long long* __restrict__ scal, long long* __restrict__ tally) {
  const AdmitRec& r = rec[blockIdx.y];
  if (blockIdx.x == 0) {
    const uint64_t* src = reinterpret_cast<const uint64_t*>(&r.q);
    uint64_t* dst = reinterpret_cast<uint64_t*>(qs + r.slot);
    for (uint32_t w = threadIdx.x; w < sizeof(QueryDev) / 8; w += kBlock) dst[w] = src[w];
    if (threadIdx.x < (uint32_t)kScalarSlots) scal[(uint64_t)r.slot * kScalarSlots + threadIdx.x] = 0;
  }
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < r.tally_words; i += (uint64_t)gridDim.x * kBlock)
    tally[r.tally_off + i] = 0;
}

}  // namespace

void launch_admit(const AdmitRec* rec, uint32_t n, uint64_t max_words, QueryDev* qs, long long* scal,
                  long long* tally, hipStream_t st) {
  const uint64_t gx = (max_words + kBlock - 1) / kBlock;
  const dim3 g((uint32_t)(gx < 1 ? 1 : (gx > 1024 ? 1024 : gx)), n);
  admit_kernel<<<g, kBlock, 0, st>>>(rec, qs, scal, tally);
}

// Check of the two-stage seeding's estimate: over particles [0, n) of one
// query, the largest distance between the estimated and the exact ray as a
// fraction of the margin (out[0], the bits of a non-negative double: they
// order as integers), and the number of particles the estimate covered
// (out[1]).  Distance = |o_est - o| + 2 r |w_est / |w_est| - w / |w||: how
// far apart the two rays can get along the at most 2 r of path in the CV.
__global__ __launch_bounds__(kBlock) void precull_check_kernel(const QueryDev* __restrict__ qp, uint64_t n,
                                                               unsigned long long* __restrict__ out) {
  const QueryDev& q = *qp;
  double worst = 0.0;
  unsigned long long cnt = 0;
  for (uint64_t pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x; pid < n; pid += (uint64_t)gridDim.x * kBlock) {
    float o[3], w[3];
    if (!precull_estimate(q, g_lat_fine, g_vn_start, pid, o, w)) continue;
    double x[3], we[3];
    seed_particle(q, g_lat_start, g_lat_fine, g_vn_start, g_sc_tab, g_ee_tab, pid, x, we);
    double dp = 0.0, nw = 0.0, ne = 0.0, dd = 0.0;
    for (int c = 0; c < 3; ++c) {
      dp += ((double)o[c] - x[c]) * ((double)o[c] - x[c]);
      nw += (double)w[c] * (double)w[c];
      ne += we[c] * we[c];
    }
    nw = sqrt(nw);
    ne = sqrt(ne);
    for (int c = 0; c < 3; ++c) dd += ((double)w[c] / nw - we[c] / ne) * ((double)w[c] / nw - we[c] / ne);
    const double ratio = (sqrt(dp) + 2.0 * q.r * sqrt(dd)) / ((double)kPrecullMargin * q.r);
    worst = ratio == ratio ? fmax(worst, ratio) : __builtin_inf();  // a NaN estimate counts as unbounded
    ++cnt;
  }
  atomicMax(out, (unsigned long long)__double_as_longlong(worst));
  atomicAdd(out + 1, cnt);
}

void launch_precull_check(const QueryDev* d_q, uint64_t n, unsigned long long* out, int grid, hipStream_t st) {
  zero_i64_kernel<<<1, kBlock, 0, st>>>(reinterpret_cast<long long*>(out), 2);
  precull_check_kernel<<<grid, kBlock, 0, st>>>(d_q, n, out);
}

#if TPMC_PHASE_PROBE
bool probe_built() { return true; }

hipError_t probe_read(unsigned long long* out, bool reset, hipStream_t st) {
  unsigned long long* d = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&d, HIP_SYMBOL(g_probe));
  if (e == hipSuccess) e = hipMemcpyAsync(out, d, kProbeSlots * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && reset) {
    zero_i64_kernel<<<1, kBlock, 0, st>>>(reinterpret_cast<long long*>(d), kProbeSlots);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}
#else
bool probe_built() { return false; }

hipError_t probe_read(unsigned long long*, bool, hipStream_t) { return hipErrorNotSupported; }
#endif

hipError_t init_seed_tables(hipStream_t st) {
  float* tab = nullptr;
  float* lat = nullptr;
  float* fine = nullptr;
  double* sc = nullptr;
  double* ee = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&tab, HIP_SYMBOL(g_vn_start));
  if (e == hipSuccess) e = hipGetSymbolAddress((void**)&lat, HIP_SYMBOL(g_lat_start));
  if (e == hipSuccess) e = hipGetSymbolAddress((void**)&fine, HIP_SYMBOL(g_lat_fine));
  if (e == hipSuccess) e = hipGetSymbolAddress((void**)&sc, HIP_SYMBOL(g_sc_tab));
  if (e == hipSuccess) e = hipGetSymbolAddress((void**)&ee, HIP_SYMBOL(g_ee_tab));
  if (e != hipSuccess) return e;
  sc_table_kernel<<<1, 256, 0, st>>>(sc);
  ee_table_kernel<<<(kExpErfcN + 255) / 256, 256, 0, st>>>(ee);  // before the solves that read it
  vn_table_kernel<<<(kVnNS * kVnNT + 255) / 256, 256, 0, st>>>(tab, ee);
  lat_table_kernel<<<(kLatNS * kLatNT + 255) / 256, 256, 0, st>>>(lat, ee);
  lat_fine_kernel<<<(kLatFNS * kLatFNT + 255) / 256, 256, 0, st>>>(fine, ee);
  e = hipGetLastError();
  return e != hipSuccess ? e : hipStreamSynchronize(st);
}

void zero_i64(long long* p, uint64_t n, hipStream_t st) {
  if (n) zero_i64_kernel<<<grid_for(n, 4096), kBlock, 0, st>>>(p, n);
}

void zero_u32(uint32_t* p, uint64_t n, hipStream_t st) {
  if (n) zero_u32_kernel<<<grid_for(n, 4096), kBlock, 0, st>>>(p, n);
}

int stack_slots_for_depth(uint32_t depth) {
  if (depth <= 4) return 4;
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
    case 4: launch_trace_stack<4>(a, mode, grid, st); break;
    case 8: launch_trace_stack<8>(a, mode, grid, st); break;
    case 16: launch_trace_stack<16>(a, mode, grid, st); break;
    case 32: launch_trace_stack<32>(a, mode, grid, st); break;
    default: launch_trace_stack<64>(a, mode, grid, st); break;
  }
}

void launch_batch(const BatchArgs& a, int stack_slots, TallyMode mode, int grid, hipStream_t st) {
  switch (stack_slots) {
    case 4: launch_batch_mode<4>(a, mode, grid, st); break;
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

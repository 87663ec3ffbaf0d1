// tpmc_launch.h -- host-side launchers of the HIP kernels (defined in the .hip files).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tpmc_internal.h"

namespace tpmc {

// Tally strategy of the trace kernels.
// Auto: per query, global per-triangle atomics or register totals (serving steps
// that mix both kinds of request).
enum TallyMode { kTallyGlobal = 0, kTallyLds = 1, kTallyLane = 2, kTallyTotals = 3, kTallyAuto = 4 };

struct TraceArgs {
  const Node* nodes;
  const TriRec* tris;
  const uint32_t* orig;
  const QueryDev* q;          // device pointer, one query
  const float* x[3];          // SoA planes, already offset to the query
  const float* w[3];
  uint64_t n;
  long long* tally;           // [nt][7] or null (totals mode)
  long long* scal;            // [kScalarSlots]
  int32_t* first_tri;         // optional, already offset to the query
  unsigned long long* counters;  // optional [2]: BVH nodes visited, triangle tests
  uint32_t nt;
  uint32_t refill;            // serve ended segments when fewer lanes of a wave traverse (1..64)
};

// One persistent launch covers n_entries entries; entry j is entry_tiles[j]
// tiles of query entry_query[j] starting at tile entry_tile0[j] (a whole batch:
// entry j = query j from tile 0; a serving step: any slots, any ranges).
// Waves claim work entry by entry in units of a quarter tile (a whole tile
// when the tile is not a multiple of 256 particles; entry_next[j] counts the
// claimed units), so a wave stays on one query and flushes its partial sums
// only when it moves to another.  With workgroup LDS tallies the workgroup's
// waves move to another entry together.
struct BatchArgs {
  const QueryDev* qs;              // query / slot table (meshes referenced per query)
  const uint32_t* entry_query;     // [n_entries] or null (entry j is query j)
  const uint64_t* entry_tile0;     // [n_entries] or null (start at tile 0)
  const uint64_t* entry_tiles;     // [n_entries] tiles to trace per entry
  unsigned long long* entry_next;  // [n_entries] claim counters, zeroed before the launch
  long long* tally_base;           // per-triangle tallies, indexed by QueryDev::tally_offset
  long long* scal_base;            // scalar blocks, indexed by QueryDev::scalar_offset
  uint32_t n_entries;
  uint32_t refill;                 // as TraceArgs::refill
  uint64_t tile;                   // particles per tile (multiple of 64)
  uint32_t lds_tris;               // largest nt of an entry with an LDS tally (kTallyLds / kTallyAuto)
  uint32_t wave_totals;            // kTallyAuto: some entry keeps totals only (per-wave LDS totals allocated)
  // Where each XCD's workgroups start claiming: XCD x (workgroups x, x + 8, ...; the
  // hardware deals workgroups to the eight XCDs in turn) starts in entries
  // [xcd_start[x], xcd_start[x + 1]) (entries grouped by mesh, ranges by tile share),
  // so that each XCD's L2 holds the hierarchies of few meshes; all 0: entry
  // blockIdx % n_entries.
  uint32_t xcd_start[9];
};

void zero_i64(long long* p, uint64_t n, hipStream_t st);
// Fills the seeding start table of the current device (once per device).
hipError_t init_seed_tables(hipStream_t st);
void zero_u32(uint32_t* p, uint64_t n, hipStream_t st);

size_t bvh_scratch_bytes(uint64_t nt);
// Supporting-plane flags in bits 30 / 31 of orig[] (after build_bvh; see tpmc_bvh.hip).
void mark_support(const float* d_xyz, uint64_t nv, const TriRec* d_tris, uint64_t nt, uint32_t* d_orig,
                  hipStream_t st);
constexpr uint32_t kOrigIdMask = 0x3FFFFFFFu;  // orig[] bits 0..29: original triangle index
hipError_t build_bvh(const float* d_xyz, const uint32_t* d_tri, uint64_t nt, const float box_lo[3],
                     const float box_hi[3], void* scratch, Node* d_nodes, TriRec* d_tris, uint32_t* d_orig,
                     uint32_t* h_depth, hipStream_t st);

// Top-down binned-SAH hierarchy in the same node / leaf format (default builder).
size_t sah_scratch_bytes(uint64_t nt);
hipError_t build_bvh_sah(const float* d_xyz, const uint32_t* d_tri, uint64_t nt, void* scratch, Node* d_nodes,
                         TriRec* d_tris, uint32_t* d_orig, uint32_t* h_depth, hipStream_t st);

int stack_slots_for_depth(uint32_t depth);  // 0 when too deep
void launch_seed(const QueryDev* d_q, uint64_t n, float* const x[3], float* const w[3], int grid, hipStream_t st);
void launch_trace(const TraceArgs& a, int stack_slots, TallyMode mode, int grid, hipStream_t st);
void launch_reduce(const long long* tally, uint32_t nt, long long* scal, hipStream_t st);
void launch_finalize(const QueryDev* d_qs, const uint32_t* d_idx, const long long* scal_base, uint32_t nq, double xr,
                     double yr, double zr, double A_ref, ResultDev* out, hipStream_t st);
void launch_reduce_slots(const QueryDev* d_qs, const uint32_t* d_idx, uint32_t n, long long* tally_base,
                         long long* scal_base, uint32_t max_nt, hipStream_t st);
void launch_batch(const BatchArgs& a, int stack_slots, TallyMode mode, int grid, hipStream_t st);
// Check of the two-stage seeding's estimate (precull_check_kernel): out[0] the
// bits of the largest error / margin, out[1] the particles estimated.
void launch_precull_check(const QueryDev* d_q, uint64_t n, unsigned long long* out, int grid, hipStream_t st);
// Phase probe: whether this library was built with it; the readout copies the
// kProbeSlots sums of the current device into out (after the stream's work)
// and clears them when reset.
bool probe_built();
hipError_t probe_read(unsigned long long* out, bool reset, hipStream_t st);
// Serving admission: n records (device) -> constants into qs[slot], cleared
// scalar block and per-triangle tally words; max_words is the largest tally.
void launch_admit(const AdmitRec* rec, uint32_t n, uint64_t max_words, QueryDev* qs, long long* scal,
                  long long* tally, hipStream_t st);

// Ceiling microkernels (tpmc_ceilings.hip).  kind 0: FP32 FMA, 1: FP64 FMA,
// 2: int32 multiply and add; each lane performs ceiling_valu_ops_per_lane(iters)
// of them.
void launch_ceiling_valu(uint32_t kind, int grid, uint32_t iters, void* sink, hipStream_t st);
uint64_t ceiling_valu_ops_per_lane(uint32_t iters);
void launch_ceiling_read(const void* p, uint64_t bytes, uint32_t passes, int grid, hipStream_t st);
void launch_ceiling_atomic(void* p, uint32_t slots, uint32_t per_thread, int grid, hipStream_t st);
void launch_ceiling_lds_atomic(void* sink, uint32_t slots, uint32_t per_thread, int grid, hipStream_t st);
void launch_reduce_batch(const QueryDev* d_qs, uint32_t nq, long long* tally_base, long long* scal_base,
                         uint32_t max_nt, hipStream_t st);

}  // namespace tpmc

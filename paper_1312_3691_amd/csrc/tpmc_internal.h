// tpmc_internal.h -- layouts shared by the host side of libtpmc and its HIP kernels.
#pragma once

#include <stdint.h>

namespace tpmc {

constexpr int kBlock = 256;            // threads per workgroup (4 wave64s)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxReflections = 64;
constexpr int kLdsTallyMaxTris = 512;  // per-workgroup LDS tallies up to this mesh size
constexpr int kLaneTallyMaxTris = 2;   // per-lane LDS tallies for tiny meshes
constexpr int kScalarSlots = 21;       // int64 per query, see ScalarSlot

// Per-query int64 block.  D is the momentum one particle gives the body along
// the free stream (sum over its hits of (w - w').U); D and D^2 are quantised
// per particle, so every sum is an exact integer sum and independent of order.
enum ScalarSlot {
  kSD = 0, kSD2 = 1, kRays = 2, kHits = 3, kSegments = 4, kMissed = 5, kEscaped = 6, kCapped = 7,
  kFx = 8, kFy = 9, kFz = 10, kLx = 11, kLy = 12, kLz = 13, kCount = 14,
  kSE = 15, kSE2 = 16,  // per-particle energy E = sum over hits of |w|^2 - |w'|^2, and E^2
  kTrCap = 17,          // diffuse re-emissions whose temperature the kernel's bound limited
  kGuard = 18,          // ray segments ended by the traversal step bound (a damaged tree)
  kPreculled = 19,      // particles the seeding estimate showed to miss the root's boxes (batched kernel)
  kPrecullOff = 20      // nonzero once the batched kernel has switched the estimate off for this query
};

// Phase probe of the batched kernel (compiled in only with TPMC_PHASE_PROBE=1):
// sums over the waves of every launch since the last reset.  Cycles are
// shader-clock ticks a wave spends in a phase; lanes are the active lanes of
// each pass, summed.  The slot numbers are the TPMC_PROBE_* ones of the
// public header.
enum ProbeSlot {
  kPrWaves = 0, kPrCycles = 1,                                                    // waves; cycles start to exit
  kPrClaimCyc = 2, kPrClaims = 3,                                                 // tile claims and tile ends
  kPrTravCyc = 4, kPrTravSteps = 5, kPrTravLanes = 6,                             // traversal steps
  kPrLeafCyc = 7, kPrLeafPasses = 8, kPrLeafLanes = 9,                            // leaf phases
  kPrServeCyc = 10, kPrServes = 11, kPrServeLanes = 12,                           // service passes
  kPrEstCyc = 13, kPrEstBatches = 14, kPrEstLanes = 15, kPrEstKept = 16,          // estimate (stage 1)
  kPrSeedCyc = 17, kPrSeedBatches = 18, kPrSeedLanes = 19, kPrSeedKept = 20,      // exact seeding + root test
  kPrAssignCyc = 21, kPrAssigns = 22, kPrAssignLanes = 23,                        // queue -> idle lanes
  kProbeSlots = 24
};

// Fine table of the latitude root mu of G(mu) = u Z(S): the seeding estimate
// takes it as it is (no iteration), the exact FP64 solve starts from it (one
// Halley step then ends the solve).  Rows ln S = kLatFL0 +
// i kLatFDL (S from about 0.23 to 10.6), interpolated by the four-point
// Lagrange cubic in ln S whose rows and weights the host sets per query
// (QueryDev::lat_f0, lat_fw), columns t = kLatFT0 + j kLatFDT in the logit
// t = ln(u / (1 - u)), linear.  Filled once per device by FP64 bisection.
// Its error in mu is below 1e-5 (a dense host evaluation of the interpolation
// against FP64 roots found at most 9e-6 where cos(phi) >= 0.05, 3.5e-5 of
// cos(phi), and 5.5e-6 over draws from the whole range, poles included);
// tpmc_precull_check measures the rays it gives against the exact seeding.
constexpr int kLatFNS = 192, kLatFNT = 3073;
constexpr double kLatFL0 = -1.45, kLatFDL = 0.02;
constexpr float kLatFT0 = -24.0f, kLatFDT = 1.0f / 64.0f;
constexpr double kLatFSmin = 0.25, kLatFSmax = 10.0;  // the S range the estimate takes from it

struct Node;
struct TriRec;

// Device-side constants of one query (a1: FP64 set-up done on the host).
struct alignas(16) QueryDev {
  double U[3], e1[3], e2[3], c0[3];  // free stream and seeding frame, CV centre (body frame)
  double r;                          // CV radius
  double S;                          // speed ratio
  double Z;                          // normaliser of the latitude density, = G(1)
  double erfS, erfcS, expmS2;        // erf(S), erfc(S), exp(-S^2)
  double inv_scaleF, inv_scaleL, inv_scaleD, inv_scaleD2;
  double Gamma_hat;
  uint64_t N;                        // particles of this query
  uint64_t p_offset;                 // first particle in the SoA planes (plain path)
  uint64_t tally_offset;             // first int64 of this query's per-triangle tallies
  uint64_t scalar_offset;            // first int64 of this query's scalar block
  const Node* nodes;                 // the query's mesh (resident BVH)
  const TriRec* tris;
  const uint32_t* orig;
  float Uf[3], c0f[3];
  float tau, alpha;
  float scaleF, scaleL, scaleD, scaleD2;  // fixed-point scales, powers of two
  uint32_t key0, key1;               // Philox key = seed
  uint32_t rmax;
  uint32_t s_zero;                   // S treated as exactly 0
  uint32_t per_tri;                  // per-triangle tallies kept
  uint32_t nt;                       // triangles of the query's mesh
  uint32_t box;                      // box control volume (faces f = 2k: outward -e_k, 2k + 1: +e_k)
  uint32_t pad_;
  double h[3];                       // box half-extents
  double face_s[6];                  // s_f = S U.n_f, n_f the inward normal of face f
  double face_cum[6];                // cumulative A_f chi(s_f)
  double inv_scaleE, inv_scaleE2;
  float alpha_E;                     // energy accommodation of diffuse re-emission
  float tr_cap2;                     // cap of the re-emission temperature tau_r^2
  float scaleE, scaleE2;             // fixed-point scales of E and E^2
  uint32_t eacc;                     // energy accommodation on (else tau_r = tau)
  uint32_t pad2_;
  double lat_k;                      // sqrt(pi) / (4 S), the erf term's factor in the latitude CDF
  // FP32 copies for the seeding estimate of the pre-cull (precull_may_enter)
  float e1f[3], e2f[3];
  float Sf, rf;
  int32_t lat_f0;     // first of the four fine-table rows around ln S (-1: S outside the table)
  float lat_fw[4];    // their cubic Lagrange weights at ln S
};

// Device result of the finalisation kernel (mirrors tpmc_result).
struct ResultDev {
  double F_over_q[3], M_over_q[3], Fhat[3];
  double CD, CD_sigma, Gamma_hat;
  uint64_t rays, hits, segments, missed, escaped, capped;
  double Qhat, CH, CH_sigma;
  double Mhat[3];
  uint64_t tr_capped, guard_trips, preculled;
};

// One slot admitted by a serving step's admission kernel: its constants and
// the per-triangle tally words it clears (none for totals-only requests).
struct alignas(16) AdmitRec {
  QueryDev q;
  uint32_t slot, pad;
  uint64_t tally_off, tally_words;
};

// BVH node: the boxes of both children and the two child links (64 bytes).
// A link >= 0 is an internal node; a link < 0 is the leaf ~link, a position in
// the Morton-sorted triangle array.
struct alignas(16) Node {
  float lo0x, lo0y, lo0z, hi0x;
  float hi0y, hi0z, lo1x, lo1y;
  float lo1z, hi1x, hi1y, hi1z;
  int32_t c0, c1, parent, pad;
};

// Triangle record in Morton order: vertices and unit geometric normal (48 bytes).
struct alignas(16) TriRec {
  float v0x, v0y, v0z, nx;
  float v1x, v1y, v1z, ny;
  float v2x, v2y, v2z, nz;
};

}  // namespace tpmc

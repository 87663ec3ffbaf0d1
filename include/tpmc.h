/*
 * tpmc.h -- C ABI of the MI355X test-particle Monte Carlo (TPMC) drag library.
 *
 * Method: J. B. Parham and L. A. Barba, "Finding the Force -- Consistent
 * Particle Seeding for Satellite Aerodynamics" (AIAA).  A drag query seeds N
 * test particles on a spherical control volume (CV) enclosing the body with
 * the flux-correct drifting-Maxwellian boundary distribution (Sec. III.A),
 * follows each through a triangulated surface by closest-hit ray tracing with
 * specular / diffuse (Maxwell) re-emission (Sec. II.A, multiple reflections
 * Sec. I), and sums the momentum each particle gives each triangle into force,
 * moment and drag coefficient (eq. drag; effective mass Sec. II.A).
 *
 * Conventions
 *  - Every function returns tpmc_status; TPMC_OK = 0.  No C++ exception
 *    crosses the ABI.  tpmc_last_error() returns the calling thread's last
 *    error message (valid until that thread's next call).
 *  - Handles are opaque and owned by the caller, who destroys them.  Destroy
 *    functions accept NULL.
 *  - Host arrays passed in are read during the call and never retained.
 *  - "Device" pointers are HIP device memory of the context's device.  The
 *    library allocates device memory only in tpmc_build_mesh (the resident
 *    BVH); every per-query buffer lives in a caller-provided workspace.
 *  - Work is enqueued on the context's HIP stream.  tpmc_seed, tpmc_trace and
 *    tpmc_batch_launch are asynchronous; tpmc_forces, tpmc_tally_copy,
 *    tpmc_batch_results and tpmc_server_results synchronise the stream.
 *  - Velocities are dimensionless, w = v / c_mp (Nomenclature: c_mp is the
 *    most probable thermal speed of the free stream).  Lengths are metres in
 *    the body frame.  All results are in the body frame.
 *  - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef TPMC_H
#define TPMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPMC_ABI_VERSION 9

typedef enum {
  TPMC_OK = 0,
  TPMC_E_INVALID = 1,   /* bad argument: NULL handle, non-finite or out-of-range query field */
  TPMC_E_MESH = 2,      /* nt == 0, index >= nv, non-finite vertex, BVH deeper than supported */
  TPMC_E_CV = 3,        /* the control volume does not enclose every vertex */
  TPMC_E_WORKSPACE = 4, /* workspace NULL, misaligned (256 B) or smaller than required */
  TPMC_E_DEVICE = 5,    /* a HIP call failed; message has the HIP error string */
  TPMC_E_BUSY = 6       /* handle belongs to another context / batch not launched */
} tpmc_status;

typedef struct tpmc_ctx_s* tpmc_ctx;
typedef struct tpmc_mesh_s* tpmc_mesh;
typedef struct tpmc_particles_s* tpmc_particles;
typedef struct tpmc_tally_s* tpmc_tally;
typedef struct tpmc_batch_s* tpmc_batch;

/* One drag query: the paper's problem statement (mesh separately). */
typedef struct {
  double q_wxyz[4];          /* attitude: unit quaternion (|q| within 1e-6 of 1) of the rotation
                                body -> wind axes; the free stream runs along +x of the wind axes,
                                so its body-frame direction U is the first row of R(q), and the
                                second and third rows are the seeding tangents e1, e2 */
  double S;                  /* speed ratio U_inf / c_mp (Sec. II.B), 0 <= S <= 100; S == 0 is
                                a gas at rest (then CD, CD_sigma and F_over_q are NaN) */
  double T_inf, T_w;         /* free-stream and wall temperature, K, > 0; only
                                tau = sqrt(T_w / T_inf) enters the dimensionless results */
  double alpha;              /* Maxwell accommodation: probability of diffuse re-emission, [0, 1] */
  uint64_t n_particles;      /* N >= 1 test particles */
  uint64_t seed;             /* Philox4x32-10 key; particle p uses counter (p lo, p hi, step, 0) */
  uint32_t max_reflections;  /* hit cap per particle, 1..64; a particle reaching it retires as capped */
  uint32_t flags;            /* TPMC_Q_* bits */
  double cv_center[3];       /* control-volume centre, used when cv_radius > 0 */
  double cv_radius;          /* CV radius (m); <= 0: centre = vertex-box centre, radius = largest
                                vertex distance times (1 + 1e-3).  With TPMC_Q_BOX_CV: the half-side
                                of a cube about cv_center; <= 0: the vertex box widened on every
                                axis by 1e-3 of its half-diagonal */
  double energy_accommodation; /* alpha_E in [0, 1], read only with TPMC_Q_ENERGY_ACC (else 1) */
} tpmc_query;

#define TPMC_Q_NO_TRIANGLE_TALLY 1u /* batched path: keep only per-query totals */
/* Seed on an axis-aligned box of the body frame instead of a sphere (the
 * rectangular control volume of Sec. III.A, with the correct inflow): a face
 * is chosen by its share A_f chi(s_f) of the inflow (s_f = S U.n_f, n_f its
 * inward normal, chi(s) = e^{-s^2} + sqrt(pi) s (1 + erf s)), the point is
 * uniform on it, the normal speed follows eq. vel_dist1 with S_n = s_f and the
 * two tangential components are Gaussian (eqs. vel_dist2-3) about the
 * tangential drift; Gamma_hat = sum_f A_f chi(s_f) / (2 sqrt(pi)).  Draws:
 * face r0.a, position r0.b and r1.b, normal speed r0.c, Box-Muller r0.d and
 * r1.a. */
#define TPMC_Q_BOX_CV 2u
/* Diffuse re-emission with incomplete energy accommodation ("momentum and
 * energy" exchange, Sec. I): with alpha_E = (E_i - E_r) / (E_i - E_w) (Sentman)
 * and E = 2kT the flux-weighted mean energy of a re-emitted Maxwellian, a
 * molecule of incident velocity w leaves diffusely at the temperature
 * tau_r^2 = alpha_E tau^2 + (1 - alpha_E) |w|^2 / 2 (units of T_inf).
 * alpha_E = 1 is the default model.  Limit of this implementation, not of the
 * model: the kernel bounds tau_r by max(tau, 8 (S + 15)) so that its
 * fixed-point tallies stay in range; inside a cavity the bound can bind only
 * at the far tail of the chain of re-emissions (tau_r^2 grows by a random
 * factor per re-emission), and every re-emission it limits is counted in
 * tpmc_result.tr_capped (a result with tr_capped > 0 departs from the model). */
#define TPMC_Q_ENERGY_ACC 4u

/* Result of one query.  Force and moment are divided by the dynamic pressure
 * q = rho U^2 / 2 (so they are areas, m^2, and m^3); Fhat = F / (rho c_mp^2)
 * and Mhat = M / (rho c_mp^2) are finite at S = 0 (a gas at rest).
 * CD = (F/q).U / A_ref; CD_sigma is its one-sigma statistical error from the
 * per-particle momentum along U. */
typedef struct {
  double F_over_q[3], M_over_q[3], Fhat[3];
  double CD, CD_sigma, Gamma_hat; /* Gamma_hat = Gamma / (n c_mp): CV number flux (Sec. III.A.1) */
  uint64_t rays;     /* particles traced (= N) */
  uint64_t hits;     /* particle-surface hits, re-hits included */
  uint64_t segments; /* rays cast: hits + particles that left the body or missed it */
  uint64_t missed;   /* particles that never hit */
  uint64_t escaped;  /* particles that hit at least once and then left */
  uint64_t capped;   /* particles retired at max_reflections */
  double Qhat;       /* energy given to the body per unit time / (n c_mp m c_mp^2 / 2) */
  double CH, CH_sigma; /* heat-transfer coefficient Q / (rho U^3 A_ref / 2) and its sigma (NaN at S = 0) */
  double Mhat[3];    /* moment about ref_point / (rho c_mp^2), m; finite at S = 0 (Fhat's counterpart) */
  uint64_t tr_capped;   /* diffuse re-emissions whose temperature the kernel's bound limited
                           (TPMC_Q_ENERGY_ACC only; 0 when the result follows the model exactly) */
  uint64_t guard_trips; /* ray segments ended by the traversal's step bound instead of by the
                           search (a damaged hierarchy); 0 for every valid mesh */
  uint64_t preculled;   /* of the missed particles, those the batched path's seeding estimate
                           showed to miss the BVH root's boxes before their exact seeding (a
                           work count: the plain path reports 0, and every other field is the
                           same either way) */
} tpmc_result;

typedef struct {
  uint64_t nv, nt;
  uint32_t depth;        /* BVH depth (root = 0) */
  uint32_t stack_slots;  /* traversal stack depth the trace kernel uses */
  double box_lo[3], box_hi[3];
  double sphere_center[3], sphere_radius; /* default control volume */
  uint64_t device_bytes; /* resident BVH + triangle records */
  uint32_t builder;      /* tpmc_bvh_builder the hierarchy was built with */
  uint32_t reserved;     /* 0 */
} tpmc_mesh_info;

const char* tpmc_last_error(void);
int tpmc_abi_version(void);

/* Context on HIP device `device` issuing work on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  Reads device properties; allocates nothing.  The
 * first context on a device also fills a small table in the library's code
 * object (starting points of the normal-speed solve, one kernel, synchronised). */
tpmc_status tpmc_create(int device, void* hip_stream, tpmc_ctx* out);
tpmc_status tpmc_set_stream(tpmc_ctx ctx, void* hip_stream);
void tpmc_destroy_ctx(tpmc_ctx ctx);

/* Launch tuning of a context.  No setting changes any result: particles are
 * independent (Sec. II.A), each draws from its own counter-based stream, and
 * every sum is an exact integer sum, so results are bit-identical under any
 * tuning.  Set by the autotuner (paper_1312_3691_amd/autotune.py) or by hand;
 * a context starts with the defaults below. */
typedef struct {
  uint32_t refill_lanes;   /* 1..64, default 32: a wave serves the lanes whose ray segment has ended
                              (re-emission, tallies, next segment or particle) once fewer than this
                              many of its 64 lanes are still traversing */
  uint32_t tile_particles; /* multiple of 64 in [64, 65536], default 16384: particles per work tile
                              of the persistent kernel; read when a batch or server is created */
  uint32_t groups_per_cu;  /* 1..32, default 8: workgroups (256 lanes) per compute unit of the
                              persistent launches (batches and server steps) */
  uint32_t plain_groups_per_cu; /* 0..32, default 4 (0 selects it): cap, in workgroups per compute
                              unit, of the grid of tpmc_trace; the grid also keeps at least four
                              particles per lane, so small queries get fewer workgroups */
} tpmc_tuning;

/* Copy out / replace the context's tuning.  set validates every field
 * (TPMC_E_INVALID, nothing changed, on any field out of range). */
tpmc_status tpmc_get_tuning(tpmc_ctx ctx, tpmc_tuning* out);
tpmc_status tpmc_set_tuning(tpmc_ctx ctx, const tpmc_tuning* t);

/* Bounding-volume hierarchy builders (both on the device, same node format).
 * The hierarchy changes only speed: the closest hit does not depend on it
 * (ties between equal t go to the lower original triangle index), so both
 * give bit-identical results. */
typedef enum {
  TPMC_BVH_SAH = 0,  /* default: top-down, binned surface-area heuristic (32 planes per axis
                        over the triangle box centres), one workgroup per node and level */
  TPMC_BVH_LBVH = 1  /* linear BVH: Karras 2012 hierarchy over 30-bit Morton codes of the
                        triangle centroids (fastest build, more node visits per ray) */
} tpmc_bvh_builder;

/* Mesh and its BVH (closest-hit tracing on a triangulation, Sec. II.A).
 *   xyz: host float [nv][3], metres, body frame.  tri: host uint32 [nt][3].
 * Triangles are two-sided; zero-area triangles are accepted and never hit.
 * Also marks, per triangle and side, whether the whole mesh lies on the other
 * side of its plane, so that a particle leaving that side provably cannot hit
 * again and escapes without being traced (exact; nt * nv FP64 distance
 * evaluations at build).  nt < 2^30, nv < 2^32.
 * Builds on the device (synchronises); the handle owns its device memory.
 * tpmc_build_mesh uses TPMC_BVH_SAH; tpmc_build_mesh_ex takes the builder
 * (TPMC_E_INVALID for any other value). */
tpmc_status tpmc_build_mesh(tpmc_ctx ctx, const float* xyz, uint64_t nv, const uint32_t* tri, uint64_t nt,
                            tpmc_mesh* out);
tpmc_status tpmc_build_mesh_ex(tpmc_ctx ctx, const float* xyz, uint64_t nv, const uint32_t* tri, uint64_t nt,
                               uint32_t builder, tpmc_mesh* out);
tpmc_status tpmc_get_mesh_info(tpmc_mesh mesh, tpmc_mesh_info* out);
void tpmc_destroy_mesh(tpmc_mesh mesh);

/* Bytes of device workspace tpmc_seed needs for these nq queries (particle
 * states 24 B each, per-triangle tallies 56 B per triangle per query, tables). */
tpmc_status tpmc_workspace_bytes(tpmc_ctx ctx, tpmc_mesh mesh, const tpmc_query* q, uint32_t nq,
                                 uint64_t* bytes);

/* Seed all particles of the nq queries (Sec. III.A.1-3) into the workspace:
 * FP64 inverse-CDF sampling of the incidence latitude (g(phi|S)) and of the
 * inward normal speed (eq. vel_dist1), Gaussian tangential components (eqs.
 * vel_dist2-3), stored as FP32 structure-of-arrays.  `dev_workspace` is device
 * memory of at least tpmc_workspace_bytes, 256-byte aligned, owned by the
 * caller and used until the particles and tally handles are destroyed. */
tpmc_status tpmc_seed(tpmc_ctx ctx, tpmc_mesh mesh, const tpmc_query* q, uint32_t nq, void* dev_workspace,
                      uint64_t ws_bytes, tpmc_particles* out);

/* Device views of the seeded states: six FP32 planes x0, x1, x2, w0, w1, w2,
 * each of n_total entries (query i occupies [sum_{j<i} N_j, ... + N_i)). */
tpmc_status tpmc_particles_planes(tpmc_particles p, float* dev_planes[6], uint64_t* n_total);

/* Trace every seeded particle: closest two-sided hit with t > 0 excluding the
 * triangle just left (equal t: lower triangle index), FP32 watertight test
 * (Woop, Benthin & Wald 2013); re-emission diffuse with probability alpha at
 * T_w (cosine law), else specular; per-triangle momentum and moment tallies in
 * exact int64 fixed point.  dev_first_tri (optional, int32 [n_total]) receives
 * each particle's first-hit triangle index, -1 when it missed.  dev_counters
 * (optional, uint64 [2], accumulated into, caller zeroes) receives the BVH
 * nodes visited and the ray-triangle tests made; it selects a counting
 * variant of the kernel, so leave it NULL when timing. */
tpmc_status tpmc_trace(tpmc_ctx ctx, tpmc_mesh mesh, tpmc_particles p, tpmc_tally* out);
tpmc_status tpmc_trace_ex(tpmc_ctx ctx, tpmc_mesh mesh, tpmc_particles p, int32_t* dev_first_tri,
                          uint64_t* dev_counters, tpmc_tally* out);

/* Reduce the tallies to force, moment about ref_point (body frame, m) and C_D
 * with reference area A_ref > 0 (eq. drag).  out: host [nq].  Synchronises. */
tpmc_status tpmc_forces(tpmc_ctx ctx, tpmc_tally t, const double ref_point[3], double A_ref, tpmc_result* out);

/* Per-triangle sums of one query, host double [nt][7]: sum of (w - w') xyz,
 * sum of p x (w - w') xyz about the body origin, hit count.  Synchronises. */
tpmc_status tpmc_tally_copy(tpmc_ctx ctx, tpmc_tally t, uint32_t query, double* host_per_tri);

void tpmc_destroy_particles(tpmc_particles p);
void tpmc_destroy_tally(tpmc_tally t);

/* ---- Batched path: many queries on one mesh in one persistent launch ----
 * Work items are (query, tile of particles); workgroups take them from a
 * device counter, seed the tile into LDS and trace it, so particle states
 * never go to HBM.  Results equal the plain path's bit for bit (same Philox
 * streams, same per-particle arithmetic, exact integer tallies). */
tpmc_status tpmc_batch_workspace_bytes(tpmc_ctx ctx, tpmc_mesh mesh, const tpmc_query* q, uint32_t nq,
                                       uint64_t* bytes);
/* Upload the query table and work map; returns a batch handle bound to the
 * workspace.  Does not launch the trace. */
tpmc_status tpmc_batch_create(tpmc_ctx ctx, tpmc_mesh mesh, const tpmc_query* q, uint32_t nq,
                              void* dev_workspace, uint64_t ws_bytes, tpmc_batch* out);
/* Enqueue zeroing, the persistent kernel and the reduction (asynchronous).
 * use_graph != 0 replays a HIP graph captured on the first call. */
tpmc_status tpmc_batch_launch(tpmc_ctx ctx, tpmc_batch b, int use_graph);
/* Wait and convert: out host [nq]. */
tpmc_status tpmc_batch_results(tpmc_ctx ctx, tpmc_batch b, const double ref_point[3], double A_ref,
                               tpmc_result* out);
void tpmc_destroy_batch(tpmc_batch b);

/* ---- Serving: continuous batching over resident meshes ----
 * A server is a table of request slots in a caller workspace.  A request is
 * admitted into a free slot (its constants uploaded, its tallies zeroed); each
 * step is ONE persistent launch over any set of (slot, tile range) entries --
 * slots of different meshes and sizes run together -- and tallies accumulate
 * exactly across steps, so a request's result does not depend on how its tiles
 * were spread over steps or which requests shared them.  Tiles hold the
 * context's tile_particles at tpmc_server_create (default 16384)
 * particles.  Slot and pool bookkeeping (admission by memory budget) is the
 * caller's policy; the library checks bounds. */
typedef struct tpmc_server_s* tpmc_server;
/* Workspace for max_slots slots and a per-triangle tally pool of tally_words int64. */
tpmc_status tpmc_server_workspace_bytes(uint32_t max_slots, uint64_t tally_words, uint64_t* bytes);
tpmc_status tpmc_server_create(tpmc_ctx ctx, uint32_t max_slots, uint64_t tally_words, void* dev_workspace,
                               uint64_t ws_bytes, tpmc_server* out);
/* Admit query q on mesh into slot (asynchronous).  Unless TPMC_Q_NO_TRIANGLE_TALLY,
 * its per-triangle tallies occupy pool words [tally_offset, tally_offset + 7 nt).
 * n_tiles receives the query's tile count. */
tpmc_status tpmc_server_admit(tpmc_server s, uint32_t slot, tpmc_mesh mesh, const tpmc_query* q,
                              uint64_t tally_offset, uint64_t* n_tiles);
/* Admit n requests at once (asynchronous): admission i puts q[i] on meshes[i]
 * into slots[i] (distinct slots) with its tallies at tally_offset[i], as
 * tpmc_server_admit does, with one upload and one launch for all of them.
 * Every admission is validated first; on any error nothing is admitted and the
 * message names the admission.  n_tiles (optional): host [n]. */
tpmc_status tpmc_server_admit_many(tpmc_server s, uint32_t n, const uint32_t* slots, const tpmc_mesh* meshes,
                                   const tpmc_query* q, const uint64_t* tally_offset, uint64_t* n_tiles);
/* One step: entry i traces tiles [tile0[i], tile0[i] + count[i]) of slots[i]
 * (n <= max_slots entries, each slot at most once).  Asynchronous; no call of
 * the server waits for a step already on the stream (its uploads go through
 * pinned host memory). */
tpmc_status tpmc_server_step(tpmc_server s, const uint32_t* slots, const uint64_t* tile0, const uint64_t* count,
                             uint32_t n);
/* Wait for the stream; results of the listed slots (out: host [n]). */
tpmc_status tpmc_server_results(tpmc_server s, const uint32_t* slots, uint32_t n, const double ref_point[3],
                                double A_ref, tpmc_result* out);
/* The same in two halves, so that a caller can enqueue its next step before it
 * reads the results of the last one: collect enqueues the reduction of the
 * listed slots and the copy of their results into host memory of the server
 * (asynchronous; ticket receives its number), collected waits for collection
 * `ticket` alone (not for later work on the stream) and copies its n results
 * out (host [n]).  At most two collections are in flight: a third collect
 * fails with TPMC_E_BUSY until the oldest is read.  A slot may be released and
 * admitted again once its collection has been enqueued. */
tpmc_status tpmc_server_collect(tpmc_server s, const uint32_t* slots, uint32_t n, const double ref_point[3],
                                double A_ref, uint32_t* ticket);
tpmc_status tpmc_server_collected(tpmc_server s, uint32_t ticket, tpmc_result* out, uint32_t n);
tpmc_status tpmc_server_release(tpmc_server s, uint32_t slot);
void tpmc_destroy_server(tpmc_server s);

/* ---- Batched path without allocation ----
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The batched
 * path (tpmc_batch_create + tpmc_batch_launch + tpmc_batch_results, same
 * kernels, same results) in one call, with its workspace in a static device
 * array of the library, TPMC_NOALLOC_MAX_BYTES bytes on each GPU it runs on,
 * held until the process ends.  No device memory is allocated or freed.
 * Queries whose batch workspace (tpmc_batch_workspace_bytes) is larger are
 * rejected with TPMC_E_WORKSPACE before any work is enqueued.  Every call on a
 * GPU uses that GPU's one array and leaves its contents behind (each call
 * clears what it accumulates into before its launch), so calls that overlap on
 * one GPU -- from two threads, or from two contexts on different streams --
 * race: the caller serialises them.  Synchronises the context's stream.
 * out: host [nq]; the other arguments as for tpmc_batch_create and
 * tpmc_batch_results. */
#define TPMC_NOALLOC_MAX_BYTES (32ull << 20)
tpmc_status tpmc_batch_run_noalloc(tpmc_ctx ctx, tpmc_mesh mesh, const tpmc_query* q, uint32_t nq,
                                   const double ref_point[3], double A_ref, tpmc_result* out);

/* Host-only checks (no device needed): the validation the entry points above
 * apply.  tpmc_check_query also needs the mesh vertices for the CV test. */
tpmc_status tpmc_check_mesh(const float* xyz, uint64_t nv, const uint32_t* tri, uint64_t nt);
tpmc_status tpmc_check_query(const tpmc_query* q, const float* xyz, uint64_t nv);

/* ---- Measured ceilings of the roofline ----
 * The path is not a dense contraction and its working set stays in the
 * caches, so it is bound by VALU issue, cache bandwidth and atomics rather
 * than by HBM.  These entry points time microkernels on the context's device
 * and stream (one untimed launch, then one launch between two events; they
 * synchronise the stream) and return the measured rate.  Buffers are the
 * caller's device memory; the library allocates nothing.  They change no
 * other state: the VALU and LDS kernels never write their sink (they keep
 * their work live through a store that only a one-thread workgroup would make).
 *   tpmc_ceiling_valu: kind 0 FP32 FMA, 1 FP64 FMA (lane FMAs per second), 2
 *     32-bit integer multiply plus add (lane multiplies per second; the
 *     Philox rounds are made of such products); sink >= 16 bytes.
 *   tpmc_ceiling_read: streams reads of 16 bytes per lane over bytes (a
 *     positive multiple of 16) of buf, passes times (>= 1); read bytes per
 *     second.  The buffer's size chooses the level: a few MB stay in each
 *     XCD's L2, tens of MB in the Infinity Cache, larger ones come from HBM.
 *   tpmc_ceiling_atomic: per_thread (1..4096) int64 atomic adds per lane into
 *     slots (1..2^26) int64 words of buf (adds 1 to them: zero or reuse it
 *     afterwards as needed); atomics per second.
 *   tpmc_ceiling_lds_atomic: the same into slots (1..1024) int64 words of each
 *     workgroup's LDS; sink >= 16 bytes. */
tpmc_status tpmc_ceiling_valu(tpmc_ctx ctx, uint32_t kind, void* dev_sink, double* lane_ops_per_s);
tpmc_status tpmc_ceiling_read(tpmc_ctx ctx, const void* dev_buf, uint64_t bytes, uint32_t passes,
                              double* bytes_per_s);
tpmc_status tpmc_ceiling_atomic(tpmc_ctx ctx, void* dev_buf, uint32_t slots, uint32_t per_thread,
                                double* atomics_per_s);
tpmc_status tpmc_ceiling_lds_atomic(tpmc_ctx ctx, void* dev_sink, uint32_t slots, uint32_t per_thread,
                                    double* atomics_per_s);

/* ---- Check of the batched path's two-stage seeding ----
 * The persistent kernel (batches and server steps) seeds in two stages: an
 * FP32 estimate of each particle's first ray from its own variates (Sec.
 * III.A.1-3 in FP32: the latitude from a fine table without iteration, the
 * normal speed from a tabulated start and two Halley steps) is tested against
 * the BVH root's boxes grown on every side by 2 % of
 * the CV radius, and only the particles it does not rule out are seeded
 * exactly (FP64) and traced; the others are misses either way, so no result
 * field other than tpmc_result.preculled depends on it.  The margin rests on
 * the estimate's error, which this entry point measures: for particles
 * [0, q->n_particles) of the query it returns the largest distance between
 * the estimated and the exact ray (|o_est - o| + 2 r |w_est/|w_est| - w/|w||)
 * as a fraction of the margin, over the particles the estimate covers (it
 * gives up near the poles mu = +-1, outside its tables' ranges and when the
 * speed's solve has not converged; those particles are always seeded
 * exactly), and their number.  Workspace: the
 * caller's device memory, >= TPMC_PRECULL_CHECK_BYTES, 256-byte aligned.
 * Synchronises the context's stream. */
#define TPMC_PRECULL_CHECK_BYTES 1024
tpmc_status tpmc_precull_check(tpmc_ctx ctx, tpmc_mesh mesh, const tpmc_query* q, void* dev_ws, uint64_t ws_bytes,
                               double* max_err_over_margin, uint64_t* estimated);

/* ---- Phase probe of the persistent kernel (a measuring aid) ----
 * A library compiled with TPMC_PHASE_PROBE=1 (libtpmc_probe.so, built next to
 * libtpmc.so by the package's build script) has every wave of the batched
 * kernel read the shader clock around its phases and count each phase's passes
 * and active lanes; the ordinary library has no such code.  tpmc_phase_probe
 * waits for the context's stream, copies the sums of every batched launch on
 * the context's device since the last reset into out[0 .. TPMC_PROBE_SLOTS)
 * (caller's host memory, n_slots >= TPMC_PROBE_SLOTS) and, when reset is
 * nonzero, clears them.  It returns TPMC_E_INVALID, writing nothing, from a
 * library built without the probe.  Slots (sums over waves; cycles are
 * shader-clock ticks, lanes the active lanes of each pass):
 *   0 waves, 1 cycles from a wave's start to its exit,
 *   2-3 cycles and count of tile claims (with the ends of tiles),
 *   4-6 traversal steps: cycles, steps, lanes,
 *   7-9 leaf phases (the batched triangle tests): cycles, passes, lanes,
 *   10-12 service passes (hit, re-emission, tally): cycles, passes, lanes,
 *   13-16 seeding estimate (first stage): cycles, batches, particles, kept,
 *   17-20 exact seeding with the root test: cycles, batches, particles, kept,
 *   21-23 queue hand-out to idle lanes: cycles, passes, lanes.
 * The probe's own clock reads lengthen a launch by some per cent. */
#define TPMC_PROBE_SLOTS 24
tpmc_status tpmc_phase_probe(tpmc_ctx ctx, uint64_t* out, uint32_t n_slots, int reset);

#ifdef __cplusplus
}
#endif
#endif

// tpmc_capi.hip -- host side of the libtpmc C ABI (include/tpmc.h): argument
// validation, per-query FP64 set-up (a1), workspace layout, kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <mutex>
#include <algorithm>
#include <vector>

#include "../../include/tpmc.h"
#include "tpmc_internal.h"
#include "tpmc_launch.h"

using namespace tpmc;

// default cap of the plain trace grid, workgroups per compute unit
static constexpr uint32_t kPlainGroupsPerCu = 4;

// Workspace of tpmc_batch_run_noalloc: a device array in the library's code
// object, one copy per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): the address each device gives for it at context creation
// (hipGetSymbolAddress) is kept in g_scratch_ptr and used instead.
static constexpr uint64_t kScratchBytes = TPMC_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;  // [device], null until that device's first context

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static tpmc_status fail(tpmc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return fail(TPMC_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

#define HIP_CHECK_LAUNCH(what)                                                                     \
  do {                                                                                             \
    hipError_t e_ = hipGetLastError();                                                             \
    if (e_ != hipSuccess) return fail(TPMC_E_DEVICE, "%s launch: %s", what, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct tpmc_ctx_s {
  int device;
  hipStream_t stream;
  hipStream_t capture_stream;
  int n_cu;
  tpmc_tuning tune;
};

struct tpmc_mesh_s {
  tpmc_ctx ctx;
  int device;  // the context's device, kept so that destruction never reads the context
  uint64_t nv, nt;
  uint32_t depth;
  uint32_t builder;  // tpmc_bvh_builder
  int stack_slots;
  Node* nodes;
  TriRec* tris;
  uint32_t* orig;
  std::vector<float> host_xyz;  // for control-volume checks
  double lo[3], hi[3], c0[3], r;
  uint64_t device_bytes;
};

struct Layout {
  QueryDev* qs;
  ResultDev* res;
  long long* scal;
  long long* tally;
  uint64_t* tiles;       // batch: tiles per query
  unsigned long long* next;  // batch: claim counter per query
  float* planes[6];
  uint64_t bytes;
};

struct tpmc_particles_s {
  tpmc_ctx ctx;
  tpmc_mesh mesh;
  uint32_t nq;
  std::vector<QueryDev> hq;
  Layout lay;
  uint64_t n_total;
};

struct tpmc_tally_s {
  tpmc_particles p;
};

struct tpmc_batch_s {
  tpmc_ctx ctx;
  int device;  // as tpmc_mesh_s::device
  tpmc_mesh mesh;
  uint32_t nq;
  std::vector<QueryDev> hq;
  std::vector<uint64_t> tiles;
  Layout lay;
  uint64_t total_tiles;
  uint64_t tally_words;
  TallyMode mode;
  int grid;
  uint32_t tile;
  uint32_t refill;
  hipGraphExec_t exec;
  bool launched;
};

// ---------------------------------------------------------------------------
// validation and per-query set-up
// ---------------------------------------------------------------------------
static bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

extern "C" tpmc_status tpmc_check_mesh(const float* xyz, uint64_t nv, const uint32_t* tri, uint64_t nt) {
  if (!xyz || !tri) return fail(TPMC_E_INVALID, "mesh arrays must not be NULL");
  if (nt == 0) return fail(TPMC_E_MESH, "mesh has no triangles");
  if (nv == 0) return fail(TPMC_E_MESH, "mesh has no vertices");
  if (nv > 0xFFFFFFFFull) return fail(TPMC_E_MESH, "mesh has too many vertices (%llu)", (unsigned long long)nv);
  if (nt >= (1ull << 30)) return fail(TPMC_E_MESH, "mesh has too many triangles (%llu)", (unsigned long long)nt);
  for (uint64_t i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(xyz[i])) return fail(TPMC_E_MESH, "vertex %llu is not finite", (unsigned long long)(i / 3));
  for (uint64_t i = 0; i < 3 * nt; ++i)
    if (tri[i] >= nv)
      return fail(TPMC_E_MESH, "triangle %llu names vertex %u >= nv = %llu", (unsigned long long)(i / 3), tri[i],
                  (unsigned long long)nv);
  return TPMC_OK;
}

static void bounding_sphere(const float* xyz, uint64_t nv, double lo[3], double hi[3], double c0[3], double* r) {
  for (int k = 0; k < 3; ++k) {
    lo[k] = INFINITY;
    hi[k] = -INFINITY;
  }
  for (uint64_t i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::fmin(lo[k], (double)xyz[3 * i + k]);
      hi[k] = std::fmax(hi[k], (double)xyz[3 * i + k]);
    }
  for (int k = 0; k < 3; ++k) c0[k] = 0.5 * (lo[k] + hi[k]);
  double rr = 0.0;
  for (uint64_t i = 0; i < nv; ++i) {
    const double a = xyz[3 * i] - c0[0], b = xyz[3 * i + 1] - c0[1], c = xyz[3 * i + 2] - c0[2];
    rr = std::fmax(rr, std::sqrt(a * a + b * b + c * c));
  }
  *r = rr * (1.0 + 1e-3);
}

static tpmc_status check_query_fields(const tpmc_query* q) {
  if (!q) return fail(TPMC_E_INVALID, "query is NULL");
  const double n2 = q->q_wxyz[0] * q->q_wxyz[0] + q->q_wxyz[1] * q->q_wxyz[1] + q->q_wxyz[2] * q->q_wxyz[2] +
                    q->q_wxyz[3] * q->q_wxyz[3];
  if (!std::isfinite(n2) || std::fabs(std::sqrt(n2) - 1.0) > 1e-6)
    return fail(TPMC_E_INVALID, "attitude quaternion must have unit norm (|q| = %g)", std::sqrt(n2));
  if (!std::isfinite(q->S) || q->S < 0.0 || q->S > 100.0)
    return fail(TPMC_E_INVALID, "speed ratio S = %g outside [0, 100]", q->S);
  if (!std::isfinite(q->T_inf) || !(q->T_inf > 0.0) || !std::isfinite(q->T_w) || !(q->T_w > 0.0))
    return fail(TPMC_E_INVALID, "temperatures must be finite and > 0 (T_inf = %g, T_w = %g)", q->T_inf, q->T_w);
  if (!std::isfinite(q->alpha) || q->alpha < 0.0 || q->alpha > 1.0)
    return fail(TPMC_E_INVALID, "accommodation alpha = %g outside [0, 1]", q->alpha);
  if (q->n_particles == 0 || q->n_particles > (1ull << 40))
    return fail(TPMC_E_INVALID, "n_particles = %llu outside [1, 2^40]", (unsigned long long)q->n_particles);
  if (q->max_reflections == 0 || q->max_reflections > (uint32_t)kMaxReflections)
    return fail(TPMC_E_INVALID, "max_reflections = %u outside [1, %d]", q->max_reflections, kMaxReflections);
  if (q->flags & ~(TPMC_Q_NO_TRIANGLE_TALLY | TPMC_Q_BOX_CV | TPMC_Q_ENERGY_ACC))
    return fail(TPMC_E_INVALID, "unknown query flags 0x%x", q->flags);
  if ((q->flags & TPMC_Q_ENERGY_ACC) &&
      (!std::isfinite(q->energy_accommodation) || q->energy_accommodation < 0.0 || q->energy_accommodation > 1.0))
    return fail(TPMC_E_INVALID, "energy accommodation %g outside [0, 1]", q->energy_accommodation);
  if (!finite3(q->cv_center) || !std::isfinite(q->cv_radius))
    return fail(TPMC_E_INVALID, "control volume must be finite");
  return TPMC_OK;
}

static tpmc_status check_cv(const tpmc_query* q, const float* xyz, uint64_t nv) {
  if (!(q->cv_radius > 0.0)) return TPMC_OK;
  if (q->flags & TPMC_Q_BOX_CV) {
    double worst = 0.0;  // largest |v_k - c_k| over vertices and axes
    for (uint64_t i = 0; i < nv; ++i)
      for (int k = 0; k < 3; ++k) worst = std::fmax(worst, std::fabs(xyz[3 * i + k] - q->cv_center[k]));
    if (worst > q->cv_radius)
      return fail(TPMC_E_CV, "control box (half-side %g) does not enclose the mesh (a vertex at %g on one axis)",
                  q->cv_radius, worst);
    return TPMC_OK;
  }
  double worst = 0.0;
  for (uint64_t i = 0; i < nv; ++i) {
    const double a = xyz[3 * i] - q->cv_center[0], b = xyz[3 * i + 1] - q->cv_center[1],
                 c = xyz[3 * i + 2] - q->cv_center[2];
    worst = std::fmax(worst, std::sqrt(a * a + b * b + c * c));
  }
  if (worst > q->cv_radius)
    return fail(TPMC_E_CV, "control volume (radius %g) does not enclose the mesh (farthest vertex at %g)",
                q->cv_radius, worst);
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_check_query(const tpmc_query* q, const float* xyz, uint64_t nv) {
  tpmc_status s = check_query_fields(q);
  if (s != TPMC_OK) return s;
  if (!xyz && q->cv_radius > 0.0) return fail(TPMC_E_INVALID, "vertices needed for the control-volume check");
  return xyz ? check_cv(q, xyz, nv) : TPMC_OK;
}

static double pow2_floor(double v) { return std::ldexp(1.0, (int)std::floor(std::log2(v))); }

// a1: FP64 constants of one query (Sec. II.B, III.A.1, III.A.3).
static void setup_query(const tpmc_query* in, const tpmc_mesh m, QueryDev* q) {
  std::memset(q, 0, sizeof *q);
  double w = in->q_wxyz[0], x = in->q_wxyz[1], y = in->q_wxyz[2], z = in->q_wxyz[3];
  const double n = std::sqrt(w * w + x * x + y * y + z * z);
  w /= n; x /= n; y /= n; z /= n;
  // rows of the body->wind rotation: free stream U, seeding tangents e1, e2
  const double U[3] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)};
  const double e1[3] = {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)};
  const double e2[3] = {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  for (int k = 0; k < 3; ++k) {
    q->U[k] = U[k];
    q->e1[k] = e1[k];
    q->e2[k] = e2[k];
    q->Uf[k] = (float)U[k];
  }
  if (in->cv_radius > 0.0) {
    for (int k = 0; k < 3; ++k) q->c0[k] = in->cv_center[k];
    q->r = in->cv_radius;
  } else {
    for (int k = 0; k < 3; ++k) q->c0[k] = m->c0[k];
    q->r = m->r;
  }
  const double S = in->S;
  q->S = S;
  q->s_zero = S < 1e-8 ? 1u : 0u;
  const double sqrtpi = 1.77245385090551602730, pi = 3.14159265358979323846;
  q->erfS = std::erf(S);
  q->erfcS = std::erfc(S);
  q->expmS2 = std::exp(-S * S);
  q->lat_k = q->s_zero ? 0.0 : sqrtpi / (4.0 * S);
  // Z(S) = e^{-S^2} + sqrt(pi) (S + 1/(2S)) erf S; Gamma/(n c_mp) = sqrt(pi) r^2 Z (Sec. III.A.1)
  q->Z = q->s_zero ? 2.0 : q->expmS2 + sqrtpi * (S + 0.5 / S) * q->erfS;
  q->Gamma_hat = q->s_zero ? 2.0 * sqrtpi * q->r * q->r
                           : (sqrtpi * q->expmS2 + (pi / (2.0 * S) + pi * S) * q->erfS) * q->r * q->r;
  if (in->flags & TPMC_Q_BOX_CV) {
    // Box CV: the cube of half-side cv_radius, or the vertex box widened by 1e-3
    // of its half-diagonal; inflow through face f = A_f chi(s_f) / (2 sqrt(pi)).
    q->box = 1u;
    if (in->cv_radius > 0.0) {
      for (int k = 0; k < 3; ++k) q->h[k] = in->cv_radius;
    } else {
      double hd = 0.0;
      for (int k = 0; k < 3; ++k) {
        q->h[k] = 0.5 * (m->hi[k] - m->lo[k]);
        hd += q->h[k] * q->h[k];
      }
      hd = std::sqrt(hd);
      for (int k = 0; k < 3; ++k) q->h[k] += 1e-3 * hd;
    }
    q->r = std::sqrt(q->h[0] * q->h[0] + q->h[1] * q->h[1] + q->h[2] * q->h[2]);  // lever bound
    double cum = 0.0;
    for (int f = 0; f < 6; ++f) {
      const int k = f / 2, j = (k + 1) % 3, l = (k + 2) % 3;
      const double n_k = f % 2 == 0 ? 1.0 : -1.0;
      const double s_f = q->s_zero ? 0.0 : S * U[k] * n_k;
      q->face_s[f] = s_f;
      cum += 4.0 * q->h[j] * q->h[l] * (std::exp(-s_f * s_f) + sqrtpi * s_f * std::erfc(-s_f));
      q->face_cum[f] = cum;
    }
    q->Gamma_hat = cum / (2.0 * sqrtpi);
  }
  for (int k = 0; k < 3; ++k) {
    q->c0f[k] = (float)q->c0[k];
    q->e1f[k] = (float)q->e1[k];
    q->e2f[k] = (float)q->e2[k];
  }
  q->Sf = (float)q->S;
  q->rf = (float)q->r;
  // the fine latitude table (seeding estimate, exact solve start): the four rows around ln S and
  // their cubic Lagrange weights (nodes -1, 0, 1, 2 around the row below ln S)
  q->lat_f0 = -1;
  for (int k = 0; k < 4; ++k) q->lat_fw[k] = 0.0f;
  if (!q->s_zero && S >= kLatFSmin && S <= kLatFSmax) {
    const double pos = (std::log(S) - kLatFL0) / kLatFDL;
    const int i = (int)std::floor(pos);
    const double f = pos - i;
    if (i - 1 >= 0 && i + 2 <= kLatFNS - 1) {
      q->lat_f0 = i - 1;
      q->lat_fw[0] = (float)(-f * (f - 1.0) * (f - 2.0) / 6.0);
      q->lat_fw[1] = (float)((f + 1.0) * (f - 1.0) * (f - 2.0) / 2.0);
      q->lat_fw[2] = (float)(-(f + 1.0) * f * (f - 2.0) / 2.0);
      q->lat_fw[3] = (float)((f + 1.0) * f * (f - 1.0) / 6.0);
    }
  }
  const double tau = std::sqrt(in->T_w / in->T_inf);
  q->tau = (float)tau;
  q->alpha = (float)in->alpha;
  q->N = in->n_particles;
  q->key0 = (uint32_t)in->seed;
  q->key1 = (uint32_t)(in->seed >> 32);
  q->rmax = in->max_reflections;
  q->per_tri = (in->flags & TPMC_Q_NO_TRIANGLE_TALLY) ? 0u : 1u;
  q->nodes = m->nodes;
  q->tris = m->tris;
  q->orig = m->orig;
  q->nt = (uint32_t)m->nt;
  // Fixed point: every sampled speed is bounded (the variates never reach 0 or 1),
  // |w| <= S + 15 for seeded and specular velocities and |w| <= 8 tau after a
  // diffuse re-emission, so one hit moves at most Dmax; scales are the largest
  // powers of two keeping N * rmax hits of Dmax inside 2^62.
  // With energy accommodation a re-emitted speed is at most ~7.1 tau_r; the
  // kernel bounds tau_r by max(tau, 8 (S + 15)) (a limit of these fixed-point
  // tallies, not of the model: each re-emission it limits is counted in the
  // result's tr_capped), so every |w| stays below B = max(8 tau, 57 (S + 15)).
  // Inside a cavity tau_r follows a multiplicative chain with a power-law
  // tail (tau_r^2 grows by a Gamma(2)-distributed factor times
  // (1 - alpha_E) / 2 per re-emission), so the bound sits far above
  // (S + 15)^2 / 2: at alpha_E = 0.2 in a cup that smaller bound is reached
  // by about one particle in 1e5, this one by far fewer than one in 1e10.
  q->eacc = (in->flags & TPMC_Q_ENERGY_ACC) ? 1u : 0u;
  q->alpha_E = q->eacc ? (float)in->energy_accommodation : 1.0f;
  q->tr_cap2 = (float)std::fmax(tau * tau, 64.0 * (S + 15.0) * (S + 15.0));
  const double Dmax = q->eacc ? 2.0 * std::fmax(8.0 * tau, 57.0 * (S + 15.0)) : 2.0 * std::fmax(S + 15.0, 8.0 * tau);
  const double hits_max = (double)in->n_particles * (double)in->max_reflections;
  // One hit's scaled momentum (and moment) also stays below 2^30, so the
  // kernels convert it with a 32-bit conversion.
  const double sF = std::fmin(std::fmin(pow2_floor(std::ldexp(1.0, 62) / (hits_max * Dmax)), std::ldexp(1.0, 50)),
                              pow2_floor(std::ldexp(1.0, 30) / Dmax));
  const double sL = std::fmin(std::fmin(pow2_floor(std::ldexp(1.0, 62) / (hits_max * Dmax * q->r * 1.01)),
                                        std::ldexp(1.0, 50)),
                              pow2_floor(std::ldexp(1.0, 30) / (Dmax * q->r * 1.01)));
  const double pD = (double)in->max_reflections * Dmax;
  const double sD2 = std::fmin(pow2_floor(std::ldexp(1.0, 62) / ((double)in->n_particles * pD * pD)),
                               std::ldexp(1.0, 50));
  q->scaleF = (float)sF;
  q->scaleL = (float)sL;
  q->scaleD = (float)sF;
  q->scaleD2 = (float)sD2;
  q->inv_scaleF = 1.0 / sF;
  q->inv_scaleL = 1.0 / sL;
  q->inv_scaleD = 1.0 / sF;
  q->inv_scaleD2 = 1.0 / sD2;
  // energy per hit |w|^2 - |w'|^2 is at most (Dmax / 2)^2 in magnitude
  const double Emax = 0.25 * Dmax * Dmax;
  const double sE = std::fmin(pow2_floor(std::ldexp(1.0, 62) / (hits_max * Emax)), std::ldexp(1.0, 50));
  const double pE = (double)in->max_reflections * Emax;
  const double sE2 = std::fmin(pow2_floor(std::ldexp(1.0, 62) / ((double)in->n_particles * pE * pE)),
                               std::ldexp(1.0, 50));
  q->scaleE = (float)sE;
  q->scaleE2 = (float)sE2;
  q->inv_scaleE = 1.0 / sE;
  q->inv_scaleE2 = 1.0 / sE2;
}

static tpmc_status make_queries(tpmc_mesh m, const tpmc_query* q, uint32_t nq, std::vector<QueryDev>& out) {
  if (!q || nq == 0) return fail(TPMC_E_INVALID, "need at least one query");
  out.resize(nq);
  for (uint32_t i = 0; i < nq; ++i) {
    tpmc_status s = check_query_fields(&q[i]);
    if (s != TPMC_OK) return fail(s, "query %u: %s", i, g_err.c_str());
    s = check_cv(&q[i], m->host_xyz.data(), m->nv);
    if (s != TPMC_OK) return fail(s, "query %u: %s", i, g_err.c_str());
    setup_query(&q[i], m, &out[i]);
  }
  return TPMC_OK;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
static uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

// Lays out [queries | results | scalar blocks | tallies | tiles | claim counters | 6 planes].
static void layout(std::vector<QueryDev>& hq, uint64_t nt, uint64_t n_planes, bool batch, uint8_t* base, Layout& L) {
  const uint64_t nq = hq.size();
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const uint64_t o_q = take(nq * sizeof(QueryDev));
  const uint64_t o_r = take(nq * sizeof(ResultDev));
  const uint64_t o_s = take(nq * kScalarSlots * sizeof(long long));
  uint64_t words = 0;
  for (uint64_t i = 0; i < nq; ++i) {
    hq[i].scalar_offset = i * kScalarSlots;
    hq[i].tally_offset = words;
    if (hq[i].per_tri) words += nt * 7;
  }
  const uint64_t o_t = take(words * sizeof(long long));
  const uint64_t o_te = take(batch ? nq * sizeof(uint64_t) : 0);
  const uint64_t o_c = take(batch ? nq * sizeof(uint64_t) : 0);
  uint64_t o_p[6];
  for (int k = 0; k < 6; ++k) o_p[k] = take(n_planes * sizeof(float));
  L.bytes = off;
  L.qs = reinterpret_cast<QueryDev*>(base + o_q);
  L.res = reinterpret_cast<ResultDev*>(base + o_r);
  L.scal = reinterpret_cast<long long*>(base + o_s);
  L.tally = reinterpret_cast<long long*>(base + o_t);
  L.tiles = reinterpret_cast<uint64_t*>(base + o_te);
  L.next = reinterpret_cast<unsigned long long*>(base + o_c);
  for (int k = 0; k < 6; ++k) L.planes[k] = reinterpret_cast<float*>(base + o_p[k]);
}

static uint64_t total_particles(const std::vector<QueryDev>& hq) {
  uint64_t n = 0;
  for (const auto& q : hq) n += q.N;
  return n;
}

static TallyMode plain_mode(const QueryDev& q, uint64_t nt) {
  if (!q.per_tri) return kTallyTotals;
  if (nt <= (uint64_t)kLaneTallyMaxTris) return kTallyLane;
  if (nt <= (uint64_t)kLdsTallyMaxTris) return kTallyLds;
  return kTallyGlobal;
}

// ---------------------------------------------------------------------------
// context and mesh
// ---------------------------------------------------------------------------
extern "C" const char* tpmc_last_error(void) { return g_err.c_str(); }
extern "C" int tpmc_abi_version(void) { return TPMC_ABI_VERSION; }

extern "C" tpmc_status tpmc_create(int device, void* hip_stream, tpmc_ctx* out) {
  if (!out) return fail(TPMC_E_INVALID, "out is NULL");
  *out = nullptr;
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(TPMC_E_INVALID, "device %d not present (%d devices)", device, count);
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  {
    // the seeding start table lives in the code object of each device; fill it once
    static std::mutex mu;
    static std::vector<char> ready;
    std::lock_guard<std::mutex> lock(mu);
    if (ready.size() < (size_t)count) ready.resize(count, 0);
    if (!ready[device]) {
      hipError_t e = init_seed_tables(static_cast<hipStream_t>(hip_stream));
      if (e != hipSuccess) return fail(TPMC_E_DEVICE, "seeding tables: %s", hipGetErrorString(e));
      void* sp = nullptr;  // this device's copy of the no-allocation workspace
      e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !sp) return fail(TPMC_E_DEVICE, "static workspace address: %s", hipGetErrorString(e));
      {
        std::lock_guard<std::mutex> lock2(g_scratch_mu);
        if (g_scratch_ptr.size() < (size_t)count) g_scratch_ptr.resize(count, nullptr);
        g_scratch_ptr[device] = sp;
      }
      ready[device] = 1;
    }
  }
  tpmc_ctx c = new (std::nothrow) tpmc_ctx_s;
  if (!c) return fail(TPMC_E_INVALID, "out of host memory");
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->capture_stream = nullptr;
  c->n_cu = prop.multiProcessorCount;
  c->tune.refill_lanes = 32;
  c->tune.tile_particles = 16384;
  c->tune.groups_per_cu = 8;
  c->tune.plain_groups_per_cu = kPlainGroupsPerCu;
  *out = c;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_get_tuning(tpmc_ctx ctx, tpmc_tuning* out) {
  if (!ctx || !out) return fail(TPMC_E_INVALID, "ctx and out must not be NULL");
  *out = ctx->tune;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_set_tuning(tpmc_ctx ctx, const tpmc_tuning* t) {
  if (!ctx || !t) return fail(TPMC_E_INVALID, "ctx and tuning must not be NULL");
  if (t->refill_lanes < 1 || t->refill_lanes > 64)
    return fail(TPMC_E_INVALID, "refill_lanes = %u outside 1..64", t->refill_lanes);
  if (t->tile_particles < 64 || t->tile_particles > (1u << 16) || t->tile_particles % 64 != 0)
    return fail(TPMC_E_INVALID, "tile_particles = %u is not a multiple of 64 in [64, 65536]", t->tile_particles);
  if (t->groups_per_cu < 1 || t->groups_per_cu > 32)
    return fail(TPMC_E_INVALID, "groups_per_cu = %u outside 1..32", t->groups_per_cu);
  if (t->plain_groups_per_cu > 32)
    return fail(TPMC_E_INVALID, "plain_groups_per_cu = %u outside 0..32", t->plain_groups_per_cu);
  ctx->tune = *t;
  if (ctx->tune.plain_groups_per_cu == 0) ctx->tune.plain_groups_per_cu = kPlainGroupsPerCu;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_set_stream(tpmc_ctx ctx, void* hip_stream) {
  if (!ctx) return fail(TPMC_E_INVALID, "ctx is NULL");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return TPMC_OK;
}

extern "C" void tpmc_destroy_ctx(tpmc_ctx ctx) {
  if (!ctx) return;
  if (ctx->capture_stream) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamDestroy(ctx->capture_stream);
    (void)hipGetLastError();
  }
  delete ctx;
}

extern "C" tpmc_status tpmc_build_mesh(tpmc_ctx ctx, const float* xyz, uint64_t nv, const uint32_t* tri, uint64_t nt,
                                       tpmc_mesh* out) {
  return tpmc_build_mesh_ex(ctx, xyz, nv, tri, nt, TPMC_BVH_SAH, out);
}

extern "C" tpmc_status tpmc_build_mesh_ex(tpmc_ctx ctx, const float* xyz, uint64_t nv, const uint32_t* tri,
                                          uint64_t nt, uint32_t builder, tpmc_mesh* out) {
  if (!ctx || !out) return fail(TPMC_E_INVALID, "ctx and out must not be NULL");
  *out = nullptr;
  if (builder != TPMC_BVH_SAH && builder != TPMC_BVH_LBVH)
    return fail(TPMC_E_INVALID, "unknown BVH builder %u", builder);
  tpmc_status s = tpmc_check_mesh(xyz, nv, tri, nt);
  if (s != TPMC_OK) return s;
  HIP_TRY(hipSetDevice(ctx->device));
  tpmc_mesh m = new (std::nothrow) tpmc_mesh_s;
  if (!m) return fail(TPMC_E_INVALID, "out of host memory");
  m->ctx = ctx;
  m->device = ctx->device;
  m->nv = nv;
  m->nt = nt;
  m->host_xyz.assign(xyz, xyz + 3 * nv);
  bounding_sphere(xyz, nv, m->lo, m->hi, m->c0, &m->r);
  m->nodes = nullptr;
  m->tris = nullptr;
  m->orig = nullptr;
  const uint64_t nnodes = nt > 1 ? nt - 1 : 1;
  float* d_xyz = nullptr;
  uint32_t* d_tri = nullptr;
  void* scratch = nullptr;
  hipError_t e = hipMalloc(&d_xyz, 3 * nv * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&d_tri, 3 * nt * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&scratch, builder == TPMC_BVH_SAH ? sah_scratch_bytes(nt) : bvh_scratch_bytes(nt));
  if (e == hipSuccess) e = hipMalloc(&m->nodes, nnodes * sizeof(Node));
  if (e == hipSuccess) e = hipMalloc(&m->tris, nt * sizeof(TriRec));
  if (e == hipSuccess) e = hipMalloc(&m->orig, nt * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemcpyAsync(d_xyz, xyz, 3 * nv * sizeof(float), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_tri, tri, 3 * nt * sizeof(uint32_t), hipMemcpyHostToDevice, ctx->stream);
  uint32_t depth = 0;
  if (e == hipSuccess) {
    const float lo[3] = {(float)m->lo[0], (float)m->lo[1], (float)m->lo[2]};
    const float hi[3] = {(float)m->hi[0], (float)m->hi[1], (float)m->hi[2]};
    e = builder == TPMC_BVH_SAH
            ? build_bvh_sah(d_xyz, d_tri, nt, scratch, m->nodes, m->tris, m->orig, &depth, ctx->stream)
            : build_bvh(d_xyz, d_tri, nt, lo, hi, scratch, m->nodes, m->tris, m->orig, &depth, ctx->stream);
  }
  if (e == hipSuccess) {
    mark_support(d_xyz, nv, m->tris, nt, m->orig, ctx->stream);
    e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = hipGetLastError();
  }
  if (d_xyz) (void)hipFree(d_xyz);
  if (d_tri) (void)hipFree(d_tri);
  if (scratch) (void)hipFree(scratch);
  if (e != hipSuccess) {
    tpmc_destroy_mesh(m);
    return fail(TPMC_E_DEVICE, "BVH build: %s", hipGetErrorString(e));
  }
  m->depth = depth;
  m->builder = builder;
  m->stack_slots = stack_slots_for_depth(depth);
  if (m->stack_slots == 0) {
    tpmc_destroy_mesh(m);
    return fail(TPMC_E_MESH, "BVH depth %u exceeds the supported 64 levels", depth);
  }
  m->device_bytes = nnodes * sizeof(Node) + nt * (sizeof(TriRec) + sizeof(uint32_t));
  *out = m;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_get_mesh_info(tpmc_mesh m, tpmc_mesh_info* out) {
  if (!m || !out) return fail(TPMC_E_INVALID, "mesh and out must not be NULL");
  out->nv = m->nv;
  out->nt = m->nt;
  out->depth = m->depth;
  out->stack_slots = (uint32_t)m->stack_slots;
  for (int k = 0; k < 3; ++k) {
    out->box_lo[k] = m->lo[k];
    out->box_hi[k] = m->hi[k];
    out->sphere_center[k] = m->c0[k];
  }
  out->sphere_radius = m->r;
  out->device_bytes = m->device_bytes;
  out->builder = m->builder;
  out->reserved = 0;
  return TPMC_OK;
}

// Destruction may run after the context's (a garbage collector finalises in
// any order), so it uses the handle's own device id, and it clears the error
// state of the calls it makes so that no later check reports them.
extern "C" void tpmc_destroy_mesh(tpmc_mesh m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  if (m->nodes) (void)hipFree(m->nodes);
  if (m->tris) (void)hipFree(m->tris);
  if (m->orig) (void)hipFree(m->orig);
  (void)hipGetLastError();
  delete m;
}

// ---------------------------------------------------------------------------
// plain path: seed -> trace -> forces
// ---------------------------------------------------------------------------
static tpmc_status check_ws(void* ws, uint64_t ws_bytes, uint64_t need) {
  if (!ws) return fail(TPMC_E_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(TPMC_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(TPMC_E_WORKSPACE, "workspace of %llu bytes is smaller than the %llu needed",
                (unsigned long long)ws_bytes, (unsigned long long)need);
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_workspace_bytes(tpmc_ctx ctx, tpmc_mesh m, const tpmc_query* q, uint32_t nq,
                                            uint64_t* bytes) {
  if (!ctx || !m || !bytes) return fail(TPMC_E_INVALID, "ctx, mesh and bytes must not be NULL");
  std::vector<QueryDev> hq;
  tpmc_status s = make_queries(m, q, nq, hq);
  if (s != TPMC_OK) return s;
  Layout L;
  layout(hq, m->nt, total_particles(hq), false, nullptr, L);
  *bytes = L.bytes;
  return TPMC_OK;
}

static int seed_grid(tpmc_ctx ctx, uint64_t n) {
  const uint64_t g = (n + kBlock - 1) / kBlock;
  const uint64_t cap = (uint64_t)ctx->n_cu * 16;
  return (int)(g < cap ? (g ? g : 1) : cap);
}

extern "C" tpmc_status tpmc_seed(tpmc_ctx ctx, tpmc_mesh m, const tpmc_query* q, uint32_t nq, void* ws,
                                 uint64_t ws_bytes, tpmc_particles* out) {
  if (!ctx || !m || !out) return fail(TPMC_E_INVALID, "ctx, mesh and out must not be NULL");
  *out = nullptr;
  if (m->ctx != ctx) return fail(TPMC_E_BUSY, "mesh belongs to another context");
  tpmc_particles p = new (std::nothrow) tpmc_particles_s;
  if (!p) return fail(TPMC_E_INVALID, "out of host memory");
  tpmc_status s = make_queries(m, q, nq, p->hq);
  if (s != TPMC_OK) {
    delete p;
    return s;
  }
  p->ctx = ctx;
  p->mesh = m;
  p->nq = nq;
  p->n_total = total_particles(p->hq);
  uint64_t off = 0;
  for (auto& hq : p->hq) {
    hq.p_offset = off;
    off += hq.N;
  }
  layout(p->hq, m->nt, p->n_total, false, static_cast<uint8_t*>(ws), p->lay);
  s = check_ws(ws, ws_bytes, p->lay.bytes);
  if (s != TPMC_OK) {
    delete p;
    return s;
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->lay.qs, p->hq.data(), nq * sizeof(QueryDev), hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) {
    delete p;
    return fail(TPMC_E_DEVICE, "query upload: %s", hipGetErrorString(e));
  }
  uint64_t words = 0;
  for (const auto& hq : p->hq) words += hq.per_tri ? m->nt * 7 : 0;
  zero_i64(p->lay.scal, (uint64_t)nq * kScalarSlots, ctx->stream);
  zero_i64(p->lay.tally, words, ctx->stream);
  for (uint32_t i = 0; i < nq; ++i) {
    const QueryDev& hq = p->hq[i];
    float* const x[3] = {p->lay.planes[0] + hq.p_offset, p->lay.planes[1] + hq.p_offset,
                         p->lay.planes[2] + hq.p_offset};
    float* const w[3] = {p->lay.planes[3] + hq.p_offset, p->lay.planes[4] + hq.p_offset,
                         p->lay.planes[5] + hq.p_offset};
    launch_seed(p->lay.qs + i, hq.N, x, w, seed_grid(ctx, hq.N), ctx->stream);
  }
  e = hipGetLastError();
  if (e != hipSuccess) {
    delete p;
    return fail(TPMC_E_DEVICE, "seed launch: %s", hipGetErrorString(e));
  }
  *out = p;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_particles_planes(tpmc_particles p, float* dev_planes[6], uint64_t* n_total) {
  if (!p || !dev_planes) return fail(TPMC_E_INVALID, "particles and planes must not be NULL");
  for (int k = 0; k < 6; ++k) dev_planes[k] = p->lay.planes[k];
  if (n_total) *n_total = p->n_total;
  return TPMC_OK;
}

// Plain trace grid: at least four particles per lane (so that lanes whose
// particle retires have another to take), at most plain_groups_per_cu per CU.
// Every workgroup of a plain launch flushes its tallies and scalars with
// device atomics once, onto the same few addresses for a small mesh, so the
// cap is kept lower than the persistent launches' (whose workgroups flush once
// per query they took part in).
static int trace_grid(tpmc_ctx ctx, uint64_t n) {
  const uint64_t g = (n + 4 * kBlock - 1) / (4 * kBlock);
  const uint64_t cap = (uint64_t)ctx->n_cu * ctx->tune.plain_groups_per_cu;
  return (int)(g < cap ? (g ? g : 1) : cap);
}

extern "C" tpmc_status tpmc_trace_ex(tpmc_ctx ctx, tpmc_mesh m, tpmc_particles p, int32_t* dev_first_tri,
                                     uint64_t* dev_counters, tpmc_tally* out) {
  if (!ctx || !m || !p || !out) return fail(TPMC_E_INVALID, "ctx, mesh, particles and out must not be NULL");
  *out = nullptr;
  if (p->mesh != m || p->ctx != ctx) return fail(TPMC_E_BUSY, "particles were seeded for another mesh or context");
  HIP_TRY(hipSetDevice(ctx->device));
  for (uint32_t i = 0; i < p->nq; ++i) {
    const QueryDev& hq = p->hq[i];
    TraceArgs a;
    a.nodes = m->nodes;
    a.tris = m->tris;
    a.orig = m->orig;
    a.q = p->lay.qs + i;
    for (int k = 0; k < 3; ++k) {
      a.x[k] = p->lay.planes[k] + hq.p_offset;
      a.w[k] = p->lay.planes[3 + k] + hq.p_offset;
    }
    a.n = hq.N;
    a.tally = hq.per_tri ? p->lay.tally + hq.tally_offset : nullptr;
    a.scal = p->lay.scal + hq.scalar_offset;
    a.first_tri = dev_first_tri ? dev_first_tri + hq.p_offset : nullptr;
    a.counters = reinterpret_cast<unsigned long long*>(dev_counters);
    a.nt = (uint32_t)m->nt;
    a.refill = ctx->tune.refill_lanes;
    launch_trace(a, m->stack_slots, plain_mode(hq, m->nt), trace_grid(ctx, hq.N), ctx->stream);
    HIP_CHECK_LAUNCH("trace");
  }
  tpmc_tally t = new (std::nothrow) tpmc_tally_s;
  if (!t) return fail(TPMC_E_INVALID, "out of host memory");
  t->p = p;
  *out = t;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_trace(tpmc_ctx ctx, tpmc_mesh m, tpmc_particles p, tpmc_tally* out) {
  return tpmc_trace_ex(ctx, m, p, nullptr, nullptr, out);
}

static void copy_result(const ResultDev& r, tpmc_result* o) {
  for (int k = 0; k < 3; ++k) {
    o->F_over_q[k] = r.F_over_q[k];
    o->M_over_q[k] = r.M_over_q[k];
    o->Fhat[k] = r.Fhat[k];
  }
  o->CD = r.CD;
  o->CD_sigma = r.CD_sigma;
  o->Gamma_hat = r.Gamma_hat;
  o->rays = r.rays;
  o->hits = r.hits;
  o->segments = r.segments;
  o->missed = r.missed;
  o->escaped = r.escaped;
  o->capped = r.capped;
  o->Qhat = r.Qhat;
  o->CH = r.CH;
  o->CH_sigma = r.CH_sigma;
  for (int k = 0; k < 3; ++k) o->Mhat[k] = r.Mhat[k];
  o->tr_capped = r.tr_capped;
  o->guard_trips = r.guard_trips;
  o->preculled = r.preculled;
}

// Clears the per-query totals the reduction writes (slots kFx..kCount).
static void clear_totals(long long* scal, uint32_t nq, const std::vector<QueryDev>& hq, hipStream_t st) {
  for (uint32_t i = 0; i < nq; ++i)
    if (hq[i].per_tri) zero_i64(scal + hq[i].scalar_offset + kFx, 7, st);
}

static tpmc_status finalize_results(tpmc_ctx ctx, const Layout& L, uint32_t nq, const double ref_point[3],
                                    double A_ref, tpmc_result* out) {
  const double xr = ref_point ? ref_point[0] : 0.0, yr = ref_point ? ref_point[1] : 0.0,
               zr = ref_point ? ref_point[2] : 0.0;
  launch_finalize(L.qs, nullptr, L.scal, nq, xr, yr, zr, A_ref, L.res, ctx->stream);
  HIP_CHECK_LAUNCH("finalize");
  std::vector<ResultDev> hr(nq);
  HIP_TRY(hipMemcpyAsync(hr.data(), L.res, nq * sizeof(ResultDev), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (uint32_t i = 0; i < nq; ++i) copy_result(hr[i], out + i);
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_forces(tpmc_ctx ctx, tpmc_tally t, const double ref_point[3], double A_ref,
                                   tpmc_result* out) {
  if (!ctx || !t || !out) return fail(TPMC_E_INVALID, "ctx, tally and out must not be NULL");
  if (!(A_ref > 0.0) || !std::isfinite(A_ref)) return fail(TPMC_E_INVALID, "A_ref = %g must be > 0", A_ref);
  if (ref_point && !finite3(ref_point)) return fail(TPMC_E_INVALID, "reference point must be finite");
  tpmc_particles p = t->p;
  if (p->ctx != ctx) return fail(TPMC_E_BUSY, "tally belongs to another context");
  HIP_TRY(hipSetDevice(ctx->device));
  clear_totals(p->lay.scal, p->nq, p->hq, ctx->stream);
  for (uint32_t i = 0; i < p->nq; ++i)
    if (p->hq[i].per_tri)
      launch_reduce(p->lay.tally + p->hq[i].tally_offset, (uint32_t)p->mesh->nt,
                    p->lay.scal + p->hq[i].scalar_offset, ctx->stream);
  HIP_CHECK_LAUNCH("reduce");
  return finalize_results(ctx, p->lay, p->nq, ref_point, A_ref, out);
}

extern "C" tpmc_status tpmc_tally_copy(tpmc_ctx ctx, tpmc_tally t, uint32_t query, double* host_per_tri) {
  if (!ctx || !t || !host_per_tri) return fail(TPMC_E_INVALID, "ctx, tally and output must not be NULL");
  tpmc_particles p = t->p;
  if (query >= p->nq) return fail(TPMC_E_INVALID, "query %u >= nq = %u", query, p->nq);
  const QueryDev& q = p->hq[query];
  if (!q.per_tri) return fail(TPMC_E_INVALID, "query %u keeps no per-triangle tallies", query);
  const uint64_t nt = p->mesh->nt;
  std::vector<long long> raw(nt * 7);
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipMemcpyAsync(raw.data(), p->lay.tally + q.tally_offset, nt * 7 * sizeof(long long),
                         hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (uint64_t k = 0; k < nt; ++k) {
    double F[3], L[3];
    for (int c = 0; c < 3; ++c) {
      F[c] = (double)raw[7 * k + c] * q.inv_scaleF;
      L[c] = (double)raw[7 * k + 3 + c] * q.inv_scaleL;
    }
    // moment about the body origin: (p - c0) x dw + c0 x dw
    double* o = host_per_tri + 7 * k;
    o[0] = F[0];
    o[1] = F[1];
    o[2] = F[2];
    o[3] = L[0] + (q.c0[1] * F[2] - q.c0[2] * F[1]);
    o[4] = L[1] + (q.c0[2] * F[0] - q.c0[0] * F[2]);
    o[5] = L[2] + (q.c0[0] * F[1] - q.c0[1] * F[0]);
    o[6] = (double)raw[7 * k + 6];
  }
  return TPMC_OK;
}

extern "C" void tpmc_destroy_particles(tpmc_particles p) { delete p; }
extern "C" void tpmc_destroy_tally(tpmc_tally t) { delete t; }

// ---------------------------------------------------------------------------
// batched path
// ---------------------------------------------------------------------------

static tpmc_status batch_prepare(tpmc_mesh m, const tpmc_query* q, uint32_t nq, uint32_t tile,
                                 std::vector<QueryDev>& hq, std::vector<uint64_t>& tiles, Layout& L, uint8_t* base) {
  tpmc_status s = make_queries(m, q, nq, hq);
  if (s != TPMC_OK) return s;
  tiles.resize(nq);
  for (uint32_t i = 0; i < nq; ++i) tiles[i] = (hq[i].N + tile - 1) / tile;
  layout(hq, m->nt, 0, true, base, L);
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_batch_workspace_bytes(tpmc_ctx ctx, tpmc_mesh m, const tpmc_query* q, uint32_t nq,
                                                  uint64_t* bytes) {
  if (!ctx || !m || !bytes) return fail(TPMC_E_INVALID, "ctx, mesh and bytes must not be NULL");
  std::vector<QueryDev> hq;
  std::vector<uint64_t> te;
  Layout L;
  tpmc_status s = batch_prepare(m, q, nq, ctx->tune.tile_particles, hq, te, L, nullptr);
  if (s != TPMC_OK) return s;
  *bytes = L.bytes;
  return TPMC_OK;
}

// Fills b for the queries q on mesh m with its workspace at ws (ws_bytes) and
// uploads the query table and tile counts (synchronises).  Allocates nothing.
static tpmc_status batch_init(tpmc_ctx ctx, tpmc_mesh m, const tpmc_query* q, uint32_t nq, void* ws,
                              uint64_t ws_bytes, tpmc_batch_s* b) {
  tpmc_status s = batch_prepare(m, q, nq, ctx->tune.tile_particles, b->hq, b->tiles, b->lay,
                                static_cast<uint8_t*>(ws));
  if (s == TPMC_OK) s = check_ws(ws, ws_bytes, b->lay.bytes);
  if (s != TPMC_OK) return s;
  b->ctx = ctx;
  b->device = ctx->device;
  b->mesh = m;
  b->nq = nq;
  b->total_tiles = 0;
  for (uint64_t t : b->tiles) b->total_tiles += t;
  b->tally_words = 0;
  bool any_tri = false, all_tri = true;
  for (const auto& hq : b->hq) {
    b->tally_words += hq.per_tri ? m->nt * 7 : 0;
    any_tri = any_tri || hq.per_tri;
    all_tri = all_tri && hq.per_tri;
  }
  if (any_tri && !all_tri)
    return fail(TPMC_E_INVALID, "a batch must use one tally kind (TPMC_Q_NO_TRIANGLE_TALLY on all or none)");
  b->mode = !any_tri ? kTallyTotals
                     : (m->nt <= (uint64_t)kLaneTallyMaxTris ? kTallyLane
                                                            : (m->nt <= (uint64_t)kLdsTallyMaxTris ? kTallyLds : kTallyGlobal));
  b->grid = ctx->n_cu * (int)ctx->tune.groups_per_cu;
  b->tile = ctx->tune.tile_particles;
  b->refill = ctx->tune.refill_lanes;
  b->exec = nullptr;
  b->launched = false;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->lay.qs, b->hq.data(), nq * sizeof(QueryDev), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->lay.tiles, b->tiles.data(), nq * sizeof(uint64_t), hipMemcpyHostToDevice,
                       ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(TPMC_E_DEVICE, "batch upload: %s", hipGetErrorString(e));
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_batch_create(tpmc_ctx ctx, tpmc_mesh m, const tpmc_query* q, uint32_t nq, void* ws,
                                         uint64_t ws_bytes, tpmc_batch* out) {
  if (!ctx || !m || !out) return fail(TPMC_E_INVALID, "ctx, mesh and out must not be NULL");
  *out = nullptr;
  if (m->ctx != ctx) return fail(TPMC_E_BUSY, "mesh belongs to another context");
  tpmc_batch b = new (std::nothrow) tpmc_batch_s;
  if (!b) return fail(TPMC_E_INVALID, "out of host memory");
  const tpmc_status s = batch_init(ctx, m, q, nq, ws, ws_bytes, b);
  if (s != TPMC_OK) {
    delete b;
    return s;
  }
  *out = b;
  return TPMC_OK;
}

static void batch_enqueue(tpmc_batch b, hipStream_t st) {
  tpmc_mesh m = b->mesh;
  zero_i64(reinterpret_cast<long long*>(b->lay.next), b->nq, st);
  zero_i64(b->lay.scal, (uint64_t)b->nq * kScalarSlots, st);
  zero_i64(b->lay.tally, b->tally_words, st);
  BatchArgs a{};
  a.qs = b->lay.qs;
  a.entry_query = nullptr;
  a.entry_tile0 = nullptr;
  a.entry_tiles = b->lay.tiles;
  a.entry_next = b->lay.next;
  a.tally_base = b->lay.tally;
  a.scal_base = b->lay.scal;
  a.n_entries = b->nq;
  a.refill = b->refill;
  a.tile = b->tile;
  a.lds_tris = b->mode == kTallyLds ? (uint32_t)m->nt : 0u;
  a.wave_totals = b->mode == kTallyTotals ? 1u : 0u;
  launch_batch(a, m->stack_slots, b->mode, b->grid, st);
  if (b->mode != kTallyTotals) launch_reduce_batch(b->lay.qs, b->nq, b->lay.tally, b->lay.scal, (uint32_t)m->nt, st);
}

extern "C" tpmc_status tpmc_batch_launch(tpmc_ctx ctx, tpmc_batch b, int use_graph) {
  if (!ctx || !b) return fail(TPMC_E_INVALID, "ctx and batch must not be NULL");
  if (b->ctx != ctx) return fail(TPMC_E_BUSY, "batch belongs to another context");
  HIP_TRY(hipSetDevice(ctx->device));
  if (!use_graph) {
    batch_enqueue(b, ctx->stream);
    HIP_CHECK_LAUNCH("batch");
    b->launched = true;
    return TPMC_OK;
  }
  if (!b->exec) {
    if (!ctx->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
    batch_enqueue(b, ctx->capture_stream);
    hipError_t e = hipStreamEndCapture(ctx->capture_stream, &graph);
    if (e != hipSuccess) return fail(TPMC_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return fail(TPMC_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
    }
  }
  HIP_TRY(hipGraphLaunch(b->exec, ctx->stream));
  b->launched = true;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_batch_results(tpmc_ctx ctx, tpmc_batch b, const double ref_point[3], double A_ref,
                                          tpmc_result* out) {
  if (!ctx || !b || !out) return fail(TPMC_E_INVALID, "ctx, batch and out must not be NULL");
  if (!(A_ref > 0.0) || !std::isfinite(A_ref)) return fail(TPMC_E_INVALID, "A_ref = %g must be > 0", A_ref);
  if (ref_point && !finite3(ref_point)) return fail(TPMC_E_INVALID, "reference point must be finite");
  if (!b->launched) return fail(TPMC_E_BUSY, "batch has not been launched");
  HIP_TRY(hipSetDevice(ctx->device));
  return finalize_results(ctx, b->lay, b->nq, ref_point, A_ref, out);
}

extern "C" void tpmc_destroy_batch(tpmc_batch b) {
  if (!b) return;
  if (b->exec) {
    (void)hipSetDevice(b->device);
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGetLastError();
  }
  delete b;
}

// The batched path (tpmc_batch_create + tpmc_batch_launch + tpmc_batch_results)
// in one call, with its workspace in the library's static device array: no
// device memory is allocated or freed.  The same kernels, so the same results.
extern "C" tpmc_status tpmc_batch_run_noalloc(tpmc_ctx ctx, tpmc_mesh m, const tpmc_query* q, uint32_t nq,
                                              const double ref_point[3], double A_ref, tpmc_result* out) {
  if (!ctx || !m || !out) return fail(TPMC_E_INVALID, "ctx, mesh and out must not be NULL");
  if (m->ctx != ctx) return fail(TPMC_E_BUSY, "mesh belongs to another context");
  if (!(A_ref > 0.0) || !std::isfinite(A_ref)) return fail(TPMC_E_INVALID, "A_ref = %g must be > 0", A_ref);
  if (ref_point && !finite3(ref_point)) return fail(TPMC_E_INVALID, "reference point must be finite");
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)ctx->device < g_scratch_ptr.size()) ws = g_scratch_ptr[ctx->device];
  }
  if (!ws) return fail(TPMC_E_DEVICE, "no static workspace address for device %d", ctx->device);
  tpmc_batch_s b;
  std::vector<QueryDev> hq;
  std::vector<uint64_t> te;
  Layout L;
  tpmc_status s = batch_prepare(m, q, nq, ctx->tune.tile_particles, hq, te, L, nullptr);
  if (s != TPMC_OK) return s;
  if (L.bytes > kScratchBytes)
    return fail(TPMC_E_WORKSPACE, "these queries need %llu bytes of workspace; the static workspace holds %llu",
                (unsigned long long)L.bytes, (unsigned long long)kScratchBytes);
  s = batch_init(ctx, m, q, nq, ws, kScratchBytes, &b);
  if (s != TPMC_OK) return s;
  batch_enqueue(&b, ctx->stream);  // zeroes the claim counters, scalars and tallies it uses
  HIP_CHECK_LAUNCH("batch");
  return finalize_results(ctx, b.lay, nq, ref_point, A_ref, out);
}

// ---------------------------------------------------------------------------
// serving: a slot table plus one persistent launch per continuous-batching step
// ---------------------------------------------------------------------------
// Every host-to-device upload of the server goes through a ring of pinned
// host chunks, each guarded by an event recorded after its copy, so that no
// call waits for the kernels already on the stream (a copy from pageable
// memory may), and a chunk is rewritten only once its copy has run.
constexpr int kUploadRing = 8;

struct tpmc_server_s {
  tpmc_ctx ctx;
  int device;  // as tpmc_mesh_s::device
  uint32_t max_slots;
  uint64_t tally_words;
  uint32_t tile;         // particles per tile, fixed at creation
  QueryDev* qs;          // [max_slots]
  ResultDev* res;        // [2][max_slots]: the two collections that may be in flight
  long long* scal;       // [max_slots][kScalarSlots]
  long long* tally;      // pool of tally_words
  uint8_t* entries;      // step entries: tile0 [n] u64, tiles [n] u64, slot [n] u32 (packed for n)
  uint8_t* admits;       // admission staging: [max_slots] AdmitRec
  uint32_t* r_idx;       // [2][max_slots] slots whose results are collected
  unsigned long long* e_next;
  std::vector<QueryDev> hq;
  std::vector<tpmc_mesh> mesh_of;
  std::vector<uint8_t> used;
  // pinned upload ring
  uint8_t* ring_host = nullptr;
  uint64_t chunk = 0;
  hipEvent_t ring_ev[kUploadRing] = {};
  bool ring_used[kUploadRing] = {};
  uint32_t ring_next = 0;
  // collections: pinned result buffers and events, two in flight at most
  ResultDev* res_host = nullptr;  // [2][max_slots]
  hipEvent_t coll_ev[2] = {};
  uint32_t coll_n[2] = {0, 0};
  uint32_t coll_seq = 0;          // collections issued
  bool coll_pending[2] = {false, false};
};

static void server_layout(uint32_t max_slots, uint64_t tally_words, uint8_t* base, tpmc_server_s* s,
                          uint64_t* bytes) {
  uint64_t off = 0;
  auto take = [&](uint64_t b) {
    const uint64_t o = off;
    off = align256(off + b);
    return o;
  };
  const uint64_t oq = take(max_slots * sizeof(QueryDev)), orr = take(2ull * max_slots * sizeof(ResultDev)),
                 os = take((uint64_t)max_slots * kScalarSlots * 8), ot = take(tally_words * 8),
                 oe = take(max_slots * 20ull), oa = take(max_slots * sizeof(AdmitRec)),
                 ori = take(2ull * max_slots * 4), oc = take(max_slots * 8ull);
  *bytes = off;
  if (!s) return;
  s->qs = reinterpret_cast<QueryDev*>(base + oq);
  s->res = reinterpret_cast<ResultDev*>(base + orr);
  s->scal = reinterpret_cast<long long*>(base + os);
  s->tally = reinterpret_cast<long long*>(base + ot);
  s->entries = base + oe;
  s->admits = base + oa;
  s->r_idx = reinterpret_cast<uint32_t*>(base + ori);
  s->e_next = reinterpret_cast<unsigned long long*>(base + oc);
}

static void server_free_host(tpmc_server s) {
  for (int i = 0; i < kUploadRing; ++i)
    if (s->ring_ev[i]) (void)hipEventDestroy(s->ring_ev[i]);
  for (int i = 0; i < 2; ++i)
    if (s->coll_ev[i]) (void)hipEventDestroy(s->coll_ev[i]);
  if (s->ring_host) (void)hipHostFree(s->ring_host);
  if (s->res_host) (void)hipHostFree(s->res_host);
}

// Copy bytes from host src to device dst on the server's stream through the next ring chunk.
static tpmc_status server_upload(tpmc_server s, void* dst, const void* src, uint64_t bytes) {
  if (bytes > s->chunk) return fail(TPMC_E_INVALID, "upload of %llu bytes exceeds the %llu-byte chunk",
                                    (unsigned long long)bytes, (unsigned long long)s->chunk);
  const uint32_t k = s->ring_next;
  s->ring_next = (k + 1) % kUploadRing;
  if (s->ring_used[k]) HIP_TRY(hipEventSynchronize(s->ring_ev[k]));
  uint8_t* h = s->ring_host + (uint64_t)k * s->chunk;
  std::memcpy(h, src, bytes);
  hipStream_t st = s->ctx->stream;
  HIP_TRY(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(s->ring_ev[k], st));
  s->ring_used[k] = true;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_server_workspace_bytes(uint32_t max_slots, uint64_t tally_words, uint64_t* bytes) {
  if (!bytes || max_slots == 0) return fail(TPMC_E_INVALID, "need max_slots >= 1 and an output");
  server_layout(max_slots, tally_words, nullptr, nullptr, bytes);
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_server_create(tpmc_ctx ctx, uint32_t max_slots, uint64_t tally_words, void* ws,
                                          uint64_t ws_bytes, tpmc_server* out) {
  if (!ctx || !out || max_slots == 0) return fail(TPMC_E_INVALID, "ctx, out and max_slots >= 1 required");
  *out = nullptr;
  uint64_t need = 0;
  server_layout(max_slots, tally_words, nullptr, nullptr, &need);
  tpmc_status st = check_ws(ws, ws_bytes, need);
  if (st != TPMC_OK) return st;
  tpmc_server s = new (std::nothrow) tpmc_server_s;
  if (!s) return fail(TPMC_E_INVALID, "out of host memory");
  s->ctx = ctx;
  s->device = ctx->device;
  s->max_slots = max_slots;
  s->tally_words = tally_words;
  s->tile = ctx->tune.tile_particles;
  server_layout(max_slots, tally_words, static_cast<uint8_t*>(ws), s, &need);
  s->hq.assign(max_slots, QueryDev{});
  s->mesh_of.assign(max_slots, nullptr);
  s->used.assign(max_slots, 0);
  s->chunk = align256(std::max<uint64_t>(max_slots * sizeof(AdmitRec), max_slots * 20ull));
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->ring_host), s->chunk * kUploadRing);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->res_host), 2ull * max_slots * sizeof(ResultDev));
  for (int i = 0; e == hipSuccess && i < kUploadRing; ++i) e = hipEventCreateWithFlags(&s->ring_ev[i], hipEventDisableTiming);
  for (int i = 0; e == hipSuccess && i < 2; ++i) e = hipEventCreateWithFlags(&s->coll_ev[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    server_free_host(s);
    delete s;
    return fail(TPMC_E_DEVICE, "server host buffers: %s", hipGetErrorString(e));
  }
  *out = s;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_server_admit_many(tpmc_server s, uint32_t n, const uint32_t* slots, const tpmc_mesh* meshes,
                                              const tpmc_query* q, const uint64_t* tally_offset, uint64_t* n_tiles) {
  if (!s || (n && (!slots || !meshes || !q || !tally_offset)))
    return fail(TPMC_E_INVALID, "server, slots, meshes, queries and offsets must not be NULL");
  if (n == 0) return TPMC_OK;
  if (n > s->max_slots) return fail(TPMC_E_INVALID, "%u admissions > max_slots %u", n, s->max_slots);
  // validate everything before changing any state
  std::vector<AdmitRec> rec(n);
  std::vector<uint8_t> seen(s->max_slots, 0);
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t slot = slots[i];
    const tpmc_mesh m = meshes[i];
    if (!m) return fail(TPMC_E_INVALID, "admission %u: mesh is NULL", i);
    if (slot >= s->max_slots) return fail(TPMC_E_INVALID, "admission %u: slot %u >= max_slots %u", i, slot, s->max_slots);
    if (seen[slot]) return fail(TPMC_E_INVALID, "admission %u: slot %u listed twice", i, slot);
    seen[slot] = 1;
    if (m->ctx != s->ctx) return fail(TPMC_E_BUSY, "admission %u: mesh belongs to another context", i);
    std::vector<QueryDev> one;
    tpmc_status st = make_queries(m, q + i, 1, one);
    if (st != TPMC_OK) return fail(st, "admission %u: %s", i, g_err.c_str());
    QueryDev& d = one[0];
    d.scalar_offset = (uint64_t)slot * kScalarSlots;
    d.tally_offset = tally_offset[i];
    if (d.per_tri && (tally_offset[i] > s->tally_words || m->nt * 7 > s->tally_words - tally_offset[i]))
      return fail(TPMC_E_WORKSPACE, "admission %u: per-triangle tallies of %llu words at offset %llu exceed the pool "
                  "of %llu", i, (unsigned long long)(m->nt * 7), (unsigned long long)tally_offset[i],
                  (unsigned long long)s->tally_words);
    rec[i].q = d;
    rec[i].slot = slot;
    rec[i].pad = 0;
    rec[i].tally_off = tally_offset[i];
    rec[i].tally_words = d.per_tri ? m->nt * 7 : 0;
  }
  HIP_TRY(hipSetDevice(s->ctx->device));
  uint64_t max_words = 0;
  for (uint32_t i = 0; i < n; ++i) {
    s->hq[slots[i]] = rec[i].q;
    s->mesh_of[slots[i]] = meshes[i];
    s->used[slots[i]] = 1;
    if (rec[i].tally_words > max_words) max_words = rec[i].tally_words;
    if (n_tiles) n_tiles[i] = (rec[i].q.N + s->tile - 1) / s->tile;
  }
  tpmc_status st = server_upload(s, s->admits, rec.data(), n * sizeof(AdmitRec));
  if (st != TPMC_OK) return st;
  launch_admit(reinterpret_cast<const AdmitRec*>(s->admits), n, max_words, s->qs, s->scal, s->tally, s->ctx->stream);
  HIP_CHECK_LAUNCH("admit");
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_server_admit(tpmc_server s, uint32_t slot, tpmc_mesh m, const tpmc_query* q,
                                         uint64_t tally_offset, uint64_t* n_tiles) {
  if (!s || !m || !q) return fail(TPMC_E_INVALID, "server, mesh and query must not be NULL");
  return tpmc_server_admit_many(s, 1, &slot, &m, q, &tally_offset, n_tiles);
}

extern "C" tpmc_status tpmc_server_step(tpmc_server s, const uint32_t* slots, const uint64_t* tile0,
                                        const uint64_t* count, uint32_t n) {
  if (!s || (n && (!slots || !tile0 || !count))) return fail(TPMC_E_INVALID, "server and step arrays required");
  if (n == 0) return TPMC_OK;
  if (n > s->max_slots) return fail(TPMC_E_INVALID, "%u entries > max_slots %u", n, s->max_slots);
  uint64_t acc = 0;
  int stack = 4;
  uint32_t lds_tris = 0;  // largest per-triangle tally kept in LDS by the auto mode
  bool any_totals = false, any_tri = false;
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t sl = slots[i];
    if (sl >= s->max_slots || !s->used[sl]) return fail(TPMC_E_INVALID, "entry %u names an empty slot %u", i, sl);
    for (uint32_t j = 0; j < i; ++j)
      if (slots[j] == sl) return fail(TPMC_E_INVALID, "entry %u repeats slot %u", i, sl);
    const uint64_t tiles = (s->hq[sl].N + s->tile - 1) / s->tile;
    if (tile0[i] > tiles || count[i] > tiles - tile0[i])
      return fail(TPMC_E_INVALID, "entry %u: tiles [%llu, +%llu) beyond the slot's %llu", i,
                  (unsigned long long)tile0[i], (unsigned long long)count[i], (unsigned long long)tiles);
    acc += count[i];
    if (s->mesh_of[sl]->stack_slots > stack) stack = s->mesh_of[sl]->stack_slots;
    const QueryDev& hq = s->hq[sl];
    if (hq.per_tri && hq.nt <= (uint32_t)kLdsTallyMaxTris && hq.nt > lds_tris) lds_tris = hq.nt;
    if (!hq.per_tri) any_totals = true;
    else any_tri = true;
  }
  if (acc == 0) return TPMC_OK;
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t st = s->ctx->stream;
  // one packed upload: tile0 [n] u64, tiles [n] u64, slot [n] u32, the entries
  // grouped by mesh (largest first; the order changes no result), and where
  // each XCD's workgroups start: XCD x at the entry holding tile x * acc / 8
  std::vector<uint32_t> ord(n);
  for (uint32_t i = 0; i < n; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) {
    return s->mesh_of[slots[x]]->nt > s->mesh_of[slots[y]]->nt;
  });
  std::vector<uint8_t> pk(20ull * n);
  uint32_t xs[9];
  {
    uint64_t c = 0;
    uint32_t x = 0;
    for (uint32_t i = 0; i < n; ++i) {
      std::memcpy(pk.data() + 8ull * i, tile0 + ord[i], 8);
      std::memcpy(pk.data() + 8ull * n + 8ull * i, count + ord[i], 8);
      std::memcpy(pk.data() + 16ull * n + 4ull * i, slots + ord[i], 4);
      while (x < 8 && c >= x * acc / 8) xs[x++] = i;
      c += count[ord[i]];
    }
    while (x < 9) xs[x++] = n;
    for (int k = 0; k < 8; ++k)
      if (xs[k] >= n) xs[k] = n - 1;
    for (int k = 1; k < 8; ++k)
      if (xs[k] < xs[k - 1]) xs[k] = xs[k - 1];
  }
  tpmc_status ust = server_upload(s, s->entries, pk.data(), pk.size());
  if (ust != TPMC_OK) return ust;
  zero_i64(reinterpret_cast<long long*>(s->e_next), n, st);
  BatchArgs a{};
  a.qs = s->qs;
  a.entry_tile0 = reinterpret_cast<const uint64_t*>(s->entries);
  a.entry_tiles = reinterpret_cast<const uint64_t*>(s->entries + 8ull * n);
  a.entry_query = reinterpret_cast<const uint32_t*>(s->entries + 16ull * n);
  a.entry_next = s->e_next;
  a.tally_base = s->tally;
  a.scal_base = s->scal;
  a.n_entries = n;
  a.refill = s->ctx->tune.refill_lanes;
  a.tile = s->tile;
  // The single-kind instances use fewer registers than the mixed one (four
  // waves per SIMD instead of three); every kind gives the same exact sums.
  const TallyMode mode = !any_tri ? kTallyTotals : (!any_totals && lds_tris == 0 ? kTallyGlobal : kTallyAuto);
  a.lds_tris = mode == kTallyAuto ? lds_tris : 0u;
  a.wave_totals = any_totals ? 1u : 0u;
  for (int k = 0; k < 9; ++k) a.xcd_start[k] = xs[k];
  launch_batch(a, stack, mode, s->ctx->n_cu * (int)s->ctx->tune.groups_per_cu, st);
  HIP_CHECK_LAUNCH("server step");
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_server_collect(tpmc_server s, const uint32_t* slots, uint32_t n, const double ref_point[3],
                                           double A_ref, uint32_t* ticket) {
  if (!s || !slots || !ticket || n == 0) return fail(TPMC_E_INVALID, "server, slots, ticket and n >= 1 required");
  if (n > s->max_slots) return fail(TPMC_E_INVALID, "%u slots > max_slots %u", n, s->max_slots);
  if (!(A_ref > 0.0) || !std::isfinite(A_ref)) return fail(TPMC_E_INVALID, "A_ref = %g must be > 0", A_ref);
  if (ref_point && !finite3(ref_point)) return fail(TPMC_E_INVALID, "reference point must be finite");
  const uint32_t b = s->coll_seq % 2;
  if (s->coll_pending[b])
    return fail(TPMC_E_BUSY, "two collections are already in flight; read collection %u first", s->coll_seq - 2);
  uint32_t max_nt = 1;
  for (uint32_t i = 0; i < n; ++i) {
    if (slots[i] >= s->max_slots || !s->used[slots[i]]) return fail(TPMC_E_INVALID, "slot %u is empty", slots[i]);
    if (s->hq[slots[i]].nt > max_nt) max_nt = s->hq[slots[i]].nt;
  }
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t st = s->ctx->stream;
  uint32_t* idx = s->r_idx + (uint64_t)b * s->max_slots;
  ResultDev* res = s->res + (uint64_t)b * s->max_slots;
  tpmc_status ust = server_upload(s, idx, slots, 4ull * n);
  if (ust != TPMC_OK) return ust;
  launch_reduce_slots(s->qs, idx, n, s->tally, s->scal, max_nt, st);
  const double xr = ref_point ? ref_point[0] : 0.0, yr = ref_point ? ref_point[1] : 0.0,
               zr = ref_point ? ref_point[2] : 0.0;
  launch_finalize(s->qs, idx, s->scal, n, xr, yr, zr, A_ref, res, st);
  HIP_CHECK_LAUNCH("server collect");
  HIP_TRY(hipMemcpyAsync(s->res_host + (uint64_t)b * s->max_slots, res, n * sizeof(ResultDev), hipMemcpyDeviceToHost,
                         st));
  HIP_TRY(hipEventRecord(s->coll_ev[b], st));
  s->coll_n[b] = n;
  s->coll_pending[b] = true;
  *ticket = s->coll_seq++;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_server_collected(tpmc_server s, uint32_t ticket, tpmc_result* out, uint32_t n) {
  if (!s || !out) return fail(TPMC_E_INVALID, "server and out must not be NULL");
  const uint32_t b = ticket % 2;
  if (ticket >= s->coll_seq || s->coll_seq - ticket > 2 || !s->coll_pending[b])
    return fail(TPMC_E_INVALID, "collection %u is not in flight", ticket);
  if (n != s->coll_n[b]) return fail(TPMC_E_INVALID, "collection %u holds %u results, not %u", ticket, s->coll_n[b], n);
  HIP_TRY(hipSetDevice(s->ctx->device));
  HIP_TRY(hipEventSynchronize(s->coll_ev[b]));
  const ResultDev* h = s->res_host + (uint64_t)b * s->max_slots;
  for (uint32_t i = 0; i < n; ++i) copy_result(h[i], out + i);
  s->coll_pending[b] = false;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_server_results(tpmc_server s, const uint32_t* slots, uint32_t n, const double ref_point[3],
                                           double A_ref, tpmc_result* out) {
  if (!s || !slots || !out || n == 0) return fail(TPMC_E_INVALID, "server, slots and out required");
  uint32_t ticket = 0;
  tpmc_status st = tpmc_server_collect(s, slots, n, ref_point, A_ref, &ticket);
  if (st != TPMC_OK) return st;
  return tpmc_server_collected(s, ticket, out, n);
}

extern "C" tpmc_status tpmc_server_release(tpmc_server s, uint32_t slot) {
  if (!s || slot >= s->max_slots) return fail(TPMC_E_INVALID, "bad server or slot");
  s->used[slot] = 0;
  s->mesh_of[slot] = nullptr;
  return TPMC_OK;
}

extern "C" void tpmc_destroy_server(tpmc_server s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();  // pending uploads and collections read the pinned host buffers
  server_free_host(s);
  (void)hipGetLastError();
  delete s;
}

// ---------------------------------------------------------------------------
// measured ceilings (tpmc_ceilings.hip)
// ---------------------------------------------------------------------------
// One untimed launch, then one launch between two events on the context's stream.
template <class F>
static tpmc_status time_launch(tpmc_ctx ctx, F launch, double* ms) {
  HIP_TRY(hipSetDevice(ctx->device));
  launch();
  HIP_CHECK_LAUNCH("ceiling");
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  hipError_t e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipEventRecord(a, ctx->stream);
  if (e == hipSuccess) {
    launch();
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float f = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
  (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail(TPMC_E_DEVICE, "ceiling timing: %s", hipGetErrorString(e));
  if (!(f > 0.0f)) return fail(TPMC_E_DEVICE, "ceiling timing: elapsed time %g ms", (double)f);
  *ms = (double)f;
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_precull_check(tpmc_ctx ctx, tpmc_mesh m, const tpmc_query* q, void* dev_ws,
                                          uint64_t ws_bytes, double* max_err_over_margin, uint64_t* estimated) {
  if (!ctx || !m || !q || !dev_ws || !max_err_over_margin || !estimated)
    return fail(TPMC_E_INVALID, "ctx, mesh, query, workspace and outputs must not be NULL");
  if (m->ctx != ctx) return fail(TPMC_E_BUSY, "mesh belongs to another context");
  if (ws_bytes < TPMC_PRECULL_CHECK_BYTES || (uintptr_t)dev_ws % 256 != 0)
    return fail(TPMC_E_WORKSPACE, "workspace of %llu bytes at %p: need %d bytes, 256-byte aligned",
                (unsigned long long)ws_bytes, dev_ws, TPMC_PRECULL_CHECK_BYTES);
  std::vector<QueryDev> hq;
  tpmc_status s = make_queries(m, q, 1, hq);
  if (s != TPMC_OK) return s;
  static_assert(sizeof(QueryDev) + 16 <= TPMC_PRECULL_CHECK_BYTES, "check workspace too small");
  QueryDev* dq = static_cast<QueryDev*>(dev_ws);
  unsigned long long* dout = reinterpret_cast<unsigned long long*>(static_cast<uint8_t*>(dev_ws) +
                                                                   ((sizeof(QueryDev) + 15) & ~(size_t)15));
  unsigned long long h[2] = {0, 0};
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMemcpyAsync(dq, hq.data(), sizeof(QueryDev), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    launch_precull_check(dq, hq[0].N, dout, ctx->n_cu * 4, ctx->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h, dout, sizeof h, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(TPMC_E_DEVICE, "pre-cull check: %s", hipGetErrorString(e));
  double r;
  std::memcpy(&r, &h[0], sizeof r);
  *max_err_over_margin = r;
  *estimated = h[1];
  return TPMC_OK;
}

static_assert(TPMC_PROBE_SLOTS == kProbeSlots, "phase probe layout");

extern "C" tpmc_status tpmc_phase_probe(tpmc_ctx ctx, uint64_t* out, uint32_t n_slots, int reset) {
  if (!probe_built()) return fail(TPMC_E_INVALID, "library built without the phase probe (TPMC_PHASE_PROBE=1)");
  if (!ctx || !out) return fail(TPMC_E_INVALID, "ctx and out must not be NULL");
  if (n_slots < (uint32_t)kProbeSlots)
    return fail(TPMC_E_INVALID, "n_slots = %u, the probe has %d", n_slots, kProbeSlots);
  unsigned long long h[kProbeSlots];
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = probe_read(h, reset != 0, ctx->stream);
  if (e != hipSuccess) return fail(TPMC_E_DEVICE, "phase probe: %s", hipGetErrorString(e));
  for (int k = 0; k < kProbeSlots; ++k) out[k] = h[k];
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_ceiling_valu(tpmc_ctx ctx, uint32_t kind, void* dev_sink, double* lane_ops_per_s) {
  if (!ctx || !dev_sink || !lane_ops_per_s) return fail(TPMC_E_INVALID, "ctx, sink and out must not be NULL");
  if (kind > 2) return fail(TPMC_E_INVALID, "kind = %u outside 0..2", kind);
  const int grid = ctx->n_cu * 8;
  const uint32_t iters = kind == 1 ? 1024u : 2048u;
  double ms = 0.0;
  const tpmc_status st =
      time_launch(ctx, [&] { launch_ceiling_valu(kind, grid, iters, dev_sink, ctx->stream); }, &ms);
  if (st != TPMC_OK) return st;
  *lane_ops_per_s = (double)grid * kBlock * (double)ceiling_valu_ops_per_lane(iters) / (ms * 1e-3);
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_ceiling_read(tpmc_ctx ctx, const void* dev_buf, uint64_t bytes, uint32_t passes,
                                         double* bytes_per_s) {
  if (!ctx || !dev_buf || !bytes_per_s) return fail(TPMC_E_INVALID, "ctx, buffer and out must not be NULL");
  if (bytes == 0 || bytes % 16 != 0) return fail(TPMC_E_INVALID, "bytes = %llu is not a positive multiple of 16",
                                                 (unsigned long long)bytes);
  if (passes < 1) return fail(TPMC_E_INVALID, "passes must be >= 1");
  const int grid = ctx->n_cu * 8;
  double ms = 0.0;
  const tpmc_status st =
      time_launch(ctx, [&] { launch_ceiling_read(dev_buf, bytes, passes, grid, ctx->stream); }, &ms);
  if (st != TPMC_OK) return st;
  *bytes_per_s = (double)bytes * passes / (ms * 1e-3);
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_ceiling_atomic(tpmc_ctx ctx, void* dev_buf, uint32_t slots, uint32_t per_thread,
                                           double* atomics_per_s) {
  if (!ctx || !dev_buf || !atomics_per_s) return fail(TPMC_E_INVALID, "ctx, buffer and out must not be NULL");
  if (slots < 1 || slots > (1u << 26)) return fail(TPMC_E_INVALID, "slots = %u outside 1..2^26", slots);
  if (per_thread < 1 || per_thread > 4096) return fail(TPMC_E_INVALID, "per_thread = %u outside 1..4096", per_thread);
  const int grid = ctx->n_cu * 8;
  double ms = 0.0;
  const tpmc_status st =
      time_launch(ctx, [&] { launch_ceiling_atomic(dev_buf, slots, per_thread, grid, ctx->stream); }, &ms);
  if (st != TPMC_OK) return st;
  *atomics_per_s = (double)grid * kBlock * per_thread / (ms * 1e-3);
  return TPMC_OK;
}

extern "C" tpmc_status tpmc_ceiling_lds_atomic(tpmc_ctx ctx, void* dev_sink, uint32_t slots, uint32_t per_thread,
                                               double* atomics_per_s) {
  if (!ctx || !dev_sink || !atomics_per_s) return fail(TPMC_E_INVALID, "ctx, sink and out must not be NULL");
  if (slots < 1 || slots > 1024) return fail(TPMC_E_INVALID, "slots = %u outside 1..1024", slots);
  if (per_thread < 1 || per_thread > 4096) return fail(TPMC_E_INVALID, "per_thread = %u outside 1..4096", per_thread);
  const int grid = ctx->n_cu * 8;
  double ms = 0.0;
  const tpmc_status st =
      time_launch(ctx, [&] { launch_ceiling_lds_atomic(dev_sink, slots, per_thread, grid, ctx->stream); }, &ms);
  if (st != TPMC_OK) return st;
  *atomics_per_s = (double)grid * kBlock * per_thread / (ms * 1e-3);
  return TPMC_OK;
}

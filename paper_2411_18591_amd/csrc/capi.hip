// C-ABI of the propagation library: argument validation, workspace and
// table management, and the launch sequence of each entry point.  The
// operations are documented in include/toprop.h.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/toprop.h"
#include "accum.hpp"
#include "coherence.hpp"
#include <complex>

#include "launch.hpp"
#include "noalloc.hpp"
#include "plain.hpp"
#include "plan.hpp"
#include "queue.hpp"
#include "resample.hpp"
#include "transfer.hpp"

using namespace toprop;

namespace {

thread_local std::string g_last_error;

to_status fail(to_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

to_status hip_fail(hipError_t e, const char* what) {
  return fail(TO_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2i(int64_t n) {
  int k = 0;
  while ((int64_t(1) << k) < n) ++k;
  return k;
}

// Twiddle table of length L: exp(-2 pi i m / L), m < L, each entry from its
// own long-double sine and cosine (no recurrences).  All lengths 8..8192 are
// packed in one buffer; length L starts at element L - 8 (sum of the
// smaller power-of-two lengths from 8).
constexpr int kTwTotal = 2 * kMaxLen - kMinLen;
inline int tw_offset(int L) { return L - kMinLen; }

template <typename T>
std::vector<cx<T>> build_twiddles() {
  std::vector<cx<T>> h(kTwTotal);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int L = kMinLen; L <= kMaxLen; L *= 2) {
    for (int m = 0; m < L; ++m) {
      long double a = -two_pi * (long double)m / (long double)L;
      h[tw_offset(L) + m] = {(T)cosl(a), (T)sinl(a)};
    }
  }
  return h;
}

// Independent jobs of one call run concurrently on up to kLanes "lanes":
// lane 0 is the caller's stream, lanes 1.. are library streams (default
// priority) forked from and joined back into it with events.  Each lane has
// its own scratch, reduction partials and transfer-function tables.
constexpr int kLanes = 4;
// Longest chain of propagations run with fused layer boundaries (one set of
// transfer-function tables per layer).
constexpr int kMaxChain = 16;
constexpr size_t kTableSlotBytes = (size_t)kMaxLen * 2 * (sizeof(cx<float>) + sizeof(float));

struct Lane {
  hipStream_t stream = nullptr;  // null for lane 0 (the caller's stream is used)
  hipEvent_t done = nullptr;
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  double* partial = nullptr;
  size_t partial_count = 0;
  // separable transfer-function tables: ex, ey (complex64) and sx, sy
  // (float), kMaxLen entries each, one slot per layer of a chain
  void* tf = nullptr;
  // fixed: scratch and partials are a caller-provided area that is never
  // grown (the no-allocation entry point); jobs are chunked to fit it
  bool fixed = false;
};

struct DeviceCtx {
  bool init = false;
  cx<float>* tw32 = nullptr;
  cx<double>* tw64 = nullptr;
  Lane lane[kLanes];
  hipEvent_t fork = nullptr;
  void* plain = nullptr;  // workspace of the unfused baseline
  size_t plain_bytes = 0;
  void* coh = nullptr;    // workspace of the coherence propagation
  size_t coh_bytes = 0;
  void* di = nullptr;     // direct-integration tables built within a call
  size_t di_bytes = 0;
  std::vector<const void*> di_t;  // those of the current call stored transposed ([px][py])
  void* sep = nullptr;    // separable complex64 transfer-function tables of a call
  size_t sep_bytes = 0;
  void* rs = nullptr;     // per-axis tables of a resampling call
  size_t rs_bytes = 0;
  void* acc = nullptr;    // private intensity accumulators of the lanes of a call
  size_t acc_bytes = 0;
  // Tables of the non-power-of-two lengths used so far: Bluestein's chirp
  // and kernel spectrum (M > 0), or the twiddles of a mixed-radix length
  // (M = -1, twiddles in w)
  struct Blue {
    int L;
    bool dbl;
    int M;
    void* w;
    void* Bf;
  };
  std::vector<Blue> blue;
};

std::mutex g_mutex;
std::vector<DeviceCtx> g_ctx;

to_status get_ctx(DeviceCtx** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mutex);
  if ((int)g_ctx.size() <= dev) g_ctx.resize(dev + 1);
  DeviceCtx& c = g_ctx[dev];
  if (!c.init) {
    auto h32 = build_twiddles<float>();
    auto h64 = build_twiddles<double>();
    if ((e = hipMalloc(&c.tw32, sizeof(cx<float>) * kTwTotal)) != hipSuccess)
      return fail(TO_E_NOMEM, "twiddle table allocation failed: %s", hipGetErrorString(e));
    if ((e = hipMalloc(&c.tw64, sizeof(cx<double>) * kTwTotal)) != hipSuccess)
      return fail(TO_E_NOMEM, "twiddle table allocation failed: %s", hipGetErrorString(e));
    if ((e = hipMemcpy(c.tw32, h32.data(), sizeof(cx<float>) * kTwTotal, hipMemcpyHostToDevice)) !=
        hipSuccess)
      return hip_fail(e, "twiddle upload");
    if ((e = hipMemcpy(c.tw64, h64.data(), sizeof(cx<double>) * kTwTotal, hipMemcpyHostToDevice)) !=
        hipSuccess)
      return hip_fail(e, "twiddle upload");
    for (int l = 0; l < kLanes; ++l) {
      Lane& ln = c.lane[l];
      if ((e = hipMalloc(&ln.tf, kTableSlotBytes * kMaxChain)) != hipSuccess)
        return fail(TO_E_NOMEM, "table allocation failed: %s", hipGetErrorString(e));
      if (l > 0) {
        if ((e = hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking)) != hipSuccess)
          return hip_fail(e, "hipStreamCreateWithFlags");
      }
      if ((e = hipEventCreateWithFlags(&ln.done, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "hipEventCreateWithFlags");
    }
    if ((e = hipEventCreateWithFlags(&c.fork, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "hipEventCreateWithFlags");
    c.init = true;
  }
  *out = &c;
  return TO_OK;
}

// Captured calls (to_graph_create) hold the addresses of the workspaces they
// were captured with.  While any is alive, a workspace that grows is not
// freed but retired, and retired buffers are freed when the last graph is
// destroyed.
int g_live_graphs = 0;                            // under g_mutex
std::vector<std::pair<int, void*>> g_retired;     // (device, buffer), under g_mutex

void free_workspace(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mutex);
  if (g_live_graphs > 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    g_retired.emplace_back(dev, p);
  } else {
    (void)hipFree(p);
  }
}

// Grow a lane's scratch buffer to at least `bytes` (synchronizes the device
// when it has to reallocate, since queued work may still use the old buffer).
to_status ensure_scratch(Lane* c, size_t bytes) {
  if (c->scratch_bytes >= bytes) return TO_OK;
  if (c->fixed)
    return fail(TO_E_UNSUPPORTED, "the job needs %zu bytes of scratch, more than the %zu of the static area", bytes,
                c->scratch_bytes);
  hipError_t e;
  if (c->scratch) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    free_workspace(c->scratch);
    c->scratch = nullptr;
    c->scratch_bytes = 0;
  }
  if ((e = hipMalloc(&c->scratch, bytes)) != hipSuccess)
    return fail(TO_E_NOMEM, "scratch allocation of %zu bytes failed: %s", bytes,
                hipGetErrorString(e));
  c->scratch_bytes = bytes;
  return TO_OK;
}

to_status ensure_plain(DeviceCtx* c, size_t bytes) {
  if (c->plain_bytes >= bytes) return TO_OK;
  hipError_t e;
  if (c->plain) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    free_workspace(c->plain);
    c->plain = nullptr;
    c->plain_bytes = 0;
  }
  if ((e = hipMalloc(&c->plain, bytes)) != hipSuccess)
    return fail(TO_E_NOMEM, "workspace allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  c->plain_bytes = bytes;
  return TO_OK;
}

// Grow a device-wide table area (synchronizes the device when it has to
// reallocate, since queued work may still read the old one).
to_status ensure_area(void** area, size_t* have, size_t bytes, const char* what) {
  if (*have >= bytes) return TO_OK;
  hipError_t e;
  if (*area) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    free_workspace(*area);
    *area = nullptr;
    *have = 0;
  }
  if ((e = hipMalloc(area, bytes)) != hipSuccess)
    return fail(TO_E_NOMEM, "%s of %zu bytes failed: %s", what, bytes, hipGetErrorString(e));
  *have = bytes;
  return TO_OK;
}

to_status ensure_di(DeviceCtx* c, size_t bytes) {
  return ensure_area(&c->di, &c->di_bytes, bytes, "direct-integration table");
}

to_status ensure_partial(Lane* c, size_t count) {
  if (c->partial_count >= count) return TO_OK;
  if (c->fixed)
    return fail(TO_E_UNSUPPORTED, "the job needs %zu partial sums, more than the %zu of the static area", count,
                c->partial_count);
  hipError_t e;
  if (c->partial) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    free_workspace(c->partial);
    c->partial = nullptr;
    c->partial_count = 0;
  }
  if ((e = hipMalloc(&c->partial, count * sizeof(double))) != hipSuccess)
    return fail(TO_E_NOMEM, "partial-sum allocation failed: %s", hipGetErrorString(e));
  c->partial_count = count;
  return TO_OK;
}

// Launch schedule of a job: column-pass configuration (ColCfg variant) and
// chunk budget.  Precedence: the autotuner's candidate being timed (this
// thread) > TOPROP_COL_VARIANT / TOPROP_CHUNK_MB > plan table > defaults.
constexpr int kDefaultColVariant = 1;
constexpr int kDefaultChunkMb = 128;
thread_local const PlanEntry* t_force_plan = nullptr;

int env_col_variant() {  // -1: not set
  static int v = [] {
    const char* s = getenv("TOPROP_COL_VARIANT");
    if (!s) return -1;
    int x = atoi(s);
    return (x >= 0 && x < kColVariants) ? x : -1;
  }();
  return v;
}

long env_chunk_mb() {  // -1: not set
  static long mb = [] {
    const char* s = getenv("TOPROP_CHUNK_MB");
    if (!s) return -1L;
    long x = atol(s);
    return x >= 1 ? x : -1L;
  }();
  return mb;
}

int env_row_fpb() {  // 0: not set
  static int v = [] {
    const char* s = getenv("TOPROP_ROW_FPB");
    const int x = s ? atoi(s) : 0;
    return (x >= 1 && x <= kPlanMaxRowFpb) ? x : 0;
  }();
  return v;
}

struct Schedule {
  int col_variant;
  size_t chunk_bytes;
  int row_fpb;  // fields per row-pass workgroup, 0: from the occupancy target
};

// Built-in column configuration: complex64 columns of 4096 points and more
// take variant 0 (one 1024-thread workgroup per CU holding 4 or 2 columns,
// twice the columns per cache-line segment of variant 1; measured 95 against
// 107 us at 4096 points and 540 against 675 us at 8192 on one 2048^2 and
// one 4096^2 field; with the split transforms also ahead of variant 4 at
// 8192: 1569 against 1722 us per launch in the uneven batch), everything
// else variant 1.
int default_col_variant(int dtype, int ly) {
  return (dtype == 0 && ly >= 4096) ? 0 : kDefaultColVariant;
}

Schedule schedule_for(int dtype, int ly, int lx) {
  if (t_force_plan)
    return {t_force_plan->col_variant, (size_t)t_force_plan->chunk_mb << 20, t_force_plan->row_fpb};
  Schedule sc{default_col_variant(dtype, ly), (size_t)kDefaultChunkMb << 20, 0};
  PlanEntry pe;
  const bool have = plan_lookup(dtype, ly, lx, &pe);
  if (env_col_variant() >= 0)
    sc.col_variant = env_col_variant();
  else if (have)
    sc.col_variant = pe.col_variant;
  if (env_chunk_mb() >= 1)
    sc.chunk_bytes = (size_t)env_chunk_mb() << 20;
  else if (have)
    sc.chunk_bytes = (size_t)pe.chunk_mb << 20;
  if (env_row_fpb() >= 1)
    sc.row_fpb = env_row_fpb();
  else if (have)
    sc.row_fpb = pe.row_fpb;
  return sc;
}

// ---------------------------------------------------------------------------
// Kernel timing (diagnostics): while enabled, every launch is bracketed by a
// pair of HIP events recorded on its own stream; to_profile_end() waits for
// them and aggregates the elapsed times per kernel name.
// ---------------------------------------------------------------------------
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
  bool valid;  // both events recorded
};
struct ProfAgg {
  std::string name;
  int64_t launches;
  double ms;
};
std::mutex g_prof_mutex;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;
size_t g_prof_pool_used = 0;
std::vector<ProfAgg> g_prof_agg;

hipEvent_t prof_event() {
  if (g_prof_pool_used == g_prof_pool.size()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    g_prof_pool.push_back(ev);
  }
  return g_prof_pool[g_prof_pool_used++];
}

// Set while a call must not create HIP objects (the no-allocation entry
// point): its launches are not timed.
thread_local bool g_prof_suspended = false;

int prof_start(const char* name, int L, bool dbl, hipStream_t s) {
  if (!g_prof_on || g_prof_suspended) return -1;
  std::lock_guard<std::mutex> lk(g_prof_mutex);
  ProfRec r;
  char buf[96];
  snprintf(buf, sizeof(buf), "%s_%s_L%d", name, dbl ? "c128" : "c64", L);
  r.name = buf;
  r.a = prof_event();
  r.b = prof_event();
  if (!r.a || !r.b) return -1;
  if (hipEventRecord(r.a, s) != hipSuccess) return -1;  // launch not timed
  r.valid = false;
  g_prof_recs.push_back(r);
  return (int)g_prof_recs.size() - 1;
}

void prof_stop(int tok, hipStream_t s) {
  if (tok < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mutex);
  g_prof_recs[tok].valid = hipEventRecord(g_prof_recs[tok].b, s) == hipSuccess;
}

template <typename F>
hipError_t timed(const char* name, int L, bool dbl, hipStream_t s, F&& f) {
  const int tok = prof_start(name, L, dbl, s);
  hipError_t e = f();
  prof_stop(tok, s);
  return e;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Padded extents: powers of two in [kMinLen, kMaxLen] (the fused path), or
// other lengths up to kMaxAnyLen, transformed in the plain path by the
// mixed-radix passes (2^a 3^b 5^c 7^d) or by Bluestein's method (whose
// convolution length, a power of two >= 2L - 1, stays within kMaxLen).
constexpr int kMaxAnyLen = 4096;
bool extent_ok(int64_t L) {
  return is_pow2(L) ? (L >= kMinLen && L <= kMaxLen) : (L >= 3 && L <= kMaxAnyLen);
}
bool pow2_grid(const to_job& j) { return is_pow2(j.py) && is_pow2(j.px); }
bool has_jones(const to_job& j);

// Critical distance of Eq. (sampling_condition), L dx / lambda with the
// aperture length L = n d of each axis; the smaller axis value is taken, so
// the automatic choice keeps the AS method only where both axes favour it.
double critical_distance(const to_job& j) {
  return std::min((double)j.ny * j.dy * j.dy, (double)j.nx * j.dx * j.dx) / j.wavelength;
}

// The method a job runs with (TO_AUTO resolved: DI at or beyond the critical
// distance, AS below it and for z <= 0, where AS at -z is the exact adjoint).
int resolved_method(const to_job& j) {
  if (j.method != TO_AUTO) return j.method;
  return (j.z > 0.0 && j.z >= critical_distance(j)) ? TO_DI : TO_ASM;
}

// Host-side validation of one job.  `what` selects which pointers matter.
enum Mode { MODE_FWD, MODE_BWD, MODE_MOD, MODE_COH };

to_status validate(const to_job& j, int idx, to_dtype dt, Mode mode) {
  if (dt != TO_C64 && dt != TO_C128) return fail(TO_E_INVAL, "dtype %d is not TO_C64/TO_C128", (int)dt);
  if (j.ny < 1 || j.nx < 1) return fail(TO_E_INVAL, "job %d: grid %dx%d must be >= 1", idx, j.ny, j.nx);
  if (mode != MODE_MOD) {
    const int64_t ly = j.py, lx = j.px;
    if (ly < j.ny || lx < j.nx)
      return fail(TO_E_INVAL, "job %d: padded grid %lldx%lld smaller than the field %dx%d", idx,
                  (long long)ly, (long long)lx, j.ny, j.nx);
    if (!extent_ok(ly) || !extent_ok(lx))
      return fail(TO_E_UNSUPPORTED,
                  "job %d: padded grid %lldx%lld: each extent must be a power of two in [%d, %d] or any "
                  "length in [3, %d]",
                  idx, (long long)ly, (long long)lx, kMinLen, kMaxLen, kMaxAnyLen);
    if (j.method != TO_ASM && j.method != TO_FRESNEL && j.method != TO_DI && j.method != TO_AUTO)
      return fail(TO_E_INVAL, "job %d: unknown method %d", idx, j.method);
    if (!std::isfinite(j.z)) return fail(TO_E_INVAL, "job %d: z is not finite", idx);
  }
  if (!finite_pos(j.dy) || !finite_pos(j.dx))
    return fail(TO_E_INVAL, "job %d: spacing must be finite and > 0", idx);
  if (!finite_pos(j.wavelength)) return fail(TO_E_INVAL, "job %d: wavelength must be finite and > 0", idx);
  if (mode != MODE_MOD && resolved_method(j) == TO_DI) {
    if (!(j.z > 0.0))
      return fail(TO_E_INVAL, "job %d: direct integration needs z > 0 (got %g)", idx, j.z);
    if ((int64_t)j.py < 2 * (int64_t)j.ny - 1 || (int64_t)j.px < 2 * (int64_t)j.nx - 1)
      return fail(TO_E_UNSUPPORTED,
                  "job %d: direct integration needs a padded grid of at least 2n-1 per axis (field %dx%d, "
                  "padded %dx%d)",
                  idx, j.ny, j.nx, j.py, j.px);
  }
  if (!std::isfinite(j.y0) || !std::isfinite(j.x0)) return fail(TO_E_INVAL, "job %d: offset not finite", idx);
  if (j.batch < 0) return fail(TO_E_INVAL, "job %d: batch %lld < 0", idx, (long long)j.batch);
  if (j.ncomp != 1 && j.ncomp != 3) return fail(TO_E_INVAL, "job %d: ncomp must be 1 or 3", idx);
  const uint32_t known = TO_EL_PHASE | TO_EL_COMPLEX | TO_EL_LENS | TO_EL_JONES | TO_EL_JONES_MAP;
  if (j.el_flags & ~known) return fail(TO_E_INVAL, "job %d: unknown element flags 0x%x", idx, j.el_flags);
  if ((j.el_flags & (TO_EL_JONES | TO_EL_JONES_MAP)) && j.ncomp != 3)
    return fail(TO_E_INVAL, "job %d: a Jones element needs ncomp == 3", idx);
  if ((j.el_flags & TO_EL_JONES) && (j.el_flags & TO_EL_JONES_MAP))
    return fail(TO_E_INVAL, "job %d: uniform and mapped Jones matrices are exclusive", idx);
  if ((j.el_flags & TO_EL_JONES_MAP) && !j.el_jones_map)
    return fail(TO_E_INVAL, "job %d: el_jones_map is NULL", idx);
  if ((j.el_flags & TO_EL_PHASE) && !j.el_phase) return fail(TO_E_INVAL, "job %d: el_phase is NULL", idx);
  if ((j.el_flags & TO_EL_COMPLEX) && !j.el_complex)
    return fail(TO_E_INVAL, "job %d: el_complex is NULL", idx);
  if ((j.el_flags & TO_EL_LENS) && (!std::isfinite(j.el_f) || j.el_f == 0.0))
    return fail(TO_E_INVAL, "job %d: lens focal length must be finite and non-zero", idx);
  if (j.el_flags & TO_EL_JONES)
    for (int k = 0; k < 18; ++k)
      if (!std::isfinite(j.el_jones[k])) return fail(TO_E_INVAL, "job %d: Jones matrix not finite", idx);
  const bool intensity_only = mode == MODE_FWD && j.epi == TO_EPI_INTENSITY;
  if (j.batch > 0 && mode != MODE_BWD && (!j.in || (!j.out && !intensity_only)))
    return fail(TO_E_INVAL, "job %d: in/out is NULL", idx);
  if (mode == MODE_FWD && j.batch > 0) {
    if (j.epi != TO_EPI_NONE && j.epi != TO_EPI_MSE && j.epi != TO_EPI_WEIGHTED && j.epi != TO_EPI_INTENSITY)
      return fail(TO_E_INVAL, "job %d: unknown epilogue %d", idx, j.epi);
    if ((j.epi == TO_EPI_MSE || j.epi == TO_EPI_WEIGHTED) && (!j.epi_ref || !j.epi_grad || !j.epi_loss))
      return fail(TO_E_INVAL, "job %d: epilogue needs epi_ref, epi_grad and epi_loss", idx);
    if (j.epi == TO_EPI_INTENSITY && !j.epi_out)
      return fail(TO_E_INVAL, "job %d: the intensity epilogue needs epi_out", idx);
    if (j.epi != TO_EPI_NONE && !std::isfinite(j.epi_scale))
      return fail(TO_E_INVAL, "job %d: epi_scale not finite", idx);
  }
  const int64_t npix = (int64_t)j.ny * j.nx;
  if (j.batch > 0 && npix * j.ncomp > (int64_t(1) << 40) / j.batch)
    return fail(TO_E_UNSUPPORTED, "job %d: batch too large", idx);
  return TO_OK;
}

TransferParams make_transfer(const to_job& j, bool conj) {
  TransferParams p;
  const int m = resolved_method(j);
  p.method = m == TO_DI ? 2 : m;
  p.table = m == TO_DI ? j.tf_table : nullptr;
  p.conj = conj ? 1 : 0;
  const double lam = j.wavelength, z = j.z;
  p.lam2 = lam * lam;
  p.q = z / lam;
  // frac(z / lambda) without losing the fractional digits of a large ratio:
  // q_hat = fl(z/lambda), remainder r = z - q_hat lambda is exact with fma.
  const double qh = z / lam;
  const double r = std::fma(-qh, lam, z);
  p.q_frac = (qh - std::floor(qh)) + r / lam;
  p.fres_a = 0.5 * lam * z;
  p.inv_lxdx = 1.0 / ((double)j.px * j.dx);
  p.inv_lydy = 1.0 / ((double)j.py * j.dy);
  p.fast = 0;
  p.qh = (float)(0.5 * p.q);
  p.ex = p.ey = nullptr;
  p.sx = p.sy = nullptr;
  return p;
}

// Largest non-paraxial remainder (q/2) t^2 of the angular spectrum over the
// padded grid, in cycles (infinite when some bin is evanescent).  The
// largest |f| on a length-L grid of spacing d is 1/(2d) (bin -L/2).
double asm_remainder_cycles(const to_job& j) {
  const double fx = 0.5 / j.dx, fy = 0.5 / j.dy;
  const double s = j.wavelength * j.wavelength * (fx * fx + fy * fy);
  if (!(s < 1.0)) return INFINITY;
  const double t = s / (1.0 + std::sqrt(1.0 - s));
  return 0.5 * std::fabs(j.z / j.wavelength) * t * t;
}

// complex64 jobs use the separable transfer function when its FP32 remainder
// term stays below this many cycles (error ~1e-7 cycles); otherwise, and for
// complex128, the phase is evaluated per bin in FP64.
constexpr double kFastRemainderCycles = 1.0;

template <typename T>
hipError_t prepare_transfer(const to_job& j, Lane* c, hipStream_t s, TransferParams* h, int slot = 0) {
  if (sizeof(T) != 4 || h->table) return hipSuccess;
  if (h->method == TO_ASM && !(asm_remainder_cycles(j) <= kFastRemainderCycles)) return hipSuccess;
  if (j.tf_table) {  // built for the whole call at entry (prepare_jobs)
    h->fast = 1;
    h->ex = (const cx<float>*)j.tf_table;
    h->ey = h->ex + j.px;
    h->sx = (const float*)(h->ey + j.py);
    h->sy = h->sx + j.px;
    return hipSuccess;
  }
  cx<float>* ex = (cx<float>*)((char*)c->tf + (size_t)slot * kTableSlotBytes);
  cx<float>* ey = ex + kMaxLen;
  float* sx = (float*)(ey + kMaxLen);
  float* sy = sx + kMaxLen;
  hipError_t e = timed("tf_tables", j.px, false, s, [&] {
    return launch_tf_tables(ex, sx, j.px, h->inv_lxdx, ey, sy, j.py, h->inv_lydy, h->fres_a,
                            h->q_frac, h->lam2, s);
  });
  if (e != hipSuccess) return e;
  h->fast = 1;
  h->ex = ex;
  h->ey = ey;
  h->sx = sx;
  h->sy = sy;
  return hipSuccess;
}

// Fields per row block: a block pipelines the loads of its next field behind
// the transform of the current one (and evaluates the element's modulation
// once for all of them), while the launch keeps >= ~2048 blocks.
// Target block count of a row-pass launch: as many blocks as fit on the
// device at once (one round of workgroups, each taking its share of the
// fields), or TOPROP_ROW_BLOCKS.
int device_cus() {
  static int n = [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      return 256;
    return cus;
  }();
  return n;
}

int row_blocks_target(int lx, bool dbl, bool heavy) {
  static int env = [] {
    const char* s = getenv("TOPROP_ROW_BLOCKS");
    const int x = s ? atoi(s) : 0;
    return x >= 64 ? x : 0;
  }();
  return env ? env : device_cus() * row_blocks_per_cu(lx, dbl, heavy);
}

int fields_per_block_rows(int row_blocks, int nfields, int target) {
  int fpb = (int)((int64_t)row_blocks * nfields / std::max(1, target));
  if (fpb < 1) fpb = 1;
  if (fpb > 8) fpb = 8;
  if (fpb > nfields) fpb = nfields;
  return fpb;
}

template <typename T>
ElementParams<T> make_element(const to_job& j, uint32_t flags) {
  ElementParams<T> e;
  memset(&e, 0, sizeof(e));
  e.flags = flags;
  e.phase = (const T*)j.el_phase;
  e.cmask = (const cx<T>*)j.el_complex;
  e.lens_a = (flags & TO_EL_LENS) ? 1.0 / (2.0 * j.wavelength * j.el_f) : 0.0;
  e.dy = j.dy;
  e.dx = j.dx;
  e.y0 = j.y0;
  e.x0 = j.x0;
  for (int k = 0; k < 9; ++k) e.jones[k] = {(T)j.el_jones[2 * k], (T)j.el_jones[2 * k + 1]};
  e.jones_map = (const cx<T>*)j.el_jones_map;
  e.plane = (int64_t)j.ny * j.nx;
  return e;
}

template <typename T>
const cx<T>* twiddles(DeviceCtx* c, int L);
template <>
const cx<float>* twiddles<float>(DeviceCtx* c, int L) { return c->tw32 + tw_offset(L); }
template <>
const cx<double>* twiddles<double>(DeviceCtx* c, int L) { return c->tw64 + tw_offset(L); }

// Transforms of length L: the power-of-two twiddles, or the Bluestein tables
// of L (built on first use, on `s`, which is then synchronized: a first use
// is not for graph capture).
template <typename T>
to_status line_fft(DeviceCtx* c, int L, hipStream_t s, LineFft<T>* out) {
  out->L = L;
  out->M = 0;
  out->w = out->Bf = nullptr;
  out->mp.np = 0;
  if (is_pow2(L)) {
    out->tw = twiddles<T>(c, L);
    return TO_OK;
  }
  const bool dbl = sizeof(T) == 8;
  MixedPlan mp;
  if (mixed_plan(L, &mp)) {
    // 2^a 3^b 5^c 7^d: the mixed-radix passes with twiddles of length L
    // (kept in the Bluestein cache with M = -1 and no chirp tables)
    for (const auto& b : c->blue)
      if (b.L == L && b.dbl == dbl && b.M < 0) {
        out->tw = (const cx<T>*)b.w;
        out->mp = mp;
        return TO_OK;
      }
    DeviceCtx::Blue b{L, dbl, -1, nullptr, nullptr};
    hipError_t e = hipMalloc(&b.w, sizeof(cx<T>) * L);
    if (e != hipSuccess) return fail(TO_E_NOMEM, "mixed-radix twiddles: %s", hipGetErrorString(e));
    if ((e = Mixed<T>::twiddles(L, (cx<T>*)b.w, s)) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess) {
      (void)hipFree(b.w);
      return hip_fail(e, "mixed-radix twiddles");
    }
    c->blue.push_back(b);
    return line_fft<T>(c, L, s, out);
  }
  int M = 1;
  while (M < 2 * L - 1) M *= 2;
  if (M > kMaxLen) return fail(TO_E_UNSUPPORTED, "length %d is too long for Bluestein's transform", L);
  for (const auto& b : c->blue)
    if (b.L == L && b.dbl == dbl) {
      out->M = b.M;
      out->tw = twiddles<T>(c, b.M);
      out->w = (const cx<T>*)b.w;
      out->Bf = (const cx<T>*)b.Bf;
      return TO_OK;
    }
  DeviceCtx::Blue b{L, dbl, M, nullptr, nullptr};
  hipError_t e;
  if ((e = hipMalloc(&b.w, sizeof(cx<T>) * L)) != hipSuccess ||
      (e = hipMalloc(&b.Bf, sizeof(cx<T>) * M)) != hipSuccess) {
    if (b.w) (void)hipFree(b.w);
    return fail(TO_E_NOMEM, "Bluestein tables: %s", hipGetErrorString(e));
  }
  if ((e = Bluestein<T>::build(L, M, (cx<T>*)b.w, (cx<T>*)b.Bf, twiddles<T>(c, M), s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    (void)hipFree(b.w);
    (void)hipFree(b.Bf);
    return hip_fail(e, "Bluestein tables");
  }
  c->blue.push_back(b);
  return line_fft<T>(c, L, s, out);
}

// Geometry shared by the forward and backward launch sequences.
struct Geometry {
  int lx, ly, tc, tm, tc_shift;
  bool half_x, half_y;
  int nc_kernel;          // 3 when a Jones element couples the components
  int64_t nfields;        // independent field groups seen by the row kernels
  int64_t in_stride;      // elements between field groups
  int64_t comp_stride;    // elements between components
  int64_t s_stride;       // scratch elements per (field group, component)
  int64_t chunk;          // field groups per chunk
  int rows_per_block;     // rows handled by one row-pass workgroup
  int col_variant;        // column-pass configuration (see ColCfg)
  int row_fpb = 0;        // fields per row-pass workgroup from the schedule (0: automatic)
};

// Fields per row-pass workgroup: the schedule's value (at most the chunk's
// fields) or, when it leaves the choice open, as many as keep the launch at
// one round of resident workgroups.
int row_fields_per_block(const Geometry& g, int row_blocks, int nf, bool heavy, bool dbl) {
  if (g.row_fpb > 0) return std::max(1, std::min(g.row_fpb, nf));
  return fields_per_block_rows(row_blocks, nf, row_blocks_target(g.lx, dbl, heavy));
}

// Components of a field processed together by one workgroup: a Jones
// element mixes them, and the intensity epilogue sums over them.
bool has_jones(const to_job& j) { return (j.el_flags & (TO_EL_JONES | TO_EL_JONES_MAP)) != 0; }

bool coupled(const to_job& j) { return has_jones(j) || (j.epi == TO_EPI_INTENSITY && j.ncomp == 3); }

bool has_loss(const to_job& j) { return j.epi == TO_EPI_MSE || j.epi == TO_EPI_WEIGHTED; }

// Fields per column-pass block: as many as keep at least two blocks per
// CU in flight (512 on 256 CUs), so the transfer function each block forms
// is reused across fields.
// Fields per column-pass block: the transfer function is formed once per
// block and reused for its fields, while the launch keeps enough blocks:
// 512 for columns of 2048 points and more, proportionally more for shorter
// columns (whose per-field work is too short to hide latency in few blocks).
int col_fields_per_block(int ntiles, int nfields, int ly) {
  const int64_t target = 512 * std::max(1, std::min(16, 2048 / std::max(ly, 1)));
  const int64_t f = (int64_t)nfields * ntiles / target;
  return (int)std::max<int64_t>(1, std::min<int64_t>(nfields, f));
}

template <typename T>
to_status make_geometry(const to_job& j, bool jones, Geometry* g) {
  g->lx = j.px;
  g->ly = j.py;
  // Pruned first/last passes when the field fills at most half of the
  // padded extent along that axis.
  g->half_x = 2 * j.nx <= g->lx;
  g->half_y = 2 * j.ny <= g->ly;
  const Schedule sc = schedule_for(sizeof(T) == 8 ? 1 : 0, g->ly, g->lx);
  g->col_variant = sc.col_variant;
  g->row_fpb = sc.row_fpb;
  // columns per column-pass block (cpb) and the scratch tile width (tm):
  // a tile row segment is one 128-byte cache line when the rows allow it
  g->tc = col_tile_width(g->ly, sizeof(T) == 8, g->col_variant);
  if (g->tc <= 0) {  // configuration not available at this length
    g->col_variant = kDefaultColVariant;
    g->tc = col_tile_width(g->ly, sizeof(T) == 8, g->col_variant);
  }
  if (g->tc > g->lx) g->tc = g->lx;
  g->tm = std::max<int>(g->tc, (int)(128 / sizeof(cx<T>)));
  if (g->tm > g->lx) g->tm = g->lx;
  if (g->tc <= 0 || g->lx % g->tc != 0 || g->tm % g->tc != 0)
    return fail(TO_E_UNSUPPORTED, "no column configuration for %dx%d", g->ly, g->lx);
  g->tc_shift = ilog2i(g->tm);
  g->rows_per_block = row_rows_per_block(g->lx, sizeof(T) == 8, jones);
  g->nc_kernel = jones ? 3 : 1;
  const int64_t npix = (int64_t)j.ny * j.nx;
  g->nfields = jones ? j.batch : j.batch * j.ncomp;
  g->in_stride = jones ? 3 * npix : npix;
  g->comp_stride = npix;
  g->s_stride = (int64_t)g->lx * j.ny;
  const size_t per = (size_t)g->s_stride * g->nc_kernel * sizeof(cx<T>);
  int64_t ch = (int64_t)(sc.chunk_bytes / per);
  if (ch < 1) ch = 1;
  if (ch > g->nfields) ch = g->nfields;
  if (ch > 65535) ch = 65535;
  g->chunk = ch;
  return TO_OK;
}

struct Span {
  uintptr_t lo, hi;
};
Span span(const void* p, size_t bytes) {
  const uintptr_t a = (uintptr_t)p;
  return p ? Span{a, a + bytes} : Span{0, 0};
}
bool overlaps(const Span& a, const Span& b) { return a.hi > a.lo && b.hi > b.lo && a.lo < b.hi && b.lo < a.hi; }

size_t field_bytes(const to_job& j, to_dtype dt) {
  return (size_t)j.batch * j.ncomp * j.ny * j.nx * (dt == TO_C64 ? sizeof(cx<float>) : sizeof(cx<double>));
}

// Ranges a job reads besides its field: the element's mask tables and the
// epilogue's reference.
void element_spans(const to_job& j, to_dtype dt, std::vector<Span>* rd) {
  const size_t px = (size_t)j.ny * j.nx, re = dt == TO_C64 ? sizeof(float) : sizeof(double);
  if (j.el_flags & TO_EL_PHASE) rd->push_back(span(j.el_phase, px * re));
  if (j.el_flags & TO_EL_COMPLEX) rd->push_back(span(j.el_complex, px * 2 * re));
  if (j.el_flags & TO_EL_JONES_MAP) rd->push_back(span(j.el_jones_map, 9 * px * 2 * re));
  if (has_loss(j)) rd->push_back(span(j.epi_ref, px * re));
  if (resolved_method(j) == TO_DI && j.tf_table) rd->push_back(span(j.tf_table, (size_t)j.py * j.px * 2 * re));
}

// Argument records of the three passes for one chunk of `nf` fields.
template <typename T>
RowFwdArgs<T> row_fwd_args(const to_job& j, const Geometry& g, DeviceCtx* c, cx<T>* scratch, const cx<T>* in,
                           int64_t in_stride, int nf, const ElementParams<T>& el, const cx<T>* coh_m,
                           int64_t f0) {
  RowFwdArgs<T> ra;
  memset(&ra, 0, sizeof(ra));
  ra.fpb = row_fields_per_block(g, (j.ny + g.rows_per_block - 1) / g.rows_per_block, nf, g.nc_kernel == 3,
                                sizeof(T) == 8);
  ra.coh_m = coh_m;
  ra.f_off = f0;
  ra.in = in;
  ra.scratch = scratch;
  ra.in_stride = in_stride;
  ra.comp_stride = g.comp_stride;
  ra.s_stride = g.s_stride;
  ra.ny = j.ny;
  ra.nx = j.nx;
  ra.tc_shift = g.tc_shift;
  ra.nfields = nf;
  ra.el = el;
  ra.tw = twiddles<T>(c, g.lx);
  return ra;
}

template <typename T>
ColArgs<T> col_args(const to_job& j, const Geometry& g, DeviceCtx* c, cx<T>* scratch, int nf,
                    const TransferParams& h) {
  ColArgs<T> ca;
  ca.scratch = scratch;
  ca.s_stride = g.s_stride;
  ca.ny = j.ny;
  ca.lx = g.lx;
  ca.tm = g.tm;
  ca.cpb = g.tc;
  ca.nfields = nf;
  ca.fpc = col_fields_per_block(g.lx / g.tc, nf, g.ly);
  ca.h = h;
  ca.tw = twiddles<T>(c, g.ly);
  return ca;
}

template <typename T>
RowInvArgs<T> row_inv_args(const to_job& j, const Geometry& g, DeviceCtx* c, cx<T>* scratch, int nf) {
  RowInvArgs<T> ia;
  memset(&ia, 0, sizeof(ia));
  ia.scratch = scratch;
  ia.s_stride = g.s_stride;
  ia.comp_stride = g.comp_stride;
  ia.out_stride = g.in_stride;
  ia.ny = j.ny;
  ia.nx = j.nx;
  ia.tc_shift = g.tc_shift;
  ia.nfields = nf;
  ia.scale = (T)(1.0 / ((double)g.lx * (double)g.ly));
  ia.tw = twiddles<T>(c, g.lx);
  ia.epi = TO_EPI_NONE;
  return ia;
}

// Launches of one chunk's passes (profiled under `phase`).
template <typename T>
hipError_t launch_row_fwd(const char* phase, const Geometry& g, int ny, int nf, int nc, const RowFwdArgs<T>& ra,
                          hipStream_t s) {
  return timed(phase, g.lx, sizeof(T) == 8, s,
               [&] { return Launch<T>::row_fwd(g.lx, g.half_x, nc, ny, nf, ra, s); });
}

template <typename T>
hipError_t launch_col(const char* phase, const Geometry& g, const ColArgs<T>& ca, hipStream_t s) {
  return timed(phase, g.ly, sizeof(T) == 8, s, [&] {
    return Launch<T>::col(g.ly, g.half_y, g.lx / g.tc, ca.nfields, g.col_variant, ca, s);
  });
}

// Row passes of a job without element (forward row_inv: nor epilogue)
// through the job-queue kernels, with one job and one workgroup per block:
// the per-job passes with the element and epilogue branches folded away
// (fewer registers; no spills at 4096 and 8192 points).  The records must
// have the scalar-field layout those kernels assume.
template <typename T>
bool row_fwd_plain(const Geometry& g, int nc, const RowFwdArgs<T>& ra) {
  const int64_t npix = (int64_t)ra.ny * ra.nx;
  return nc == 1 && ra.el.flags == 0 && !ra.coh_m && ra.in_stride == npix && ra.comp_stride == npix &&
         ra.s_stride == (int64_t)g.lx * ra.ny && queue_row_len_ok(g.lx);
}

template <typename T>
bool row_inv_plain(const Geometry& g, int nc, const RowInvArgs<T>& ia) {
  const int64_t npix = (int64_t)ia.ny * ia.nx;
  return nc == 1 && ia.el.flags == 0 && ia.epi == TO_EPI_NONE && !ia.lens_partial && ia.out_stride == npix &&
         ia.comp_stride == npix && ia.s_stride == (int64_t)g.lx * ia.ny && queue_row_len_ok(g.lx);
}

template <typename T>
QueueArgs<T> plain_args(const Geometry& g, const cx<T>* tw, const cx<T>* in, cx<T>* out, const cx<T>* scratch,
                        int ny, int nx, int nf, int fpb) {
  QueueArgs<T> q;
  memset(&q, 0, sizeof(q));
  q.njobs = 1;
  q.lx = g.lx;
  q.tc_shift = g.tc_shift;
  q.scale = (T)(1.0 / ((double)g.lx * (double)g.ly));
  q.tw = tw;
  q.job[0].in = in;
  q.job[0].out = out;
  q.job[0].scratch = const_cast<cx<T>*>(scratch);
  q.job[0].ny = ny;
  q.job[0].nx = nx;
  q.job[0].nfields = nf;
  q.job[0].fpb = fpb > 0 ? fpb : 1;
  return q;
}

template <typename T>
hipError_t launch_row_fwd_any(const char* phase, const Geometry& g, int ny, int nf, int nc, const RowFwdArgs<T>& ra,
                              hipStream_t s) {
  if (!row_fwd_plain<T>(g, nc, ra)) return launch_row_fwd<T>(phase, g, ny, nf, nc, ra, s);
  QueueArgs<T> q = plain_args<T>(g, ra.tw, ra.in, nullptr, ra.scratch, ra.ny, ra.nx, nf, ra.fpb);
  const bool exact = ra.nx == (g.half_x ? g.lx / 2 : g.lx);
  return timed(phase, g.lx, sizeof(T) == 8, s,
               [&] { return QueueLaunch<T>::row_fwd(g.lx, g.half_x, exact, q, 0, s); });
}

template <typename T>
hipError_t launch_row_inv_any(const char* phase, const Geometry& g, int nc, int nblocks_y, const RowInvArgs<T>& ia,
                              hipStream_t s) {
  const bool dbl = sizeof(T) == 8;
  if (!row_inv_plain<T>(g, nc, ia))
    return timed(phase, g.lx, dbl, s,
                 [&] { return Launch<T>::row_inv(g.lx, g.half_x, nc, ia.ny, nblocks_y, ia, s); });
  QueueArgs<T> q = plain_args<T>(g, ia.tw, nullptr, ia.out, ia.scratch, ia.ny, ia.nx, ia.nfields, ia.fpb);
  q.scale = ia.scale;
  const bool exact = ia.nx == (g.half_x ? g.lx / 2 : g.lx);
  return timed(phase, g.lx, dbl, s,
               [&] { return QueueLaunch<T>::row_inv(g.lx, g.half_x, exact, ia.backward != 0, q, 0, s); });
}

// Forward row_inv with the job's epilogue, then the loss reduction.
template <typename T>
to_status finish_forward_chunk(const to_job& j, const Geometry& g, DeviceCtx* c, Lane* ln, cx<T>* scratch,
                               int64_t f0, int nf, hipStream_t s) {
  RowInvArgs<T> ia = row_inv_args<T>(j, g, c, scratch, nf);
  ia.out = j.out ? (cx<T>*)j.out + f0 * g.in_stride : nullptr;
  ia.epi_out = j.epi == TO_EPI_INTENSITY ? (T*)j.epi_out + f0 * (int64_t)j.ny * j.nx : nullptr;
  ia.epi = j.epi;
  ia.epi_ref = (const T*)j.epi_ref;
  ia.epi_scale = (T)j.epi_scale;
  ia.epi_grad = j.epi_grad ? (cx<T>*)j.epi_grad + f0 * g.in_stride : nullptr;
  ia.row_partial = ln->partial;
  ia.backward = 0;
  ia.fpb = row_fields_per_block(g, (j.ny + g.rows_per_block - 1) / g.rows_per_block, nf, g.nc_kernel == 3,
                                sizeof(T) == 8);
  const int inv_blocks_y = (nf + ia.fpb - 1) / ia.fpb;
  ia.el = make_element<T>(j, 0);
  const bool dbl = sizeof(T) == 8;
  hipError_t e = launch_row_inv_any<T>("fwd.row_inv", g, g.nc_kernel, inv_blocks_y, ia, s);
  if (e != hipSuccess) return hip_fail(e, "row_inv launch");
  if (has_loss(j)) {
    e = timed("fwd.loss_reduce", 0, dbl, s, [&] {
      return launch_reduce_add(ln->partial, (int64_t)nf * j.ny, j.epi_scale, j.epi_loss, s);
    });
    if (e != hipSuccess) return hip_fail(e, "loss reduction launch");
  }
  return TO_OK;
}

// Backward row_inv of one chunk (element adjoint, parameter gradients), then
// the lens-gradient reduction.
template <typename T>
to_status finish_backward_chunk(const to_job& j, const to_grad& gr, const Geometry& g, DeviceCtx* c, Lane* ln,
                                cx<T>* scratch, int64_t f0, int nf, hipStream_t s) {
  const bool want_f = (j.el_flags & TO_EL_LENS) && gr.grad_f;
  RowInvArgs<T> ia = row_inv_args<T>(j, g, c, scratch, nf);
  ia.out = gr.grad_in ? (cx<T>*)gr.grad_in + f0 * g.in_stride : nullptr;
  ia.backward = 1;
  ia.fpb = nf;
  ia.el = make_element<T>(j, j.el_flags);
  ia.saved_in = gr.saved_in ? (const cx<T>*)gr.saved_in + f0 * g.in_stride : nullptr;
  ia.grad_phase = (T*)gr.grad_phase;
  ia.lens_f = j.el_f;
  ia.lens_partial = want_f ? ln->partial : nullptr;
  const bool dbl = sizeof(T) == 8;
  hipError_t e = launch_row_inv_any<T>("bwd.row_inv", g, g.nc_kernel, 1, ia, s);
  if (e != hipSuccess) return hip_fail(e, "row_inv launch");
  if (want_f) {
    e = timed("bwd.lens_reduce", 0, dbl, s,
              [&] { return launch_reduce_add(ln->partial, j.ny, 1.0, gr.grad_f, s); });
    if (e != hipSuccess) return hip_fail(e, "lens gradient reduction launch");
  }
  return TO_OK;
}

// A fixed-area lane: fewer fields per chunk, so that a chunk's scratch and
// loss partials fit the area (at least one field must).
template <typename T>
void fit_chunk(const to_job& j, const Lane* ln, Geometry* g) {
  if (!ln->fixed) return;
  const size_t per = (size_t)g->s_stride * g->nc_kernel * sizeof(cx<T>);
  int64_t ch = std::min<int64_t>(g->chunk, (int64_t)(ln->scratch_bytes / per));
  if (has_loss(j)) ch = std::min<int64_t>(ch, (int64_t)(ln->partial_count / (size_t)j.ny));
  g->chunk = std::max<int64_t>(1, ch);
}

template <typename T>
to_status run_forward(const to_job& j, DeviceCtx* c, Lane* ln, hipStream_t s, bool conj_h = false,
                      const cx<T>* coh_m = nullptr) {
  if (j.batch == 0) return TO_OK;
  Geometry g;
  to_status st = make_geometry<T>(j, coupled(j), &g);
  if (st != TO_OK) return st;
  fit_chunk<T>(j, ln, &g);
  st = ensure_scratch(ln, (size_t)g.s_stride * g.nc_kernel * g.chunk * sizeof(cx<T>));
  if (st != TO_OK) return st;
  if (has_loss(j)) {
    st = ensure_partial(ln, (size_t)g.chunk * j.ny);
    if (st != TO_OK) return st;
  }
  cx<T>* scratch = (cx<T>*)ln->scratch;
  TransferParams h = make_transfer(j, conj_h);
  const ElementParams<T> el = make_element<T>(j, coh_m ? 0u : j.el_flags);
  hipError_t e = prepare_transfer<T>(j, ln, s, &h);
  if (e != hipSuccess) return hip_fail(e, "transfer table launch");
  for (int64_t f0 = 0; f0 < g.nfields; f0 += g.chunk) {
    const int nf = (int)std::min<int64_t>(g.chunk, g.nfields - f0);
    RowFwdArgs<T> ra = row_fwd_args<T>(j, g, c, scratch, (const cx<T>*)j.in + f0 * g.in_stride, g.in_stride, nf,
                                       el, coh_m, f0);
    if ((e = launch_row_fwd_any<T>("fwd.row_fwd", g, j.ny, nf, g.nc_kernel, ra, s)) != hipSuccess)
      return hip_fail(e, "row_fwd launch");
    if ((e = launch_col<T>("fwd.col", g, col_args<T>(j, g, c, scratch, nf * g.nc_kernel, h), s)) != hipSuccess)
      return hip_fail(e, "col launch");
    if ((st = finish_forward_chunk<T>(j, g, c, ln, scratch, f0, nf, s)) != TO_OK) return st;
  }
  return TO_OK;
}

template <typename T>
to_status run_backward(const to_job& j, const to_grad& gr, DeviceCtx* c, Lane* ln, hipStream_t s) {
  if (j.batch == 0) return TO_OK;
  Geometry g;
  to_status st = make_geometry<T>(j, has_jones(j), &g);
  if (st != TO_OK) return st;
  st = ensure_scratch(ln, (size_t)g.s_stride * g.nc_kernel * g.chunk * sizeof(cx<T>));
  if (st != TO_OK) return st;
  if ((j.el_flags & TO_EL_LENS) && gr.grad_f) {
    st = ensure_partial(ln, (size_t)j.ny);
    if (st != TO_OK) return st;
  }
  cx<T>* scratch = (cx<T>*)ln->scratch;
  TransferParams h = make_transfer(j, true);
  hipError_t e = prepare_transfer<T>(j, ln, s, &h);
  if (e != hipSuccess) return hip_fail(e, "transfer table launch");
  // The gradient rows carry no element: the first two passes treat every
  // component as an independent field.
  const ElementParams<T> none = make_element<T>(j, 0);
  for (int64_t f0 = 0; f0 < g.nfields; f0 += g.chunk) {
    const int nf = (int)std::min<int64_t>(g.chunk, g.nfields - f0);
    const int flat = nf * g.nc_kernel;
    RowFwdArgs<T> ra = row_fwd_args<T>(j, g, c, scratch, (const cx<T>*)gr.grad_out + f0 * g.in_stride,
                                       g.comp_stride, flat, none, nullptr, 0);
    if ((e = launch_row_fwd_any<T>("bwd.row_fwd", g, j.ny, flat, 1, ra, s)) != hipSuccess)
      return hip_fail(e, "row_fwd launch");
    if ((e = launch_col<T>("bwd.col", g, col_args<T>(j, g, c, scratch, flat, h), s)) != hipSuccess)
      return hip_fail(e, "col launch");
    if ((st = finish_backward_chunk<T>(j, gr, g, c, ln, scratch, f0, nf, s)) != TO_OK) return st;
  }
  return TO_OK;
}

// ---------------------------------------------------------------------------
// Chains: consecutive jobs of one call where each propagation's input is the
// previous one's output (the layers of a diffractive network).  They run
// chunk by chunk through all layers, the boundary between two layers in one
// fused row pass (row_mid), so a chunk's intermediate stays in the last-level
// cache across layers and no layer output is read back.  Results equal those
// of running the jobs one by one.
// ---------------------------------------------------------------------------
bool same_grid(const to_job& a, const to_job& b) {
  return a.ny == b.ny && a.nx == b.nx && a.py == b.py && a.px == b.px && a.batch == b.batch &&
         a.ncomp == b.ncomp && !has_jones(a) && !has_jones(b) && a.batch > 0 && pow2_grid(a);
}

// Field buffers of a chain may be shared between layers only whole (same
// start, same layout), so that processing chunk by chunk reads and writes
// every field in the order the one-by-one run would.
bool whole_or_disjoint(const std::vector<Span>& v) {
  for (size_t i = 0; i < v.size(); ++i)
    for (size_t k = i + 1; k < v.size(); ++k)
      if (overlaps(v[i], v[k]) && (v[i].lo != v[k].lo || v[i].hi != v[k].hi)) return false;
  return true;
}

bool env_no_chain() {
  static const bool v = getenv("TOPROP_NO_CHAIN") != nullptr;
  return v;
}

// Length of the forward chain starting at jobs[i] (1 = no chain).
int forward_chain_len(const to_job* jobs, int n, int i, to_dtype dt) {
  if (env_no_chain()) return 1;
  int len = 1;
  while (i + len < n && len < kMaxChain) {
    const to_job& a = jobs[i + len - 1];
    const to_job& b = jobs[i + len];
    if (!same_grid(a, b) || a.epi != TO_EPI_NONE || b.in != a.out || a.out == nullptr) break;
    if (coupled(b)) break;
    std::vector<Span> v;
    for (int k = i; k <= i + len; ++k) {
      const size_t fb = field_bytes(jobs[k], dt);
      v.push_back(span(jobs[k].in, fb));
      v.push_back(span(jobs[k].out, fb));
      if (has_loss(jobs[k])) v.push_back(span(jobs[k].epi_grad, fb));
    }
    if (!whole_or_disjoint(v)) break;
    ++len;
  }
  return len;
}

int backward_chain_len(const to_job* jobs, const to_grad* grads, int n, int i, to_dtype dt) {
  if (env_no_chain()) return 1;
  int len = 1;
  while (i + len < n && len < kMaxChain) {
    const int a = i + len - 1, b = i + len;
    if (!same_grid(jobs[a], jobs[b]) || !grads[a].grad_in || grads[b].grad_out != grads[a].grad_in) break;
    std::vector<Span> v;
    for (int k = i; k <= b; ++k) {
      const size_t fb = field_bytes(jobs[k], dt);
      v.push_back(span(grads[k].grad_out, fb));
      v.push_back(span(grads[k].grad_in, fb));
      v.push_back(span(grads[k].saved_in, fb));
    }
    if (!whole_or_disjoint(v)) break;
    ++len;
  }
  return len;
}

template <typename T>
to_status run_forward_chain(const to_job* jobs, int n, DeviceCtx* c, Lane* ln, hipStream_t s) {
  const to_job& j0 = jobs[0];
  const to_job& jl = jobs[n - 1];
  Geometry g;
  to_status st = make_geometry<T>(j0, false, &g);
  if (st != TO_OK) return st;
  st = ensure_scratch(ln, (size_t)g.s_stride * g.chunk * sizeof(cx<T>));
  if (st != TO_OK) return st;
  if (has_loss(jl) && (st = ensure_partial(ln, (size_t)g.chunk * j0.ny)) != TO_OK) return st;
  cx<T>* scratch = (cx<T>*)ln->scratch;
  TransferParams h[kMaxChain];
  ElementParams<T> el[kMaxChain];
  hipError_t e;
  for (int l = 0; l < n; ++l) {
    h[l] = make_transfer(jobs[l], false);
    if ((e = prepare_transfer<T>(jobs[l], ln, s, &h[l], l)) != hipSuccess) return hip_fail(e, "transfer table launch");
    el[l] = make_element<T>(jobs[l], jobs[l].el_flags);
  }
  const int row_blocks = (j0.ny + g.rows_per_block - 1) / g.rows_per_block;
  for (int64_t f0 = 0; f0 < g.nfields; f0 += g.chunk) {
    const int nf = (int)std::min<int64_t>(g.chunk, g.nfields - f0);
    RowFwdArgs<T> ra = row_fwd_args<T>(j0, g, c, scratch, (const cx<T>*)j0.in + f0 * g.in_stride, g.in_stride,
                                       nf, el[0], nullptr, f0);
    if ((e = launch_row_fwd_any<T>("fwd.row_fwd", g, j0.ny, nf, 1, ra, s)) != hipSuccess)
      return hip_fail(e, "row_fwd launch");
    if ((e = launch_col<T>("fwd.col", g, col_args<T>(j0, g, c, scratch, nf, h[0]), s)) != hipSuccess)
      return hip_fail(e, "col launch");
    for (int l = 0; l + 1 < n; ++l) {
      RowMidArgs<T> ma;
      ma.scratch = scratch;
      ma.s_stride = g.s_stride;
      ma.out = (cx<T>*)jobs[l].out + f0 * g.in_stride;
      ma.out_stride = g.in_stride;
      ma.ny = j0.ny;
      ma.nx = j0.nx;
      ma.tc_shift = g.tc_shift;
      ma.nfields = nf;
      ma.fpb = row_fields_per_block(g, row_blocks, nf, false, sizeof(T) == 8);
      ma.scale = (T)(1.0 / ((double)g.lx * (double)g.ly));
      ma.el = el[l + 1];
      ma.tw = twiddles<T>(c, g.lx);
      e = timed("fwd.row_mid", g.lx, sizeof(T) == 8, s, [&] {
        return Launch<T>::row_mid(g.lx, g.half_x, j0.ny, (nf + ma.fpb - 1) / ma.fpb, ma, s);
      });
      if (e != hipSuccess) return hip_fail(e, "row_mid launch");
      if ((e = launch_col<T>("fwd.col", g, col_args<T>(jobs[l + 1], g, c, scratch, nf, h[l + 1]), s)) != hipSuccess)
        return hip_fail(e, "col launch");
    }
    if ((st = finish_forward_chunk<T>(jl, g, c, ln, scratch, f0, nf, s)) != TO_OK) return st;
  }
  return TO_OK;
}

// Field groups of the fused backward boundary: each block takes `fpb`
// fields, and the groups' gradient partials are combined in order.
template <typename T>
int mid_bwd_fields_per_block(int row_blocks, int nf, const Geometry& g) {
  return row_fields_per_block(g, row_blocks, nf, false, sizeof(T) == 8);
}

// Reduction partials (doubles) of a backward chain's fused boundaries: lens
// partials [groups][ny], then phase-gradient partials [groups][ny][nx] of
// type T when there is more than one group.
template <typename T>
size_t chain_bwd_partial_count(const to_job& j, const Geometry& g) {
  const int row_blocks = (j.ny + g.rows_per_block - 1) / g.rows_per_block;
  const int nf = (int)g.chunk;
  const int fpb = mid_bwd_fields_per_block<T>(row_blocks, nf, g);
  const int groups = (nf + fpb - 1) / fpb;
  size_t n = (size_t)groups * j.ny;
  if (groups > 1) n += ((size_t)groups * j.ny * j.nx * sizeof(T) + sizeof(double) - 1) / sizeof(double);
  return n;
}

template <typename T>
to_status run_backward_chain(const to_job* jobs, const to_grad* grads, int n, DeviceCtx* c, Lane* ln,
                             hipStream_t s) {
  const to_job& j0 = jobs[0];
  Geometry g;
  to_status st = make_geometry<T>(j0, false, &g);
  if (st != TO_OK) return st;
  st = ensure_scratch(ln, (size_t)g.s_stride * g.chunk * sizeof(cx<T>));
  if (st != TO_OK) return st;
  if ((st = ensure_partial(ln, chain_bwd_partial_count<T>(j0, g))) != TO_OK) return st;
  const int row_blocks = (j0.ny + g.rows_per_block - 1) / g.rows_per_block;
  cx<T>* scratch = (cx<T>*)ln->scratch;
  TransferParams h[kMaxChain];
  hipError_t e;
  for (int l = 0; l < n; ++l) {
    h[l] = make_transfer(jobs[l], true);
    if ((e = prepare_transfer<T>(jobs[l], ln, s, &h[l], l)) != hipSuccess) return hip_fail(e, "transfer table launch");
  }
  const ElementParams<T> none = make_element<T>(j0, 0);
  const bool dbl = sizeof(T) == 8;
  for (int64_t f0 = 0; f0 < g.nfields; f0 += g.chunk) {
    const int nf = (int)std::min<int64_t>(g.chunk, g.nfields - f0);
    RowFwdArgs<T> ra = row_fwd_args<T>(j0, g, c, scratch, (const cx<T>*)grads[0].grad_out + f0 * g.in_stride,
                                       g.comp_stride, nf, none, nullptr, 0);
    if ((e = launch_row_fwd_any<T>("bwd.row_fwd", g, j0.ny, nf, 1, ra, s)) != hipSuccess)
      return hip_fail(e, "row_fwd launch");
    if ((e = launch_col<T>("bwd.col", g, col_args<T>(j0, g, c, scratch, nf, h[0]), s)) != hipSuccess)
      return hip_fail(e, "col launch");
    for (int l = 0; l + 1 < n; ++l) {
      const to_job& j = jobs[l];
      const to_grad& gr = grads[l];
      const bool want_f = (j.el_flags & TO_EL_LENS) && gr.grad_f;
      RowMidBwdArgs<T> mb;
      mb.scratch = scratch;
      mb.s_stride = g.s_stride;
      // the link to the next layer: left unwritten when only that layer reads it
      mb.grad_in = (gr.flags & TO_GRAD_IN_TRANSIENT) ? nullptr : (cx<T>*)gr.grad_in + f0 * g.in_stride;
      mb.saved_in = gr.saved_in ? (const cx<T>*)gr.saved_in + f0 * g.in_stride : nullptr;
      mb.stride = g.in_stride;
      mb.ny = j.ny;
      mb.nx = j.nx;
      mb.tc_shift = g.tc_shift;
      mb.nfields = nf;
      mb.fpb = mid_bwd_fields_per_block<T>(row_blocks, nf, g);
      const int groups = (nf + mb.fpb - 1) / mb.fpb;
      mb.scale = (T)(1.0 / ((double)g.lx * (double)g.ly));
      mb.el = make_element<T>(j, j.el_flags);
      const bool want_phase = (j.el_flags & TO_EL_PHASE) && gr.grad_phase && gr.saved_in;
      mb.grad_phase = (T*)gr.grad_phase;
      mb.gphase_part = (want_phase && groups > 1) ? (T*)(ln->partial + (size_t)groups * j.ny) : nullptr;
      mb.lens_f = j.el_f;
      mb.lens_partial = want_f ? ln->partial : nullptr;
      mb.tw = twiddles<T>(c, g.lx);
      e = timed("bwd.row_mid", g.lx, dbl, s,
                [&] { return Launch<T>::row_mid_bwd(g.lx, g.half_x, j.ny, groups, mb, s); });
      if (e != hipSuccess) return hip_fail(e, "row_mid_bwd launch");
      if (mb.gphase_part) {
        e = timed("bwd.phase_combine", 0, dbl, s, [&] {
          return launch_sum_parts<T>(mb.gphase_part, groups, (int64_t)j.ny * j.nx, (T*)gr.grad_phase, s);
        });
        if (e != hipSuccess) return hip_fail(e, "phase gradient combine launch");
      }
      if (want_f) {
        e = timed("bwd.lens_reduce", 0, dbl, s,
                  [&] { return launch_reduce_add(ln->partial, (int64_t)groups * j.ny, 1.0, gr.grad_f, s); });
        if (e != hipSuccess) return hip_fail(e, "lens gradient reduction launch");
      }
      if ((e = launch_col<T>("bwd.col", g, col_args<T>(jobs[l + 1], g, c, scratch, nf, h[l + 1]), s)) != hipSuccess)
        return hip_fail(e, "col launch");
    }
    if ((st = finish_backward_chunk<T>(jobs[n - 1], grads[n - 1], g, c, ln, scratch, f0, nf, s)) != TO_OK)
      return st;
  }
  return TO_OK;
}

template <typename T>
to_status run_modulate(const to_job& j, int adjoint, hipStream_t s) {
  if (j.batch == 0) return TO_OK;
  const bool jones = has_jones(j);
  const int64_t npix = (int64_t)j.ny * j.nx;
  const int nc = jones ? 3 : 1;
  const int64_t nfields = jones ? j.batch : j.batch * j.ncomp;
  if (nfields > INT32_MAX) return fail(TO_E_UNSUPPORTED, "too many fields");
  const ElementParams<T> el = make_element<T>(j, j.el_flags);
  hipError_t e = Launch<T>::modulate(nc, (const cx<T>*)j.in, (cx<T>*)j.out, nc * npix, npix, j.ny,
                                     j.nx, (int)nfields, adjoint, el, s);
  if (e != hipSuccess) return hip_fail(e, "modulate launch");
  return TO_OK;
}

// ---------------------------------------------------------------------------
// Scheduling of the jobs of one call over the lanes.
// ---------------------------------------------------------------------------
// Relative cost of a job: FFT work of its padded grid.
double job_cost(const to_job& j) {
  const double n = (double)j.px * (double)j.py;
  return (double)j.batch * j.ncomp * n * std::log2(n > 2 ? n : 2.0);
}

template <typename T>
void workspace_need(const to_job& j, bool backward, size_t* scratch_bytes, size_t* partial_count) {
  *scratch_bytes = 0;
  *partial_count = 0;
  if (j.batch == 0 || !pow2_grid(j)) return;
  Geometry g;
  if (make_geometry<T>(j, backward ? has_jones(j) : coupled(j), &g) != TO_OK) return;
  *scratch_bytes = (size_t)g.s_stride * g.nc_kernel * g.chunk * sizeof(cx<T>);
  if (!backward && has_loss(j)) *partial_count = (size_t)g.chunk * j.ny;
  if (backward && (j.el_flags & TO_EL_LENS)) *partial_count = (size_t)j.ny;
}

// An accumulation into a shared real array by the intensity epilogue of
// job `job` (an index into the call's prepared jobs) of scheduling unit
// `unit`.
struct AccUse {
  int unit;
  int job;
  Span span;
};

bool same_span(const Span& a, const Span& b) { return a.lo == b.lo && a.hi == b.hi; }

// Runs jobs 0..n-1.  Jobs whose written ranges overlap another job's read or
// written ranges form one group and stay in call order on one lane; groups
// are assigned longest-first to the least-loaded lane.  Lane 0 is the
// caller's stream; the other lanes fork from it and join back with events,
// so the whole call can be captured in a hipGraph.
// Accumulations (`acc`) into the same array do not conflict with each
// other: when they land on several lanes, every lane but the lowest
// accumulates into a private zeroed copy (its jobs' epi_out is redirected
// in `jobs`), and the copies are added into the array in lane order after
// the join.  `elt` is the array's element size.
template <typename Run, typename Need>
to_status run_on_lanes(DeviceCtx* c, hipStream_t s, int n, const std::vector<std::vector<Span>>& rd,
                       const std::vector<std::vector<Span>>& wr, const std::vector<double>& cost, Run&& run,
                       Need&& need, const std::vector<AccUse>* acc = nullptr, to_job* jobs = nullptr,
                       size_t elt = 0) {
  // union-find over conflicting jobs
  std::vector<int> parent(n);
  for (int i = 0; i < n; ++i) parent[i] = i;
  auto find = [&](int i) {
    while (parent[i] != i) i = parent[i] = parent[parent[i]];
    return i;
  };
  std::vector<std::vector<Span>> accs(n);
  if (acc)
    for (const AccUse& a : *acc) accs[a.unit].push_back(a.span);
  for (int i = 0; i < n; ++i)
    for (int k = i + 1; k < n; ++k) {
      bool conflict = false;
      for (const Span& w : wr[i]) {
        for (const Span& r : rd[k]) conflict |= overlaps(w, r);
        for (const Span& r : wr[k]) conflict |= overlaps(w, r);
      }
      for (const Span& w : wr[k])
        for (const Span& r : rd[i]) conflict |= overlaps(w, r);
      // accumulations: against everything else as writes; against each
      // other only when they overlap without being the same array
      for (int side = 0; side < 2; ++side) {
        const int a = side ? k : i, b = side ? i : k;
        for (const Span& w : accs[a]) {
          for (const Span& r : rd[b]) conflict |= overlaps(w, r);
          for (const Span& r : wr[b]) conflict |= overlaps(w, r);
        }
      }
      for (const Span& x : accs[i])
        for (const Span& y : accs[k]) conflict |= overlaps(x, y) && !same_span(x, y);
      if (conflict) parent[find(i)] = find(k);
    }
  std::vector<int> root(n);
  std::vector<double> gcost(n, 0.0);
  for (int i = 0; i < n; ++i) {
    root[i] = find(i);
    gcost[root[i]] += cost[i];
  }
  std::vector<int> groups;
  for (int i = 0; i < n; ++i)
    if (root[i] == i) groups.push_back(i);
  const int nl = std::min<int>(kLanes, (int)groups.size());
  std::vector<int> lane_of(n, 0);
  if (nl > 1) {
    std::sort(groups.begin(), groups.end(), [&](int a, int b) { return gcost[a] > gcost[b]; });
    std::vector<double> load(nl, 0.0);
    std::vector<int> glane(n, 0);
    for (int gi : groups) {
      int best = 0;
      for (int l = 1; l < nl; ++l)
        if (load[l] < load[best]) best = l;
      glane[gi] = best;
      load[best] += gcost[gi];
    }
    for (int i = 0; i < n; ++i) lane_of[i] = glane[root[i]];
  }
  // private accumulators: per distinct array, every lane using it but the
  // lowest gets a zeroed copy
  struct Private {
    int lane;
    Span target;
    size_t offset;
  };
  std::vector<Private> privs;
  size_t priv_total = 0;
  if (acc && nl > 1) {
    std::vector<Span> arrays;
    for (const AccUse& a : *acc) {
      bool seen = false;
      for (const Span& x : arrays) seen |= same_span(x, a.span);
      if (!seen) arrays.push_back(a.span);
    }
    for (const Span& arr : arrays) {
      int lo_lane = kLanes;
      for (const AccUse& a : *acc)
        if (same_span(a.span, arr)) lo_lane = std::min(lo_lane, lane_of[a.unit]);
      for (int l = lo_lane + 1; l < nl; ++l) {
        bool used = false;
        for (const AccUse& a : *acc) used |= same_span(a.span, arr) && lane_of[a.unit] == l;
        if (!used) continue;
        privs.push_back({l, arr, priv_total});
        priv_total += ((size_t)(arr.hi - arr.lo) + 255) & ~(size_t)255;
      }
    }
  }
  if (!privs.empty()) {
    to_status st = ensure_area(&c->acc, &c->acc_bytes, priv_total, "private accumulators");
    if (st != TO_OK) return st;
    for (const AccUse& a : *acc)
      for (const Private& p : privs)
        if (p.lane == lane_of[a.unit] && same_span(p.target, a.span)) jobs[a.job].epi_out = (char*)c->acc + p.offset;
  }
  auto accum_zero = [&](const Private& p, hipStream_t ls) {
    const int64_t cnt = (int64_t)((p.target.hi - p.target.lo) / elt);
    void* ptr = (char*)c->acc + p.offset;
    return elt == sizeof(double) ? Accum<double>::zero((double*)ptr, cnt, ls) : Accum<float>::zero((float*)ptr, cnt, ls);
  };
  auto accum_add = [&](const Private& p) {
    const int64_t cnt = (int64_t)((p.target.hi - p.target.lo) / elt);
    const void* ptr = (char*)c->acc + p.offset;
    void* dst = (void*)p.target.lo;
    return elt == sizeof(double) ? Accum<double>::add((double*)dst, (const double*)ptr, cnt, s)
                                 : Accum<float>::add((float*)dst, (const float*)ptr, cnt, s);
  };
  // size every lane's workspace before anything is enqueued
  for (int l = 0; l < nl || l == 0; ++l) {
    size_t sb = 0, pc = 0;
    for (int i = 0; i < n; ++i) {
      if (lane_of[i] != l) continue;
      size_t a, b;
      need(i, &a, &b);
      sb = std::max(sb, a);
      pc = std::max(pc, b);
    }
    to_status st;
    if (sb && (st = ensure_scratch(&c->lane[l], sb)) != TO_OK) return st;
    if (pc && (st = ensure_partial(&c->lane[l], pc)) != TO_OK) return st;
  }
  hipError_t e;
  if (nl > 1) {
    if ((e = hipEventRecord(c->fork, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int l = 1; l < nl; ++l)
      if ((e = hipStreamWaitEvent(c->lane[l].stream, c->fork, 0)) != hipSuccess)
        return hip_fail(e, "hipStreamWaitEvent");
  }
  to_status result = TO_OK;
  for (const Private& p : privs)
    if (result == TO_OK && (e = accum_zero(p, c->lane[p.lane].stream)) != hipSuccess)
      result = hip_fail(e, "accumulator reset");
  for (int i = 0; i < n && result == TO_OK; ++i) {
    const int l = lane_of[i];
    result = run(i, &c->lane[l], l == 0 ? s : c->lane[l].stream);
  }
  if (nl > 1) {  // join even after an error so no lane is left detached
    for (int l = 1; l < nl; ++l) {
      if ((e = hipEventRecord(c->lane[l].done, c->lane[l].stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
      if ((e = hipStreamWaitEvent(s, c->lane[l].done, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    }
  }
  for (const Private& p : privs)  // in lane order: deterministic
    if (result == TO_OK && (e = accum_add(p)) != hipSuccess) result = hip_fail(e, "accumulator combine");
  return result;
}

// ---------------------------------------------------------------------------
// Coherence propagation: Gamma (n x n, n = ny nx) -> P (M Gamma M^H) P^H as
// two batched field propagations around transposes.
//   forward:  A  rows r1:  row <- conj(P)(M(r1) conj(M) row)   [= Gm P^H]
//             B  transpose
//             C  rows r2:  row <- P row                         [= (P Gm P^H)^T]
//             D  transpose                                      [= Gamma_z]
//   adjoint:  A' rows: row <- P row [= G P]; B; C' rows: row <- conj(P) row
//             [= (P^H G P)^T]; D transpose with the element adjoint M^H . M.
// conj(P) = P^H because H is even in fx and fy.
// ---------------------------------------------------------------------------
to_status ensure_coh(DeviceCtx* c, size_t bytes) {
  if (c->coh_bytes >= bytes) return TO_OK;
  hipError_t e;
  if (c->coh) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    free_workspace(c->coh);
    c->coh = nullptr;
    c->coh_bytes = 0;
  }
  if ((e = hipMalloc(&c->coh, bytes)) != hipSuccess)
    return fail(TO_E_NOMEM, "coherence workspace of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  c->coh_bytes = bytes;
  return TO_OK;
}

template <typename T>
to_status run_batch_plain(const to_job& j, DeviceCtx* c, bool conj_h, const cx<T>* coh_mc, hipStream_t s);

template <typename T>
to_status run_coherence(const to_job& j, int adjoint, const to_grad* gr, DeviceCtx* c, hipStream_t s) {
  const int n = j.ny * j.nx;
  const size_t nn = (size_t)n * n;
  const size_t bytes = (nn + 2 * (size_t)n) * sizeof(cx<T>) + (2 + kCohRowChunks) * (size_t)n * sizeof(double);
  to_status st = ensure_coh(c, bytes);
  if (st != TO_OK) return st;
  cx<T>* W = (cx<T>*)c->coh;
  cx<T>* mt = W + nn;   // M(r)
  cx<T>* mtc = mt + n;  // conj(M(r))
  double* rowsum = (double*)(mtc + n);
  double* part = rowsum + n;
  double* colsum = part + n;  // kCohRowChunks * n column partials
  const bool dbl = sizeof(T) == 8;
  const bool has_el = (j.el_flags & (TO_EL_PHASE | TO_EL_COMPLEX | TO_EL_LENS)) != 0;
  const ElementParams<T> el = make_element<T>(j, j.el_flags);
  hipError_t e;
  if (has_el) {
    if ((e = Coh<T>::mtable(mt, j.ny, j.nx, el, 0, s)) != hipSuccess) return hip_fail(e, "element table");
    if ((e = Coh<T>::mtable(mtc, j.ny, j.nx, el, 1, s)) != hipSuccess) return hip_fail(e, "element table");
  }
  to_job rj = j;
  rj.batch = n;
  rj.ncomp = 1;
  rj.el_flags = 0;
  rj.epi = TO_EPI_NONE;
  cx<T>* out = (cx<T>*)j.out;
  auto transpose = [&](const cx<T>* a, cx<T>* b, const cx<T>* m) -> to_status {
    hipError_t ee = timed("coh.transpose", n, dbl, s, [&] { return Coh<T>::transpose(a, b, n, m, s); });
    return ee == hipSuccess ? TO_OK : hip_fail(ee, "transpose");
  };
  rj.in = j.in;
  rj.out = out;
  // the n batched propagations: fused kernels, or the plain path's any-length
  // sequence one field at a time (its element applied as a separate step)
  const bool fused = pow2_grid(j);
  auto batch = [&](bool conj_h, const cx<T>* m) -> to_status {
    return fused ? run_forward<T>(rj, c, &c->lane[0], s, conj_h, m)
                 : run_batch_plain<T>(rj, c, conj_h, m ? mtc : nullptr, s);
  };
  if (!adjoint) {
    if ((st = batch(true, has_el ? mt : nullptr)) != TO_OK) return st;
    if ((st = transpose(out, W, nullptr)) != TO_OK) return st;
    rj.in = W;
    rj.out = W;
    if ((st = batch(false, nullptr)) != TO_OK) return st;
    if ((st = transpose(W, out, nullptr)) != TO_OK) return st;
    if (j.epi == TO_EPI_INTENSITY) {
      e = timed("coh.diag_intensity", n, dbl, s,
                [&] { return Coh<T>::diag_intensity(out, (T*)j.epi_out, n, (T)j.epi_scale, s); });
      if (e != hipSuccess) return hip_fail(e, "coherence intensity");
    } else if (j.epi != TO_EPI_NONE) {
      e = timed("coh.diag_loss", n, dbl, s, [&] {
        return Coh<T>::diag_loss(out, (const T*)j.epi_ref, (cx<T>*)j.epi_grad, part, n, j.epi, (T)j.epi_scale,
                                 s);
      });
      if (e != hipSuccess) return hip_fail(e, "coherence loss");
      if ((e = launch_reduce_add(part, n, j.epi_scale, j.epi_loss, s)) != hipSuccess)
        return hip_fail(e, "coherence loss reduction");
    }
    return TO_OK;
  }
  if ((st = batch(false, nullptr)) != TO_OK) return st;
  if ((st = transpose(out, W, nullptr)) != TO_OK) return st;
  rj.in = W;
  rj.out = W;
  if ((st = batch(true, nullptr)) != TO_OK) return st;
  const bool want_phase = gr && gr->grad_phase && (j.el_flags & TO_EL_PHASE);
  if (!want_phase) return transpose(W, out, has_el ? mtc : nullptr);
  // G' = P^H G P in `out`, then the phase gradient, then M^H G' M in place
  if ((st = transpose(W, out, nullptr)) != TO_OK) return st;
  e = timed("coh.phase_grad", n, dbl, s, [&] {
    return Coh<T>::phase_grad(out, (const cx<T>*)gr->saved_in, mt, rowsum, colsum, (T*)gr->grad_phase, n, s);
  });
  if (e != hipSuccess) return hip_fail(e, "coherence phase gradient");
  if ((e = Coh<T>::scale(out, mt, n, s)) != hipSuccess) return hip_fail(e, "element adjoint");
  return TO_OK;
}

// ---------------------------------------------------------------------------
// Plain (unfused) form: one field at a time, one kernel per pipeline step.
// ---------------------------------------------------------------------------
template <typename T>
struct PlainWork {
  LineFft<T> fx, fy;
  cx<T>* H;
  cx<T>* pad;
  cx<T>* tmp;
  cx<T>* tmp2;
  double* partial;
  cx<T>* tr;  // transpose buffer of the column passes of non-power-of-two grids, or null
  bool fast;  // Plain::run_mixed applies (the table is stored transposed)
  int64_t chunk;  // fields per batched run_mixed pass (pad and tr hold that many)
  bool hcalc;     // run_mixed forms the transfer function in its column launch (no table built)
  TransferParams tp;
};

// Fields that go through one pass of the mixed-radix sequence together
// (Plain::run_mixed with nbatch): up to 64 MiB of [ny][px] rows per
// pass; 1 where that sequence does not apply.
template <typename T>
int64_t plain_chunk(const to_job& j) {
  MixedPlan a, b;
  if ((is_pow2(j.py) && is_pow2(j.px)) || !mixed_plan(j.py, &a, true) || !mixed_plan(j.px, &b, true)) return 1;
  const int64_t per = (int64_t)j.ny * j.px * (int64_t)sizeof(cx<T>);
  const int64_t fields = std::max<int64_t>(1, j.batch * j.ncomp);
  return std::max<int64_t>(1, std::min<int64_t>(fields, (int64_t(64) << 20) / per));
}

template <typename T>
size_t plain_bytes(const to_job& j) {
  const size_t npad = (size_t)j.py * j.px, nf = (size_t)j.ny * j.nx;
  const size_t padsz = std::max(npad, (size_t)plain_chunk<T>(j) * j.ny * j.px);
  const size_t tr = (is_pow2(j.py) && is_pow2(j.px)) ? 0 : padsz;  // columns run as transposed rows
  const size_t nt = has_jones(j) ? 3 * nf : nf;                      // a Jones element mixes three components
  return (npad + padsz + 2 * nt + tr) * sizeof(cx<T>) + 1024 * sizeof(double);
}

// Jobs of to_propagate / to_propagate_backward whose padded grid is not a
// power of two run through the plain path; its workspace and Bluestein
// tables are made ready before the lanes fork (both may synchronize).
template <typename T>
to_status prepare_plain_jobs(const to_job* jobs, int n, DeviceCtx* c, hipStream_t s) {
  size_t bytes = 0;
  for (int i = 0; i < n; ++i) {
    const to_job& j = jobs[i];
    if (j.batch == 0 || pow2_grid(j)) continue;
    bytes = std::max(bytes, plain_bytes<T>(j));
    LineFft<T> f;
    to_status st;
    if ((st = line_fft<T>(c, j.px, s, &f)) != TO_OK || (st = line_fft<T>(c, j.py, s, &f)) != TO_OK) return st;
  }
  return bytes ? ensure_plain(c, bytes) : TO_OK;
}

template <typename T>
to_status plain_setup(const to_job& j, DeviceCtx* c, bool conj, hipStream_t s, PlainWork<T>* w) {
  const size_t npad = (size_t)j.py * j.px, nf = (size_t)j.ny * j.nx;
  const size_t bytes = plain_bytes<T>(j);
  to_status st = ensure_plain(c, bytes);
  if (st != TO_OK) return st;
  if ((st = line_fft<T>(c, j.px, s, &w->fx)) != TO_OK) return st;
  if ((st = line_fft<T>(c, j.py, s, &w->fy)) != TO_OK) return st;
  w->H = (cx<T>*)c->plain;
  w->pad = w->H + npad;
  const size_t nt = has_jones(j) ? 3 * nf : nf;
  w->chunk = plain_chunk<T>(j);
  w->tmp = w->pad + std::max(npad, (size_t)w->chunk * j.ny * j.px);
  w->tmp2 = w->tmp + nt;
  w->partial = (double*)(w->tmp2 + nt);
  const bool pow2 = is_pow2(j.py) && is_pow2(j.px);
  w->tr = pow2 ? nullptr : (cx<T>*)(w->partial + 1024);
  MixedPlan qy, qx;
  w->fast = !pow2 && mixed_plan(j.py, &qy, true) && mixed_plan(j.px, &qx, true);
  TransferParams h = make_transfer(j, conj);
  hipError_t e;
  // one or two fields: AS / Fresnel formed where it is used, no table per call
  w->hcalc = w->fast && !h.table && j.batch * j.ncomp <= 2;
  w->tp = h;
  if (w->hcalc) return TO_OK;
  if (h.table) {  // direct integration: the call's (or the caller's) table
    const bool built_t = std::find(c->di_t.begin(), c->di_t.end(), h.table) != c->di_t.end();
    if (!w->fast || built_t) {  // the table as it is, or built transposed by this call
      w->H = (cx<T>*)h.table;
      return TO_OK;
    }
    e = timed("plain.table", j.px, sizeof(T) == 8, s,
              [&] { return Bluestein<T>::transpose((const cx<T>*)h.table, w->H, j.py, j.px, s); });
    return e == hipSuccess ? TO_OK : hip_fail(e, "plain table transpose");
  }
  h.conj = 0;  // the table holds H; the multiply kernel conjugates
  e = timed("plain.table", j.px, sizeof(T) == 8, s,
            [&] { return Plain<T>::table(w->H, j.py, j.px, h, s, w->fast); });
  if (e != hipSuccess) return hip_fail(e, "plain table launch");
  return TO_OK;
}

template <typename T>
to_status run_forward_plain(const to_job& j, DeviceCtx* c, hipStream_t s) {
  if (j.batch == 0) return TO_OK;
  const bool intensity = j.epi == TO_EPI_INTENSITY;
  const bool jones = has_jones(j);
  PlainWork<T> w;
  to_status st = plain_setup<T>(j, c, false, s, &w);
  if (st != TO_OK) return st;
  const int64_t nf = (int64_t)j.ny * j.nx;
  const int64_t fields = j.batch * j.ncomp;
  const bool dbl = sizeof(T) == 8;
  const ElementParams<T> el = make_element<T>(j, j.el_flags);
  // fields stored to `out` go through the mixed-radix sequence in batches
  const int64_t step = (w.fast && !jones && j.out) ? w.chunk : 1;
  for (int64_t b = 0; b < fields; b += step) {
    const int64_t nb = std::min(step, fields - b);
    if (jones && b % 3 == 0) {
      // the element of the three components of field b / 3 (M J E) into tmp
      hipError_t e = Launch<T>::modulate(3, (const cx<T>*)j.in + b * nf, w.tmp, 3 * nf, nf, j.ny, j.nx, 1, 0, el,
                                         s);
      if (e != hipSuccess) return hip_fail(e, "plain Jones element");
    }
    PlainJob<T> pj;
    pj.ny = j.ny;
    pj.nx = j.nx;
    pj.py = j.py;
    pj.px = j.px;
    pj.in = jones ? w.tmp + (b % 3) * nf : (const cx<T>*)j.in + b * nf;
    pj.out = j.out ? (cx<T>*)j.out + b * nf : w.tmp2;  // an intensity-only job keeps the field in the workspace
    pj.tmp = w.tmp;
    pj.pad = w.pad;
    pj.H = w.H;
    pj.conj = 0;
    pj.el = jones ? make_element<T>(j, 0) : el;  // with a Jones element, applied above
    pj.fx = w.fx;
    pj.fy = w.fy;
    pj.tr = w.tr;
    pj.ht = w.fast ? 1 : 0;
    pj.hcalc = w.hcalc ? 1 : 0;
    pj.tp = w.tp;
    pj.nbatch = nb;
    hipError_t e = timed("plain.propagate", j.px, dbl, s, [&] { return Plain<T>::run(pj, s); });
    if (e != hipSuccess) return hip_fail(e, "plain propagation");
    for (int64_t k = 0; k < nb; ++k) {
      const int64_t fb = b + k;
      const cx<T>* field = pj.out + k * nf;
      if (intensity) {
        // epi_out[fb / ncomp] += epi_scale |field|^2, the components in order
        e = Plain<T>::intensity(field, (T*)j.epi_out + (fb / j.ncomp) * nf, nf, (T)j.epi_scale, s);
        if (e != hipSuccess) return hip_fail(e, "plain intensity");
      } else if (j.epi != TO_EPI_NONE) {
        int nblk = 0;
        e = Plain<T>::loss(field, (const T*)j.epi_ref, (cx<T>*)j.epi_grad + fb * nf, w.partial, nf, j.epi,
                           (T)j.epi_scale, &nblk, s);
        if (e != hipSuccess) return hip_fail(e, "plain loss");
        if ((e = launch_reduce_add(w.partial, nblk, j.epi_scale, j.epi_loss, s)) != hipSuccess)
          return hip_fail(e, "plain loss reduction");
      }
    }
  }
  return TO_OK;
}

// Backward of a job with a Jones element, one three-component field at a
// time: g_mod = P^H grad_out per component (into tmp2), the modulated
// input M J saved_in (into tmp) for the parameter gradients, which sum
// Im(g_mod conj(M J saved_in)) over the components in order, and
// grad_in = J^H conj(M) g_mod.
template <typename T>
to_status run_backward_plain_jones(const to_job& j, const to_grad& gr, const PlainWork<T>& w,
                                   const ElementParams<T>& el, hipStream_t s) {
  const int64_t nf = (int64_t)j.ny * j.nx;
  const bool dbl = sizeof(T) == 8;
  ElementParams<T> none = el;  // the grid geometry and lens coefficient, no modulation
  none.flags = 0;
  const bool want_phase = gr.grad_phase && (j.el_flags & TO_EL_PHASE) && gr.saved_in;
  const bool want_f = gr.grad_f && (j.el_flags & TO_EL_LENS) && gr.saved_in;
  for (int64_t f = 0; f < j.batch; ++f) {
    hipError_t e = hipSuccess;
    for (int comp = 0; comp < 3 && e == hipSuccess; ++comp) {
      PlainJob<T> pj;
      pj.ny = j.ny;
      pj.nx = j.nx;
      pj.py = j.py;
      pj.px = j.px;
      pj.in = (const cx<T>*)gr.grad_out + (3 * f + comp) * nf;
      pj.out = w.tmp2 + comp * nf;
      pj.tmp = w.tmp;
      pj.pad = w.pad;
      pj.H = w.H;
      pj.conj = 1;
      pj.el = none;
      pj.fx = w.fx;
      pj.fy = w.fy;
      pj.tr = w.tr;
      pj.ht = w.fast ? 1 : 0;
      pj.hcalc = w.hcalc ? 1 : 0;
      pj.tp = w.tp;
      e = timed("plain.adjoint", j.px, dbl, s, [&] { return Plain<T>::run(pj, s); });
    }
    if (e != hipSuccess) return hip_fail(e, "plain adjoint");
    if (want_phase || want_f) {
      e = Launch<T>::modulate(3, (const cx<T>*)gr.saved_in + 3 * f * nf, w.tmp, 3 * nf, nf, j.ny, j.nx, 1, 0, el,
                              s);
      for (int comp = 0; comp < 3 && e == hipSuccess; ++comp) {
        if (want_phase)
          e = Plain<T>::phase_grad(w.tmp2 + comp * nf, w.tmp + comp * nf, (T*)gr.grad_phase, j.ny, j.nx, none, s);
        if (want_f && e == hipSuccess) {
          int nb = 0;
          e = Plain<T>::lens_grad(w.tmp2 + comp * nf, w.tmp + comp * nf, w.partial, j.ny, j.nx, none, j.el_f, &nb,
                                  s);
          if (e == hipSuccess) e = launch_reduce_add(w.partial, nb, 1.0, gr.grad_f, s);
        }
      }
      if (e != hipSuccess) return hip_fail(e, "plain parameter gradients");
    }
    if (gr.grad_in) {
      e = Launch<T>::modulate(3, w.tmp2, (cx<T>*)gr.grad_in + 3 * f * nf, 3 * nf, nf, j.ny, j.nx, 1, 1, el, s);
      if (e != hipSuccess) return hip_fail(e, "plain input gradient");
    }
  }
  return TO_OK;
}

template <typename T>
to_status run_backward_plain(const to_job& j, const to_grad& gr, DeviceCtx* c, hipStream_t s) {
  if (j.batch == 0) return TO_OK;
  PlainWork<T> w;
  to_status st = plain_setup<T>(j, c, true, s, &w);
  if (st != TO_OK) return st;
  const int64_t nf = (int64_t)j.ny * j.nx;
  const int64_t fields = j.batch * j.ncomp;
  const bool dbl = sizeof(T) == 8;
  const ElementParams<T> el = make_element<T>(j, j.el_flags);
  if (has_jones(j)) return run_backward_plain_jones<T>(j, gr, w, el, s);
  // with grad_in given, g_mod = P^H grad_out goes there (in batches through
  // the mixed-radix sequence) and is modulated in place; else into tmp2
  const bool direct = gr.grad_in != nullptr;
  const int64_t step = (w.fast && direct) ? w.chunk : 1;
  const bool has_el = (j.el_flags & (TO_EL_PHASE | TO_EL_COMPLEX | TO_EL_LENS)) != 0;
  for (int64_t b = 0; b < fields; b += step) {
    const int64_t nb = std::min(step, fields - b);
    PlainJob<T> pj;
    pj.ny = j.ny;
    pj.nx = j.nx;
    pj.py = j.py;
    pj.px = j.px;
    pj.in = (const cx<T>*)gr.grad_out + b * nf;
    pj.out = direct ? (cx<T>*)gr.grad_in + b * nf : w.tmp2;  // g_mod = P^H grad_out
    pj.tmp = w.tmp;
    pj.pad = w.pad;
    pj.H = w.H;
    pj.conj = 1;
    pj.el = make_element<T>(j, 0);
    pj.fx = w.fx;
    pj.fy = w.fy;
    pj.tr = w.tr;
    pj.ht = w.fast ? 1 : 0;
    pj.hcalc = w.hcalc ? 1 : 0;
    pj.tp = w.tp;
    pj.nbatch = nb;
    hipError_t e = timed("plain.adjoint", j.px, dbl, s, [&] { return Plain<T>::run(pj, s); });
    if (e != hipSuccess) return hip_fail(e, "plain adjoint");
    for (int64_t k = 0; k < nb; ++k) {
      const int64_t fb = b + k;
      cx<T>* gm = pj.out + k * nf;
      if (gr.grad_phase && (j.el_flags & TO_EL_PHASE) && gr.saved_in) {
        e = Plain<T>::phase_grad(gm, (const cx<T>*)gr.saved_in + fb * nf, (T*)gr.grad_phase, j.ny, j.nx, el, s);
        if (e != hipSuccess) return hip_fail(e, "plain phase gradient");
      }
      if (gr.grad_f && (j.el_flags & TO_EL_LENS) && gr.saved_in) {
        int nblk = 0;
        e = Plain<T>::lens_grad(gm, (const cx<T>*)gr.saved_in + fb * nf, w.partial, j.ny, j.nx, el, j.el_f, &nblk,
                                s);
        if (e == hipSuccess) e = launch_reduce_add(w.partial, nblk, 1.0, gr.grad_f, s);
        if (e != hipSuccess) return hip_fail(e, "plain lens gradient");
      }
      if (direct && has_el) {
        e = Plain<T>::modulate(gm, gm, j.ny, j.nx, el, 1, s);  // grad_in = conj(M) g_mod, in place
        if (e != hipSuccess) return hip_fail(e, "plain input gradient");
      }
    }
  }
  return TO_OK;
}


// The batched propagations of a coherence matrix on a padded grid that is
// not a power of two: j.batch fields [ny][nx] from j.in to j.out (in place
// allowed), P or P^H (conj_h), one field at a time through the plain path.
// coh_mc = conj(M): the element as the coherence modulation
// Gamma(r1, r2) M(r1) conj(M(r2)), applied first (into j.out).
template <typename T>
to_status run_batch_plain(const to_job& j, DeviceCtx* c, bool conj_h, const cx<T>* coh_mc, hipStream_t s) {
  if (j.batch == 0) return TO_OK;
  const int64_t nf = (int64_t)j.ny * j.nx;
  const bool dbl = sizeof(T) == 8;
  const cx<T>* src = (const cx<T>*)j.in;
  hipError_t e;
  if (coh_mc) {
    if (j.in != j.out &&
        (e = hipMemcpyAsync(j.out, j.in, (size_t)j.batch * nf * sizeof(cx<T>), hipMemcpyDeviceToDevice, s)) !=
            hipSuccess)
      return hip_fail(e, "coherence copy");
    if ((e = Coh<T>::scale((cx<T>*)j.out, coh_mc, (int)nf, s)) != hipSuccess) return hip_fail(e, "element");
    src = (const cx<T>*)j.out;
  }
  PlainWork<T> w;
  to_status st = plain_setup<T>(j, c, conj_h, s, &w);
  if (st != TO_OK) return st;
  const int64_t step = w.fast ? w.chunk : 1;
  for (int64_t b = 0; b < j.batch; b += step) {
    PlainJob<T> pj;
    pj.ny = j.ny;
    pj.nx = j.nx;
    pj.py = j.py;
    pj.px = j.px;
    pj.in = src + b * nf;
    pj.out = (cx<T>*)j.out + b * nf;
    pj.tmp = w.tmp;
    pj.pad = w.pad;
    pj.H = w.H;
    pj.conj = conj_h ? 1 : 0;
    pj.el = make_element<T>(j, 0);
    pj.fx = w.fx;
    pj.fy = w.fy;
    pj.tr = w.tr;
    pj.ht = w.fast ? 1 : 0;
    pj.hcalc = w.hcalc ? 1 : 0;
    pj.tp = w.tp;
    pj.nbatch = std::min(step, j.batch - b);
    e = timed("plain.coh_batch", j.px, dbl, s, [&] { return Plain<T>::run(pj, s); });
    if (e != hipSuccess) return hip_fail(e, "plain propagation");
  }
  return TO_OK;
}

// Times one forward propagation of `j` under the schedule `pe` (lane 0,
// stream s): one untimed run, then the mean of `reps` runs between events.
template <typename T>
to_status time_candidate(const to_job& j, DeviceCtx* c, hipStream_t s, const PlanEntry& pe, int reps,
                         hipEvent_t ea, hipEvent_t eb, double* us) {
  t_force_plan = &pe;
  size_t sb, pc;
  workspace_need<T>(j, false, &sb, &pc);
  to_status st = TO_OK;
  if (sb) st = ensure_scratch(&c->lane[0], sb);
  if (st == TO_OK && pc) st = ensure_partial(&c->lane[0], pc);
  if (st == TO_OK) st = run_forward<T>(j, c, &c->lane[0], s);
  hipError_t e = hipSuccess;
  if (st == TO_OK) e = hipEventRecord(ea, s);
  for (int r = 0; r < reps && st == TO_OK && e == hipSuccess; ++r) st = run_forward<T>(j, c, &c->lane[0], s);
  if (st == TO_OK && e == hipSuccess) e = hipEventRecord(eb, s);
  if (st == TO_OK && e == hipSuccess) e = hipEventSynchronize(eb);
  float ms = 0.f;
  if (st == TO_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, ea, eb);
  t_force_plan = nullptr;
  if (st != TO_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "autotune timing");
  *us = 1000.0 * ms / reps;
  return TO_OK;
}

// frac(z / lambda), exact: see make_transfer.
double exact_cycles_frac(double z, double lam) {
  const double qh = z / lam;
  const double r = std::fma(-qh, lam, z);
  return (qh - std::floor(qh)) + r / lam;
}

DiParams di_params(const to_job& j) {
  DiParams p;
  p.ny = j.ny;
  p.nx = j.nx;
  p.py = j.py;
  p.px = j.px;
  p.dy = j.dy;
  p.dx = j.dx;
  p.z = j.z;
  p.lam = j.wavelength;
  p.q_frac = exact_cycles_frac(j.z, j.wavelength);
  return p;
}

bool same_di_geometry(const to_job& a, const to_job& b) {
  return a.ny == b.ny && a.nx == b.nx && a.py == b.py && a.px == b.px && a.dy == b.dy && a.dx == b.dx &&
         a.wavelength == b.wavelength && a.z == b.z;
}

// Copies the (validated) jobs of a call with TO_AUTO resolved, and gives every
// direct-integration job that carries no table of its own one built on `s`
// before any other work of the call (one table per distinct geometry, in the
// device's DI area; every lane forks from `s` after it, and the area is only
// rebuilt by a later call, which `s` orders after this one).
bool same_sep_geometry(const to_job& a, const to_job& b) {
  return a.py == b.py && a.px == b.px && a.dy == b.dy && a.dx == b.dx && a.wavelength == b.wavelength &&
         a.z == b.z;
}

// complex64 jobs whose transfer function takes the separable form get their
// 1-D tables from one batched launch for the whole call (one table per
// distinct padded grid, spacing, wavelength and distance), carried in the
// prepared copy's tf_table.
to_status prepare_separable(std::vector<to_job>* jobs, DeviceCtx* c, hipStream_t s) {
  const int n = (int)jobs->size();
  std::vector<int> first, table_of(n, -1);
  std::vector<size_t> offset;
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    const to_job& j = (*jobs)[i];
    if (j.batch == 0 || j.method == TO_DI || !pow2_grid(j)) continue;
    if (j.method == TO_ASM && !(asm_remainder_cycles(j) <= kFastRemainderCycles)) continue;
    int k = 0;
    while (k < (int)first.size() && !same_sep_geometry((*jobs)[first[k]], j)) ++k;
    if (k == (int)first.size()) {
      first.push_back(i);
      offset.push_back(total);
      total += ((size_t)(j.px + j.py) * (sizeof(cx<float>) + sizeof(float)) + 255) & ~(size_t)255;
    }
    table_of[i] = k;
  }
  if (first.empty()) return TO_OK;
  to_status st = ensure_area(&c->sep, &c->sep_bytes, total, "transfer-function tables");
  if (st != TO_OK) return st;
  for (size_t k0 = 0; k0 < first.size(); k0 += kSepBatch) {
    SepTableBatch b;
    memset(&b, 0, sizeof(b));
    for (size_t k = k0; k < first.size() && k < k0 + kSepBatch; ++k) {
      const to_job& j = (*jobs)[first[k]];
      const TransferParams h = make_transfer(j, false);
      SepTableDesc& d = b.d[b.count++];
      d.base = (char*)c->sep + offset[k];
      d.lx = j.px;
      d.ly = j.py;
      d.inv_lxdx = h.inv_lxdx;
      d.inv_lydy = h.inv_lydy;
      d.fres_a = h.fres_a;
      d.q_frac = h.q_frac;
      d.lam2 = h.lam2;
      b.maxlen = std::max(b.maxlen, j.px + j.py);
    }
    hipError_t e = timed("tf_tables", b.maxlen, false, s, [&] { return separable_tables(b, s); });
    if (e != hipSuccess) return hip_fail(e, "transfer-function tables");
  }
  for (int i = 0; i < n; ++i)
    if (table_of[i] >= 0) (*jobs)[i].tf_table = (char*)c->sep + offset[table_of[i]];
  return TO_OK;
}

template <typename T>
to_status prepare_jobs(const to_job* jobs, int n, DeviceCtx* c, hipStream_t s, std::vector<to_job>* out) {
  out->assign(jobs, jobs + n);
  std::vector<int> first;       // index of the job whose geometry each table has
  std::vector<size_t> offset;   // byte offset of each table in the DI area
  std::vector<int> table_of(n, -1);
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    to_job& j = (*out)[i];
    j.method = resolved_method(j);
    if (j.method != TO_DI) j.tf_table = nullptr;  // the field is read for DI only
    if (j.method != TO_DI || j.tf_table || j.batch == 0) continue;
    int k = 0;
    while (k < (int)first.size() && !same_di_geometry((*out)[first[k]], j)) ++k;
    if (k == (int)first.size()) {
      first.push_back(i);
      offset.push_back(total);
      total += ((size_t)j.py * j.px * sizeof(cx<T>) + 255) & ~(size_t)255;
    }
    table_of[i] = k;
  }
  c->di_t.clear();
  if (first.empty()) return TO_OK;
  // Tables of grids that take the any-length mixed-radix sequence are built
  // transposed, the layout its column launch reads; others with a column
  // length that is not a power of two transform their columns as rows of
  // the transposed table.  Both use scratch after the tables.
  auto transposed = [](const to_job& j) {
    MixedPlan a, b;
    return !(is_pow2(j.py) && is_pow2(j.px)) && mixed_plan(j.py, &a, true) && mixed_plan(j.px, &b, true);
  };
  size_t scratch = 0;
  for (int k : first)
    if (!is_pow2((*out)[k].py) || transposed((*out)[k]))
      scratch = std::max(scratch, (size_t)(*out)[k].py * (*out)[k].px * sizeof(cx<T>));
  to_status st = ensure_di(c, total + scratch);
  if (st != TO_OK) return st;
  cx<T>* tr = scratch ? (cx<T>*)((char*)c->di + total) : nullptr;
  for (size_t k = 0; k < first.size(); ++k) {
    const to_job& j = (*out)[first[k]];
    cx<T>* H = (cx<T>*)((char*)c->di + offset[k]);
    LineFft<T> fx, fy;
    if ((st = line_fft<T>(c, j.px, s, &fx)) != TO_OK) return st;
    if ((st = line_fft<T>(c, j.py, s, &fy)) != TO_OK) return st;
    const bool t = transposed(j);
    if (t) c->di_t.push_back(H);
    hipError_t e = timed("di_table", j.px, sizeof(T) == 8, s, [&] {
      return t ? TransferTable<T>::direct_integration_t(H, tr, di_params(j), fx, fy, s)
               : TransferTable<T>::direct_integration(H, di_params(j), fx, fy, s, tr);
    });
    if (e != hipSuccess) return hip_fail(e, "direct-integration table");
  }
  for (int i = 0; i < n; ++i)
    if (table_of[i] >= 0) (*out)[i].tf_table = (char*)c->di + offset[table_of[i]];
  return TO_OK;
}

template <typename T>
to_status prepare_all(const to_job* jobs, int n, DeviceCtx* c, hipStream_t s, std::vector<to_job>* out) {
  to_status st = prepare_jobs<T>(jobs, n, c, s, out);
  if (st == TO_OK && sizeof(T) == 4) st = prepare_separable(out, c, s);
  return st;
}

to_status prepare_jobs_dt(const to_job* jobs, int n, to_dtype dt, DeviceCtx* c, hipStream_t s,
                          std::vector<to_job>* out) {
  return dt == TO_C64 ? prepare_all<float>(jobs, n, c, s, out) : prepare_all<double>(jobs, n, c, s, out);
}

// ---------------------------------------------------------------------------
// Job-queue groups: independent propagations of one shape class, each too
// small to fill the device with its own launches, run as one launch per pass
// over all of them (QueueLaunch) instead of three launches per job.  A group
// is one scheduling unit on the lanes.  Every eligible job runs through the
// queue kernels, alone or not, so its result does not depend on the other
// jobs of the call.
// ---------------------------------------------------------------------------
// Upper bound of a group's summed intermediates: a group's passes then
// hand their intermediate to the next pass through the last-level cache
// (256 MiB, shared by the lanes) instead of HBM.
constexpr size_t kQueueScratchCap = (size_t)64 << 20;

bool env_no_queue() { return getenv("TOPROP_NO_QUEUE") != nullptr; }  // read per call

struct QueueKey {
  int lx, ly, variant, tc, tm;
  bool half_x, half_y, ex_x, ex_y;
  bool operator==(const QueueKey& o) const {
    return lx == o.lx && ly == o.ly && variant == o.variant && tc == o.tc && tm == o.tm && half_x == o.half_x &&
           half_y == o.half_y && ex_x == o.ex_x && ex_y == o.ex_y;
  }
};

// Shape class of job j for a job-queue launch and the size of its padded
// intermediate; false where the job runs on its own: grids beyond the
// queue's lengths, coupled components, elements, epilogues, more fields
// than one chunk, or a transfer function whose tables would be built in the
// lane (one slot, not one per job).
template <typename T>
bool queue_class(const to_job& j, bool backward, QueueKey* key, size_t* scratch_bytes) {
  if (j.batch == 0 || !pow2_grid(j) || !queue_len_ok(j.px) || !queue_len_ok(j.py)) return false;
  if (j.el_flags != 0 || coupled(j) || has_jones(j)) return false;
  if (!backward && j.epi != TO_EPI_NONE) return false;
  Geometry g;
  if (make_geometry<T>(j, false, &g) != TO_OK || g.nc_kernel != 1 || g.chunk < g.nfields) return false;
  if (sizeof(T) == 4) {
    const TransferParams h = make_transfer(j, backward);
    const bool exact_phase = h.method == TO_ASM && !(asm_remainder_cycles(j) <= kFastRemainderCycles);
    if (!h.table && !exact_phase && !j.tf_table) return false;
  }
  key->lx = g.lx;
  key->ly = g.ly;
  key->variant = g.col_variant;
  key->tc = g.tc;
  key->tm = g.tm;
  key->half_x = g.half_x;
  key->half_y = g.half_y;
  key->ex_x = j.nx == (g.half_x ? g.lx / 2 : g.lx);
  key->ex_y = j.ny == (g.half_y ? g.ly / 2 : g.ly);
  *scratch_bytes = ((size_t)g.s_stride * g.nfields * sizeof(cx<T>) + 255) & ~(size_t)255;
  return true;
}

// Scheduling units of a call: a chain of `len` jobs from `beg` (len 1: one
// job), or a job-queue group (`group` >= 0, an index into the call's groups).
struct Unit {
  int beg, len, group;
};

// Groups the single-job units whose jobs share a class and touch no range
// any other job of the call touches (so they may run in any order, in one
// launch); a job joins the first open group of its class.  An eligible job
// that conflicts with another job forms a group of its own.  `jrd` / `jwr`:
// each job's read and written ranges.
template <typename T>
std::vector<Unit> group_units(const to_job* jobs, const std::vector<Unit>& units, bool backward,
                              const std::vector<std::vector<Span>>& jrd, const std::vector<std::vector<Span>>& jwr,
                              std::vector<std::vector<int>>* groups) {
  groups->clear();
  const int n = (int)jrd.size();
  auto touches = [&](int a, int b) {  // a writes what b reads or writes, or the reverse
    for (const Span& w : jwr[a]) {
      for (const Span& r : jrd[b]) if (overlaps(w, r)) return true;
      for (const Span& r : jwr[b]) if (overlaps(w, r)) return true;
    }
    for (const Span& w : jwr[b])
      for (const Span& r : jrd[a]) if (overlaps(w, r)) return true;
    return false;
  };
  std::vector<QueueKey> gkey;
  std::vector<size_t> gbytes;
  std::vector<bool> gopen;  // whether other jobs may join
  std::vector<int> group_of(units.size(), -1);
  for (size_t u = 0; u < units.size(); ++u) {
    if (units[u].len != 1) continue;
    const int i = units[u].beg;
    QueueKey key;
    size_t bytes = 0;
    if (!queue_class<T>(jobs[i], backward, &key, &bytes)) continue;
    bool alone = true;
    for (int k = 0; k < n && alone; ++k) alone = k == i || !touches(i, k);
    int gi = 0;
    while (alone && gi < (int)groups->size() &&
           !(gkey[gi] == key && gopen[gi] && (int)(*groups)[gi].size() < kQueueJobs &&
             gbytes[gi] + bytes <= kQueueScratchCap))
      ++gi;
    if (!alone) gi = (int)groups->size();
    if (gi == (int)groups->size()) {
      groups->emplace_back();
      gkey.push_back(key);
      gbytes.push_back(0);
      gopen.push_back(alone);
    }
    (*groups)[gi].push_back((int)u);
    gbytes[gi] += bytes;
    group_of[u] = gi;
  }
  // a group takes the place of its first unit
  std::vector<int> renum(groups->size(), -1);
  std::vector<std::vector<int>> kept;
  std::vector<Unit> out;
  for (size_t u = 0; u < units.size(); ++u) {
    const int gi = group_of[u];
    if (gi < 0) {
      out.push_back(units[u]);
      continue;
    }
    if ((*groups)[gi].front() != (int)u) continue;
    renum[gi] = (int)kept.size();
    std::vector<int> members;
    for (int v : (*groups)[gi]) members.push_back(units[v].beg);
    kept.push_back(members);
    out.push_back(Unit{units[u].beg, 1, renum[gi]});
  }
  *groups = kept;
  return out;
}

// Scratch of a group: each member's intermediate at its own offset.
template <typename T>
size_t queue_scratch(const to_job* jobs, const std::vector<int>& members, bool backward,
                     std::vector<size_t>* offsets) {
  size_t total = 0;
  for (int i : members) {
    QueueKey key;
    size_t bytes = 0;
    queue_class<T>(jobs[i], backward, &key, &bytes);
    if (offsets) offsets->push_back(total);
    total += bytes;
  }
  return total;
}

// Forward (grads == nullptr) or adjoint propagation of a job-queue group.
template <typename T>
to_status run_queue(const to_job* jobs, const to_grad* grads, const std::vector<int>& members, DeviceCtx* c,
                    Lane* ln, hipStream_t s) {
  const bool bwd = grads != nullptr;
  const bool dbl = sizeof(T) == 8;
  std::vector<size_t> off;
  const size_t total = queue_scratch<T>(jobs, members, bwd, &off);
  to_status st = ensure_scratch(ln, total);
  if (st != TO_OK) return st;
  Geometry g0;
  if ((st = make_geometry<T>(jobs[members[0]], false, &g0)) != TO_OK) return st;
  QueueArgs<T> rf, ri;
  ColQueueArgs<T> cq;
  memset(&rf, 0, sizeof(rf));
  memset(&ri, 0, sizeof(ri));
  memset(&cq, 0, sizeof(cq));
  rf.njobs = ri.njobs = cq.q.njobs = (int)members.size();
  rf.lx = ri.lx = cq.q.lx = g0.lx;
  rf.tc_shift = ri.tc_shift = cq.q.tc_shift = g0.tc_shift;
  cq.q.tm = g0.tm;
  cq.q.cpb = g0.tc;
  ri.scale = (T)(1.0 / ((double)g0.lx * (double)g0.ly));
  rf.tw = ri.tw = twiddles<T>(c, g0.lx);
  cq.q.tw = twiddles<T>(c, g0.ly);
  for (size_t k = 0; k < members.size(); ++k) {
    const to_job& j = jobs[members[k]];
    Geometry g;
    if ((st = make_geometry<T>(j, false, &g)) != TO_OK) return st;
    const int nf = (int)g.nfields;
    cx<T>* scratch = (cx<T>*)((char*)ln->scratch + off[k]);
    const int row_blocks = (j.ny + g.rows_per_block - 1) / g.rows_per_block;
    TransferParams h = make_transfer(j, bwd);
    hipError_t e = prepare_transfer<T>(j, ln, s, &h);  // takes the call's table; launches nothing here
    if (e != hipSuccess) return hip_fail(e, "transfer table");
    QueueJob<T> base;
    memset(&base, 0, sizeof(base));
    base.scratch = scratch;
    base.ny = j.ny;
    base.nx = j.nx;
    base.nfields = nf;
    rf.job[k] = base;
    rf.job[k].in = (const cx<T>*)(bwd ? grads[members[k]].grad_out : j.in);
    rf.job[k].fpb = row_fields_per_block(g, row_blocks, nf, false, dbl);
    cq.q.job[k] = base;
    cq.q.job[k].fpb = col_fields_per_block(g.lx / g.tc, nf, g.ly);
    cq.h[k] = h;
    ri.job[k] = base;
    ri.job[k].out = (cx<T>*)(bwd ? grads[members[k]].grad_in : j.out);
    ri.job[k].fpb = bwd ? nf : row_fields_per_block(g, row_blocks, nf, false, dbl);
  }
  const int cus = device_cus();
  const QueueKey* kp = nullptr;
  QueueKey key;
  size_t bytes;
  if (queue_class<T>(jobs[members[0]], bwd, &key, &bytes)) kp = &key;
  if (!kp) return fail(TO_E_INVAL, "job-queue group of an ineligible job");
  hipError_t e = timed(bwd ? "bwd.queue_row_fwd" : "fwd.queue_row_fwd", g0.lx, dbl, s,
                       [&] { return QueueLaunch<T>::row_fwd(g0.lx, key.half_x, key.ex_x, rf, cus, s); });
  if (e != hipSuccess) return hip_fail(e, "queue row_fwd launch");
  e = timed(bwd ? "bwd.queue_col" : "fwd.queue_col", g0.ly, dbl, s,
            [&] { return QueueLaunch<T>::col(g0.ly, key.half_y, key.ex_y, key.variant, cq, cus, s); });
  if (e != hipSuccess) return hip_fail(e, "queue col launch");
  e = timed(bwd ? "bwd.queue_row_inv" : "fwd.queue_row_inv", g0.lx, dbl, s,
            [&] { return QueueLaunch<T>::row_inv(g0.lx, key.half_x, key.ex_x, bwd, ri, cus, s); });
  if (e != hipSuccess) return hip_fail(e, "queue row_inv launch");
  return TO_OK;
}

to_status plan_args(int32_t py, int32_t px, to_dtype dtype) {
  if (dtype != TO_C64 && dtype != TO_C128) return fail(TO_E_INVAL, "dtype must be TO_C64 or TO_C128");
  (void)py;
  (void)px;
  return TO_OK;
}

}  // namespace

namespace toprop {

to_status set_error(to_status st, const char* msg) { return fail(st, "%s", msg); }

to_status hip_error(hipError_t e, const char* what) { return hip_fail(e, what); }

// to_propagate's work with every workspace carved from `ws` and everything
// on `stream`: no allocation, no library streams or events, no profiling.
// `tw` holds the twiddle tables in the packed layout of build_twiddles
// (complex64 tables first, then complex128).
// Layout of a fixed area: one transfer-function table slot, the loss
// partial sums, then the chunk scratch.
constexpr size_t kFixedPartialBytes = (size_t)1 << 20;
size_t fixed_scratch_bytes(size_t ws_bytes) {
  const size_t head = kTableSlotBytes + kFixedPartialBytes;
  return ws_bytes > head ? ws_bytes - head : 0;
}

to_status validate_forward(const to_job* jobs, int32_t njobs, to_dtype dtype, size_t ws_bytes) {
  const size_t avail = fixed_scratch_bytes(ws_bytes);
  for (int i = 0; i < njobs; ++i) {
    to_status st = validate(jobs[i], i, dtype, MODE_FWD);
    if (st != TO_OK) return st;
    const to_job& j = jobs[i];
    if (j.batch == 0) continue;
    if (!pow2_grid(j))
      return fail(TO_E_UNSUPPORTED, "job %d: padded grid %dx%d: the no-allocation entry point needs powers of two",
                  i, j.py, j.px);
    if (resolved_method(j) == TO_DI && !j.tf_table)
      return fail(TO_E_UNSUPPORTED,
                  "job %d: direct integration without a caller table (to_transfer_table) needs workspace", i);
    const size_t per = (size_t)j.px * j.ny * (coupled(j) ? 3 : 1) *
                       (dtype == TO_C64 ? sizeof(cx<float>) : sizeof(cx<double>));
    if (per > avail)
      return fail(TO_E_UNSUPPORTED,
                  "job %d: one field needs %zu bytes of scratch (ny x px x coupled components), more than the %zu "
                  "bytes of the static area",
                  i, per, avail);
    if (has_loss(j) && (size_t)j.ny * sizeof(double) > kFixedPartialBytes)
      return fail(TO_E_UNSUPPORTED, "job %d: %d rows exceed the static partial sums", i, j.ny);
  }
  return TO_OK;
}

to_status propagate_fixed(const to_job* jobs, int32_t njobs, to_dtype dtype, hipStream_t s, const void* tw,
                          void* ws, size_t ws_bytes) {
  static_assert(kTwTotal == kTwPacked, "packed twiddle layout");
  DeviceCtx c;
  c.tw32 = (cx<float>*)tw;
  c.tw64 = (cx<double>*)((char*)tw + sizeof(cx<float>) * kTwTotal);
  Lane ln;
  ln.fixed = true;
  char* p = (char*)ws;
  ln.tf = p;
  p += kTableSlotBytes;
  ln.partial = (double*)p;
  ln.partial_count = kFixedPartialBytes / sizeof(double);
  p += kFixedPartialBytes;
  ln.scratch = p;
  ln.scratch_bytes = fixed_scratch_bytes(ws_bytes);
  g_prof_suspended = true;
  to_status st = TO_OK;
  for (int i = 0; i < njobs && st == TO_OK; ++i)
    st = dtype == TO_C64 ? run_forward<float>(jobs[i], &c, &ln, s) : run_forward<double>(jobs[i], &c, &ln, s);
  g_prof_suspended = false;
  return st;
}

}  // namespace toprop

extern "C" {

to_status to_propagate_plain(const to_job* jobs, int32_t njobs, to_dtype dtype, void* stream) {
  if (njobs < 0) return fail(TO_E_INVAL, "njobs < 0");
  if (njobs > 0 && !jobs) return fail(TO_E_INVAL, "jobs is NULL");
  for (int i = 0; i < njobs; ++i) {
    to_status st = validate(jobs[i], i, dtype, MODE_FWD);
    if (st != TO_OK) return st;
  }
  if (njobs == 0) return TO_OK;
  DeviceCtx* c;
  to_status st = get_ctx(&c);
  if (st != TO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  std::vector<to_job> prepared;
  if ((st = prepare_jobs_dt(jobs, njobs, dtype, c, s, &prepared)) != TO_OK) return st;
  jobs = prepared.data();
  for (int i = 0; i < njobs; ++i) {
    st = dtype == TO_C64 ? run_forward_plain<float>(jobs[i], c, s) : run_forward_plain<double>(jobs[i], c, s);
    if (st != TO_OK) return st;
  }
  return TO_OK;
}

to_status to_propagate_backward_plain(const to_job* jobs, const to_grad* grads, int32_t njobs,
                                      to_dtype dtype, void* stream) {
  if (njobs < 0) return fail(TO_E_INVAL, "njobs < 0");
  if (njobs > 0 && (!jobs || !grads)) return fail(TO_E_INVAL, "jobs or grads is NULL");
  for (int i = 0; i < njobs; ++i) {
    to_status st = validate(jobs[i], i, dtype, MODE_BWD);
    if (st != TO_OK) return st;
    if (jobs[i].batch > 0 && !grads[i].grad_out) return fail(TO_E_INVAL, "job %d: grad_out is NULL", i);
    if (jobs[i].batch > 0 && grads[i].grad_phase && (jobs[i].el_flags & TO_EL_PHASE) && !grads[i].saved_in)
      return fail(TO_E_INVAL, "job %d: a parameter gradient needs saved_in", i);
  }
  if (njobs == 0) return TO_OK;
  DeviceCtx* c;
  to_status st = get_ctx(&c);
  if (st != TO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  std::vector<to_job> prepared;
  if ((st = prepare_jobs_dt(jobs, njobs, dtype, c, s, &prepared)) != TO_OK) return st;
  jobs = prepared.data();
  for (int i = 0; i < njobs; ++i) {
    st = dtype == TO_C64 ? run_backward_plain<float>(jobs[i], grads[i], c, s)
                         : run_backward_plain<double>(jobs[i], grads[i], c, s);
    if (st != TO_OK) return st;
  }
  return TO_OK;
}

to_status to_propagate(const to_job* jobs, int32_t njobs, to_dtype dtype, void* stream) {
  if (njobs < 0) return fail(TO_E_INVAL, "njobs < 0");
  if (njobs > 0 && !jobs) return fail(TO_E_INVAL, "jobs is NULL");
  for (int i = 0; i < njobs; ++i) {
    to_status st = validate(jobs[i], i, dtype, MODE_FWD);
    if (st != TO_OK) return st;
  }
  if (njobs == 0) return TO_OK;
  DeviceCtx* c;
  to_status st = get_ctx(&c);
  if (st != TO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  std::vector<to_job> prepared;
  if ((st = prepare_jobs_dt(jobs, njobs, dtype, c, s, &prepared)) != TO_OK) return st;
  jobs = prepared.data();
  st = dtype == TO_C64 ? prepare_plain_jobs<float>(jobs, njobs, c, s) : prepare_plain_jobs<double>(jobs, njobs, c, s);
  if (st != TO_OK) return st;
  // scheduling units: single jobs, chains of layers, job-queue groups
  std::vector<Unit> units;
  for (int i = 0; i < njobs;) {
    const int len = forward_chain_len(jobs, njobs, i, dtype);
    units.push_back(Unit{i, len, -1});
    i += len;
  }
  const size_t relt = dtype == TO_C64 ? sizeof(float) : sizeof(double);
  std::vector<std::vector<Span>> jrd(njobs), jwr(njobs);
  for (int i = 0; i < njobs; ++i) {
    const to_job& j = jobs[i];
    const size_t fb = field_bytes(j, dtype);
    jrd[i].push_back(span(j.in, fb));
    jwr[i].push_back(span(j.out, fb));
    element_spans(j, dtype, &jrd[i]);
    if (has_loss(j)) {
      jwr[i].push_back(span(j.epi_grad, fb));
      jwr[i].push_back(span(j.epi_loss, sizeof(double)));
    }
    if (!pow2_grid(j)) jwr[i].push_back(Span{1, 2});  // the plain path's one workspace
  }
  std::vector<std::vector<int>> groups;
  if (!env_no_queue()) {
    // for grouping, an intensity accumulation counts as a write
    std::vector<std::vector<Span>> jw = jwr;
    for (int i = 0; i < njobs; ++i)
      if (jobs[i].epi == TO_EPI_INTENSITY && jobs[i].batch > 0)
        jw[i].push_back(span(jobs[i].epi_out, (size_t)jobs[i].batch * jobs[i].ny * jobs[i].nx * relt));
    units = dtype == TO_C64 ? group_units<float>(jobs, units, false, jrd, jw, &groups)
                            : group_units<double>(jobs, units, false, jrd, jw, &groups);
  }
  auto members = [&](int u) {
    std::vector<int> m;
    if (units[u].group >= 0) return groups[units[u].group];
    for (int i = units[u].beg; i < units[u].beg + units[u].len; ++i) m.push_back(i);
    return m;
  };
  const int nu = (int)units.size();
  std::vector<std::vector<Span>> rd(nu), wr(nu);
  std::vector<double> cost(nu, 0.0);
  std::vector<AccUse> acc;
  for (int u = 0; u < nu; ++u) {
    for (int i : members(u)) {
      const to_job& j = jobs[i];
      rd[u].insert(rd[u].end(), jrd[i].begin(), jrd[i].end());
      wr[u].insert(wr[u].end(), jwr[i].begin(), jwr[i].end());
      if (j.epi == TO_EPI_INTENSITY && j.batch > 0)
        acc.push_back({u, i, span(j.epi_out, (size_t)j.batch * j.ny * j.nx * relt)});
      cost[u] += job_cost(j);
    }
  }
  auto run = [&](int u, Lane* ln, hipStream_t ls) {
    const Unit& un = units[u];
    if (un.group >= 0)
      return dtype == TO_C64 ? run_queue<float>(jobs, nullptr, groups[un.group], c, ln, ls)
                             : run_queue<double>(jobs, nullptr, groups[un.group], c, ln, ls);
    const to_job* js = jobs + un.beg;
    if (!pow2_grid(*js))
      return dtype == TO_C64 ? run_forward_plain<float>(*js, c, ls) : run_forward_plain<double>(*js, c, ls);
    if (un.len > 1)
      return dtype == TO_C64 ? run_forward_chain<float>(js, un.len, c, ln, ls)
                             : run_forward_chain<double>(js, un.len, c, ln, ls);
    return dtype == TO_C64 ? run_forward<float>(*js, c, ln, ls) : run_forward<double>(*js, c, ln, ls);
  };
  auto need = [&](int u, size_t* sb, size_t* pc) {
    *sb = 0;
    *pc = 0;
    if (units[u].group >= 0) {
      *sb = dtype == TO_C64 ? queue_scratch<float>(jobs, groups[units[u].group], false, nullptr)
                            : queue_scratch<double>(jobs, groups[units[u].group], false, nullptr);
      return;
    }
    for (int i : members(u)) {
      size_t a = 0, b = 0;
      if (dtype == TO_C64)
        workspace_need<float>(jobs[i], false, &a, &b);
      else
        workspace_need<double>(jobs[i], false, &a, &b);
      *sb = std::max(*sb, a);
      *pc = std::max(*pc, b);
    }
  };
  return run_on_lanes(c, s, nu, rd, wr, cost, run, need, &acc, prepared.data(), relt);
}

to_status to_modulate(const to_job* jobs, int32_t njobs, to_dtype dtype, int32_t adjoint,
                      void* stream) {
  if (njobs < 0) return fail(TO_E_INVAL, "njobs < 0");
  if (njobs > 0 && !jobs) return fail(TO_E_INVAL, "jobs is NULL");
  for (int i = 0; i < njobs; ++i) {
    to_status st = validate(jobs[i], i, dtype, MODE_MOD);
    if (st != TO_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < njobs; ++i) {
    to_status st = dtype == TO_C64 ? run_modulate<float>(jobs[i], adjoint, s)
                                   : run_modulate<double>(jobs[i], adjoint, s);
    if (st != TO_OK) return st;
  }
  return TO_OK;
}

to_status to_propagate_backward(const to_job* jobs, const to_grad* grads, int32_t njobs,
                                to_dtype dtype, void* stream) {
  if (njobs < 0) return fail(TO_E_INVAL, "njobs < 0");
  if (njobs > 0 && (!jobs || !grads)) return fail(TO_E_INVAL, "jobs or grads is NULL");
  for (int i = 0; i < njobs; ++i) {
    to_status st = validate(jobs[i], i, dtype, MODE_BWD);
    if (st != TO_OK) return st;
    const to_grad& g = grads[i];
    if (g.flags & ~TO_GRAD_IN_TRANSIENT) return fail(TO_E_INVAL, "job %d: unknown gradient flags 0x%x", i, g.flags);
    if (jobs[i].batch > 0) {
      if (!g.grad_out) return fail(TO_E_INVAL, "job %d: grad_out is NULL", i);
      const bool want_param = (g.grad_phase && (jobs[i].el_flags & TO_EL_PHASE)) ||
                              (g.grad_f && (jobs[i].el_flags & TO_EL_LENS));
      if (want_param && !g.saved_in)
        return fail(TO_E_INVAL, "job %d: a parameter gradient needs saved_in", i);
    }
  }
  if (njobs == 0) return TO_OK;
  DeviceCtx* c;
  to_status st = get_ctx(&c);
  if (st != TO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  std::vector<to_job> prepared;
  if ((st = prepare_jobs_dt(jobs, njobs, dtype, c, s, &prepared)) != TO_OK) return st;
  jobs = prepared.data();
  st = dtype == TO_C64 ? prepare_plain_jobs<float>(jobs, njobs, c, s) : prepare_plain_jobs<double>(jobs, njobs, c, s);
  if (st != TO_OK) return st;
  std::vector<Unit> units;
  for (int i = 0; i < njobs;) {
    const int len = backward_chain_len(jobs, grads, njobs, i, dtype);
    units.push_back(Unit{i, len, -1});
    i += len;
  }
  std::vector<std::vector<Span>> jrd(njobs), jwr(njobs);
  for (int i = 0; i < njobs; ++i) {
    const to_job& j = jobs[i];
    const to_grad& g = grads[i];
    const size_t fb = field_bytes(j, dtype);
    const size_t rb = (size_t)j.ny * j.nx * (dtype == TO_C64 ? sizeof(float) : sizeof(double));
    jrd[i].push_back(span(g.grad_out, fb));
    jrd[i].push_back(span(g.saved_in, fb));
    element_spans(j, dtype, &jrd[i]);
    jwr[i].push_back(span(g.grad_in, fb));
    jwr[i].push_back(span(g.grad_phase, rb));
    jwr[i].push_back(span(g.grad_f, sizeof(double)));
    if (!pow2_grid(j)) jwr[i].push_back(Span{1, 2});  // the plain path's one workspace
  }
  std::vector<std::vector<int>> groups;
  if (!env_no_queue())
    units = dtype == TO_C64 ? group_units<float>(jobs, units, true, jrd, jwr, &groups)
                            : group_units<double>(jobs, units, true, jrd, jwr, &groups);
  auto members = [&](int u) {
    std::vector<int> m;
    if (units[u].group >= 0) return groups[units[u].group];
    for (int i = units[u].beg; i < units[u].beg + units[u].len; ++i) m.push_back(i);
    return m;
  };
  const int nu = (int)units.size();
  std::vector<std::vector<Span>> rd(nu), wr(nu);
  std::vector<double> cost(nu, 0.0);
  for (int u = 0; u < nu; ++u) {
    for (int i : members(u)) {
      rd[u].insert(rd[u].end(), jrd[i].begin(), jrd[i].end());
      wr[u].insert(wr[u].end(), jwr[i].begin(), jwr[i].end());
      cost[u] += job_cost(jobs[i]);
    }
  }
  auto run = [&](int u, Lane* ln, hipStream_t ls) {
    const Unit& un = units[u];
    if (un.group >= 0)
      return dtype == TO_C64 ? run_queue<float>(jobs, grads, groups[un.group], c, ln, ls)
                             : run_queue<double>(jobs, grads, groups[un.group], c, ln, ls);
    const int i = un.beg;
    if (!pow2_grid(jobs[i]))
      return dtype == TO_C64 ? run_backward_plain<float>(jobs[i], grads[i], c, ls)
                             : run_backward_plain<double>(jobs[i], grads[i], c, ls);
    if (un.len > 1)
      return dtype == TO_C64 ? run_backward_chain<float>(jobs + i, grads + i, un.len, c, ln, ls)
                             : run_backward_chain<double>(jobs + i, grads + i, un.len, c, ln, ls);
    return dtype == TO_C64 ? run_backward<float>(jobs[i], grads[i], c, ln, ls)
                           : run_backward<double>(jobs[i], grads[i], c, ln, ls);
  };
  auto need = [&](int u, size_t* sb, size_t* pc) {
    *sb = 0;
    *pc = 0;
    if (units[u].group >= 0) {
      *sb = dtype == TO_C64 ? queue_scratch<float>(jobs, groups[units[u].group], true, nullptr)
                            : queue_scratch<double>(jobs, groups[units[u].group], true, nullptr);
      return;
    }
    for (int i : members(u)) {
      size_t a = 0, b = 0;
      if (dtype == TO_C64)
        workspace_need<float>(jobs[i], true, &a, &b);
      else
        workspace_need<double>(jobs[i], true, &a, &b);
      *sb = std::max(*sb, a);
      *pc = std::max(*pc, b);
    }
    if (units[u].len > 1) {
      Geometry g;
      const to_job& j0 = jobs[units[u].beg];
      if (dtype == TO_C64 && make_geometry<float>(j0, false, &g) == TO_OK)
        *pc = std::max(*pc, chain_bwd_partial_count<float>(j0, g));
      if (dtype == TO_C128 && make_geometry<double>(j0, false, &g) == TO_OK)
        *pc = std::max(*pc, chain_bwd_partial_count<double>(j0, g));
    }
  };
  return run_on_lanes(c, s, nu, rd, wr, cost, run, need);
}

to_status to_coherence_propagate(const to_job* job, to_dtype dtype, int32_t adjoint,
                                 const to_grad* grad, void* stream) {
  if (!job) return fail(TO_E_INVAL, "job is NULL");
  to_status st = validate(*job, 0, dtype, MODE_COH);
  if (st != TO_OK) return st;
  const to_job& j = *job;
  if (j.batch != 1 || j.ncomp != 1) return fail(TO_E_INVAL, "coherence job needs batch == 1 and ncomp == 1");
  if (has_jones(j)) return fail(TO_E_UNSUPPORTED, "coherence job with a Jones element");
  if ((int64_t)j.ny * j.nx > 46340) return fail(TO_E_UNSUPPORTED, "coherence grid too large");
  if (adjoint && j.epi != TO_EPI_NONE) return fail(TO_E_INVAL, "the adjoint has no epilogue");
  if (j.epi != TO_EPI_NONE) {
    if (j.epi != TO_EPI_MSE && j.epi != TO_EPI_WEIGHTED && j.epi != TO_EPI_INTENSITY)
      return fail(TO_E_INVAL, "unknown epilogue %d", j.epi);
    if (has_loss(j) && (!j.epi_ref || !j.epi_grad || !j.epi_loss))
      return fail(TO_E_INVAL, "epilogue needs epi_ref, epi_grad and epi_loss");
    if (j.epi == TO_EPI_INTENSITY && !j.epi_out) return fail(TO_E_INVAL, "the intensity epilogue needs epi_out");
    if (!std::isfinite(j.epi_scale)) return fail(TO_E_INVAL, "epi_scale not finite");
  }
  if (adjoint && grad && grad->grad_phase && (j.el_flags & TO_EL_PHASE)) {
    if (!grad->saved_in) return fail(TO_E_INVAL, "the phase gradient needs saved_in (the forward input)");
    if (grad->saved_in == j.out) return fail(TO_E_INVAL, "saved_in must not alias out");
  }
  DeviceCtx* c;
  if ((st = get_ctx(&c)) != TO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  std::vector<to_job> prepared;
  if ((st = prepare_jobs_dt(job, 1, dtype, c, s, &prepared)) != TO_OK) return st;
  return dtype == TO_C64 ? run_coherence<float>(prepared[0], adjoint, grad, c, s)
                         : run_coherence<double>(prepared[0], adjoint, grad, c, s);
}

to_status to_autotune(const to_job* job, to_dtype dtype, void* stream, to_plan* result) {
  if (!job) return fail(TO_E_INVAL, "job is NULL");
  to_status st = validate(*job, 0, dtype, MODE_FWD);
  if (st != TO_OK) return st;
  if (job->batch == 0) return fail(TO_E_INVAL, "autotune needs a job with batch >= 1");
  if (!pow2_grid(*job)) return fail(TO_E_UNSUPPORTED, "autotune needs power-of-two padded extents");
  DeviceCtx* c;
  if ((st = get_ctx(&c)) != TO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int dt = dtype == TO_C64 ? 0 : 1;
  // tuning copy: no epilogue, output into a temporary buffer (the job may be
  // in place, and every candidate runs it several times)
  std::vector<to_job> prepared;
  if ((st = prepare_jobs_dt(job, 1, dtype, c, s, &prepared)) != TO_OK) return st;
  to_job tj = prepared[0];
  tj.epi = TO_EPI_NONE;
  tj.epi_grad = nullptr;
  tj.epi_loss = nullptr;
  tj.epi_ref = nullptr;
  tj.epi_out = nullptr;
  void* tmp = nullptr;
  hipError_t e = hipMalloc(&tmp, field_bytes(*job, dtype));
  if (e != hipSuccess) return fail(TO_E_NOMEM, "autotune output allocation failed: %s", hipGetErrorString(e));
  tj.out = tmp;
  hipEvent_t ea = nullptr, eb = nullptr;
  if ((e = hipEventCreate(&ea)) != hipSuccess || (e = hipEventCreate(&eb)) != hipSuccess) {
    if (ea) (void)hipEventDestroy(ea);
    (void)hipFree(tmp);
    return hip_fail(e, "hipEventCreate");
  }
  static const int kChunkMb[] = {32, 64, 128, 256};
  PlanEntry best{kDefaultColVariant, kDefaultChunkMb, -1.0};
  std::vector<std::pair<int, int64_t>> seen;  // (variant, chunk fields) already timed
  for (int v = 0; v < kColVariants && st == TO_OK; ++v) {
    if (v == 4 && tj.py < 8192) continue;  // the same kernels as variant 0 below 8192 points
    for (int mb : kChunkMb) {
      PlanEntry pe{v, mb, 0.0};
      Geometry g;
      t_force_plan = &pe;
      const to_status gs = dtype == TO_C64 ? make_geometry<float>(tj, coupled(tj), &g)
                                           : make_geometry<double>(tj, coupled(tj), &g);
      t_force_plan = nullptr;
      if (gs != TO_OK || g.col_variant != v) continue;
      const std::pair<int, int64_t> key(v, g.chunk);
      bool dup = false;
      for (auto& k : seen) dup |= k == key;
      if (dup) continue;  // a larger budget that changes nothing
      seen.push_back(key);
      double us = 0.0;
      st = dtype == TO_C64 ? time_candidate<float>(tj, c, s, pe, 3, ea, eb, &us)
                           : time_candidate<double>(tj, c, s, pe, 3, ea, eb, &us);
      if (st != TO_OK) break;
      if (best.us < 0 || us < best.us) {
        best = pe;
        best.us = us;
      }
    }
  }
  // then the fields per row-pass workgroup, with the best column
  // configuration and chunk (0: the occupancy rule)
  static const int kRowFpb[] = {1, 2, 4, 8};
  for (int fpb : kRowFpb) {
    if (st != TO_OK) break;
    const int64_t nf = (int64_t)tj.batch * (coupled(tj) ? 1 : tj.ncomp);
    if (fpb > 1 && fpb > nf) continue;  // the same as the largest already timed
    PlanEntry pe{best.col_variant, best.chunk_mb, 0.0, fpb};
    double us = 0.0;
    st = dtype == TO_C64 ? time_candidate<float>(tj, c, s, pe, 3, ea, eb, &us)
                         : time_candidate<double>(tj, c, s, pe, 3, ea, eb, &us);
    if (st == TO_OK && us < best.us) {
      best = pe;
      best.us = us;
    }
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  (void)hipFree(tmp);  // the timed runs were synchronized above
  if (st != TO_OK) return st;
  plan_store(dt, job->py, job->px, best);
  if (!plan_env_path().empty()) {
    std::string err;
    plan_save_file(plan_env_path().c_str(), &err);  // best effort: the table holds the plan
  }
  if (result) *result = {best.col_variant, best.chunk_mb, best.row_fpb, best.us};
  // the job itself, once, under the stored plan
  return to_propagate(job, 1, dtype, stream);
}

to_status to_plan_get(int32_t py, int32_t px, to_dtype dtype, to_plan* plan, int32_t* found) {
  to_status st = plan_args(py, px, dtype);
  if (st != TO_OK) return st;
  if (!plan || !found) return fail(TO_E_INVAL, "plan or found is NULL");
  PlanEntry pe;
  *found = plan_lookup(dtype == TO_C64 ? 0 : 1, py, px, &pe) ? 1 : 0;
  if (*found) *plan = {pe.col_variant, pe.chunk_mb, pe.row_fpb, pe.us};
  return TO_OK;
}

to_status to_plan_set(int32_t py, int32_t px, to_dtype dtype, const to_plan* plan) {
  to_status st = plan_args(py, px, dtype);
  if (st != TO_OK) return st;
  if (!plan) return fail(TO_E_INVAL, "plan is NULL");
  const PlanEntry pe{plan->col_variant, plan->chunk_mb, plan->us, plan->row_fpb};
  std::string err;
  const int dt = dtype == TO_C64 ? 0 : 1;
  if (!plan_entry_valid(dt, py, px, pe, &err)) return fail(TO_E_INVAL, "%s", err.c_str());
  plan_store(dt, py, px, pe);
  return TO_OK;
}

to_status to_plan_clear(void) {
  plan_clear();
  return TO_OK;
}

to_status to_plan_load(const char* path) {
  if (!path) return fail(TO_E_INVAL, "path is NULL");
  std::string err;
  if (plan_load_file(path, &err) != 0) return fail(TO_E_INVAL, "%s", err.c_str());
  return TO_OK;
}

to_status to_plan_save(const char* path) {
  if (!path) return fail(TO_E_INVAL, "path is NULL");
  std::string err;
  if (plan_save_file(path, &err) != 0) return fail(TO_E_INVAL, "%s", err.c_str());
  return TO_OK;
}

const char* to_last_error(void) { return g_last_error.c_str(); }

to_status to_release(void) {
  std::lock_guard<std::mutex> lk(g_mutex);
  if (g_live_graphs > 0) return fail(TO_E_INVAL, "%d captured call(s) still hold the workspaces", g_live_graphs);
  // release everything even after an error; report the first one
  hipError_t first = hipSuccess;
  auto note = [&](hipError_t e) {
    if (first == hipSuccess && e != hipSuccess) first = e;
  };
  int cur = 0;
  note(hipGetDevice(&cur));
  for (size_t d = 0; d < g_ctx.size(); ++d) {
    DeviceCtx& c = g_ctx[d];
    if (!c.init) continue;
    note(hipSetDevice((int)d));
    note(hipDeviceSynchronize());
    if (c.tw32) note(hipFree(c.tw32));
    if (c.tw64) note(hipFree(c.tw64));
    for (int l = 0; l < kLanes; ++l) {
      Lane& ln = c.lane[l];
      if (ln.scratch) note(hipFree(ln.scratch));
      if (ln.partial) note(hipFree(ln.partial));
      if (ln.tf) note(hipFree(ln.tf));
      if (ln.done) note(hipEventDestroy(ln.done));
      if (l > 0 && ln.stream) note(hipStreamDestroy(ln.stream));
    }
    if (c.fork) note(hipEventDestroy(c.fork));
    if (c.plain) note(hipFree(c.plain));
    if (c.coh) note(hipFree(c.coh));
    if (c.di) note(hipFree(c.di));
    if (c.sep) note(hipFree(c.sep));
    if (c.rs) note(hipFree(c.rs));
    if (c.acc) note(hipFree(c.acc));
    for (auto& b : c.blue) {
      if (b.w) note(hipFree(b.w));
      if (b.Bf) note(hipFree(b.Bf));
    }
    c = DeviceCtx();
  }
  note(hipSetDevice(cur));
  return first == hipSuccess ? TO_OK : hip_fail(first, "to_release");
}

to_status to_transfer_table(const to_job* job, to_dtype dtype, void* table, void* stream) {
  if (!job) return fail(TO_E_INVAL, "job is NULL");
  if (!table) return fail(TO_E_INVAL, "table is NULL");
  to_job j = *job;
  j.batch = 0;  // the field pointers, element and epilogue play no part
  j.el_flags = 0;
  j.epi = TO_EPI_NONE;
  to_status st = validate(j, 0, dtype, MODE_FWD);
  if (st != TO_OK) return st;
  DeviceCtx* c;
  if ((st = get_ctx(&c)) != TO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  j.method = resolved_method(j);
  const bool dbl = dtype == TO_C128;
  hipError_t e;
  if (j.method == TO_DI) {
    if (dbl) {
      LineFft<double> fx, fy;
      if ((st = line_fft<double>(c, j.px, s, &fx)) != TO_OK || (st = line_fft<double>(c, j.py, s, &fy)) != TO_OK)
        return st;
      e = TransferTable<double>::direct_integration((cx<double>*)table, di_params(j), fx, fy, s);
    } else {
      LineFft<float> fx, fy;
      if ((st = line_fft<float>(c, j.px, s, &fx)) != TO_OK || (st = line_fft<float>(c, j.py, s, &fy)) != TO_OK)
        return st;
      e = TransferTable<float>::direct_integration((cx<float>*)table, di_params(j), fx, fy, s);
    }
  } else {
    const TransferParams h = make_transfer(j, false);
    e = dbl ? TransferTable<double>::analytic((cx<double>*)table, j.py, j.px, h, s)
            : TransferTable<float>::analytic((cx<float>*)table, j.py, j.px, h, s);
  }
  return e == hipSuccess ? TO_OK : hip_fail(e, "transfer table");
}

to_status to_resample(const void* src, void* dst, const to_grid* grid_in, const to_grid* grid_out, int64_t batch,
                      int32_t interp, int32_t adjoint, to_dtype dtype, void* stream) {
  if (dtype != TO_C64 && dtype != TO_C128) return fail(TO_E_INVAL, "dtype %d is not TO_C64/TO_C128", (int)dtype);
  if (!grid_in || !grid_out) return fail(TO_E_INVAL, "grid_in or grid_out is NULL");
  if (interp != TO_NEAREST && interp != TO_BILINEAR) return fail(TO_E_INVAL, "unknown interpolation %d", interp);
  if (batch < 0) return fail(TO_E_INVAL, "batch %lld < 0", (long long)batch);
  const to_grid* gs[2] = {grid_in, grid_out};
  for (const to_grid* g : gs) {
    if (g->ny < 1 || g->nx < 1) return fail(TO_E_INVAL, "grid %dx%d must be >= 1", g->ny, g->nx);
    if (!finite_pos(g->dy) || !finite_pos(g->dx)) return fail(TO_E_INVAL, "grid spacing must be finite and > 0");
    if (!std::isfinite(g->y0) || !std::isfinite(g->x0)) return fail(TO_E_INVAL, "grid offset not finite");
  }
  const int64_t pin = (int64_t)grid_in->ny * grid_in->nx, pout = (int64_t)grid_out->ny * grid_out->nx;
  if (batch > 0 && std::max(pin, pout) > (int64_t(1) << 40) / batch)
    return fail(TO_E_UNSUPPORTED, "resampling batch too large");
  if (batch == 0) return TO_OK;
  if (!src || !dst) return fail(TO_E_INVAL, "src or dst is NULL");
  const size_t elt = dtype == TO_C64 ? sizeof(cx<float>) : sizeof(cx<double>);
  const size_t sb = (size_t)batch * (adjoint ? pout : pin) * elt, db = (size_t)batch * (adjoint ? pin : pout) * elt;
  if (overlaps(span(src, sb), span(dst, db))) return fail(TO_E_INVAL, "src and dst overlap");
  auto axis = [](int n_in, double d_in, double o_in, int n_out, double d_out, double o_out) {
    AxisMap m;
    m.n_in = n_in;
    m.n_out = n_out;
    m.half_in = n_in / 2;
    m.half_out = n_out / 2;
    m.ratio = d_out / d_in;
    m.shift = (o_out - o_in) / d_in;
    return m;
  };
  const AxisMap ay = axis(grid_in->ny, grid_in->dy, grid_in->y0, grid_out->ny, grid_out->dy, grid_out->y0);
  const AxisMap ax = axis(grid_in->nx, grid_in->dx, grid_in->x0, grid_out->nx, grid_out->dx, grid_out->x0);
  DeviceCtx* c;
  to_status st = get_ctx(&c);
  if (st != TO_OK) return st;
  if ((st = ensure_area(&c->rs, &c->rs_bytes, resample_table_bytes(ay, ax), "resampling tables")) != TO_OK)
    return st;
  hipStream_t s = (hipStream_t)stream;
  const bool dbl = dtype == TO_C128;
  hipError_t e = timed(adjoint ? "resample_adjoint" : "resample", 0, dbl, s, [&] {
    return dbl ? Resample<double>::run((const cx<double>*)src, (cx<double>*)dst, batch, ay, ax, interp, adjoint != 0,
                                       c->rs, s)
               : Resample<float>::run((const cx<float>*)src, (cx<float>*)dst, batch, ay, ax, interp, adjoint != 0,
                                      c->rs, s);
  });
  return e == hipSuccess ? TO_OK : hip_fail(e, "resample");
}

to_status to_resolve_method(const to_job* job, int32_t* method) {
  if (!job || !method) return fail(TO_E_INVAL, "job or method is NULL");
  to_job j = *job;
  j.batch = 0;
  j.el_flags = 0;
  j.epi = TO_EPI_NONE;
  to_status st = validate(j, 0, TO_C64, MODE_FWD);
  if (st != TO_OK) return st;
  *method = resolved_method(j);
  return TO_OK;
}

// Jones matrices of standard elements (section "Polarization"), embedded in
// 3x3 with the z component passed through; host only.
namespace {
void jones_store(const std::complex<double> (&J)[2][2], double* out) {
  for (int k = 0; k < 18; ++k) out[k] = 0.0;
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      out[2 * (3 * r + c)] = J[r][c].real();
      out[2 * (3 * r + c) + 1] = J[r][c].imag();
    }
  out[2 * 8] = 1.0;
}
}  // namespace

to_status to_jones_linear_polarizer(double theta, double* out) {
  if (!out) return fail(TO_E_INVAL, "out is NULL");
  if (!std::isfinite(theta)) return fail(TO_E_INVAL, "theta must be finite");
  // projector onto the transmission axis (cos theta, sin theta)
  const double c = std::cos(theta), s = std::sin(theta);
  const std::complex<double> J[2][2] = {{c * c, c * s}, {c * s, s * s}};
  jones_store(J, out);
  return TO_OK;
}

to_status to_jones_waveplate(double theta, double retardance, double* out) {
  if (!out) return fail(TO_E_INVAL, "out is NULL");
  if (!std::isfinite(theta) || !std::isfinite(retardance)) return fail(TO_E_INVAL, "angles must be finite");
  // rotate to the plate's axes, delay the slow axis by the retardance,
  // rotate back: R(theta) diag(1, e^{i Gamma}) R(-theta)
  const double c = std::cos(theta), s = std::sin(theta);
  const std::complex<double> e = std::polar(1.0, retardance);
  const std::complex<double> J[2][2] = {{c * c + e * (s * s), (1.0 - e) * (c * s)},
                                        {(1.0 - e) * (c * s), s * s + e * (c * c)}};
  jones_store(J, out);
  return TO_OK;
}

to_status to_jones_compose(const double* first, const double* then, double* out) {
  if (!first || !then || !out) return fail(TO_E_INVAL, "a matrix pointer is NULL");
  std::complex<double> A[3][3], B[3][3], C[3][3];
  for (int k = 0; k < 9; ++k) {
    A[k / 3][k % 3] = {first[2 * k], first[2 * k + 1]};
    B[k / 3][k % 3] = {then[2 * k], then[2 * k + 1]};
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      C[r][c] = 0.0;
      for (int k = 0; k < 3; ++k) C[r][c] += B[r][k] * A[k][c];
    }
  for (int k = 0; k < 9; ++k) {
    out[2 * k] = C[k / 3][k % 3].real();
    out[2 * k + 1] = C[k / 3][k % 3].imag();
  }
  return TO_OK;
}

const char* to_version(void) { return "toprop 0.1.0 gfx950"; }

to_status to_profile_begin(void) {
  std::lock_guard<std::mutex> lk(g_prof_mutex);
  g_prof_recs.clear();
  g_prof_agg.clear();
  g_prof_pool_used = 0;
  g_prof_on = true;
  return TO_OK;
}

to_status to_profile_end(void) {
  std::lock_guard<std::mutex> lk(g_prof_mutex);
  g_prof_on = false;
  g_prof_agg.clear();
  for (const ProfRec& r : g_prof_recs) {
    if (!r.valid) continue;
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, r.a, r.b)) != hipSuccess)
      return hip_fail(e, "hipEventElapsedTime");
    size_t k = 0;
    while (k < g_prof_agg.size() && g_prof_agg[k].name != r.name) ++k;
    if (k == g_prof_agg.size()) g_prof_agg.push_back({r.name, 0, 0.0});
    g_prof_agg[k].launches += 1;
    g_prof_agg[k].ms += ms;
  }
  g_prof_recs.clear();
  g_prof_pool_used = 0;
  return TO_OK;
}

int32_t to_profile_count(void) {
  std::lock_guard<std::mutex> lk(g_prof_mutex);
  return (int32_t)g_prof_agg.size();
}

to_status to_profile_entry(int32_t i, char* name, int32_t name_len, int64_t* launches,
                           double* total_ms) {
  std::lock_guard<std::mutex> lk(g_prof_mutex);
  if (i < 0 || i >= (int32_t)g_prof_agg.size() || !name || name_len < 1 || !launches || !total_ms)
    return fail(TO_E_INVAL, "bad profile entry query");
  snprintf(name, (size_t)name_len, "%s", g_prof_agg[i].name.c_str());
  *launches = g_prof_agg[i].launches;
  *total_ms = g_prof_agg[i].ms;
  return TO_OK;
}


// ---------------------------------------------------------------------------
// Captured calls.
// ---------------------------------------------------------------------------
struct to_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;  // the private stream the call was captured on
};

void graph_free(to_graph g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

to_status to_graph_destroy(to_graph g) {
  if (!g) return fail(TO_E_INVAL, "graph is NULL");
  graph_free(g);
  std::lock_guard<std::mutex> lk(g_mutex);
  if (--g_live_graphs == 0 && !g_retired.empty()) {
    // replays may still be queued: wait for the devices before freeing
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& r : g_retired) {
      (void)hipSetDevice(r.first);
      (void)hipDeviceSynchronize();
      (void)hipFree(r.second);
    }
    g_retired.clear();
    (void)hipSetDevice(cur);
  }
  return TO_OK;
}

to_status to_graph_create(const to_job* jobs, const to_grad* grads, int32_t njobs, to_dtype dtype,
                          void* stream, to_graph* out) {
  if (!out) return fail(TO_E_INVAL, "out is NULL");
  *out = nullptr;
  if (njobs < 1 || !jobs) return fail(TO_E_INVAL, "a captured call needs at least one job");
  auto call = [&](void* s) {
    return grads ? to_propagate_backward(jobs, grads, njobs, dtype, s) : to_propagate(jobs, njobs, dtype, s);
  };
  // the eager call: results, workspaces, tables
  to_status st = call(stream);
  if (st != TO_OK) return st;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  to_graph g = new to_graph_s;
  if ((e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking)) != hipSuccess) {
    delete g;
    return hip_fail(e, "hipStreamCreate");
  }
  if ((e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    graph_free(g);
    return hip_fail(e, "hipStreamBeginCapture");
  }
  st = call(g->stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(g->stream, &graph);
  g->graph = graph;
  if (st != TO_OK) {
    graph_free(g);
    return st;
  }
  if (e != hipSuccess) {
    graph_free(g);
    return hip_fail(e, "hipStreamEndCapture");
  }
  if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess) {
    graph_free(g);
    return hip_fail(e, "hipGraphInstantiate");
  }
  {
    std::lock_guard<std::mutex> lk(g_mutex);
    ++g_live_graphs;
  }
  *out = g;
  return TO_OK;
}

to_status to_graph_launch(to_graph g, void* stream) {
  if (!g || !g->exec) return fail(TO_E_INVAL, "graph is NULL");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return TO_OK;
}

}  // extern "C"

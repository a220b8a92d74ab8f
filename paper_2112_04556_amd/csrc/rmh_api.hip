// C ABI of the adjoint-Laplacian library: argument checks, workspace planning and the
// host drivers (Chebyshev moment recursion, multi-shift CG with reliable updates and
// per-shift refinement, rational combination, kinetic force).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rmh.h"
#include "rmh_host.h"
#include "rmh_internal.h"
#include "rmh_tune.h"

using namespace rmh;

namespace {

thread_local std::string g_err = "no error";

rmh_status fail(rmh_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(RMH_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

#define RMH_TRY(expr)                  \
  do {                                 \
    rmh_status st_ = (expr);           \
    if (st_ != RMH_OK) return st_;     \
  } while (0)

constexpr int64_t kMaxSites = int64_t(1) << 28;

rmh_status make_geom(const int32_t* L, Geom* g) {
  if (!L) return fail(RMH_E_ARG, "lattice extents pointer is NULL");
  int64_t V = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (L[mu] < 2) return fail(RMH_E_SHAPE, "lattice extent L[%d] = %d must be >= 2", mu, L[mu]);
    V *= L[mu];
    if (V > kMaxSites) return fail(RMH_E_SHAPE, "lattice volume exceeds %lld sites", (long long)kMaxSites);
  }
  g->L0 = L[0];
  g->L1 = L[1];
  g->L2 = L[2];
  g->L3 = L[3];
  g->V = (int32_t)V;
  return RMH_OK;
}

size_t dsize(int32_t dtype) { return dtype == RMH_F64 ? 8 : 4; }

rmh_status check_dtype(int32_t dtype) {
  if (dtype != RMH_F64 && dtype != RMH_F32) return fail(RMH_E_ARG, "dtype %d is neither RMH_F64 nor RMH_F32", dtype);
  return RMH_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

rmh_status check_ptr(const void* p, const char* name) {
  if (!p) return fail(RMH_E_ARG, "%s is NULL", name);
  if (((uintptr_t)p) & 255) return fail(RMH_E_ARG, "%s is not 256-byte aligned", name);
  return RMH_OK;
}

// Workspace carving: the same code computes sizes (base == nullptr) and pointers.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t n) {
    const size_t bytes = ((n * sizeof(T) + 255) / 256) * 256;
    T* p = base ? (T*)(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

// Pinned host staging for the drivers' small transfers (coefficient tables, solver state): one
// buffer per calling thread, allocated with hipHostMalloc, grown on demand and freed when the
// thread ends, so the copies skip the runtime's bounce through pageable memory.
struct PinnedStage {
  void* p = nullptr;
  size_t cap = 0;
  ~PinnedStage() {
    if (p) (void)hipHostFree(p);
  }
};
static thread_local PinnedStage t_stage;

static rmh_status pinned(size_t bytes, void** out) {
  if (t_stage.cap < bytes) {
    if (t_stage.p) HIP_TRY(hipHostFree(t_stage.p));   // no copy is in flight: every user waits
    t_stage.p = nullptr;
    t_stage.cap = 0;
    const size_t cap = std::max<size_t>(bytes, (size_t)1 << 16);
    HIP_TRY(hipHostMalloc(&t_stage.p, cap, hipHostMallocDefault));
    t_stage.cap = cap;
  }
  *out = t_stage.p;
  return RMH_OK;
}

// copies host -> device on the stream through the pinned stage and waits
rmh_status h2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return RMH_OK;
  void* st = nullptr;
  RMH_TRY(pinned(bytes, &st));
  memcpy(st, src, bytes);
  HIP_TRY(hipMemcpyAsync(dst, st, bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return RMH_OK;
}
rmh_status d2h(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return RMH_OK;
  void* st = nullptr;
  RMH_TRY(pinned(bytes, &st));
  HIP_TRY(hipMemcpyAsync(st, src, bytes, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  memcpy(dst, st, bytes);
  return RMH_OK;
}

// ------------------------------------------------------------------------------------------
// Static device scratch for the entry point that allocates nothing (rmh_power_spectrum_noalloc).
// Each device holds its own copy of the array at its own address for the life of the process; host
// code must never pass the array's name to a kernel (in host code it is a host-side stand-in), only
// the address hipGetSymbolAddress returns for the current device, kept here per device.  Every call
// on a device shares its array: calls that overlap on one device race.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_addr;

static rmh_status scratch_ptr(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(RMH_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    it = g_scratch_addr.emplace(dev, p).first;
  }
  *out = it->second;
  return RMH_OK;
}

// ------------------------------------------------------------------------------------------
// kernel timing (HIP events around launches of the instrumented classes)

struct ProfRec {
  int cls;
  hipEvent_t e0, e1;
  double bytes, items;
};

struct ProfState {
  std::mutex mu;
  bool on = false;
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> pool;
  int64_t launches[RMH_PROF_N] = {};
  double ms[RMH_PROF_N] = {};
  double bytes[RMH_PROF_N] = {};
  double items[RMH_PROF_N] = {};
};
ProfState g_prof;

hipEvent_t prof_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_flush_locked() {
  for (auto& r : g_prof.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
      g_prof.launches[r.cls] += 1;
      g_prof.ms[r.cls] += ms;
      g_prof.bytes[r.cls] += r.bytes;
      g_prof.items[r.cls] += r.items;
    }
    g_prof.pool.push_back(r.e0);
    g_prof.pool.push_back(r.e1);
  }
  g_prof.pending.clear();
}

// Records an event pair around the enclosed launch when timing is enabled.
struct ProfScope {
  int cls;
  double bytes, items;
  hipStream_t s;
  hipEvent_t e0 = nullptr;
  ProfScope(int c, double b, hipStream_t st, double it = 0.0) : cls(c), bytes(b), items(it), s(st) {
    if (!g_prof.on) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    e0 = prof_event();
    if (e0 && hipEventRecord(e0, s) != hipSuccess) e0 = nullptr;
  }
  ~ProfScope() {
    if (!e0) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    hipEvent_t e1 = prof_event();
    if (e1 && hipEventRecord(e1, s) == hipSuccess) g_prof.pending.push_back({cls, e0, e1, bytes, items});
    if (g_prof.pending.size() > 4096) prof_flush_locked();
  }
};

void prof_add_bytes(int cls, double bytes, double items = 0.0) {
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.bytes[cls] += bytes;
  g_prof.items[cls] += items;
}

// algorithmic bytes of one stencil launch over n fields: links once, x, optional z, optional out
double hop_bytes(const Geom& g, int32_t n, size_t ts, bool z, bool store) {
  // links: the 12 reals of rows 0 and 1 per direction (row 2 is rebuilt in registers)
  return (double)g.V * ts * (48.0 + (double)n * 32.0 * (1.0 + (z ? 1.0 : 0.0) + (store ? 1.0 : 0.0)));
}

HopConfig hop_config(const Geom& g, int32_t dtype, int32_t n_rhs, int32_t purpose) {
  return tune_hop(g, dtype, n_rhs, purpose);
}

// ------------------------------------------------------------------------------------------
// Chebyshev plans

struct ChebPlan {
  void* bufA;
  void* bufB;
  double* partials;
  double* sums;
};

ChebPlan plan_cheb(Carver& c, const Geom& g, int32_t dtype, int32_t n_rhs, int32_t sweeps, bool moments) {
  ChebPlan p{};
  const size_t fb = (size_t)n_rhs * 32 * g.V * dsize(dtype);
  p.bufA = c.take<char>(fb);
  p.bufB = c.take<char>(fb);
  if (moments) {
    const int nblk = hop_max_blocks(g);
    p.partials = c.take<double>((size_t)sweeps * n_rhs * 3 * nblk);
    p.sums = c.take<double>((size_t)sweeps * n_rhs * 3);
  }
  return p;
}

// The filter keeps its recursion vectors in a ring of R slots and folds them into the window
// outputs every R sweeps (and at the end): each output is read and written once per R sweeps
// instead of once per sweep.
struct FilterPlan {
  void* ring;     // [R][n_rhs][4][8][V]
  double* coef;   // [nw][D + 1]
  int32_t R;
};

int32_t filter_ring_slots(int32_t D) { return std::min(kMaxFold, std::max(3, D)); }

FilterPlan plan_filter(Carver& c, const Geom& g, int32_t dtype, int32_t n_rhs, int32_t D, int32_t nw) {
  FilterPlan p{};
  p.R = filter_ring_slots(D);
  p.ring = c.take<char>((size_t)p.R * n_rhs * 32 * g.V * dsize(dtype));
  p.coef = c.take<double>((size_t)std::max(1, nw) * (D + 1));
  return p;
}

// ------------------------------------------------------------------------------------------
// multi-shift CG engine

struct Engine {
  Geom g;
  int32_t n_rhs = 0, n_shift = 0, mode = 0, nslot = 2, nslot32 = 4;   // FP64 and FP32 ring slots
  // seed vectors: direction and its image, FP64 (FP64 phase) and FP32 (FP32 phase)
  double* p64 = nullptr;   // [n_rhs]
  double* Ap64 = nullptr;  // [n_rhs]
  float* p32 = nullptr;
  float* Ap32 = nullptr;
  double* r64 = nullptr;   // [n_rhs] FP64 residual of a reliable update (mixed)
  float* x_lo = nullptr;   // [n_rhs] FP32 increment of the seed's solution since the last reliable update
  double* ring = nullptr;  // [n_rhs][nslot] seed residuals of the FP64 phase
  float* ring32 = nullptr; // [n_rhs][nslot32] seed residuals of the FP32 phase (mixed)
  double* pj = nullptr;    // [n_rhs][n_shift] shift directions at the segment start (n_shift > 1)
  double* coef = nullptr;  // [n_rhs][n_shift][2 + 2 nslot32]
  // scalar state, contiguous so one copy brings it to the host: sc then flags
  double* sc = nullptr;
  int32_t* flags = nullptr;
  size_t state_bytes = 0;
  double* sh = nullptr;
  int32_t* act = nullptr;
  int32_t* act_next = nullptr;
  // parameters, uploaded by one copy per solve
  char* params = nullptr;
  size_t params_bytes = 0;
  double* sigma = nullptr;   // [n_rhs][n_shift]
  double* b_hop = nullptr;   // [n_rhs]  8 + sigma0
  double* b_ru = nullptr;    // [n_rhs]  -(8 + sigma0)
  double* b_true = nullptr;  // [n_rhs][n_shift]  -(8 + sigma_j)
  double* tol_rhs = nullptr; // [n_rhs]
  int32_t* seed = nullptr;   // [n_rhs]
  double* part = nullptr;      // [n_rhs][max(3 nblk_hop, nblk_e)]
  double* part_ru = nullptr;   // [n_rhs][3][nblk_hop]  (mixed precision)
  double* part_true = nullptr; // [n_rhs][n_shift][3][nblk_hop]
  double* sums_true = nullptr; // [n_rhs][n_shift][3]
  int32_t nblk_hop = 0, nblk_e = 0;
};

size_t rup(size_t b) { return ((b + 255) / 256) * 256; }

// Residual ring length for a solver: basis iterations per segment + 1 (single-shift engines
// keep only the current and the next residual).  Default segments: 32 iterations in FP64 engines
// (a solve of up to 32 iterations folds its shifts once), 16 in mixed ones (whose FP64 phase
// ends near there; the open segment then goes on in the FP32 ring).
int32_t ring_slots(int32_t n_shift, int32_t basis, int32_t mode) {
  if (n_shift <= 1) return 2;
  const int32_t m = basis > 0 ? basis : (mode ? 16 : 32);
  return std::min<int32_t>(m, kMaxSlots - 1) + 1;
}

void plan_engine(Carver& c, Engine& e, const Geom& g, int32_t n_rhs, int32_t n_shift, int32_t mode,
                 int32_t basis) {
  e.g = g;
  e.n_rhs = n_rhs;
  e.n_shift = n_shift;
  e.mode = mode;
  e.nslot = ring_slots(n_shift, basis, mode);
  e.nslot32 = std::min<int32_t>(2 * e.nslot, kMaxSlots);
  const int64_t n = field_reals(g);
  const size_t nr = n_rhs, np = (size_t)n_rhs * n_shift;
  e.p64 = c.take<double>(nr * n);
  e.Ap64 = c.take<double>(nr * n);
  if (mode) {
    e.p32 = c.take<float>(nr * n);
    e.Ap32 = c.take<float>(nr * n);
    e.r64 = c.take<double>(nr * n);
    e.x_lo = c.take<float>(nr * n);
  }
  e.ring = c.take<double>(nr * e.nslot * n);
  if (mode) e.ring32 = c.take<float>(nr * e.nslot32 * n);
  if (n_shift > 1) e.pj = c.take<double>(np * n);
  e.coef = c.take<double>(np * (2 + 2 * std::max(e.nslot, e.nslot32)));
  const size_t scb = rup(nr * kScN * 8), flb = rup(nr * kFlN * 4);
  char* st = c.take<char>(scb + flb);
  e.sc = (double*)st;
  e.flags = st ? (int32_t*)(st + scb) : nullptr;
  e.state_bytes = scb + flb;
  e.sh = c.take<double>(np * kShN);
  e.act = c.take<int32_t>(np);
  e.act_next = c.take<int32_t>(np);
  const size_t pb = rup(np * 8) * 2 + rup(nr * 8) * 3 + rup(nr * 4);
  e.params = c.take<char>(pb);
  e.params_bytes = pb;
  if (e.params) {
    char* q = e.params;
    e.sigma = (double*)q;   q += rup(np * 8);
    e.b_true = (double*)q;  q += rup(np * 8);
    e.b_hop = (double*)q;   q += rup(nr * 8);
    e.b_ru = (double*)q;    q += rup(nr * 8);
    e.tol_rhs = (double*)q; q += rup(nr * 8);
    e.seed = (int32_t*)q;
  }
  e.nblk_hop = hop_max_blocks(g);
  e.nblk_e = red_num_blocks(n);
  e.part = c.take<double>(nr * std::max<int64_t>(3 * e.nblk_hop, e.nblk_e));
  if (mode) e.part_ru = c.take<double>(nr * 3 * e.nblk_hop);
  e.part_true = c.take<double>(np * 3 * e.nblk_hop);
  e.sums_true = c.take<double>(np * 3);
}

CgDev cg_view(const Engine& e, int32_t nblk_hop, bool fp32) {
  CgDev d;
  d.n_rhs = e.n_rhs;
  d.n_shift = e.n_shift;
  d.sc = e.sc;
  d.sh = e.sh;
  d.flags = e.flags;
  d.act = e.act;
  d.act_next = e.act_next;
  d.sigma = e.sigma;
  d.seed = e.seed;
  d.part = e.part;
  d.part_ru = e.part_ru;
  d.coef = e.coef;
  d.cslots = std::max(e.nslot, e.nslot32);
  d.nslot = fp32 ? d.cslots : e.nslot;
  d.ring64 = e.ring;
  d.rb64 = (int64_t)e.nslot * field_reals(e.g) * 8;
  d.nslot64 = e.nslot;
  d.ring32 = e.ring32;
  d.rb32 = (int64_t)e.nslot32 * field_reals(e.g) * 4;
  d.nslot32 = e.nslot32;
  d.ring_on = e.n_shift > 1 ? 1 : 0;
  // the seed's solution is updated each iteration where reliable updates read it
  d.seed_explicit = (e.n_shift == 1 || fp32) ? 1 : 0;
  d.nblk_hop = nblk_hop;
  d.nblk_e = e.nblk_e;
  d.nblk_ru = 0;
  return d;
}

int log_level() {
  static int lvl = -1;
  if (lvl < 0) {
    const char* e = getenv("RMH_LOG");
    lvl = e ? atoi(e) : 0;
  }
  return lvl;
}

struct SolveInfo {
  int32_t iters = 0;
  int32_t ru = 0;
  int32_t fp64_iters = 0;  // iterations done in the FP64 phase
  int32_t status = kStOk;
};

// Solve (Delta + sigma[v][j]) x[v][j] = b[v] for all v, j to recursive residual tol_rel[v] * ||b_v||.
// x_hi (FP64, [n_rhs][n_shift]) receives the solutions (zeroed here).
// FP64 engines iterate in FP64 throughout.  Mixed engines iterate in FP64 while the seed residual
// is above switch_rel * ||b|| (switch_rel <= 0: not at all), then in FP32 with FP64 reliable updates.
// Every shift solution is accumulated in FP64: the seed's each iteration, the others at flushes.
rmh_status engine_solve(Engine& e, const double* U64, const float* U32, const double* b, double* x_hi,
                        const std::vector<double>& sigma, const std::vector<double>& tol_rel, int32_t maxiter,
                        double delta, int32_t check_every, double switch_rel, hipStream_t s, SolveInfo* info) {
  const Geom& g = e.g;
  const int64_t n = field_reals(g);
  const int32_t nr = e.n_rhs, ns = e.n_shift;
  const bool mixed = e.mode != 0;
  // parameters: seeds and shift coefficients, one upload
  std::vector<char> hp(e.params_bytes, 0);
  std::vector<int32_t> seed(nr);
  {
    const size_t np = (size_t)nr * ns;
    double* h_sigma = (double*)hp.data();
    double* h_btrue = (double*)(hp.data() + rup(np * 8));
    double* h_bhop = (double*)(hp.data() + 2 * rup(np * 8));
    double* h_bru = h_bhop + rup(nr * 8) / 8;
    double* h_tol = h_bru + rup(nr * 8) / 8;
    int32_t* h_seed = (int32_t*)(h_tol + rup(nr * 8) / 8);
    for (int v = 0; v < nr; ++v) {
      int j0 = 0;
      for (int j = 1; j < ns; ++j)
        if (sigma[(size_t)v * ns + j] < sigma[(size_t)v * ns + j0]) j0 = j;
      seed[v] = j0;
      h_seed[v] = j0;
      h_bhop[v] = 8.0 + sigma[(size_t)v * ns + j0];
      h_bru[v] = -h_bhop[v];
      h_tol[v] = tol_rel[v];
      for (int j = 0; j < ns; ++j) {
        h_sigma[(size_t)v * ns + j] = sigma[(size_t)v * ns + j];
        h_btrue[(size_t)v * ns + j] = -(8.0 + sigma[(size_t)v * ns + j]);
      }
    }
    for (int v = 1; v < nr; ++v)
      if (seed[v] != seed[0]) return fail(RMH_E_ARG, "internal: non-uniform seed shift");
    HIP_TRY(hipMemcpyAsync(e.params, hp.data(), hp.size(), hipMemcpyHostToDevice, s));
  }
  // iterations in each precision, and the FP64 residual of the reliable updates
  const HopConfig c32 = hop_config(g, RMH_F32, nr, RMH_PURPOSE_CG);
  const HopConfig c64 = hop_config(g, RMH_F64, nr, RMH_PURPOSE_CG);
  // The reliable-update stencil is launched every FP32 iteration and usually finds nothing pending
  // (its blocks exit at once); an empty launch costs in proportion to its block count, so where the
  // FP64 residual shape is the hop-split one (four lanes per site) it runs one thread per site
  // instead (16^4, one field, 12 poles: the mixed solve 3 % faster).
  HopConfig cru = hop_config(g, RMH_F64, nr, RMH_PURPOSE_CG64);
  if (cru.order >= 2) {
    cru.form = kFormStream;
    cru.block = 256;
    cru.nv = 4;
    cru.order = 0;
    cru.walk = 0;
    cru.ns = 1;
    cru.tile2 = 1;
  }
  const int32_t nblk_32 = hop_num_blocks(g, c32), nblk_64 = hop_num_blocks(g, c64);
  CgDev cg64 = cg_view(e, nblk_64, false);
  CgDev cg32 = cg_view(e, nblk_32, true);
  cg32.nblk_ru = hop_num_blocks(g, cru);

  bool fp32_phase = mixed && !(switch_rel > 0.0);
  // a seed solution kept outside the ring starts from zero; the flushes write x of the others
  if (ns == 1)
    HIP_TRY(launch_zero(x_hi, (size_t)nr * n * 8, s));
  else if (fp32_phase)
    for (int v = 0; v < nr; ++v) HIP_TRY(launch_zero(x_hi + ((size_t)v * ns + seed[v]) * n, (size_t)n * 8, s));
  if (fp32_phase) HIP_TRY(launch_zero(e.x_lo, (size_t)nr * n * 4, s));
  if (fp32_phase)
    HIP_TRY(launch_cg_start<float>(b, e.ring32, e.p32, nr, cg32.rb32, n, s));
  else
    HIP_TRY(launch_cg_start<double>(b, e.ring, e.p64, nr, cg64.rb64, n, s));
  HIP_TRY(launch_dot<double>(b, b, n, nr, e.part, s));
  HIP_TRY(launch_cg_init(cg64, e.part, e.nblk_e, e.tol_rhs, delta, maxiter, fp32_phase ? 1 : 0, s));

  // FP64 stencil on the seed direction: Ap = (8 + sigma0) p - H p, partial <p, Ap>
  HopArgs<double> h64{};
  h64.g = g;
  h64.U = U64;
  h64.x = e.p64;
  h64.x_mul = 1;
  h64.out = e.Ap64;
  h64.z_div = 1;
  h64.a = -1.0;
  h64.b_rhs = e.b_hop;
  h64.n_rhs = nr;
  h64.run = e.flags + kFlRun;
  h64.run_stride = kFlN;
  h64.store = 1;
  h64.partials = e.part;
  h64.dot_mask = 2;
  // FP32 stencil of the mixed phase
  HopArgs<float> h32{};
  h32.g = g;
  h32.U = U32;
  h32.x = e.p32;
  h32.x_mul = 1;
  h32.out = e.Ap32;
  h32.z_div = 1;
  h32.a = -1.0;
  h32.b_rhs = e.b_hop;
  h32.n_rhs = nr;
  h32.run = e.flags + kFlRun;
  h32.run_stride = kFlN;
  h32.store = 1;
  h32.partials = e.part;
  h32.dot_mask = 2;
  // FP64 true residual of the seed for reliable updates: r64 = b - (Delta + sigma0) x_seed
  HopArgs<double> hr{};
  hr.g = g;
  hr.U = U64;
  hr.x = x_hi;
  hr.x_mul = ns;
  hr.x_add = seed[0];
  hr.out = e.r64;
  hr.z = b;
  hr.z_div = 1;
  hr.a = 1.0;
  hr.b_rhs = e.b_ru;
  hr.c = 1.0;
  hr.n_rhs = nr;
  hr.run = e.flags + kFlNeedRU;
  hr.run_stride = kFlN;
  hr.store = 1;
  hr.partials = e.part_ru;
  hr.dot_mask = 4;

  // shift solutions through the residual ring (more than one shift): flush before a segment
  // would outgrow its ring; a single shift updates its solution each iteration.  The segment
  // open at the switch to FP32 goes on in the FP32 ring (its FP64 entries stay where they are),
  // so the switch folds only the seed's solution, which the FP32 phase keeps explicitly.
  const bool multi = ns > 1;
  const int32_t seg64 = cg64.nslot - 1, seg32 = cg32.nslot - 1;
  if (check_every <= 0) check_every = 8;
  if (multi) check_every = std::min(check_every, std::min(seg64, seg32));
  int32_t since = 0;     // iterations in the open segment
  int32_t k64 = 0;       // FP64 entries of the open FP32-phase segment
  bool first = true;
  auto flush = [&](bool fin) -> rmh_status {
    if (!multi) return RMH_OK;
    const double res = fp32_phase ? k64 * 8.0 + (since + 1 - k64) * 4.0 : (since + 1) * 8.0;
    const double bytes = (double)nr * n * (res + ns * (16.0 + (first ? 0.0 : 8.0) + (fin ? 0.0 : 8.0)));
    ProfScope ps(RMH_PROF_CG_SHIFTS, bytes, s, nr);
    if (fp32_phase)
      HIP_TRY(launch_cg_flush(cg32, x_hi, e.pj, fin ? 1 : 0, first ? 1 : 0, 0, 1, n, s));
    else
      HIP_TRY(launch_cg_flush(cg64, x_hi, e.pj, fin ? 1 : 0, first ? 1 : 0, 0, 0, n, s));
    first = false;
    since = 0;
    k64 = 0;
    return RMH_OK;
  };

  std::vector<char> st(e.state_bytes);
  const double* hsc = (const double*)st.data();
  const int32_t* hfl = (const int32_t*)(st.data() + ((char*)e.flags - (char*)e.sc));
  int32_t it = 0;
  info->fp64_iters = 0;
  // Iterations until the next host check.  From the second check on, the seed's convergence rate
  // so far predicts when its relative residual reaches the next threshold (the switch to FP32, then
  // tol: the seed is the last shift to converge, |zeta_j| <= 1), and the check is placed there, at
  // most check_every iterations away, so the switch is not held back to a fixed grid of checks and
  // fewer launches run past convergence.  Only where the checks fall depends on it; the device
  // decides convergence.
  int32_t chunk = check_every;
  double rel_prev = 1.0;   // the worst running seed's relative residual at it_prev (r_0 = b)
  int32_t it_prev = 0;
  double tol_min = 1.0;
  for (int v = 0; v < nr; ++v) tol_min = std::min(tol_min, tol_rel[v]);
  while (true) {
    if (multi && since + chunk > (fp32_phase ? seg32 : seg64)) RMH_TRY(flush(false));
    for (int i = 0; i < chunk; ++i) {
      if (!fp32_phase) {
        {
          ProfScope ps(RMH_PROF_STENCIL, hop_bytes(g, nr, 8, false, true), s, nr);
          HIP_TRY(launch_hop<double>(h64, c64, s));
        }
        HIP_TRY(launch_cg_alpha(cg64, s));
        {
          ProfScope ps(RMH_PROF_CG_RESIDUAL, (double)nr * n * (3 * 8.0 + (multi ? 0.0 : 24.0)), s, nr);
          HIP_TRY(launch_cg_r_update<double>(cg64, e.Ap64, e.p64, multi ? nullptr : x_hi, nullptr, n, s));
        }
        HIP_TRY(launch_cg_beta(cg64, 0, s));
        {
          ProfScope ps(RMH_PROF_CG_RESIDUAL, (double)nr * n * 3 * 8.0, s, nr);
          HIP_TRY(launch_cg_p_update<double>(cg64, e.p64, nullptr, nullptr, n, s));
        }
      } else {
        {
          ProfScope ps(RMH_PROF_STENCIL, hop_bytes(g, nr, 4, false, true), s, nr);
          HIP_TRY(launch_hop<float>(h32, c32, s));
        }
        HIP_TRY(launch_cg_alpha(cg32, s));
        {
          ProfScope ps(RMH_PROF_CG_RESIDUAL, (double)nr * n * 3 * 4.0, s, nr);
          HIP_TRY(launch_cg_r_update<float>(cg32, e.Ap32, e.p32, nullptr, e.r64, n, s));
        }
        HIP_TRY(launch_cg_beta(cg32, 1, s));
        {
          ProfScope ps(RMH_PROF_CG_RESIDUAL, (double)nr * n * 5 * 4.0, s, nr);
          HIP_TRY(launch_cg_p_update<float>(cg32, e.p32, e.x_lo, x_hi, n, s));
        }
        // reliable update decided by this iteration's beta kernel (blocks of rhs without a
        // pending update exit at once): the p update has folded the seed solution into FP64,
        // now its FP64 residual; the stencil's bytes are added once the update count is known
        {
          ProfScope ps(RMH_PROF_STENCIL, 0.0, s, 0.0);
          HIP_TRY(launch_hop<double>(hr, cru, s));
        }
      }
    }
    it += chunk;
    since += chunk;
    if (!fp32_phase) info->fp64_iters = it;
    RMH_TRY(d2h(st.data(), e.sc, e.state_bytes, s));
    bool running = false, below = true;
    double rel = 0.0;
    for (int v = 0; v < nr; ++v) {
      if (hfl[(size_t)v * kFlN + kFlRun] == 0) continue;
      running = true;
      const double rr = hsc[(size_t)v * kScN + kScRR], bb = hsc[(size_t)v * kScN + kScBnorm2];
      if (!(sqrt(rr) <= switch_rel * sqrt(bb))) below = false;
      if (bb > 0.0) rel = std::max(rel, sqrt(rr / bb));
    }
    if (!running) break;
    if (mixed && !fp32_phase && below) {
      // switch to FP32: the remaining increments are small, so their rounding no longer matters
      if (multi) {
        ProfScope ps(RMH_PROF_CG_SHIFTS, (double)nr * n * ((since + 1) * 8.0 + (first ? 8.0 : 16.0)), s, nr);
        HIP_TRY(launch_cg_flush(cg64, x_hi, e.pj, 0, first ? 1 : 0, 1, 0, n, s));
        k64 = since + 1;
      }
      HIP_TRY(launch_cg_to_f32(cg64, e.p64, e.p32, n, s));
      HIP_TRY(launch_zero(e.x_lo, (size_t)nr * n * 4, s));
      fp32_phase = true;
    }
    chunk = check_every;
    const double target = (mixed && !fp32_phase) ? switch_rel : tol_min;
    if (it > it_prev && rel > target && target > 0.0 && rel < rel_prev) {
      const double k = ceil(log(target / rel) / (log(rel / rel_prev) / (it - it_prev)));
      if (k >= 1.0 && k < (double)check_every) chunk = (int32_t)k;
    }
    rel_prev = rel;
    it_prev = it;
    if (it > maxiter + 2 * check_every) break;  // safety net; the device sets NoConv first
  }
  RMH_TRY(flush(true));
  if (fp32_phase) HIP_TRY(launch_cg_xfold(cg32, e.x_lo, x_hi, 1, n, s));
  RMH_TRY(d2h(st.data(), e.sc, e.state_bytes, s));
  if (log_level() > 0) {
    for (int v = 0; v < nr; ++v)
      fprintf(stderr, "[rmh] engine mode=%d rhs %d/%d shifts=%d sigma0=%.4g iters=%g (fp64 %d) ru=%g status=%d |b|^2=%.4g rr=%.4g tol=%.3g\n",
              e.mode, v, nr, ns, sigma[(size_t)v * ns + seed[v]], hsc[(size_t)v * kScN + kScIters], info->fp64_iters,
              hsc[(size_t)v * kScN + kScRU], hfl[(size_t)v * kFlN + kFlStatus], hsc[(size_t)v * kScN + kScBnorm2],
              hsc[(size_t)v * kScN + kScRR], tol_rel[v]);
  }
  info->iters = 0;
  info->ru = 0;
  info->status = kStOk;
  for (int v = 0; v < nr; ++v) {
    info->iters = std::max(info->iters, (int32_t)hsc[(size_t)v * kScN + kScIters]);
    info->ru += (int32_t)hsc[(size_t)v * kScN + kScRU];
    // the reliable-update stencils that ran (links, x_seed, b and r64 of one field each)
    prof_add_bytes(RMH_PROF_STENCIL, hsc[(size_t)v * kScN + kScRU] * hop_bytes(g, 1, 8, true, true),
                   hsc[(size_t)v * kScN + kScRU]);
    const int32_t stv = hfl[(size_t)v * kFlN + kFlStatus];
    if (stv == kStBreakdown) info->status = kStBreakdown;
    else if (stv == kStNoConv && info->status == kStOk) info->status = kStNoConv;
  }
  return RMH_OK;
}

// FP64 true relative residuals ||b_v - (Delta + sigma_j) x_vj|| / ||b_v|| for all pairs.
rmh_status true_residuals(Engine& e, const double* U64, const double* b, const double* x_hi,
                          const std::vector<double>& bnorm, hipStream_t s, std::vector<double>* res) {
  const Geom& g = e.g;
  const int32_t nr = e.n_rhs, ns = e.n_shift;
  const HopConfig c64 = hop_config(g, RMH_F64, nr * ns, RMH_PURPOSE_CG64);
  const int32_t nblk = hop_num_blocks(g, c64);
  HopArgs<double> h{};
  h.g = g;
  h.U = U64;
  h.x = x_hi;
  h.x_mul = 1;
  h.x_add = 0;
  h.out = nullptr;
  h.z = b;
  h.z_div = ns;
  h.a = 1.0;
  h.b_rhs = e.b_true;
  h.c = 1.0;
  h.n_rhs = nr * ns;
  h.store = 0;
  h.partials = e.part_true;
  h.dot_mask = 4;
  {
    ProfScope ps(RMH_PROF_STENCIL, hop_bytes(g, nr * ns, 8, true, false), s, nr * ns);
    HIP_TRY(launch_hop<double>(h, c64, s));
  }
  // rows: for pair q the <out,out> partials sit at row 3 q + 2
  HIP_TRY(launch_reduce_rows(e.part_true, nblk, nr * ns * 3, e.sums_true, s));
  std::vector<double> sums((size_t)nr * ns * 3);
  RMH_TRY(d2h(sums.data(), e.sums_true, sums.size() * 8, s));
  res->resize((size_t)nr * ns);
  for (int v = 0; v < nr; ++v)
    for (int j = 0; j < ns; ++j) {
      const double rr = sums[((size_t)v * ns + j) * 3 + 2];
      (*res)[(size_t)v * ns + j] = bnorm[v] > 0 ? sqrt(rr) / bnorm[v] : 0.0;
    }
  return RMH_OK;
}

// Refinement buffers for a batch of (rhs, shift) pairs solved as independent single-shift systems.
struct RefinePlan {
  Engine eng;
  double* X;      // [nb] copies of the pairs' solutions
  double* Bsrc;   // [nb] copies of their sources
  double* Res;    // [nb] residual vectors (sources of the correction solve)
  double* E;      // [nb] corrections
  int32_t* idx;   // [nb] pair indices, then [nb] doubles -(8 + sigma) (one upload)
  double* bneg;
  int32_t nb;
};

// pairs refined together (a refinement is rare; its buffers cost some 11 link fields a pair)
int32_t refine_batch(int32_t n_rhs, int32_t n_shift) { return std::max(1, std::min(n_rhs * n_shift, 4)); }

void plan_refine(Carver& c, RefinePlan& rp, const Geom& g, int32_t nb, int32_t mode) {
  const int64_t n = field_reals(g);
  rp.nb = nb;
  rp.X = c.take<double>((size_t)nb * n);
  rp.Bsrc = c.take<double>((size_t)nb * n);
  rp.Res = c.take<double>((size_t)nb * n);
  rp.E = c.take<double>((size_t)nb * n);
  char* q = c.take<char>(rup((size_t)nb * 4) + rup((size_t)nb * 8));
  rp.idx = (int32_t*)q;
  rp.bneg = q ? (double*)(q + rup((size_t)nb * 4)) : nullptr;
  plan_engine(c, rp.eng, g, nb, 1, mode, 0);
}

struct SolvePlan {
  Engine eng;
  RefinePlan ref;
  float* U32 = nullptr;
};

void plan_solve(Carver& c, SolvePlan& sp, const Geom& g, int32_t n_rhs, int32_t n_shift, int32_t mode,
                int32_t basis) {
  plan_engine(c, sp.eng, g, n_rhs, n_shift, mode, basis);
  plan_refine(c, sp.ref, g, refine_batch(n_rhs, n_shift), mode);
  if (mode) sp.U32 = c.take<float>((size_t)72 * g.V);
}

struct SolveResult {
  int32_t iters = 0, ru = 0, refine_iters = 0, refine_rounds = 0, fp64_iters = 0;
  double relres_max = 0.0;
  int32_t status = kStOk;
};

// Full solve of every shift to the FP64 true residual tol: multi-shift CG, then per-shift
// refinement of any pair above tol (batched as independent single-shift systems).
rmh_status solve_all(SolvePlan& sp, const double* U64, const double* b, double* x_hi, const std::vector<double>& sig,
                     const rmh_solver& sv, hipStream_t s, SolveResult* out) {
  Engine& e = sp.eng;
  const Geom& g = e.g;
  const int64_t n = field_reals(g);
  const int32_t nr = e.n_rhs, ns = e.n_shift;
  const int32_t mode = e.mode;
  if ((int64_t)sig.size() != ns) return fail(RMH_E_ARG, "internal: %zu shifts for a %d-shift plan", sig.size(), ns);
  if (mode) HIP_TRY(launch_f64_to_f32(U64, sp.U32, (int64_t)72 * g.V, s));
  std::vector<double> sigma((size_t)nr * ns);
  for (int v = 0; v < nr; ++v)
    for (int j = 0; j < ns; ++j) sigma[(size_t)v * ns + j] = sig[j];
  // the recursive residual is driven below the target so the true residual lands under it; the
  // correction solves of the refinement aim at half of tol whatever the multi-shift target
  const double target = 0.5 * sv.tol;
  const double ms_target = (sv.multishift_target > 0.0 ? sv.multishift_target : 0.5) * sv.tol;
  const double sw = sv.mixed_switch > 0.0 ? sv.mixed_switch : (sv.mixed_switch < 0.0 ? 0.0 : 1e-4);
  std::vector<double> tol_rel(nr, ms_target);
  SolveInfo info;
  RMH_TRY(engine_solve(e, U64, sp.U32, b, x_hi, sigma, tol_rel, sv.maxiter, sv.delta, sv.check_every, sw, s,
                       &info));
  out->iters = info.iters;
  out->ru = info.ru;
  out->fp64_iters = info.fp64_iters;
  out->status = info.status;
  if (info.status == kStBreakdown) return RMH_OK;
  std::vector<double> bnorm(nr);
  {
    std::vector<double> scv((size_t)nr * kScN);
    RMH_TRY(d2h(scv.data(), e.sc, scv.size() * 8, s));
    for (int v = 0; v < nr; ++v) bnorm[v] = sqrt(scv[(size_t)v * kScN + kScBnorm2]);
  }
  std::vector<double> res;
  RMH_TRY(true_residuals(e, U64, b, x_hi, bnorm, s, &res));
  RefinePlan& rp = sp.ref;
  for (int round = 0; round < 4; ++round) {
    if (log_level() > 0)
      for (int q = 0; q < nr * ns; ++q)
        fprintf(stderr, "[rmh] round %d pair %d (rhs %d shift %d sigma %.4g) true relres %.3e\n", round, q, q / ns,
                q % ns, sig[q % ns], res[q]);
    std::vector<int32_t> bad;
    for (int q = 0; q < nr * ns; ++q)
      if (!(res[q] <= sv.tol)) bad.push_back(q);
    if (bad.empty()) break;
    out->refine_rounds = round + 1;
    for (size_t i0 = 0; i0 < bad.size(); i0 += rp.nb) {
      const int32_t nb = (int32_t)std::min<size_t>(rp.nb, bad.size() - i0);
      std::vector<double> rsig(nb), rtol(nb);
      std::vector<char> up(rup((size_t)rp.nb * 4) + rup((size_t)rp.nb * 8), 0);
      int32_t* hidx = (int32_t*)up.data();
      double* hbn = (double*)(up.data() + rup((size_t)rp.nb * 4));
      for (int i = 0; i < nb; ++i) {
        const int q = bad[i0 + i];
        hidx[i] = q;
        rsig[i] = sig[q % ns];
        hbn[i] = -(8.0 + rsig[i]);
        // correction solve target relative to its own source ||r|| = res * ||b||
        rtol[i] = std::min(0.5, target / std::max(res[q], 1e-300));
      }
      HIP_TRY(hipMemcpyAsync(rp.idx, up.data(), up.size(), hipMemcpyHostToDevice, s));
      HIP_TRY(launch_gather_pairs(x_hi, b, rp.idx, ns, rp.X, rp.Bsrc, nb, n, s));
      // residual vectors Res_i = Bsrc_i - (Delta + sigma_i) X_i
      HopArgs<double> h{};
      h.g = g;
      h.U = U64;
      h.x = rp.X;
      h.x_mul = 1;
      h.out = rp.Res;
      h.z = rp.Bsrc;
      h.z_div = 1;
      h.a = 1.0;
      h.b_rhs = rp.bneg;
      h.c = 1.0;
      h.n_rhs = nb;
      h.store = 1;
      {
        ProfScope ps(RMH_PROF_STENCIL, hop_bytes(g, nb, 8, true, true), s, nb);
        HIP_TRY(launch_hop<double>(h, hop_config(g, RMH_F64, nb, RMH_PURPOSE_CG64), s));
      }
      Engine& re = rp.eng;
      re.n_rhs = nb;
      SolveInfo ri;
      // corrections need only a few digits: FP32 from the start when mixed
      RMH_TRY(engine_solve(re, U64, sp.U32, rp.Res, rp.E, rsig, rtol, sv.maxiter, sv.delta, sv.check_every, 0.0,
                           s, &ri));
      out->refine_iters += ri.iters;
      if (ri.status == kStBreakdown) out->status = kStBreakdown;
      HIP_TRY(launch_scatter_add_pairs(x_hi, rp.idx, rp.E, nb, n, s));
    }
    RMH_TRY(true_residuals(e, U64, b, x_hi, bnorm, s, &res));
  }
  out->relres_max = 0.0;
  for (double r : res) out->relres_max = std::max(out->relres_max, r);
  if (!(out->relres_max <= sv.tol) && out->status == kStOk) out->status = kStNoConv;
  return RMH_OK;
}

rmh_status check_rational(const rmh_rational* rat) {
  if (!rat) return fail(RMH_E_ARG, "rational is NULL");
  if (rat->n_poles < 1 || rat->n_poles > 64) return fail(RMH_E_ARG, "n_poles = %d outside [1, 64]", rat->n_poles);
  if (!rat->r || !rat->sigma) return fail(RMH_E_ARG, "rational r or sigma is NULL");
  for (int j = 0; j < rat->n_poles; ++j) {
    if (!(rat->sigma[j] > 0.0) || !isfinite(rat->sigma[j]))
      return fail(RMH_E_POLES, "sigma[%d] = %g must be positive and finite", j, rat->sigma[j]);
    if (!isfinite(rat->r[j])) return fail(RMH_E_POLES, "r[%d] is not finite", j);
  }
  if (!isfinite(rat->c)) return fail(RMH_E_POLES, "c is not finite");
  return RMH_OK;
}

rmh_status check_solver(const rmh_solver* sv) {
  if (!sv) return fail(RMH_E_ARG, "solver is NULL");
  if (!(sv->tol > 0.0) || sv->tol >= 1.0) return fail(RMH_E_ARG, "solver tol = %g must lie in (0, 1)", sv->tol);
  if (sv->maxiter < 1) return fail(RMH_E_ARG, "solver maxiter = %d must be >= 1", sv->maxiter);
  if (sv->mode != 0 && sv->mode != 1) return fail(RMH_E_ARG, "solver mode = %d must be 0 or 1", sv->mode);
  if (sv->mode == 1 && !(sv->delta > 0.0 && sv->delta < 1.0))
    return fail(RMH_E_ARG, "solver delta = %g must lie in (0, 1)", sv->delta);
  if (!(sv->mixed_switch < 1.0) || sv->mixed_switch != sv->mixed_switch)
    return fail(RMH_E_ARG, "solver mixed_switch = %g must be < 1", sv->mixed_switch);
  if (sv->basis < 0 || sv->basis > kMaxSlots - 1)
    return fail(RMH_E_ARG, "solver basis = %d outside [0, %d]", sv->basis, kMaxSlots - 1);
  if (!(sv->multishift_target >= 0.0 && sv->multishift_target <= 1e6) || !(sv->multishift_target * sv->tol < 1.0))
    return fail(RMH_E_ARG, "solver multishift_target = %g must lie in [0, 1e6] with multishift_target * tol < 1",
                sv->multishift_target);
  return RMH_OK;
}

rmh_status status_of(const SolveResult& r, const char* what) {
  if (r.status == kStBreakdown) return fail(RMH_E_BREAKDOWN, "%s: CG breakdown (non-finite or non-positive scalar)", what);
  if (r.status == kStNoConv)
    return fail(RMH_E_NOCONV, "%s: not converged (max true relative residual %g)", what, r.relres_max);
  return RMH_OK;
}

void fill_stats(rmh_stats* st, const SolveResult* rs, int n, double seconds) {
  if (!st) return;
  memset(st, 0, sizeof(*st));
  for (int i = 0; i < n; ++i) {
    st->iters += rs[i].iters;
    st->reliable_updates += rs[i].ru;
    st->refine_iters += rs[i].refine_iters;
    st->refine_rounds += rs[i].refine_rounds;
    st->fp64_iters += rs[i].fp64_iters;
    st->true_relres_max = std::max(st->true_relres_max, rs[i].relres_max);
  }
  st->seconds = seconds;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct RationalPlan {
  SolvePlan sp;
  double* X = nullptr;     // x_j of the first solve (if not caller-provided)
  double* Z = nullptr;     // z_j of the second solve
  double* Y = nullptr;     // combined vector (if not caller-provided)
  double* coef = nullptr;  // c, r_0.. (device)
  double* partK = nullptr; // partials for K
  double* sumsK = nullptr;
};

void plan_rational(Carver& c, RationalPlan& rp, const Geom& g, int32_t n_rhs, int32_t n_poles, int32_t mode,
                   int32_t basis,
                   int32_t op) {
  const int64_t n = field_reals(g);
  plan_solve(c, rp.sp, g, n_rhs, n_poles, mode, basis);
  rp.X = c.take<double>((size_t)n_rhs * n_poles * n);
  if (op == RMH_OP_RATIONAL_APPLY_BWD || op == RMH_OP_KINETIC_FORCE)
    rp.Z = c.take<double>((size_t)n_rhs * n_poles * n);
  if (op != RMH_OP_RATIONAL_APPLY) rp.Y = c.take<double>((size_t)n_rhs * n);
  rp.coef = c.take<double>(n_poles + 1);
  rp.partK = c.take<double>((size_t)n_rhs * red_num_blocks(n));
  rp.sumsK = c.take<double>(n_rhs);
}

// workspace of one implicit leapfrog step (one momentum field)
struct LeapfrogPlan {
  RationalPlan rp;       // solves of the kinetic term: X, Z, Y, coefficients
  double* Fg = nullptr;  // gauge force
  double* dK = nullptr;  // dK/d omega
  double* Ph = nullptr;  // half-step momentum
  double* Pi0 = nullptr; // Pi(U, P_h)
  double* PiA = nullptr; // Pi(U', P_h), newest
  double* PiB = nullptr; // Pi(U', P_h), previous
  double* part = nullptr;  // [2][red_num_blocks] partials of the fixed-point norms
  double* sums = nullptr;  // [2]
};

void plan_leapfrog(Carver& c, LeapfrogPlan& lp, const Geom& g, int32_t n_poles, int32_t mode, int32_t basis) {
  const int64_t n = field_reals(g);
  plan_rational(c, lp.rp, g, 1, n_poles, mode, basis, RMH_OP_KINETIC_FORCE);
  lp.Fg = c.take<double>(n);
  lp.dK = c.take<double>(n);
  lp.Ph = c.take<double>(n);
  lp.Pi0 = c.take<double>(n);
  lp.PiA = c.take<double>(n);
  lp.PiB = c.take<double>(n);
  lp.part = c.take<double>(2 * (size_t)red_num_blocks(n));
  lp.sums = c.take<double>(2);
}

template <typename T>
rmh_status power_spectrum_t(const Geom& g, const T* U, const T* F, int32_t n_rhs, int32_t D,
                                   const ChebPlan& cp, std::vector<double>* sums_h, bool direct_copy, hipStream_t s) {
  const int32_t K = std::max(1, (D + 1) / 2);
  const HopConfig cfg = hop_config(g, sizeof(T) == 8 ? RMH_F64 : RMH_F32, n_rhs, RMH_PURPOSE_MOMENTS);
  const int32_t nblk = hop_num_blocks(g, cfg);
  T* A = (T*)cp.bufA;
  T* B = (T*)cp.bufB;
  const T* cur = F;
  const T* prev = nullptr;
  for (int32_t k = 0; k < K; ++k) {
    HopArgs<T> h{};
    h.g = g;
    h.U = U;
    h.x_mul = 1;
    h.z_div = 1;
    h.n_rhs = n_rhs;
    h.store = (k + 1 < K) ? 1 : 0;   // the last sweep only needs its dot products
    h.partials = cp.partials + (size_t)k * n_rhs * 3 * nblk;
    h.dot_mask = 7;
    h.x = cur;
    T* out;
    if (k == 0) {
      out = A;              // t1 = A t0 = -H t0 / 8
      h.a = -0.125;
      h.b = 0.0;
    } else {
      out = (k & 1) ? B : A;  // t_{k+1} = 2 A t_k - t_{k-1} = -H t_k / 4 - t_{k-1}, over t_{k-1}
      h.a = -0.25;
      h.b = 0.0;
      h.c = -1.0;
      h.z = prev;
    }
    h.out = out;
    {
      ProfScope ps(RMH_PROF_STENCIL, hop_bytes(g, n_rhs, sizeof(T), k > 0, h.store != 0), s, n_rhs);
      HIP_TRY(launch_hop<T>(h, cfg, s));
    }
    prev = cur;
    cur = out;
  }
  HIP_TRY(launch_reduce_rows(cp.partials, nblk, K * n_rhs * 3, cp.sums, s));
  sums_h->resize((size_t)K * n_rhs * 3);
  if (direct_copy) {
    HIP_TRY(hipMemcpyAsync(sums_h->data(), cp.sums, sums_h->size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  } else {
    RMH_TRY(d2h(sums_h->data(), cp.sums, sums_h->size() * 8, s));
  }
  return RMH_OK;
}

template <typename T>
rmh_status cheb_filter_t(const Geom& g, const T* U, const T* x, int32_t n_rhs, int32_t D, int32_t nw,
                         const std::vector<double>& coef, const FilterPlan& fp, T* y, hipStream_t s) {
  const HopConfig cfg = hop_config(g, sizeof(T) == 8 ? RMH_F64 : RMH_F32, n_rhs, RMH_PURPOSE_FILTER);
  const int64_t n = (int64_t)n_rhs * 32 * g.V;
  RMH_TRY(h2d(fp.coef, coef.data(), coef.size() * sizeof(double), s));
  T* ring = (T*)fp.ring;
  const int32_t R = fp.R;
  const T* cur = x;       // t_k
  const T* prev = nullptr;  // t_{k-1}
  int32_t pending = 1;    // first t_k not yet folded
  for (int32_t k = 0; k < D; ++k) {
    // t_{k+1} into slot (k+1) % R: that slot held t_{k+1-R}, folded already, and R >= 3 keeps it
    // apart from t_k and t_{k-1}
    T* out = ring + (int64_t)((k + 1) % R) * n;
    HopArgs<T> h{};
    h.g = g;
    h.U = U;
    h.x_mul = 1;
    h.z_div = 1;
    h.n_rhs = n_rhs;
    h.store = 1;
    h.x = cur;
    h.out = out;
    if (k == 0) {
      h.a = -0.125;      // t_1 = A t_0 = -H t_0 / 8
    } else {
      h.a = -0.25;       // t_{k+1} = 2 A t_k - t_{k-1} = -H t_k / 4 - t_{k-1}
      h.c = -1.0;
      h.z = prev;
    }
    {
      ProfScope ps(RMH_PROF_STENCIL, hop_bytes(g, n_rhs, sizeof(T), k > 0, true), s, n_rhs);
      HIP_TRY(launch_hop<T>(h, cfg, s));
    }
    prev = cur;
    cur = out;
    const int32_t cnt = k + 2 - pending;   // t_pending .. t_{k+1}
    if (cnt == R || k + 1 == D) {
      const int32_t first = pending == 1 ? 1 : 0;
      // reads cnt vectors (and x on the first fold), reads (after the first) and writes nw outputs
      const double fb = (double)n * sizeof(T);
      ProfScope ps(RMH_PROF_CHEB_FOLD, fb * (cnt + first + (double)nw * (first ? 1.0 : 2.0)), s, n_rhs);
      HIP_TRY(launch_cheb_fold<T>(x, ring, R, pending, cnt, first, fp.coef, D, nw, y, n, s));
      pending = k + 2;
    }
  }
  return RMH_OK;
}

// Reverse sweep of the Chebyshev recursion (FP64).  For L = sum_v sum_k <G_k[v], T_k(A) x[v]> with
// A = Delta/8 - 1 and G_k[v] = sum_y c[v][y][k] Y[y][v], the adjoint vectors of t_k = T_k(A) x obey
//   tb_k = G_k + 2A tb_{k+1} - tb_{k+2}  (tb_{D+1} = tb_{D+2} = 0),
// and, since t_1 = A t_0 and t_k = 2A t_{k-1} - t_{k-2},
//   dL/d omega = (1/8) <tb_1, dDelta t_0> + (1/4) sum_{k=2..D} <tb_k, dDelta t_{k-1}>,
//   dL/dx      = tb_0 = G_0 + A tb_1 - tb_2  (through the recursion only).
// t_D, t_{D-1} come from a forward sweep; the reverse sweep then runs the recursion backwards,
// t_{k-2} = 2A t_{k-1} - t_k, so only two t and two tb vectors are held.  2A = -H/4.
// tb_j lives in B[(j-1) % 2] and t_j (j >= 1) in T[(j-1) % 2], and B[i] is followed by T[i] in
// memory: the two recursion steps of a reverse step (tb_k from tb_{k+1}, tb_{k+2} and t_{k-2} from
// t_{k-1}, t_k) then read one 2 n_rhs-field batch and write another, and go out as one launch.
struct ChebBwdPlan {
  double* T[2];
  double* B[2];
  double* coef;   // [n_rhs][n_y][D+1], then [n_rhs][n_y] scaled k = 0 coefficients
};

ChebBwdPlan plan_cheb_bwd(Carver& c, const Geom& g, int32_t n_rhs, int32_t n_y, int32_t D) {
  ChebBwdPlan p{};
  const size_t fr = (size_t)n_rhs * 32 * g.V;
  for (int i = 0; i < 2; ++i) {
    p.B[i] = c.take<double>(2 * fr);
    p.T[i] = p.B[i] + fr;
  }
  p.coef = c.take<double>((size_t)n_rhs * n_y * (D + 2));
  return p;
}

rmh_status cheb_bwd(const Geom& g, const double* U, const double* x, int32_t n_rhs, int32_t D, const double* Y,
                    int32_t n_y, const std::vector<double>& coef_h, const ChebBwdPlan& p, double* grad_x,
                    double xscale, double* grad_omega, int32_t per_rhs, hipStream_t s) {
  const int64_t n = field_reals(g);
  const int32_t nk = D + 1;
  {
    std::vector<double> up(coef_h);
    up.resize((size_t)n_rhs * n_y * (D + 2));
    for (size_t i = 0; i < (size_t)n_rhs * n_y; ++i) up[(size_t)n_rhs * n_y * nk + i] = xscale * coef_h[i * nk];
    RMH_TRY(h2d(p.coef, up.data(), up.size() * 8, s));
  }
  const double* coef_x = p.coef + (size_t)n_rhs * n_y * nk;
  const HopConfig cfg = hop_config(g, RMH_F64, n_rhs, RMH_PURPOSE_CHEB_BWD);
  const HopConfig cfg2 = hop_config(g, RMH_F64, 2 * n_rhs, RMH_PURPOSE_CHEB_BWD);
  // nf fields (n_rhs, or 2 n_rhs for a B[i]-T[i] pair)
  auto hopn = [&](const double* in, const double* z, double* out, double a, double c, int32_t nf) -> rmh_status {
    HopArgs<double> h{};
    h.g = g;
    h.U = U;
    h.x = in;
    h.x_mul = 1;
    h.z = z;
    h.z_div = 1;
    h.out = out;
    h.a = a;
    h.c = c;
    h.n_rhs = nf;
    h.store = 1;
    ProfScope ps(RMH_PROF_STENCIL, hop_bytes(g, nf, 8, z != nullptr, true), s, nf);
    HIP_TRY(launch_hop<double>(h, nf == n_rhs ? cfg : cfg2, s));
    return RMH_OK;
  };
  auto hop = [&](const double* in, const double* z, double* out, double a, double c) -> rmh_status {
    return hopn(in, z, out, a, c, n_rhs);
  };
  const int64_t fr = n * n_rhs;
  // forward: prv = t_{D-1}, cur = t_D
  const double* prv = x;
  double* cur = p.T[0];
  RMH_TRY(hop(x, nullptr, cur, -0.125, 0.0));
  for (int32_t k = 2; k <= D; ++k) {
    double* out = (k == 2) ? p.T[1] : (double*)prv;   // t_{k-2}'s buffer (x itself is never written)
    RMH_TRY(hop(cur, prv, out, -0.25, -1.0));
    prv = cur;
    cur = out;
  }
  // reverse
  double* nb = p.B[D % 2];         // tb_{k+1}
  double* nb2 = p.B[(D - 1) % 2];  // tb_{k+2}
  HIP_TRY(launch_zero(nb, (size_t)n * n_rhs * 8, s));
  HIP_TRY(launch_zero(nb2, (size_t)n * n_rhs * 8, s));
  for (int32_t k = D; k >= 1; --k) {
    // tb_k into tb_{k+2}'s buffer (for k < D), t_{k-2} = 2A t_{k-1} - t_k into t_k's buffer (for
    // k >= 3; t_{k-1} stays for the link term below): one launch over the pairs B[i]-T[i] when both
    // run (tb_{D+1} is the zeroed buffer, so its z term adds nothing)
    const bool tb_hop = k < D, t_hop = k >= 3;
    if (tb_hop && t_hop) {
      if (prv != nb + fr || cur != nb2 + fr) return fail(RMH_E_HOST, "Chebyshev backward: buffer pairing broken");
      RMH_TRY(hopn(nb, nb2, nb2, -0.25, -1.0, 2 * n_rhs));
    } else if (tb_hop) {
      RMH_TRY(hop(nb, k + 1 < D ? nb2 : nullptr, nb2, -0.25, k + 1 < D ? -1.0 : 0.0));
    } else if (t_hop) {
      RMH_TRY(hop(prv, cur, cur, -0.25, -1.0));
    }
    HIP_TRY(launch_cheb_source(nb2, Y, p.coef, n_rhs, n_y, nk, k, n, s));
    std::swap(nb, nb2);   // nb = tb_k, nb2 = tb_{k+1}
    if (grad_omega) {
      ForceArgs fa{};
      fa.g = g;
      fa.U = U;
      fa.A = nb;
      fa.B = prv;     // t_{k-1}
      fa.n_rhs = n_rhs;
      fa.n_pair = 1;
      fa.w[0] = (k == 1) ? 0.125 : 0.25;
      fa.grad = grad_omega;
      fa.per_rhs = per_rhs ? 1 : 0;
      fa.accumulate = (k == D) ? 0 : 1;
      const double fbytes = (double)g.V * 8.0 * (48.0 + 64.0 * n_rhs + 32.0 * (per_rhs ? n_rhs : 1) * (k == D ? 1.0 : 2.0));
      ProfScope ps(RMH_PROF_FORCE, fbytes, s, n_rhs);
      HIP_TRY(launch_force(fa, s));
    }
    if (k >= 3) {
      const double* t_km2 = cur;
      cur = (double*)prv;
      prv = t_km2;
    } else if (k == 2) {
      cur = (double*)prv;   // t_0 is x itself
      prv = x;
    }
  }
  if (grad_x) {
    // tb_0 = G_0 + A tb_1 - tb_2, scaled by xscale (nb = tb_1, nb2 = tb_2, zero when D = 1)
    RMH_TRY(hop(nb, D >= 2 ? nb2 : nullptr, grad_x, -0.125 * xscale, D >= 2 ? -xscale : 0.0));
    HIP_TRY(launch_cheb_source(grad_x, Y, coef_x, n_rhs, n_y, 1, 0, n, s));
  }
  return RMH_OK;
}

}  // namespace

// =============================================================================================
// One timing unit of the autotuner: the two stencil epilogues the drivers use, the plain
// y = (8 - H) x of the CG and the Chebyshev recursion step y = -H x / 4 - z with z = y (the sweeps
// write t_{k+1} over t_{k-1}), so the pick fits the solves and the spectra alike.
// partials/dot_mask (optional): the per-block FP64 dot products the drivers of a purpose fuse into
// the same launch (the CG's <p, Ap>, the moments' three), so the unit runs the kernel they run.
template <typename T>
static hipError_t tune_unit(const Geom& g, const T* U, const T* x, T* y, int32_t n_rhs, const HopConfig& cfg,
                            int32_t kind, double* partials, int32_t dot_mask, hipStream_t s) {
  HopArgs<T> h{};
  h.g = g;
  h.U = U;
  h.x = x;
  h.x_mul = 1;
  h.out = y;
  h.z_div = 1;
  h.n_rhs = n_rhs;
  h.store = 1;
  h.partials = partials;
  h.dot_mask = partials ? dot_mask : 0;
  if (kind & 1) {   // the plain application y = (8 - H) x
    h.a = -1.0;
    h.b = 8.0;
    hipError_t e = launch_hop<T>(h, cfg, s);
    if (e != hipSuccess) return e;
  }
  if (kind & 2) {   // the recursion step y = -H x / 4 - y, written over its z input as the sweeps do
    h.a = -0.25;
    h.b = 0.0;
    h.c = -1.0;
    h.z = y;
    return launch_hop<T>(h, cfg, s);
  }
  return hipSuccess;
}

// degree and window count, checked before any host buffer is sized by them
static rmh_status check_cheb_dims(const rmh_cheb* cheb, int32_t min_degree, int32_t max_windows) {
  if (!cheb) return fail(RMH_E_ARG, "cheb is NULL");
  if (cheb->degree < min_degree || cheb->degree > kMaxChebDegree)
    return fail(RMH_E_ARG, "degree = %d must be in [%d, %d]", cheb->degree, min_degree, kMaxChebDegree);
  if (cheb->n_windows < 1 || cheb->n_windows > max_windows)
    return fail(RMH_E_ARG, "n_windows = %d must be in [1, %d]", cheb->n_windows, max_windows);
  return RMH_OK;
}

// The power spectrum on a given workspace.  static_ws: the workspace is the library's static
// scratch (ws == nullptr here; it is looked up once the call is known to fit in it), and nothing is
// allocated: the sums come back by a plain copy into host memory instead of the pinned stage.
static rmh_status power_spectrum_impl(const int32_t L[4], const void* U, int32_t dtype, const void* F,
                                      int32_t n_rhs, const rmh_cheb* cheb, double* moments, double* power,
                                      void* ws, size_t ws_bytes, bool static_ws, rmh_stream stream) {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_dtype(dtype));
  RMH_TRY(check_cheb_dims(cheb, 1, kMaxSpectrumWindows));
  if (n_rhs < 0) return fail(RMH_E_ARG, "n_rhs < 0");
  const int32_t D = cheb->degree, nw = cheb->n_windows;
  std::vector<double> coef((size_t)nw * (D + 1));
  RMH_TRY(rmh_cheb_coefficients(cheb, coef.data()));
  if (n_rhs == 0) return RMH_OK;
  RMH_TRY(check_ptr(U, "U"));
  RMH_TRY(check_ptr(F, "F"));
  const int32_t K = std::max(1, (D + 1) / 2);
  if (static_ws) {
    Carver need(nullptr);
    plan_cheb(need, g, dtype, n_rhs, K, true);
    if (need.off > kScratchBytes)
      return fail(RMH_E_WORKSPACE, "the call needs %zu bytes of scratch, more than the %zu of the static scratch",
                  need.off, kScratchBytes);
    RMH_TRY(scratch_ptr(&ws));
    ws_bytes = kScratchBytes;
  }
  RMH_TRY(check_ptr(ws, "ws"));
  Carver c(ws);
  ChebPlan cp = plan_cheb(c, g, dtype, n_rhs, K, true);
  if (c.off > ws_bytes) return fail(RMH_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, c.off);
  const size_t fb = (size_t)n_rhs * 32 * g.V * dsize(dtype);
  if (overlap(ws, c.off, F, fb) || overlap(ws, c.off, U, (size_t)72 * g.V * dsize(dtype)))
    return fail(RMH_E_ARG, "workspace overlaps an input");
  std::vector<double> sums;
  hipStream_t s = (hipStream_t)stream;
  if (dtype == RMH_F64)
    RMH_TRY(power_spectrum_t<double>(g, (const double*)U, (const double*)F, n_rhs, D, cp, &sums, static_ws, s));
  else
    RMH_TRY(power_spectrum_t<float>(g, (const float*)U, (const float*)F, n_rhs, D, cp, &sums, static_ws, s));
  // moments from the doubling identities
  std::vector<double> mu((size_t)n_rhs * (2 * K + 1));
  for (int32_t n = 0; n < n_rhs; ++n) {
    double* m = mu.data() + (size_t)n * (2 * K + 1);
    auto S = [&](int k, int q) { return sums[((size_t)k * n_rhs + n) * 3 + q]; };
    m[0] = S(0, 0);
    m[1] = S(0, 1);
    m[2] = 2.0 * S(0, 2) - m[0];
    for (int32_t k = 1; k < K; ++k) {
      m[2 * k + 1] = 2.0 * S(k, 1) - m[1];
      m[2 * k + 2] = 2.0 * S(k, 2) - m[0];
    }
  }
  for (int32_t n = 0; n < n_rhs; ++n) {
    const double* m = mu.data() + (size_t)n * (2 * K + 1);
    if (moments)
      for (int32_t k = 0; k <= D; ++k) moments[(size_t)n * (D + 1) + k] = m[k];
    if (power)
      for (int32_t w = 0; w < nw; ++w) {
        double acc = 0.0;
        for (int32_t k = 0; k <= D; ++k) acc += coef[(size_t)w * (D + 1) + k] * m[k];
        power[(size_t)n * nw + w] = acc;
      }
  }
  return RMH_OK;
}

extern "C" {

const char* rmh_last_error(void) { return g_err.c_str(); }

// the autotuner's per-block dot-product partials: n_rhs x 3 rows of the largest block count
static double* plan_autotune(Carver& c, const Geom& g, int32_t n_rhs) {
  return c.take<double>((size_t)std::max(n_rhs, 1) * 3 * hop_max_blocks(g));
}

int32_t rmh_version(void) { return 101; }

size_t rmh_workspace_bytes(int32_t op, const int32_t L[4], int32_t dtype, int32_t n_rhs, int32_t aux,
                           int32_t degree, int32_t mode) try {
  Geom g;
  if (make_geom(L, &g) != RMH_OK) return 0;
  if (check_dtype(dtype) != RMH_OK) return 0;
  if (n_rhs < 0) {
    fail(RMH_E_ARG, "n_rhs < 0");
    return 0;
  }
  Carver c(nullptr);
  switch (op) {
    case RMH_OP_LAPLACIAN:
    case RMH_OP_LAPLACIAN_BWD:
      c.take<char>(256);
      break;
    case RMH_OP_POWER_SPECTRUM:
      plan_cheb(c, g, dtype, n_rhs, std::max(1, (degree + 1) / 2), true);
      break;
    case RMH_OP_CHEB_FILTER:
      plan_filter(c, g, dtype, n_rhs, std::max(1, degree), std::min(std::max(aux, 1), kMaxFilterWindows));
      break;
    case RMH_OP_CHEB_FILTER_BWD:
      plan_cheb_bwd(c, g, n_rhs, std::max(1, aux), std::max(1, degree));
      break;
    case RMH_OP_POWER_SPECTRUM_BWD:
      plan_cheb_bwd(c, g, n_rhs, 1, std::max(1, degree));
      break;
    case RMH_OP_GAUGE_FORCE:
      c.take<double>(gauge_force_blocks(g));   // the same carve as rmh_wilson_gauge_force
      c.take<double>(1);
      break;
    case RMH_OP_RATIONAL_APPLY:
    case RMH_OP_RATIONAL_APPLY_BWD:
    case RMH_OP_KINETIC_FORCE:
    case RMH_OP_HEATBATH: {
      if (aux < 1) {
        fail(RMH_E_ARG, "n_poles < 1");
        return 0;
      }
      RationalPlan rp;
      plan_rational(c, rp, g, n_rhs, aux, mode ? 1 : 0, degree, op);
      break;
    }
    case RMH_OP_LEAPFROG: {
      if (aux < 1) {
        fail(RMH_E_ARG, "n_poles < 1");
        return 0;
      }
      LeapfrogPlan lp;
      plan_leapfrog(c, lp, g, aux, mode ? 1 : 0, degree);
      break;
    }
    case RMH_OP_AUTOTUNE:
      plan_autotune(c, g, n_rhs);
      break;
    default:
      fail(RMH_E_ARG, "unknown op %d", op);
      return 0;
  }
  return c.off;
} catch (...) {   // no C++ exception crosses the C ABI
  return 0;
}

rmh_status rmh_pack_links(const int32_t L[4], const double* U_aos, void* U_soa, int32_t dtype, rmh_stream stream) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_dtype(dtype));
  RMH_TRY(check_ptr(U_aos, "U_aos"));
  RMH_TRY(check_ptr(U_soa, "U_soa"));
  if (overlap(U_aos, (size_t)72 * g.V * 8, U_soa, (size_t)72 * g.V * dsize(dtype)))
    return fail(RMH_E_ARG, "U_soa overlaps U_aos");
  HIP_TRY(launch_pack_links(g, U_aos, U_soa, dtype, (hipStream_t)stream));
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_unpack_links(const int32_t L[4], const double* U_soa, double* U_aos, rmh_stream stream) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_ptr(U_aos, "U_aos"));
  RMH_TRY(check_ptr(U_soa, "U_soa"));
  if (overlap(U_aos, (size_t)72 * g.V * 8, U_soa, (size_t)72 * g.V * 8)) return fail(RMH_E_ARG, "U_aos overlaps U_soa");
  HIP_TRY(launch_unpack_links(g, U_soa, U_aos, (hipStream_t)stream));
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_pack_fields(const int32_t L[4], int32_t n, const double* F_aos, void* F_soa, int32_t dtype,
                           rmh_stream stream) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_dtype(dtype));
  if (n < 0) return fail(RMH_E_ARG, "n < 0");
  if (n == 0) return RMH_OK;
  RMH_TRY(check_ptr(F_aos, "F_aos"));
  RMH_TRY(check_ptr(F_soa, "F_soa"));
  if (overlap(F_aos, (size_t)n * 32 * g.V * 8, F_soa, (size_t)n * 32 * g.V * dsize(dtype)))
    return fail(RMH_E_ARG, "F_soa overlaps F_aos");
  HIP_TRY(launch_fields_aos_to_soa(g, n, F_aos, F_soa, dtype, (hipStream_t)stream));
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_unpack_fields(const int32_t L[4], int32_t n, const void* F_soa, int32_t dtype, double* F_aos,
                             rmh_stream stream) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_dtype(dtype));
  if (n < 0) return fail(RMH_E_ARG, "n < 0");
  if (n == 0) return RMH_OK;
  RMH_TRY(check_ptr(F_aos, "F_aos"));
  RMH_TRY(check_ptr(F_soa, "F_soa"));
  if (overlap(F_aos, (size_t)n * 32 * g.V * 8, F_soa, (size_t)n * 32 * g.V * dsize(dtype)))
    return fail(RMH_E_ARG, "F_aos overlaps F_soa");
  HIP_TRY(launch_fields_soa_to_aos(g, n, F_soa, dtype, F_aos, (hipStream_t)stream));
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_convert_f64_f32(const double* in, float* out, int64_t n, rmh_stream stream) try {
  if (n < 0) return fail(RMH_E_ARG, "n < 0");
  if (n == 0) return RMH_OK;
  RMH_TRY(check_ptr(in, "in"));
  RMH_TRY(check_ptr(out, "out"));
  if (overlap(in, n * 8, out, n * 4)) return fail(RMH_E_ARG, "out overlaps in");
  HIP_TRY(launch_f64_to_f32(in, out, n, (hipStream_t)stream));
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_laplacian_apply(const int32_t L[4], const void* U, int32_t dtype, const void* x, void* y,
                               int32_t n_rhs, double shift, rmh_stream stream) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_dtype(dtype));
  if (n_rhs < 0) return fail(RMH_E_ARG, "n_rhs < 0");
  if (!isfinite(shift)) return fail(RMH_E_ARG, "shift is not finite");
  if (n_rhs == 0) return RMH_OK;
  RMH_TRY(check_ptr(U, "U"));
  RMH_TRY(check_ptr(x, "x"));
  RMH_TRY(check_ptr(y, "y"));
  const size_t fb = (size_t)n_rhs * 32 * g.V * dsize(dtype), ub = (size_t)72 * g.V * dsize(dtype);
  if (overlap(x, fb, y, fb) || overlap(U, ub, y, fb)) return fail(RMH_E_ARG, "y overlaps x or U");
  const HopConfig cfg = hop_config(g, dtype, n_rhs, RMH_PURPOSE_APPLY);
  if (dtype == RMH_F64) {
    HopArgs<double> h{};
    h.g = g;
    h.U = (const double*)U;
    h.x = (const double*)x;
    h.x_mul = 1;
    h.out = (double*)y;
    h.z_div = 1;
    h.a = -1.0;
    h.b = 8.0 + shift;
    h.n_rhs = n_rhs;
    h.store = 1;
    ProfScope ps(RMH_PROF_STENCIL, hop_bytes(g, n_rhs, 8, false, true), (hipStream_t)stream, n_rhs);
    HIP_TRY(launch_hop<double>(h, cfg, (hipStream_t)stream));
  } else {
    HopArgs<float> h{};
    h.g = g;
    h.U = (const float*)U;
    h.x = (const float*)x;
    h.x_mul = 1;
    h.out = (float*)y;
    h.z_div = 1;
    h.a = -1.0;
    h.b = 8.0 + shift;
    h.n_rhs = n_rhs;
    h.store = 1;
    ProfScope ps(RMH_PROF_STENCIL, hop_bytes(g, n_rhs, 4, false, true), (hipStream_t)stream, n_rhs);
    HIP_TRY(launch_hop<float>(h, cfg, (hipStream_t)stream));
  }
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_laplacian_apply_bwd(const int32_t L[4], const void* U, int32_t dtype, const void* x, const void* g_,
                                   int32_t n_rhs, double shift, void* grad_x, double* grad_omega, int32_t per_rhs,
                                   rmh_stream stream) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_dtype(dtype));
  if (n_rhs < 0) return fail(RMH_E_ARG, "n_rhs < 0");
  if (n_rhs == 0) return RMH_OK;
  RMH_TRY(check_ptr(U, "U"));
  RMH_TRY(check_ptr(g_, "g"));
  const size_t fb = (size_t)n_rhs * 32 * g.V * dsize(dtype);
  if (grad_x) {
    RMH_TRY(check_ptr(grad_x, "grad_x"));
    if (overlap(grad_x, fb, g_, fb) || overlap(grad_x, fb, x, fb)) return fail(RMH_E_ARG, "grad_x overlaps an input");
    RMH_TRY(rmh_laplacian_apply(L, U, dtype, g_, grad_x, n_rhs, shift, stream));
  }
  if (grad_omega) {
    if (dtype != RMH_F64) return fail(RMH_E_ARG, "grad_omega needs RMH_F64 inputs");
    RMH_TRY(check_ptr(x, "x"));
    RMH_TRY(check_ptr(grad_omega, "grad_omega"));
    const size_t gb = (size_t)(per_rhs ? n_rhs : 1) * 32 * g.V * 8;
    if (overlap(grad_omega, gb, x, fb) || overlap(grad_omega, gb, g_, fb) || overlap(grad_omega, gb, grad_x, fb))
      return fail(RMH_E_ARG, "grad_omega overlaps another buffer");
    ForceArgs fa{};
    fa.g = g;
    fa.U = (const double*)U;
    fa.A = (const double*)g_;
    fa.B = (const double*)x;
    fa.n_rhs = n_rhs;
    fa.n_pair = 1;
    fa.w[0] = 1.0;
    fa.grad = grad_omega;
    fa.per_rhs = per_rhs ? 1 : 0;
    const double fbytes = (double)g.V * 8.0 * (48.0 + 64.0 * n_rhs + 32.0 * (per_rhs ? n_rhs : 1));
    ProfScope ps(RMH_PROF_FORCE, fbytes, (hipStream_t)stream, n_rhs);
    HIP_TRY(launch_force(fa, (hipStream_t)stream));
  }
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}


rmh_status rmh_cheb_coefficients(const rmh_cheb* cheb, double* coef) try {
  if (!cheb || !coef) return fail(RMH_E_ARG, "cheb or coef is NULL");
  RMH_TRY(check_cheb_dims(cheb, 0, kMaxSpectrumWindows));
  if (cheb->kernel != 0 && cheb->kernel != 1) return fail(RMH_E_ARG, "kernel must be 0 or 1");
  if (cheb_window_coefficients(cheb->degree, cheb->n_windows, cheb->edges, cheb->kernel, coef) != 0)
    return fail(RMH_E_ARG, "window edges must ascend strictly within [0, 16]");
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_power_ratio(const rmh_cheb* cheb, const double* trace_moments, const double* power, int32_t n_rhs,
                           double* ratio) try {
  if (!cheb || !trace_moments || !power || !ratio) return fail(RMH_E_ARG, "NULL argument");
  RMH_TRY(check_cheb_dims(cheb, 0, kMaxSpectrumWindows));
  const int32_t D = cheb->degree, nw = cheb->n_windows;
  std::vector<double> coef((size_t)nw * (D + 1));
  RMH_TRY(rmh_cheb_coefficients(cheb, coef.data()));
  for (int32_t w = 0; w < nw; ++w) {
    double den = 0.0;
    for (int32_t k = 0; k <= D; ++k) den += coef[(size_t)w * (D + 1) + k] * trace_moments[k];
    for (int32_t n = 0; n < n_rhs; ++n) ratio[(size_t)n * nw + w] = power[(size_t)n * nw + w] / den;
  }
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_trace_moments_free(const int32_t L[4], int32_t degree, double* trace_moments) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  if (degree < 0 || degree > kMaxChebDegree || !trace_moments)
    return fail(RMH_E_ARG, "degree = %d outside [0, %d] or NULL output", degree, kMaxChebDegree);
  trace_moments_free(L, degree, trace_moments);
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_power_spectrum(const int32_t L[4], const void* U, int32_t dtype, const void* F, int32_t n_rhs,
                              const rmh_cheb* cheb, double* moments, double* power, void* ws, size_t ws_bytes,
                              rmh_stream stream) try {
  return power_spectrum_impl(L, U, dtype, F, n_rhs, cheb, moments, power, ws, ws_bytes, false, stream);
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_power_spectrum_noalloc(const int32_t L[4], const void* U, int32_t dtype, const void* F,
                                      int32_t n_rhs, const rmh_cheb* cheb, double* moments, double* power,
                                      rmh_stream stream) try {
  return power_spectrum_impl(L, U, dtype, F, n_rhs, cheb, moments, power, nullptr, 0, true, stream);
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_cheb_filter(const int32_t L[4], const void* U, int32_t dtype, const void* x, int32_t n_rhs,
                           const rmh_cheb* cheb, void* y, void* ws, size_t ws_bytes, rmh_stream stream) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_dtype(dtype));
  RMH_TRY(check_cheb_dims(cheb, 1, kMaxFilterWindows));
  if (n_rhs < 0) return fail(RMH_E_ARG, "n_rhs < 0");
  const int32_t D = cheb->degree, nw = cheb->n_windows;
  std::vector<double> coef((size_t)nw * (D + 1));
  RMH_TRY(rmh_cheb_coefficients(cheb, coef.data()));
  if (n_rhs == 0) return RMH_OK;
  RMH_TRY(check_ptr(U, "U"));
  RMH_TRY(check_ptr(x, "x"));
  RMH_TRY(check_ptr(y, "y"));
  RMH_TRY(check_ptr(ws, "ws"));
  Carver c(ws);
  FilterPlan fp = plan_filter(c, g, dtype, n_rhs, D, nw);
  if (c.off > ws_bytes) return fail(RMH_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, c.off);
  const size_t fb = (size_t)n_rhs * 32 * g.V * dsize(dtype);
  if (overlap(y, fb * nw, x, fb) || overlap(y, fb * nw, ws, c.off) || overlap(y, fb * nw, U, (size_t)72 * g.V * dsize(dtype)))
    return fail(RMH_E_ARG, "y overlaps an input or the workspace");
  hipStream_t s = (hipStream_t)stream;
  if (dtype == RMH_F64)
    return cheb_filter_t<double>(g, (const double*)U, (const double*)x, n_rhs, D, nw, coef, fp, (double*)y, s);
  return cheb_filter_t<float>(g, (const float*)U, (const float*)x, n_rhs, D, nw, coef, fp, (float*)y, s);
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

static rmh_status cheb_bwd_common(const int32_t L[4], const double* U, const double* x, int32_t n_rhs,
                                  const rmh_cheb* cheb, const void* grad_x, const double* grad_omega, Geom* g,
                                  std::vector<double>* coef) {
  RMH_TRY(make_geom(L, g));
  RMH_TRY(check_cheb_dims(cheb, 1, kMaxSpectrumWindows));
  if (n_rhs < 0) return fail(RMH_E_ARG, "n_rhs < 0");
  const int32_t D = cheb->degree, nw = cheb->n_windows;
  coef->resize((size_t)nw * (D + 1));
  RMH_TRY(rmh_cheb_coefficients(cheb, coef->data()));
  if (!grad_x && !grad_omega) return fail(RMH_E_ARG, "neither grad_x nor grad_omega requested");
  if (n_rhs == 0) return RMH_OK;
  RMH_TRY(check_ptr(U, "U"));
  RMH_TRY(check_ptr(x, "x"));
  if (grad_x) RMH_TRY(check_ptr(grad_x, "grad_x"));
  if (grad_omega) RMH_TRY(check_ptr(grad_omega, "grad_omega"));
  return RMH_OK;
}

rmh_status rmh_cheb_filter_bwd(const int32_t L[4], const double* U, const double* x, const double* gy, int32_t n_rhs,
                               const rmh_cheb* cheb, double* grad_x, double* grad_omega, int32_t per_rhs, void* ws,
                               size_t ws_bytes, rmh_stream stream) try {
  Geom g;
  std::vector<double> coef;
  RMH_TRY(cheb_bwd_common(L, U, x, n_rhs, cheb, grad_x, grad_omega, &g, &coef));
  if (n_rhs == 0) return RMH_OK;
  RMH_TRY(check_ptr(gy, "gy"));
  RMH_TRY(check_ptr(ws, "ws"));
  const int32_t D = cheb->degree, nw = cheb->n_windows;
  Carver c(ws);
  ChebBwdPlan p = plan_cheb_bwd(c, g, n_rhs, nw, D);
  if (c.off > ws_bytes) return fail(RMH_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, c.off);
  const size_t fb = (size_t)n_rhs * 32 * g.V * 8, gb = (size_t)(per_rhs ? n_rhs : 1) * 32 * g.V * 8;
  const void* ins[4] = {U, x, gy, ws};
  const size_t insz[4] = {(size_t)72 * g.V * 8, fb, fb * nw, c.off};
  for (int i = 0; i < 4; ++i) {
    if (grad_x && overlap(grad_x, fb, ins[i], insz[i])) return fail(RMH_E_ARG, "grad_x overlaps an input or the workspace");
    if (grad_omega && overlap(grad_omega, gb, ins[i], insz[i]))
      return fail(RMH_E_ARG, "grad_omega overlaps an input or the workspace");
  }
  if (grad_x && grad_omega && overlap(grad_x, fb, grad_omega, gb)) return fail(RMH_E_ARG, "grad_x overlaps grad_omega");
  // G_k[v] = sum_w coef[w][k] gy[w][v]
  std::vector<double> ch((size_t)n_rhs * nw * (D + 1));
  for (int32_t v = 0; v < n_rhs; ++v)
    for (int32_t w = 0; w < nw; ++w)
      for (int32_t k = 0; k <= D; ++k) ch[((size_t)v * nw + w) * (D + 1) + k] = coef[(size_t)w * (D + 1) + k];
  return cheb_bwd(g, U, x, n_rhs, D, gy, nw, ch, p, grad_x, 1.0, grad_omega, per_rhs, (hipStream_t)stream);
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_power_spectrum_bwd(const int32_t L[4], const double* U, const double* F, int32_t n_rhs,
                                  const rmh_cheb* cheb, const double* gamma, double* grad_F, double* grad_omega,
                                  int32_t per_rhs, void* ws, size_t ws_bytes, rmh_stream stream) try {
  Geom g;
  std::vector<double> coef;
  RMH_TRY(cheb_bwd_common(L, U, F, n_rhs, cheb, grad_F, grad_omega, &g, &coef));
  if (n_rhs == 0) return RMH_OK;
  if (!gamma) return fail(RMH_E_ARG, "gamma is NULL");
  RMH_TRY(check_ptr(ws, "ws"));
  const int32_t D = cheb->degree, nw = cheb->n_windows;
  for (size_t i = 0; i < (size_t)n_rhs * nw; ++i)
    if (!isfinite(gamma[i])) return fail(RMH_E_ARG, "gamma[%zu] is not finite", i);
  Carver c(ws);
  ChebBwdPlan p = plan_cheb_bwd(c, g, n_rhs, 1, D);
  if (c.off > ws_bytes) return fail(RMH_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, c.off);
  const size_t fb = (size_t)n_rhs * 32 * g.V * 8, gb = (size_t)(per_rhs ? n_rhs : 1) * 32 * g.V * 8;
  const void* ins[3] = {U, F, ws};
  const size_t insz[3] = {(size_t)72 * g.V * 8, fb, c.off};
  for (int i = 0; i < 3; ++i) {
    if (grad_F && overlap(grad_F, fb, ins[i], insz[i])) return fail(RMH_E_ARG, "grad_F overlaps an input or the workspace");
    if (grad_omega && overlap(grad_omega, gb, ins[i], insz[i]))
      return fail(RMH_E_ARG, "grad_omega overlaps an input or the workspace");
  }
  if (grad_F && grad_omega && overlap(grad_F, fb, grad_omega, gb)) return fail(RMH_E_ARG, "grad_F overlaps grad_omega");
  // one source vector per field, G_k = beta_k F with beta_k = sum_w gamma_w coef[w][k]
  std::vector<double> ch((size_t)n_rhs * (D + 1), 0.0);
  for (int32_t v = 0; v < n_rhs; ++v)
    for (int32_t w = 0; w < nw; ++w)
      for (int32_t k = 0; k <= D; ++k)
        ch[(size_t)v * (D + 1) + k] += gamma[(size_t)v * nw + w] * coef[(size_t)w * (D + 1) + k];
  // F enters both slots of <F, p(A) F>: grad_F = tb_0 + p(A) F = 2 tb_0 (p(A) symmetric)
  return cheb_bwd(g, U, F, n_rhs, D, F, 1, ch, p, grad_F, 2.0, grad_omega, per_rhs, (hipStream_t)stream);
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_wilson_gauge_force(const int32_t L[4], const double* U, double beta, double* F, double* S, void* ws,
                                  size_t ws_bytes, rmh_stream stream) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  if (!isfinite(beta)) return fail(RMH_E_ARG, "beta is not finite");
  if (!F && !S) return fail(RMH_E_ARG, "neither F nor S requested");
  RMH_TRY(check_ptr(U, "U"));
  if (F) RMH_TRY(check_ptr(F, "F"));
  if (F && overlap(F, (size_t)32 * g.V * 8, U, (size_t)72 * g.V * 8)) return fail(RMH_E_ARG, "F overlaps U");
  hipStream_t s = (hipStream_t)stream;
  double* part = nullptr;
  double* sum = nullptr;
  if (S) {
    RMH_TRY(check_ptr(ws, "ws"));
    Carver c(ws);
    part = c.take<double>(gauge_force_blocks(g));
    sum = c.take<double>(1);
    if (c.off > ws_bytes) return fail(RMH_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, c.off);
    if (F && overlap(F, (size_t)32 * g.V * 8, ws, c.off)) return fail(RMH_E_ARG, "F overlaps the workspace");
  }
  {
    ProfScope ps(RMH_PROF_FORCE, (double)g.V * 8.0 * (48.0 + (F ? 32.0 : 0.0)), s, 1.0);
    HIP_TRY(launch_gauge_force(g, U, beta, F, part, s));
  }
  if (S) {
    HIP_TRY(launch_reduce_rows(part, gauge_force_blocks(g), 1, sum, s));
    double tr = 0.0;
    RMH_TRY(d2h(&tr, sum, 8, s));
    // every plaquette enters the staple sums of its four links
    *S = beta * (6.0 * g.V - tr / 12.0);
  }
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_rational_from_quadratics(int32_t n_terms, const double* a0, const double* a1, const double* b0,
                                        const double* b1, double* r, double* sigma) try {
  if (n_terms < 1 || !a0 || !a1 || !b0 || !b1 || !r || !sigma) return fail(RMH_E_ARG, "bad arguments");
  if (rational_from_quadratics(n_terms, a0, a1, b0, b1, r, sigma) != 0)
    return fail(RMH_E_POLES, "a quadratic term has no two distinct real roots with positive shifts");
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_rational_kappa(double kappa, int32_t n, double* c, double* r, double* sigma) try {
  if (!c || !r || !sigma) return fail(RMH_E_ARG, "NULL output");
  if (rational_kappa(kappa, n, c, r, sigma) != 0) return fail(RMH_E_ARG, "need 0 < kappa < 1 and n >= 1");
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

static rmh_status rational_common(const int32_t L[4], const double* U, int32_t n_rhs, const rmh_rational* rat,
                                  const rmh_solver* sv, Geom* g) {
  RMH_TRY(make_geom(L, g));
  if (n_rhs < 0) return fail(RMH_E_ARG, "n_rhs < 0");
  RMH_TRY(check_rational(rat));
  RMH_TRY(check_solver(sv));
  RMH_TRY(check_ptr(U, "U"));
  return RMH_OK;
}

rmh_status rmh_rational_apply(const int32_t L[4], const double* U, const double* x, int32_t n_rhs,
                              const rmh_rational* rat, const rmh_solver* solver, double* y, double* x_poles,
                              double* K, rmh_stats* stats, void* ws, size_t ws_bytes, rmh_stream stream) try {
  const double t0 = now_s();
  Geom g;
  RMH_TRY(rational_common(L, U, n_rhs, rat, solver, &g));
  if (n_rhs == 0) return RMH_OK;
  RMH_TRY(check_ptr(x, "x"));
  RMH_TRY(check_ptr(y, "y"));
  RMH_TRY(check_ptr(ws, "ws"));
  const int32_t np = rat->n_poles;
  Carver c(ws);
  RationalPlan rp;
  plan_rational(c, rp, g, n_rhs, np, solver->mode, solver->basis, RMH_OP_RATIONAL_APPLY);
  if (c.off > ws_bytes) return fail(RMH_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, c.off);
  const int64_t n = field_reals(g);
  const size_t fb = (size_t)n_rhs * n * 8, pb = fb * np;
  if (overlap(y, fb, x, fb) || overlap(y, fb, ws, c.off) || overlap(ws, c.off, x, fb) || overlap(ws, c.off, U, 72 * (size_t)g.V * 8))
    return fail(RMH_E_ARG, "overlapping buffers");
  if (x_poles) {
    RMH_TRY(check_ptr(x_poles, "x_poles"));
    if (overlap(x_poles, pb, x, fb) || overlap(x_poles, pb, y, fb) || overlap(x_poles, pb, ws, c.off))
      return fail(RMH_E_ARG, "x_poles overlaps another buffer");
  }
  hipStream_t s = (hipStream_t)stream;
  double* X = x_poles ? x_poles : rp.X;
  std::vector<double> sig(rat->sigma, rat->sigma + np);
  SolveResult res;
  RMH_TRY(solve_all(rp.sp, U, x, X, sig, *solver, s, &res));
  std::vector<double> coef(np + 1);
  coef[0] = rat->c;
  for (int j = 0; j < np; ++j) coef[1 + j] = rat->r[j];
  RMH_TRY(h2d(rp.coef, coef.data(), coef.size() * 8, s));
  HIP_TRY(launch_rational_combine(x, X, n_rhs, np, rp.coef, y, n, rp.partK, s));
  if (K) {
    HIP_TRY(launch_reduce_rows(rp.partK, red_num_blocks(n), n_rhs, rp.sumsK, s));
    RMH_TRY(d2h(K, rp.sumsK, n_rhs * 8, s));
    for (int v = 0; v < n_rhs; ++v) K[v] *= 0.5;
  } else {
    HIP_TRY(hipStreamSynchronize(s));
  }
  fill_stats(stats, &res, 1, now_s() - t0);
  return status_of(res, "rational_apply");
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_heatbath_momenta(const int32_t L[4], const double* U, const double* xi, int32_t n_rhs, double kappa,
                                const rmh_rational* rat, const rmh_solver* solver, double* P, rmh_stats* stats,
                                void* ws, size_t ws_bytes, rmh_stream stream) try {
  const double t0 = now_s();
  Geom g;
  RMH_TRY(rational_common(L, U, n_rhs, rat, solver, &g));
  if (!(kappa >= 0.0 && kappa <= 1.0)) return fail(RMH_E_ARG, "kappa = %g must lie in [0, 1]", kappa);
  // kappa = 0: P = R(Delta)^{-1} xi through the partial fractions of 1/R,
  // a Delta + b + sum_k rho_k (Delta + tau_k)^{-1}
  const int32_t np = rat->n_poles;
  double ia = 0.0, ib = 0.0;
  std::vector<double> rho(np), tau(np);
  int32_t m = 0;
  if (kappa == 0.0 &&
      rational_inverse(rat->c, np, rat->r, rat->sigma, &ia, &ib, rho.data(), tau.data(), &m) != 0)
    return fail(RMH_E_POLES, "1/R(Delta) has no partial-fraction form with positive shifts (needs c >= 0, r_j > 0, "
                             "distinct sigma_j > 0)");
  if (n_rhs == 0) return RMH_OK;
  RMH_TRY(check_ptr(xi, "xi"));
  RMH_TRY(check_ptr(P, "P"));
  RMH_TRY(check_ptr(ws, "ws"));
  Carver c(ws);
  RationalPlan rp;
  // the exact inverse solves over the m shifts tau_k (m <= n_poles, within the queried workspace)
  plan_rational(c, rp, g, n_rhs, kappa == 0.0 ? std::max(m, 1) : np, solver->mode, solver->basis,
                RMH_OP_HEATBATH);
  if (c.off > ws_bytes) return fail(RMH_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, c.off);
  const int64_t n = field_reals(g);
  const size_t fb = (size_t)n_rhs * n * 8;
  if (overlap(P, fb, xi, fb) || overlap(P, fb, ws, c.off) || overlap(P, fb, U, (size_t)72 * g.V * 8) ||
      overlap(ws, c.off, xi, fb) || overlap(ws, c.off, U, (size_t)72 * g.V * 8))
    return fail(RMH_E_ARG, "overlapping buffers");
  hipStream_t s = (hipStream_t)stream;
  SolveResult res;
  HopArgs<double> h{};
  h.g = g;
  h.U = U;
  h.x_mul = 1;
  h.z_div = 1;
  h.out = P;
  h.n_rhs = n_rhs;
  h.store = 1;
  if (kappa > 0.0) {
    std::vector<double> sig(rat->sigma, rat->sigma + np);
    RMH_TRY(solve_all(rp.sp, U, xi, rp.X, sig, *solver, s, &res));
    std::vector<double> coef(np + 1);
    coef[0] = rat->c;
    for (int j = 0; j < np; ++j) coef[1 + j] = rat->r[j];
    RMH_TRY(h2d(rp.coef, coef.data(), coef.size() * 8, s));
    HIP_TRY(launch_rational_combine(xi, rp.X, n_rhs, np, rp.coef, rp.Y, n, nullptr, s));
    // P = (1 - kappa) y + kappa Delta y = -kappa H y + (1 + 7 kappa) y,  y = R(Delta) xi
    h.x = rp.Y;
    h.a = -kappa;
    h.b = 1.0 + 7.0 * kappa;
  } else {
    // Y = b xi + sum_k rho_k (Delta + tau_k)^{-1} xi, then P = a Delta xi + Y = -a H xi + 8 a xi + Y
    if (m > 0) {
      std::vector<double> sig(tau.begin(), tau.begin() + m);
      RMH_TRY(solve_all(rp.sp, U, xi, rp.X, sig, *solver, s, &res));
      std::vector<double> coef(m + 1);
      coef[0] = ib;
      for (int k = 0; k < m; ++k) coef[1 + k] = rho[k];
      RMH_TRY(h2d(rp.coef, coef.data(), coef.size() * 8, s));
      HIP_TRY(launch_rational_combine(xi, rp.X, n_rhs, m, rp.coef, rp.Y, n, nullptr, s));
      h.z = rp.Y;
      h.c = 1.0;
      h.b = 8.0 * ia;
    } else {
      h.b = 8.0 * ia + ib;
    }
    h.x = xi;
    h.a = -ia;
  }
  {
    ProfScope ps(RMH_PROF_STENCIL, hop_bytes(g, n_rhs, 8, h.z != nullptr, true), s, n_rhs);
    HIP_TRY(launch_hop<double>(h, hop_config(g, RMH_F64, n_rhs, RMH_PURPOSE_HEATBATH), s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  fill_stats(stats, &res, 1, now_s() - t0);
  return status_of(res, "heatbath_momenta");
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

// second solve (source g) and the force; X holds the pole solutions of the first solve
static rmh_status force_from_solves(RationalPlan& rp, const Geom& g, const double* U, const double* X,
                                    const double* gsrc, int32_t n_rhs, const rmh_rational* rat,
                                    const rmh_solver* sv, double* grad_x, double* grad_omega, int32_t per_rhs,
                                    hipStream_t s, SolveResult* res2) {
  const int32_t np = rat->n_poles;
  const int64_t n = field_reals(g);
  std::vector<double> sig(rat->sigma, rat->sigma + np);
  RMH_TRY(solve_all(rp.sp, U, gsrc, rp.Z, sig, *sv, s, res2));
  if (grad_x) HIP_TRY(launch_rational_combine(gsrc, rp.Z, n_rhs, np, rp.coef, grad_x, n, nullptr, s));
  ForceArgs fa{};
  for (int j = 0; j < np; ++j) fa.w[j] = -rat->r[j];
  fa.g = g;
  fa.U = U;
  fa.A = rp.Z;
  fa.B = X;
  fa.n_rhs = n_rhs;
  fa.n_pair = np;
  fa.grad = grad_omega;
  fa.per_rhs = per_rhs ? 1 : 0;
  {
    const double fbytes = (double)g.V * 8.0 * (48.0 + 64.0 * n_rhs * np + 32.0 * (per_rhs ? n_rhs : 1));
    ProfScope ps(RMH_PROF_FORCE, fbytes, s, n_rhs);
    HIP_TRY(launch_force(fa, s));
  }
  return RMH_OK;
}

rmh_status rmh_rational_apply_bwd(const int32_t L[4], const double* U, const double* x, const double* g_,
                                  int32_t n_rhs, const rmh_rational* rat, const rmh_solver* solver, double* grad_x,
                                  double* grad_omega, int32_t per_rhs, rmh_stats* stats, void* ws, size_t ws_bytes,
                                  rmh_stream stream) try {
  const double t0 = now_s();
  Geom g;
  RMH_TRY(rational_common(L, U, n_rhs, rat, solver, &g));
  if (n_rhs == 0) return RMH_OK;
  RMH_TRY(check_ptr(x, "x"));
  RMH_TRY(check_ptr(g_, "g"));
  RMH_TRY(check_ptr(grad_omega, "grad_omega"));
  RMH_TRY(check_ptr(ws, "ws"));
  const int32_t np = rat->n_poles;
  Carver c(ws);
  RationalPlan rp;
  plan_rational(c, rp, g, n_rhs, np, solver->mode, solver->basis, RMH_OP_RATIONAL_APPLY_BWD);
  if (c.off > ws_bytes) return fail(RMH_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, c.off);
  const int64_t n = field_reals(g);
  const size_t fb = (size_t)n_rhs * n * 8, gb = (size_t)(per_rhs ? n_rhs : 1) * n * 8;
  if (overlap(grad_omega, gb, x, fb) || overlap(grad_omega, gb, g_, fb) || overlap(grad_omega, gb, ws, c.off) ||
      (grad_x && (overlap(grad_x, fb, x, fb) || overlap(grad_x, fb, g_, fb) || overlap(grad_x, fb, ws, c.off) ||
                  overlap(grad_x, fb, grad_omega, gb))) ||
      overlap(ws, c.off, x, fb) || overlap(ws, c.off, g_, fb))
    return fail(RMH_E_ARG, "overlapping buffers");
  hipStream_t s = (hipStream_t)stream;
  std::vector<double> coef(np + 1);
  coef[0] = rat->c;
  for (int j = 0; j < np; ++j) coef[1 + j] = rat->r[j];
  RMH_TRY(h2d(rp.coef, coef.data(), coef.size() * 8, s));
  std::vector<double> sig(rat->sigma, rat->sigma + np);
  SolveResult res[2];
  RMH_TRY(solve_all(rp.sp, U, x, rp.X, sig, *solver, s, &res[0]));
  RMH_TRY(force_from_solves(rp, g, U, rp.X, g_, n_rhs, rat, solver, grad_x, grad_omega, per_rhs, s, &res[1]));
  HIP_TRY(hipStreamSynchronize(s));
  fill_stats(stats, res, 2, now_s() - t0);
  RMH_TRY(status_of(res[0], "rational_apply_bwd (solve of x)"));
  return status_of(res[1], "rational_apply_bwd (solve of g)");
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_kinetic_force(const int32_t L[4], const double* U, const double* P, int32_t n_rhs,
                             const rmh_rational* rat, const rmh_solver* solver, double* Y, double* K,
                             double* dK_domega, int32_t per_rhs, rmh_stats* stats, void* ws, size_t ws_bytes,
                             rmh_stream stream) try {
  const double t0 = now_s();
  Geom g;
  RMH_TRY(rational_common(L, U, n_rhs, rat, solver, &g));
  if (n_rhs == 0) return RMH_OK;
  RMH_TRY(check_ptr(P, "P"));
  RMH_TRY(check_ptr(dK_domega, "dK_domega"));
  RMH_TRY(check_ptr(ws, "ws"));
  const int32_t np = rat->n_poles;
  Carver c(ws);
  RationalPlan rp;
  plan_rational(c, rp, g, n_rhs, np, solver->mode, solver->basis, RMH_OP_KINETIC_FORCE);
  if (c.off > ws_bytes) return fail(RMH_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, c.off);
  const int64_t n = field_reals(g);
  const size_t fb = (size_t)n_rhs * n * 8, gb = (size_t)(per_rhs ? n_rhs : 1) * n * 8;
  if (Y) RMH_TRY(check_ptr(Y, "Y"));
  if (overlap(dK_domega, gb, P, fb) || overlap(dK_domega, gb, ws, c.off) || overlap(ws, c.off, P, fb) ||
      (Y && (overlap(Y, fb, P, fb) || overlap(Y, fb, ws, c.off) || overlap(Y, fb, dK_domega, gb))))
    return fail(RMH_E_ARG, "overlapping buffers");
  hipStream_t s = (hipStream_t)stream;
  double* Yb = Y ? Y : rp.Y;
  std::vector<double> coef(np + 1);
  coef[0] = rat->c;
  for (int j = 0; j < np; ++j) coef[1 + j] = rat->r[j];
  RMH_TRY(h2d(rp.coef, coef.data(), coef.size() * 8, s));
  std::vector<double> sig(rat->sigma, rat->sigma + np);
  SolveResult res[2];
  RMH_TRY(solve_all(rp.sp, U, P, rp.X, sig, *solver, s, &res[0]));
  HIP_TRY(launch_rational_combine(P, rp.X, n_rhs, np, rp.coef, Yb, n, rp.partK, s));
  if (K) {
    HIP_TRY(launch_reduce_rows(rp.partK, red_num_blocks(n), n_rhs, rp.sumsK, s));
    RMH_TRY(d2h(K, rp.sumsK, n_rhs * 8, s));
    for (int v = 0; v < n_rhs; ++v) K[v] *= 0.5;
  }
  RMH_TRY(force_from_solves(rp, g, U, rp.X, Yb, n_rhs, rat, solver, nullptr, dK_domega, per_rhs, s, &res[1]));
  HIP_TRY(hipStreamSynchronize(s));
  fill_stats(stats, res, 2, now_s() - t0);
  RMH_TRY(status_of(res[0], "kinetic_force (solve of P)"));
  return status_of(res[1], "kinetic_force (solve of Y)");
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

// dK/d omega at (U, P) into lp.dK: the kinetic force's two solves and its link derivative
static rmh_status lf_kinetic_grad(LeapfrogPlan& lp, const Geom& g, const double* U, const double* P,
                                  const rmh_rational* rat, const rmh_solver* sv, hipStream_t s,
                                  std::vector<SolveResult>& res) {
  const int32_t np = rat->n_poles;
  const int64_t n = field_reals(g);
  std::vector<double> sig(rat->sigma, rat->sigma + np);
  SolveResult r1, r2;
  RMH_TRY(solve_all(lp.rp.sp, U, P, lp.rp.X, sig, *sv, s, &r1));
  HIP_TRY(launch_rational_combine(P, lp.rp.X, 1, np, lp.rp.coef, lp.rp.Y, n, nullptr, s));
  RMH_TRY(force_from_solves(lp.rp, g, U, lp.rp.X, lp.rp.Y, 1, rat, sv, nullptr, lp.dK, 0, s, &r2));
  res.push_back(r1);
  res.push_back(r2);
  return RMH_OK;
}

// Pi = R(Delta[U])^2 P into out
static rmh_status lf_velocity(LeapfrogPlan& lp, const Geom& g, const double* U, const double* P, double* out,
                              const rmh_rational* rat, const rmh_solver* sv, hipStream_t s,
                              std::vector<SolveResult>& res) {
  const int32_t np = rat->n_poles;
  const int64_t n = field_reals(g);
  std::vector<double> sig(rat->sigma, rat->sigma + np);
  SolveResult r1, r2;
  RMH_TRY(solve_all(lp.rp.sp, U, P, lp.rp.X, sig, *sv, s, &r1));
  HIP_TRY(launch_rational_combine(P, lp.rp.X, 1, np, lp.rp.coef, lp.rp.Y, n, nullptr, s));
  RMH_TRY(solve_all(lp.rp.sp, U, lp.rp.Y, lp.rp.Z, sig, *sv, s, &r2));
  HIP_TRY(launch_rational_combine(lp.rp.Y, lp.rp.Z, 1, np, lp.rp.coef, out, n, nullptr, s));
  res.push_back(r1);
  res.push_back(r2);
  return RMH_OK;
}

// -dK/d omega weights of the pole pairs at the solves held in lp.rp (X of P, Z of Y = R(Delta) P)
static rmh_status lf_force_from_held(LeapfrogPlan& lp, const Geom& g, const double* U, const rmh_rational* rat,
                                     hipStream_t s) {
  ForceArgs fa{};
  for (int j = 0; j < rat->n_poles; ++j) fa.w[j] = -rat->r[j];
  fa.g = g;
  fa.U = U;
  fa.A = lp.rp.Z;
  fa.B = lp.rp.X;
  fa.n_rhs = 1;
  fa.n_pair = rat->n_poles;
  fa.grad = lp.dK;
  ProfScope ps(RMH_PROF_FORCE, (double)g.V * 8.0 * (48.0 + 64.0 * rat->n_poles + 32.0), s, 1.0);
  HIP_TRY(launch_force(fa, s));
  return RMH_OK;
}

// out = x + h (y - z); returns |out - prev| and |out|
static rmh_status lf_update(LeapfrogPlan& lp, const double* x, const double* y, const double* z, double h,
                            const double* prev, double* out, int64_t n, hipStream_t s, double* diff, double* norm) {
  HIP_TRY(launch_axpy_diff(x, y, z, h, prev, out, n, lp.part, s));
  if (!diff) return RMH_OK;
  HIP_TRY(launch_reduce_rows(lp.part, red_num_blocks(n), 2, lp.sums, s));
  double hs[2];
  RMH_TRY(d2h(hs, lp.sums, sizeof(hs), s));
  *diff = sqrt(hs[0]);
  *norm = sqrt(hs[1]);
  return RMH_OK;
}

rmh_status rmh_leapfrog_step(const int32_t L[4], const double* U0, const double* P0, const rmh_rational* rat,
                             const rmh_solver* solver, const rmh_leapfrog* lf, double* U1, double* P1,
                             rmh_leapfrog_stats* stats, void* ws, size_t ws_bytes, rmh_stream stream) try {
  const double t0 = now_s();
  Geom g;
  RMH_TRY(rational_common(L, U0, 1, rat, solver, &g));
  if (!lf) return fail(RMH_E_ARG, "NULL step controls");
  if (!(isfinite(lf->eps) && isfinite(lf->beta))) return fail(RMH_E_ARG, "eps and beta must be finite");
  if (!(lf->fp_tol > 0.0) || lf->fp_maxiter < 1) return fail(RMH_E_ARG, "need fp_tol > 0 and fp_maxiter >= 1");
  RMH_TRY(check_ptr(P0, "P0"));
  RMH_TRY(check_ptr(U1, "U1"));
  RMH_TRY(check_ptr(P1, "P1"));
  RMH_TRY(check_ptr(ws, "ws"));
  Carver c(ws);
  LeapfrogPlan lp;
  plan_leapfrog(c, lp, g, rat->n_poles, solver->mode, solver->basis);
  if (c.off > ws_bytes) return fail(RMH_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, c.off);
  const int64_t n = field_reals(g);
  const size_t fb = (size_t)n * 8, ub = (size_t)72 * g.V * 8;
  const void* bufs[5] = {U0, P0, U1, P1, ws};
  const size_t lens[5] = {ub, fb, ub, fb, c.off};
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j)
      if (overlap(bufs[i], lens[i], bufs[j], lens[j])) return fail(RMH_E_ARG, "overlapping buffers");
  hipStream_t s = (hipStream_t)stream;
  const int32_t np = rat->n_poles;
  std::vector<double> coef(np + 1);
  coef[0] = rat->c;
  for (int j = 0; j < np; ++j) coef[1 + j] = rat->r[j];
  RMH_TRY(h2d(lp.rp.coef, coef.data(), coef.size() * 8, s));
  const double h = 0.5 * lf->eps, tol = lf->fp_tol;
  std::vector<SolveResult> res;
  bool noconv = false;
  // Each fixed point keeps the first iterate whose successor changes it by at most tol: the solves
  // of the kept iterate are then the ones in the workspace, and the next stage starts from them.
  // (i) P_h = P0 + h F(U0, P_h), F = F_G - dK/d omega, from P_h = P0
  HIP_TRY(launch_gauge_force(g, U0, lf->beta, lp.Fg, nullptr, s));
  HIP_TRY(hipMemcpyAsync(lp.Ph, P0, fb, hipMemcpyDeviceToDevice, s));
  double* ph = lp.Ph;    // current iterate
  double* pn = lp.PiB;   // its successor (PiB is free until stage ii)
  int32_t ip = 0;
  double dp = 0.0, np_ = 0.0;
  while (true) {
    ++ip;
    RMH_TRY(lf_kinetic_grad(lp, g, U0, ph, rat, solver, s, res));
    RMH_TRY(lf_update(lp, P0, lp.Fg, lp.dK, h, ph, pn, n, s, &dp, &np_));
    if (dp <= tol * np_) break;
    if (ip >= lf->fp_maxiter || !(dp == dp)) {
      noconv = true;
      break;
    }
    std::swap(ph, pn);
  }
  // (ii) U1 = exp(i h (Pi(U0, P_h) + Pi(U1, P_h))) U0, from Pi(U1) = Pi(U0).  Pi(U0, P_h) =
  // R(Delta) Y from the held solves of P_h (X) and of Y = R(Delta) P_h (Z).
  HIP_TRY(launch_rational_combine(lp.rp.Y, lp.rp.Z, 1, np, lp.rp.coef, lp.Pi0, n, nullptr, s));
  double* pib = pn;   // the Pi that U1 was built from (in the buffer ph does not use)
  HIP_TRY(hipMemcpyAsync(pib, lp.Pi0, fb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_link_exp(g, U0, lp.Pi0, pib, h, U1, s));
  int32_t iu = 0;
  double du = 0.0, nu = 0.0;
  while (true) {
    ++iu;
    RMH_TRY(lf_velocity(lp, g, U1, ph, lp.PiA, rat, solver, s, res));
    RMH_TRY(lf_update(lp, lp.PiA, lp.PiA, lp.PiA, 0.0, pib, pib, n, s, &du, &nu));   // change; pib = PiA
    if (du <= tol * nu) break;
    if (iu >= lf->fp_maxiter || !(du == du)) {
      noconv = true;
      break;
    }
    HIP_TRY(launch_link_exp(g, U0, lp.Pi0, lp.PiA, h, U1, s));
  }
  // (iii) P1 = P_h + h F(U1, P_h), the kinetic part from the solves at the kept U1
  HIP_TRY(launch_gauge_force(g, U1, lf->beta, lp.Fg, nullptr, s));
  RMH_TRY(lf_force_from_held(lp, g, U1, rat, s));
  RMH_TRY(lf_update(lp, ph, lp.Fg, lp.dK, h, P1, P1, n, s, nullptr, nullptr));
  HIP_TRY(hipStreamSynchronize(s));
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->p_iters = ip;
    stats->u_iters = iu;
    stats->p_res = np_ > 0.0 ? dp / np_ : dp;
    stats->u_res = nu > 0.0 ? du / nu : du;
    fill_stats(&stats->solver, res.data(), (int)res.size(), now_s() - t0);
  }
  for (const SolveResult& r : res) RMH_TRY(status_of(r, "leapfrog_step (a shifted solve)"));
  if (noconv)
    return fail(RMH_E_NOCONV, "leapfrog_step: a fixed point did not reach fp_tol = %g in %d iterations (%d, %d)",
                tol, lf->fp_maxiter, ip, iu);
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_link_exp(const int32_t L[4], const double* U0, const double* omega, double* U1, rmh_stream stream) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_ptr(U0, "U0"));
  RMH_TRY(check_ptr(omega, "omega"));
  RMH_TRY(check_ptr(U1, "U1"));
  const size_t ub = (size_t)72 * g.V * 8, wb = (size_t)32 * g.V * 8;
  if (overlap(U0, ub, U1, ub) || overlap(omega, wb, U1, ub)) return fail(RMH_E_ARG, "U1 overlaps U0 or omega");
  HIP_TRY(launch_link_exp(g, U0, omega, nullptr, 1.0, U1, (hipStream_t)stream));
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_link_exp_vjp(const int32_t L[4], const double* omega, const double* g_, double* out,
                            rmh_stream stream) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_ptr(omega, "omega"));
  RMH_TRY(check_ptr(g_, "g"));
  RMH_TRY(check_ptr(out, "out"));
  const size_t wb = (size_t)32 * g.V * 8;
  if (overlap(omega, wb, out, wb)) return fail(RMH_E_ARG, "out overlaps omega");
  if (out != g_ && overlap(g_, wb, out, wb)) return fail(RMH_E_ARG, "out partially overlaps g");
  HIP_TRY(launch_dexp_vjp(g, omega, g_, out, (hipStream_t)stream));
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

static HopConfig from_abi(const rmh_hop_config& c) {
  HopConfig h;
  h.form = c.form;
  h.block = c.block;
  h.xcd_remap = c.xcd_remap;
  h.nv = c.nv;
  h.order = c.order;
  h.walk = c.walk;
  h.ns = c.ns;
  h.tile2 = c.tile2;
  return h;
}

static rmh_hop_config to_abi(const HopConfig& h) {
  rmh_hop_config c;
  c.form = h.form;
  c.block = h.block;
  c.xcd_remap = h.xcd_remap;
  c.nv = h.nv;
  c.order = h.order;
  c.walk = h.walk;
  c.ns = h.ns;
  c.tile2 = h.tile2;
  return c;
}

static rmh_status check_purpose(int32_t purpose) {
  if (purpose < RMH_PURPOSE_ANY || purpose > RMH_PURPOSE_HEATBATH)
    return fail(RMH_E_ARG, "purpose = %d outside [%d, %d]", purpose, (int)RMH_PURPOSE_ANY, (int)RMH_PURPOSE_HEATBATH);
  return RMH_OK;
}

// architecture name of the current device and the HIP runtime version, the stamp of a tuning file
// ("no-device" on a host without a GPU, where the cache can still be saved and loaded)
static rmh_status device_stamp(std::string* arch, int32_t* runtime) {
  int dev = 0, ndev = 0;
  *arch = "no-device";
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    *arch = prop.gcnArchName;
  }
  (void)hipGetLastError();
  int rt = 0;
  if (hipRuntimeGetVersion(&rt) != hipSuccess) rt = 0;
  *runtime = rt;
  return RMH_OK;
}

rmh_status rmh_tune_set(const int32_t L[4], int32_t dtype, int32_t n_rhs, int32_t purpose, const rmh_hop_config* cfg) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_dtype(dtype));
  RMH_TRY(check_purpose(purpose));
  if (n_rhs < 1) return fail(RMH_E_ARG, "n_rhs must be >= 1");
  if (!cfg) return fail(RMH_E_ARG, "cfg is NULL");
  const HopConfig c = from_abi(*cfg);
  if (const char* why = hop_config_error(c, dtype)) return fail(RMH_E_ARG, "%s", why);
  tune_store(g, dtype, n_rhs, purpose, c, 0.0);
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_tune_clear(void) try {
  tune_clear();
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_tune_save(const char* path, int32_t* n_saved) try {
  if (!path) return fail(RMH_E_ARG, "path is NULL");
  std::string arch;
  int32_t rt = 0;
  RMH_TRY(device_stamp(&arch, &rt));
  if (tune_save_file(path, arch, rt, n_saved) != 0) return fail(RMH_E_HOST, "cannot write %s", path);
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_tune_load(const char* path, int32_t* n_loaded) try {
  if (!path) return fail(RMH_E_ARG, "path is NULL");
  std::string arch;
  int32_t rt = 0;
  RMH_TRY(device_stamp(&arch, &rt));
  const int r = tune_load_file(path, arch, rt, n_loaded);
  if (r == -1) return fail(RMH_E_HOST, "cannot read %s", path);
  if (r == -2) return fail(RMH_E_ARG, "%s is not a valid tuning file", path);
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_autotune_laplacian(const int32_t L[4], const void* U, int32_t dtype, const void* x, void* y,
                                  int32_t n_rhs, int32_t purpose, int32_t reps, rmh_hop_config* best, double* best_ms,
                                  void* ws, size_t ws_bytes, rmh_stream stream) try {
  Geom g;
  RMH_TRY(make_geom(L, &g));
  RMH_TRY(check_dtype(dtype));
  RMH_TRY(check_purpose(purpose));
  if (n_rhs < 1 || reps < 1) return fail(RMH_E_ARG, "n_rhs and reps must be >= 1");
  RMH_TRY(check_ptr(U, "U"));
  RMH_TRY(check_ptr(x, "x"));
  RMH_TRY(check_ptr(y, "y"));
  RMH_TRY(check_ptr(ws, "ws"));
  Carver cw(ws);
  double* partials = plan_autotune(cw, g, n_rhs);
  if (cw.off > ws_bytes) return fail(RMH_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, cw.off);
  {
    const size_t fb = (size_t)n_rhs * 32 * g.V * dsize(dtype), ub = (size_t)72 * g.V * dsize(dtype);
    if (overlap(x, fb, y, fb) || overlap(U, ub, y, fb)) return fail(RMH_E_ARG, "y overlaps x or U");
    if (overlap(ws, cw.off, x, fb) || overlap(ws, cw.off, y, fb) || overlap(ws, cw.off, U, ub))
      return fail(RMH_E_ARG, "ws overlaps x, y or U");
  }
  // timing unit: 1 = plain application, 2 = recursion step, 3 = both
  const int32_t unit_kind = (purpose == RMH_PURPOSE_MOMENTS || purpose == RMH_PURPOSE_FILTER ||
                             purpose == RMH_PURPOSE_CHEB_BWD)
                                ? 2
                                : (purpose == RMH_PURPOSE_ANY ? 3 : 1);
  // the dot products fused into the purpose's launches: <p, Ap> in the CG iterations and the FP64
  // residuals, the three moment sums in the power-spectrum sweeps
  const int32_t dot_mask = (purpose == RMH_PURPOSE_CG || purpose == RMH_PURPOSE_CG64) ? 2
                           : purpose == RMH_PURPOSE_MOMENTS                           ? 7
                                                                                      : 0;
  hipStream_t s = (hipStream_t)stream;
  // y is the recursion unit's z input: start it from zeros (it then stays bounded, y <- A x - y)
  HIP_TRY(launch_zero(y, (size_t)n_rhs * 32 * g.V * dsize(dtype), s));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HopConfig bestc = tune_hop(g, dtype, n_rhs, purpose);
  float bt = 1e30f;
  rmh_status st = RMH_OK;
  for (int form = 0; form < 3 && st == RMH_OK; ++form)
    for (int nv : {4, 2, 1})
    for (int ns : {1, 2, 4})
    for (int tile2 : {1, 2, 4})
    for (int block : {64, 128, 256})
    for (int walk : {0, 4, 8, 16})
    for (int order = 0; order < 4 && st == RMH_OK; ++order) {
      for (int xcd = 0; xcd < 2 && st == RMH_OK; ++xcd) {
        HopConfig c;
        c.form = form;
        c.block = block;
        c.xcd_remap = xcd;
        c.nv = nv;
        c.order = order;
        c.walk = walk;
        c.ns = ns;
        c.tile2 = tile2;
        if (hop_config_error(c, dtype)) continue;
        if (ns > 1 && n_rhs % ns) continue;
        if ((order == 1 || order == 3) && !hop_order_ok(g, c)) continue;
        if (walk && (order || !hop_walk_ok(g, c))) continue;
        tune_store(g, dtype, n_rhs, purpose, c, 0.0);
        auto unit = [&]() -> rmh_status {
          const hipError_t e =
              dtype == RMH_F64
                  ? tune_unit<double>(g, (const double*)U, (const double*)x, (double*)y, n_rhs, c, unit_kind,
                                      partials, dot_mask, s)
                  : tune_unit<float>(g, (const float*)U, (const float*)x, (float*)y, n_rhs, c, unit_kind,
                                     partials, dot_mask, s);
          return e == hipSuccess ? RMH_OK : fail(RMH_E_HIP, "stencil launch: %s", hipGetErrorString(e));
        };
        st = unit();  // warm-up
        if (st != RMH_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) st = fail(RMH_E_HIP, "hipEventRecord");
        for (int r = 0; r < reps && st == RMH_OK; ++r) st = unit();
        if (st != RMH_OK) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          st = fail(RMH_E_HIP, "hipEventRecord/Synchronize");
          break;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = 1e30f;
        ms /= reps;
        if (log_level() > 0)
          fprintf(stderr, "[rmh] tune L=%dx%dx%dx%d dtype=%d n=%d purpose=%d form=%d nv=%d ns=%d block=%d order=%d walk=%d tile2=%d xcd=%d: %.4f ms\n",
                  g.L0, g.L1, g.L2, g.L3, dtype, n_rhs, purpose, form, nv, ns, block, order, walk, tile2, xcd, ms);
        if (ms < bt) {
          bt = ms;
          bestc = c;
        }
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the candidates were stored one by one while they were timed: leave the best one measured (or,
  // after a failure before any was, the configuration looked up at the start) in the table
  tune_store(g, dtype, n_rhs, purpose, bestc, bt < 1e30f ? bt : 0.0);
  if (st != RMH_OK) return st;
  if (best) *best = to_abi(bestc);
  if (best_ms) *best_ms = bt;
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_profile_enable(int32_t enable) try {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  prof_flush_locked();
  g_prof.on = enable != 0;
  for (int c = 0; c < RMH_PROF_N; ++c) {
    g_prof.launches[c] = 0;
    g_prof.ms[c] = 0.0;
    g_prof.bytes[c] = 0.0;
    g_prof.items[c] = 0.0;
  }
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

rmh_status rmh_profile_read(int32_t cls, int64_t* launches, double* total_ms, double* total_bytes,
                            double* total_items) try {
  if (cls < 0 || cls >= RMH_PROF_N) return fail(RMH_E_ARG, "profile class %d out of range", cls);
  std::lock_guard<std::mutex> lk(g_prof.mu);
  prof_flush_locked();
  if (launches) *launches = g_prof.launches[cls];
  if (total_ms) *total_ms = g_prof.ms[cls];
  if (total_bytes) *total_bytes = g_prof.bytes[cls];
  if (total_items) *total_items = g_prof.items[cls];
  return RMH_OK;
} catch (...) {   // no C++ exception crosses the C ABI
  return fail(RMH_E_HOST, "host-side failure (out of host memory?)");
}

}  // extern "C"

// Stencil launch configuration cache.  Entries are keyed by lattice extents, dtype, the number of
// link fields per launch and the purpose of the launch (rmh_purpose); the autotuner
// (rmh_autotune_laplacian) fills them from timed candidates, rmh_tune_save / rmh_tune_load keep
// them in a JSON file stamped with the device architecture and the HIP runtime version, and
// otherwise the built-in defaults apply.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "rmh.h"
#include "rmh_tune.h"

namespace rmh {

namespace {
using Key = std::tuple<int32_t, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t>;  // L0..L3, dtype, n, purpose
struct Entry {
  HopConfig cfg;
  double ms;
};
std::mutex g_mu;
std::map<Key, Entry> g_cache;

Key key_of(const Geom& g, int32_t dtype, int32_t n_rhs, int32_t purpose) {
  return Key(g.L0, g.L1, g.L2, g.L3, dtype, n_rhs, purpose);
}

// Untuned defaults, from the sweeps of the autotuner on MI355X.  Lattices of a million sites and
// more: one thread per x0-x1-x2 column and all four directions, walking 8 consecutive x3 sites
// (fewest re-reads past L2: about 1.7 times the algorithmic reads in FP32, against 2.5 for one
// thread per site); a batch of fields below a million sites, when the batch gives every SIMD
// several waves: one thread per site, the adjoint matrix streamed two columns at a time; below
// that the hop-split shape (four lanes per site, one per direction), whose four times as many waves
// hide the memory latency that one thread per site leaves exposed when the lattice gives only a
// few waves per SIMD, except FP64 from 2^18 sites on, where one thread per site and direction pair
// in the x3-fastest order is as fast.
HopConfig defaults(const Geom& g, int32_t dtype, int32_t n_rhs) {
  HopConfig c;
  if (g.V < (1 << 20) && (int64_t)g.V * n_rhs >= (1 << 19)) {
    c.form = kFormStream;
    c.block = 64;
    c.xcd_remap = 1;
    c.nv = 4;
    c.walk = 0;
    c.order = 1;
    if (!hop_order_ok(g, c)) c.order = 0;
  } else if (g.V >= (1 << 20)) {
    c.form = dtype == RMH_F64 ? kFormStream : kFormAdjoint;
    c.block = dtype == RMH_F64 ? 128 : 256;
    c.xcd_remap = dtype == RMH_F64 ? 0 : 1;
    c.nv = 4;
    c.order = 0;
    c.walk = 0;
    for (int k : {8, 4, 16, 2})
      if (g.L3 % k == 0) {
        c.walk = k;
        break;
      }
  } else if (dtype == RMH_F64 && g.V >= (1 << 18)) {
    c.form = kFormMatrix;
    c.block = 256;
    c.xcd_remap = 1;
    c.nv = 2;
    c.walk = 0;
    c.order = 1;
    if (!hop_order_ok(g, c)) c.order = 0;
  } else {
    c.form = dtype == RMH_F64 ? kFormMatrix : kFormStream;
    c.block = dtype == RMH_F64 ? 128 : 256;
    c.xcd_remap = dtype == RMH_F64 ? 0 : 1;
    c.nv = dtype == RMH_F64 ? 2 : 4;
    c.walk = 0;
    c.order = 2;
  }
  return c;
}

// nearest batch size among the entries of (L, dtype, purpose)
const HopConfig* nearest(const Geom& g, int32_t dtype, int32_t n_rhs, int32_t purpose) {
  const HopConfig* best = nullptr;
  int32_t dist = 0;
  for (auto& kv : g_cache) {
    const Key& k = kv.first;
    if (std::get<0>(k) != g.L0 || std::get<1>(k) != g.L1 || std::get<2>(k) != g.L2 || std::get<3>(k) != g.L3 ||
        std::get<4>(k) != dtype || std::get<6>(k) != purpose)
      continue;
    const int32_t d = std::abs(std::get<5>(k) - n_rhs);
    if (!best || d < dist) {
      best = &kv.second.cfg;
      dist = d;
    }
  }
  return best;
}

// a configuration that was stored for another batch size keeps only what fits this one
HopConfig fit_batch(HopConfig c, int32_t n_rhs) {
  if (c.ns > 1 && n_rhs % c.ns) c.ns = 1;
  return c;
}
}  // namespace

const char* hop_config_error(const HopConfig& c, int32_t dtype) {
  if (c.form < kFormAdjoint || c.form > kFormStream) return "form must be 0, 1 or 2";
  if (c.block != 64 && c.block != 128 && c.block != 256) return "block must be 64, 128 or 256";
  if (c.nv != 1 && c.nv != 2 && c.nv != 4) return "nv must be 1, 2 or 4";
  if (c.nv == 1 && c.form != kFormMatrix) return "nv = 1 needs form 1 (3x3 products)";
  if ((c.block * c.nv / 4) % 64) return "block * nv / 4 must be a multiple of 64";
  if (c.order < 0 || c.order > 3) return "order must be 0, 1, 2 or 3";
  if (c.walk < 0 || c.walk > 64) return "walk must be in [0, 64]";
  if (c.xcd_remap != 0 && c.xcd_remap != 1) return "xcd_remap must be 0 or 1";
  if (c.ns != 1 && c.ns != 2 && c.ns != 4) return "ns must be 1, 2 or 4";
  if (c.tile2 != 1 && c.tile2 != 2 && c.tile2 != 4) return "tile2 must be 1, 2 or 4";
  if (c.tile2 > 1 && c.walk == 0) return "tile2 > 1 needs a walk";
  if (c.ns > 1) {
    if (c.nv != 4 || c.walk != 0 || c.order > 1 || c.form == kFormMatrix)
      return "ns > 1 needs nv = 4, form 0 or 2, order 0 or 1 and no walk";
    if (c.ns == 4 && dtype == RMH_F64) return "ns = 4 is FP32 only";
  }
  return nullptr;
}

HopConfig tune_hop(const Geom& g, int32_t dtype, int32_t n_rhs, int32_t purpose) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find(key_of(g, dtype, n_rhs, purpose));
  if (it != g_cache.end()) return it->second.cfg;
  it = g_cache.find(key_of(g, dtype, n_rhs, RMH_PURPOSE_ANY));
  if (it != g_cache.end()) return it->second.cfg;
  if (const HopConfig* c = nearest(g, dtype, n_rhs, purpose)) return fit_batch(*c, n_rhs);
  if (const HopConfig* c = nearest(g, dtype, n_rhs, RMH_PURPOSE_ANY)) return fit_batch(*c, n_rhs);
  return defaults(g, dtype, n_rhs);
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache.clear();
}

void tune_store(const Geom& g, int32_t dtype, int32_t n_rhs, int32_t purpose, const HopConfig& cfg, double ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[key_of(g, dtype, n_rhs, purpose)] = Entry{cfg, ms};
}

// ------------------------------------------------------------------------------------------
// JSON file: {"format": "rmh-tune-1", "arch": "...", "hip_runtime": N, "entries": [{...}, ...]}

static const char* kFields[] = {"L0", "L1", "L2", "L3", "dtype", "n_rhs", "purpose", "form", "block",
                                "xcd_remap", "nv", "order", "walk", "ns", "tile2"};
constexpr int kNumFields = 15;

int tune_save_file(const char* path, const std::string& arch, int32_t runtime, int32_t* n_saved) {
  std::lock_guard<std::mutex> lk(g_mu);
  FILE* f = fopen(path, "w");
  if (!f) return -1;
  fprintf(f, "{\"format\": \"rmh-tune-1\", \"arch\": \"%s\", \"hip_runtime\": %d, \"entries\": [", arch.c_str(),
          runtime);
  int n = 0;
  for (auto& kv : g_cache) {
    const Key& k = kv.first;
    const HopConfig& c = kv.second.cfg;
    const int32_t v[kNumFields] = {std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                                   std::get<5>(k), std::get<6>(k), c.form, c.block, c.xcd_remap, c.nv, c.order,
                                   c.walk, c.ns, c.tile2};
    fprintf(f, "%s\n  {", n ? "," : "");
    for (int i = 0; i < kNumFields; ++i) fprintf(f, "%s\"%s\": %d", i ? ", " : "", kFields[i], v[i]);
    fprintf(f, ", \"ms\": %.6g}", kv.second.ms);
    ++n;
  }
  fprintf(f, "\n]}\n");
  const bool ok = ferror(f) == 0;
  if (fclose(f) != 0 || !ok) return -1;
  if (n_saved) *n_saved = n;
  return 0;
}

// value of "name": <int> inside [b, e); false when absent or not an integer
static bool json_int(const char* b, const char* e, const char* name, long* out) {
  const std::string key = std::string("\"") + name + "\"";
  const char* p = b;
  while (p < e) {
    const char* q = strstr(p, key.c_str());
    if (!q || q >= e) return false;
    q += key.size();
    while (q < e && (*q == ' ' || *q == '\t' || *q == '\n' || *q == '\r')) ++q;
    if (q < e && *q == ':') {
      ++q;
      char* end = nullptr;
      const long v = strtol(q, &end, 10);
      if (end == q || end > e) return false;
      *out = v;
      return true;
    }
    p = q;
  }
  return false;
}

static bool json_str(const char* b, const char* e, const char* name, std::string* out) {
  const std::string key = std::string("\"") + name + "\"";
  const char* q = strstr(b, key.c_str());
  if (!q || q >= e) return false;
  q += key.size();
  while (q < e && *q != '"') {
    if (*q != ' ' && *q != ':' && *q != '\t' && *q != '\n' && *q != '\r') return false;
    ++q;
  }
  if (q >= e) return false;
  const char* s = ++q;
  while (q < e && *q != '"') ++q;
  if (q >= e) return false;
  out->assign(s, q);
  return true;
}

// 0: loaded (or skipped for another device/runtime), -1: unreadable, -2: malformed or invalid
int tune_load_file(const char* path, const std::string& arch, int32_t runtime, int32_t* n_loaded) {
  if (n_loaded) *n_loaded = 0;
  FILE* f = fopen(path, "rb");
  if (!f) return -1;
  std::string text;
  char buf[4096];
  size_t r;
  while ((r = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, r);
  const bool bad = ferror(f) != 0;
  fclose(f);
  if (bad) return -1;
  const char* b = text.c_str();
  const char* e = b + text.size();
  std::string fmt, farch;
  long frt = 0;
  if (!json_str(b, e, "format", &fmt) || fmt != "rmh-tune-1" || !json_str(b, e, "arch", &farch) ||
      !json_int(b, e, "hip_runtime", &frt))
    return -2;
  if (farch != arch || frt != runtime) return 0;
  const char* ent = strstr(b, "\"entries\"");
  if (!ent) return -2;
  const char* p = strchr(ent, '[');
  if (!p) return -2;
  // parse every entry first, store only if all are valid
  std::map<Key, Entry> add;
  for (;;) {
    const char* ob = strchr(p, '{');
    const char* close = strchr(p, ']');
    if (!ob || (close && close < ob)) break;
    const char* cb = strchr(ob, '}');
    if (!cb) return -2;
    long v[kNumFields];
    for (int i = 0; i < kNumFields; ++i)
      if (!json_int(ob, cb, kFields[i], &v[i])) return -2;
    HopConfig c;
    c.form = (int32_t)v[7];
    c.block = (int32_t)v[8];
    c.xcd_remap = (int32_t)v[9];
    c.nv = (int32_t)v[10];
    c.order = (int32_t)v[11];
    c.walk = (int32_t)v[12];
    c.ns = (int32_t)v[13];
    c.tile2 = (int32_t)v[14];
    const int32_t dtype = (int32_t)v[4];
    if ((dtype != RMH_F64 && dtype != RMH_F32) || v[5] < 1 || v[5] > (1L << 24) || v[6] < RMH_PURPOSE_ANY ||
        v[6] > RMH_PURPOSE_HEATBATH)
      return -2;
    for (int i = 0; i < 4; ++i)
      if (v[i] < 2 || v[i] > (1 << 20)) return -2;
    if (hop_config_error(c, dtype)) return -2;
    add[Key((int32_t)v[0], (int32_t)v[1], (int32_t)v[2], (int32_t)v[3], dtype, (int32_t)v[5], (int32_t)v[6])] =
        Entry{c, 0.0};
    p = cb + 1;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : add) g_cache[kv.first] = kv.second;
  if (n_loaded) *n_loaded = (int32_t)add.size();
  return 0;
}

}  // namespace rmh

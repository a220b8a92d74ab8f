// Stencil launch configuration cache.  Entries are keyed by lattice extents, dtype and
// the number of link fields per launch; the autotuner (rmh_autotune_laplacian) fills
// them from timed candidates, otherwise the defaults apply.  RMH_HOP_FORM (0 adjoint,
// 1 matrix, 2 streamed adjoint) and RMH_HOP_BLOCK override the defaults for experiments.
#include <stdlib.h>

#include <cstdlib>

#include <map>
#include <mutex>
#include <tuple>

#include "rmh.h"
#include "rmh_tune.h"

namespace rmh {

namespace {
using Key = std::tuple<int32_t, int32_t, int32_t, int32_t, int32_t, int32_t>;
std::mutex g_mu;
std::map<Key, HopConfig> g_cache;

Key key_of(const Geom& g, int32_t dtype, int32_t n_rhs) {
  return Key(g.L0, g.L1, g.L2, g.L3, dtype, n_rhs);
}

// Untuned defaults, from the sweeps of the autotuner: on lattices of a million sites and more
// the x3-walking kernel with four directions per thread (the streamed form in FP64, the
// materialised adjoint matrix in FP32); below that the hop-split shape (four lanes per site, one
// per direction), whose four times as many waves hide the memory latency that one thread per
// site leaves exposed when the lattice gives only a few waves per SIMD, except FP64 from 2^18
// sites on, where one thread per site and direction pair in the x3-fastest order is as fast.
HopConfig defaults(const Geom& g, int32_t dtype, int32_t n_rhs) {
  HopConfig c;
  if (g.V < (1 << 20) && (int64_t)g.V * n_rhs >= (1 << 19)) {
    // a batch of fields already gives every SIMD several waves: one thread per site and all four
    // directions, the adjoint matrix streamed two columns at a time and shared by them
    c.form = kFormStream;
    c.block = 64;
    c.xcd_remap = 1;
    c.nv = 4;
    c.walk = 0;
    c.order = 1;
    if (!hop_order_ok(g, c)) c.order = 0;
  } else if (g.V >= (1 << 20)) {
    c.form = dtype == RMH_F64 ? kFormStream : kFormAdjoint;
    c.block = 128;
    c.xcd_remap = 0;
    c.nv = 4;
    c.order = 0;
    c.walk = 0;
    const int32_t P = g.V / g.L3;
    const int32_t cpb = c.block * c.nv / 4;
    for (int k : {16, 8, 4, 2}) {
      if (g.L3 % k) continue;
      if ((int64_t)((P + cpb - 1) / cpb) * (g.L3 / k) >= 1024) {
        c.walk = k;
        break;
      }
    }
  } else if (dtype == RMH_F64 && g.V >= (1 << 18)) {
    // one thread per site and direction pair, 3x3 products, x3-fastest block order
    c.form = kFormMatrix;
    c.block = 256;
    c.xcd_remap = 1;
    c.nv = 2;
    c.walk = 0;
    c.order = 1;
    if (!hop_order_ok(g, c)) c.order = 0;
  } else {
    // the hop-split shape: four lanes per site
    c.form = dtype == RMH_F64 ? kFormMatrix : kFormStream;
    c.block = dtype == RMH_F64 ? 128 : 256;
    c.xcd_remap = dtype == RMH_F64 ? 0 : 1;
    c.nv = dtype == RMH_F64 ? 2 : 4;
    c.walk = 0;
    c.order = 2;
  }
  if (const char* e = getenv("RMH_HOP_FORM")) c.form = atoi(e);
  if (const char* e = getenv("RMH_HOP_BLOCK")) {
    const int b = atoi(e);
    if (b == 64 || b == 128 || b == 256) c.block = b;
  }
  return c;
}
}  // namespace

HopConfig tune_hop(const Geom& g, int32_t dtype, int32_t n_rhs, int32_t /*purpose*/) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find(key_of(g, dtype, n_rhs));
  if (it != g_cache.end()) return it->second;
  // else the entry of this lattice and dtype with the nearest batch size
  const HopConfig* best = nullptr;
  int32_t dist = 0;
  for (auto& kv : g_cache) {
    const Key& k = kv.first;
    if (std::get<0>(k) != g.L0 || std::get<1>(k) != g.L1 || std::get<2>(k) != g.L2 || std::get<3>(k) != g.L3 ||
        std::get<4>(k) != dtype)
      continue;
    const int32_t d = std::abs(std::get<5>(k) - n_rhs);
    if (!best || d < dist) {
      best = &kv.second;
      dist = d;
    }
  }
  return best ? *best : defaults(g, dtype, n_rhs);
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache.clear();
}

void tune_store(const Geom& g, int32_t dtype, int32_t n_rhs, const HopConfig& cfg) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[key_of(g, dtype, n_rhs)] = cfg;
}

}  // namespace rmh

// The adjoint-Laplacian stencil for gfx950: one hop per direction and sign, fused epilogues
// (axpby, dot products), the site-per-thread kernel, the hop-split kernel and the
// x3-walking kernel, and their launch dispatch.  Every kernel writes its output with
// non-temporal stores (and reads a per-field z input with non-temporal loads): neither is touched
// again in the launch, and streaming them past the L2 leaves that cache to the neighbour fields
// and links the blocks share.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "rmh_internal.h"
#include "rmh_reduce.h"

namespace rmh {

// ------------------------------------------------------------------------------------------
// the stencil

// Block -> (field v, lattice block lb). The grid is one-dimensional, nblk lattice blocks times
// n_rhs fields, taken in groups of fg fields (the largest divisor of n_rhs up to 4): within a
// group the fields are fastest, so consecutive blocks take the same sites of successive fields
// and a link loaded for the first is an L2 hit for the others (with the XCD remap each XCD owns
// a contiguous range); the groups are not interleaved, which keeps the neighbour fields of at
// most fg fields in the L2 at a time.
struct HopBlock {
  int32_t v, lb, nblk;
};
__host__ __device__ __forceinline__ int32_t hop_field_group(int32_t n_rhs) {
  for (int32_t f = 4; f > 1; --f)
    if (n_rhs % f == 0) return f;
  return 1;
}
__device__ __forceinline__ HopBlock hop_block(int32_t xcd, int32_t n_rhs) {
  const int32_t b = remap_block(blockIdx.x, gridDim.x, xcd);
  const int32_t fg = hop_field_group(n_rhs);
  HopBlock h;
  h.nblk = gridDim.x / n_rhs;
  const int32_t gsize = h.nblk * fg;   // blocks per field group
  const int32_t grp = b / gsize, r = b - grp * gsize;
  h.v = grp * fg + r % fg;
  h.lb = r / fg;
  return h;
}

// One hop's contribution to NV vectors: forward (kT = false, link U_mu(x), neighbour x+mu) or
// backward (kT = true, link U_mu(x-mu), neighbour x-mu).
template <typename T, int FORM, int NV, bool kT>
__device__ __forceinline__ void hop_apply(const T* u, const T (*phi)[8], T (*acc)[8]) {
  if (FORM == kFormAdjoint) {
    T R[64];
    adjoint_matrix<T>(u, R);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (!kT)
        adj_apply<T>(R, phi[v], acc[v]);
      else
        adj_apply_t<T>(R, phi[v], acc[v]);
    }
  } else if (FORM == kFormMatrix) {
#pragma unroll
    for (int v = 0; v < NV; ++v) mat_hop<T, kT>(u, phi[v], acc[v]);
  } else {
    adj_stream<T, NV, kT>(u, phi, acc);
  }
}

// An element of the z input: read once when each field has its own z (z_div = 1), so it is loaded
// non-temporally and does not take L2 space from the neighbour fields; a z shared by several
// fields (z_div > 1) is loaded normally for the others to hit.
template <typename T>
__device__ __forceinline__ T load_z(const T* p, bool once) {
  return once ? __builtin_nontemporal_load(p) : *p;
}

// The link at site s (component c at Um[c V + s]): rows 0 and 1 are loaded, row 2 is rebuilt
// from them (SU(3)), so a hop moves 12 link reals instead of 18.
template <typename T>
__device__ __forceinline__ void load_link(const T* __restrict__ Um, int32_t s, int32_t V, T (&u)[18]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) u[c] = (Um + (size_t)c * V)[s];
  su3_row2<T>(u);
}

// out[v] = a (H x)[v] + b x[v] + c z[v]: a block of B threads covers B * NV / 4 sites; the
// 4 / NV thread groups of a site (direction subsets) are wave-aligned slices of the block.
// One backward hop: link and field both read at the neighbour site sb.
template <typename T, int FORM, int NV, bool kT>
__device__ __forceinline__ void hop_term(const T* __restrict__ Um, int32_t sb, const T* __restrict__ xf,
                                         int nu0, int32_t V, T (&acc)[NV][8]) {
  T u[18], phi[NV][8];
  load_link<T>(Um, sb, V, u);
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int b = 0; b < 8; ++b) phi[i][b] = (xf + (size_t)((nu0 + i) * 8 + b) * V)[sb];
  hop_apply<T, FORM, NV, kT>(u, phi, acc);
}

// One forward hop: link at s, field at the neighbour sf.
template <typename T, int FORM, int NV>
__device__ __forceinline__ void hop_term_fwd(const T* __restrict__ Um, int32_t s, int32_t sf,
                                             const T* __restrict__ xf, int nu0, int32_t V,
                                             T (&acc)[NV][8]) {
  T u[18], phi[NV][8];
  load_link<T>(Um, s, V, u);
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int b = 0; b < 8; ++b) phi[i][b] = (xf + (size_t)((nu0 + i) * 8 + b) * V)[sf];
  hop_apply<T, FORM, NV, false>(u, phi, acc);
}

template <typename T, int FORM, int NV, bool DOTS>
__global__ void __launch_bounds__(256) k_hop(const HopArgs<T> A, int32_t xcd, int32_t order) {
  constexpr int G = 4 / NV;  // thread groups per site
  const HopBlock hb = hop_block(xcd, A.n_rhs);
  const int32_t v = hb.v;
  if (A.run && A.run[(int64_t)v * A.run_stride] == 0) return;
  const int32_t V = A.g.V;
  const int32_t lb = hb.lb;
  const int32_t spb = blockDim.x / G;              // sites per block
  // direction subset of this thread: wave-uniform (spb is a multiple of the wave size), so the
  // per-component base addresses stay in scalar registers
  const int32_t grp = __builtin_amdgcn_readfirstlane(threadIdx.x / spb);
  int32_t blk = lb;
  if (order) {
    // lb = ((chunk * L2) + x2) * L3 + x3  ->  lexicographic block of that (x0 x1 chunk, x2, x3)
    const int32_t x3 = lb % A.g.L3;
    const int32_t t = lb / A.g.L3;
    const int32_t x2 = t % A.g.L2;
    const int32_t chunk = t / A.g.L2;
    const int32_t cpp = (A.g.L0 * A.g.L1) / spb;   // chunks per (x2, x3) plane
    blk = (x3 * A.g.L2 + x2) * cpp + chunk;
  }
  const int32_t s = blk * spb + (threadIdx.x - grp * spb);
  const int nu0 = grp * NV;
  double dsum[3] = {0.0, 0.0, 0.0};
  if (s < V) {
    const int64_t FV = 32 * (int64_t)V;
    const T* __restrict__ xf = A.x + ((int64_t)v * A.x_mul + A.x_add) * FV;
    const T* __restrict__ U = A.U;
    T acc[NV][8];
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int a = 0; a < 8; ++a) acc[i][a] = T(0);
    int32_t xc[4];
    site_coords(A.g, s, xc);
    // term order (shared with k_hop_walk, so every launch shape rounds alike): the x3
    // backward hop, the x0, x1, x2 forward and backward hops, the x3 forward hop
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      const int mb = (mu + 3) & 3;   // backward hop of the previous direction, x3 first
      hop_term<T, FORM, NV, true>(U + (int64_t)mb * 18 * V, site_shift(A.g, s, xc, mb, -1), xf, nu0, V, acc);
      hop_term_fwd<T, FORM, NV>(U + (int64_t)mu * 18 * V, s, site_shift(A.g, s, xc, mu, +1), xf, nu0, V, acc);
    }
    // epilogue: out = a H x + b x + c z
    const T ca = T(A.a);
    const T cb = T(A.b_rhs ? A.b_rhs[v] : A.b);
    const T cc = T(A.c);
    const T* zf = A.z ? A.z + (int64_t)(v / A.z_div) * FV : nullptr;  // may alias out
    T* outf = A.out + (int64_t)v * FV;
    // per direction: the 8 z values are loaded before any of the 8 stores (z may be the output
    // itself, each element read and written by this thread only), so those loads overlap
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int64_t e0 = (int64_t)((nu0 + i) * 8) * V + s;
      T xs[8], zv[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        xs[a] = xf[e0 + (int64_t)a * V];
        zv[a] = zf ? load_z(&zf[e0 + (int64_t)a * V], A.z_div == 1) : T(0);
      }
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int64_t e = e0 + (int64_t)a * V;
        const T xv = xs[a];
        T o = fmadd(ca, acc[i][a], cb * xv);
        if (zf) o = fmadd(cc, zv[a], o);
        if (A.store) __builtin_nontemporal_store(o, &outf[e]);
        if (DOTS) {
          const double xd = (double)xv, od = (double)o;
          dsum[0] = fma(xd, xd, dsum[0]);
          dsum[1] = fma(od, xd, dsum[1]);
          dsum[2] = fma(od, od, dsum[2]);
        }
      }
    }
  }
  if (DOTS) {
    __shared__ double lds[3][16];
    block_sum<3>(dsum, lds);
    if (threadIdx.x == 0) {
      const int32_t nblk = hb.nblk;
      double* p = A.partials + (int64_t)v * 3 * nblk + lb;
      if (A.dot_mask & 1) p[0] = dsum[0];
      if (A.dot_mask & 2) p[nblk] = dsum[1];
      if (A.dot_mask & 4) p[2 * nblk] = dsum[2];
    }
  }
}

// Hop-split variant of k_hop for lattices too small to fill the chip with one thread per site:
// the four lanes l, l+16, l+32, l+48 of a wave share a site, lane group mu doing the forward and the
// backward hop along mu; two butterfly shuffles sum the four partial results (in the fixed order
// (mu0 + mu1) + (mu2 + mu3)), and each of the four lanes stores a quarter of the components.  A wave
// covers 16 consecutive sites for one direction group; a block of B threads has B/64 waves.
template <typename T, int FORM, int NV, bool DOTS>
__global__ void __launch_bounds__(256) k_hop_split(const HopArgs<T> A, int32_t xcd, int32_t order) {
  constexpr int G = 4 / NV;
  const HopBlock hb = hop_block(xcd, A.n_rhs);
  const int32_t v = hb.v;
  if (A.run && A.run[(int64_t)v * A.run_stride] == 0) return;
  const int32_t V = A.g.V;
  const int32_t lb = hb.lb;
  const int32_t wi = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int32_t W = blockDim.x >> 6;
  const int32_t grp = wi % G;   // wave-uniform direction group
  const int32_t spb = (W / G) * 16;
  const int32_t lane = threadIdx.x & 63;
  const int32_t mu = lane >> 4;
  int32_t blk = lb;
  if (order) {
    // x3 fastest, then x2, then the (x0, x1) chunks: a contiguous range of blocks (one XCD's,
    // with the remap) sweeps whole x3 columns of a few chunks, so the x3 and x2 neighbours of a
    // block were loaded moments before by the same XCD
    const int32_t x3 = lb % A.g.L3;
    const int32_t t = lb / A.g.L3;
    const int32_t x2 = t % A.g.L2;
    const int32_t chunk = t / A.g.L2;
    const int32_t cpp = (A.g.L0 * A.g.L1) / spb;
    blk = (x3 * A.g.L2 + x2) * cpp + chunk;
  }
  const int32_t s = blk * spb + (wi / G) * 16 + (lane & 15);
  const int nu0 = grp * NV;
  const bool live = s < V;
  const int64_t FV = 32 * (int64_t)V;
  const T* __restrict__ xf = A.x + ((int64_t)v * A.x_mul + A.x_add) * FV;
  T acc[NV][8];
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int a = 0; a < 8; ++a) acc[i][a] = T(0);
  if (live) {
    int32_t xc[4];
    site_coords(A.g, s, xc);
    const T* __restrict__ Um = A.U + (int64_t)mu * 18 * V;
    hop_term<T, FORM, NV, true>(Um, site_shift(A.g, s, xc, mu, -1), xf, nu0, V, acc);
    hop_term_fwd<T, FORM, NV>(Um, s, site_shift(A.g, s, xc, mu, +1), xf, nu0, V, acc);
  }
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      acc[i][a] += __shfl_xor(acc[i][a], 16, 64);
      acc[i][a] += __shfl_xor(acc[i][a], 32, 64);
    }
  // lane group mu keeps the components 4q + mu of its direction group (q < 2 NV), picked with
  // bit masks (a select chain here tends to become a lane-indexed array in scratch), then one
  // full-wave load/store per q; every z value is loaded before the first store (z may be the
  // output itself, each element read and written by this lane only), so those loads overlap
  double dsum[3] = {0.0, 0.0, 0.0};
  if (live) {
    const T ca = T(A.a);
    const T cb = T(A.b_rhs ? A.b_rhs[v] : A.b);
    const T cc = T(A.c);
    const T* zf = A.z ? A.z + (int64_t)(v / A.z_div) * FV : nullptr;  // may alias out
    T* outf = A.out + (int64_t)v * FV;
    using Bits = typename std::conditional<sizeof(T) == 8, uint64_t, uint32_t>::type;
    const Bits m0 = mu == 0 ? ~Bits(0) : Bits(0), m1 = mu == 1 ? ~Bits(0) : Bits(0);
    const Bits m2 = mu == 2 ? ~Bits(0) : Bits(0), m3 = mu == 3 ? ~Bits(0) : Bits(0);
    T hs[2 * NV], xs[2 * NV], zv[2 * NV];
#pragma unroll
    for (int q = 0; q < 2 * NV; ++q) {
      const int i = q >> 1, a0 = (q & 1) * 4;
      const Bits hb_ = (m0 & __builtin_bit_cast(Bits, acc[i][a0])) | (m1 & __builtin_bit_cast(Bits, acc[i][a0 + 1])) |
                       (m2 & __builtin_bit_cast(Bits, acc[i][a0 + 2])) | (m3 & __builtin_bit_cast(Bits, acc[i][a0 + 3]));
      hs[q] = __builtin_bit_cast(T, hb_);
      const int64_t e = (int64_t)(nu0 * 8 + 4 * q + mu) * V + s;
      xs[q] = xf[e];
      zv[q] = zf ? load_z(&zf[e], A.z_div == 1) : T(0);
    }
#pragma unroll
    for (int q = 0; q < 2 * NV; ++q) {
      const T h = hs[q];
      const int64_t e = (int64_t)(nu0 * 8 + 4 * q + mu) * V + s;
      const T xv = xs[q];
      T o = fmadd(ca, h, cb * xv);
      if (zf) o = fmadd(cc, zv[q], o);
      if (A.store) __builtin_nontemporal_store(o, &outf[e]);
      if (DOTS) {
        const double xd = (double)xv, od = (double)o;
        dsum[0] = fma(xd, xd, dsum[0]);
        dsum[1] = fma(od, xd, dsum[1]);
        dsum[2] = fma(od, od, dsum[2]);
      }
    }
  }
  if (DOTS) {
    __shared__ double lds[3][16];
    block_sum<3>(dsum, lds);
    if (threadIdx.x == 0) {
      const int32_t nblk = hb.nblk;
      double* p = A.partials + (int64_t)v * 3 * nblk + lb;
      if (A.dot_mask & 1) p[0] = dsum[0];
      if (A.dot_mask & 2) p[nblk] = dsum[1];
      if (A.dot_mask & 4) p[2 * nblk] = dsum[2];
    }
  }
}

// Waves per SIMD the walking kernel is compiled for.  The FP32 3x3-form walk over all four
// directions needs about 170 registers left to itself (two waves per SIMD); capped at 168 it keeps
// three waves, and its batched Chebyshev sweeps ran 4-5 % faster (they move fewer bytes than one
// thread per site but were latency-bound at two waves).  Under the cap the variant with the fused
// dot products (the sweeps, the CG) does not spill; the plain one spills about 130 B per lane since
// the x0 hops take their neighbours from other lanes.  The other walks keep the compiler's choice
// (FP64 and the 8x8 forms do not fit three waves without spilling).
template <typename T, int FORM, int NV>
constexpr int hop_walk_waves() {
  return (sizeof(T) == 4 && FORM == kFormMatrix && NV == 4) ? 3 : 1;
}

// Walking variant of k_hop: a block of B threads covers B * NV / 4 columns (x0, x1, x2) of the
// lattice; each thread walks K consecutive x3 values of its column.  Per step the x1 and x2 hops
// load their links and neighbours as in k_hop, the x0 hops too unless lane_x0 (then they take the
// neighbours from the other lanes of the x0 row); the x3 forward hop loads U_3(x) and phi(x+3),
// which stay in registers as the backward link and the centre field of the next step.
template <typename T, int FORM, int NV, bool DOTS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(hop_walk_waves<T, FORM, NV>())))
k_hop_walk(const HopArgs<T> A, int32_t xcd, int32_t K, int32_t tile2, int32_t lane_x0) {
  constexpr int G = 4 / NV;
  const HopBlock hb = hop_block(xcd, A.n_rhs);
  const int32_t v = hb.v;
  if (A.run && A.run[(int64_t)v * A.run_stride] == 0) return;
  const int32_t V = A.g.V;
  const int32_t P = A.g.L0 * A.g.L1 * A.g.L2;            // sites per x3 plane
  const int32_t cpb = blockDim.x / G;                    // columns per block
  const int32_t nchunk = (P + cpb - 1) / cpb;
  const int32_t lb = hb.lb;
  const int32_t chunk = lb % nchunk;
  const int32_t x3_0 = (lb / nchunk) * K;
  const int32_t grp = __builtin_amdgcn_readfirstlane(threadIdx.x / cpb);  // wave-uniform
  const int32_t tc = threadIdx.x - grp * cpb;
  int32_t col;
  if (tile2 > 1) {
    // the block's columns form an L0 x R1 x tile2 tile of the (x0, x1, x2) plane (tiles with x1
    // fastest), so its x2 neighbours are partly its own columns; hop_walk_ok checks the tiling
    const int32_t R1 = cpb / (A.g.L0 * tile2);
    const int32_t nc1 = A.g.L1 / R1;
    const int32_t c1 = chunk % nc1, c2 = chunk / nc1;
    const int32_t x0 = tc % A.g.L0, r = tc / A.g.L0;
    col = x0 + A.g.L0 * ((c1 * R1 + r % R1) + A.g.L1 * (c2 * tile2 + r / R1));
  } else {
    col = chunk * cpb + tc;
  }
  const int nu0 = grp * NV;
  double dsum[3] = {0.0, 0.0, 0.0};
  if (col < P) {
    const int64_t FV = 32 * (int64_t)V;
    const T* __restrict__ xf = A.x + ((int64_t)v * A.x_mul + A.x_add) * FV;
    const T* __restrict__ U = A.U;
    const T* __restrict__ U3 = U + (int64_t)3 * 18 * V;
    const T ca = T(A.a);
    const T cb = T(A.b_rhs ? A.b_rhs[v] : A.b);
    const T cc = T(A.c);
    const T* zf = A.z ? A.z + (int64_t)(v / A.z_div) * FV : nullptr;  // may alias out
    T* outf = A.out + (int64_t)v * FV;
    int32_t xc[4];
    site_coords(A.g, col + x3_0 * P, xc);
    // carried state: the centre field, the x-3 field and the 12 loaded reals of the link U_3(x-3)
    // (this thread's forward x3 link of the step before; row 2 is rebuilt from them each step)
    T cen[NV][8], bwd[NV][8], l3[12];
    {
      const int32_t s0 = col + x3_0 * P;
      const int32_t sb = (x3_0 == 0) ? s0 + (A.g.L3 - 1) * P : s0 - P;
#pragma unroll
      for (int c = 0; c < 12; ++c) l3[c] = (U3 + (size_t)c * V)[sb];
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          cen[i][b] = (xf + (size_t)((nu0 + i) * 8 + b) * V)[s0];
          bwd[i][b] = (xf + (size_t)((nu0 + i) * 8 + b) * V)[sb];
        }
    }
#pragma unroll 1
    for (int32_t t = 0; t < K; ++t) {
      const int32_t x3 = x3_0 + t;
      const int32_t s = col + x3 * P;
      xc[3] = x3;
      T acc[NV][8];
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int a = 0; a < 8; ++a) acc[i][a] = T(0);
      // x3 backward hop: carried field, link U_3(x - 3)
      {
        T u[18];
#pragma unroll
        for (int c = 0; c < 12; ++c) u[c] = l3[c];
        su3_row2<T>(u);
        hop_apply<T, FORM, NV, true>(u, bwd, acc);
      }
      int32_t mu_begin = 0;
      if (lane_x0) {
        // x0 hops from the other lanes of this x0 row (a row of L0 lanes lies within the wave):
        // the field at x +- 0 is that lane's carried centre, and the backward link U_0(x - 0) is
        // the forward link that lane loads, passed as its 12 loaded reals (row 2 rebuilt here, as
        // load_link does) -- the same values the loads would give, in the same order of terms
        const int32_t lane = threadIdx.x & 63;
        const int32_t x0 = xc[0];
        const int32_t row = lane - x0;
        const int32_t lp = row + (x0 + 1 == A.g.L0 ? 0 : x0 + 1);
        const int32_t lm = row + (x0 == 0 ? A.g.L0 - 1 : x0 - 1);
        T u[18], u12[12], phi[NV][8];
#pragma unroll
        for (int c = 0; c < 12; ++c) u12[c] = (U + (size_t)c * V)[s];
#pragma unroll
        for (int c = 0; c < 12; ++c) u[c] = u12[c];
        su3_row2<T>(u);
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
          for (int b = 0; b < 8; ++b) phi[i][b] = __shfl(cen[i][b], lp, 64);
        hop_apply<T, FORM, NV, false>(u, phi, acc);
#pragma unroll
        for (int c = 0; c < 12; ++c) u[c] = __shfl(u12[c], lm, 64);
        su3_row2<T>(u);
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
          for (int b = 0; b < 8; ++b) phi[i][b] = __shfl(cen[i][b], lm, 64);
        hop_apply<T, FORM, NV, true>(u, phi, acc);
        mu_begin = 1;
      }
#pragma unroll 1
      for (int mu = mu_begin; mu < 3; ++mu) {
        const T* __restrict__ Um = U + (int64_t)mu * 18 * V;
        hop_term_fwd<T, FORM, NV>(Um, s, site_shift(A.g, s, xc, mu, +1), xf, nu0, V, acc);
        hop_term<T, FORM, NV, true>(Um, site_shift(A.g, s, xc, mu, -1), xf, nu0, V, acc);
      }
      // x3 forward hop: phi(x + 3) becomes the centre of the next step
      T fwd[NV][8];
      {
        const int32_t sf = (x3 == A.g.L3 - 1) ? s - (A.g.L3 - 1) * P : s + P;
        T u[18];
#pragma unroll
        for (int c = 0; c < 12; ++c) l3[c] = (U3 + (size_t)c * V)[s];
#pragma unroll
        for (int c = 0; c < 12; ++c) u[c] = l3[c];
        su3_row2<T>(u);
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
          for (int b = 0; b < 8; ++b) fwd[i][b] = (xf + (size_t)((nu0 + i) * 8 + b) * V)[sf];
        hop_apply<T, FORM, NV, false>(u, fwd, acc);
      }
      // epilogue
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        // the 8 z values before the 8 stores (z may be the output itself, element by element)
        const int64_t e0 = (int64_t)((nu0 + i) * 8) * V + s;
        T zv[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) zv[a] = zf ? load_z(&zf[e0 + (int64_t)a * V], A.z_div == 1) : T(0);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int64_t e = e0 + (int64_t)a * V;
          const T xv = cen[i][a];
          T o = fmadd(ca, acc[i][a], cb * xv);
          if (zf) o = fmadd(cc, zv[a], o);
          if (A.store) __builtin_nontemporal_store(o, &outf[e]);
          if (DOTS) {
            const double xd = (double)xv, od = (double)o;
            dsum[0] = fma(xd, xd, dsum[0]);
            dsum[1] = fma(od, xd, dsum[1]);
            dsum[2] = fma(od, od, dsum[2]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          bwd[i][b] = cen[i][b];
          cen[i][b] = fwd[i][b];
        }
    }
  }
  if (DOTS) {
    __shared__ double lds[3][16];
    block_sum<3>(dsum, lds);
    if (threadIdx.x == 0) {
      const int32_t nblk = hb.nblk;
      double* p = A.partials + (int64_t)v * 3 * nblk + lb;
      if (A.dot_mask & 1) p[0] = dsum[0];
      if (A.dot_mask & 2) p[nblk] = dsum[1];
      if (A.dot_mask & 4) p[2 * nblk] = dsum[2];
    }
  }
}


// Multi-field variant of k_hop (one thread per site, all four directions): the thread applies the
// operator at its site to NS consecutive fields of the batch.  The grid is lattice blocks times field
// groups of NS, laid out as hop_block lays out fields.  Per hop the link is loaded once and its
// adjoint matrix built once for all 4 NS vectors: form 0 keeps the 8x8 matrix in registers and
// streams the fields through it one at a time (registers: the matrix, one field, the NS
// accumulators); form 2 builds each column pair once and applies it to all 4 NS vectors.  Term order
// and per-vector arithmetic are those of k_hop, so every field's result is bitwise that of k_hop with
// the same form.
template <typename T, int FORM, int NS, bool kT>
__device__ __forceinline__ void hop_term_ns(const T* __restrict__ Um, int32_t sl, int32_t sn,
                                            const T* const (&xf)[NS], int32_t V, T (&acc)[NS * 4][8]) {
  T u[18];
  load_link<T>(Um, sl, V, u);
  if (FORM == kFormAdjoint) {
    T R[64];
    adjoint_matrix<T>(u, R);
#pragma unroll
    for (int f = 0; f < NS; ++f) {
      T phi[4][8];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < 8; ++b) phi[i][b] = (xf[f] + (size_t)(i * 8 + b) * V)[sn];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (!kT)
          adj_apply<T>(R, phi[i], acc[f * 4 + i]);
        else
          adj_apply_t<T>(R, phi[i], acc[f * 4 + i]);
      }
    }
  } else {
    T phi[NS * 4][8];
#pragma unroll
    for (int f = 0; f < NS; ++f)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < 8; ++b) phi[f * 4 + i][b] = (xf[f] + (size_t)(i * 8 + b) * V)[sn];
    adj_stream<T, NS * 4, kT>(u, phi, acc);
  }
}

template <typename T, int FORM, int NS, bool DOTS>
__global__ void __launch_bounds__(256) k_hop_ns(const HopArgs<T> A, int32_t xcd, int32_t order) {
  const int32_t ngrp = A.n_rhs / NS;
  const HopBlock hb = hop_block(xcd, ngrp);
  const int32_t v0 = hb.v * NS;
  bool runs[NS];
  bool any = false;
#pragma unroll
  for (int f = 0; f < NS; ++f) {
    runs[f] = !A.run || A.run[(int64_t)(v0 + f) * A.run_stride] != 0;
    any = any || runs[f];
  }
  if (!any) return;
  const int32_t V = A.g.V;
  const int32_t lb = hb.lb;
  const int32_t spb = blockDim.x;
  int32_t blk = lb;
  if (order) {
    const int32_t x3 = lb % A.g.L3;
    const int32_t t = lb / A.g.L3;
    const int32_t x2 = t % A.g.L2;
    const int32_t chunk = t / A.g.L2;
    const int32_t cpp = (A.g.L0 * A.g.L1) / spb;
    blk = (x3 * A.g.L2 + x2) * cpp + chunk;
  }
  const int32_t s = blk * spb + threadIdx.x;
  double dsum[NS * 3];
#pragma unroll
  for (int q = 0; q < NS * 3; ++q) dsum[q] = 0.0;
  if (s < V) {
    const int64_t FV = 32 * (int64_t)V;
    const T* xf[NS];
#pragma unroll
    for (int f = 0; f < NS; ++f) xf[f] = A.x + ((int64_t)(v0 + f) * A.x_mul + A.x_add) * FV;
    const T* __restrict__ U = A.U;
    T acc[NS * 4][8];
#pragma unroll
    for (int i = 0; i < NS * 4; ++i)
#pragma unroll
      for (int a = 0; a < 8; ++a) acc[i][a] = T(0);
    int32_t xc[4];
    site_coords(A.g, s, xc);
    // the term order of k_hop: x3 backward, then x0, x1, x2 forward and backward, x3 forward
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      const int mb = (mu + 3) & 3;
      const int32_t sb = site_shift(A.g, s, xc, mb, -1);
      hop_term_ns<T, FORM, NS, true>(U + (int64_t)mb * 18 * V, sb, sb, xf, V, acc);
      hop_term_ns<T, FORM, NS, false>(U + (int64_t)mu * 18 * V, s, site_shift(A.g, s, xc, mu, +1), xf, V, acc);
    }
    const T ca = T(A.a);
    const T cc = T(A.c);
#pragma unroll
    for (int f = 0; f < NS; ++f) {
      const int32_t v = v0 + f;
      const T cb = T(A.b_rhs ? A.b_rhs[v] : A.b);
      const T* zf = A.z ? A.z + (int64_t)(v / A.z_div) * FV : nullptr;  // may alias out
      T* outf = A.out + (int64_t)v * FV;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t e0 = (int64_t)(i * 8) * V + s;
        T xs[8], zv[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          xs[a] = xf[f][e0 + (int64_t)a * V];
          zv[a] = zf ? load_z(&zf[e0 + (int64_t)a * V], A.z_div == 1) : T(0);
        }
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int64_t e = e0 + (int64_t)a * V;
          const T xv = xs[a];
          T o = fmadd(ca, acc[f * 4 + i][a], cb * xv);
          if (zf) o = fmadd(cc, zv[a], o);
          if (A.store && runs[f]) __builtin_nontemporal_store(o, &outf[e]);
          if (DOTS) {
            const double xd = (double)xv, od = (double)o;
            dsum[f * 3 + 0] = fma(xd, xd, dsum[f * 3 + 0]);
            dsum[f * 3 + 1] = fma(od, xd, dsum[f * 3 + 1]);
            dsum[f * 3 + 2] = fma(od, od, dsum[f * 3 + 2]);
          }
        }
      }
    }
  }
  if (DOTS) {
    __shared__ double lds[NS * 3][16];
    block_sum<NS * 3>(dsum, lds);
    if (threadIdx.x == 0) {
      const int32_t nblk = hb.nblk;
#pragma unroll
      for (int f = 0; f < NS; ++f) {
        if (!runs[f]) continue;
        double* p = A.partials + (int64_t)(v0 + f) * 3 * nblk + lb;
        if (A.dot_mask & 1) p[0] = dsum[f * 3 + 0];
        if (A.dot_mask & 2) p[nblk] = dsum[f * 3 + 1];
        if (A.dot_mask & 4) p[2 * nblk] = dsum[f * 3 + 2];
      }
    }
  }
}

int hop_walk_ok(const Geom& g, const HopConfig& cfg) {
  if (!(cfg.walk > 0 && (g.L3 % cfg.walk) == 0)) return 0;
  if (cfg.tile2 > 1) {
    // an L0 x R1 x tile2 column tile per block that tiles the (x0, x1, x2) plane exactly
    const int cpb = cfg.block * cfg.nv / 4;
    if (cpb % (g.L0 * cfg.tile2) || g.L2 % cfg.tile2) return 0;
    const int R1 = cpb / (g.L0 * cfg.tile2);
    if (R1 < 1 || g.L1 % R1) return 0;
  }
  return 1;
}

int hop_ns_ok(const HopConfig& cfg, int32_t n_rhs) {
  return (cfg.ns > 1 && n_rhs % cfg.ns == 0 && cfg.nv == 4 && cfg.walk == 0 && (cfg.order == 0 || cfg.order == 1) &&
          (cfg.form == kFormAdjoint || cfg.form == kFormStream))
             ? 1
             : 0;
}

// hop-split shape (order 2, or 3 with the x3-fastest block order): each wave covers 16 sites
// of one direction group
int hop_split_ok(const HopConfig& cfg) {
  return ((cfg.order == 2 || cfg.order == 3) && (cfg.block / 64) % (4 / cfg.nv) == 0) ? 1 : 0;
}
static int hop_split_spb(const HopConfig& cfg) { return (cfg.block / 64) / (4 / cfg.nv) * 16; }

int hop_num_blocks(const Geom& g, const HopConfig& cfg) {
  if (hop_split_ok(cfg)) {
    const int spb = hop_split_spb(cfg);
    return (g.V + spb - 1) / spb;
  }
  const int spb = cfg.block * cfg.nv / 4;
  if (hop_walk_ok(g, cfg)) {
    const int P = g.L0 * g.L1 * g.L2;
    return ((P + spb - 1) / spb) * (g.L3 / cfg.walk);
  }
  return (g.V + spb - 1) / spb;
}

int hop_order_ok(const Geom& g, const HopConfig& cfg) {
  const int spb = hop_split_ok(cfg) ? hop_split_spb(cfg) : cfg.block * cfg.nv / 4;
  return ((g.L0 * g.L1) % spb) == 0 ? 1 : 0;
}

template <typename T, int FORM, int NV>
static hipError_t launch_hop_form(const HopArgs<T>& A, const HopConfig& cfg, hipStream_t s) {
  const int64_t nblk = hop_num_blocks(A.g, cfg);
  // one-dimensional grid, fields fastest (hop_block)
  if (nblk * A.n_rhs > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((uint32_t)(nblk * A.n_rhs)), block(cfg.block);
  const bool dots = A.partials && A.dot_mask;
  // the partial-sum buffers hold hop_max_blocks entries per field and dot product
  if (dots && nblk > hop_max_blocks(A.g)) return hipErrorInvalidValue;
  if constexpr (NV == 4 && FORM != kFormMatrix) {
    if (hop_ns_ok(cfg, A.n_rhs)) {
      const int32_t ord = (cfg.order == 1 && hop_order_ok(A.g, cfg)) ? 1 : 0;
      dim3 g2((uint32_t)(nblk * (A.n_rhs / cfg.ns)));
      if (cfg.ns == 2) {
        if (dots)
          hipLaunchKernelGGL((k_hop_ns<T, FORM, 2, true>), g2, block, 0, s, A, cfg.xcd_remap, ord);
        else
          hipLaunchKernelGGL((k_hop_ns<T, FORM, 2, false>), g2, block, 0, s, A, cfg.xcd_remap, ord);
      } else if (cfg.ns == 4) {
        // four fields per thread: FP32 only (the FP64 kernel would spill)
        if constexpr (sizeof(T) == 4) {
          if (dots)
            hipLaunchKernelGGL((k_hop_ns<T, FORM, 4, true>), g2, block, 0, s, A, cfg.xcd_remap, ord);
          else
            hipLaunchKernelGGL((k_hop_ns<T, FORM, 4, false>), g2, block, 0, s, A, cfg.xcd_remap, ord);
        } else {
          return hipErrorInvalidValue;
        }
      } else {
        return hipErrorInvalidValue;
      }
      return hipGetLastError();
    }
  }
  if (hop_split_ok(cfg)) {
    const int32_t ord = (cfg.order == 3 && hop_order_ok(A.g, cfg)) ? 1 : 0;
    if (dots)
      hipLaunchKernelGGL((k_hop_split<T, FORM, NV, true>), grid, block, 0, s, A, cfg.xcd_remap, ord);
    else
      hipLaunchKernelGGL((k_hop_split<T, FORM, NV, false>), grid, block, 0, s, A, cfg.xcd_remap, ord);
    return hipGetLastError();
  }
  const int32_t order = (cfg.order == 1 && hop_order_ok(A.g, cfg)) ? 1 : 0;
  if (hop_walk_ok(A.g, cfg)) {
    const int32_t K = cfg.walk;
    // the x0 rows lie whole within a wave (L0 divides 64 and the columns per block): their x0
    // neighbours come from other lanes instead of the caches
    const int32_t cpb = cfg.block * cfg.nv / 4;
    const int32_t lane_x0 = (64 % A.g.L0 == 0 && cpb % A.g.L0 == 0) ? 1 : 0;
    if (dots)
      hipLaunchKernelGGL((k_hop_walk<T, FORM, NV, true>), grid, block, 0, s, A, cfg.xcd_remap, K, cfg.tile2, lane_x0);
    else
      hipLaunchKernelGGL((k_hop_walk<T, FORM, NV, false>), grid, block, 0, s, A, cfg.xcd_remap, K, cfg.tile2,
                         lane_x0);
    return hipGetLastError();
  }
  if (dots)
    hipLaunchKernelGGL((k_hop<T, FORM, NV, true>), grid, block, 0, s, A, cfg.xcd_remap, order);
  else
    hipLaunchKernelGGL((k_hop<T, FORM, NV, false>), grid, block, 0, s, A, cfg.xcd_remap, order);
  return hipGetLastError();
}

template <typename T, int FORM>
static hipError_t launch_hop_nv(const HopArgs<T>& A, const HopConfig& cfg, hipStream_t s) {
  if (cfg.nv == 1) {
    // one direction per thread: only the 3x3 form, whose work does not repeat across directions
    if constexpr (FORM == kFormMatrix) return launch_hop_form<T, FORM, 1>(A, cfg, s);
    return hipErrorInvalidValue;
  }
  if (cfg.nv == 2) return launch_hop_form<T, FORM, 2>(A, cfg, s);
  if (cfg.nv == 4) return launch_hop_form<T, FORM, 4>(A, cfg, s);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_hop(const HopArgs<T>& A, const HopConfig& cfg, hipStream_t s) {
  if (A.n_rhs == 0 || A.g.V == 0) return hipSuccess;
  if (cfg.form == kFormMatrix) return launch_hop_nv<T, kFormMatrix>(A, cfg, s);
  if (cfg.form == kFormAdjoint) return launch_hop_nv<T, kFormAdjoint>(A, cfg, s);
  return launch_hop_nv<T, kFormStream>(A, cfg, s);
}
template hipError_t launch_hop<double>(const HopArgs<double>&, const HopConfig&, hipStream_t);
template hipError_t launch_hop<float>(const HopArgs<float>&, const HopConfig&, hipStream_t);

}  // namespace rmh

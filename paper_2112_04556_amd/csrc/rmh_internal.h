// Internal declarations shared by the kernel and ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "rmh_device.h"

namespace rmh {

constexpr int kBlock = 256;        // threads per block for site and element kernels
constexpr int kRedBlock = 256;     // threads of the per-rhs scalar kernels
constexpr int kCgBlock = 512;      // threads of the CG alpha and beta kernels: one (shift, coefficient)
                                   // pair each for 12 shifts over segments of up to 40 iterations
constexpr int kMaxFilterWindows = 64;
constexpr int kMaxSpectrumWindows = 4096;   // windows of a power spectrum (host-side sums only)
constexpr int kMaxChebDegree = 100000;
constexpr int kMaxShifts = 64;      // poles of one rational (shifts of one multi-shift solve)

// Stencil variants chosen by the tuner.
// kFormAdjoint: the 8x8 adjoint matrix R(U) built once per hop and applied to every vector;
// kFormMatrix: U phi U^dag as 3x3 complex products per vector;
// kFormStream: R(U) built and applied two columns at a time (fewest registers).
enum HopForm : int32_t { kFormAdjoint = 0, kFormMatrix = 1, kFormStream = 2 };

// nv = directions nu per thread (4: a whole link field, 2: half of one; the threads of a
// site's halves sit in the same block).
// order = 1 walks the blocks with x3 fastest, then x2, then the (x0, x1) chunks, so the blocks
// holding a site's x2 and x3 neighbours are resident at the same time and share the L2; it needs
// L0 * L1 to be a multiple of the sites per block (else the lexicographic order 0 is used).
// order = 2 (hop split) gives each site four lanes of one wave, lane group mu doing the two hops
// along mu, summed by wave shuffles: four times the threads of order 0, for lattices too small to
// fill the chip (walk is then ignored); order = 3 is the same shape with the x3-fastest block
// order of order 1.
// walk = K > 0: each thread walks K consecutive sites along x3 (K divides L3), carrying the
// centre field, the x-3 field and the x-3 link in registers, so every x3-direction field and
// link is fetched once per column instead of being re-read from the caches.
// ns = S > 1 (with nv = 4, orders 0 and 1, no walk; S divides the batch): each thread applies the
// operator at its site to S fields of the batch, so every link it loads and every adjoint matrix it
// builds serves 4 S vectors instead of 4 (form 0: the 8x8 matrix is built once per hop and the
// fields are streamed through it one at a time; form 2: its column pairs are built once per hop
// and applied to all 4 S vectors).  The per-vector arithmetic is that of nv = 4, so results are
// bitwise those of ns = 1 with the same form.
struct HopConfig {
  int32_t form = kFormStream;
  int32_t block = 256;
  int32_t xcd_remap = 1;
  int32_t nv = 4;
  int32_t order = 0;
  int32_t walk = 0;
  int32_t ns = 1;
  int32_t tile2 = 1;   // walk only: 2 or 4 gives each block an L0 x R1 x tile2 tile of columns
};

// out[v] = a * (H x)[v] + b_v * x[v] + c * z[v / z_div]   for v in [0, n_rhs) link fields,
// where H = sum_mu (forward hop + backward hop), so Delta = 8 - H.
// Optional: per-block partial dot products.
template <typename T>
struct HopArgs {
  Geom g;
  const T* U;               // [4][18][V]
  const T* x;               // field index v * x_mul + x_add, [*][4][8][V]
  int32_t x_mul, x_add;
  T* out;                   // [n_rhs][4][8][V] (may alias z)
  const T* z;               // optional, [*][4][8][V]
  int32_t z_div;            // z field index = v / z_div
  double a, b, c;
  const double* b_rhs;      // optional per-field b (device), replaces b
  int32_t n_rhs;
  const int32_t* run;       // optional per-field flag (device) run[v * run_stride]: 0 = skip
  int32_t run_stride;
  int32_t store;            // write out
  double* partials;         // [n_rhs][3][nblk]: <x,x>, <out,x>, <out,out>
  int32_t dot_mask;         // bit q set -> compute dot q
};

int hop_num_blocks(const Geom& g, const HopConfig& cfg);
// whether the x3-fastest block order applies to this lattice and configuration
int hop_order_ok(const Geom& g, const HopConfig& cfg);
// whether the hop-split shape applies (order 2)
int hop_split_ok(const HopConfig& cfg);
// whether the x3 walk applies (K divides L3)
int hop_walk_ok(const Geom& g, const HopConfig& cfg);
// whether the multi-field shape applies (ns > 1 divides n_rhs, nv = 4, no walk, orders 0 and 1)
int hop_ns_ok(const HopConfig& cfg, int32_t n_rhs);
// upper bound of hop_num_blocks over every configuration: 16 sites per block at least (the
// hop-split shape with one direction group per block), plus one partial block per x3 slice of
// the walking shape; every per-block partial-sum buffer is sized with it
inline int hop_max_blocks(const Geom& g) { return (g.V + 15) / 16 + g.L3; }

template <typename T>
hipError_t launch_hop(const HopArgs<T>& args, const HopConfig& cfg, hipStream_t s);

// Element-wise helpers over link fields of 32 V reals each.
int64_t field_reals(const Geom& g);
int elem_num_blocks(int64_t n_reals);
// Element-wise kernels with a reduction: each block covers red_steps(n) chunks of 4 kBlock
// reals, so the per-block partials stay few on large lattices; red_num_blocks(n) partials
// per row.
int red_steps(int64_t n_reals);
int red_num_blocks(int64_t n_reals);

hipError_t launch_pack_links(const Geom& g, const double* aos, void* soa, int dtype, hipStream_t s);
hipError_t launch_unpack_links(const Geom& g, const double* soa, double* aos, hipStream_t s);
hipError_t launch_fields_aos_to_soa(const Geom& g, int32_t n, const double* aos, void* soa, int dtype,
                                    hipStream_t s);
hipError_t launch_fields_soa_to_aos(const Geom& g, int32_t n, const void* soa, int dtype, double* aos,
                                    hipStream_t s);
hipError_t launch_f64_to_f32(const double* in, float* out, int64_t n, hipStream_t s);
hipError_t launch_f32_to_f64(const float* in, double* out, int64_t n, hipStream_t s);

// Reduce partials[m][nblk] -> sums[m] (fixed order), one block per m.
hipError_t launch_reduce_rows(const double* partials, int32_t nblk, int32_t m, double* sums, hipStream_t s);

// Dot products <a_v, b_v> of n fields (per-block partials [n][nblk_e]).
template <typename T>
hipError_t launch_dot(const T* a, const T* b, int64_t n_reals, int32_t n, double* partials, hipStream_t s);

// ---------------------------------------------------------------------------------------------
// Multi-shift CG engine state (all device pointers, carved from the caller's workspace).
//
// The seed system (smallest shift) is iterated with explicit vectors: residual, direction p and
// A p.  The shift solutions and directions are not updated vector by vector: they are linear
// combinations of the seed residuals of the current segment (a ring of stored residuals) and of
// their own vectors at the segment start,
//   x_j = x_j0 + a_j p_j0 + sum_i d_ji r_i,   p_j = b_j p_j0 + sum_i e_ji r_i,
// with the scalar coefficients updated each iteration on the device and the combination folded
// into x_j, p_j (flush) when the ring is full, at a precision switch and at the end.  The seed's
// own solution is kept outside the ring where reliable updates read it: in FP32 phases it
// accumulates in an FP32 vector that each reliable update moves into FP64; single-shift engines
// update it each iteration in FP64 phases.
struct CgDev {
  int32_t n_rhs, n_shift;
  double* sc;            // [n_rhs][kScN]
  double* sh;            // [n_rhs][n_shift][kShN]
  int32_t* flags;        // [n_rhs][kFlN]
  int32_t* act;          // [n_rhs][n_shift]
  int32_t* act_next;     // [n_rhs][n_shift]
  const double* sigma;   // [n_rhs][n_shift]
  const int32_t* seed;   // [n_rhs]
  double* part;          // partials scratch [n_rhs][nblk_max]
  double* part_ru;       // partials of the FP64 residual stencil [n_rhs][3][nblk_ru] (mixed precision)
  double* coef;          // [n_rhs][n_shift][2 + 2 cslots]: a, b, d[cslots], e[cslots]
  int32_t nslot;         // segment capacity guard of this view: FP64 ring slots, or (FP32 view)
                         // the coefficient slots
  int32_t cslots;        // coefficient slots: entries a segment can hold
  // the residual rings: FP64 slots (nslot64 per rhs, rb64 bytes per rhs) and, with mixed
  // precision, FP32 slots (nslot32 per rhs, rb32 bytes per rhs) in a region of their own
  void* ring64;
  int64_t rb64;
  int32_t nslot64;
  void* ring32;
  int64_t rb32;
  int32_t nslot32;
  int32_t ring_on;       // shift solutions through the ring (n_shift > 1); else the seed's
                         // solution is updated each iteration and nslot = 2
  int32_t seed_explicit; // the seed's solution is kept outside the ring (single shift, FP32 phase)
  int32_t nblk_hop, nblk_e, nblk_ru;
};
// Segment entries: entry i < K64 is FP64 slot (Base + i) % nslot64; entry i >= K64 is FP32 slot
// (Base32 + i - K0) % nslot32 (K0: the entry held in FP32 slot Base32).  FP64 phases have
// K64 = kAllFp64; at the switch to FP32 the segment goes on, K64 = M + 1 and the current FP64
// residual is copied to FP32 slot Base32 as entry K0 = M; after an FP32-phase flush K64 = K0 = 0.
constexpr int kMaxSlots = 33;
constexpr int32_t kAllFp64 = 1 << 30;
// scalar slots per rhs
enum : int { kScRR = 0, kScAlpha, kScAlphaPrev, kScBetaPrev, kScBnorm2, kScMaxR, kScTolAbs, kScIters,
             kScRU, kScDelta, kScMaxIter, kScN };
// per (rhs, shift) slots; Seg: the shift was updated in the current segment
enum : int { kShZeta = 0, kShZetaPrev, kShZetaNext, kShCx, kShCr, kShCp, kShSeg, kShN };
// int flags per rhs
// Run: the rhs still iterates (read by the stencil of the next iteration);
// Live: the current iteration is being carried out (set by the alpha kernel), so the
// update kernels of the iteration in which a rhs converges still run once.
// Base, M: FP64 ring slot of the segment's first residual, index of the current residual in it;
// K64, K0, Base32: the FP64 entries of the segment and the FP32 slot of entry K0 (above).
enum : int { kFlRun = 0, kFlLive, kFlStatus, kFlNeedRU, kFlRUMask, kFlBase, kFlM, kFlK64, kFlK0, kFlBase32, kFlN };
enum : int { kStOk = 0, kStNoConv = 1, kStBreakdown = 2 };

// fp32_start: the solve runs in FP32 from its first iteration (its segment has no FP64 entries)
hipError_t launch_cg_init(const CgDev& cg, const double* bn2_partials, int32_t nblk, const double* tol_rel,
                          double delta, int32_t maxiter, int32_t fp32_start, hipStream_t s);
hipError_t launch_cg_alpha(const CgDev& cg, hipStream_t s);
hipError_t launch_cg_beta(const CgDev& cg, int32_t mixed, hipStream_t s);
// slot 0 of the ring region (ring, rhs_bytes per rhs) = (T) b, p = (T) b for every rhs
template <typename T>
hipError_t launch_cg_start(const double* b, void* ring, T* p, int32_t nr, int64_t rhs_bytes, int64_t n_reals,
                           hipStream_t s);
// next residual r' = r - alpha Ap into the next segment entry (r taken from r64 when a reliable
// update was consumed), partial <r', r'>; with x_hi non-null also x_hi[seed] += alpha p
template <typename T>
hipError_t launch_cg_r_update(const CgDev& cg, const T* Ap, const T* p, double* x_hi, const double* r64,
                              int64_t n_reals, hipStream_t s);
// seed direction p = r' + beta p (while the rhs runs); with x_lo non-null also x_lo += alpha p
// (the FP32 increment of the seed's solution, FP32 phase), and with x_hi non-null, for the rhs
// with a pending reliable update, x_hi[seed] += x_lo, x_lo = 0 in the same pass
template <typename T>
hipError_t launch_cg_p_update(const CgDev& cg, T* p, float* x_lo, double* x_hi, int64_t n_reals, hipStream_t s);
// x_hi[seed] += x_lo, x_lo = 0 for every rhs (all, the end of a mixed solve) or those with a
// pending reliable update
hipError_t launch_cg_xfold(const CgDev& cg, float* x_lo, double* x_hi, int32_t all, int64_t n_reals, hipStream_t s);
// fold the segment (FP64 and FP32 entries alike) into x_j (and p_j unless final) of every shift
// updated in it (p_j0 is read only where its coefficient is nonzero: before the first flush it
// holds nothing); then, unless seed_only, reset the coefficients and restart the segment at the
// current residual (fp32: in the FP32 ring).  first: no flush yet in this solve (x_j holds
// nothing: written, not accumulated).  seed_only: fold the seed's solution alone, nothing reset
// (the switch to FP32, after which the seed's solution is kept explicitly).
hipError_t launch_cg_flush(const CgDev& cg, double* x_hi, double* pj, int32_t final_, int32_t first,
                           int32_t seed_only, int32_t fp32, int64_t n_reals, hipStream_t s);
// precision switch (no flush: the segment goes on in FP32): the current FP64 residual -> FP32
// slot 0, p64 -> p32, K64 = M + 1, K0 = M, Base32 = 0; the reliable-update reference becomes the
// current residual norm
hipError_t launch_cg_to_f32(const CgDev& cg64, const double* p64, float* p32, int64_t n_reals, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_gather_pairs(const double* x_hi, const double* b, const int32_t* idx, int32_t ns, double* X,
                               double* B, int32_t nb, int64_t n, hipStream_t s);
hipError_t launch_scatter_add_pairs(double* x_hi, const int32_t* idx, const double* E, int32_t nb, int64_t n,
                                    hipStream_t s);
template <typename T>
hipError_t launch_copy_cast(const double* in, T* out, int64_t n, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// y[v] = c * x[v] + sum_j r_j * xp[v][j]  (FP64), with optional partial <y,y>
hipError_t launch_rational_combine(const double* x, const double* xp, int32_t n_rhs, int32_t n_poles,
                                   const double* coef /* device: c, r_0..r_{n-1} */, double* y,
                                   int64_t n_reals, double* partials, hipStream_t s);
// x[v] += e[v] (FP64 axpy with unit weight)
hipError_t launch_add(double* x, const double* e, int64_t n, hipStream_t s);

// Link derivative: grad[o][mu][c][V] (+)= sum_k w_k d<A_k, Delta B_k>/d omega
struct ForceArgs {
  Geom g;
  const double* U;
  const double* A;   // [n_rhs][n_pair][4][8][V]
  const double* B;   // same layout
  int32_t n_rhs, n_pair;
  double w[64];      // weight of each pair
  double* grad;      // [n_out][4][8][V]
  int32_t per_rhs;
  int32_t accumulate;  // grad += (else grad =)
};
hipError_t launch_force(const ForceArgs& a, hipStream_t s);

// Wilson gauge force F = -dS_W/d omega ([4][8][V], optional) and per-block partials of
// sum_mu Re Tr(U_mu A_mu) (gauge_force_blocks of them, optional).
int gauge_force_blocks(const Geom& g);
hipError_t launch_gauge_force(const Geom& g, const double* U, double beta, double* F, double* partials,
                              hipStream_t s);

// Molecular-dynamics link update: U1_mu(x) = exp(i h (A + B)^c_mu(x) T^c) U0_mu(x) for every link
// (FP64 SoA links, A and B FP64 [4][8][V], B may be null; U1 must not overlap U0)
hipError_t launch_link_exp(const Geom& g, const double* U0, const double* A, const double* B, double h, double* U1,
                           hipStream_t s);
// gout = J(omega)^T gin per link ([4][8][V] FP64 each): the derivative of f(exp(i omega.T) U) with
// respect to omega from the left-multiplication derivative gin at the displaced links
hipError_t launch_dexp_vjp(const Geom& g, const double* omega, const double* gin, double* gout, hipStream_t s);
// out = x + h (y - z) over n reals (FP64), with per-block partials of |out - prev|^2 and |out|^2
// written to partials[0][nblk], partials[1][nblk], nblk = red_num_blocks(n); prev may be out itself
// (each element is read before it is written, by the same thread)
hipError_t launch_axpy_diff(const double* x, const double* y, const double* z, double h, const double* prev,
                            double* out, int64_t n, double* partials, hipStream_t s);

// Chebyshev filter fold over a ring of R recursion vectors of n elements each (t_k in slot k % R):
//   y_w = (first ? coef[w][0] x : y_w) + sum_{j < cnt} coef[w][k0 + j] t_{k0 + j},   w < nw,
// coef [nw][D + 1] on the device, y_w = y + w * n; accumulated in FP64.  cnt <= kMaxFold.
constexpr int kMaxFold = 16;
template <typename T>
hipError_t launch_cheb_fold(const T* x, const T* ring, int32_t R, int32_t k0, int32_t cnt, int32_t first,
                            const double* coef, int32_t D, int32_t nw, T* y, int64_t n, hipStream_t s);

// Chebyshev reverse sweep source term: tb[v] += sum_y coef[(v * n_y + y) * n_k + k] Y[y][v] (FP64;
// Y laid out [n_y][n_rhs][n_reals], coef on the device)
hipError_t launch_cheb_source(double* tb, const double* Y, const double* coef, int32_t n_rhs, int32_t n_y,
                              int32_t n_k, int32_t k, int64_t n_reals, hipStream_t s);

}  // namespace rmh

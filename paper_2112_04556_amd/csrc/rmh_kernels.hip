// HIP kernels for gfx950 besides the stencil: layout conversion, element-wise kernels with
// deterministic reductions, the multi-shift CG vector and scalar kernels, mixed-precision
// reliable updates, and the link-derivative (force) kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rmh_internal.h"
#include "rmh_reduce.h"

namespace rmh {

// ------------------------------------------------------------------------------------------
// element-wise helpers

int64_t field_reals(const Geom& g) { return 32 * (int64_t)g.V; }
int elem_num_blocks(int64_t n_reals) { return (int)((n_reals / 4 + kBlock - 1) / kBlock); }
int red_steps(int64_t n_reals) {
  const int64_t s = n_reals / (4LL * kBlock * 2048);   // keep at least ~2048 blocks
  return (int)std::max<int64_t>(1, std::min<int64_t>(8, s));
}
int red_num_blocks(int64_t n_reals) {
  const int64_t c = 4LL * kBlock * red_steps(n_reals);
  return (int)((n_reals + c - 1) / c);
}

template <typename T>
__global__ void k_dot(const T* __restrict__ a, const T* __restrict__ b, int64_t n, int32_t steps, double* partials) {
  const int32_t v = blockIdx.y;
  const T* av = a + (int64_t)v * n;
  const T* bv = b + (int64_t)v * n;
  double d[1] = {0.0};
  for (int32_t t = 0; t < steps; ++t) {
    const int64_t i0 = (((int64_t)blockIdx.x * steps + t) * blockDim.x + threadIdx.x) * 4;
    if (i0 < n) {
#pragma unroll
      for (int k = 0; k < 4; ++k) d[0] = fma((double)av[i0 + k], (double)bv[i0 + k], d[0]);
    }
  }
  __shared__ double lds[1][16];
  block_sum<1>(d, lds);
  if (threadIdx.x == 0) partials[(int64_t)v * gridDim.x + blockIdx.x] = d[0];
}

template <typename T>
hipError_t launch_dot(const T* a, const T* b, int64_t n_reals, int32_t n, double* partials, hipStream_t s) {
  if (n == 0) return hipSuccess;
  dim3 grid(red_num_blocks(n_reals), n);
  hipLaunchKernelGGL((k_dot<T>), grid, dim3(kBlock), 0, s, a, b, n_reals, red_steps(n_reals), partials);
  return hipGetLastError();
}
template hipError_t launch_dot<double>(const double*, const double*, int64_t, int32_t, double*, hipStream_t);
template hipError_t launch_dot<float>(const float*, const float*, int64_t, int32_t, double*, hipStream_t);

__global__ void k_reduce_rows(const double* partials, int32_t nblk, double* sums) {
  __shared__ double lds[1][16];
  const double v = block_sum_array(partials + (int64_t)blockIdx.x * nblk, nblk, lds);
  if (threadIdx.x == 0) sums[blockIdx.x] = v;
}

hipError_t launch_reduce_rows(const double* partials, int32_t nblk, int32_t m, double* sums, hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_rows, dim3(m), dim3(kRedBlock), 0, s, partials, nblk, sums);
  return hipGetLastError();
}

// Fills stride over the grid: a launch holds fewer than 2^32 threads, and buffers of 16 GiB and
// more (a batch of FP64 link fields at 32^3 x 64) have more 4-byte words than that.
static unsigned fill_blocks(int64_t n) { return (unsigned)std::min<int64_t>((n + kBlock - 1) / kBlock, 1 << 20); }

__global__ void k_zero(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  // every buffer is carved at 256-byte granularity, so bytes is a multiple of 4
  const int64_t n = (int64_t)(bytes / 4);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(fill_blocks(n)), dim3(kBlock), 0, s, (uint32_t*)p, n);
  return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_blocks(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

template <typename TI, typename TO>
__global__ void k_cast(const TI* __restrict__ in, TO* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (TO)in[i];  // FP64 -> FP32 rounds to nearest even
}

hipError_t launch_f64_to_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_cast<double, float>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     in, out, n);
  return hipGetLastError();
}
hipError_t launch_f32_to_f64(const float* in, double* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_cast<float, double>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     in, out, n);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_copy_cast(const double* in, T* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_cast<double, T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, in,
                     out, n);
  return hipGetLastError();
}
template hipError_t launch_copy_cast<double>(const double*, double*, int64_t, hipStream_t);
template hipError_t launch_copy_cast<float>(const double*, float*, int64_t, hipStream_t);

__global__ void k_add(double* __restrict__ x, const double* __restrict__ e, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += e[i];
}
hipError_t launch_add(double* x, const double* e, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_add, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, x, e, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// layout conversion (bitwise: pure data movement plus FP64 -> FP32 round to nearest even)

template <typename T>
__global__ void k_pack_links(Geom g, const double* __restrict__ aos, T* __restrict__ soa) {
  const int32_t mu = blockIdx.y;
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const double* src = aos + ((int64_t)mu * g.V + s) * 18;
#pragma unroll
  for (int c = 0; c < 18; ++c) soa[((int64_t)mu * 18 + c) * g.V + s] = (T)src[c];
}

__global__ void k_unpack_links(Geom g, const double* __restrict__ soa, double* __restrict__ aos) {
  const int32_t mu = blockIdx.y;
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  double* dst = aos + ((int64_t)mu * g.V + s) * 18;
#pragma unroll
  for (int c = 0; c < 18; ++c) dst[c] = soa[((int64_t)mu * 18 + c) * g.V + s];
}

hipError_t launch_pack_links(const Geom& g, const double* aos, void* soa, int dtype, hipStream_t s) {
  dim3 grid((g.V + kBlock - 1) / kBlock, 4);
  if (dtype == 0)
    hipLaunchKernelGGL((k_pack_links<double>), grid, dim3(kBlock), 0, s, g, aos, (double*)soa);
  else
    hipLaunchKernelGGL((k_pack_links<float>), grid, dim3(kBlock), 0, s, g, aos, (float*)soa);
  return hipGetLastError();
}

hipError_t launch_unpack_links(const Geom& g, const double* soa, double* aos, hipStream_t s) {
  dim3 grid((g.V + kBlock - 1) / kBlock, 4);
  hipLaunchKernelGGL(k_unpack_links, grid, dim3(kBlock), 0, s, g, soa, aos);
  return hipGetLastError();
}

// fields: AoS [n][V][4][8]  <->  SoA [n][4][8][V]
template <typename T>
__global__ void k_fields_aos_to_soa(Geom g, const double* __restrict__ aos, T* __restrict__ soa) {
  const int32_t n = blockIdx.y;
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const double* src = aos + ((int64_t)n * g.V + s) * 32;
  T* dst = soa + (int64_t)n * 32 * g.V;
#pragma unroll
  for (int c = 0; c < 32; ++c) dst[(int64_t)c * g.V + s] = (T)src[c];
}

template <typename T>
__global__ void k_fields_soa_to_aos(Geom g, const T* __restrict__ soa, double* __restrict__ aos) {
  const int32_t n = blockIdx.y;
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  double* dst = aos + ((int64_t)n * g.V + s) * 32;
  const T* src = soa + (int64_t)n * 32 * g.V;
#pragma unroll
  for (int c = 0; c < 32; ++c) dst[c] = (double)src[(int64_t)c * g.V + s];
}

hipError_t launch_fields_aos_to_soa(const Geom& g, int32_t n, const double* aos, void* soa, int dtype,
                                    hipStream_t s) {
  if (n == 0) return hipSuccess;
  dim3 grid((g.V + kBlock - 1) / kBlock, n);
  if (dtype == 0)
    hipLaunchKernelGGL((k_fields_aos_to_soa<double>), grid, dim3(kBlock), 0, s, g, aos, (double*)soa);
  else
    hipLaunchKernelGGL((k_fields_aos_to_soa<float>), grid, dim3(kBlock), 0, s, g, aos, (float*)soa);
  return hipGetLastError();
}

hipError_t launch_fields_soa_to_aos(const Geom& g, int32_t n, const void* soa, int dtype, double* aos,
                                    hipStream_t s) {
  if (n == 0) return hipSuccess;
  dim3 grid((g.V + kBlock - 1) / kBlock, n);
  if (dtype == 0)
    hipLaunchKernelGGL((k_fields_soa_to_aos<double>), grid, dim3(kBlock), 0, s, g, (const double*)soa, aos);
  else
    hipLaunchKernelGGL((k_fields_soa_to_aos<float>), grid, dim3(kBlock), 0, s, g, (const float*)soa, aos);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// multi-shift CG (Jegerlehner's shifted recurrences on a seed system; every shift's
// residual is zeta_j times the seed residual)

__global__ void k_cg_init(CgDev cg, const double* bn2_part, int32_t nblk, const double* tol_rel, double delta,
                          int32_t maxiter, int32_t fp32_start) {
  __shared__ double lds[1][16];
  const int32_t v = blockIdx.x;
  const double bn2 = block_sum_array(bn2_part + (int64_t)v * nblk, nblk, lds);
  __shared__ double s_bn2;
  if (threadIdx.x == 0) {
    double* sc = cg.sc + (int64_t)v * kScN;
    int32_t* fl = cg.flags + (int64_t)v * kFlN;
    sc[kScRR] = bn2;
    sc[kScBnorm2] = bn2;
    sc[kScAlpha] = 0.0;
    sc[kScAlphaPrev] = 1.0;
    sc[kScBetaPrev] = 0.0;
    sc[kScMaxR] = sqrt(bn2);
    sc[kScTolAbs] = tol_rel[v] * sqrt(bn2);
    sc[kScIters] = 0.0;
    sc[kScRU] = 0.0;
    sc[kScDelta] = delta;
    sc[kScMaxIter] = (double)maxiter;
    fl[kFlRun] = (bn2 > 0.0) ? 1 : 0;
    fl[kFlStatus] = (bn2 == bn2) ? kStOk : kStBreakdown;   // NaN source
    if (!(bn2 == bn2)) fl[kFlRun] = 0;
    fl[kFlNeedRU] = 0;
    fl[kFlRUMask] = 0;
    fl[kFlLive] = 0;
    fl[kFlBase] = 0;
    fl[kFlM] = 0;
    fl[kFlK64] = fp32_start ? 0 : kAllFp64;
    fl[kFlK0] = 0;
    fl[kFlBase32] = 0;
    s_bn2 = bn2;
  }
  __syncthreads();
  const int32_t nc = 2 + 2 * cg.cslots;
  for (int j = threadIdx.x; j < cg.n_shift; j += blockDim.x) {
    const int64_t vj = (int64_t)v * cg.n_shift + j;
    double* sh = cg.sh + vj * kShN;
    sh[kShZeta] = 1.0;
    sh[kShZetaPrev] = 1.0;
    sh[kShZetaNext] = 1.0;
    sh[kShCx] = 0.0;
    sh[kShCr] = 0.0;
    sh[kShCp] = 0.0;
    sh[kShSeg] = 0.0;
    // x_j = 0, p_j = b = ring slot 0
    double* cf = cg.coef + vj * nc;
    for (int i = 0; i < nc; ++i) cf[i] = 0.0;
    cf[2 + cg.cslots] = 1.0;
    const int32_t on = (s_bn2 > 0.0) ? 1 : 0;
    cg.act[vj] = on;
    cg.act_next[vj] = on;
  }
}

hipError_t launch_cg_init(const CgDev& cg, const double* bn2_partials, int32_t nblk, const double* tol_rel,
                          double delta, int32_t maxiter, int32_t fp32_start, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init, dim3(cg.n_rhs), dim3(kRedBlock), 0, s, cg, bn2_partials, nblk, tol_rel, delta,
                     maxiter, fp32_start);
  return hipGetLastError();
}

// alpha_k = rr / <p, A0 p>;  zeta_{k+1}^j and the x-update coefficient of every active shift,
// applied to the segment coefficients of the non-seed shifts: x_j += cx_j p_j
__global__ void k_cg_alpha(CgDev cg) {
  const int32_t v = blockIdx.x;
  int32_t* fl = cg.flags + (int64_t)v * kFlN;
  double* sc = cg.sc + (int64_t)v * kScN;
  const int32_t ns = cg.n_shift;
  const int32_t nc = 2 + 2 * cg.cslots;
  const int32_t tid = threadIdx.x;
  // Every load that does not need alpha is issued first (each address is valid whatever the
  // flags hold), so the block waits on memory a few times instead of once per dependent step.
  const int32_t run = fl[kFlRun];
  const int32_t m = fl[kFlM];
  const int32_t ru = cg.part_ru ? fl[kFlNeedRU] : 0;
  const int32_t seed = cg.seed[v];
  const double rr_sc = sc[kScRR], ap = sc[kScAlphaPrev], bp = sc[kScBetaPrev];
  // this thread's shift (n_shift <= blockDim)
  int32_t on = 0;
  double z = 0.0, zp = 0.0, sig = 0.0;
  if (tid < ns) {
    const int64_t vj = (int64_t)v * ns + tid;
    on = cg.act_next[vj];
    z = cg.sh[vj * kShN + kShZeta];
    zp = cg.sh[vj * kShN + kShZetaPrev];
    sig = cg.sigma[vj];
  }
  const double s0 = cg.sigma[(int64_t)v * ns + seed];
  // this thread's (shift, coefficient) pair when they all fit in the block: q = 0 the p_j0
  // coefficient (x_j0 += cx p_j0), q = 1 + i the ring entry i <= m (d_ji += cx e_ji).  A shift is
  // updated only while m < nslot <= cslots; past that (a single shift's segment index grows
  // without flushes) the pairs stop at the last coefficient slot so every read stays in its row.
  const int32_t per = min(m, cg.cslots - 1) + 2;
  const bool one_pass = ns * per <= (int32_t)blockDim.x;
  int32_t pj = 0, pq = 0;
  double c_dst = 0.0, c_src = 0.0;
  if (one_pass && tid < ns * per) {
    pj = tid / per;
    pq = tid - pj * per;
    const double* cf = cg.coef + ((int64_t)v * ns + pj) * nc;
    c_dst = pq == 0 ? cf[0] : cf[1 + pq];
    c_src = pq == 0 ? cf[1] : cf[1 + pq + cg.cslots];
  }
  if (run == 0) {
    if (tid == 0) fl[kFlLive] = 0;
    return;
  }
  __shared__ double lds[1][16];
  // a reliable update issued at the end of the previous iteration: its FP64 residual
  // r64 = b - (Delta + sigma0) x_seed replaces the recursive residual from now on
  double rr_true = 0.0;
  if (ru) rr_true = block_sum_array(cg.part_ru + ((int64_t)v * 3 + 2) * cg.nblk_ru, cg.nblk_ru, lds);
  const double pAp = block_sum_array(cg.part + ((int64_t)v * 3 + 1) * cg.nblk_hop, cg.nblk_hop, lds);
  __shared__ double s_alpha;
  __shared__ int s_ok;
  if (tid == 0) {
    if (ru) {
      sc[kScRR] = rr_true;
      sc[kScMaxR] = sqrt(rr_true);
      sc[kScRU] += 1.0;
      fl[kFlNeedRU] = 0;
      fl[kFlRUMask] = 1;
    }
    const double rr = ru ? rr_true : rr_sc;
    const double alpha = rr / pAp;
    s_ok = (pAp > 0.0 && alpha == alpha && alpha < 1e300) ? 1 : 0;
    s_alpha = alpha;
    if (s_ok) {
      sc[kScAlpha] = alpha;
      fl[kFlLive] = 1;
    } else {
      fl[kFlStatus] = kStBreakdown;
      fl[kFlRun] = 0;
      fl[kFlLive] = 0;
    }
  }
  __syncthreads();
  if (!s_ok) return;
  const double alpha = s_alpha;
  __shared__ double s_cx[kMaxShifts];
  __shared__ int s_upd[kMaxShifts];
  // per shift: zeta_{k+1} and the x coefficient
  if (tid < ns) {
    const int64_t vj = (int64_t)v * ns + tid;
    cg.act[vj] = on;
    double* sh = cg.sh + vj * kShN;
    int upd = 0;
    if (on) {
      const double ds = sig - s0;
      const double zn = z * zp * ap / (ap * zp * (1.0 + alpha * ds) + alpha * bp * (zp - z));
      const double cx = alpha * zn / z;
      sh[kShZetaNext] = zn;
      sh[kShCx] = cx;
      upd = (cg.ring_on && m < cg.nslot && !(cg.seed_explicit && tid == seed)) ? 1 : 0;
      if (upd) sh[kShSeg] = 1.0;
      s_cx[tid] = cx;
    } else {
      sh[kShCx] = 0.0;
    }
    s_upd[tid] = upd;
  }
  __syncthreads();
  // x_j += cx_j p_j on the segment coefficients, one (shift, coefficient) pair per thread
  if (one_pass) {
    if (tid < ns * per && s_upd[pj]) {
      double* cf = cg.coef + ((int64_t)v * ns + pj) * nc;
      cf[pq == 0 ? 0 : 1 + pq] = fma(s_cx[pj], c_src, c_dst);
    }
  } else {
    for (int t = tid; t < ns * per; t += blockDim.x) {
      const int32_t jj = t / per, q = t - jj * per;
      if (!s_upd[jj]) continue;
      double* cf = cg.coef + ((int64_t)v * ns + jj) * nc;
      if (q == 0)
        cf[0] = fma(s_cx[jj], cf[1], cf[0]);
      else
        cf[1 + q] = fma(s_cx[jj], cf[1 + q + cg.cslots], cf[1 + q]);
    }
  }
}

hipError_t launch_cg_alpha(const CgDev& cg, hipStream_t s) {
  if (cg.n_shift > kMaxShifts) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cg_alpha, dim3(cg.n_rhs), dim3(kCgBlock), 0, s, cg);
  return hipGetLastError();
}

// beta_k = rr_new / rr; shifted beta and p-update coefficients (applied to the segment
// coefficients of the non-seed shifts: p_j = cr_j r' + cp_j p_j); convergence and freezing;
// the new residual becomes the current ring entry
__global__ void k_cg_beta(CgDev cg, int32_t mixed) {
  const int32_t v = blockIdx.x;
  int32_t* fl = cg.flags + (int64_t)v * kFlN;
  double* sc = cg.sc + (int64_t)v * kScN;
  const int32_t ns = cg.n_shift;
  const int32_t nc = 2 + 2 * cg.cslots;
  const int32_t tid = threadIdx.x;
  // loads that do not need the new residual norm go out first (valid addresses whatever the
  // flags hold)
  const int32_t live = fl[kFlLive];
  const int32_t m = fl[kFlM];
  const int32_t seed = cg.seed[v];
  const double rr_old = sc[kScRR], tolabs = sc[kScTolAbs];
  // the scalars thread 0 updates after the shift pass, loaded now so that pass ends in no load
  double alpha0 = 0.0, iters0 = 0.0, maxit0 = 0.0, maxr0 = 0.0, delta0 = 0.0;
  if (tid == 0) {
    alpha0 = sc[kScAlpha];
    iters0 = sc[kScIters];
    maxit0 = sc[kScMaxIter];
    maxr0 = sc[kScMaxR];
    delta0 = sc[kScDelta];
  }
  int32_t act = 0;
  double z = 0.0, zn = 0.0;
  if (tid < ns) {
    const int64_t vj = (int64_t)v * ns + tid;
    act = cg.act[vj];
    z = cg.sh[vj * kShN + kShZeta];
    zn = cg.sh[vj * kShN + kShZetaNext];
  }
  // this thread's (shift, coefficient) pair when they all fit in the block: q = 0 the p_j0
  // coefficient, q = 1 + i the ring entry i <= m (both scaled by cp_j), q = m + 2 the new
  // entry m + 1 (set to cr_j).  Updates need m + 1 < nslot <= cslots; the pairs stop at the
  // last coefficient slot for larger m (reads in the row, nothing written).
  const int32_t mc = min(m, cg.cslots - 2);
  const int32_t per = mc + 3;
  const bool one_pass = ns * per <= (int32_t)blockDim.x;
  int32_t pj = 0, pq = 0;
  double c_old = 0.0;
  if (one_pass && tid < ns * per) {
    pj = tid / per;
    pq = tid - pj * per;
    const double* cf = cg.coef + ((int64_t)v * ns + pj) * nc;
    if (pq == 0)
      c_old = cf[1];
    else if (pq <= mc + 1)
      c_old = cf[2 + cg.cslots + pq - 1];
  }
  if (live == 0) return;
  __shared__ double lds[1][16];
  __shared__ double s_rrn;
  {
    const double t = block_sum_array(cg.part + (int64_t)v * cg.nblk_e, cg.nblk_e, lds);
    if (tid == 0) s_rrn = t;  // the block sum is valid in thread 0 only
    __syncthreads();
  }
  const double rrn = s_rrn;
  const double beta = rrn / rr_old;
  const double rnorm = sqrt(rrn);
  __shared__ double s_cp[kMaxShifts], s_cr[kMaxShifts];
  __shared__ int s_upd[kMaxShifts];
  __shared__ int s_seed_act, s_seed_keep;   // the seed's act and act_next, for thread 0
  int any_other = 0;
  // per shift: beta_j, the p coefficients, convergence
  if (tid < ns) {
    const int64_t vj = (int64_t)v * ns + tid;
    double* sh = cg.sh + vj * kShN;
    int upd = 0;
    if (act) {
      const double ratio = zn / z;
      const double cr = zn, cp = beta * ratio * ratio;
      sh[kShCr] = cr;
      sh[kShCp] = cp;
      s_cr[tid] = cr;
      s_cp[tid] = cp;
      const int32_t keep = (fabs(zn) * rnorm > tolabs) ? 1 : 0;
      cg.act_next[vj] = keep;
      if (tid != seed) any_other |= keep;
      if (tid == seed) s_seed_keep = keep;
      upd = (!(cg.seed_explicit && tid == seed) && cg.ring_on && keep && m + 1 < cg.nslot) ? 1 : 0;
      sh[kShZetaPrev] = z;
      sh[kShZeta] = zn;
    } else {
      cg.act_next[vj] = 0;
      if (tid == seed) s_seed_keep = 0;
    }
    if (tid == seed) s_seed_act = act;
    s_upd[tid] = upd;
  }
  any_other = __syncthreads_or(any_other);
  if (tid == 0) {
    const int64_t vs = (int64_t)v * ns + seed;
    int32_t seed_next = s_seed_keep;
    if (any_other && !seed_next && s_seed_act) {
      // the seed carries the Krylov space for the others: its direction keeps being updated
      if (cg.ring_on && !cg.seed_explicit && m + 1 < cg.nslot) s_upd[seed] = 1;
    }
    if (any_other) seed_next = 1;
    if (seed_next != s_seed_keep) cg.act_next[vs] = seed_next;
    const int32_t any = any_other | seed_next;
    const double iters = iters0 + 1.0;
    sc[kScAlphaPrev] = alpha0;
    sc[kScBetaPrev] = beta;
    sc[kScRR] = rrn;
    sc[kScIters] = iters;
    fl[kFlRUMask] = 0;  // the residual update of this iteration has consumed it
    fl[kFlM] = m + 1;
    if (!(rrn == rrn)) {
      fl[kFlStatus] = kStBreakdown;
      fl[kFlRun] = 0;
    } else if (!any) {
      fl[kFlRun] = 0;
    } else if (iters >= maxit0) {
      fl[kFlStatus] = kStNoConv;
      fl[kFlRun] = 0;
    }
    if (mixed) {
      const double maxr = rnorm > maxr0 ? rnorm : maxr0;
      if (rnorm > maxr0) sc[kScMaxR] = rnorm;
      if (rnorm < delta0 * maxr) fl[kFlNeedRU] = 1;
    }
  }
  __syncthreads();
  // p_j = cr_j r' + cp_j p_j on the segment coefficients, one (shift, coefficient) pair per thread
  if (one_pass) {
    if (tid < ns * per && s_upd[pj]) {
      double* cf = cg.coef + ((int64_t)v * ns + pj) * nc;
      if (pq == 0)
        cf[1] = c_old * s_cp[pj];
      else if (pq <= m + 1)
        cf[2 + cg.cslots + pq - 1] = c_old * s_cp[pj];
      else
        cf[2 + cg.cslots + m + 1] = s_cr[pj];
    }
  } else {
    for (int t = tid; t < ns * per; t += blockDim.x) {
      const int32_t jj = t / per, q = t - jj * per;
      if (!s_upd[jj]) continue;
      double* cf = cg.coef + ((int64_t)v * ns + jj) * nc;
      double* e = cf + 2 + cg.cslots;
      if (q == 0)
        cf[1] *= s_cp[jj];
      else if (q <= m + 1)
        e[q - 1] *= s_cp[jj];
      else
        e[m + 1] = s_cr[jj];
    }
  }
}

hipError_t launch_cg_beta(const CgDev& cg, int32_t mixed, hipStream_t s) {
  if (cg.n_shift > kMaxShifts) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cg_beta, dim3(cg.n_rhs), dim3(kCgBlock), 0, s, cg, mixed);
  return hipGetLastError();
}

// ring slot i of rhs v in a ring region of rhs_bytes per rhs, viewed as T (slots of n_reals)
template <typename T>
__device__ __forceinline__ T* ring_slot(const void* ring, int64_t rhs_bytes, int32_t v, int32_t i, int64_t n) {
  return (T*)((char*)ring + (int64_t)v * rhs_bytes + (int64_t)i * n * (int64_t)sizeof(T));
}

// segment entry i of rhs v: in the FP64 ring from the segment's FP64 base slot, or in the FP32
// ring counted from entry k0, which sits in FP32 slot base32
__device__ __forceinline__ double* entry64(const CgDev& cg, int32_t v, int32_t base, int32_t i, int64_t n) {
  return ring_slot<double>(cg.ring64, cg.rb64, v, (base + i) % cg.nslot64, n);
}
__device__ __forceinline__ float* entry32(const CgDev& cg, int32_t v, int32_t base32, int32_t k0, int32_t i,
                                          int64_t n) {
  return ring_slot<float>(cg.ring32, cg.rb32, v, (base32 + i - k0) % cg.nslot32, n);
}
// entry i of the phase whose arithmetic type is T (the FP32 phase only touches entries >= k0)
template <typename T>
__device__ __forceinline__ T* entry(const CgDev& cg, int32_t v, const int32_t* st, int32_t i, int64_t n) {
  if constexpr (sizeof(T) == 8)
    return entry64(cg, v, st[0], i, n);
  else
    return entry32(cg, v, st[1], st[2], i, n);
}

template <typename T>
__global__ void k_cg_start(const double* __restrict__ b, void* ring, T* __restrict__ p, int64_t rhs_bytes,
                           int64_t n) {
  const int32_t v = blockIdx.y;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
  T* r0 = ring_slot<T>(ring, rhs_bytes, v, 0, n);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T x = (T)b[(int64_t)v * n + i0 + k];
    r0[i0 + k] = x;
    p[(int64_t)v * n + i0 + k] = x;
  }
}

template <typename T>
hipError_t launch_cg_start(const double* b, void* ring, T* p, int32_t nr, int64_t rhs_bytes, int64_t n_reals,
                           hipStream_t s) {
  if (nr == 0) return hipSuccess;
  dim3 grid(elem_num_blocks(n_reals), nr);
  hipLaunchKernelGGL((k_cg_start<T>), grid, dim3(kBlock), 0, s, b, ring, p, rhs_bytes, n_reals);
  return hipGetLastError();
}
template hipError_t launch_cg_start<double>(const double*, void*, double*, int32_t, int64_t, int64_t, hipStream_t);
template hipError_t launch_cg_start<float>(const double*, void*, float*, int32_t, int64_t, int64_t, hipStream_t);

template <typename T>
__global__ void k_cg_r(CgDev cg, const T* __restrict__ Ap, const T* __restrict__ p, double* __restrict__ x_hi,
                       const double* __restrict__ r64, int64_t n, int32_t steps) {
  const int32_t v = blockIdx.y;
  const int32_t* fl = cg.flags + (int64_t)v * kFlN;
  // the per-rhs state in one batch of independent loads, ahead of any branch on it
  const int32_t live = fl[kFlLive], ru_mask = fl[kFlRUMask];
  const int32_t m = fl[kFlM];
  const int32_t st[3] = {fl[kFlBase], fl[kFlBase32], fl[kFlK0]};
  const int32_t seed = cg.seed[v];
  const double alpha_d = cg.sc[(int64_t)v * kScN + kScAlpha];
  if (live == 0) return;
  const int32_t from64 = r64 ? ru_mask : 0;
  const T* rc = entry<T>(cg, v, st, m, n);
  T* rn = entry<T>(cg, v, st, m + 1, n);
  const T alpha = (T)alpha_d;
  const T* av = Ap + (int64_t)v * n;
  const T* pv = p + (int64_t)v * n;
  double* xs = x_hi ? x_hi + ((int64_t)v * cg.n_shift + seed) * n : nullptr;
  const double* r64v = r64 ? r64 + (int64_t)v * n : nullptr;
  double d[1] = {0.0};
  for (int32_t t = 0; t < steps; ++t) {
    const int64_t i0 = (((int64_t)blockIdx.x * steps + t) * blockDim.x + threadIdx.x) * 4;
    if (i0 < n) {
      // (the residual source is uniform per field: one branch around whole vector loads)
      T r0[4], a4[4];
      if (from64) {
        double rd[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) rd[k] = r64v[i0 + k];
#pragma unroll
        for (int k = 0; k < 4; ++k) r0[k] = (T)rd[k];
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) r0[k] = rc[i0 + k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) a4[k] = av[i0 + k];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const T r1 = fmadd(-alpha, a4[k], r0[k]);
        rn[i0 + k] = r1;
        d[0] = fma((double)r1, (double)r1, d[0]);
      }
      if (xs) {
#pragma unroll
        for (int k = 0; k < 4; ++k) xs[i0 + k] = fma(alpha_d, (double)pv[i0 + k], xs[i0 + k]);
      }
    }
  }
  __shared__ double lds[1][16];
  block_sum<1>(d, lds);
  if (threadIdx.x == 0) cg.part[(int64_t)v * cg.nblk_e + blockIdx.x] = d[0];
}

template <typename T>
hipError_t launch_cg_r_update(const CgDev& cg, const T* Ap, const T* p, double* x_hi, const double* r64,
                              int64_t n_reals, hipStream_t s) {
  if (cg.nblk_e != red_num_blocks(n_reals)) return hipErrorInvalidValue;
  if (sizeof(T) == 4 && !cg.ring32) return hipErrorInvalidValue;
  dim3 grid(cg.nblk_e, cg.n_rhs);
  hipLaunchKernelGGL((k_cg_r<T>), grid, dim3(kBlock), 0, s, cg, Ap, p, x_hi, r64, n_reals, red_steps(n_reals));
  return hipGetLastError();
}
template hipError_t launch_cg_r_update<double>(const CgDev&, const double*, const double*, double*, const double*,
                                               int64_t, hipStream_t);
template hipError_t launch_cg_r_update<float>(const CgDev&, const float*, const float*, double*, const double*,
                                              int64_t, hipStream_t);

template <typename T>
__global__ void k_cg_p(CgDev cg, T* __restrict__ p, float* __restrict__ x_lo, double* __restrict__ x_hi, int64_t n) {
  const int32_t v = blockIdx.y;
  const int32_t* fl = cg.flags + (int64_t)v * kFlN;
  const double* scv = cg.sc + (int64_t)v * kScN;
  // the per-rhs state in one batch of independent loads, ahead of any branch on it
  const int32_t live = fl[kFlLive], upd_p = fl[kFlRun], need_ru = fl[kFlNeedRU];
  const int32_t m = fl[kFlM];
  const int32_t st[3] = {fl[kFlBase], fl[kFlBase32], fl[kFlK0]};
  const int32_t seed = cg.seed[v];
  const double beta_d = scv[kScBetaPrev], alpha_d = scv[kScAlpha];
  if (live == 0) return;
  if (!upd_p && !x_lo) return;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
  const T* r = entry<T>(cg, v, st, m, n);
  const T beta = (T)beta_d;
  const float alpha = (float)alpha_d;
  T* pv = p + (int64_t)v * n;
  T pold[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) pold[k] = pv[i0 + k];
  if (x_lo) {
    // the seed's increment of this iteration, alpha p, in FP32 until the next reliable update;
    // when this iteration's beta kernel asked for one, the increment goes into the FP64 seed
    // solution now (x_hi[seed] += x_lo, x_lo = 0), ahead of the update's FP64 residual stencil
    float* xv = x_lo + (int64_t)v * n + i0;
    float xl[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) xl[k] = xv[k];
    if (x_hi && need_ru) {
      double* xh = x_hi + ((int64_t)v * cg.n_shift + seed) * n + i0;
      double xo[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) xo[k] = xh[k];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xh[k] = xo[k] + (double)fmaf(alpha, (float)pold[k], xl[k]);
        xv[k] = 0.0f;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) xv[k] = fmaf(alpha, (float)pold[k], xl[k]);
    }
  }
  if (upd_p) {
#pragma unroll
    for (int k = 0; k < 4; ++k) pv[i0 + k] = fmadd(beta, pold[k], r[i0 + k]);
  }
}

template <typename T>
hipError_t launch_cg_p_update(const CgDev& cg, T* p, float* x_lo, double* x_hi, int64_t n_reals, hipStream_t s) {
  if (sizeof(T) == 4 && !cg.ring32) return hipErrorInvalidValue;
  dim3 grid(elem_num_blocks(n_reals), cg.n_rhs);
  hipLaunchKernelGGL((k_cg_p<T>), grid, dim3(kBlock), 0, s, cg, p, x_lo, x_hi, n_reals);
  return hipGetLastError();
}

// x_hi[seed] += x_lo, x_lo = 0: for the rhs with a pending reliable update, or for all
__global__ void k_cg_xfold(CgDev cg, float* __restrict__ x_lo, double* __restrict__ x_hi, int32_t all, int64_t n) {
  const int32_t v = blockIdx.y;
  if (!all && cg.flags[(int64_t)v * kFlN + kFlNeedRU] == 0) return;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
  float* xl = x_lo + (int64_t)v * n;
  double* xh = x_hi + ((int64_t)v * cg.n_shift + cg.seed[v]) * n;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    xh[i0 + k] += (double)xl[i0 + k];
    xl[i0 + k] = 0.0f;
  }
}

hipError_t launch_cg_xfold(const CgDev& cg, float* x_lo, double* x_hi, int32_t all, int64_t n_reals, hipStream_t s) {
  dim3 grid(elem_num_blocks(n_reals), cg.n_rhs);
  hipLaunchKernelGGL(k_cg_xfold, grid, dim3(kBlock), 0, s, cg, x_lo, x_hi, all, n_reals);
  return hipGetLastError();
}

template hipError_t launch_cg_p_update<double>(const CgDev&, double*, float*, double*, int64_t, hipStream_t);
template hipError_t launch_cg_p_update<float>(const CgDev&, float*, float*, double*, int64_t, hipStream_t);

// One element per thread: the segment's residuals at this element are loaded once and every
// non-seed shift touched in the segment is folded from registers (seed_only: the seed alone,
// its solution only).  F32: an FP32-phase segment, whose entries from K64 on are FP32 (those
// below K64, in the segment that spans the switch of precision, are FP64).
template <bool F32>
__global__ void __launch_bounds__(256) k_cg_flush(CgDev cg, double* __restrict__ x_hi, double* __restrict__ pj,
                                                  int32_t final_, int32_t first, int32_t seed_only, int64_t n) {
  const int32_t v = blockIdx.y;
  const int32_t* fl = cg.flags + (int64_t)v * kFlN;
  const int32_t m = min(fl[kFlM], cg.nslot - 1);   // the host flushes before m passes nslot - 1
  const int32_t base = fl[kFlBase], base32 = fl[kFlBase32], k0 = fl[kFlK0], k64 = fl[kFlK64];
  const int32_t seed = cg.seed[v];
  const int32_t nc = 2 + 2 * cg.cslots;
  const int32_t ns = cg.n_shift;
  // the segment coefficients of this rhs (and per shift: updated in the segment, still active)
  extern __shared__ double s_cf[];
  int32_t* s_fl = (int32_t*)(s_cf + (size_t)ns * nc);
  for (int i = threadIdx.x; i < ns * nc; i += blockDim.x) s_cf[i] = cg.coef[(int64_t)v * ns * nc + i];
  for (int j = threadIdx.x; j < ns; j += blockDim.x) {
    const int64_t vj = (int64_t)v * ns + j;
    s_fl[2 * j] = cg.sh[vj * kShN + kShSeg] != 0.0 ? 1 : 0;
    s_fl[2 * j + 1] = cg.act_next[vj];
  }
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double rv[kMaxSlots];
  if constexpr (!F32) {
#pragma unroll
    for (int i = 0; i < kMaxSlots; ++i) {
      rv[i] = 0.0;
      if (i <= m) rv[i] = entry64(cg, v, base, i, n)[e];
    }
  } else {
    // FP32 entries: every load is issued unconditionally so they overlap (the conditional form
    // waits on each); indices outside [k0, m] re-read an end of that range (a cache hit) and are
    // never used
    float rt[kMaxSlots];
#pragma unroll
    for (int i = 0; i < kMaxSlots; ++i) rt[i] = entry32(cg, v, base32, k0, min(max(i, k0), m), n)[e];
#pragma unroll
    for (int i = 0; i < kMaxSlots; ++i) rv[i] = (double)rt[i];
    if (k64 > 0) {   // uniform per rhs: only the segment that spans the switch
#pragma unroll
      for (int i = 0; i < kMaxSlots; ++i)
        if (i < k64) rv[i] = entry64(cg, v, base, i, n)[e];
    }
  }
  for (int j = 0; j < ns; ++j) {
    if (seed_only ? j != seed : (cg.seed_explicit && j == seed)) continue;   // kept current by the residual update
    const int64_t vj = (int64_t)v * ns + j;
    const double* cf = s_cf + (size_t)j * nc;
    const double* d = cf + 2;
    const double* ec = cf + 2 + cg.cslots;
    double* xj = x_hi + vj * n + e;
    double* pp = pj + vj * n + e;
    if (!s_fl[2 * j]) {
      if (first) *xj = 0.0;   // never updated (zero source)
      continue;
    }
    // p_j0 exists once a flush has written it; before that its coefficients are exactly zero
    const double p0 = (cf[0] != 0.0 || cf[1] != 0.0) ? *pp : 0.0;
    double x = fma(cf[0], p0, first ? 0.0 : *xj);
#pragma unroll
    for (int i = 0; i < kMaxSlots; ++i)
      if (i <= m) x = fma(d[i], rv[i], x);
    *xj = x;
    if (!final_ && !seed_only && s_fl[2 * j + 1]) {
      double q = cf[1] * p0;
#pragma unroll
      for (int i = 0; i < kMaxSlots; ++i)
        if (i <= m) q = fma(ec[i], rv[i], q);
      *pp = q;
    }
  }
}

// after a flush: coefficients of the fresh segment (x_j = x_j0, p_j = p_j0), which starts at the
// current residual (fp32: in the FP32 ring, with no FP64 entries)
__global__ void k_cg_flush_reset(CgDev cg, int32_t fp32) {
  const int32_t v = blockIdx.x;
  int32_t* fl = cg.flags + (int64_t)v * kFlN;
  const int32_t nc = 2 + 2 * cg.cslots;
  for (int j = threadIdx.x; j < cg.n_shift; j += blockDim.x) {
    const int64_t vj = (int64_t)v * cg.n_shift + j;
    double* cf = cg.coef + vj * nc;
    for (int i = 0; i < nc; ++i) cf[i] = 0.0;
    cf[1] = 1.0;
    cg.sh[vj * kShN + kShSeg] = 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int32_t m = fl[kFlM];
    if (fp32) {
      fl[kFlBase32] = (fl[kFlBase32] + m - fl[kFlK0]) % cg.nslot32;
      fl[kFlK0] = 0;
      fl[kFlK64] = 0;
    } else {
      fl[kFlBase] = (fl[kFlBase] + m) % cg.nslot64;
    }
    fl[kFlM] = 0;
  }
}

size_t flush_lds_bytes(const CgDev& cg) {
  return (size_t)cg.n_shift * (2 + 2 * cg.cslots) * 8 + (size_t)cg.n_shift * 2 * 4;
}

hipError_t launch_cg_flush(const CgDev& cg, double* x_hi, double* pj, int32_t final_, int32_t first,
                           int32_t seed_only, int32_t fp32, int64_t n_reals, hipStream_t s) {
  if (cg.nslot > kMaxSlots || cg.nslot > cg.cslots || cg.nslot64 > kMaxSlots) return hipErrorInvalidValue;
  if (fp32 && (!cg.ring32 || cg.nslot32 < cg.nslot || seed_only)) return hipErrorInvalidValue;
  dim3 grid((unsigned)((n_reals + kBlock - 1) / kBlock), cg.n_rhs);
  if (fp32)
    hipLaunchKernelGGL((k_cg_flush<true>), grid, dim3(kBlock), flush_lds_bytes(cg), s, cg, x_hi, pj, final_, first,
                       0, n_reals);
  else
    hipLaunchKernelGGL((k_cg_flush<false>), grid, dim3(kBlock), flush_lds_bytes(cg), s, cg, x_hi, pj, final_,
                       first, seed_only, n_reals);
  if (!seed_only) hipLaunchKernelGGL(k_cg_flush_reset, dim3(cg.n_rhs), dim3(kRedBlock), 0, s, cg, fp32);
  return hipGetLastError();
}

// the switch of precision: the current FP64 entry M -> FP32 slot 0, which holds entry K0 = M from
// now on; p64 -> p32
__global__ void k_cg_to_f32(CgDev cg, const double* __restrict__ p64, float* __restrict__ p32, int64_t n) {
  const int32_t v = blockIdx.y;
  const int32_t* fl = cg.flags + (int64_t)v * kFlN;
  const double* r = entry64(cg, v, fl[kFlBase], fl[kFlM], n);
  float* r32 = ring_slot<float>(cg.ring32, cg.rb32, v, 0, n);
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r32[i0 + k] = (float)r[i0 + k];
    p32[(int64_t)v * n + i0 + k] = (float)p64[(int64_t)v * n + i0 + k];
  }
}

__global__ void k_cg_to_f32_scalars(CgDev cg) {
  for (int v = threadIdx.x; v < cg.n_rhs; v += blockDim.x) {
    int32_t* fl = cg.flags + (int64_t)v * kFlN;
    double* sc = cg.sc + (int64_t)v * kScN;
    fl[kFlK64] = fl[kFlM] + 1;
    fl[kFlK0] = fl[kFlM];
    fl[kFlBase32] = 0;
    sc[kScMaxR] = sqrt(sc[kScRR]);
  }
}

hipError_t launch_cg_to_f32(const CgDev& cg64, const double* p64, float* p32, int64_t n_reals, hipStream_t s) {
  if (!cg64.ring32) return hipErrorInvalidValue;
  dim3 grid(elem_num_blocks(n_reals), cg64.n_rhs);
  hipLaunchKernelGGL(k_cg_to_f32, grid, dim3(kBlock), 0, s, cg64, p64, p32, n_reals);
  hipLaunchKernelGGL(k_cg_to_f32_scalars, dim3(1), dim3(kRedBlock), 0, s, cg64);
  return hipGetLastError();
}

// X[i] = x_hi[idx[i]], B[i] = b[idx[i] / ns] for the pairs of a refinement batch
__global__ void k_gather_pairs(const double* __restrict__ x_hi, const double* __restrict__ b,
                               const int32_t* __restrict__ idx, int32_t ns, double* __restrict__ X,
                               double* __restrict__ B, int64_t n) {
  const int32_t i = blockIdx.y;
  const int32_t q = idx[i];
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    X[(int64_t)i * n + i0 + k] = x_hi[(int64_t)q * n + i0 + k];
    B[(int64_t)i * n + i0 + k] = b[(int64_t)(q / ns) * n + i0 + k];
  }
}

hipError_t launch_gather_pairs(const double* x_hi, const double* b, const int32_t* idx, int32_t ns, double* X,
                               double* B, int32_t nb, int64_t n, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_pairs, dim3(elem_num_blocks(n), nb), dim3(kBlock), 0, s, x_hi, b, idx, ns, X, B, n);
  return hipGetLastError();
}

// x_hi[idx[i]] += E[i]
__global__ void k_scatter_add_pairs(double* __restrict__ x_hi, const int32_t* __restrict__ idx,
                                    const double* __restrict__ E, int64_t n) {
  const int32_t i = blockIdx.y;
  const int32_t q = idx[i];
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) x_hi[(int64_t)q * n + i0 + k] += E[(int64_t)i * n + i0 + k];
}

hipError_t launch_scatter_add_pairs(double* x_hi, const int32_t* idx, const double* E, int32_t nb, int64_t n,
                                    hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_add_pairs, dim3(elem_num_blocks(n), nb), dim3(kBlock), 0, s, x_hi, idx, E, n);
  return hipGetLastError();
}

// y = c x + sum_j r_j x_j  (FP64) with partial <y, y>
__global__ void k_rational_combine(const double* __restrict__ x, const double* __restrict__ xp, int32_t n_poles,
                                   const double* __restrict__ coef, double* __restrict__ y, int64_t n,
                                   int32_t steps, double* partials) {
  const int32_t v = blockIdx.y;
  double d[1] = {0.0};
  const double c = coef[0];
  for (int32_t t = 0; t < steps; ++t) {
    const int64_t i0 = (((int64_t)blockIdx.x * steps + t) * blockDim.x + threadIdx.x) * 4;
    if (i0 < n) {
      double acc[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] = c * x[(int64_t)v * n + i0 + k];
      for (int j = 0; j < n_poles; ++j) {
        const double* xj = xp + ((int64_t)v * n_poles + j) * n + i0;
        const double rj = coef[1 + j];
        double t4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) t4[k] = xj[k];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = fma(rj, t4[k], acc[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        y[(int64_t)v * n + i0 + k] = acc[k];
        d[0] = fma(acc[k], acc[k], d[0]);
      }
    }
  }
  if (partials) {
    __shared__ double lds[1][16];
    block_sum<1>(d, lds);
    if (threadIdx.x == 0) partials[(int64_t)v * gridDim.x + blockIdx.x] = d[0];
  }
}

hipError_t launch_rational_combine(const double* x, const double* xp, int32_t n_rhs, int32_t n_poles,
                                   const double* coef, double* y, int64_t n_reals, double* partials,
                                   hipStream_t s) {
  if (n_rhs == 0) return hipSuccess;
  dim3 grid(red_num_blocks(n_reals), n_rhs);
  hipLaunchKernelGGL(k_rational_combine, grid, dim3(kBlock), 0, s, x, xp, n_poles, coef, y, n_reals,
                     red_steps(n_reals), partials);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// link derivative
//
// For the link U = U_mu(x):  d<A, Delta B>/d omega^c = sum_{d,e} f^{dec} (R(U) C)^{de},
// C^{be} = B(x+mu)^b A(x)^e + A(x+mu)^b B(x)^e (summed over nu and over the pairs with
// weights w_k).  f^{abc} are the su(3) structure constants; with the antisymmetric part
// S = RC - (RC)^T each independent triple (a, b, c; f) contributes
// f S_ab to component c, f S_bc to component a and f S_ca to component b.

struct FTriple {
  int a, b, c;
  double f;
};
// compile-time table: with the loop over it unrolled every index is a constant, so the 8x8
// products stay in registers
constexpr FTriple kF[9] = {{0, 1, 2, 1.0},
                           {0, 3, 6, 0.5},
                           {0, 4, 5, -0.5},
                           {1, 3, 5, 0.5},
                           {1, 4, 6, 0.5},
                           {2, 3, 4, 0.5},
                           {2, 5, 6, -0.5},
                           {3, 4, 7, 0.86602540378443864676},
                           {5, 6, 7, 0.86602540378443864676}};

// G += R[:, b1] x C[b1, :] + R[:, b2] x C[b2, :] for the column group q of R(U) (columns b1, b2)
template <int q, int b1, int b2>
__device__ __forceinline__ void force_cross_cols(const double* u, const double* C, double* G) {
  double c1[8], c2[8];
  adjoint_columns<double, q>(u, c1, c2);
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int a = kF[t].a, b = kF[t].b, c = kF[t].c;
    const double f = kF[t].f;
    // (p x q)_c += f (p_a q_b - p_b q_a), cyclically in (a, b, c)
    G[c] += f * ((c1[a] * C[b1 * 8 + b] - c1[b] * C[b1 * 8 + a]) + (c2[a] * C[b2 * 8 + b] - c2[b] * C[b2 * 8 + a]));
    G[a] += f * ((c1[b] * C[b1 * 8 + c] - c1[c] * C[b1 * 8 + b]) + (c2[b] * C[b2 * 8 + c] - c2[c] * C[b2 * 8 + b]));
    G[b] += f * ((c1[c] * C[b1 * 8 + a] - c1[a] * C[b1 * 8 + c]) + (c2[c] * C[b2 * 8 + a] - c2[a] * C[b2 * 8 + c]));
  }
}

// One thread per (site, mu): a block of 256 threads is four waves, wave w taking direction mu = w
// for 64 consecutive sites, so every link and field base address is wave-uniform.
__global__ void __launch_bounds__(256) k_force(const ForceArgs F, int32_t xcd) {
  const int32_t o = blockIdx.y;
  const int32_t V = F.g.V;
  const int32_t blk = remap_block(blockIdx.x, gridDim.x, xcd);
  const int32_t mu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int32_t s = blk * 64 + (threadIdx.x & 63);
  if (s >= V) return;
  const int64_t FV = 32 * (int64_t)V;
  int32_t xc[4];
  site_coords(F.g, s, xc);
  const int32_t r0 = F.per_rhs ? o : 0;
  const int32_t r1 = F.per_rhs ? o + 1 : F.n_rhs;
  {
    const int32_t sf = site_shift(F.g, s, xc, mu, +1);
    double C[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) C[i] = 0.0;
#pragma unroll 1
    for (int32_t rh = r0; rh < r1; ++rh)
#pragma unroll 1
      for (int32_t k = 0; k < F.n_pair; ++k) {
        const double w = F.w[k];
        const double* Ak = F.A + ((int64_t)rh * F.n_pair + k) * FV;
        const double* Bk = F.B + ((int64_t)rh * F.n_pair + k) * FV;
#pragma unroll 1
        for (int nu = 0; nu < 4; ++nu) {
          double ax[8], bx[8], af[8], bf[8];
#pragma unroll
          for (int a = 0; a < 8; ++a) {
            const int64_t e = (int64_t)(nu * 8 + a) * V;
            ax[a] = w * Ak[e + s];
            bx[a] = w * Bk[e + s];
            af[a] = Ak[e + sf];
            bf[a] = Bk[e + sf];
          }
#pragma unroll
          for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int e = 0; e < 8; ++e) C[b * 8 + e] = fma(af[b], bx[e], fma(bf[b], ax[e], C[b * 8 + e]));
        }
      }
    // rows 0 and 1 of U_mu(x) (12 reals), row 2 rebuilt (SU(3))
    double u[18];
    const double* Um = F.U + (int64_t)mu * 18 * V;
#pragma unroll
    for (int c = 0; c < 12; ++c) u[c] = (Um + (size_t)c * V)[s];
    su3_row2<double>(u);
    // G = sum_b R[:, b] x C[b, :], x the su(3) product (p x q)_c = sum_{a,e} f^{aec} p_a q_e, with
    // the columns of R(U) formed two at a time (the whole of R is never held)
    double G[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) G[c] = 0.0;
    force_cross_cols<0, 0, 1>(u, C, G);
    force_cross_cols<1, 3, 4>(u, C, G);
    force_cross_cols<2, 5, 6>(u, C, G);
    force_cross_cols<3, 2, 7>(u, C, G);
    double* go = F.grad + ((int64_t)o * 4 + mu) * 8 * V;
    if (F.accumulate) {
#pragma unroll
      for (int c = 0; c < 8; ++c) go[(int64_t)c * V + s] += G[c];
    } else {
#pragma unroll
      for (int c = 0; c < 8; ++c) go[(int64_t)c * V + s] = G[c];
    }
  }
}

__global__ void k_cheb_source(double* __restrict__ tb, const double* __restrict__ Y, const double* __restrict__ coef,
                              int32_t n_rhs, int32_t n_y, int32_t n_k, int32_t k, int64_t n) {
  const int32_t v = blockIdx.y;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
  double acc[4];
  double* t = tb + (int64_t)v * n + i0;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = t[q];
  for (int32_t y = 0; y < n_y; ++y) {
    const double c = coef[((int64_t)v * n_y + y) * n_k + k];
    const double* yv = Y + ((int64_t)y * n_rhs + v) * n + i0;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = fma(c, yv[q], acc[q]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) t[q] = acc[q];
}

hipError_t launch_cheb_source(double* tb, const double* Y, const double* coef, int32_t n_rhs, int32_t n_y,
                              int32_t n_k, int32_t k, int64_t n_reals, hipStream_t s) {
  if (n_rhs == 0 || n_y == 0) return hipSuccess;
  dim3 grid(elem_num_blocks(n_reals), n_rhs);
  hipLaunchKernelGGL(k_cheb_source, grid, dim3(kBlock), 0, s, tb, Y, coef, n_rhs, n_y, n_k, k, n_reals);
  return hipGetLastError();
}

// Chebyshev filter fold: two consecutive elements per thread; the block's t_k are loaded once
// into registers and every window output is read, updated and written once per fold.
template <typename T>
__global__ void __launch_bounds__(256) k_cheb_fold(const T* __restrict__ x, const T* __restrict__ ring, int32_t R,
                                                   int32_t k0, int32_t cnt, int32_t first,
                                                   const double* __restrict__ coef, int32_t D1, int32_t nw,
                                                   T* __restrict__ y, int64_t n) {
  // this fold's coefficients (window w, vector j: coef[w][k0 + j]; column 0 for x on the first
  // fold) staged in LDS by the whole block, so the window loop reads no global scalars
  __shared__ double s_c[kMaxFilterWindows][kMaxFold + 1];
  for (int t = threadIdx.x; t < nw * (kMaxFold + 1); t += blockDim.x) {
    const int w = t / (kMaxFold + 1), j = t - w * (kMaxFold + 1);
    double c = 0.0;
    if (j == 0)
      c = first ? coef[(int64_t)w * D1] : 0.0;
    else if (j <= cnt)
      c = coef[(int64_t)w * D1 + k0 + j - 1];
    s_c[w][j] = c;
  }
  __syncthreads();
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
  if (i0 >= n) return;
  // every load is issued unconditionally so they overlap: entries past cnt re-read the last
  // vector of the fold (a cache hit) and are never used
  T tt[kMaxFold][2];
#pragma unroll
  for (int j = 0; j < kMaxFold; ++j) {
    const T* t = ring + (int64_t)((k0 + min(j, cnt - 1)) % R) * n + i0;
    tt[j][0] = t[0];
    tt[j][1] = t[1];
  }
  double tv[kMaxFold][2];
#pragma unroll
  for (int j = 0; j < kMaxFold; ++j) {
    tv[j][0] = (double)tt[j][0];
    tv[j][1] = (double)tt[j][1];
  }
  double x0 = 0.0, x1 = 0.0;
  if (first) {
    x0 = (double)x[i0];
    x1 = (double)x[i0 + 1];
  }
  // windows four at a time: their outputs are loaded together
  for (int32_t w0 = 0; w0 < nw; w0 += 4) {
    double a[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t w = w0 + u;
      if (w < nw && !first) {
        const T* yw = y + (int64_t)w * n + i0;
        a[u][0] = (double)yw[0];
        a[u][1] = (double)yw[1];
      } else {
        a[u][0] = 0.0;
        a[u][1] = 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t w = w0 + u;
      if (w >= nw) break;
      const double* c = s_c[w];
      if (first) {
        a[u][0] = c[0] * x0;
        a[u][1] = c[0] * x1;
      }
      // branch-free: the coefficients past cnt are zero (their vectors are finite re-reads)
#pragma unroll
      for (int j = 0; j < kMaxFold; ++j) {
        a[u][0] = fma(c[1 + j], tv[j][0], a[u][0]);
        a[u][1] = fma(c[1 + j], tv[j][1], a[u][1]);
      }
      T* yw = y + (int64_t)w * n + i0;
      yw[0] = (T)a[u][0];
      yw[1] = (T)a[u][1];
    }
  }
}

template <typename T>
hipError_t launch_cheb_fold(const T* x, const T* ring, int32_t R, int32_t k0, int32_t cnt, int32_t first,
                            const double* coef, int32_t D, int32_t nw, T* y, int64_t n, hipStream_t s) {
  if (n == 0 || nw == 0) return hipSuccess;
  if (cnt < 1 || cnt > kMaxFold || nw > kMaxFilterWindows || (n & 1)) return hipErrorInvalidValue;
  const int64_t nb = (n / 2 + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_cheb_fold<T>, dim3((uint32_t)nb), dim3(kBlock), 0, s, x, ring, R, k0, cnt, first, coef, D + 1,
                     nw, y, n);
  return hipGetLastError();
}
template hipError_t launch_cheb_fold<double>(const double*, const double*, int32_t, int32_t, int32_t, int32_t,
                                             const double*, int32_t, int32_t, double*, int64_t, hipStream_t);
template hipError_t launch_cheb_fold<float>(const float*, const float*, int32_t, int32_t, int32_t, int32_t,
                                            const double*, int32_t, int32_t, float*, int64_t, hipStream_t);

hipError_t launch_force(const ForceArgs& a, hipStream_t s) {
  const int32_t n_out = a.per_rhs ? a.n_rhs : 1;
  if (a.n_pair < 0 || a.n_pair > (int32_t)(sizeof(a.w) / sizeof(a.w[0]))) return hipErrorInvalidValue;
  if (n_out == 0) return hipSuccess;
  dim3 grid((a.g.V + 63) / 64, n_out);
  hipLaunchKernelGGL(k_force, grid, dim3(256), 0, s, a, 1);
  return hipGetLastError();
}

}  // namespace rmh

namespace rmh {

// ------------------------------------------------------------------------------------------
// Wilson gauge force
//
// 3x3 complex matrices as separate real and imaginary parts, row-major.
struct M3 {
  double re[9], im[9];
};

// U_mu(x) at site s: rows 0 and 1 loaded (12 reals), row 2 rebuilt from them (SU(3)).
__device__ __forceinline__ void load_link(const double* __restrict__ U, int32_t mu, int32_t s, int32_t V, M3& m) {
  const double* Um = U + (int64_t)mu * 18 * V;
  double u[18];
#pragma unroll
  for (int c = 0; c < 12; ++c) u[c] = (Um + (size_t)c * V)[s];
  su3_row2<double>(u);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    m.re[k] = u[2 * k];
    m.im[k] = u[2 * k + 1];
  }
}

// C = op(A) op(B) (kAcc: C += op(A) op(B)), op = identity or Hermitian conjugate
template <bool kDa, bool kDb, bool kAcc = false>
__device__ __forceinline__ void mul3(const M3& A, const M3& B, M3& C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double re = kAcc ? C.re[i * 3 + j] : 0.0, im = kAcc ? C.im[i * 3 + j] : 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int ia = kDa ? k * 3 + i : i * 3 + k;
        const int ib = kDb ? j * 3 + k : k * 3 + j;
        const double ar = A.re[ia], ai = kDa ? -A.im[ia] : A.im[ia];
        const double br = B.re[ib], bi = kDb ? -B.im[ib] : B.im[ib];
        re = fma(ar, br, fma(-ai, bi, re));
        im = fma(ar, bi, fma(ai, br, im));
      }
      C.re[i * 3 + j] = re;
      C.im[i * 3 + j] = im;
    }
}

// F^c_mu(x) = -(beta/3) Im Tr(T^c U_mu(x) A_mu(x)), A the sum of the six staples; partials of
// sum_mu Re Tr(U_mu A_mu) per block (each plaquette enters four times).  A block is four waves over
// the same 64 consecutive sites, wave w computing the force on U_w: the direction is wave-uniform,
// every load is a coalesced 64-site row of one component, and a lattice gives four times as many
// waves as sites / 64 to hide the staples' dependent loads.
__global__ void __launch_bounds__(256) k_gauge_force(Geom g, const double* __restrict__ U, double beta,
                                                     double* __restrict__ F, double* __restrict__ partials) {
  const int32_t V = g.V;
  const int32_t mu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int32_t s = blockIdx.x * 64 + (threadIdx.x & 63);
  double tr[1] = {0.0};
  if (s < V) {
    int32_t xc[4];
    site_coords(g, s, xc);
    const int32_t s_pm = site_shift(g, s, xc, mu, +1);
    int32_t xm[4];
    site_coords(g, s_pm, xm);
    M3 A;
#pragma unroll
    for (int k = 0; k < 9; ++k) A.re[k] = A.im[k] = 0.0;
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
      if (nu == mu) continue;
      const int32_t s_pn = site_shift(g, s, xc, nu, +1);
      const int32_t s_mn = site_shift(g, s, xc, nu, -1);
      const int32_t s_pm_mn = site_shift(g, s_pm, xm, nu, -1);
      M3 a, b, t;
      // upper staple U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
      load_link(U, nu, s_pm, V, a);
      load_link(U, mu, s_pn, V, b);
      mul3<false, true>(a, b, t);
      load_link(U, nu, s, V, a);
      mul3<false, true, true>(t, a, A);
      // lower staple U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
      load_link(U, nu, s_pm_mn, V, a);
      load_link(U, mu, s_mn, V, b);
      mul3<true, true>(a, b, t);
      load_link(U, nu, s_mn, V, a);
      mul3<false, false, true>(t, a, A);
    }
    M3 u, m;
    load_link(U, mu, s, V, u);
    mul3<false, false>(u, A, m);
    tr[0] = m.re[0] + m.re[4] + m.re[8];
    // Im Tr(lambda^c M) for the eight Gell-Mann matrices; T^c = lambda^c / 2
    double q[8];
    q[0] = m.im[3] + m.im[1];
    q[1] = m.re[1] - m.re[3];
    q[2] = m.im[0] - m.im[4];
    q[3] = m.im[6] + m.im[2];
    q[4] = m.re[2] - m.re[6];
    q[5] = m.im[7] + m.im[5];
    q[6] = m.re[5] - m.re[7];
    q[7] = (m.im[0] + m.im[4] - 2.0 * m.im[8]) * 0.57735026918962576451;
    if (F) {
      double* f = F + (int64_t)mu * 8 * V + s;
      const double k = -beta / 6.0;
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) f[(int64_t)cc * V] = k * q[cc];
    }
  }
  if (partials) {
    __shared__ double lds[1][16];
    block_sum<1>(tr, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = tr[0];
  }
}

int gauge_force_blocks(const Geom& g) { return (g.V + 63) / 64; }

hipError_t launch_gauge_force(const Geom& g, const double* U, double beta, double* F, double* partials,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_gauge_force, dim3(gauge_force_blocks(g)), dim3(256), 0, s, g, U, beta, F, partials);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// molecular-dynamics updates of the implicit leapfrog

// 3x3 complex matrices as separate real and imaginary parts, row major
struct Cm3 {
  double re[9], im[9];
};

__device__ __forceinline__ void cm3_mul(const Cm3& a, const Cm3& b, Cm3& c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sr = fma(a.re[3 * i + k], b.re[3 * k + j], fma(-a.im[3 * i + k], b.im[3 * k + j], sr));
        si = fma(a.re[3 * i + k], b.im[3 * k + j], fma(a.im[3 * i + k], b.re[3 * k + j], si));
      }
      c.re[3 * i + j] = sr;
      c.im[3 * i + j] = si;
    }
}

// exp(i H) U per link, H = sum_c a^c T^c: scaling and squaring of the Taylor series.  X = i H is
// scaled by 2^-q until its Frobenius norm is at most 1/4, the series is summed to degree 12 in
// Horner form (remainder below 0.25^13 / 13! < 3e-18 relative), and the result is squared q
// times.  The exponential of an anti-Hermitian traceless matrix is in SU(3), so U1 stays in SU(3)
// to rounding.
__global__ void k_link_exp(Geom g, const double* __restrict__ U0, const double* __restrict__ A,
                           const double* __restrict__ B, double h, double* __restrict__ U1) {
  const int32_t mu = blockIdx.y;
  const int64_t V = g.V;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  double a[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int64_t e = ((int64_t)mu * 8 + c) * V + s;
    a[c] = h * (B ? A[e] + B[e] : A[e]);
  }
  // H = sum_c a^c lambda^c / 2 (Gell-Mann), Hermitian traceless
  const double r3 = 0.57735026918962576451;   // 1 / sqrt(3)
  double hre[9], him[9];
  hre[0] = 0.5 * (a[2] + r3 * a[7]);
  hre[4] = 0.5 * (-a[2] + r3 * a[7]);
  hre[8] = -r3 * a[7];
  him[0] = him[4] = him[8] = 0.0;
  hre[1] = 0.5 * a[0]; him[1] = -0.5 * a[1];
  hre[2] = 0.5 * a[3]; him[2] = -0.5 * a[4];
  hre[5] = 0.5 * a[5]; him[5] = -0.5 * a[6];
  hre[3] = hre[1]; him[3] = -him[1];
  hre[6] = hre[2]; him[6] = -him[2];
  hre[7] = hre[5]; him[7] = -him[5];
  double nrm2 = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) nrm2 += hre[k] * hre[k] + him[k] * him[k];
  double nrm = sqrt(nrm2), scale = 1.0;
  int q = 0;
  while (nrm > 0.25 && q < 64) {   // false for NaN: a NaN momentum gives a NaN link
    nrm *= 0.5;
    scale *= 0.5;
    ++q;
  }
  // Y = i H * scale
  Cm3 Y, E, T;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    Y.re[k] = -him[k] * scale;
    Y.im[k] = hre[k] * scale;
  }
  // E = I + Y/1 (I + Y/2 (I + ... (I + Y/12)))
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    E.re[k] = (k % 4 == 0) ? 1.0 : 0.0;
    E.im[k] = 0.0;
  }
#pragma unroll 1
  for (int m = 12; m >= 1; --m) {
    cm3_mul(Y, E, T);
    const double w = 1.0 / (double)m;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      E.re[k] = ((k % 4 == 0) ? 1.0 : 0.0) + w * T.re[k];
      E.im[k] = w * T.im[k];
    }
  }
#pragma unroll 1
  for (int i = 0; i < q; ++i) {
    cm3_mul(E, E, T);
    E = T;
  }
  Cm3 u;
  const double* um = U0 + (int64_t)mu * 18 * V + s;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    u.re[k] = um[(int64_t)(2 * k) * V];
    u.im[k] = um[(int64_t)(2 * k + 1) * V];
  }
  cm3_mul(E, u, T);
  double* uo = U1 + (int64_t)mu * 18 * V + s;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    uo[(int64_t)(2 * k) * V] = T.re[k];
    uo[(int64_t)(2 * k + 1) * V] = T.im[k];
  }
}

hipError_t launch_link_exp(const Geom& g, const double* U0, const double* A, const double* B, double h, double* U1,
                           hipStream_t s) {
  dim3 grid((unsigned)((g.V + kBlock - 1) / kBlock), 4);
  hipLaunchKernelGGL(k_link_exp, grid, dim3(kBlock), 0, s, g, U0, A, B, h, U1);
  return hipGetLastError();
}

// The transposed left-trivialised differential of the exponential map, per link:
// out = J(omega)^T g with exp(i(omega + eps e_c).T) = exp(i eps (J e_c).T + O(eps^2)) exp(i omega.T),
// so that d/d omega f(exp(i omega.T) U) = J^T (the derivative at the displaced link under left
// multiplication).  In the adjoint representation J = sum_k M^k / (k+1)!, (M v)^d = f^{adc} omega^a v^c,
// and M is antisymmetric, so J^T g = sum_k t_k with t_0 = g, t_k = (omega x t_{k-1}) / (k + 1) and
// (p x q)^d = sum f^{acd} p^a q^c.  The series is summed until a term no longer changes the sum
// (at most 64 terms: enough for |omega| up to about 10).
__global__ void k_dexp_vjp(Geom g, const double* __restrict__ omega, const double* __restrict__ gin,
                           double* __restrict__ gout) {
  const int32_t mu = blockIdx.y;
  const int64_t V = g.V;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  double w[8], t[8], acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int64_t e = ((int64_t)mu * 8 + c) * V + s;
    w[c] = omega[e];
    t[c] = gin[e];
    acc[c] = t[c];
  }
#pragma unroll 1
  for (int k = 1; k <= 64; ++k) {
    double n[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) n[c] = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int a = kF[q].a, b = kF[q].b, c = kF[q].c;
      const double f = kF[q].f;
      // (w x t)_c += f (w_a t_b - w_b t_a), cyclically in (a, b, c)
      n[c] += f * (w[a] * t[b] - w[b] * t[a]);
      n[a] += f * (w[b] * t[c] - w[c] * t[b]);
      n[b] += f * (w[c] * t[a] - w[a] * t[c]);
    }
    const double inv = 1.0 / (double)(k + 1);
    bool changed = false;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      t[c] = n[c] * inv;
      const double nxt = acc[c] + t[c];
      changed = changed || (nxt != acc[c]);
      acc[c] = nxt;
    }
    if (!changed) break;
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) gout[((int64_t)mu * 8 + c) * V + s] = acc[c];
}

hipError_t launch_dexp_vjp(const Geom& g, const double* omega, const double* gin, double* gout, hipStream_t s) {
  dim3 grid((unsigned)((g.V + kBlock - 1) / kBlock), 4);
  hipLaunchKernelGGL(k_dexp_vjp, grid, dim3(kBlock), 0, s, g, omega, gin, gout);
  return hipGetLastError();
}

__global__ void k_axpy_diff(const double* x, const double* __restrict__ y, const double* __restrict__ z, double h,
                            const double* prev, double* out, int64_t n, int32_t steps,
                            double* __restrict__ partials) {
  double d[2] = {0.0, 0.0};
  for (int32_t t = 0; t < steps; ++t) {
    const int64_t i0 = (((int64_t)blockIdx.x * steps + t) * blockDim.x + threadIdx.x) * 4;
    if (i0 < n) {
      double xv[4], yv[4], zv[4], ov[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xv[k] = x[i0 + k];
        yv[k] = y[i0 + k];
        zv[k] = z[i0 + k];
        ov[k] = prev[i0 + k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double o = fma(h, yv[k] - zv[k], xv[k]);
        const double e = o - ov[k];
        out[i0 + k] = o;
        d[0] = fma(e, e, d[0]);
        d[1] = fma(o, o, d[1]);
      }
    }
  }
  __shared__ double lds[2][16];
  block_sum<2>(d, lds);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = d[0];
    partials[gridDim.x + blockIdx.x] = d[1];
  }
}

hipError_t launch_axpy_diff(const double* x, const double* y, const double* z, double h, const double* prev,
                            double* out, int64_t n, double* partials, hipStream_t s) {
  if (n % 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_axpy_diff, dim3(red_num_blocks(n)), dim3(kBlock), 0, s, x, y, z, h, prev, out, n,
                     red_steps(n), partials);
  return hipGetLastError();
}

}  // namespace rmh

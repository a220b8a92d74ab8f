/*
 * rmh.h -- C ABI of the MI355X (gfx950) adjoint-Laplacian library.
 *
 * The hot path of Riemannian-manifold HMC tooling for lattice QCD: the SU(3)
 * gauge-covariant Laplacian in the adjoint representation (section 2, Eq. 3),
 * applied to su(3)-valued link fields inside
 *   - a Chebyshev bandpass recursion giving power spectra per mode (section 2, Eq. 4),
 *   - a multi-shift conjugate-gradient solve applying the rational kinetic mass
 *     term M^{-1} = R(Delta)^2 (section 3, Eq. 5 and Eq. 6),
 * and the derivatives of both with respect to the links (section 3, the mass-term
 * force F_M, with the left-multiplication derivative of section 2).
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice      periodic L[0] x L[1] x L[2] x L[3], every L[mu] >= 2, V = product.
 *              Site index s = x0 + L0*(x1 + L1*(x2 + L2*x3)) (x0 fastest).
 * Operator     Delta = -nabla^2_G >= 0 with spectrum in [0, 16]:
 *              (Delta phi)(x) = 8 phi(x) - sum_mu [ U_mu(x) phi(x+mu) U_mu(x)^dag
 *                                          + U_mu(x-mu)^dag phi(x-mu) U_mu(x-mu) ],
 *              acting on each direction nu of a link field separately.  All spectral
 *              quantities (window edges, shifts sigma) are in Delta units; the paper's
 *              normalised operator -nabla^2_G/16 is Delta/16.
 * su(3) basis  T^a = lambda^a/2 (Gell-Mann), component a = 0..7 is Gell-Mann a+1,
 *              phi = sum_a phi^a T^a, <phi, psi> = sum_a phi^a psi^a.
 * Links        "SoA" U[mu][18][V]: component 2*(3i+j) = Re U_ij, 2*(3i+j)+1 = Im U_ij.
 *              "AoS" U[mu][V][3][3] complex interleaved (re, im) doubles.
 *              Links are SU(3) matrices (unitary, unit determinant, to rounding): the
 *              Laplacian reads rows 0 and 1 of each link and rebuilds row 2 as the complex
 *              conjugate of their cross product, U_2j = conj(U_0k U_1l - U_0l U_1k) for
 *              (j, k, l) cyclic; components 12..17 of the SoA links are not read by it.
 * Link fields  "SoA" F[n][nu][a][V] = F[n][4][8][V] (n counts independent fields).
 *              "AoS" F[n][V][4][8].
 * dtype        RMH_F64 (double) or RMH_F32 (float) for links and fields where a call
 *              takes a dtype; the computation runs in that precision, every dot product
 *              and moment is accumulated in FP64.
 * Pointers     "device" pointers are HIP device memory on the current device, 256-byte
 *              aligned; "host" pointers are ordinary host memory.  The caller owns
 *              every buffer.  The library never allocates device memory; scratch comes
 *              from a caller-provided workspace sized by rmh_workspace_bytes().
 *              Outputs must not overlap inputs (checked by address range: RMH_E_ARG).
 * Streams      rmh_stream is a hipStream_t (NULL = the default stream).  Work is
 *              ordered on that stream.  Calls that return host scalars (moments,
 *              power, K, stats) synchronize the stream before returning; the others
 *              return after enqueueing.
 * Errors       every call returns an rmh_status; nothing is thrown.  rmh_last_error()
 *              gives a thread-local message for the last failing call.
 *              Reductions are deterministic (fixed order): repeated calls give
 *              bitwise-identical results.
 * Environment  RMH_LOG=1 prints the solver's and the autotuner's diagnostics to stderr;
 *              nothing else is read from the environment (launch shapes come only from
 *              rmh_tune_set, rmh_tune_load, rmh_autotune_laplacian or the built-in defaults).
 */
#ifndef RMH_H
#define RMH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* rmh_stream; /* a hipStream_t */

typedef enum {
  RMH_OK = 0,
  RMH_E_ARG = 1,           /* bad pointer, size, aliasing or option */
  RMH_E_SHAPE = 2,         /* lattice extent < 2 or too large */
  RMH_E_WORKSPACE = 3,     /* workspace smaller than rmh_workspace_bytes() */
  RMH_E_POLES = 4,         /* shift sigma_j <= 0, complex or repeated roots */
  RMH_E_NOCONV = 5,        /* solver hit maxiter; outputs hold the last iterate */
  RMH_E_BREAKDOWN = 6,     /* non-finite or non-positive CG scalar (e.g. NaN source) */
  RMH_E_HIP = 7,           /* a HIP runtime call failed */
  RMH_E_UNIMPLEMENTED = 8,
  RMH_E_HOST = 9           /* host-side failure (e.g. out of host memory); nothing is thrown */
} rmh_status;

typedef enum { RMH_F64 = 0, RMH_F32 = 1 } rmh_dtype;

/* Chebyshev bandpass windows (section 2): B_w(Delta) = sum_{k=0}^{degree} g_k c^w_k T_k(Delta/8 - 1),
 * c^w_k the Chebyshev coefficients of the indicator of window w, g_k the Jackson kernel
 * (kernel = 1) or 1 (kernel = 0).  edges: host, n_windows + 1 ascending values in [0, 16],
 * or NULL for n_windows equal windows.  degree <= 100000 and 1 <= n_windows <= 4096 (64 for
 * rmh_cheb_filter); the device calls need degree >= 1; RMH_E_ARG outside. */
typedef struct {
  int32_t degree;
  int32_t n_windows;
  const double* edges;
  int32_t kernel;
} rmh_cheb;

/* R(Delta) = c + sum_j r_j (Delta + sigma_j)^{-1} (section 3, Eq. 6 in partial fractions,
 * Delta units).  r, sigma: host arrays of n_poles values, sigma_j > 0; 1 <= n_poles <= 64
 * (RMH_E_ARG outside). */
typedef struct {
  double c;
  int32_t n_poles;
  const double* r;
  const double* sigma;
} rmh_rational;

/* Shifted-solve controls.  tol: per-shift FP64 true relative residual
 * ||x - (Delta + sigma_j) x_j|| / ||x|| that every shift must reach.  mode 0: FP64 multi-shift
 * CG; mode 1: mixed precision -- FP64 iterations while the seed residual is above
 * mixed_switch * ||x|| (0 = default 1e-4, negative = none), then FP32 stencil and vectors with
 * FP64 reliable updates of the seed residual (delta = reliable-update threshold in (0, 1): an update
 * once the seed residual fell below delta times its largest value since the last one, e.g. 0.01).
 * check_every: at most this many iterations between host convergence checks (0 = 8); after the
 * first, each check is placed where the seed's convergence rate so far predicts the next threshold
 * (the switch to FP32, then tol).  basis: iterations per
 * segment of the shift solutions (0 = 32 in mode 0, 16 in mode 1; at most 32): the shifts other
 * than the seed are carried as coefficients over the stored seed residuals of a segment and
 * folded into their FP64 vectors once per segment, so the workspace holds basis + 1 extra link
 * fields per source
 * (mode 1: plus min(2 (basis + 1), 33) FP32 residuals, where the FP32 phase, and the segment open
 * at the switch of precision, go on).  multishift_target: the multi-shift recursion stops once every
 * shift's recursive residual is below multishift_target * tol (0 = default 0.5); every pair whose
 * FP64 true residual is then above tol is refined by its own correction solve (targets above 1
 * leave pairs for that refinement on purpose; range [0, 1e6] with multishift_target * tol < 1). */
typedef struct {
  double tol;
  int32_t maxiter;
  int32_t mode;
  double delta;
  int32_t check_every;
  double mixed_switch;
  int32_t basis;
  double multishift_target;
} rmh_solver;

/* Per-call solver statistics (host). */
typedef struct {
  int32_t iters;            /* multi-shift iterations (summed over the solves of the call) */
  int32_t reliable_updates; /* FP64 reliable updates */
  int32_t refine_iters;     /* iterations spent in per-shift refinement */
  int32_t refine_rounds;
  int32_t fp64_iters;       /* iterations done in FP64 (mode 1: before the switch) */
  int32_t reserved;
  double true_relres_max;   /* max over fields and shifts of the final FP64 true residual */
  double seconds;           /* wall time of the call */
} rmh_stats;

/* Operations for rmh_workspace_bytes(). */
typedef enum {
  RMH_OP_LAPLACIAN = 0,
  RMH_OP_LAPLACIAN_BWD = 1,
  RMH_OP_POWER_SPECTRUM = 2,
  RMH_OP_CHEB_FILTER = 3,
  RMH_OP_RATIONAL_APPLY = 4,
  RMH_OP_RATIONAL_APPLY_BWD = 5,
  RMH_OP_KINETIC_FORCE = 6,
  RMH_OP_CHEB_FILTER_BWD = 7,
  RMH_OP_POWER_SPECTRUM_BWD = 8,
  RMH_OP_GAUGE_FORCE = 9,
  RMH_OP_HEATBATH = 10,
  RMH_OP_LEAPFROG = 11,
  RMH_OP_AUTOTUNE = 12
} rmh_op;

/* ---------------------------------------------------------------------------------------- */
/* library */

/* Thread-local description of the last error (never NULL). */
const char* rmh_last_error(void);
/* ABI version (major * 100 + minor). */
int32_t rmh_version(void);
/* Workspace bytes for op at this shape.  aux = n_windows (POWER_SPECTRUM, CHEB_FILTER) or
 * n_poles (RATIONAL_*, KINETIC_FORCE); degree = Chebyshev degree (POWER_SPECTRUM,
 * CHEB_FILTER) or the solver's basis (RATIONAL_*, KINETIC_FORCE; 0 = default), else 0;
 * mode = solver mode (else 0).  Returns 0 on a bad argument (and sets the error string). */
size_t rmh_workspace_bytes(int32_t op, const int32_t L[4], int32_t dtype, int32_t n_rhs, int32_t aux,
                           int32_t degree, int32_t mode);

/* ---------------------------------------------------------------------------------------- */
/* layout (ingest); pure data movement, bitwise, plus FP64 -> FP32 round-to-nearest-even */

/* U_soa[mu][18][V] (dtype) <- U_aos[mu][V][3][3] complex doubles.  Both device. */
rmh_status rmh_pack_links(const int32_t L[4], const double* U_aos, void* U_soa, int32_t dtype,
                          rmh_stream stream);
/* U_aos <- U_soa (FP64 only).  Both device. */
rmh_status rmh_unpack_links(const int32_t L[4], const double* U_soa, double* U_aos, rmh_stream stream);
/* F_soa[n][4][8][V] (dtype) <- F_aos[n][V][4][8] doubles.  Both device. */
rmh_status rmh_pack_fields(const int32_t L[4], int32_t n, const double* F_aos, void* F_soa, int32_t dtype,
                           rmh_stream stream);
/* F_aos (doubles) <- F_soa (dtype).  Both device. */
rmh_status rmh_unpack_fields(const int32_t L[4], int32_t n, const void* F_soa, int32_t dtype, double* F_aos,
                             rmh_stream stream);
/* out[i] = (float) in[i] (round to nearest even), n elements, device. */
rmh_status rmh_convert_f64_f32(const double* in, float* out, int64_t n, rmh_stream stream);

/* ---------------------------------------------------------------------------------------- */
/* the operator (section 2, Eq. 3) */

/* y = (Delta + shift) x for n_rhs link fields.  U: device SoA links; x, y: device SoA link
 * fields [n_rhs][4][8][V]; all of the given dtype.  y must not overlap x or U. */
rmh_status rmh_laplacian_apply(const int32_t L[4], const void* U, int32_t dtype, const void* x, void* y,
                               int32_t n_rhs, double shift, rmh_stream stream);

/* Vector-Jacobian product of y = (Delta[U] + shift) x with cotangent g.
 * grad_x (optional, device, dtype) = (Delta + shift) g.
 * grad_omega (optional, device, FP64 [n_out][4][8][V]) = d<g, Delta[U] x>/d omega^c_mu(x) for
 * U_mu(x) -> exp(i omega^c T^c) U_mu(x) (the left-multiplication derivative of section 2);
 * n_out = n_rhs when per_rhs != 0 (one gradient per field pair) else 1 (summed).
 * Computed in FP64: U, x, g must be RMH_F64 when grad_omega is requested. */
rmh_status rmh_laplacian_apply_bwd(const int32_t L[4], const void* U, int32_t dtype, const void* x,
                                   const void* g, int32_t n_rhs, double shift, void* grad_x,
                                   double* grad_omega, int32_t per_rhs, rmh_stream stream);

/* ---------------------------------------------------------------------------------------- */
/* Chebyshev bandpass filters and power spectra (section 2, Eq. 4) */

/* Host: coef[w][k] = g_k c^w_k, n_windows x (degree + 1); 0 <= degree <= 100000,
 * 1 <= n_windows <= 4096 (RMH_E_ARG outside). */
rmh_status rmh_cheb_coefficients(const rmh_cheb* cheb, double* coef);

/* Moments mu[n][k] = <F_n, T_k(A) F_n>, A = Delta/8 - 1, k = 0..degree, summed over nu, and
 * power[n][w] = <F_n, B_w F_n> = sum_k g_k c^w_k mu[n][k] (the numerator of Eq. 4).
 * The recursion t_{k+1} = 2 A t_k - t_{k-1} runs for ceil(degree/2) stencil sweeps and uses
 * mu_{2k} = 2<t_k,t_k> - mu_0, mu_{2k+1} = 2<t_{k+1},t_k> - mu_1.
 * U, F: device (dtype); moments: host [n_rhs][degree+1] (or NULL); power: host
 * [n_rhs][n_windows] (or NULL).  Synchronizes the stream. */
rmh_status rmh_power_spectrum(const int32_t L[4], const void* U, int32_t dtype, const void* F, int32_t n_rhs,
                              const rmh_cheb* cheb, double* moments, double* power, void* ws, size_t ws_bytes,
                              rmh_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): rmh_power_spectrum with its recursion vectors and
 * partial sums in the library's static device scratch instead of a workspace argument.  The
 * scratch is 64 MiB per device (a file-scope device array, held until the process ends); a call
 * that needs more (the same amount rmh_workspace_bytes(RMH_OP_POWER_SPECTRUM, ...) reports, e.g.
 * more than one FP64 source at 16^4) returns RMH_E_WORKSPACE before touching any pointer.  The
 * call allocates nothing: no hipMalloc, hipFree or pinned host staging (the sums come back by a
 * plain device-to-host copy).  Every call on one device shares that device's scratch, so calls that
 * overlap on one device (other threads, other streams) race; successive calls are independent
 * (nothing in the scratch needs to start at zero).  Results equal rmh_power_spectrum's bit for bit. */
rmh_status rmh_power_spectrum_noalloc(const int32_t L[4], const void* U, int32_t dtype, const void* F,
                                      int32_t n_rhs, const rmh_cheb* cheb, double* moments, double* power,
                                      rmh_stream stream);

/* Host: ratio[n][w] = power[n][w] / Tr B_w with Tr B_w = sum_k g_k c^w_k trace_moments[k]
 * (Eq. 4, power per mode).  trace_moments[k] = Tr T_k(A) over the link-field space
 * (e.g. rmh_trace_moments_free, or the mean moments of Gaussian sources). */
rmh_status rmh_power_ratio(const rmh_cheb* cheb, const double* trace_moments, const double* power,
                           int32_t n_rhs, double* ratio);

/* Host: exact Tr T_k(A), k = 0..degree (0 <= degree <= 100000), over the link-field space (32 V) at U = 1, where the
 * eigenvalues of Delta are 4 sum_mu sin^2(p_mu/2), p_mu = 2 pi n_mu / L_mu. */
rmh_status rmh_trace_moments_free(const int32_t L[4], int32_t degree, double* trace_moments);

/* y[w][n] = B_w x_n for every window (vector output).  x: device [n_rhs][4][8][V]; y: device
 * [n_windows][n_rhs][4][8][V]; dtype for both.  At most 64 windows.  Runs degree sweeps; the
 * recursion vectors go into a workspace ring of min(16, max(3, degree)) fields and are folded
 * into y once per ring (sums in FP64), so y is read and written once per 16 sweeps.  The
 * window coefficients are copied to the workspace first (the stream is synchronized once). */
rmh_status rmh_cheb_filter(const int32_t L[4], const void* U, int32_t dtype, const void* x, int32_t n_rhs,
                           const rmh_cheb* cheb, void* y, void* ws, size_t ws_bytes, rmh_stream stream);

/* Vector-Jacobian product of the filters y_w = B_w x (section 2, the bandpass of Eq. 4) with
 * cotangents gy (device FP64 [n_windows][n_rhs][4][8][V]):
 * grad_x (optional, device FP64 [n_rhs][4][8][V]) = sum_w B_w gy_w (B_w is symmetric);
 * grad_omega (optional, device FP64 [n_out][4][8][V], n_out = per_rhs ? n_rhs : 1)
 *   = d(sum_w <gy_w, y_w>)/d omega^c_mu(x) for U_mu(x) -> exp(i omega^c T^c) U_mu(x).
 * U, x: device FP64.  At least one output.  Reverse Chebyshev sweep: 3 degree stencil sweeps and
 * degree link-derivative passes; workspace: 4 link fields per source (RMH_OP_CHEB_FILTER_BWD,
 * aux = n_windows).  Outputs are overwritten and must not overlap an input or the workspace. */
rmh_status rmh_cheb_filter_bwd(const int32_t L[4], const double* U, const double* x, const double* gy, int32_t n_rhs,
                               const rmh_cheb* cheb, double* grad_x, double* grad_omega, int32_t per_rhs, void* ws,
                               size_t ws_bytes, rmh_stream stream);
/* Vector-Jacobian product of power[n][w] = <F_n, B_w F_n> (Eq. 4 numerator) with host cotangent
 * gamma[n_rhs][n_windows]:
 * grad_F (optional, device FP64 [n_rhs][4][8][V]) = 2 sum_w gamma[n][w] B_w F_n;
 * grad_omega (optional, as above) = d(sum_{n,w} gamma[n][w] power[n][w])/d omega.
 * U, F: device FP64.  Workspace: RMH_OP_POWER_SPECTRUM_BWD.  Same conventions as
 * rmh_cheb_filter_bwd. */
rmh_status rmh_power_spectrum_bwd(const int32_t L[4], const double* U, const double* F, int32_t n_rhs,
                                  const rmh_cheb* cheb, const double* gamma, double* grad_F, double* grad_omega,
                                  int32_t per_rhs, void* ws, size_t ws_bytes, rmh_stream stream);

/* ---------------------------------------------------------------------------------------- */
/* rational mass term (section 3, Eq. 5 and Eq. 6) */

/* Host: Eq. 6 terms (a0_i + a1_i L)/(b0_i + b1_i L + L^2), L = Delta/16, split into 2 n_terms
 * real poles r/(Delta + sigma) (r = 16 rho, sigma = 16 s).  RMH_E_POLES when a term has no
 * two distinct real roots or a root gives sigma <= 0.  r, sigma: host, 2 n_terms each. */
rmh_status rmh_rational_from_quadratics(int32_t n_terms, const double* a0, const double* a1, const double* b0,
                                        const double* b1, double* r, double* sigma);

/* Host: n-pole R with R(Delta)^2 ~ (1 - kappa + kappa Delta)^{-1} on [0, 16] (midpoint rule on
 * y^{-1/2} = (2/pi) sqrt(s) int_0^{pi/2} dt / (s sin^2 t + y cos^2 t), s = sqrt((1-kappa)(1+15 kappa))).
 * c = 0; r, sigma: host, n values each.  0 < kappa < 1. */
rmh_status rmh_rational_kappa(double kappa, int32_t n, double* c, double* r, double* sigma);

/* y_n = c x_n + sum_j r_j (Delta + sigma_j)^{-1} x_n for n_rhs link fields, every shift solved to
 * the FP64 true relative residual solver->tol by multi-shift CG (seed = smallest sigma),
 * followed by per-shift refinement of any shift above tol.
 * U: device FP64 SoA links; x, y: device FP64 [n_rhs][4][8][V];
 * x_poles: optional device FP64 [n_rhs][n_poles][4][8][V] receiving x_j;
 * K: optional host [n_rhs] receiving 1/2 <y_n, y_n> (Eq. 5 with M^{-1} = R^2);
 * stats: optional host.  Synchronizes the stream.  RMH_E_NOCONV leaves the last iterate. */
rmh_status rmh_rational_apply(const int32_t L[4], const double* U, const double* x, int32_t n_rhs,
                              const rmh_rational* rat, const rmh_solver* solver, double* y, double* x_poles,
                              double* K, rmh_stats* stats, void* ws, size_t ws_bytes, rmh_stream stream);

/* RMHMC heat-bath momenta for the kinetic term 1/2 P M^{-1} P with M = R(Delta)^{-2} (section 3):
 * P = M^{1/2} xi = R(Delta)^{-1} xi for Gaussian xi.
 * kappa in (0, 1]: rat must be a pole set with R(Delta)^2 ~ (1 - kappa + kappa Delta)^{-1}
 * (rmh_rational_kappa(kappa, n)), and R^{-1} is taken as (1 - kappa + kappa Delta) R, exact to the
 * pole set's accuracy: one multi-shift solve (to the solver's true residual) and one stencil.
 * kappa = 0: R^{-1} exactly, for any rat with c >= 0, r_j > 0 and distinct sigma_j > 0, through the
 * partial fractions 1/R(l) = a l + b + sum_k rho_k / (l + tau_k) (tau_k > 0 the negated zeros of R,
 * n_poles - 1 of them for c = 0, n_poles for c > 0; RMH_E_POLES when R has no such form): one
 * multi-shift solve with the shifts tau_k and one stencil, exact to the solver's tolerance.
 * xi, P: device FP64 [n_rhs][4][8][V]; U: device FP64.  Workspace: RMH_OP_HEATBATH (aux = n_poles,
 * degree = solver basis, mode).  Synchronizes the stream.  Projection onto a spectral window
 * (section 3) is rmh_cheb_filter of P. */
rmh_status rmh_heatbath_momenta(const int32_t L[4], const double* U, const double* xi, int32_t n_rhs, double kappa,
                                const rmh_rational* rat, const rmh_solver* solver, double* P, rmh_stats* stats,
                                void* ws, size_t ws_bytes, rmh_stream stream);

/* Vector-Jacobian product of y = R(Delta[U]) x with cotangent g (both FP64 [n_rhs][4][8][V]):
 * grad_x (optional, device FP64) = R(Delta) g;
 * grad_omega (device FP64 [n_out][4][8][V], n_out = per_rhs ? n_rhs : 1)
 *   = d<g, R(Delta[U]) x>/d omega = -sum_j r_j d<z_j, Delta x_j>/d omega,
 *   x_j = (Delta + sigma_j)^{-1} x, z_j = (Delta + sigma_j)^{-1} g.
 * Both multi-shift solves are recomputed; nothing is kept from a forward call.
 * The kinetic force of section 3 is F_M = -grad_omega with g = y = R(Delta) P. */
rmh_status rmh_rational_apply_bwd(const int32_t L[4], const double* U, const double* x, const double* g,
                                  int32_t n_rhs, const rmh_rational* rat, const rmh_solver* solver,
                                  double* grad_x, double* grad_omega, int32_t per_rhs, rmh_stats* stats,
                                  void* ws, size_t ws_bytes, rmh_stream stream);

/* One RMHMC kinetic-force evaluation: Y = R(Delta) P, K_n = 1/2 <Y_n, Y_n>, and
 * dK/domega (device FP64 [n_out][4][8][V]); two multi-shift solves (P, then Y) and the link
 * derivative.  Y (optional device FP64), K (optional host [n_rhs]).  Synchronizes. */
rmh_status rmh_kinetic_force(const int32_t L[4], const double* U, const double* P, int32_t n_rhs,
                             const rmh_rational* rat, const rmh_solver* solver, double* Y, double* K,
                             double* dK_domega, int32_t per_rhs, rmh_stats* stats, void* ws, size_t ws_bytes,
                             rmh_stream stream);

/* ---------------------------------------------------------------------------------------- */
/* gauge force (the force whose power spectra section 2 measures, Fig. 1) */

/* Wilson plaquette action S_W = beta sum_x sum_{mu<nu} (1 - Re Tr U_{mu nu}(x) / 3) and its gauge
 * force F_G = -dS_W / d omega^c_mu(x) for U_mu(x) -> exp(i omega^c T^c) U_mu(x) (the
 * left-multiplication derivative of section 2): F^c_mu(x) = -(beta/3) Im Tr(T^c U_mu(x) A_mu(x)),
 * A_mu(x) the sum of the six staples.  U: device FP64 SoA links.  F (optional): device FP64
 * [4][8][V], a link field ready for rmh_power_spectrum.  S (optional): host, the action; needs a
 * workspace (RMH_OP_GAUGE_FORCE) and synchronizes the stream.  At least one of F, S. */
rmh_status rmh_wilson_gauge_force(const int32_t L[4], const double* U, double beta, double* F, double* S, void* ws,
                                  size_t ws_bytes, rmh_stream stream);

/* ---------------------------------------------------------------------------------------- */
/* molecular dynamics: the implicit leapfrog step of RMHMC (section 3) */

/* Step controls: step size eps (molecular-dynamics time), Wilson coupling beta, and the
 * fixed points' relative tolerance and iteration limit. */
typedef struct {
  double eps;
  double beta;
  double fp_tol;
  int32_t fp_maxiter;
} rmh_leapfrog;

typedef struct {
  int32_t p_iters;   /* fixed-point iterations of the half-step momentum */
  int32_t u_iters;   /* fixed-point iterations of the link update */
  double p_res;      /* last relative change of the half-step momentum */
  double u_res;      /* last relative change of Pi(U', P_h) */
  rmh_stats solver;  /* every multi-shift solve of the step, summed */
} rmh_leapfrog_stats;

/* One implicit (generalized) leapfrog step for the non-separable Hamiltonian of section 3,
 * H(U, P) = 1/2 <R(Delta) P, R(Delta) P> + S_W(U) (Eq. 5 with M^-1 = R^2; the log|M| term is not
 * included: the paper realises it with auxiliary fields it does not define).  Links move by left
 * multiplication, dU/dt = i Pi^a T^a U with Pi = dH/dP = R(Delta)^2 P, and dP/dt = F = F_G - dK/d omega.
 * With h = eps / 2:
 *   P_h = P + h F(U, P_h)                               (fixed point, from P_h = P),
 *   U'  = exp(i h (Pi(U, P_h) + Pi(U', P_h))^a T^a) U   (fixed point, from Pi(U') = Pi(U)),
 *   P'  = P_h + h F(U', P_h).
 * A fixed point keeps the first iterate whose successor differs from it by at most fp_tol relative
 * to the successor (stage 1: P_h; stage 2: U', comparing Pi(U', P_h) with the Pi that built U'), so
 * the solves of the kept iterate serve the next stage: 2 (n_1 + n_2) multi-shift solves for n_1, n_2
 * iterations.  After fp_maxiter iterations the step goes on with the last iterate and returns
 * RMH_E_NOCONV.  Every solve runs to solver->tol.  The step is time reversible: from (U', -P') it
 * returns to (U, -P) up to the tolerances.
 * U0, U1: device FP64 SoA links (distinct buffers); P0, P1: device FP64 [4][8][V] (distinct).
 * Workspace: RMH_OP_LEAPFROG (n_rhs = 1, aux = n_poles, degree = solver basis, mode).
 * stats: optional host.  Synchronizes the stream. */
rmh_status rmh_leapfrog_step(const int32_t L[4], const double* U0, const double* P0, const rmh_rational* rat,
                             const rmh_solver* solver, const rmh_leapfrog* lf, double* U1, double* P1,
                             rmh_leapfrog_stats* stats, void* ws, size_t ws_bytes, rmh_stream stream);

/* ---------------------------------------------------------------------------------------- */
/* stencil launch tuning */

/* A stencil launch configuration.  form 0 = adjoint 8x8 action R(U) built per hop, 1 = 3x3 matrix
 * products U phi U^dag, 2 = R(U) built and applied two columns at a time; block = 64, 128 or 256
 * threads; xcd_remap = 1 maps consecutive lattice blocks onto one XCD (L2 locality); nv = 4, 2 or 1
 * directions per thread (1 with form 1 only, and block * nv / 4 a multiple of the 64-wide wave);
 * order = 1 visits the blocks with x3 fastest (x2/x3 neighbours resident together; used when
 * L0*L1 is a multiple of the sites per block); order = 2 splits each site over four lanes, one per
 * direction mu, summed by wave shuffles (four times the threads, for small lattices; walk is then
 * ignored), and order = 3 is that shape visiting its blocks with x3 fastest (as order 1); walk =
 * K > 0 makes each thread walk K consecutive x3 sites carrying the x3 neighbours in registers
 * (used when K divides L3); ns = 2 or 4 (nv = 4, form 0 or 2, order 0 or 1, no walk; 4 in FP32
 * only) makes each thread apply the operator to ns fields of a batch, so each link and adjoint
 * matrix serves 4 ns vectors (used when ns divides the batch); tile2 = 2 or 4 (with a walk) gives
 * each walking block an L0 x R x tile2 tile of (x0, x1, x2) columns instead of consecutive
 * columns, so part of its x2 neighbours are its own (used when the tile divides the plane).  Every
 * configuration computes the
 * same operator; a form fixes the per-site arithmetic, so results are bitwise identical across
 * block sizes, remaps, nv, ns, orders 0 and 1 and walks of one form (orders 2 and 3 sum the eight
 * hops in another order: equal to rounding). */
typedef struct {
  int32_t form, block, xcd_remap, nv, order, walk, ns, tile2;
} rmh_hop_config;

/* What a stencil launch is for: the drivers look up their configurations under these purposes
 * (an entry stored for RMH_PURPOSE_ANY serves every purpose without one of its own). */
typedef enum {
  RMH_PURPOSE_ANY = -1,
  RMH_PURPOSE_APPLY = 0,     /* rmh_laplacian_apply */
  RMH_PURPOSE_CG = 1,        /* multi-shift CG iterations in the working precision */
  RMH_PURPOSE_CG64 = 2,      /* FP64 residuals: reliable updates, true residuals, refinement */
  RMH_PURPOSE_MOMENTS = 3,   /* power-spectrum sweeps (recursion step with FP64 dot products) */
  RMH_PURPOSE_FILTER = 4,    /* vector-filter sweeps (recursion step) */
  RMH_PURPOSE_CHEB_BWD = 5,  /* backward Chebyshev sweeps */
  RMH_PURPOSE_HEATBATH = 6   /* the Delta of the heat-bath momenta */
} rmh_purpose;

/* Store the configuration for lattice L, dtype, launches over n_rhs link fields and a purpose
 * (RMH_E_ARG for an invalid configuration or purpose).  Lookups take the entry of that key, else the
 * RMH_PURPOSE_ANY entry of that batch, else the nearest batch size of the purpose, else of
 * RMH_PURPOSE_ANY, else built-in defaults by lattice size, dtype and batch. */
rmh_status rmh_tune_set(const int32_t L[4], int32_t dtype, int32_t n_rhs, int32_t purpose, const rmh_hop_config* cfg);
/* Time every stencil configuration on the caller's buffers and keep the fastest for (L, dtype, n_rhs,
 * purpose).  The timing unit: for RMH_PURPOSE_MOMENTS, _FILTER and _CHEB_BWD the recursion step
 * y = -H x / 4 - y (written over its z input, as the sweeps write t_{k+1} over t_{k-1}; y is zeroed
 * first); for _APPLY, _CG, _CG64 and _HEATBATH the plain y = (8 - H) x; for _ANY both (the
 * pair); with the per-block FP64 dot products that the purpose's drivers fuse into the launch
 * (_CG, _CG64: one, _MOMENTS: three), written into the workspace ws (device, ws_bytes >=
 * rmh_workspace_bytes(RMH_OP_AUTOTUNE, L, dtype, n_rhs, 0, 0, 0)); reps units each, HIP events on
 * the stream, y overwritten.  best (optional, host) receives the configuration, best_ms (optional)
 * the mean time of one unit.  RMH_E_ARG for null pointers or y or ws overlapping x, U or each
 * other, RMH_E_WORKSPACE for a short workspace.  Synchronizes the stream. */
rmh_status rmh_autotune_laplacian(const int32_t L[4], const void* U, int32_t dtype, const void* x, void* y,
                                  int32_t n_rhs, int32_t purpose, int32_t reps, rmh_hop_config* best,
                                  double* best_ms, void* ws, size_t ws_bytes, rmh_stream stream);
/* Write every stored configuration to a JSON file at path (host), stamped with the current
 * device's architecture name (gcnArchName) and the HIP runtime version; *n_saved (optional) receives
 * the entry count.  RMH_E_HOST if the file cannot be written. */
rmh_status rmh_tune_save(const char* path, int32_t* n_saved);
/* Read a file written by rmh_tune_save and store its entries, if its architecture and runtime
 * version match the current device's (else nothing is stored and *n_loaded = 0); *n_loaded
 * (optional) receives the count stored.  RMH_E_HOST if the file cannot be read, RMH_E_ARG if it
 * is not such a file or holds an invalid configuration. */
rmh_status rmh_tune_load(const char* path, int32_t* n_loaded);
/* Forget every stored configuration. */
rmh_status rmh_tune_clear(void);

/* ---------------------------------------------------------------------------------------- */
/* Link displacements (section 2: links vary by left multiplication with exp(i omega^c T^c)) */

/* U1_mu(x) = exp(i omega^c_mu(x) T^c) U0_mu(x) for every link.  U0, U1: device FP64 SoA links
 * [4][18][V] (U1 must not overlap U0); omega: device FP64 [4][8][V].  The exponential is summed by
 * scaling and squaring of its Taylor series, so U1 stays in SU(3) to rounding. */
rmh_status rmh_link_exp(const int32_t L[4], const double* U0, const double* omega, double* U1, rmh_stream stream);

/* The chain rule through that displacement: out = J(omega)^T g per link, where g is the derivative
 * of a function f with respect to a left-multiplication displacement at the displaced links
 * exp(i omega.T) U0 (what the backward calls return) and out the derivative of
 * f(exp(i omega.T) U0) with respect to omega itself.  J is the left-trivialised differential of
 * the exponential map, J = sum_k M^k / (k+1)!, (M v)^d = f^{adc} omega^a v^c.  omega, g, out: device
 * FP64 [4][8][V]; out may alias g.  Converges for |omega| up to about 10 per link. */
rmh_status rmh_link_exp_vjp(const int32_t L[4], const double* omega, const double* g, double* out,
                            rmh_stream stream);

/* ---------------------------------------------------------------------------------------- */
/* kernel timing */

/* Kernel classes of rmh_profile_read. */
typedef enum {
  RMH_PROF_STENCIL = 0,      /* every Delta application (all drivers) */
  RMH_PROF_CG_RESIDUAL = 1,  /* the seed's vector updates: r -= alpha A p with <r, r>, p = r + beta p */
  RMH_PROF_CG_SHIFTS = 2,    /* folds of the shift solutions and directions over the residual ring */
  RMH_PROF_FORCE = 3,        /* link derivative */
  RMH_PROF_CHEB_FOLD = 4,    /* folds of the Chebyshev filter's recursion vectors into its window outputs */
  RMH_PROF_N = 5
} rmh_prof_class;

/* enable != 0: record a HIP event pair on the call's stream around every launch of the classes
 * above and accumulate launches, event time and algorithmic bytes (links, inputs and outputs
 * counted once per launch; for the shift updates only the shifts still active).  Enabling or
 * disabling resets the counters. */
rmh_status rmh_profile_enable(int32_t enable);
/* Totals of one class since the last reset (waits for the recorded events).  total_items counts
 * link fields processed (for the stencil: link-field applications of Delta). */
rmh_status rmh_profile_read(int32_t cls, int64_t* launches, double* total_ms, double* total_bytes,
                            double* total_items);

#ifdef __cplusplus
}
#endif

#endif /* RMH_H */

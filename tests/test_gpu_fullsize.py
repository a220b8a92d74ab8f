"""GPU checks at the full workload sizes, on outputs the oracle can compute site by site and on
properties that hold at any size, plus the batched spectrum's grid at a size the oracle affords.

* The batched FP32 power spectrum of 32 Gaussian sources on Haar links, degree 256, 64 windows: on
  an 8x8x4x4 lattice every moment and window power of four sources (one from each of four field
  groups of the batched grid) against the oracle's recursion, with the launch shape the 24^4
  workload uses and with the small-lattice default; at 24^4 the first moments of two sources in
  different field groups against the oracle, and the U = 1 control of all 32 sources, whose moments
  the oracle gives exactly through the FFT.
* 32^3 x 64, eps = 0.4 links: the stencil (FP64 and FP32) and the Wilson gauge force at sampled
  sites, a 16-pole
  mixed-precision rational solve checked shift by shift at sampled sites, and the kinetic force of
  two momentum fields (16 poles, mixed precision) at sampled links against the oracle's per-link
  derivative fed the pole solutions (each verified by its residual at sampled sites), then the
  first moments of the 128-window spectrum of those forces against dot products of the verified
  stencil.

FP32 moment tolerance at degree 256: the stable recursion's error grows at most linearly in k;
the test takes |mu_gpu - mu_orc| <= 1e-4 mu_0 (2.6e-5 expected from 256 steps of ~1e-7), and a
window power within sum_k |coef_wk| times that.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import announce, dev
from oracle import chebyshev as och
from oracle import gauge as ogauge
from oracle import laplacian as olap
from oracle import rational as orat
from paper_2112_04556_amd import api, inputs

pytestmark = pytest.mark.gpu


def _sample_sites(V, n, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, V - 1], rng.integers(0, V, n)]))


_SPECTRUM_ORACLE = {}


def _haar_spectrum_reference(L, n, D, nw, picks):
    """Oracle moments and powers of the FP32-rounded inputs for the picked sources (cached: two
    launch shapes are checked against one reference)."""
    key = (L, n, D, nw, picks)
    if key not in _SPECTRUM_ORACLE:
        U = inputs.random_links(L, "haar", seed=3)
        F = inputs.gaussian_fields(L, n, seed=3)
        U32 = U.numpy().astype(np.complex64).astype(np.complex128)
        F32 = F.numpy().astype(np.float32).astype(np.float64)
        mu, pw = och.power_spectrum(U32, F32[list(picks)], L, D, och.equal_windows(nw))
        _SPECTRUM_ORACLE[key] = (U, F, mu, pw)
    return _SPECTRUM_ORACLE[key]


@pytest.mark.parametrize("shape", ["default", "24^4 launch shape"])
def test_batched_spectrum_haar_parity(shape):
    """32 sources (eight field groups of four) at degree 256 with 64 windows, FP32 stencil with FP64
    moments, one batched call; four sources from field groups 0, 1, 4 and 7 against the oracle."""
    L = (8, 8, 4, 4)
    n, D, nw = 32, 256, 64
    picks = (0, 5, 18, 31)
    announce(f"8x8x4x4 haar: 32 sources, D=256, 64 windows, fp32, {shape}")
    U, F, mu_ref, pw_ref = _haar_spectrum_reference(L, n, D, nw, picks)
    Ud = api.pack_links(L, U.to(dev()), torch.float32)
    Fd = F.to(dev()).to(torch.float32)
    if shape != "default":
        # the shape the 24^4, 32-source spectrum runs with: one thread per site and all four
        # directions, streamed adjoint form, block 64, XCD remap, x3-fastest block order
        api.tune_set(L, torch.float32, n, form=2, block=64, xcd_remap=1, nv=4, order=1, walk=0)
    try:
        mom, pw = api.power_spectrum(L, Ud, Fd, D, nw)
    finally:
        api.tune_clear()
    mu0 = mom[list(picks), :1]
    assert np.all(np.abs(mom[list(picks)] - mu_ref) <= 1e-4 * mu0)
    coef = och.window_coefficients(och.equal_windows(nw), D)
    bound = 1e-4 * mu0 * np.abs(coef).sum(axis=1)[None, :]
    assert np.all(np.abs(pw[list(picks)] - pw_ref) <= bound)
    # every source: mu_0 = |F|^2 of the FP32 input (exact FP64 sum), |mu_k| <= mu_0
    F32 = Fd.double().cpu().numpy().reshape(n, -1)
    assert np.allclose(mom[:, 0], np.einsum("ni,ni->n", F32, F32), rtol=1e-12)
    assert np.all(np.abs(mom) <= mom[:, :1] * (1 + 1e-4))


def test_batched_spectrum_24_haar():
    L = (24, 24, 24, 24)
    V = api.volume(L)
    announce("24^4 haar: 32 sources, D=256, 64 windows, fp32")
    U = inputs.random_links(L, "haar", seed=3)
    F = inputs.gaussian_fields(L, 32, seed=3)
    Ud = api.pack_links(L, U.to(dev()), torch.float32)
    Fd = F.to(dev()).to(torch.float32)
    mom, pw = api.power_spectrum(L, Ud, Fd, 256, 64)
    F32 = Fd.double().cpu().numpy()
    mu0 = np.einsum("ni,ni->n", F32.reshape(32, -1), F32.reshape(32, -1))
    assert np.allclose(mom[:, 0], mu0, rtol=1e-12)
    # the first moments of two sources in different field groups (0 and 7) against the oracle's
    # recursion on the FP32-rounded inputs
    U32 = U.numpy().astype(np.complex64).astype(np.complex128)
    ref = och.moments(U32, F32[[1, 30]], L, 2)
    assert np.all(np.abs(mom[[1, 30], :3] - ref) <= 1e-5 * ref[:, :1])
    # sanity only (not a check of the higher moments): the windows partition [0, 16], so the powers
    # of any moment sequence sum to mu_0; Jackson-damped windows are non-negative on the true moments
    assert np.allclose(pw.sum(axis=1), mom[:, 0], rtol=1e-11)
    assert pw.min() >= -1e-4 * mom[:, 0].max()
    assert np.all(np.abs(mom) <= mom[:, :1] * (1 + 1e-4))
    # the stencil of this launch at sampled sites
    sites = _sample_sites(V, 48, 3)
    y = api.laplacian_apply(L, Ud, Fd[:2].contiguous()).double().cpu().numpy()
    ref = olap.laplacian_at(U32, F32[:2], L, sites)
    assert np.abs(y[..., sites] - ref).max() <= 1e-5 * np.abs(ref).max()


def test_batched_spectrum_24_free_control():
    """U = 1 control: all 32 sources (every field group of the batched grid) against the exact
    plane-wave moments."""
    L = (24, 24, 24, 24)
    announce("24^4 U=1 control, 32 sources")
    U = inputs.random_links(L, "unit")
    F = inputs.gaussian_fields(L, 32, seed=33)
    Ud = api.pack_links(L, U.to(dev()), torch.float32)
    Fd = F.to(dev()).to(torch.float32)
    mom, pw = api.power_spectrum(L, Ud, Fd, 256, 64)
    ref = och.free_moments_fft(Fd.double().cpu().numpy(), L, 256)
    assert np.all(np.abs(mom - ref) <= 1e-4 * ref[:, :1])
    # FP64 path on the same control: within 1e-12 mu_0
    mom64, _ = api.power_spectrum(L, api.pack_links(L, U.to(dev())), F[:4].to(dev()), 64, 16)
    ref64 = och.free_moments_fft(F[:4].numpy(), L, 64)
    assert np.all(np.abs(mom64 - ref64) <= 1e-12 * ref64[:, :1])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_stencil_32x64_sampled(dtype):
    L = (32, 32, 32, 64)
    V = api.volume(L)
    announce(f"32^3x64 stencil sampled {dtype}")
    U = inputs.random_links(L, "eps", 0.4, seed=5)
    F = inputs.gaussian_fields(L, 1, seed=5)
    Ud = api.pack_links(L, U.to(dev()), dtype)
    api.autotune_laplacian(L, Ud, F.to(dev()).to(dtype), reps=1)
    y = api.laplacian_apply(L, Ud, F.to(dev()).to(dtype)).double().cpu().numpy()
    sites = _sample_sites(V, 64, 5)
    Un = U.numpy()
    Fn = F.numpy()
    if dtype == torch.float32:
        Un = Un.astype(np.complex64).astype(np.complex128)
        Fn = Fn.astype(np.float32).astype(np.float64)
        tol = 1e-5
    else:
        tol = 1e-12
    ref = olap.laplacian_at(Un, Fn, L, sites)
    assert np.abs(y[..., sites] - ref).max() <= tol * np.abs(ref).max()
    api.tune_clear()


def test_gauge_force_32x64_sampled():
    """The Wilson gauge force (beta = 6.4, the bench's workload: eps = 0.4 links, seed 7) at 32^3 x 64
    against the oracle's site-local staples at sampled sites, all four directions and eight
    components (the action is checked against the oracle at the small lattices of the gauge tests)."""
    L = (32, 32, 32, 64)
    V = api.volume(L)
    announce("32^3x64 gauge force sampled")
    U = inputs.random_links(L, "eps", 0.4, seed=7)
    Ud = api.pack_links(L, U.to(dev()))
    F, S = api.wilson_gauge_force(L, Ud, 6.4)
    assert np.isfinite(S)
    sites = _sample_sites(V, 64, 7)
    ref = ogauge.gauge_force_at(U.numpy(), L, 6.4, sites)
    got = F[..., torch.as_tensor(sites, device=dev())].cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("walk", [8, 16])
def test_headline_launch_configurations_32x64(walk):
    """The launch configurations the headline is timed and profiled in (streamed adjoint columns,
    block 256, a walk of 8 or 16 x3 slices, x2 tiles of 2): FP64 at 32^3 x 64 against the oracle at
    sampled sites, and bitwise equal to the one-thread-per-site kernel of the same form."""
    L = (32, 32, 32, 64)
    V = api.volume(L)
    announce(f"32^3x64 headline configuration walk={walk}")
    U = inputs.random_links(L, "eps", 0.4, seed=1)
    F = inputs.gaussian_fields(L, 1, seed=1)
    Ud = api.pack_links(L, U.to(dev()))
    Fd = F.to(dev())
    try:
        api.tune_set(L, torch.float64, 1, form=2, block=256, xcd_remap=0, nv=4, order=0, walk=0, purpose="apply")
        y0 = api.laplacian_apply(L, Ud, Fd)
        api.tune_set(L, torch.float64, 1, form=2, block=256, xcd_remap=0, nv=4, order=0, walk=walk, tile2=2,
                     purpose="apply")
        y = api.laplacian_apply(L, Ud, Fd)
        torch.cuda.synchronize()
        assert torch.equal(y, y0)
        sites = _sample_sites(V, 64, 11)
        ref = olap.laplacian_at(U.numpy(), F.numpy(), L, sites)
        assert np.abs(y.cpu().numpy()[..., sites] - ref).max() <= 1e-12 * np.abs(ref).max()
    finally:
        api.tune_clear()


def test_rational_32x64_mixed_sampled():
    """16-pole kappa = 0.9 rational on one 32^3 x 64 momentum field, mixed precision to 1e-10."""
    L = (32, 32, 32, 64)
    V = api.volume(L)
    announce("32^3x64 16-pole mixed solve")
    U = inputs.random_links(L, "eps", 0.4, seed=5)
    P = inputs.gaussian_fields(L, 1, seed=55)
    Ud = api.pack_links(L, U.to(dev()))
    c, r, s = orat.kappa_poles(0.9, 16)
    out = api.rational_apply(L, Ud, P.to(dev()), api.Rational(c, r, s), api.Solver(tol=1e-10, mode=1),
                             want_poles=True)
    announce(f"  stats {out['stats']}")
    assert out["stats"]["true_relres_max"] <= 1e-10
    xp = out["x_poles"][0]
    sites = _sample_sites(V, 32, 55)
    Pn = P.numpy()
    bnorm = np.linalg.norm(Pn)
    for j in (0, 7, 15):
        xj = xp[j].cpu().numpy()[None]
        res = olap.laplacian_at(U.numpy(), xj, L, sites, s[j]) - Pn[..., sites]
        # every component of a residual is bounded by its norm <= tol ||P||
        assert np.abs(res).max() <= 1e-10 * bnorm
    y = out["y"][0].cpu().numpy()
    ys = c * Pn[0][..., sites] + sum(r[j] * xp[j].cpu().numpy()[..., sites] for j in range(16))
    assert np.allclose(y[..., sites], ys, rtol=0, atol=1e-12 * np.abs(ys).max())
    assert out["K"][0] > 0


def test_kinetic_force_32x64_sampled():
    """Kinetic force of two momentum fields at 32^3 x 64 (16-pole kappa = 0.9 rational, mixed
    precision to 1e-10, section 3 F_M), per field, at sampled links: against the oracle's per-link
    derivative -sum_j r_j d<z_j, Delta x_j>/d omega fed the pole solutions x_j = (Delta + sigma_j)^-1 P
    and z_j = (Delta + sigma_j)^-1 Y, each verified by its FP64 residual at the sampled sites.
    Then the degree-256, 128-window FP32 spectrum of the two forces: mu_0, mu_1 and mu_2 against
    dot products of the FP64 stencil, itself checked at sampled sites."""
    L = (32, 32, 32, 64)
    V = api.volume(L)
    announce("32^3x64 kinetic force, 2 fields, 16 poles, mixed")
    U = inputs.random_links(L, "eps", 0.4, seed=5)
    P = inputs.gaussian_fields(L, 2, seed=57)
    Un = U.numpy()
    Pn = P.numpy()
    Ud = api.pack_links(L, U.to(dev()))
    Pd = P.to(dev())
    c, r, s = orat.kappa_poles(0.9, 16)
    rat = api.Rational(c, r, s)
    sv = api.Solver(tol=1e-10, mode=1)
    out = api.kinetic_force(L, Ud, Pd, rat, sv, per_rhs=True, want_Y=True)
    announce(f"  force stats {out['stats']}")
    assert out["stats"]["true_relres_max"] <= 1e-10
    dK = out["dK"]
    Y = out["Y"]
    torch.cuda.empty_cache()
    sites = _sample_sites(V, 24, 57)
    tab = np.stack([olap_neighbours(L, sites, mu) for mu in range(4)])        # (4, m): x + mu
    idx_all = torch.as_tensor(np.concatenate([sites, tab.ravel()]), device=dev())
    m = len(sites)

    def poles_at(src, field, src_full):
        """Pole solutions at the sampled sites and their neighbours; shifts 0 and 15 of one field
        are checked by their FP64 residual at the sampled sites (which needs the whole field)."""
        res = api.rational_apply(L, Ud, src, rat, sv, want_poles=True, want_K=False)
        assert res["stats"]["true_relres_max"] <= 1e-10
        xp = res["x_poles"]
        g = xp[..., idx_all].cpu().numpy()                                       # (2, 16, 4, 8, 5 m)
        bn = np.linalg.norm(src_full)
        for j in (0, 15):
            full = xp[field, j].cpu().numpy()[None]
            rr = olap.laplacian_at(Un, full, L, sites, s[j]) - src_full[None][..., sites]
            assert np.abs(rr).max() <= 1e-10 * bn, (field, j)
        y = res["y"]
        del res, xp
        torch.cuda.empty_cache()
        return g, y

    xg, yP = poles_at(Pd, 0, Pn[0])
    # the force's own first solve (bitwise when both calls take the same launch shapes; in any case
    # within both solves' tolerance)
    same = bool(torch.equal(yP, Y))
    announce(f"  R(Delta) P of rational_apply and of the force bitwise equal: {same}")
    for i in range(2):
        bound = sum(abs(rj) * 2e-10 * np.linalg.norm(Pn[i]) / sj for rj, sj in zip(r, s))
        assert float(torch.linalg.vector_norm(yP[i] - Y[i])) <= bound
    del yP
    zg, _ = poles_at(Y, 1, Y[1].cpu().numpy())
    dKs = dK[..., idx_all[:m]].cpu().numpy()                                     # (2, 4, 8, m)
    for i in range(2):
        ref = np.zeros((4, 8, m))
        for mu in range(4):
            cols_x = np.arange(m)
            cols_f = m + mu * m + np.arange(m)
            for j in range(16):
                ref[mu] -= r[j] * olap.bilinear_link_derivative_local(
                    Un[mu][sites], zg[i, j][..., cols_x], zg[i, j][..., cols_f], xg[i, j][..., cols_x],
                    xg[i, j][..., cols_f])
        err = np.abs(dKs[i] - ref).max() / np.abs(ref).max()
        announce(f"  field {i}: max |dK - oracle| / max |oracle| at {m} sites x 4 links = {err:.2e}")
        assert err <= 1e-9
    # the 128-window spectrum of the two forces (FP32 sweeps, FP64 moments)
    F32 = dK.to(torch.float32)
    Ud32 = api.pack_links(L, U.to(dev()), torch.float32)
    mom, pw = api.power_spectrum(L, Ud32, F32, 256, 128)
    Fr = F32.double()
    DF = api.laplacian_apply(L, Ud, Fr)                       # FP64 stencil on the FP32-rounded forces
    Fr0 = Fr[:1].cpu().numpy()
    ref = olap.laplacian_at(Un, Fr0, L, sites)
    assert np.abs(DF[:1].cpu().numpy()[..., sites] - ref).max() <= 1e-12 * np.abs(ref).max()
    mu0 = (Fr * Fr).sum(dim=(1, 2, 3)).cpu().numpy()
    t1 = DF / 8.0 - Fr
    mu1 = (Fr * t1).sum(dim=(1, 2, 3)).cpu().numpy()
    mu2 = 2.0 * (t1 * t1).sum(dim=(1, 2, 3)).cpu().numpy() - mu0
    assert np.allclose(mom[:, 0], mu0, rtol=1e-12)
    assert np.all(np.abs(mom[:, 1] - mu1) <= 1e-5 * mu0)
    assert np.all(np.abs(mom[:, 2] - mu2) <= 1e-5 * mu0)
    assert np.allclose(pw.sum(axis=1), mom[:, 0], rtol=1e-11)     # sanity: the windows partition [0, 16]


def olap_neighbours(L, sites, mu):
    """Flat index of x + mu for the given sites (periodic)."""
    sites = np.asarray(sites, np.int64)
    stride = [1, L[0], L[0] * L[1], L[0] * L[1] * L[2]]
    x = (sites // stride[mu]) % L[mu]
    return np.where(x == L[mu] - 1, sites - (L[mu] - 1) * stride[mu], sites + stride[mu])

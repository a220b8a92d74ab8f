"""GPU parity of the Chebyshev moments, power spectra (Eq. 4) and vector filters.

FP64: the library gets its moments from ceil(D/2) sweeps and the doubling identities
mu_2k = 2<t_k,t_k> - mu_0, mu_2k+1 = 2<t_k+1,t_k> - mu_1; the oracle runs the plain
D-step recursion.  Both are exact up to rounding of O(u) * ||t_k||^2 <= O(u) mu_0, so
|mu_gpu - mu_orc| <= 1e-12 mu_0 and the window powers (sum_w |coef| bounded by ~3)
agree to 1e-12 mu_0.  FP32 stencil with FP64 accumulation: the recursion is stable on
[-1, 1], so the error of t_k grows at most linearly in k; at D = 64 the test takes
|mu_gpu - mu_orc| <= 2e-5 mu_0.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import announce, dev, rel_max, setup
from oracle import chebyshev as och
from paper_2112_04556_amd import api, inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,kind,seed,D,nw", [((4, 4, 4, 4), "eps", 1, 64, 16), ((2, 2, 2, 2), "haar", 2, 17, 4),
                                               ((3, 5, 2, 7), "eps", 3, 40, 8), ((4, 6, 2, 8), "unit", 4, 33, 5)])
def test_power_spectrum_fp64(L, kind, seed, D, nw):
    announce(f"power_spectrum fp64 {L} D={D}")
    eps = 0.3 if L == (4, 4, 4, 4) else 0.5
    U, F, Ud, Fd = setup(L, kind, eps, seed, n=2)
    mom, pw = api.power_spectrum(L, Ud, Fd, D, nw)
    mref, pref = och.power_spectrum(U, F, L, D, och.equal_windows(nw))
    mu0 = mref[:, :1]
    assert np.all(np.abs(mom - mref) <= 1e-12 * mu0)
    assert np.all(np.abs(pw - pref) <= 1e-12 * mu0)
    # partition of unity: the windows add up to <F, F> at any U
    assert np.allclose(pw.sum(axis=1), mom[:, 0], rtol=1e-12)


def test_power_spectrum_fp32():
    L = (4, 4, 4, 4)
    announce("power_spectrum fp32")
    U, F, Ud, Fd = setup(L, "eps", 0.3, 1, n=1, dtype=torch.float32)
    mom, pw = api.power_spectrum(L, Ud, Fd, 64, 16)
    # the oracle on the same FP32-rounded inputs isolates the recursion error
    U32 = U.astype(np.complex64).astype(np.complex128)
    F32 = F.astype(np.float32).astype(np.float64)
    mref, pref = och.power_spectrum(U32, F32, L, 64, och.equal_windows(16))
    assert np.all(np.abs(mom - mref) <= 2e-5 * mref[:, :1])
    assert np.all(np.abs(pw - pref) <= 2e-5 * mref[:, :1])


def test_power_ratio_free_field():
    """At U = 1 on an anisotropic lattice, the Gaussian-source power per mode averages to 1."""
    L = (8, 4, 6, 4)
    announce("power ratio free field")
    _, F, Ud, Fd = setup(L, "unit", 0.0, 5, n=8)
    D, nw = 32, 4
    mom, pw = api.power_spectrum(L, Ud, Fd, D, nw)
    tau = api.trace_moments_free(L, D)
    ratio = api.power_ratio(D, nw, tau, pw)
    # moments at U = 1 are exact through the FFT (pinned oracle function) for every source
    for i in range(2):
        mref = och.moments(inputs.random_links(L, "unit").numpy(), F[i:i + 1], L, D)
        assert np.all(np.abs(mom[i] - mref[0]) <= 1e-12 * mref[0, 0])
    assert abs(ratio.mean() - 1.0) < 0.1


# degrees around the fold ring of 16 recursion vectors: one short ring (D < 3), exactly one
# ring, one ring and a partial one, two rings and a one-vector remainder
@pytest.mark.parametrize("dtype,D", [(torch.float64, 1), (torch.float64, 2), (torch.float64, 16),
                                     (torch.float64, 24), (torch.float64, 33), (torch.float32, 24)])
def test_cheb_filter(dtype, D):
    L = (3, 5, 2, 7)
    announce(f"cheb_filter {dtype} D={D}")
    U, x, Ud, xd = setup(L, "eps", 0.5, 6, n=2, dtype=dtype)
    nw = 5
    edges = np.array([0.0, 2.0, 5.0, 9.5, 12.0, 16.0])
    y = api.cheb_filter(L, Ud, xd, D, nw, edges).cpu().numpy().astype(np.float64)
    if dtype == torch.float64:
        ref = och.cheb_filter(U, x, L, D, edges)
        assert rel_max(y, ref) <= 1e-12
        assert np.allclose(y.sum(axis=0), x, atol=1e-12)
    else:
        U32 = U.astype(np.complex64).astype(np.complex128)
        x32 = x.astype(np.float32).astype(np.float64)
        ref = och.cheb_filter(U32, x32, L, D, edges)
        assert np.abs(y - ref).max() <= 2e-5 * np.abs(x32).max()


def test_power_spectrum_deterministic_and_batched():
    L = (4, 4, 6, 2)
    _, F, Ud, Fd = setup(L, "haar", 0.0, 8, n=3)
    m1, p1 = api.power_spectrum(L, Ud, Fd, 20, 4)
    m2, p2 = api.power_spectrum(L, Ud, Fd, 20, 4)
    assert np.array_equal(m1, m2) and np.array_equal(p1, p2)
    m3, _ = api.power_spectrum(L, Ud, Fd[1:2].contiguous(), 20, 4)
    assert np.array_equal(m3[0], m1[1])

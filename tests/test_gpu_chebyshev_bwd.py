"""GPU parity of the backward Chebyshev calls (link derivative of Eq. 4's power and of the
bandpass filters) against the oracle's dense spectral derivative, and properties that hold at any
size: the filter's adjoint identity, grad_F = 2 sum_w gamma_w B_w F, and central finite
differences of the GPU's own forward calls."""
import numpy as np
import pytest
import torch
from scipy.linalg import expm

from gpu_helpers import announce, dev, rel_max, setup
from oracle import chebyshev as och
from oracle import chebyshev_grad as ocg
from oracle import su3
from paper_2112_04556_amd import api

pytestmark = pytest.mark.gpu

# 72 sites: two 64-site blocks, the second ragged, under the (block 64, 4 directions) shape
L_PAR = (4, 3, 2, 3)


def _perturb(Ud, L, mu, s, c, eps):
    Ua = api.unpack_links(L, Ud).cpu().numpy()
    Ua[mu, s] = expm(1j * eps * su3.T[c]) @ Ua[mu, s]
    return api.pack_links(L, torch.from_numpy(Ua).to(dev()))


@pytest.mark.parametrize("kind", ["eps", "unit"])
@pytest.mark.parametrize("shape", ["default", "block64"])
def test_power_spectrum_bwd_parity(kind, shape):
    L = L_PAR
    announce(f"power_spectrum_bwd parity {kind} {shape}")
    U, F, Ud, Fd = setup(L, kind, 0.7, 41, n=2)
    D, nw = 14, 4
    edges = och.equal_windows(nw)
    gamma = np.random.default_rng(41).normal(size=(2, nw))
    if shape == "block64":
        api.tune_set(L, torch.float64, 2, 0, 64, 0, 4, 0, 0)
    try:
        gF, go = api.power_spectrum_bwd(L, Ud, Fd, gamma, D, nw)
        _, gop = api.power_spectrum_bwd(L, Ud, Fd, gamma, D, nw, grad_F=False, per_rhs=True)
    finally:
        api.tune_clear()
    ref_op = ocg.power_spectrum_link_derivative(U, F, L, D, edges, gamma, per_rhs=True)
    ref_o = ref_op.sum(axis=0)
    ref_F = ocg.power_spectrum_source_gradient(U, F, L, D, edges, gamma)
    assert rel_max(go[0].cpu().numpy(), ref_o) <= 1e-12
    assert rel_max(gop.cpu().numpy(), ref_op) <= 1e-12
    assert rel_max(gF.cpu().numpy(), ref_F) <= 1e-12


@pytest.mark.parametrize("D", [2, 3, 4, 5])
def test_bwd_low_degrees(D):
    """Degrees 2-5, where the reverse sweep's first steps take each of its forms (the adjoint step
    alone, the recomputed forward step alone, both in one launch): power-spectrum and filter
    derivatives against the oracle."""
    L = L_PAR
    announce(f"chebyshev bwd degree {D}")
    U, F, Ud, Fd = setup(L, "eps", 0.6, 45 + D, n=2)
    nw = 3
    edges = och.equal_windows(nw)
    gamma = np.random.default_rng(D).normal(size=(2, nw))
    gF, go = api.power_spectrum_bwd(L, Ud, Fd, gamma, D, nw)
    assert rel_max(go[0].cpu().numpy(), ocg.power_spectrum_link_derivative(U, F, L, D, edges, gamma)) <= 1e-12
    assert rel_max(gF.cpu().numpy(), ocg.power_spectrum_source_gradient(U, F, L, D, edges, gamma)) <= 1e-12
    gy = np.random.default_rng(100 + D).normal(size=(nw,) + F.shape)
    gx, gop = api.cheb_filter_bwd(L, Ud, Fd, torch.from_numpy(gy).to(dev()), D, nw, edges, per_rhs=True)
    rgx, rgop = ocg.cheb_filter_vjp(U, F, gy, L, D, edges, per_rhs=True)
    assert rel_max(gx.cpu().numpy(), rgx) <= 1e-12
    assert rel_max(gop.cpu().numpy(), rgop) <= 1e-12


def test_cheb_filter_bwd_parity():
    L = L_PAR
    announce("cheb_filter_bwd parity")
    U, x, Ud, xd = setup(L, "haar", 0.0, 42, n=2)
    D = 11
    edges = np.array([0.0, 2.5, 6.0, 11.0, 16.0])
    nw = 4
    gy = np.random.default_rng(42).normal(size=(nw,) + x.shape)
    gx, go = api.cheb_filter_bwd(L, Ud, xd, torch.from_numpy(gy).to(dev()), D, nw, edges)
    _, gop = api.cheb_filter_bwd(L, Ud, xd, torch.from_numpy(gy).to(dev()), D, nw, edges, grad_x=False,
                                 per_rhs=True)
    rgx, rgop = ocg.cheb_filter_vjp(U, x, gy, L, D, edges, per_rhs=True)
    rgo = rgop.sum(axis=0)
    assert rel_max(gx.cpu().numpy(), rgx) <= 1e-12
    assert rel_max(go[0].cpu().numpy(), rgo) <= 1e-12
    assert rel_max(gop.cpu().numpy(), rgop) <= 1e-12


def test_degree_one_and_errors():
    L = (2, 2, 2, 2)
    U, F, Ud, Fd = setup(L, "eps", 0.5, 43, n=1)
    gamma = np.array([[1.0, -0.5]])
    gF, go = api.power_spectrum_bwd(L, Ud, Fd, gamma, 1, 2)
    edges = och.equal_windows(2)
    assert rel_max(go[0].cpu().numpy(), ocg.power_spectrum_link_derivative(U, F, L, 1, edges, gamma)) <= 1e-12
    assert rel_max(gF.cpu().numpy(), ocg.power_spectrum_source_gradient(U, F, L, 1, edges, gamma)) <= 1e-12
    with pytest.raises(TypeError):
        api.power_spectrum_bwd(L, Ud, Fd.float(), gamma, 4, 2)
    from paper_2112_04556_amd._lib import RmhError
    with pytest.raises(RmhError):
        api.power_spectrum_bwd(L, Ud, Fd, gamma, 4, 2, grad_F=False, grad_omega=False)


def test_filter_adjoint_and_source_gradient_8():
    """At 8^4, Haar links: <gy, B x> = <grad_x, x> and grad_F = 2 sum_w gamma_w B_w F, each side
    from a different GPU call."""
    L = (8, 8, 8, 8)
    announce("cheb bwd identities 8^4")
    _, x, Ud, xd = setup(L, "haar", 0.0, 44, n=2)
    D, nw = 40, 8
    gy = torch.randn((nw,) + tuple(xd.shape), dtype=torch.float64, device=dev(),
                     generator=torch.Generator(device=dev()).manual_seed(44))
    gx, _ = api.cheb_filter_bwd(L, Ud, xd, gy, D, nw, grad_omega=False)
    y = api.cheb_filter(L, Ud, xd, D, nw)
    lhs = float(torch.sum(gy * y))
    rhs = float(torch.sum(gx * xd))
    assert abs(lhs - rhs) <= 1e-12 * float(torch.sqrt(torch.sum(gy * gy) * torch.sum(xd * xd)))
    gamma = np.random.default_rng(44).normal(size=(2, nw))
    gF, _ = api.power_spectrum_bwd(L, Ud, xd, gamma, D, nw, grad_omega=False)
    ref = 2 * torch.einsum("w,wvabs->vabs", torch.from_numpy(gamma[0]).to(dev()), y[:, :1].contiguous())
    assert rel_max(gF[:1].cpu().numpy(), ref.cpu().numpy()) <= 1e-12


@pytest.mark.parametrize("L,D,nw,n_pert,rtol", [((8, 8, 8, 8), 24, 6, 16, 1e-6), ((16, 16, 16, 16), 64, 16, 32, 1e-4)])
def test_power_spectrum_bwd_finite_differences(L, D, nw, n_pert, rtol):
    """Central differences (h = 1e-4) of sum gamma * power from the GPU's forward call, against the
    backward call's link derivative.  Truncation O(h^2) ~ 1e-8 relative; rounding of the forward
    powers ~ 1e-15 * 32 V / h."""
    announce(f"power_spectrum_bwd FD {L}")
    _, F, Ud, Fd = setup(L, "eps", 0.5, 45, n=1)
    gamma = np.random.default_rng(45).normal(size=(1, nw))
    _, go = api.power_spectrum_bwd(L, Ud, Fd, gamma, D, nw, grad_F=False)
    go = go[0].cpu().numpy()
    scale = np.abs(go).max()
    rng = np.random.default_rng(46)
    h = 1e-4
    worst = 0.0
    for _ in range(n_pert):
        mu, c, s = int(rng.integers(4)), int(rng.integers(8)), int(rng.integers(api.volume(L)))
        pp = api.power_spectrum(L, _perturb(Ud, L, mu, s, c, h), Fd, D, nw)[1]
        pm = api.power_spectrum(L, _perturb(Ud, L, mu, s, c, -h), Fd, D, nw)[1]
        fd = float(np.sum(gamma * (pp - pm))) / (2 * h)
        worst = max(worst, abs(fd - go[mu, c, s]) / scale)
    announce(f"  FD worst relative deviation {worst:.3e}")
    assert worst <= rtol


def test_autograd_power_spectrum():
    """torch.autograd through the library's forward and backward: gradients for omega and F against
    the oracle's dense derivative."""
    from paper_2112_04556_amd import autograd
    L = (2, 3, 2, 2)
    U, F, Ud, Fd = setup(L, "eps", 0.6, 47, n=2)
    D, nw = 10, 3
    gamma = np.random.default_rng(47).normal(size=(2, nw))
    omega = torch.zeros((4, 8, api.volume(L)), dtype=torch.float64, device=dev(), requires_grad=True)
    Fg = Fd.clone().requires_grad_(True)
    pw = autograd.power_spectrum(omega, Fg, Ud, L, D, nw)
    loss = torch.sum(pw * torch.from_numpy(gamma).to(dev()))
    loss.backward()
    edges = och.equal_windows(nw)
    assert rel_max(omega.grad.cpu().numpy(), ocg.power_spectrum_link_derivative(U, F, L, D, edges, gamma)) <= 1e-12
    assert rel_max(Fg.grad.cpu().numpy(), ocg.power_spectrum_source_gradient(U, F, L, D, edges, gamma)) <= 1e-12


def test_gradcheck_power_spectrum_displaced_links():
    """torch.autograd.gradcheck of a weighted sum of window powers at a non-zero link displacement
    (2^4, degree 8, 3 windows, FP64): the omega and F gradients against central differences."""
    from paper_2112_04556_amd import autograd
    L = (2, 2, 2, 2)
    U, F, Ud, Fd = setup(L, "eps", 0.6, 49, n=1)
    rng = np.random.default_rng(49)
    gamma = torch.tensor(rng.normal(size=(1, 3)), device=dev())
    omega = torch.tensor(0.3 * rng.normal(size=(4, 8, api.volume(L))), dtype=torch.float64, device=dev(),
                         requires_grad=True)
    Fg = Fd.clone().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda w, f: torch.sum(autograd.power_spectrum(w, f, Ud, L, 8, 3) * gamma),
                                    (omega, Fg), eps=1e-6, atol=1e-7, rtol=1e-6)

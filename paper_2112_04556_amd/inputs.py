"""Seeded synthetic inputs for the adjoint-Laplacian hot path.

This module only draws random numbers and builds group elements from them; it
holds none of the method's arithmetic (no Laplacian, no Chebyshev recursion, no
solver, no force).  Both the CPU oracle (through the tests) and the HIP path
(through the tests and the benchmark) take their inputs from here, so neither
side ever generates its own.

Layouts (shared with the C ABI, site index s = x0 + L0*(x1 + L1*(x2 + L2*x3)),
so x0 runs fastest):

* links  : complex128, shape (4, V, 3, 3); U[mu, s] is U_mu(x), an SU(3) matrix.
* fields : float64, shape (n, 4, 8, V); component a (Gell-Mann index a+1) of the
           su(3) element P_nu(x) = sum_a P^a T^a with T^a = lambda^a / 2.

Link ensembles (the paper's gauge ensembles are not available, these stand in
for them at the paper's lattice shapes):

* ``"eps"``  : U = exp(i*eps*H), H = sum_a h^a T^a with h^a ~ N(0,1), then
               re-unitarised (rows 0, 1 by Gram-Schmidt, row 2 = conj(row0 x row1)).
* ``"haar"`` : Haar-random SU(3) (Gram-Schmidt on complex Gaussian rows, third
               row completed by the conjugate cross product so det U = 1).
* ``"unit"`` : U = 1, the free-field control.

Random streams are keyed by (seed, stream) so links, fields and gauge
transformations never share draws.
"""
from __future__ import annotations

import math

import torch

__all__ = [
    "volume", "make_generator", "gell_mann_half", "random_links", "gaussian_fields",
    "haar_su3", "reunitarize", "gauge_transform",
]

STREAM_LINKS = 0
STREAM_FIELDS = 1
STREAM_GAUGE = 99


def volume(L) -> int:
    """Number of sites of a periodic L0 x L1 x L2 x L3 lattice."""
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def make_generator(seed: int, stream: int) -> torch.Generator:
    """A CPU torch generator keyed by (seed, stream)."""
    g = torch.Generator(device="cpu")
    g.manual_seed((int(seed) * 1_000_003 + int(stream) * 7919 + 12345) % (2**63 - 1))
    return g


def gell_mann_half(dtype=torch.complex128) -> torch.Tensor:
    """The eight matrices lambda^a / 2, shape (8, 3, 3); used only to build H."""
    lam = torch.zeros(8, 3, 3, dtype=dtype)
    lam[0, 0, 1] = lam[0, 1, 0] = 1
    lam[1, 0, 1] = -1j
    lam[1, 1, 0] = 1j
    lam[2, 0, 0] = 1
    lam[2, 1, 1] = -1
    lam[3, 0, 2] = lam[3, 2, 0] = 1
    lam[4, 0, 2] = -1j
    lam[4, 2, 0] = 1j
    lam[5, 1, 2] = lam[5, 2, 1] = 1
    lam[6, 1, 2] = -1j
    lam[6, 2, 1] = 1j
    s3 = 1.0 / math.sqrt(3.0)
    lam[7, 0, 0] = s3
    lam[7, 1, 1] = s3
    lam[7, 2, 2] = -2 * s3
    return lam / 2


def reunitarize(U: torch.Tensor) -> torch.Tensor:
    """Project onto SU(3): Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1)."""
    r0 = U[..., 0, :]
    r0 = r0 / torch.linalg.vector_norm(r0, dim=-1, keepdim=True)
    r1 = U[..., 1, :]
    r1 = r1 - (r0.conj() * r1).sum(-1, keepdim=True) * r0
    r1 = r1 / torch.linalg.vector_norm(r1, dim=-1, keepdim=True)
    r2 = torch.linalg.cross(r0, r1, dim=-1).conj()
    return torch.stack([r0, r1, r2], dim=-2)


def haar_su3(shape, gen: torch.Generator) -> torch.Tensor:
    """Haar-random SU(3) matrices of the given batch shape (complex128)."""
    re = torch.randn(*shape, 3, 3, generator=gen, dtype=torch.float64)
    im = torch.randn(*shape, 3, 3, generator=gen, dtype=torch.float64)
    return reunitarize(torch.complex(re, im))


def random_links(L, kind: str = "eps", eps: float = 0.3, seed: int = 1) -> torch.Tensor:
    """Gauge links, complex128 of shape (4, V, 3, 3), on the CPU."""
    V = volume(L)
    gen = make_generator(seed, STREAM_LINKS)
    if kind == "unit":
        return torch.eye(3, dtype=torch.complex128).expand(4, V, 3, 3).clone()
    if kind == "haar":
        return haar_su3((4, V), gen)
    if kind != "eps":
        raise ValueError(f"unknown link kind {kind!r}")
    h = torch.randn(4, V, 8, generator=gen, dtype=torch.float64)
    T = gell_mann_half()
    out = torch.empty(4, V, 3, 3, dtype=torch.complex128)
    chunk = 1 << 18
    for mu in range(4):
        for s0 in range(0, V, chunk):
            hh = h[mu, s0:s0 + chunk].to(torch.complex128)
            H = torch.einsum("na,aij->nij", hh, T)
            out[mu, s0:s0 + chunk] = reunitarize(torch.linalg.matrix_exp(1j * eps * H))
    return out


def gaussian_fields(L, n: int = 1, seed: int = 1, stream: int = STREAM_FIELDS) -> torch.Tensor:
    """n Gaussian su(3) link fields, float64 of shape (n, 4, 8, V), P^a ~ N(0,1)."""
    gen = make_generator(seed, stream)
    return torch.randn(n, 4, 8, volume(L), generator=gen, dtype=torch.float64)


def gauge_transform(L, seed: int = 1) -> torch.Tensor:
    """A Haar-random gauge transformation Omega(x), complex128 of shape (V, 3, 3)."""
    return haar_su3((volume(L),), make_generator(seed, STREAM_GAUGE))

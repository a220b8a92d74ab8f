"""The power spectrum entry point that allocates nothing (rmh_power_spectrum_noalloc) against the
workspace entry point (rmh_power_spectrum), called through the C ABI: two calls in a row, the second
with a smaller input, each bitwise equal to the workspace call on the same input (the same kernels
in the same order), and both against the oracle within the FP64 bound of the power-spectrum tests."""
import numpy as np
import pytest
import torch

from gpu_helpers import announce, dev, setup
from oracle import chebyshev as och
from paper_2112_04556_amd import api
from paper_2112_04556_amd._lib import RmhError

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_power_spectrum_noalloc_matches_workspace_call(dtype):
    cases = [((16, 16, 16, 16), 1, 64, 16), ((4, 4, 4, 6), 3, 48, 8)]   # second call: smaller input
    if dtype == torch.float32:
        cases[0] = ((16, 16, 16, 16), 2, 64, 16)
    for L, n, D, nw in cases:
        announce(f"noalloc power spectrum L={L} n={n} D={D} {dtype}")
        U, F, Ud, Fd = setup(L, "eps", 0.4, 7, n=n, dtype=dtype)
        mom_s, pw_s = api.power_spectrum_noalloc(L, Ud, Fd, D, nw)
        mom_w, pw_w = api.power_spectrum(L, Ud, Fd, D, nw)
        assert np.array_equal(mom_s, mom_w) and np.array_equal(pw_s, pw_w)
        if dtype == torch.float64 and L[0] == 4:
            mref, pref = och.power_spectrum(U, F, L, D, och.equal_windows(nw))
            assert np.all(np.abs(mom_s - mref) <= 1e-12 * mref[:, :1])
            assert np.all(np.abs(pw_s - pref) <= 1e-12 * mref[:, :1])


def test_power_spectrum_noalloc_rejects_oversize():
    L = (16, 16, 16, 16)
    U, F, Ud, Fd = setup(L, "eps", 0.4, 7, n=2)
    with pytest.raises(RmhError, match="static scratch"):
        api.power_spectrum_noalloc(L, Ud, Fd, 64, 16)

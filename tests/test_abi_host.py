"""CPU tests of the C ABI: every declared symbol is exported, the host-side FP64 helpers
agree with the oracle, and argument validation rejects bad calls before any GPU work."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

from oracle import chebyshev as och
from oracle import rational as ora
from paper_2112_04556_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmh.h")

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="librmh.so not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rmh_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 20
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_version_and_error_string():
    L = _lib.lib()
    assert L.rmh_version() == 101
    assert isinstance(L.rmh_last_error(), bytes)


@pytest.mark.parametrize("D,nw,kernel", [(64, 16, 1), (256, 64, 1), (31, 5, 0)])
def test_cheb_coefficients_match_oracle(D, nw, kernel):
    from paper_2112_04556_amd import api
    got = api.cheb_coefficients(D, nw, None, kernel)
    ref = och.window_coefficients(och.equal_windows(nw), D, "jackson" if kernel else "none")
    assert np.allclose(got, ref, rtol=0, atol=1e-14)
    edges = np.array([0.0, 0.5, 3.0, 7.5, 16.0])
    got = api.cheb_coefficients(20, 4, edges, kernel)
    assert np.allclose(got, och.window_coefficients(edges, 20, "jackson" if kernel else "none"), atol=1e-14)


def test_cheb_coefficients_reject_bad_edges():
    from paper_2112_04556_amd import api
    with pytest.raises(_lib.RmhError) as e:
        api.cheb_coefficients(8, 2, np.array([0.0, 9.0, 4.0]))
    assert e.value.status == 1


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 6, 2, 8)])
def test_trace_moments_free_match_oracle(L):
    from paper_2112_04556_amd import api
    assert np.allclose(api.trace_moments_free(L, 40), och.trace_moments_free(L, 40), rtol=1e-12, atol=1e-9)


def test_power_ratio_host():
    from paper_2112_04556_amd import api
    L = (2, 2, 2, 2)
    tau = och.trace_moments_free(L, 16)
    power = np.random.default_rng(0).random((3, 4))
    got = api.power_ratio(16, 4, tau, power)
    den = och.window_coefficients(och.equal_windows(4), 16) @ tau
    assert np.allclose(got, power / den[None, :], rtol=1e-13)


def test_rational_kappa_matches_oracle():
    from paper_2112_04556_amd import api
    for kappa, n in [(0.9, 12), (0.5, 12), (0.9, 8), (0.3, 3)]:
        rat = api.rational_kappa(kappa, n)
        c, r, s = ora.kappa_poles(kappa, n)
        assert rat.c == c
        assert np.allclose(rat.r, r, rtol=1e-14) and np.allclose(rat.sigma, s, rtol=1e-14)


def test_rational_from_quadratics_matches_oracle():
    from paper_2112_04556_amd import api
    a0, a1, b0, b1 = [0.3, -0.2], [1.1, 0.5], [0.02, 0.5], [0.5, 1.6]
    r, s = api.rational_from_quadratics(a0, a1, b0, b1)
    _, rr, ss = ora.poles_from_quadratics(0.0, a0, a1, b0, b1)
    assert np.allclose(r, rr, rtol=1e-13) and np.allclose(s, ss, rtol=1e-13)
    with pytest.raises(_lib.RmhError) as e:
        api.rational_from_quadratics([1.0], [0.0], [1.0], [0.5])
    assert e.value.status == 4


# ---- validation paths (fake, never dereferenced device addresses) ------------------------

FAKE = 0x7F0000000000  # 256-byte aligned, never touched: every call below fails validation first


def _lap(L, U, x, y, n=1, dtype=0, shift=0.0):
    return _lib.lib().rmh_laplacian_apply(_lib.lattice_arg(L), U, dtype, x, y, n, shift, None)


def test_validation_shape_and_alignment():
    V = 16
    fb = 32 * V * 8
    assert _lap((1, 2, 2, 2), FAKE, FAKE + 10 * fb, FAKE + 20 * fb) == 2          # RMH_E_SHAPE
    assert _lap((2, 2, 2, 2), FAKE + 8, FAKE + 10 * fb, FAKE + 20 * fb) == 1      # misaligned U
    assert _lap((2, 2, 2, 2), FAKE, FAKE + 10 * fb, FAKE + 10 * fb) == 1          # y aliases x
    assert _lap((2, 2, 2, 2), FAKE, FAKE + 10 * fb, FAKE + 10 * fb + 256) == 1    # y overlaps x
    assert _lap((2, 2, 2, 2), FAKE, FAKE + 10 * fb, FAKE + 20 * fb, dtype=7) == 1
    assert _lap((2, 2, 2, 2), FAKE, FAKE + 10 * fb, FAKE + 20 * fb, n=-1) == 1
    assert _lap((2, 2, 2, 2), FAKE, FAKE + 10 * fb, FAKE + 20 * fb, shift=float("nan")) == 1
    assert _lap((2, 2, 2, 2), FAKE, FAKE + 10 * fb, FAKE + 20 * fb, n=0) == 0     # empty batch: no-op


def test_validation_rational():
    L = _lib.lattice_arg((2, 2, 2, 2))
    r = np.array([1.0, 2.0])
    s_bad = np.array([0.5, -1.0])
    rat = _lib.RmhRational(0.0, 2, r.ctypes.data_as(_lib.P_f64), s_bad.ctypes.data_as(_lib.P_f64))
    sv = _lib.RmhSolver(1e-10, 100, 0, 0.1, 8, 0.0, 0)
    st = _lib.lib().rmh_rational_apply(L, FAKE, FAKE + 2**20, 1, ctypes.byref(rat), ctypes.byref(sv), FAKE + 2**21,
                                       None, None, None, FAKE + 2**22, 1 << 30, None)
    assert st == 4                                                                # RMH_E_POLES
    s_ok = np.array([0.5, 1.0])
    rat = _lib.RmhRational(0.0, 2, r.ctypes.data_as(_lib.P_f64), s_ok.ctypes.data_as(_lib.P_f64))
    sv_bad = _lib.RmhSolver(0.0, 100, 0, 0.1, 8, 0.0, 0)
    st = _lib.lib().rmh_rational_apply(L, FAKE, FAKE + 2**20, 1, ctypes.byref(rat), ctypes.byref(sv_bad),
                                       FAKE + 2**21, None, None, None, FAKE + 2**22, 1 << 30, None)
    assert st == 1
    # multi-shift target outside [0, 1e6], or its product with tol not below 1
    for mt, tol in ((-1.0, 1e-10), (2e6, 1e-10), (2.0, 0.5), (float("nan"), 1e-10)):
        sv_mt = _lib.RmhSolver(tol, 100, 0, 0.1, 8, 0.0, 0, mt)
        st = _lib.lib().rmh_rational_apply(L, FAKE, FAKE + 2**20, 1, ctypes.byref(rat), ctypes.byref(sv_mt),
                                           FAKE + 2**21, None, None, None, FAKE + 2**22, 1 << 30, None)
        assert st == 1, (mt, tol)
    # pole count outside [1, 64]
    r65, s65 = np.ones(65), np.linspace(0.5, 10.0, 65)
    for n in (0, 65):
        rat_n = _lib.RmhRational(0.0, n, r65.ctypes.data_as(_lib.P_f64), s65.ctypes.data_as(_lib.P_f64))
        st = _lib.lib().rmh_rational_apply(L, FAKE, FAKE + 2**20, 1, ctypes.byref(rat_n), ctypes.byref(sv),
                                           FAKE + 2**21, None, None, None, FAKE + 2**22, 1 << 30, None)
        assert st == 1, n                                                         # RMH_E_ARG
    # workspace too small
    st = _lib.lib().rmh_rational_apply(L, FAKE, FAKE + 2**20, 1, ctypes.byref(rat), ctypes.byref(sv),
                                       FAKE + 2**21, None, None, None, FAKE + 2**22, 1024, None)
    assert st == 3                                                                # RMH_E_WORKSPACE


def test_workspace_query():
    L = _lib.lattice_arg((4, 4, 4, 4))
    n1 = _lib.lib().rmh_workspace_bytes(4, L, 0, 1, 12, 0, 0)
    n2 = _lib.lib().rmh_workspace_bytes(4, L, 0, 2, 12, 0, 0)
    m1 = _lib.lib().rmh_workspace_bytes(4, L, 0, 1, 12, 0, 1)
    assert 0 < n1 < n2 and m1 > 0
    assert _lib.lib().rmh_workspace_bytes(99, L, 0, 1, 1, 0, 0) == 0
    # Chebyshev backward: four link fields per source plus the coefficients
    fb = 32 * 256 * 8
    b7 = _lib.lib().rmh_workspace_bytes(7, L, 0, 2, 3, 10, 0)
    b8 = _lib.lib().rmh_workspace_bytes(8, L, 0, 2, 3, 10, 0)
    assert 4 * 2 * fb <= b8 <= b7 < 4 * 2 * fb + 4096


def test_heatbath_validation():
    L = _lib.lattice_arg((2, 2, 2, 2))
    r = np.array([1.0, 2.0])
    sg = np.array([0.5, 1.0])
    rat = _lib.RmhRational(0.0, 2, r.ctypes.data_as(_lib.P_f64), sg.ctypes.data_as(_lib.P_f64))
    sv = _lib.RmhSolver(1e-10, 100, 0, 0.1, 8, 0.0, 0)
    f = _lib.lib().rmh_heatbath_momenta
    for kappa in (-0.1, 1.5, float("nan")):
        assert f(L, FAKE, FAKE + 2**20, 1, kappa, ctypes.byref(rat), ctypes.byref(sv), FAKE + 2**21, None,
                 FAKE + 2**22, 1 << 30, None) == 1
    # kappa = 0 (the exact inverse) takes the partial fractions of 1/R, which this library forms for
    # positive residues only
    rn = np.array([1.0, -0.9])
    bad = _lib.RmhRational(0.0, 2, rn.ctypes.data_as(_lib.P_f64), sg.ctypes.data_as(_lib.P_f64))
    assert f(L, FAKE, FAKE + 2**20, 1, 0.0, ctypes.byref(bad), ctypes.byref(sv), FAKE + 2**21, None,
             FAKE + 2**22, 1 << 30, None) == 4
    assert f(L, FAKE, FAKE + 2**20, 0, 0.0, ctypes.byref(rat), ctypes.byref(sv), None, None, None, 0, None) == 0
    assert f(L, FAKE, FAKE + 2**20, 1, 0.5, ctypes.byref(rat), ctypes.byref(sv), FAKE + 2**21, None,
             FAKE + 2**22, 1024, None) == 3                                   # workspace too small
    assert f(L, FAKE, FAKE + 2**20, 1, 0.5, ctypes.byref(rat), ctypes.byref(sv), FAKE + 2**20, None,
             FAKE + 2**22, 1 << 30, None) == 1                                # P aliases xi


def test_gauge_force_workspace_and_validation():
    L = _lib.lattice_arg((4, 4, 4, 4))
    assert _lib.lib().rmh_workspace_bytes(9, L, 0, 1, 0, 0, 0) == 512      # block partials + the sum
    # the autotuner's dot-product partials: 3 rows per field of the largest block count
    a1 = _lib.lib().rmh_workspace_bytes(_lib.OP_AUTOTUNE, L, 0, 1, 0, 0, 0)
    a4 = _lib.lib().rmh_workspace_bytes(_lib.OP_AUTOTUNE, L, 0, 4, 0, 0, 0)
    assert a1 > 0 and a4 >= 4 * a1 - 256
    S = np.zeros(1)
    f = _lib.lib().rmh_wilson_gauge_force
    assert f(L, FAKE, 6.0, None, None, None, 0, None) == 1                  # nothing requested
    assert f(L, FAKE, float("nan"), FAKE + 2**20, None, None, 0, None) == 1
    assert f(L, FAKE, 6.0, FAKE + 2**20, S.ctypes.data_as(_lib.P_f64), FAKE + 2**22, 256, None) == 3
    assert f(L, FAKE, 6.0, FAKE + 4096, None, None, 0, None) == 1           # F overlaps U


def test_validation_cheb_bwd():
    L = _lib.lattice_arg((4, 4, 4, 4))
    fb = 32 * 256 * 8
    st = _lib.RmhCheb(10, 3, None, 1)
    bad = _lib.RmhCheb(0, 3, None, 1)
    gam = np.ones(3)
    args = lambda cheb, gx, go, wsb: (L, FAKE, FAKE + 2**20, FAKE + 2**21, 1, ctypes.byref(cheb), gx, go, 0,
                                      FAKE + 2**22, wsb, None)
    f = _lib.lib().rmh_cheb_filter_bwd
    assert f(*args(bad, FAKE + 2**23, None, 1 << 30)) == 1                 # degree 0
    assert f(*args(st, None, None, 1 << 30)) == 1                           # nothing requested
    assert f(*args(st, FAKE + 2**23, None, 1024)) == 3                      # workspace too small
    assert f(*args(st, FAKE + 2**20, None, 1 << 30)) == 1                   # grad_x aliases x
    g = _lib.lib().rmh_power_spectrum_bwd
    gp = gam.ctypes.data_as(_lib.P_f64)
    assert g(L, FAKE, FAKE + 2**20, 1, ctypes.byref(st), None, FAKE + 2**23, None, 0, FAKE + 2**22, 1 << 30,
             None) == 1                                                       # gamma NULL
    assert g(L, FAKE, FAKE + 2**20, 1, ctypes.byref(st), gp, FAKE + 2**20 + fb // 2, None, 0, FAKE + 2**22,
             1 << 30, None) == 1                                              # grad_F overlaps F
    nan = np.array([1.0, np.nan, 0.0])
    assert g(L, FAKE, FAKE + 2**20, 1, ctypes.byref(st), nan.ctypes.data_as(_lib.P_f64), FAKE + 2**23, None, 0,
             FAKE + 2**22, 1 << 30, None) == 1                                # non-finite gamma


def test_tune_set_validation():
    """The launch cache is host state: every accepted and rejected configuration, no GPU."""
    f = _lib.lib().rmh_tune_set
    L = _lib.lattice_arg((4, 4, 4, 4))

    def put(cfg, dtype=0, n=1, purpose=-1):
        full = tuple(cfg) + (1,) * (8 - len(cfg))
        return f(L, dtype, n, purpose, ctypes.byref(_lib.RmhHopConfig(*full)))

    ok = [(0, 256, 1, 4, 0, 0, 1), (1, 64, 0, 4, 1, 0, 1), (2, 128, 1, 2, 2, 0, 1), (1, 256, 1, 1, 2, 0, 1),
          (2, 128, 0, 4, 0, 4, 1), (1, 128, 1, 2, 3, 0, 1), (0, 64, 1, 4, 1, 0, 2), (2, 128, 0, 4, 0, 0, 2),
          (0, 256, 1, 4, 0, 8, 1, 2), (2, 128, 0, 4, 0, 4, 1, 4)]
    for cfg in ok:
        assert put(cfg) == 0, cfg
    assert put((2, 64, 1, 4, 0, 0, 4), dtype=1) == 0                # four fields per thread: FP32
    for purpose in range(-1, 7):
        assert put((0, 256, 1, 4, 0, 0, 1), purpose=purpose) == 0
    bad = [(3, 256, 1, 4, 0, 0, 1),     # form
           (0, 96, 1, 4, 0, 0, 1),      # block
           (0, 256, 1, 3, 0, 0, 1),     # nv
           (0, 256, 1, 1, 0, 0, 1),     # nv = 1 needs form 1
           (0, 64, 1, 2, 2, 0, 1),      # half a wave per direction group
           (0, 256, 1, 4, 4, 0, 1),     # order
           (0, 256, 1, 4, -1, 0, 1),
           (0, 256, 1, 4, 0, 65, 1),    # walk
           (0, 256, 2, 4, 0, 0, 1),     # xcd_remap
           (0, 256, 1, 4, 0, 0, 3),     # ns
           (1, 256, 1, 4, 0, 0, 2),     # ns > 1 with the 3x3 form
           (0, 256, 1, 2, 0, 0, 2),     # ns > 1 with nv = 2
           (0, 256, 1, 4, 2, 0, 2),     # ns > 1 with the hop-split order
           (0, 256, 1, 4, 0, 4, 2),     # ns > 1 with a walk
           (0, 256, 1, 4, 0, 0, 4),     # ns = 4 in FP64
           (0, 256, 1, 4, 0, 8, 1, 3),  # tile2
           (0, 256, 1, 4, 0, 0, 1, 2)]  # tile2 > 1 without a walk
    for cfg in bad:
        assert put(cfg) == 1, cfg                                    # RMH_E_ARG
    for purpose in (-2, 7):
        assert put((0, 256, 1, 4, 0, 0, 1), purpose=purpose) == 1
    assert put((0, 256, 1, 4, 0, 0, 1), n=0) == 1
    assert f(L, 0, 1, -1, None) == 1
    assert _lib.lib().rmh_tune_clear() == 0


def test_tune_file_round_trip(tmp_path):
    """The launch cache survives a save / clear / load round trip through its JSON file (keyed by
    lattice, dtype, batch and purpose, stamped with the device architecture and HIP runtime); a
    file stamped for another architecture loads nothing; malformed files and invalid entries are
    rejected before anything is stored."""
    lib_ = _lib.lib()
    assert lib_.rmh_tune_clear() == 0
    entries = [((4, 4, 4, 4), 0, 1, -1, (0, 256, 1, 4, 0, 0, 1, 1)),
               ((4, 4, 4, 4), 0, 1, 3, (2, 64, 1, 4, 1, 0, 1, 1)),
               ((8, 8, 4, 4), 1, 32, 3, (2, 64, 1, 4, 1, 0, 4, 1)),
               ((32, 32, 32, 64), 0, 1, 0, (0, 256, 1, 4, 0, 8, 1, 2)),
               ((16, 16, 16, 16), 0, 12, 2, (1, 128, 0, 2, 2, 0, 1, 1))]
    for L, dt, n, purpose, cfg in entries:
        assert lib_.rmh_tune_set(_lib.lattice_arg(L), dt, n, purpose, ctypes.byref(_lib.RmhHopConfig(*cfg))) == 0
    p1, p2 = str(tmp_path / "a.json"), str(tmp_path / "b.json")
    n = ctypes.c_int32(0)
    assert lib_.rmh_tune_save(p1.encode(), ctypes.byref(n)) == 0 and n.value == 5
    doc = json.load(open(p1))
    assert doc["format"] == "rmh-tune-1" and len(doc["entries"]) == 5
    got = {(tuple(e[k] for k in ("L0", "L1", "L2", "L3")), e["dtype"], e["n_rhs"], e["purpose"]):
           tuple(e[k] for k in ("form", "block", "xcd_remap", "nv", "order", "walk", "ns", "tile2"))
           for e in doc["entries"]}
    assert got == {(L, dt, n_, p): cfg for L, dt, n_, p, cfg in entries}
    assert lib_.rmh_tune_clear() == 0
    assert lib_.rmh_tune_save(p2.encode(), ctypes.byref(n)) == 0 and n.value == 0
    assert lib_.rmh_tune_load(p1.encode(), ctypes.byref(n)) == 0 and n.value == 5
    assert lib_.rmh_tune_save(p2.encode(), ctypes.byref(n)) == 0 and n.value == 5
    assert open(p1).read() == open(p2).read()
    # another architecture: nothing stored
    other = dict(doc, arch=doc["arch"] + "-other")
    p3 = str(tmp_path / "c.json")
    json.dump(other, open(p3, "w"))
    assert lib_.rmh_tune_clear() == 0
    assert lib_.rmh_tune_load(p3.encode(), ctypes.byref(n)) == 0 and n.value == 0
    # malformed file, invalid entry (ns = 4 in FP64), missing file, null path
    p4 = str(tmp_path / "d.json")
    open(p4, "w").write("{not json")
    assert lib_.rmh_tune_load(p4.encode(), ctypes.byref(n)) == 1
    bad = dict(doc, entries=[dict(doc["entries"][0], dtype=0, ns=4)])
    json.dump(bad, open(p4, "w"))
    assert lib_.rmh_tune_load(p4.encode(), ctypes.byref(n)) == 1
    assert lib_.rmh_tune_save(p2.encode(), ctypes.byref(n)) == 0 and n.value == 0     # nothing was stored
    assert lib_.rmh_tune_load(str(tmp_path / "missing.json").encode(), ctypes.byref(n)) == 9
    assert lib_.rmh_tune_load(None, None) == 1
    assert lib_.rmh_tune_save(None, None) == 1


def test_leapfrog_validation():
    """rmh_leapfrog_step rejects bad controls, a short workspace and aliased buffers before any
    device work."""
    Lt = (2, 2, 2, 2)
    L = _lib.lattice_arg(Lt)
    r = np.array([1.0, 2.0])
    sg = np.array([0.5, 1.0])
    rat = _lib.RmhRational(0.0, 2, r.ctypes.data_as(_lib.P_f64), sg.ctypes.data_as(_lib.P_f64))
    sv = _lib.RmhSolver(1e-10, 100, 0, 0.1, 8, 0.0, 0)
    f = _lib.lib().rmh_leapfrog_step
    need = _lib.lib().rmh_workspace_bytes(_lib.OP_LEAPFROG, L, 0, 1, 2, 0, 0)
    assert need > _lib.lib().rmh_workspace_bytes(_lib.OP_KINETIC_FORCE, L, 0, 1, 2, 0, 0)
    U0, P0, U1, P1, WS = FAKE, FAKE + 2**20, FAKE + 2**21, FAKE + 2**22, FAKE + 2**23

    def call(lf, u1=U1, p1=P1, ws_bytes=1 << 30):
        return f(L, U0, P0, ctypes.byref(rat), ctypes.byref(sv), ctypes.byref(lf) if lf is not None else None,
                 u1, p1, None, WS, ws_bytes, None)

    ok = _lib.RmhLeapfrog(0.1, 5.0, 1e-12, 20)
    assert call(None) == 1
    assert call(_lib.RmhLeapfrog(float("inf"), 5.0, 1e-12, 20)) == 1
    assert call(_lib.RmhLeapfrog(0.1, float("nan"), 1e-12, 20)) == 1
    assert call(_lib.RmhLeapfrog(0.1, 5.0, 0.0, 20)) == 1
    assert call(_lib.RmhLeapfrog(0.1, 5.0, 1e-12, 0)) == 1
    assert call(ok, ws_bytes=need - 8) == 3                      # workspace too small
    assert call(ok, u1=U0) == 1                                  # U1 aliases U0
    assert call(ok, p1=P0 + 64) == 1                             # P1 overlaps P0


def test_product_path_does_not_use_the_oracle():
    """Nothing in the package (Python binding, HIP and C++ sources) imports or reads the oracle;
    bench.py touches it only in its CPU-baseline leg."""
    import glob
    import os
    import re
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..")
    pkg = os.path.join(root, "paper_2112_04556_amd")
    files = [f for ext in ("py", "hip", "h", "cpp") for f in glob.glob(os.path.join(pkg, "**", f"*.{ext}"), recursive=True)]
    assert files
    pat = re.compile(r"^\s*(from\s+oracle\b|import\s+oracle\b)|[\"']oracle/", re.M)
    for f in files:
        with open(f) as fh:
            assert not pat.search(fh.read()), f
    with open(os.path.join(root, "bench.py")) as fh:
        src = fh.read()
    uses = [m.start() for m in re.finditer(r"from oracle|import oracle", src)]
    leg = src.index("# ---- the CPU-baseline leg")
    end = src.index("# ---- end of the CPU-baseline leg")
    assert leg < src.index("def cpu_baseline") < end
    assert uses and all(leg < u < end for u in uses)


@pytest.mark.parametrize("nw", [0, -1, -7, 100000])
def test_window_count_rejected_before_allocation(nw):
    """A window count outside the range is an argument error in every Chebyshev call, caught before
    any buffer is sized by it (a negative count must not become a huge allocation)."""
    L = _lib.lattice_arg((4, 4, 4, 4))
    ch = _lib.RmhCheb(8, nw, None, 1)
    mom = np.zeros(9)
    lib = _lib.lib()
    assert lib.rmh_power_spectrum(L, FAKE, 0, FAKE + 2**20, 1, ctypes.byref(ch), None, None, FAKE + 2**22, 1 << 30,
                                  None) == 1
    assert lib.rmh_cheb_filter(L, FAKE, 0, FAKE + 2**20, 1, ctypes.byref(ch), FAKE + 2**21, FAKE + 2**22, 1 << 30,
                               None) == 1
    assert lib.rmh_cheb_filter_bwd(L, FAKE, FAKE + 2**20, FAKE + 2**21, 1, ctypes.byref(ch), FAKE + 2**23, None, 0,
                                   FAKE + 2**22, 1 << 30, None) == 1
    p = mom.ctypes.data_as(_lib.P_f64)
    assert lib.rmh_power_ratio(ctypes.byref(ch), p, p, 1, p) == 1


def test_degree_out_of_range_rejected():
    L = _lib.lattice_arg((4, 4, 4, 4))
    mom = np.zeros(4)
    p = mom.ctypes.data_as(_lib.P_f64)
    lib = _lib.lib()
    for D in (-3, 100001):
        ch = _lib.RmhCheb(D, 2, None, 1)
        assert lib.rmh_power_spectrum(L, FAKE, 0, FAKE + 2**20, 1, ctypes.byref(ch), None, None, FAKE + 2**22,
                                      1 << 30, None) == 1
        assert lib.rmh_power_ratio(ctypes.byref(ch), p, p, 1, p) == 1
    ch = _lib.RmhCheb(2**31 - 1, 2, None, 1)
    assert lib.rmh_cheb_coefficients(ctypes.byref(ch), p) == 1
    assert lib.rmh_trace_moments_free(L, 2**31 - 1, p) == 1
    ch0 = _lib.RmhCheb(0, 2, None, 1)        # degree 0 is a valid host-side ratio (T_0 only)
    mom[:] = 1.0
    assert lib.rmh_power_ratio(ctypes.byref(ch0), p, p, 1, p) == 0


def test_empty_batch_is_a_no_op():
    """n_rhs = 0 returns RMH_OK after argument checks, before any pointer is used or any GPU call
    (the pointers here are never mapped)."""
    L = _lib.lattice_arg((4, 4, 4, 4))
    lib = _lib.lib()
    r, s = np.array([1.0, 2.0]), np.array([0.5, 1.0])
    rat = _lib.RmhRational(0.0, 2, r.ctypes.data_as(_lib.P_f64), s.ctypes.data_as(_lib.P_f64))
    sv = _lib.RmhSolver(1e-10, 100, 0, 0.1, 8, 0.0, 0)
    ch = _lib.RmhCheb(8, 2, None, 1)
    st = _lib.RmhStats()
    assert lib.rmh_laplacian_apply(L, FAKE, 0, FAKE + 2**20, FAKE + 2**21, 0, 0.0, None) == 0
    assert lib.rmh_power_spectrum(L, FAKE, 0, FAKE + 2**20, 0, ctypes.byref(ch), None, None, FAKE + 2**22, 1 << 30,
                                  None) == 0
    assert lib.rmh_cheb_filter(L, FAKE, 0, FAKE + 2**20, 0, ctypes.byref(ch), FAKE + 2**21, FAKE + 2**22, 1 << 30,
                               None) == 0
    assert lib.rmh_rational_apply(L, FAKE, FAKE + 2**20, 0, ctypes.byref(rat), ctypes.byref(sv), FAKE + 2**21, None,
                                  None, ctypes.byref(st), FAKE + 2**22, 1 << 30, None) == 0
    assert lib.rmh_kinetic_force(L, FAKE, FAKE + 2**20, 0, ctypes.byref(rat), ctypes.byref(sv), None, None,
                                 FAKE + 2**23, 0, ctypes.byref(st), FAKE + 2**22, 1 << 30, None) == 0


def test_every_entry_point_catches_host_exceptions():
    """Each exported definition is a function-try-block, so no C++ exception crosses the C ABI."""
    src = open(os.path.join(ROOT, "paper_2112_04556_amd", "csrc", "rmh_api.hip")).read()
    body = src[src.index('extern "C" {'):src.index('}  // extern "C"')]
    defs = re.findall(r"^(?:rmh_status|size_t) (rmh_[a-z0-9_]+)\((.*?)\)\s*(try )?\{", body, flags=re.M | re.S)
    assert len(defs) >= 25
    missing = [name for name, _, t in defs if not t]
    assert not missing, missing


def test_power_spectrum_noalloc_limits():
    """The entry point that allocates nothing rejects a call larger than its 64 MiB static scratch
    (RMH_E_WORKSPACE) and bad arguments (RMH_E_ARG) before touching any pointer or the device."""
    f = _lib.lib().rmh_power_spectrum_noalloc
    cheb = _lib.RmhCheb(64, 16, None, 1)
    big = _lib.lattice_arg((32, 32, 32, 32))          # two FP64 recursion fields alone: 1 GiB
    assert f(big, FAKE, 0, FAKE + 2**31, 1, ctypes.byref(cheb), None, None, None) == 3
    assert b"static scratch" in _lib.lib().rmh_last_error()
    # 16^4: one FP64 source fits, two do not
    L16 = _lib.lattice_arg((16, 16, 16, 16))
    ws1 = _lib.lib().rmh_workspace_bytes(2, L16, 0, 1, 16, 64, 0)
    ws2 = _lib.lib().rmh_workspace_bytes(2, L16, 0, 2, 16, 64, 0)
    assert ws1 <= 64 << 20 < ws2
    assert f(L16, FAKE, 0, FAKE + 2**31, 2, ctypes.byref(cheb), None, None, None) == 3
    bad = _lib.RmhCheb(0, 16, None, 1)                 # degree 0 on the device path
    assert f(L16, FAKE, 0, FAKE + 2**31, 1, ctypes.byref(bad), None, None, None) == 1
    assert f(L16, FAKE, 0, FAKE + 2**31, -1, ctypes.byref(cheb), None, None, None) == 1
    assert f(L16, FAKE, 0, FAKE + 2**31, 0, ctypes.byref(cheb), None, None, None) == 0   # empty batch: no-op


def test_autotune_workspace_validation():
    """The autotuner's dot-product partials come from the caller's workspace: a missing, short or
    overlapping one is refused before any device work (fake addresses, never dereferenced)."""
    L = _lib.lattice_arg((4, 4, 4, 4))
    f = _lib.lib().rmh_autotune_laplacian
    need = _lib.lib().rmh_workspace_bytes(_lib.OP_AUTOTUNE, L, 0, 2, 0, 0, 0)
    U, x, y, ws = FAKE, FAKE + 2**20, FAKE + 2**21, FAKE + 2**22

    def call(ws_ptr, ws_bytes):
        return f(L, U, 0, x, y, 2, 1, 1, None, None, ws_ptr, ws_bytes, None)

    assert call(None, need) == 1                  # RMH_E_ARG: no workspace
    assert call(ws, need - 8) == 3                # RMH_E_WORKSPACE
    assert call(y + 256, need) == 1               # the workspace overlaps y
    assert call(x, need) == 1                     # ... or x

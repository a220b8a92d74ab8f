"""GPU parity of layout conversion, the stencil and its link derivative against the oracle.

Tolerances: FP64 results within 1e-12 of the oracle relative to the largest output
magnitude.  FP32 stencil: every output is a sum of 65 terms bounded by max|x| (R(U) is
orthogonal) with R itself rounded once per entry; the typical error is ~sqrt(65) * 8 u
max|x| with u = 2^-24, so the test takes max error <= 1e-5 max|y| and rms error <= 1e-6 rms(y).
"""
import numpy as np
import pytest
import torch

from gpu_helpers import announce, dev, rel_max, setup
from oracle import laplacian as olap
from paper_2112_04556_amd import api, inputs
from paper_2112_04556_amd._lib import RmhError

pytestmark = pytest.mark.gpu

# (L, link kind, seed): L = 2 edges, ragged volumes (not a multiple of 64), anisotropic shapes
CASES = [((2, 2, 2, 2), "eps", 1), ((4, 4, 4, 4), "haar", 2), ((3, 5, 2, 7), "eps", 3),
         ((8, 4, 6, 4), "unit", 4), ((2, 6, 4, 3), "haar", 5)]


@pytest.mark.parametrize("L,kind,seed", CASES)
def test_pack_links_bitwise(L, kind, seed):
    announce(f"pack_links {L} {kind}")
    U = inputs.random_links(L, kind, 0.5, seed=seed)
    Ud = U.to(dev())
    soa = api.pack_links(L, Ud, torch.float64).cpu().numpy()
    ref = np.moveaxis(torch.view_as_real(U).numpy().reshape(4, -1, 18), 1, 2)
    assert np.array_equal(soa, ref)
    soa32 = api.pack_links(L, Ud, torch.float32).cpu().numpy()
    assert np.array_equal(soa32, ref.astype(np.float32))     # round to nearest even
    back = api.unpack_links(L, api.pack_links(L, Ud, torch.float64)).cpu()
    assert torch.equal(back, U)


def test_pack_fields_and_convert_bitwise():
    L = (3, 5, 2, 7)
    F = inputs.gaussian_fields(L, 3, seed=4)                         # (n, 4, 8, V) SoA
    aos = F.permute(0, 3, 1, 2).contiguous()                          # (n, V, 4, 8)
    soa = api.pack_fields(L, aos.to(dev()), torch.float64)
    assert torch.equal(soa.cpu(), F)
    assert torch.equal(api.unpack_fields(L, soa).cpu(), aos)
    soa32 = api.pack_fields(L, aos.to(dev()), torch.float32)
    assert np.array_equal(soa32.cpu().numpy(), F.numpy().astype(np.float32))
    c = api.convert_f64_f32(F.to(dev()))
    assert np.array_equal(c.cpu().numpy(), F.numpy().astype(np.float32))


@pytest.mark.parametrize("L,kind,seed", CASES)
@pytest.mark.parametrize("shift", [0.0, 0.7])
def test_laplacian_fp64_parity(L, kind, seed, shift):
    announce(f"laplacian fp64 {L} {kind} shift={shift}")
    U, P, Ud, Pd = setup(L, kind, 0.5, seed, n=2)
    ref = olap.laplacian(U, P, L, shift)
    for form in (0, 1, 2):
        shapes = ((4, 0, 128), (2, 0, 128), (2, L[3], 128), (4, 1, 128))
        if form == 1:
            shapes += ((1, 0, 256), (1, L[3], 256))
        for nv, walk, block in shapes:
            api.tune_set(L, torch.float64, 2, form, block, 1, nv, 1, walk)
            y = api.laplacian_apply(L, Ud, Pd, shift).cpu().numpy()
            assert rel_max(y, ref) <= 1e-12, (form, nv, walk)
    api.tune_clear()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_laplacian_reads_rows_0_and_1_only(dtype):
    """Every launch shape rebuilds row 2 of each link from rows 0 and 1: with components 12..17
    of the SoA links overwritten by NaN the output is bitwise unchanged."""
    L = (4, 4, 2, 6)
    announce(f"laplacian row-2 rebuild {dtype}")
    U, P, Ud, Pd = setup(L, "haar", 0.5, 3, n=2)
    U2 = api.pack_links(L, inputs.random_links(L, "haar", seed=3).to(dev()), dtype)
    x = Pd.to(dtype)
    bad = U2.clone()
    bad[:, 12:18, :] = float("nan")
    shapes = [(0, 128, 4, 0, 0), (1, 256, 1, 0, 0), (2, 128, 2, L[3], 0), (2, 256, 4, 0, 2), (1, 128, 2, 0, 3)]
    for form, block, nv, walk, order in shapes:
        api.tune_set(L, dtype, 2, form, block, 1, nv, order, walk)
        a = api.laplacian_apply(L, U2, x)
        b = api.laplacian_apply(L, bad, x)
        assert torch.equal(a, b), (form, block, nv, walk, order)
    api.tune_clear()


@pytest.mark.parametrize("form", [0, 1, 2])
@pytest.mark.parametrize("L,kind,seed", CASES[:3])
def test_laplacian_fp32_parity(L, kind, seed, form):
    announce(f"laplacian fp32 form={form} {L}")
    U, P, Ud, Pd = setup(L, kind, 0.5, seed, n=2, dtype=torch.float32)
    api.tune_set(L, torch.float32, 2, form, 256, 1)
    try:
        y = api.laplacian_apply(L, Ud, Pd).cpu().numpy().astype(np.float64)
    finally:
        api.tune_clear()
    ref = olap.laplacian(U, P, L)
    err = y - ref
    assert np.abs(err).max() <= 1e-5 * np.abs(ref).max()
    assert np.sqrt((err ** 2).mean()) <= 1e-6 * np.sqrt((ref ** 2).mean())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_laplacian_configs_batched_and_deterministic(dtype):
    """Bitwise identity across block sizes and XCD remaps of one form, batched vs single, run to run."""
    L = (8, 8, 5, 6)   # L0 * L1 = 64: the x3-fastest order applies for 64 sites per block
    announce(f"laplacian configs {dtype}")
    _, _, Ud, Pd = setup(L, "haar", 0.0, 7, n=3, dtype=dtype)
    for form in (0, 1, 2):
        outs = []
        for block in (64, 128, 256):
            for xcd, order, walk in ((0, 0, 0), (1, 1, 0), (0, 1, 0), (1, 0, 2), (0, 0, 3), (0, 0, 6)):
                for nv in ((4, 2, 1) if form == 1 else (4, 2)):
                    if (block * nv // 4) % 64:
                        # a direction group must span whole wavefronts
                        with pytest.raises(RmhError):
                            api.tune_set(L, dtype, 3, form, block, xcd, nv, order, walk)
                        continue
                    api.tune_set(L, dtype, 3, form, block, xcd, nv, order, walk)
                    api.tune_set(L, dtype, 1, form, block, xcd, nv, order, walk)
                    y = api.laplacian_apply(L, Ud, Pd)
                    y1 = api.laplacian_apply(L, Ud, Pd[1:2].contiguous())
                    assert torch.equal(y[1:2], y1)
                    outs.append(y)
        api.tune_clear()
        for o in outs[1:]:
            assert torch.equal(o, outs[0])
    y_a = api.laplacian_apply(L, Ud, Pd)
    y_b = api.laplacian_apply(L, Ud, Pd)
    assert torch.equal(y_a, y_b)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_laplacian_walk_tiles_bitwise(dtype):
    """The walking kernel with x2-tiled column blocks (tile2 = 2, 4) over walks of 2, 3 and 6 x3 sites,
    both XCD maps and two block sizes, on a lattice the tiles fit (and, at block 256, one they do not,
    where the shape falls back to one thread per site): bitwise equal to the untiled kernel of the
    same form, batched and single, and the FP64 result within 1e-12 of the oracle."""
    L = (8, 8, 4, 6)
    announce(f"laplacian walk tiles {dtype}")
    U, P, Ud, Pd = setup(L, "haar", 0.0, 17, n=3, dtype=dtype)
    for form in (0, 2):
        api.tune_set(L, dtype, 3, form, 64, 0, 4, 0, 0)
        ref = api.laplacian_apply(L, Ud, Pd)
        for block in (64, 128, 256):
            for walk in (2, 3, 6):
                for tile2 in (1, 2, 4):
                    for xcd in (0, 1):
                        api.tune_set(L, dtype, 3, form, block, xcd, 4, 0, walk, tile2=tile2)
                        api.tune_set(L, dtype, 1, form, block, xcd, 4, 0, walk, tile2=tile2)
                        y = api.laplacian_apply(L, Ud, Pd)
                        y1 = api.laplacian_apply(L, Ud, Pd[2:3].contiguous())
                        assert torch.equal(y, ref), (form, block, walk, tile2, xcd)
                        assert torch.equal(y[2:3], y1), (form, block, walk, tile2, xcd)
        api.tune_clear()
        if dtype == torch.float64:
            yref = olap.laplacian(U, P, L)
            assert rel_max(ref.cpu().numpy(), yref) <= 1e-12


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_laplacian_multi_field_bitwise(dtype):
    """ns fields per thread (each link and adjoint matrix serving 4 ns vectors): every field's result
    is bitwise that of one field per thread with the same form, for plain applications, the Chebyshev
    recursion step with its dot products (power spectrum) and the CG (fields that stop at different
    iterations), and within the oracle's tolerance."""
    L = (8, 8, 5, 6)
    announce(f"laplacian multi-field {dtype}")
    U, P, Ud, Pd = setup(L, "haar", 0.0, 17, n=4, dtype=dtype)
    ref = olap.laplacian(U if dtype == torch.float64 else U.astype(np.complex64).astype(np.complex128),
                         Pd.double().cpu().numpy(), L, 0.0)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    nss = (2, 4) if dtype == torch.float32 else (2,)
    for form in (0, 2):
        api.tune_set(L, dtype, 4, form, 64, 1, 4, 1, 0)
        y1 = api.laplacian_apply(L, Ud, Pd)
        assert rel_max(y1.double().cpu().numpy(), ref) <= tol
        for block, xcd, order in ((64, 1, 1), (256, 0, 0), (128, 1, 0)):
            # the dot products are summed per block: bitwise only against the same block partition
            api.tune_set(L, dtype, 4, form, block, xcd, 4, order, 0)
            m1, p1 = api.power_spectrum(L, Ud, Pd, 12, 3)
            for ns in nss:
                api.tune_set(L, dtype, 4, form, block, xcd, 4, order, 0, ns=ns)
                y = api.laplacian_apply(L, Ud, Pd)
                assert torch.equal(y, y1), (form, ns, block, xcd, order)
                m, p = api.power_spectrum(L, Ud, Pd, 12, 3)
                assert np.array_equal(m, m1) and np.array_equal(p, p1), (form, ns, block)
        api.tune_clear()
    if dtype == torch.float64:
        # the FP64 multi-shift CG over two fields: one field per thread against two
        rat = api.rational_kappa(0.9, 4)
        P2 = Pd[:2].contiguous()
        api.tune_set(L, dtype, 2, 0, 64, 1, 4, 1, 0, purpose="cg")
        a = api.rational_apply(L, Ud, P2, rat, api.Solver(tol=1e-10), want_poles=True)
        api.tune_set(L, dtype, 2, 0, 64, 1, 4, 1, 0, ns=2, purpose="cg")
        b = api.rational_apply(L, Ud, P2, rat, api.Solver(tol=1e-10), want_poles=True)
        api.tune_clear()
        assert torch.equal(a["x_poles"], b["x_poles"]) and a["stats"]["iters"] == b["stats"]["iters"]


@pytest.mark.parametrize("L,kind,seed", CASES)
def test_laplacian_hop_split_parity(L, kind, seed):
    """order = 2: four lanes per site, one per direction, summed by wave shuffles."""
    announce(f"laplacian hop split {L} {kind}")
    U, P, Ud, Pd = setup(L, kind, 0.5, seed, n=2)
    ref = olap.laplacian(U, P, L, 0.4)
    U32, P32 = Ud.float(), Pd.float()
    outs = {}
    for form in (0, 1, 2):
        for nv, block in ((4, 64), (4, 256), (2, 128), (2, 256)) + (((1, 256),) if form == 1 else ()):
            # order 3: the x3-fastest block order (when L0 * L1 holds whole blocks)
            for order, xcd in ((2, 1), (3, 1), (3, 0)):
                api.tune_set(L, torch.float64, 2, form, block, xcd, nv, order, 0)
                y = api.laplacian_apply(L, Ud, Pd, 0.4).cpu().numpy()
                assert rel_max(y, ref) <= 1e-12, (form, nv, block, order)
                # the block order does not change any site's arithmetic
                assert np.array_equal(outs.setdefault((form, nv), y), y), (form, nv, block, order)
            api.tune_set(L, torch.float32, 2, form, block, 0, nv, 2, 0)
            y32 = api.laplacian_apply(L, U32, P32, 0.4).cpu().numpy().astype(np.float64)
            assert np.abs(y32 - ref).max() <= 1e-5 * np.abs(ref).max(), (form, nv, block)
    with pytest.raises(RmhError):
        api.tune_set(L, torch.float64, 2, 0, 64, 1, 2, 2, 0)    # two direction groups need two waves
    with pytest.raises(RmhError):
        api.tune_set(L, torch.float64, 2, 0, 256, 1, 4, 4, 0)   # no order 4
    api.tune_clear()


@pytest.mark.parametrize("form,block,nv", [(1, 256, 2), (1, 128, 2), (0, 64, 4), (1, 256, 1), (2, 128, 4)])
def test_hop_split_fused_epilogues(form, block, nv):
    """The hop-split kernel's dot products (spectrum moments, CG) give the site-per-thread kernel's
    results to rounding, also in the shapes with 16 sites per block (block 64 / nv 4, block 128 /
    nv 2, block 256 / nv 1), whose block count is the largest any shape launches."""
    L = (4, 3, 2, 5)    # V = 120: 16-site blocks with a ragged tail
    announce(f"hop split fused epilogues {L} form={form} block={block} nv={nv}")
    U, F, Ud, Fd = setup(L, "eps", 0.5, 9, n=2)
    rat = api.rational_kappa(0.8, 8)
    runs = []
    for cfg in ((1, 256, 1, 2, 0, 0), (form, block, 1, nv, 2, 0)):
        api.tune_set(L, torch.float64, 1, *cfg)   # nearest-batch entry: every launch on L
        mom, pw = api.power_spectrum(L, Ud, Fd, 30, 6)
        yf = api.cheb_filter(L, Ud, Fd, 30, 6).cpu().numpy()
        out = api.rational_apply(L, Ud, Fd, rat, api.Solver(tol=1e-12))
        runs.append((mom, pw, yf, out["y"].cpu().numpy(), out["stats"]["true_relres_max"]))
    api.tune_clear()
    (m0, p0, f0, y0, r0), (m1, p1, f1, y1, r1) = runs
    assert np.all(np.abs(m1 - m0) <= 1e-12 * m0[:, :1])
    assert np.all(np.abs(p1 - p0) <= 1e-12 * m0[:, :1])
    assert rel_max(f1, f0) <= 1e-12
    assert r0 <= 1e-12 and r1 <= 1e-12
    assert rel_max(y1, y0) <= 1e-10


def test_laplacian_empty_batch_and_autotune():
    L = (4, 4, 4, 4)
    _, _, Ud, Pd = setup(L, "eps", 0.3, 1, n=1)
    empty = torch.empty((0, 4, 8, api.volume(L)), dtype=torch.float64, device=dev())
    api.laplacian_apply(L, Ud, empty)
    (form, block, xcd, nv, order, walk, ns, tile2), ms = api.autotune_laplacian(L, Ud, Pd, reps=2)
    assert form in (0, 1, 2) and block in (64, 128, 256) and nv in (1, 2, 4) and ms > 0
    assert nv != 1 or form == 1
    assert ns == 1 and tile2 in (1, 2, 4)
    U, P, _, _ = setup(L, "eps", 0.3, 1, n=1)
    assert rel_max(api.laplacian_apply(L, Ud, Pd).cpu().numpy(), olap.laplacian(U, P, L)) <= 1e-12
    api.tune_clear()


def test_autotune_per_purpose_and_cache_file(tmp_path):
    """The autotuner keys its result by purpose; the cache written to a file (stamped with this
    device's architecture) is read back into an empty cache with the same configurations."""
    L = (8, 8, 5, 6)
    _, _, Ud, Pd = setup(L, "eps", 0.3, 2, n=4)
    api.tune_clear()
    c_apply, _ = api.autotune_laplacian(L, Ud, Pd, reps=1, purpose="apply")
    c_mom, _ = api.autotune_laplacian(L, Ud, Pd, reps=1, purpose="moments")
    path = str(tmp_path / "tune.json")
    assert api.tune_save(path) == 2
    import json
    doc = json.load(open(path))
    assert doc["arch"].startswith("gfx950") and doc["hip_runtime"] > 0
    assert sorted(e["purpose"] for e in doc["entries"]) == [0, 3]
    api.tune_clear()
    assert api.tune_load(path) == 2
    path2 = str(tmp_path / "tune2.json")
    assert api.tune_save(path2) == 2
    got = {e["purpose"]: tuple(e[k] for k in ("form", "block", "xcd_remap", "nv", "order", "walk", "ns", "tile2"))
           for e in json.load(open(path2))["entries"]}
    assert got == {0: c_apply, 3: c_mom}
    api.tune_clear()


@pytest.mark.parametrize("L,kind,seed", CASES[:4])
def test_laplacian_bwd_parity(L, kind, seed):
    announce(f"laplacian bwd {L} {kind}")
    U, x, Ud, xd = setup(L, kind, 0.5, seed, n=2)
    g = inputs.gaussian_fields(L, 2, seed=seed + 100)
    gx, go = api.laplacian_apply_bwd(L, Ud, xd, g.to(dev()), 0.3, per_rhs=False)
    ref_go = olap.bilinear_link_derivative(U, g.numpy(), x, L)
    assert rel_max(go[0].cpu().numpy(), ref_go) <= 1e-12
    assert rel_max(gx.cpu().numpy(), olap.laplacian(U, g.numpy(), L, 0.3)) <= 1e-12
    _, go_r = api.laplacian_apply_bwd(L, Ud, xd, g.to(dev()), 0.0, grad_x=False, per_rhs=True)
    for i in range(2):
        ref_i = olap.bilinear_link_derivative(U, g.numpy()[i:i + 1], x[i:i + 1], L)
        assert rel_max(go_r[i].cpu().numpy(), ref_i) <= 1e-12


def test_laplacian_full_size_16():
    """The 16^4 lattice at eps = 0.5 (the FP64 rational-solve workload): whole-lattice parity."""
    L = (16, 16, 16, 16)
    announce("laplacian 16^4")
    U, P, Ud, Pd = setup(L, "eps", 0.5, 2, n=1)
    y = api.laplacian_apply(L, Ud, Pd).cpu().numpy()
    assert rel_max(y, olap.laplacian(U, P, L)) <= 1e-12

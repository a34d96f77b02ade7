"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: FP32 chain proxes and TV iterates within 1e-4 relative L-inf of
the FP64 oracle on identical FP32 inputs; cut energies bit-exact (integer and
2^-8-dyadic data make every energy an exact FP64 sum, and a certificate below
1e-3 is below the data's energy granularity).
"""
import numpy as np
import pytest

import oracle
from paper_1503_01563_amd import gen

pytestmark = pytest.mark.gpu

REL_TOL = 1e-4


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_01563_amd import mc
    mc.load_library()
    return torch.device("cuda:0")


def to_dev(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


def rel_linf(x, ref):
    return float(np.abs(np.asarray(x, np.float64) - ref).max() / max(1.0, np.abs(ref).max()))


def chain_inputs(kind, shape, rng):
    if kind == "random":
        v = rng.normal(size=shape) * 5
        a = rng.uniform(0, 2, size=shape)
    elif kind == "integer":
        v = rng.integers(-20, 21, size=shape).astype(float)
        a = rng.integers(0, 11, size=shape).astype(float)
    elif kind == "piecewise":
        v = np.repeat(rng.normal(size=shape[:-1] + ((shape[-1] + 7) // 8,)) * 10, 8, axis=-1)[..., : shape[-1]]
        v = v + rng.normal(size=shape) * 0.1
        a = np.full(shape, 0.5)
    elif kind == "staircase":
        v = np.cumsum(rng.uniform(0, 3, size=shape), axis=-1)
        a = np.full(shape, 2.0)
    elif kind == "zero_runs":
        v = rng.normal(size=shape)
        a = np.where(rng.uniform(size=shape) < 0.4, 0.0, rng.uniform(0, 1, size=shape))
    elif kind == "huge_a":
        v = rng.normal(size=shape)
        a = np.full(shape, 1e6)
    elif kind == "offset":
        v = rng.normal(size=shape) * 3 + 1e4
        a = rng.uniform(0, 10, size=shape)
    else:
        raise ValueError(kind)
    return v.astype(np.float32), a.astype(np.float32)


KINDS = ["random", "integer", "piecewise", "staircase", "zero_runs", "huge_a", "offset"]


@pytest.mark.parametrize("length", [1, 2, 3, 7, 8, 64, 127, 1024])
@pytest.mark.parametrize("kind", KINDS)
def test_prox_rows_parity(dev, length, kind):
    from paper_1503_01563_amd import mc
    rng = np.random.default_rng(length * 31 + KINDS.index(kind))
    shape = (67, length)  # 67 chains: one full wave plus a ragged tail
    v, a = chain_inputs(kind, shape, rng)
    a[:, -1] = 0
    x, p = mc.tv_prox_chains(to_dev(v, dev), to_dev(a, dev), 0, return_p=True)
    xr, pr = oracle.prox_family(shape, 0, v.astype(np.float64), a.astype(np.float64))
    assert rel_linf(x.cpu().numpy(), xr) <= REL_TOL
    pg = p.cpu().numpy()
    assert np.all(np.abs(pg) <= a)
    assert np.all(pg[:, -1] == 0)
    scale = max(1.0, np.abs(pr).max())
    assert float(np.abs(pg - pr).max()) / scale <= REL_TOL


@pytest.mark.parametrize("shape,axis", [((5, 33, 70), 0), ((5, 33, 70), 1), ((5, 33, 70), 2),
                                        ((129, 3), 1), ((3, 129), 0), ((1, 1), 0), ((1, 1), 1),
                                        ((1, 200), 1), ((200, 1), 0), ((40, 1, 9), 2)])
def test_prox_axes_parity(dev, shape, axis):
    from paper_1503_01563_amd import mc
    rng = np.random.default_rng(sum(shape) + axis)
    v = (rng.normal(size=shape) * 4).astype(np.float32)
    a = rng.uniform(0, 2, size=shape).astype(np.float32)
    x, p = mc.tv_prox_chains(to_dev(v, dev), to_dev(a, dev), axis, return_p=True)
    xr, pr = oracle.prox_family(shape, axis, v.astype(np.float64), a.astype(np.float64))
    assert rel_linf(x.cpu().numpy(), xr) <= REL_TOL


@pytest.mark.parametrize("shape,axis", [((4160, 8192), 0), ((8192, 4160), 1)])
def test_prox_long_chains_sampled(dev, shape, axis):
    """Chains long enough that the piece length hits its cap, 65 chain groups:
    sampled chains against the oracle (the whole grid is too large for it)."""
    from paper_1503_01563_amd import mc
    rng = np.random.default_rng(17 + axis)
    v = (rng.normal(size=shape) * 4).astype(np.float32)
    a = rng.uniform(0, 3, size=shape).astype(np.float32)
    if axis == 0:
        a[:, -1] = 0
    else:
        a[-1, :] = 0
    x = mc.tv_prox_chains(to_dev(v, dev), to_dev(a, dev), axis).cpu().numpy()
    nch = shape[axis]
    for c in list(rng.choice(nch, 12, replace=False)) + [0, nch - 1]:
        vc = v[c] if axis == 0 else v[:, c]
        ac = a[c] if axis == 0 else a[:, c]
        xc = x[c] if axis == 0 else x[:, c]
        xr, _ = oracle.tv1d(vc.astype(np.float64), ac[:-1].astype(np.float64))
        assert rel_linf(xc, xr) <= REL_TOL, c


@pytest.mark.parametrize("shape", [(64, 64), (37, 53), (1, 300), (300, 1), (9, 11, 13), (1, 1)])
def test_cut_energy_bit_exact(dev, shape):
    from paper_1503_01563_amd import mc
    for seed in range(3):
        w, a = gen.iid_grid(shape, 500 + seed)
        if seed == 2:
            w, a = gen.ellipse_grid(shape if len(shape) == 3 else shape, 900 + seed) \
                if min(shape) > 1 else (w, a)
        lab = (np.random.default_rng(seed).uniform(size=shape) < 0.5).astype(np.uint8)
        import torch
        e = mc.cut_energy(to_dev(w, dev), [to_dev(x, dev) for x in a], torch.from_numpy(lab).to(dev))
        assert e == oracle.cut_energy(w, a, lab)


@pytest.mark.parametrize("seed", list(range(1000, 1008)))
def test_solve_small_grid_exact(dev, seed):
    from paper_1503_01563_amd import mc
    w, a = gen.config_small(seed)
    e_star, mn, mx = oracle.mincut(w, a, "ek" if seed < 1002 else "dinic")
    res = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], max_iters=500, gap_tol=1e-3)
    assert res.converged and res.cert_gap < 1e-3
    assert res.energy == e_star
    lab = res.labels.cpu().numpy()
    assert oracle.cut_energy(w, a, lab) == e_star
    # every minimum cut lies between the minimal and the maximal optimal set
    assert np.all(lab >= mn) and np.all(lab <= mx)
    ro = oracle.dr_solve(w, a, max_iters=500, gap_tol=1e-3)
    print("seed %d: gpu iters %d, oracle iters %d" % (seed, res.iters, ro["iters"]))


@pytest.mark.parametrize("shape,variant", [((37, 53), 1), ((37, 53), 2), ((6, 17, 23), 2),
                                           ((1, 41), 1), ((41, 1), 1), ((5, 1, 7), 2)])
@pytest.mark.parametrize("iters", [1, 3, 20])
def test_dr_iterates_match_oracle(dev, shape, variant, iters):
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid(shape, 77 + iters)
    res = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], max_iters=iters, gap_tol=0.0,
                      variant=variant, return_z=True)
    assert res.iters == iters
    ro = oracle.dr_solve(w, a, variant=0 if variant == 1 else 1, max_iters=iters, gap_tol=0,
                         return_z=True)
    assert rel_linf(res.x.cpu().numpy(), ro["x"]) <= REL_TOL
    assert rel_linf(res.z.cpu().numpy(), ro["z"]) <= REL_TOL


@pytest.mark.parametrize("shape,variant", [((24, 31), 1), ((24, 31), 2), ((6, 9, 11), 2)])
def test_tv_solution_matches_oracle(dev, shape, variant):
    from paper_1503_01563_amd import mc
    # Reference: FP64 run stopped at TV gap 2e-8; by 1-strong convexity of
    # the TV objective its distance to x* is at most sqrt(2 * 2e-8) = 2e-4,
    # far below 1e-4 * |x*|_inf for these data (|x*| ~ 20).
    w, a = gen.iid_grid(shape, 5)
    ro = oracle.dr_solve(w, a, variant=0 if variant == 1 else 1, max_iters=6000, gap_tol=0,
                         tv_tol=2e-8)
    assert ro["tv_gap"] < 2e-8
    res = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], max_iters=ro["iters"],
                      gap_tol=0.0, variant=variant)
    assert rel_linf(res.x.cpu().numpy(), ro["x"]) <= REL_TOL


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 2, 4), (4, 4), (1, 16), (16, 1)])
def test_solve_tiny_against_bruteforce(dev, shape):
    from paper_1503_01563_amd import mc
    for seed in range(4):
        w, a = gen.iid_grid(shape, 40 + seed)
        if seed % 2:
            w = (np.round(w / 3.0 * 256) / 256).astype(np.float32)
        if np.prod(shape) <= 20:
            e_star, _, _, _ = oracle.bruteforce(w, a)
        else:
            e_star, _, _ = oracle.mincut(w, a, "ek")
        res = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], max_iters=2000)
        assert res.converged and res.energy == e_star


def test_degenerate_inputs(dev):
    import torch
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid((20, 30), 3)
    z = [np.zeros_like(x) for x in a]
    res = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in z], max_iters=10)
    assert res.converged and res.energy == float(np.minimum(w, 0).sum())
    np.testing.assert_allclose(res.x.cpu().numpy(), -w, atol=1e-5)
    res = mc.tv_solve(to_dev(np.zeros_like(w), dev), [to_dev(x, dev) for x in a], max_iters=10)
    assert res.converged and res.energy == 0.0
    c = np.full_like(w, -3.0)
    res = mc.tv_solve(to_dev(c, dev), [to_dev(x, dev) for x in a], max_iters=50)
    assert res.converged and res.energy == float(c.sum())
    assert int(res.labels.sum()) == c.size
    w1 = np.array([[5.0]], np.float32)
    res = mc.tv_solve(to_dev(w1, dev), [to_dev(np.zeros_like(w1), dev)] * 2, max_iters=5)
    assert res.converged and res.energy == 0.0


def test_validation_errors(dev):
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid((8, 9), 1)
    bad = [x.copy() for x in a]
    bad[0][2, 3] = -1.0
    with pytest.raises(mc.McError) as e:
        mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in bad], validate=True)
    assert e.value.code == -2
    wn = w.copy()
    wn[1, 1] = np.nan
    with pytest.raises(mc.McError) as e:
        mc.tv_solve(to_dev(wn, dev), [to_dev(x, dev) for x in a], validate=True)
    assert e.value.code == -3
    res = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], max_iters=1, gap_tol=0.0)
    assert res.status == 1 and res.iters == 1
    with pytest.raises(mc.McError):
        mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], variant=1, max_iters=0)


@pytest.mark.parametrize("shape", [(40, 57), (9, 20, 23)])
def test_debug_flag_checks_and_changes_nothing(dev, shape):
    """MC_DEBUG on valid input: the same iterates and results as without it
    (its checks only read).  With a NaN unary (not validated) it stops at
    iteration 1 with MC_ERR_NUMERIC naming the iteration, where the plain
    solve only notices at its first certificate."""
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid(shape, 77)
    tw, ta = to_dev(w, dev), [to_dev(x, dev) for x in a]
    ref = mc.tv_solve(tw, ta, max_iters=400, check_every=3, return_z=True)
    dbg = mc.tv_solve(tw, ta, max_iters=400, check_every=3, return_z=True, debug=True)
    assert dbg.converged and dbg.iters == ref.iters and dbg.energy == ref.energy
    assert bool((dbg.z == ref.z).all()) and bool((dbg.labels == ref.labels).all())
    wn = w.copy()
    wn.flat[w.size // 2] = np.nan
    with pytest.raises(mc.McError) as e:
        mc.tv_solve(to_dev(wn, dev), ta, max_iters=50, check_every=10, debug=True)
    assert e.value.code == -6 and "after iteration 1" in str(e.value)
    with pytest.raises(mc.McError) as e:
        mc.tv_solve(to_dev(wn, dev), ta, max_iters=50, check_every=10)
    assert e.value.code == -6


@pytest.mark.parametrize("shape,variant", [((33, 47), 1), ((20, 30), 2), ((6, 17, 19), 2)])
def test_fp64_state_iterates_match_oracle(dev, shape, variant):
    """MC_FP64_STATE runs the same splitting in FP64: after 150 iterations its
    state (rounded to FP32 on output) equals the FP64 oracle's to the FP32
    rounding of the output; the FP32 path's distance is printed beside it."""
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid(shape, 11)
    tw, ta = to_dev(w, dev), [to_dev(x, dev) for x in a]
    iters = 150
    kw = dict(max_iters=iters, check_every=iters, gap_tol=0.0, variant=variant, return_z=True)
    r64 = mc.tv_solve(tw, ta, fp64_state=True, **kw)
    r32 = mc.tv_solve(tw, ta, **kw)
    ro = oracle.dr_solve(w, a, variant=variant - 1, max_iters=iters, gap_tol=0, return_z=True)
    zo = ro["z"]
    e64 = rel_linf(r64.z.cpu().numpy(), zo)
    e32 = rel_linf(r32.z.cpu().numpy(), zo)
    print("%s variant %d: FP64 state %.2e, FP32 state %.2e from the oracle after %d iterations"
          % (shape, variant, e64, e32, iters))
    assert r64.iters == iters
    assert e64 <= 2e-7


@pytest.mark.parametrize("shape", [(40, 50), (8, 12, 14)])
def test_fp64_state_exact_cut(dev, shape):
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid(shape, 12)
    res = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], max_iters=3000, check_every=2,
                      fp64_state=True)
    assert res.converged and res.energy == oracle.mincut(w, a, "dinic")[0]


def test_fp64_state_rejections(dev):
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid((9, 11), 13)
    tw, ta = to_dev(w, dev), [to_dev(x, dev) for x in a]
    for kw in (dict(variant=mc.VARIANT_BCD), dict(variant=mc.VARIANT_FISTA)):
        with pytest.raises(mc.McError) as e:
            mc.tv_solve(tw, ta, fp64_state=True, **kw)
        assert e.value.code == -1


def test_image2d_full_size_exact(dev):
    """Segmentation-shaped 1024x1024 grid: exact energy against max-flow."""
    from paper_1503_01563_amd import mc
    w, a = gen.config_image2d(2000)
    e_star, mn, mx = oracle.mincut(w, a, "dinic")
    res = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], max_iters=2000, gap_tol=1e-3)
    print("1024^2: iters %d cert %.3g ms %.2f" % (res.iters, res.cert_gap, res.ms))
    assert res.converged and res.energy == e_star
    lab = res.labels.cpu().numpy()
    assert oracle.cut_energy(w, a, lab) == e_star
    assert np.all(lab >= mn) and np.all(lab <= mx)


def test_volume3d_full_size_exact(dev):
    """256x256x128 6-connected volume: exact energy against max-flow."""
    from paper_1503_01563_amd import mc
    w, a = gen.config_volume3d(3000)
    e_star, mn, mx = oracle.mincut(w, a, "dinic")
    res = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], max_iters=3000, gap_tol=1e-3,
                      check_every=5)
    print("3D: iters %d cert %.3g ms %.2f" % (res.iters, res.cert_gap, res.ms))
    assert res.converged and res.energy == e_star
    lab = res.labels.cpu().numpy()
    assert oracle.cut_energy(w, a, lab) == e_star


def test_oversize_grid_rejected(dev):
    """n above 2^31 - 2^24 is refused before any device work (int grid-stride
    indexing keeps 2^24 of headroom)."""
    import ctypes
    from paper_1503_01563_amd import mc
    lib = mc.load_library()
    ctx = mc.context(0)
    g = mc._grid((46341, 46341))  # 2,147,488,281 nodes
    st = mc.Stats()
    o = mc.make_opts()
    rc = lib.mc_tv_solve(ctx, ctypes.byref(g), None, None, None, None, None, None, ctypes.byref(st),
                         ctypes.byref(o), None)
    assert rc == -1 and b"nodes" in lib.mc_last_error()
    g = mc._grid((32768, 65024))  # 2^31 - 2^24 nodes: passes the size check, fails on the null arrays
    rc = lib.mc_tv_solve(ctx, ctypes.byref(g), None, None, None, None, None, None, ctypes.byref(st),
                         ctypes.byref(o), None)
    assert rc == -1 and b"null" in lib.mc_last_error()


@pytest.mark.parametrize("shape", [(48, 64), (6, 20, 24)])
def test_positive_homogeneity_is_exact(dev, shape):
    """Scaling w and a by 2 scales every floating-point value of the solve by 2
    exactly, so the primal doubles bit for bit and labels and iterations agree
    (x*(t w, t a) = t x*(w, a))."""
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid(shape, 8100)
    r1 = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], max_iters=4000, check_every=2)
    r2 = mc.tv_solve(to_dev(2 * w, dev), [to_dev(2 * x, dev) for x in a], max_iters=4000, check_every=2,
                     tau0=2e-3, gap_tol=2e-3)  # the thresholds and the certificate scale too
    assert r1.converged and r2.converged and r1.iters == r2.iters
    assert np.array_equal((2 * r1.x).cpu().numpy(), r2.x.cpu().numpy())
    assert np.array_equal(r1.labels.cpu().numpy(), r2.labels.cpu().numpy())
    assert r2.energy == 2 * r1.energy


def test_transposed_grid_gives_the_same_cut_energy(dev):
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid((40, 56), 8200)
    r = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], max_iters=2000, check_every=2)
    wt = np.ascontiguousarray(w.T)
    at = [np.ascontiguousarray(a[1].T), np.ascontiguousarray(a[0].T)]
    rt = mc.tv_solve(to_dev(wt, dev), [to_dev(x, dev) for x in at], max_iters=2000, check_every=2)
    assert r.converged and rt.converged
    assert r.energy == rt.energy == oracle.mincut(w, a, "dinic")[0]


@pytest.mark.parametrize("workload,iters", [("image2d", 2), ("image2d", 9), ("volume3d", 2)])
def test_full_size_iterates_match_reference(dev, workload, iters):
    """The splitting iterates at the full workload sizes, in the launch
    configuration the benchmark times (1024^2: one work item per SIMD, latency
    mode; the volume: the x, y and z families in one launch), against the FP64 reference run
    for the same number of iterations: every entry of the primal and of the
    state within 1e-4 relative to the largest magnitude."""
    from paper_1503_01563_amd import mc
    if workload == "image2d":
        w, a = gen.config_image2d(2000)
    else:
        w, a = gen.config_volume3d(3000)
    res = mc.tv_solve(to_dev(w, dev), [to_dev(x, dev) for x in a], max_iters=iters, gap_tol=0.0,
                      return_z=True, check_every=iters)
    assert res.iters == iters
    ro = oracle.dr_solve(w, a, max_iters=iters, gap_tol=0, return_z=True)
    assert rel_linf(res.x.cpu().numpy(), ro["x"]) <= REL_TOL
    assert rel_linf(res.z.cpu().numpy(), ro["z"]) <= REL_TOL

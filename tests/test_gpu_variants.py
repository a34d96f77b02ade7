"""GPU parity of the other outer iterations (cyclic projections / BCD,
alternating projections, FISTA) against their FP64 reference, exact cuts
against max-flow, and an iteration-count comparison with the splitting."""
import numpy as np
import pytest

import oracle
from oracle import variants as V
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


def T(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


def variants():
    from paper_1503_01563_amd import mc
    return {"bcd": (mc.VARIANT_BCD, V.bcd_solve), "ap": (mc.VARIANT_AP, V.ap_solve),
            "fista": (mc.VARIANT_FISTA, V.fista_solve)}


@pytest.mark.parametrize("name", ["bcd", "ap", "fista"])
@pytest.mark.parametrize("iters", [1, 3, 10])
@pytest.mark.parametrize("shape", [(20, 26), (5, 6, 7)])
def test_iterates_match_reference(dev, name, iters, shape):
    from paper_1503_01563_amd import mc
    var, ref_fn = variants()[name]
    w, a = gen.iid_grid(shape, 31)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=iters, check_every=iters, gap_tol=0.0,
                      variant=var)
    ref = ref_fn(w, a, max_iters=iters, gap_tol=0.0, check_every=iters)
    x = res.x.cpu().numpy()
    scale = max(1.0, np.abs(ref["x"]).max())
    assert np.abs(x - ref["x"]).max() / scale <= REL_TOL, (name, iters)


@pytest.mark.parametrize("name", ["bcd", "ap", "fista"])
@pytest.mark.parametrize("shape,seed", [((64, 64), 1000), ((33, 47), 32), ((8, 9, 10), 33)])
def test_exact_against_maxflow(dev, name, shape, seed):
    from paper_1503_01563_amd import mc
    var, _ = variants()[name]
    w, a = gen.iid_grid(shape, seed)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=6000, check_every=2, gap_tol=1e-3, variant=var)
    assert res.converged, (name, res.cert_gap)
    assert res.energy == oracle.mincut(w, a, "dinic")[0]


def test_iteration_comparison(dev):
    """Iterations and time to the exact cut for every outer iteration, on an
    integer grid and an image, also with all edge weights scaled by 0.1."""
    from paper_1503_01563_amd import mc
    names = [("dr", mc.VARIANT_AUTO), ("bcd", mc.VARIANT_BCD), ("ap", mc.VARIANT_AP), ("fista", mc.VARIANT_FISTA)]
    cases = [("iid 64x64", gen.iid_grid((64, 64), 1000)), ("image 512x512", gen.config_image2d(2000, (512, 512)))]
    cases += [(name + " a*0.1", (w, [x * np.float32(0.1) for x in a])) for name, (w, a) in cases[:1]]
    for cname, (w, a) in cases:
        e_star = oracle.mincut(w, a, "dinic")[0] if w.size <= 4096 else None
        line = []
        for vname, var in names:
            res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=20000, check_every=2, gap_tol=1e-3,
                              variant=var)
            assert res.converged, (cname, vname)
            if e_star is not None:
                assert res.energy == e_star, (cname, vname)
            line.append("%s %d it %.1f ms" % (vname, res.iters, res.ms))
        print("%s: %s" % (cname, "; ".join(line)))


@pytest.mark.parametrize("case", ["image2d", "iid2d", "iid3d", "ellipsoid3d"])
def test_bcd_then_splitting_is_exact(dev, case):
    """MC_VARIANT_BCD_DR: BCD for 16 iterations, then the splitting from its
    dual blocks; exact whichever phase certifies."""
    from paper_1503_01563_amd import mc
    if case == "image2d":
        w, a = gen.config_image2d(2003, (192, 256))
    elif case == "iid2d":
        w, a = gen.iid_grid((96, 112), 4400)
    elif case == "iid3d":
        w, a = gen.iid_grid((10, 18, 22), 12)
    else:
        w, a = gen.ellipse_grid((16, 32, 32), 3100, lam=1.5)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=20000, check_every=2,
                      variant=mc.VARIANT_BCD_DR)
    assert res.converged, case
    assert res.energy == oracle.mincut(w, a, "dinic")[0], case
    print("bcd+dr %s: %d iterations" % (case, res.iters))


def test_bcd_then_splitting_rejects_states(dev):
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid((8, 9), 2)
    with pytest.raises(mc.McError):
        mc.tv_solve(T(w, dev), [T(x, dev) for x in a], variant=mc.VARIANT_BCD_DR, return_z=True)

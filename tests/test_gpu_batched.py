"""GPU parity of the batched solver (many uneven 2D grids at once) against the
CPU oracle's exact max-flow energies and against single-grid solves."""
import numpy as np
import pytest

import oracle
from paper_1503_01563_amd import gen

pytestmark = pytest.mark.gpu


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


def batch_inputs(shapes, seed0, dev, dyadic=False):
    ws, As, host = [], [], []
    for k, sh in enumerate(shapes):
        w, a = gen.iid_grid(sh, seed0 + k)
        if dyadic:
            w = (np.round(w / 3.0 * 256) / 256).astype(np.float32)
        host.append((w, a))
        ws.append(to_dev(w, dev))
        As.append([to_dev(a[0], dev), to_dev(a[1], dev)])
    return ws, As, host


@pytest.mark.parametrize("check_every", [1, 2, 4])
def test_batched_small_uneven_exact(dev, check_every):
    from paper_1503_01563_amd import mc
    rng = np.random.default_rng(check_every)
    shapes = [tuple(int(v) for v in rng.integers(5, 90, size=2)) for _ in range(9)]
    shapes += [(1, 37), (41, 1), (1, 1), (2, 2)]
    ws, As, host = batch_inputs(shapes, 700, dev, dyadic=check_every == 2)
    res = mc.tv_solve_batched(ws, As, max_iters=3000, check_every=check_every, return_x=True)
    assert res.converged, res.status
    for k, (w, a) in enumerate(host):
        e_star, mn, mx = oracle.mincut(w, a, "dinic")
        assert res.energy[k] == e_star, (k, shapes[k])
        lab = res.labels[k].cpu().numpy()
        assert oracle.cut_energy(w, a, lab) == e_star
        assert res.ms[k] > 0


def test_batched_matches_single_solves(dev):
    from paper_1503_01563_amd import mc
    shapes = [(64, 64), (33, 70), (90, 17), (128, 40)]
    ws, As, host = batch_inputs(shapes, 1000, dev)
    res = mc.tv_solve_batched(ws, As, max_iters=2000, check_every=2)
    for k in range(len(shapes)):
        single = mc.tv_solve(ws[k], As[k], max_iters=2000, check_every=2)
        assert single.converged
        # same iteration sequence: the same certified iteration and energy
        assert res.energy[k] == single.energy
        assert res.iters[k] == single.iters


def test_batched_repeat_uses_tuned_config(dev):
    from paper_1503_01563_amd import mc
    shapes = [(150, 200), (130, 260)]
    ws, As, host = batch_inputs(shapes, 2000, dev)
    r1 = mc.tv_solve_batched(ws, As, max_iters=2000)
    r2 = mc.tv_solve_batched(ws, As, max_iters=2000)
    assert r1.items == r2.items and r1.items > 0
    assert r1.energy == r2.energy and r1.iters == r2.iters
    for k in range(len(shapes)):
        assert bool((r1.labels[k] == r2.labels[k]).all())
    r3 = mc.tv_solve_batched(ws, As, max_iters=2000, items=2048)
    assert r3.items == 2048 and r3.energy == r1.energy


def test_batched_config_64_uneven_grids(dev):
    """64 grids with H, W uniform in [128, 1024]: every energy exact against max-flow."""
    from paper_1503_01563_amd import mc
    grids = gen.config_batch(4000)
    ws = [to_dev(w, dev) for w, _ in grids]
    As = [[to_dev(a[0], dev), to_dev(a[1], dev)] for _, a in grids]
    runs = {}
    for ce in (2, 8):  # a check every 2 iterations, and the default cadence
        res = mc.tv_solve_batched(ws, As, max_iters=3000, check_every=ce)
        ms = np.array(res.ms)
        print("batched 64, check every %d: items %d, p50 %.2f ms, p99 %.2f ms, max iters %d"
              % (ce, res.items, np.percentile(ms, 50), np.percentile(ms, 99), max(res.iters)))
        assert res.converged
        runs[ce] = res
    for k, (w, a) in enumerate(grids):
        e_star, _, _ = oracle.mincut(w, a, "dinic")
        for ce, res in runs.items():
            assert res.energy[k] == e_star, (k, ce)


@pytest.mark.parametrize("max_iters,check_every", [(1, 4), (2, 2), (7, 4), (12, 4)])
def test_batched_stops_at_max_iters(dev, max_iters, check_every):
    """No grid runs past max_iters (the iterations left below a whole replay
    period run outside the graph), every grid ends on a check, and the state
    equals the single-grid solver's after as many iterations."""
    from paper_1503_01563_amd import mc
    shapes = [(37, 53), (64, 20), (1, 30), (9, 9)]
    ws, As, host = batch_inputs(shapes, 3100, dev)
    res = mc.tv_solve_batched(ws, As, max_iters=max_iters, check_every=check_every, gap_tol=0.0,
                              return_x=True, return_z=True)
    assert res.iters == [max_iters] * len(shapes)
    for k in range(len(shapes)):
        single = mc.tv_solve(ws[k], As[k], max_iters=max_iters, check_every=max_iters, gap_tol=0.0,
                             return_x=True, return_z=True)
        assert single.iters == max_iters
        z_b = res.z[k].cpu().numpy()
        z_s = single.z.view(shapes[k]).cpu().numpy()
        assert np.array_equal(z_b, z_s), (k, float(np.abs(z_b - z_s).max()))
        assert np.allclose(res.x[k].cpu().numpy(), single.x.view(shapes[k]).cpu().numpy(), rtol=1e-6, atol=1e-6)
        assert res.energy[k] == single.energy


def test_batched_persistent_matches_graph_replay(dev):
    """One persistent launch per check period (device work queue, device-wide
    barriers) gives the same iterates as the replayed graph of per-phase
    launches: the same certified iterations, energies, labels and states."""
    from paper_1503_01563_amd import mc
    rng = np.random.default_rng(5)
    shapes = [tuple(int(v) for v in rng.integers(20, 300, size=2)) for _ in range(12)] + [(1, 50), (3, 3)]
    ws, As, host = batch_inputs(shapes, 4100, dev)
    ref = mc.tv_solve_batched(ws, As, max_iters=3000, check_every=4, return_z=True)
    per = mc.tv_solve_batched(ws, As, max_iters=3000, check_every=4, return_z=True, persistent=True)
    assert ref.converged and per.converged
    assert per.iters == ref.iters and per.energy == ref.energy
    for k, (w, a) in enumerate(host):
        assert bool((per.labels[k] == ref.labels[k]).all()), k
        assert bool((per.z[k] == ref.z[k]).all()), k
    for k in (0, 1, len(shapes) - 1):
        w, a = host[k]
        assert per.energy[k] == oracle.mincut(w, a, "dinic")[0]


@pytest.mark.parametrize("max_iters", [3, 10])
def test_batched_persistent_stops_at_max_iters(dev, max_iters):
    from paper_1503_01563_amd import mc
    shapes = [(37, 53), (64, 20), (9, 9)]
    ws, As, host = batch_inputs(shapes, 3100, dev)
    ref = mc.tv_solve_batched(ws, As, max_iters=max_iters, check_every=4, gap_tol=0.0, return_z=True)
    per = mc.tv_solve_batched(ws, As, max_iters=max_iters, check_every=4, gap_tol=0.0, return_z=True,
                              persistent=True)
    assert per.iters == [max_iters] * len(shapes) == ref.iters
    for k in range(len(shapes)):
        assert bool((per.z[k] == ref.z[k]).all()), k

"""Batched ensembles of uneven boxes and hipGraph replay (GPU).

A box advanced inside an ensemble runs the same kernels as its single-box
plan, so the states must agree bitwise; tile shapes chosen by the autotuner
and graph replay must not change any bit either."""
import math
import os
import tempfile

import numpy as np
import pytest

from conftest import rel_max
from paper_2211_16718_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2211_16718_amd.api import Ensemble, Plan  # noqa: E402


def case(msg):
    print(f"[case] {msg}", flush=True)


def box_inputs(specs):
    """specs: list of (n, mt, re, seed) -> primitives and box dicts with a CFL dt."""
    import oracle

    out = []
    for n, mt, re, seed in specs:
        rho, vel, p = I.hit_primitives(n, seed, mt)
        mu = 1.0 / re
        smax = oracle.diag(oracle.init_state(rho, vel, p), oracle.make_phys(mu_eff=mu))[7]
        dt = I.dt_from_speed(smax, n)
        out.append(dict(shape=(n, n, n), mu_eff=mu, dt=dt, prim=(rho, vel, p)))
    return out


def single_run(b, nsteps, stream, graph=False, tiles=None):
    plan = Plan(b["shape"], mu_eff=b["mu_eff"], stream=stream)
    if tiles:
        plan.set_tiles(*tiles)
    if graph:
        plan.set_graph(True)
    with torch.cuda.stream(stream):
        u = plan.init_state(*b["prim"])
        d = plan.rk4(u, b["dt"], nsteps)
    stream.synchronize()
    return u, d


def make_ensemble(boxes, stream):
    ens = Ensemble([{k: v for k, v in b.items() if k != "prim"} for b in boxes], stream=stream)
    for i, b in enumerate(boxes):
        plan = Plan(b["shape"], mu_eff=b["mu_eff"], stream=stream)
        with torch.cuda.stream(stream):
            plan.init_state(*b["prim"], out=ens.state(i))
    stream.synchronize()
    return ens


SPECS = [(32, 0.3, 100.0, 0), (48, 0.15, 700.0, 1), (16, 0.45, 250.0, 2), (24, 0.2, 400.0, 3), (32, 0.1, 800.0, 4),
         (20, 0.35, 150.0, 5)]


def test_ensemble_boxes_equal_single_box_runs_bitwise():
    case("ensemble vs single-box, eager and graph")
    stream = torch.cuda.Stream()
    boxes = box_inputs(SPECS)
    ens = make_ensemble(boxes, stream)
    with torch.cuda.stream(stream):
        diag = ens.run(3, graph=True)
    stream.synchronize()
    for i, b in enumerate(boxes):
        u, d = single_run(b, 3, stream)
        assert torch.equal(ens.state(i), u), f"box {i}"
        assert torch.equal(diag[i], d), f"diag box {i}"


def test_autotuned_tiles_do_not_change_results():
    case("autotune")
    stream = torch.cuda.Stream()
    boxes = box_inputs(SPECS[:4])
    ens = make_ensemble(boxes, stream)
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "tiles.json")
        ens.autotune(path)
        assert os.path.exists(path)
        txt = open(path).read()
        assert "seg" in txt and "block" in txt
        tiles = [ens.get_tiles(i) for i in range(len(boxes))]
        launch = [ens.get_launch(i) for i in range(len(boxes))]
        print("autotuned tiles", tiles, "launch shapes", launch)
        assert "rows" in txt and "grid" in txt
        # a second ensemble reads the cache instead of timing again
        ens2 = make_ensemble(boxes, stream)
        ens2.autotune(path)
        assert [ens2.get_tiles(i) for i in range(len(boxes))] == tiles
        assert [ens2.get_launch(i) for i in range(len(boxes))] == launch
    with torch.cuda.stream(stream):
        ens.run(2, graph=False)
    stream.synchronize()
    for i, b in enumerate(boxes):
        u, _ = single_run(b, 2, stream)
        assert torch.equal(ens.state(i), u), f"box {i}"


def test_persistent_grids_and_rows_do_not_change_results():
    """Persistent launches (fewer blocks than virtual blocks, each looping over several;
    grids below and above the 8 XCDs) and rows-per-block counts other than the default
    power of two give bitwise the single-box results."""
    case("persistent grids and rows per block")
    stream = torch.cuda.Stream()
    boxes = box_inputs(SPECS)
    ref = [single_run(b, 2, stream) for b in boxes]
    for rows, gs, gt in ((0, 5, 3), (0, 37, 1), (3, 600, 90), (5, 1, 700)):
        ens = make_ensemble(boxes, stream)
        for i, b in enumerate(boxes):
            nx = b["shape"][2]
            r = rows if rows and rows * nx <= 1024 and 14 * rows * nx * 8 <= 65536 else 0
            ens.set_launch(i, r, gs, gt)
        assert ens.get_launch(0)[1:] == (gs, gt)
        with torch.cuda.stream(stream):
            d = ens.run(2, graph=False)
        stream.synchronize()
        for i in range(len(boxes)):
            assert torch.equal(ens.state(i), ref[i][0]), (rows, gs, gt, i)
            assert torch.equal(d[i], ref[i][1]), (rows, gs, gt, i)
    from paper_2211_16718_amd._lib import CnsError

    with pytest.raises(CnsError):
        ens.set_launch(0, 1000, 0, 0)  # 1000 rows of 32 points do not fit


def test_graph_replays_match_eager_runs():
    # replay the captured graph several times with eager work and syncs in
    # between; every replay must equal the eager result.  Calls with a new
    # diagnostics buffer, another state tensor or another dt replay the same capture.
    case("graph replays")
    stream = torch.cuda.Stream()
    b = box_inputs([(24, 0.3, 200.0, 7)])[0]
    plan_e = Plan(b["shape"], mu_eff=b["mu_eff"], stream=stream)
    plan_g = Plan(b["shape"], mu_eff=b["mu_eff"], stream=stream)
    plan_g.set_graph(True)
    with torch.cuda.stream(stream):
        ue = plan_e.init_state(*b["prim"])
        ug = plan_g.init_state(*b["prim"])
    for rep in range(4):
        dt = b["dt"] * (1.0 if rep < 2 else 0.75)
        with torch.cuda.stream(stream):
            de = plan_e.rk4(ue, dt, 2)
            dg = plan_g.rk4(ug, dt, 2)
            scratch = torch.randn(1000, device="cuda") * 2  # eager work between replays
        stream.synchronize()
        assert torch.equal(ue, ug), f"replay {rep}"
        assert torch.equal(de, dg)
        del scratch
    # another state tensor: the same capture, the new tensor advanced
    with torch.cuda.stream(stream):
        ug2 = ug.clone()
        ue2 = ue.clone()
        plan_g.rk4(ug2, b["dt"], 2)
        plan_e.rk4(ue2, b["dt"], 2)
    stream.synchronize()
    assert torch.equal(ug2, ue2) and not torch.equal(ug2, ug)
    assert plan_g.graph_captures() == 1
    # a different step count or no diagnostics needs a capture of its own
    with torch.cuda.stream(stream):
        plan_g.rk4(ug, b["dt"], 3)
        plan_g.rk4(ug, b["dt"], 3, diag=False)
    stream.synchronize()
    assert plan_g.graph_captures() == 3
    assert plan_e.graph_captures() == 0


def test_ensemble_graph_is_captured_once():
    case("ensemble graph captured once")
    stream = torch.cuda.Stream()
    boxes = box_inputs(SPECS[:3])
    ens_g = make_ensemble(boxes, stream)
    ens_e = make_ensemble(boxes, stream)
    for rep in range(3):
        with torch.cuda.stream(stream):
            dg = ens_g.run(2, graph=True)
            de = ens_e.run(2, graph=False)
        stream.synchronize()
        assert torch.equal(ens_g.u, ens_e.u), f"run {rep}"
        assert torch.equal(dg, de)
    assert ens_g.graph_captures() == 1 and ens_e.graph_captures() == 0


def test_ensemble_box_matches_oracle():
    import oracle

    case("ensemble box vs oracle")
    stream = torch.cuda.Stream()
    boxes = box_inputs(SPECS[:3])
    ens = make_ensemble(boxes, stream)
    with torch.cuda.stream(stream):
        ens.run(2, graph=True)
    stream.synchronize()
    for i, b in enumerate(boxes):
        ph = oracle.make_phys(mu_eff=b["mu_eff"])
        uf, _ = oracle.rk4(oracle.init_state(*b["prim"]), b["dt"], 2, ph, with_diag=False)
        assert rel_max(ens.state(i).cpu().numpy(), uf) <= 1e-12, f"box {i}"


def test_full_ensemble_workload():
    # 64 boxes, sizes drawn from {32, 48, 64, 96}, Mt in [0.1, 0.5], Re in [100, 800],
    # tiles from the autotuner: the first 64^3 and 96^3 boxes against the oracle over
    # 2 RK4 steps, then 50 RK4 steps in one captured graph with every box bitwise equal
    # to its own single-box run (default tiles, eager launches)
    import oracle

    case("64-box ensemble: autotune, 2 steps vs oracle, 50 steps vs single-box runs")
    stream = torch.cuda.Stream()
    boxes = []
    for i in range(64):
        box, rho, vel, p = I.ensemble_box_primitives(i)
        mu = 1.0 / box.re
        smax = oracle.diag(oracle.init_state(rho, vel, p), oracle.make_phys(mu_eff=mu))[7]
        boxes.append(dict(shape=(box.n,) * 3, mu_eff=mu, dt=I.dt_from_speed(smax, box.n), prim=(rho, vel, p)))
    ens = make_ensemble(boxes, stream)
    ens.autotune(None)
    print("tiles by size:", {b["shape"][0]: ens.get_tiles(i) for i, b in enumerate(boxes)}, flush=True)
    u0 = ens.u.clone()
    with torch.cuda.stream(stream):
        ens.run(2, graph=True)
    stream.synchronize()
    for want in (64, 96):
        i = next(i for i, b in enumerate(boxes) if b["shape"][0] == want)
        b = boxes[i]
        case(f"  box {i} ({want}^3) vs oracle, 2 steps")
        uf, _ = oracle.rk4(oracle.init_state(*b["prim"]), b["dt"], 2, oracle.make_phys(mu_eff=b["mu_eff"]),
                           with_diag=False)
        err = rel_max(ens.state(i).cpu().numpy(), uf)
        print(f"  box {i}: rel err {err:.3e}", flush=True)
        assert err <= 1e-12, f"box {i}"
    ens.u.copy_(u0)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        diag = ens.run(50, graph=True)
    stream.synchronize()
    d = diag.cpu().numpy()
    assert np.all(d[:, :, 8] == 0)
    assert np.all(d[:, -1, 0] < d[:, 0, 0])  # kinetic energy decays in every box
    for i, b in enumerate(boxes):
        u, dsingle = single_run(b, 50, stream)
        assert torch.equal(ens.state(i), u), f"box {i}"
        assert torch.equal(diag[i], dsingle), f"diag box {i}"
    print("all 64 boxes bitwise equal to their single-box runs", flush=True)

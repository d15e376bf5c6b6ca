"""Batched path: meshes of mixed size and order advanced together must give,
mesh by mesh, exactly the single-mesh result (same kernels, deterministic),
with every schedule option, eagerly and from graph replays."""
import numpy as np
import pytest

from paper_2105_02127_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(torch, specs):
    from paper_2105_02127_amd import teno
    sv, U = [], []
    for n, p, seed in specs:
        m = inputs.jittered_periodic_mesh(n, seed)
        lm = teno.Mesh(m.xy, m.tri).setup(order=p, fallback=1)
        s = teno.Solver(lm)
        sv.append(s)
        U.append(torch.as_tensor(inputs.random_lines(m)[lm.perm], device="cuda"))
    return sv, U


SPECS = [(12, 3, 501), (17, 6, 502), (9, 4, 503), (21, 5, 504), (13, 6, 505), (10, 3, 506)]


@pytest.mark.parametrize("tuning", [
    dict(order_mode=0, waves_per_cu=4, item_order=0, use_graph=0),
    dict(order_mode=1, waves_per_cu=8, item_order=1, use_graph=0),
    dict(order_mode=0, waves_per_cu=16, item_order=1, use_graph=1),
    dict(order_mode=1, waves_per_cu=1, item_order=0, use_graph=1),
    dict(order_mode=1, waves_per_cu=0, item_order=1, use_graph=1),
])
def test_batch_step_equals_single_mesh_steps(torch_cuda, tuning):
    torch = torch_cuda
    from paper_2105_02127_amd.batch import Batch
    print(f"[batch] tuning {tuning}", flush=True)
    sv, U = _setup(torch, SPECS)
    b = Batch(sv)
    b.set_tuning(**tuning)
    dt = b.max_dt(U, 0.4)
    ref_dt = torch.cat([s.max_dt(u, 0.4) for s, u in zip(sv, U)])
    torch.cuda.synchronize()
    assert torch.equal(dt, ref_dt)
    ref = [u.clone() for u in U]
    for s, u, d in zip(sv, ref, ref_dt):
        s.rk_step(u, d.reshape(1).contiguous())
    work = [u.clone() for u in U]
    b.rk_step(work, dt)
    torch.cuda.synchronize()
    for k, (w, r) in enumerate(zip(work, ref)):
        assert torch.equal(w, r), f"mesh {k} differs"


def test_graph_replays_match_eager(torch_cuda):
    torch = torch_cuda
    from paper_2105_02127_amd.batch import Batch
    sv, U = _setup(torch, SPECS[:4])
    b = Batch(sv)
    dt = b.max_dt(U, 0.4)
    eager = [u.clone() for u in U]
    b.set_tuning(use_graph=0)
    for _ in range(3):
        b.rk_step(eager, dt)
    b.set_tuning(use_graph=1)
    graph = [u.clone() for u in U]
    for r in range(3):
        b.rk_step(graph, dt)                 # replays after the first capture
        torch.cuda.synchronize()
        _ = [g.sum().item() for g in graph]  # eager work between replays
    for g, e in zip(graph, eager):
        assert torch.equal(g, e)


def test_autotune_picks_a_valid_schedule(torch_cuda, tmp_path):
    torch = torch_cuda
    from paper_2105_02127_amd.batch import Batch, autotune, CANDIDATES
    sv, U = _setup(torch, SPECS[:3])
    b = Batch(sv)
    dt = b.max_dt(U, 0.4)
    cache = str(tmp_path / "tune.json")
    best, timings = autotune(b, U, dt, steps=2, cache=cache)
    assert best in CANDIDATES and len(timings) == len(CANDIDATES)
    best2, t2 = autotune(b, U, dt, cache=cache)      # served from the cache
    assert best2 == best and t2 == {}


def test_cweno_meshes_are_not_batched(torch_cuda):
    from paper_2105_02127_amd import teno
    from paper_2105_02127_amd.batch import Batch
    m = inputs.jittered_periodic_mesh(12, 507)
    s = teno.Solver(teno.Mesh(m.xy, m.tri).setup(order=4, variant=2))
    with pytest.raises(teno.TenoError):
        Batch([s])


def test_characteristic_meshes_are_not_batched(torch_cuda):
    from paper_2105_02127_amd import teno
    from paper_2105_02127_amd.batch import Batch
    m = inputs.jittered_periodic_mesh(12, 509)
    s = teno.Solver(teno.Mesh(m.xy, m.tri).setup(order=4, characteristic=1))
    with pytest.raises(teno.TenoError):
        Batch([s])

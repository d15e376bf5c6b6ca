"""Batched path: meshes of mixed size and order advanced together must give,
mesh by mesh, exactly the single-mesh result (same kernels, deterministic),
with every schedule option, eagerly and from graph replays; and on meshes of
the 64-mesh workload itself, the oracle's result."""
import numpy as np
import pytest

from paper_2105_02127_amd import inputs
from paper_2105_02127_amd.batch import CANDIDATES

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


# --------------------------------------------------------------------------
# the batched workload's own meshes against the oracle
# --------------------------------------------------------------------------
# (N, order, seed) taken from the 64-mesh workload (inputs.batch_specs): its
# largest mesh (316^2 x 2 = 199,712 cells, order 6), the largest of orders 4
# and 5, two of order 3 and its smallest mesh (N = 32)
ORACLE_SPECS = [(316, 6, 5019), (311, 4, 5008), (309, 5, 5027), (279, 3, 5051), (74, 3, 5018),
                (32, 5, 5016)]


@pytest.fixture(scope="module")
def oracle_batch(torch_cuda, oracle_mod):
    """GPU solvers and initial states of ORACLE_SPECS, and per mesh the
    oracle's dt and one SSP-RK3 step (state, stage flags, near-tie masks)."""
    torch = torch_cuda
    from paper_2105_02127_amd import teno
    spec = {tuple(s) for s in inputs.batch_specs()}
    assert all(s in spec for s in ORACLE_SPECS)
    sv, U0, ref, perms = [], [], [], []
    for n, p, seed in ORACLE_SPECS:
        print(f"[batch oracle] N={n} order={p} seed={seed}", flush=True)
        m = inputs.jittered_periodic_mesh(n, seed)
        U = inputs.random_lines(m)
        lm = teno.Mesh(m.xy, m.tri).setup(order=p, fallback=1)
        sv.append(teno.Solver(lm))
        perms.append(lm.perm)
        U0.append(torch.as_tensor(U[lm.perm], device="cuda"))
        om = oracle_mod.OracleMesh(m.xy, m.tri)
        om.setup(oracle_mod.params(order=p, fallback=1))
        dto = om.dt(U, 0.4)
        r = om.rk_step(U, dto)
        ref.append(dict(dt=dto, U=r["U"], flags=r["flags"], ties=r["diag"]["tie_mask"]))
    return sv, U0, ref, perms


SCHEDULES = ([dict(c) for c in CANDIDATES]
             + [dict(order_mode=om, waves_per_cu=w, item_order=1, use_graph=0)
                for om, w in ((0, 0), (1, 0), (1, 8))])


def test_batch_matches_oracle_on_workload_meshes(torch_cuda, oracle_batch):
    # every schedule (the autotuner's candidates, eager and replayed): one
    # batched SSP-RK3 step with the oracle's dt per mesh, compared mesh by
    # mesh with the oracle: states to 1e-12, flags of every stage exact away
    # from near ties
    from parity_check import assert_states, check_flags
    torch = torch_cuda
    from paper_2105_02127_amd.batch import Batch
    sv, U0, ref, perms = oracle_batch
    b = Batch(sv)
    dt = torch.tensor([r["dt"] for r in ref], dtype=torch.float64, device="cuda")
    flags = [s.empty_flags(3) for s in sv]
    b.set_flags(flags)
    for tuning in SCHEDULES:
        print(f"[batch oracle] schedule {tuning}", flush=True)
        b.set_tuning(**tuning)
        work = [u.clone() for u in U0]
        for f in flags:
            f.fill_(0)
        b.rk_step(work, dt)
        torch.cuda.synchronize()
        for k, (w, r, perm, f) in enumerate(zip(work, ref, perms, flags)):
            got = np.empty_like(r["U"])
            got[perm] = w.cpu().numpy()
            assert_states(got, r["U"], what=f"mesh {k} {ORACLE_SPECS[k]} {tuning}")
            gfl = np.empty((3, len(perm)), np.uint16)
            gfl[:, perm] = f.cpu().numpy().view(np.uint16)
            for st in range(3):
                check_flags(gfl[st], r["flags"][st], r["ties"][st],
                            what=f"mesh {k} stage {st} {tuning}")


def test_batch_loop_captures_once_and_never_rewrites(torch_cuda, oracle_batch):
    # a simulation loop (dt, then step, on the same buffers) captures its
    # graph once and writes the descriptors once; replays match eager steps
    torch = torch_cuda
    from paper_2105_02127_amd.batch import Batch
    sv, U0, _, _ = oracle_batch
    small = [(s, u) for s, u in zip(sv, U0) if s.n_cell < 20000]
    b = Batch([s for s, _ in small])
    b.set_tuning(order_mode=1, waves_per_cu=0, item_order=1, use_graph=1)
    work = [u.clone() for _, u in small]
    dt = torch.empty(len(small), dtype=torch.float64, device="cuda")
    s0 = b.stats
    for _ in range(5):
        b.max_dt(work, 0.4, dt)
        b.rk_step(work, dt)
    torch.cuda.synchronize()
    st = b.stats
    assert st["captures"] - s0["captures"] == 1
    assert st["descriptor_writes"] - s0["descriptor_writes"] == 1
    assert st["replays"] - s0["replays"] == 5
    eager = [u.clone() for _, u in small]
    for _ in range(5):
        for (s, _), u in zip(small, eager):
            d = s.max_dt(u, 0.4)
            s.rk_step(u, d)
    torch.cuda.synchronize()
    for g, e in zip(work, eager):
        assert torch.equal(g, e)

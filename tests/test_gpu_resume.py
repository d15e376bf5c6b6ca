"""Checkpoint and resume (GPU): 20 steps in one go equal 10 steps, a state
saved to disk and loaded into a freshly built mesh and solver, and 10 more
steps, bit for bit (triangles with the fused time step, and tetrahedra)."""
import numpy as np
import pytest

from paper_2105_02127_amd import inputs, inputs3

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_triangles_resume_bit_identical(torch_cuda, tmp_path):
    torch = torch_cuda
    from paper_2105_02127_amd import teno
    m = inputs.jittered_periodic_mesh(48, 21)
    U0 = inputs.random_lines(m)
    print("[resume] triangles N=48 order 5", flush=True)

    def solver():
        lm = teno.Mesh(m.xy, m.tri).setup(order=5, fallback=1)
        return lm, teno.Solver(lm)

    def run(lm, sv, U, dt, steps):
        for _ in range(steps):
            sv.rk_step_dt(U, dt, 0.4)
        torch.cuda.synchronize()

    lm, sv = solver()
    U = torch.as_tensor(U0[lm.perm], device="cuda")
    dt = sv.max_dt(U, 0.4)
    run(lm, sv, U, dt, 20)
    straight = lm.to_user(U.cpu().numpy())

    lm, sv = solver()
    U = torch.as_tensor(U0[lm.perm], device="cuda")
    dt = sv.max_dt(U, 0.4)
    run(lm, sv, U, dt, 10)
    path = tmp_path / "checkpoint.npz"
    np.savez(path, U=lm.to_user(U.cpu().numpy()), dt=dt.cpu().numpy())
    del sv, lm, U, dt

    ck = np.load(path)
    lm, sv = solver()
    U = torch.as_tensor(np.ascontiguousarray(ck["U"][lm.perm]), device="cuda")
    dt = torch.as_tensor(ck["dt"], device="cuda")
    run(lm, sv, U, dt, 10)
    assert np.array_equal(lm.to_user(U.cpu().numpy()), straight)


def test_tetrahedra_resume_bit_identical(torch_cuda, tmp_path):
    torch = torch_cuda
    from paper_2105_02127_amd import teno3
    m = inputs3.jittered_periodic_cube(7, 22)
    U0 = inputs3.random_planes3(m)
    print("[resume] tetrahedra N=7 order 4", flush=True)

    def solver():
        lm = teno3.TetMesh(m.xyz, m.tet).setup(order=4, fallback=1)
        return lm, teno3.TetSolver(lm)

    def run(sv, U, steps):
        dt = torch.empty(1, dtype=torch.float64, device="cuda")
        for _ in range(steps):
            sv.max_dt(U, 0.4, dt)
            sv.rk_step(U, dt)
        torch.cuda.synchronize()

    lm, sv = solver()
    U = torch.as_tensor(U0[lm.perm], device="cuda")
    run(sv, U, 20)
    straight = lm.to_user(U.cpu().numpy())

    lm, sv = solver()
    U = torch.as_tensor(U0[lm.perm], device="cuda")
    run(sv, U, 10)
    path = tmp_path / "checkpoint3.npz"
    np.savez(path, U=lm.to_user(U.cpu().numpy()))
    del sv, lm, U

    ck = np.load(path)
    lm, sv = solver()
    U = torch.as_tensor(np.ascontiguousarray(ck["U"][lm.perm]), device="cuda")
    run(sv, U, 10)
    assert np.array_equal(lm.to_user(U.cpu().numpy()), straight)

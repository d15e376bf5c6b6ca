"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars (FP64 throughout):
  * selection flags bit-exact, except at the (cell, variable) nibbles where
    the oracle reports a near tie (|chi/C_T - 1| <= 1e-10); a differing
    nibble anywhere else fails;
  * face-point states and stage states: max_i |x - y| <= 1e-12 max_i |y|
    per conservative variable;
  * residual: max |R_gpu - R_oracle| <= 1e-12 * S, where S is the flux scale
    max_i sum_faces |A| |F(U_i) . n| / |V_i| (R is a difference of O(1/h)
    face terms, so its own size is not the right reference).
"""
import math

import numpy as np
import pytest

from paper_2105_02127_amd import inputs
from parity_check import REL, assert_adjoint, assert_states, check_flags, trajectory

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def teno():
    from paper_2105_02127_amd import teno as t
    t.load()
    return t


class Case:
    """One mesh + state on both sides (oracle in user order, GPU internal)."""

    def __init__(self, teno, oracle_mod, torch, n, seed, order, ic="random_lines", fallback=1,
                 oracle_all=True, variant=0, characteristic=0):
        print(f"[case] n={n} seed={seed} order={order} ic={ic} fallback={fallback} "
              f"variant={variant} characteristic={characteristic}", flush=True)
        self.m = inputs.jittered_periodic_mesh(n, seed)
        self.U = inputs.make_state(self.m, ic)
        self.lm = teno.Mesh(self.m.xy, self.m.tri).setup(order=order, fallback=fallback,
                                                         variant=variant,
                                                         characteristic=characteristic)
        self.sv = teno.Solver(self.lm)
        self.om = oracle_mod.OracleMesh(self.m.xy, self.m.tri)
        self.om.setup(oracle_mod.params(order=order, fallback=fallback, variant=variant,
                                        characteristic=characteristic), all_cells=oracle_all)
        self.perm = self.lm.perm
        self.torch = torch
        self.Ud = torch.as_tensor(self.U[self.perm], device="cuda")

    def dev(self, a_user):
        return self.torch.as_tensor(np.ascontiguousarray(a_user[self.perm]), device="cuda")

    def host_user(self, t):
        a = t.cpu().numpy()
        out = np.empty_like(a)
        out[self.perm] = a
        return out

    def flags_user(self, t):
        """Flags in user cell order; [..., n_cell] layouts keep their
        leading axes (one word per local edge in characteristic variables)."""
        a = t.cpu().numpy().view(np.uint16)
        out = np.empty_like(a)
        out[..., self.perm] = a
        return out

    def flux_scale(self):
        area, _, _ = self.om.geometry()
        f = self.om.faces()
        U = self.U
        g = 1.4
        r, mx, my, e = U.T
        vx, vy = mx / r, my / r
        p = (g - 1) * (e - 0.5 * r * (vx * vx + vy * vy))
        acc = np.zeros(len(U))
        for side in ("L", "R"):
            c = f[side]
            un = vx[c] * f["normal"][:, 0] + vy[c] * f["normal"][:, 1]
            Fm = np.abs(np.stack([r[c] * un, mx[c] * un + p[c] * f["normal"][:, 0],
                                  my[c] * un + p[c] * f["normal"][:, 1], un * (e[c] + p[c])], 1))
            np.add.at(acc, c, f["length"] * Fm.max(1))
        return float((acc / area).max())


# --------------------------------------------------------------------------
@pytest.mark.parametrize("order,n,seed", [(3, 13, 11), (4, 16, 12), (5, 17, 13), (6, 20, 14)])
def test_reconstruction_and_residual(teno, oracle_mod, torch_cuda, order, n, seed):
    c = Case(teno, oracle_mod, torch_cuda, n, seed, order)
    ores = c.om.residual(c.U, want_fp=True)
    flags = c.sv.empty_flags()
    fs = c.sv.reconstruct(c.Ud, flags=flags)
    torch_cuda.cuda.synchronize()
    fs_user = np.empty((c.m.n_cell, fs.shape[0], 4))
    fs_user[c.perm] = fs.permute(1, 0, 2).cpu().numpy()
    oracle_fp = ores["fp"].reshape(c.m.n_cell, -1, 4)
    check_flags(c.flags_user(flags), ores["flags"], ores["diag"]["tie_mask"])
    assert_states(fs_user, oracle_fp, what="face states")
    c.sv.diagnostics(reset=True)            # the counters accumulate per call
    R = c.sv.residual(c.Ud, flags=flags)
    torch_cuda.cuda.synchronize()
    err = np.abs(c.host_user(R) - ores["R"]).max()
    assert err <= REL * c.flux_scale(), (err, c.flux_scale())
    d = c.sv.diagnostics(reset=True)
    od = c.om.residual(c.U)["diag"]
    assert d["nonphysical"] == od["nonphysical"] and d["fallbacks"] == od["fallbacks"]
    assert d["first_bad_cell"] == od["first_bad_cell"]


@pytest.mark.parametrize("order,ic", [(3, "random_lines"), (5, "random_lines"),
                                      (6, "wave_plus_jump"), (5, "kelvin_helmholtz")])
def test_cweno_matches_oracle(teno, oracle_mod, torch_cuda, order, ic):
    # CWENO weighting (Sec. 2.4): face states, residual and an RK step
    torch = torch_cuda
    c = Case(teno, oracle_mod, torch, 17, 70 + order, order, ic=ic, variant=2)
    ores = c.om.residual(c.U, want_fp=True)
    flags = c.sv.empty_flags()
    fs = c.sv.reconstruct(c.Ud, flags=flags)
    R = c.sv.residual(c.Ud)
    torch.cuda.synchronize()
    fs_user = np.empty((c.m.n_cell, fs.shape[0], 4))
    fs_user[c.perm] = fs.permute(1, 0, 2).cpu().numpy()
    assert_states(fs_user, ores["fp"].reshape(c.m.n_cell, -1, 4), what="CWENO face states")
    assert (c.flags_user(flags) == 0).all() and (ores["flags"] == 0).all()
    assert np.abs(c.host_user(R) - ores["R"]).max() <= REL * c.flux_scale()
    dto = c.om.dt(c.U, 0.4)
    dt = torch.full((1,), dto, dtype=torch.float64, device="cuda")
    ref = c.om.rk_step(c.U, dto)
    Ud = c.Ud.clone()
    c.sv.rk_step(Ud, dt)
    torch.cuda.synchronize()
    assert_states(c.host_user(Ud), ref["U"], what="CWENO U^{n+1}")
    # no selection to freeze: frozen and adjoint calls are refused
    with pytest.raises(teno.TenoError):
        c.sv.vjp_residual(c.Ud, flags, c.Ud)
    with pytest.raises(teno.TenoError):
        c.sv.residual_frozen(c.Ud, flags)


@pytest.mark.parametrize("order,variant,ic", [(3, 0, "random_lines"), (4, 0, "random_lines"),
                                               (5, 0, "random_lines"), (6, 0, "wave_plus_jump"),
                                               (5, 2, "random_lines"), (4, 1, "random_lines"),
                                               (3, 2, "random_lines"), (4, 2, "random_lines"),
                                               (6, 2, "wave_plus_jump")])
def test_characteristic_matches_oracle(teno, oracle_mod, torch_cuda, order, variant, ic):
    # selection in characteristic variables, edge by edge (Sec. 2.3): face
    # states, per-edge flags, residual and an RK step with its flags
    torch = torch_cuda
    c = Case(teno, oracle_mod, torch, 17, 90 + order, order, ic=ic, variant=variant,
             characteristic=1)
    ores = c.om.residual(c.U, want_fp=True)
    flags = c.sv.empty_flags()
    assert tuple(flags.shape) == (3, c.m.n_cell)
    fs = c.sv.reconstruct(c.Ud, flags=flags)
    R = c.sv.residual(c.Ud)
    torch.cuda.synchronize()
    fs_user = np.empty((c.m.n_cell, fs.shape[0], 4))
    fs_user[c.perm] = fs.permute(1, 0, 2).cpu().numpy()
    assert_states(fs_user, ores["fp"].reshape(c.m.n_cell, -1, 4), what="characteristic face states")
    gfl = c.flags_user(flags)
    check_flags(gfl, ores["flags"], ores["diag"]["tie_mask"])
    if variant == 0:
        assert (ores["flags"] != 0x8888).any()     # the case exercises the selection
    assert np.abs(c.host_user(R) - ores["R"]).max() <= REL * c.flux_scale()
    dto = c.om.dt(c.U, 0.4)
    dt = torch.full((1,), dto, dtype=torch.float64, device="cuda")
    ref = c.om.rk_step(c.U, dto)
    Ud = c.Ud.clone()
    fl3 = c.sv.empty_flags(3)
    assert tuple(fl3.shape) == (3, 3, c.m.n_cell)
    c.sv.rk_step(Ud, dt, flags3=fl3)
    torch.cuda.synchronize()
    assert_states(c.host_user(Ud), ref["U"], what="characteristic U^{n+1}")
    check_flags(c.flags_user(fl3), ref["flags"], ref["diag"]["tie_mask"])
    # the frozen and adjoint paths work in conservative variables only
    with pytest.raises(teno.TenoError):
        c.sv.residual_frozen(c.Ud, flags)
    with pytest.raises(teno.TenoError):
        c.sv.vjp_residual(c.Ud, flags, c.Ud)


def test_characteristic_contact_keeps_velocity_and_pressure(teno, oracle_mod, torch_cuda):
    # a contact lies in the entropy field only: the face states keep the
    # uniform velocity and pressure, and only that field drops stencils
    torch = torch_cuda
    m = inputs.jittered_periodic_mesh(24, 95)
    cen = m.xy[m.tri].mean(1)
    rho = np.where(np.sin(2 * np.pi * (cen[:, 0] + 0.3 * cen[:, 1])) > 0, 3.0, 1.0)
    rho = rho + 0.2 * np.cos(2 * np.pi * cen[:, 1])
    vx, vy, p = 0.7, -0.3, 1.0
    U = np.stack([rho, rho * vx, rho * vy, p / 0.4 + 0.5 * rho * (vx * vx + vy * vy)], 1)
    lm = teno.Mesh(m.xy, m.tri).setup(order=5, characteristic=1)
    sv = teno.Solver(lm)
    Ud = torch.as_tensor(U[lm.perm], device="cuda")
    flags = sv.empty_flags()
    fs = sv.reconstruct(Ud, flags=flags).cpu().numpy()
    fl = flags.cpu().numpy().view(np.uint16)
    ux, uy = fs[..., 1] / fs[..., 0], fs[..., 2] / fs[..., 0]
    pf = 0.4 * (fs[..., 3] - 0.5 * fs[..., 0] * (ux * ux + uy * uy))
    assert np.abs(ux - vx).max() < 1e-12 and np.abs(uy - vy).max() < 1e-12
    assert np.abs(pf - p).max() < 1e-12
    assert ((fl >> 4) & 0xF != 8).any()
    for v in (0, 2, 3):
        assert ((fl >> (4 * v)) & 0xF == 8).all()


@pytest.mark.parametrize("order", [3, 4, 5, 6])
def test_smooth_wave_teno_equals_linear(teno, oracle_mod, torch_cuda, order):
    # Sec. 5.1 (TENO rows equal the Linear rows): on the smooth workload
    # every selection keeps the large stencil, so 10 GPU steps of TENO and of
    # the linear scheme are bit-identical, and both match the oracle
    torch = torch_cuda
    w = inputs.WORKLOADS[1]
    c = Case(teno, oracle_mod, torch, w["n"], w["seed"], order, ic="smooth_wave", fallback=0,
             oracle_all=True)
    lin = teno.Solver(teno.Mesh(c.m.xy, c.m.tri).setup(order=order, fallback=0, variant=1))
    Ut, Ul = c.Ud.clone(), c.Ud.clone()
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    fl3 = c.sv.empty_flags(3)
    U = c.U
    for step in range(w["steps"]):
        dto = c.om.dt(U, 0.4)
        dt.fill_(dto)
        c.sv.rk_step(Ut, dt, flags3=fl3)
        lin.rk_step(Ul, dt)
        torch.cuda.synchronize()
        assert (fl3.cpu().numpy().view(np.uint16) == 0x8888).all(), f"step {step}"
        U = c.om.rk_step(U, dto)["U"]
    assert torch.equal(Ut, Ul)
    assert_states(c.host_user(Ut), U, what=f"TENO{order} after {w['steps']} steps")
    assert c.sv.diagnostics(reset=True)["nonphysical"] == 0


def test_trajectory_smooth_wave_10_steps(teno, oracle_mod, torch_cuda):
    """The small smooth workload: 10 SSP-RK3 steps, compared after every stage."""
    torch = torch_cuda
    w = inputs.WORKLOADS[1]
    c = Case(teno, oracle_mod, torch, w["n"], w["seed"], w["order"], ic="smooth_wave", fallback=0)
    U = c.U.copy()
    Ud = c.Ud.clone()
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    stages = torch.empty((3, c.m.n_cell, 4), dtype=torch.float64, device="cuda")
    flags3 = c.sv.empty_flags(3)
    for step in range(w["steps"]):
        c.sv.max_dt(Ud, 0.4, dt)
        dto = c.om.dt(U, 0.4)
        assert abs(dt.item() - dto) <= 1e-14 * dto
        # both sides advance with the oracle's dt
        dt.fill_(dto)
        ref = c.om.rk_step(U, dto, want_stages=True)
        c.sv.rk_step(Ud, dt, flags3=flags3, stages=stages)
        torch.cuda.synchronize()
        for k in range(3):
            assert_states(c.host_user(stages[k]), ref["stages"][k], what=f"step {step} stage {k}")
            check_flags(c.flags_user(flags3[k]), ref["flags"][k], ref["diag"]["tie_mask"][k])
        U = ref["U"]
        assert_states(c.host_user(Ud), U, what=f"step {step}")


@pytest.mark.parametrize("order,ic", [(3, "random_lines"), (5, "random_lines"),
                                      (6, "random_lines"), (4, "kelvin_helmholtz"),
                                      (5, "kelvin_helmholtz")])
def test_rk_stages(teno, oracle_mod, torch_cuda, order, ic):
    torch = torch_cuda
    c = Case(teno, oracle_mod, torch, 18, 40 + order, order, ic=ic)
    dto = c.om.dt(c.U, 0.4)
    dt = torch.full((1,), dto, dtype=torch.float64, device="cuda")
    ref = c.om.rk_step(c.U, dto, want_stages=True)
    Ud = c.Ud.clone()
    stages = torch.empty((3, c.m.n_cell, 4), dtype=torch.float64, device="cuda")
    flags3 = c.sv.empty_flags(3)
    c.sv.rk_step(Ud, dt, flags3=flags3, stages=stages)
    torch.cuda.synchronize()
    for k in range(3):
        assert_states(c.host_user(stages[k]), ref["stages"][k], what=f"stage {k}")
        check_flags(c.flags_user(flags3[k]), ref["flags"][k], ref["diag"]["tie_mask"][k])
    assert_states(c.host_user(Ud), ref["U"], what="U^{n+1}")
    # the same step through the stage-by-stage entry point
    U1 = c.sv.empty_state()
    U2 = c.sv.empty_state()
    U3 = c.sv.empty_state()
    c.sv.rk_stage(0, c.Ud, c.Ud, U1, dt)
    c.sv.rk_stage(1, c.Ud, U1, U2, dt)
    c.sv.rk_stage(2, c.Ud, U2, U3, dt)
    torch.cuda.synchronize()
    assert torch.equal(U3, Ud)


def test_frozen_residual_and_linear_variant(teno, oracle_mod, torch_cuda):
    torch = torch_cuda
    c = Case(teno, oracle_mod, torch, 16, 51, 4)
    base = c.om.residual(c.U)
    fl = c.dev(base["flags"].view(np.int16))
    U2 = c.U * (1.0 + 1e-3 * np.random.default_rng(0).normal(size=c.U.shape))
    ref = c.om.residual(U2, frozen_flags=base["flags"])
    R = c.sv.residual_frozen(c.dev(U2), fl)
    torch.cuda.synchronize()
    assert np.abs(c.host_user(R) - ref["R"]).max() <= REL * c.flux_scale()
    lin = Case(teno, oracle_mod, torch, 16, 51, 4, variant=1)
    flags = lin.sv.empty_flags()
    R = lin.sv.residual(lin.Ud, flags=flags)
    ref = lin.om.residual(lin.U)
    torch.cuda.synchronize()
    # large stencil everywhere except cells that fell back to first order
    np.testing.assert_array_equal(lin.flags_user(flags), ref["flags"])
    assert set(np.unique(ref["flags"]).tolist()) <= {0, 0x8888}
    assert np.abs(lin.host_user(R) - ref["R"]).max() <= REL * lin.flux_scale()


def test_deterministic_and_conservative(teno, oracle_mod, torch_cuda):
    torch = torch_cuda
    c = Case(teno, oracle_mod, torch, 24, 61, 5, oracle_all=False)
    R1 = c.sv.residual(c.Ud)
    R2 = c.sv.residual(c.Ud)
    torch.cuda.synchronize()
    assert torch.equal(R1, R2)
    area, _, _ = c.om.geometry()
    a = torch.as_tensor(area[c.perm], device="cuda")
    tot = (a[:, None] * R1).sum(0).cpu().numpy()
    assert np.abs(tot).max() <= 1e-13 * (a[:, None] * R1).abs().sum(0).max().item()


@pytest.mark.parametrize("order", [3, 6])
def test_free_stream(teno, oracle_mod, torch_cuda, order):
    # Sec. 2.1: a uniform state is a steady solution.  Every stencil
    # difference is zero, so beta = 0, the large stencil is kept for every
    # variable (chi_K = 1/4), the face states equal the average, and the
    # residual cancels to round-off (relative to the flux scale).
    torch = torch_cuda
    c = Case(teno, oracle_mod, torch, 15, 81, order, oracle_all=False)
    rho, u, v, p = 1.3, 0.7, -0.4, 0.9
    U = inputs.conservative(np.full(c.m.n_cell, rho), np.full(c.m.n_cell, u),
                            np.full(c.m.n_cell, v), np.full(c.m.n_cell, p))
    Ud = torch.as_tensor(U[c.perm], device="cuda")
    flags = torch.empty(c.m.n_cell, dtype=torch.int16, device="cuda")
    fs = c.sv.reconstruct(Ud, flags=flags)
    R = c.sv.residual(Ud)
    torch.cuda.synchronize()
    assert set(np.unique(c.flags_user(flags)).tolist()) == {0x8888}
    assert torch.equal(fs, Ud[None].expand_as(fs))
    c.U = U
    assert np.abs(R.cpu().numpy()).max() <= 1e-13 * c.flux_scale()
    assert c.sv.diagnostics(reset=True)["near_ties"] == 0


def test_dt_matches_oracle(teno, oracle_mod, torch_cuda):
    torch = torch_cuda
    c = Case(teno, oracle_mod, torch, 21, 71, 3, oracle_all=False)
    dt = c.sv.max_dt(c.Ud, 0.4)
    assert dt.item() == pytest.approx(c.om.dt(c.U, 0.4), rel=1e-14)


@pytest.mark.parametrize("order", [3, 4, 6])
def test_vjp_residual_matches_oracle(teno, oracle_mod, torch_cuda, order):
    torch = torch_cuda
    c = Case(teno, oracle_mod, torch, 14, 80 + order, order)
    flags = c.om.residual(c.U)["flags"]
    lam = np.random.default_rng(order).normal(size=c.U.shape)
    ref = c.om.vjp(c.U, flags, lam)
    got = c.sv.vjp_residual(c.Ud, c.dev(flags.view(np.int16)), c.dev(lam))
    torch.cuda.synchronize()
    assert_adjoint(c.host_user(got), ref, c.om.vjp_scale(c.U, flags, lam), what=f"U_bar p={order}")


def test_vjp_rk_step_matches_oracle(teno, oracle_mod, torch_cuda):
    torch = torch_cuda
    c = Case(teno, oracle_mod, torch, 14, 91, 4)
    dto = c.om.dt(c.U, 0.4)
    base = c.om.rk_step(c.U, dto, want_stages=True)
    lam = np.random.default_rng(1).normal(size=c.U.shape)
    ref = c.om.vjp_rk_step(base["stages"], base["flags"], dto, lam)
    st = torch.stack([c.dev(base["stages"][k]) for k in range(3)]).contiguous()
    f3 = torch.stack([c.dev(base["flags"][k].view(np.int16)) for k in range(3)]).contiguous()
    dt = torch.full((1,), dto, dtype=torch.float64, device="cuda")
    got = c.sv.vjp_rk_step(st, f3, dt, c.dev(lam))
    torch.cuda.synchronize()
    scale = c.om.vjp_rk_step_scale(base["stages"], base["flags"], dto, lam)
    assert_adjoint(c.host_user(got), ref, scale, what="lam_in")
    # face states kept by a GPU step under the same selection and dt spare
    # the adjoint its reconstructions; the result must not change
    fs = c.sv.empty_face_states()
    U = c.dev(base["stages"][0])
    st2 = torch.empty_like(st)
    f32 = torch.empty_like(f3)
    c.sv.rk_step(U, dt, flags3=f32, stages=st2, face_states=fs)
    kept = c.sv.vjp_rk_step(st2, f32, dt, c.dev(lam), face_states=fs)
    again = c.sv.vjp_rk_step(st2, f32, dt, c.dev(lam))
    torch.cuda.synchronize()
    assert torch.equal(kept, again)
    assert_adjoint(c.host_user(kept), ref, scale, what="lam_in (kept face states)")


# --------------------------------------------------------------------------
# full-size workloads: sampled cells the oracle computes one by one
# --------------------------------------------------------------------------
def _sampled(teno, oracle_mod, torch, key, n_sample=160, characteristic=0, n=None, variant=0,
             order=None):
    w, m, U = inputs.make_workload(key, n=n)
    if order is not None:
        w = dict(w, order=order)
    print(f"[full-size] {w['name']} n={w['n']} cells={m.n_cell} characteristic={characteristic} "
          f"variant={variant}", flush=True)
    lm = teno.Mesh(m.xy, m.tri).setup(order=w["order"], fallback=1, characteristic=characteristic,
                                      variant=variant)
    info = lm.info()
    if n is not None and n > 1024:
        # past 2^31 operator entries: every offset into M must be 64-bit
        assert info.matrix_doubles_per_cell * m.n_cell > 2 ** 31
    sv = teno.Solver(lm)
    perm = lm.perm
    om = oracle_mod.OracleMesh(m.xy, m.tri)
    om.setup(oracle_mod.params(order=w["order"], fallback=1, characteristic=characteristic,
                               variant=variant), all_cells=False)
    rng = np.random.default_rng(key)
    cells = np.unique(np.concatenate([rng.integers(0, m.n_cell, n_sample),
                                      perm[-5:], perm[:3]]))       # include the ragged tail
    Ud = torch.as_tensor(U[perm], device="cuda")
    inv = np.empty_like(perm)
    inv[perm] = np.arange(m.n_cell)
    flags = sv.empty_flags()
    fs = sv.reconstruct(Ud, flags=flags)
    R = sv.residual(Ud)
    torch.cuda.synchronize()
    fp, ofl, _, odg = om.reconstruct_cells(U, cells)
    got = fs[:, torch.as_tensor(inv[cells], device="cuda")].permute(1, 0, 2).cpu().numpy()
    assert_states(got, fp.reshape(len(cells), -1, 4), what="face states")
    gfl = flags.cpu().numpy().view(np.uint16)[..., inv[cells]]
    if characteristic:
        gfl = gfl.T                                   # [cell][edge] like the oracle's
    check_flags(gfl, ofl, odg["tie_mask"])
    Ro, _ = om.residual_cells(U, cells)
    Rg = R.cpu().numpy()[inv[cells]]
    assert np.abs(Rg - Ro).max() <= REL * _flux_scale_cells(U, m, om, cells)
    # conservation over the whole mesh: sum |V_i| R_i cancels to round-off
    ar, _, _ = om.geometry()
    aR = torch.as_tensor(ar[perm], device="cuda")[:, None] * R
    tot = aR.sum(0).cpu().numpy()
    assert np.abs(tot).max() <= 1e-12 * aR.abs().sum(0).max().item()


def _flux_scale_cells(U, m, om, cells):
    f = om.faces()
    area, _, _ = om.geometry()
    cf = f["cell_face"][cells]
    r, mx, my, e = U[cells].T
    vx, vy = mx / r, my / r
    p = 0.4 * (e - 0.5 * r * (vx * vx + vy * vy))
    acc = np.zeros(len(cells))
    for k in range(3):
        nrm = f["normal"][cf[:, k]]
        un = vx * nrm[:, 0] + vy * nrm[:, 1]
        Fm = np.abs(np.stack([r * un, mx * un + p * nrm[:, 0], my * un + p * nrm[:, 1],
                              un * (e + p)], 1)).max(1)
        acc += f["length"][cf[:, k]] * Fm
    return float((acc / area[cells]).max())


def test_full_size_teno5_lines_sampled(teno, oracle_mod, torch_cuda):
    _sampled(teno, oracle_mod, torch_cuda, 2)


def test_full_size_teno6_wavejump_sampled(teno, oracle_mod, torch_cuda):
    _sampled(teno, oracle_mod, torch_cuda, 3, n_sample=64)


def _trajectory_full(teno, oracle_mod, torch, key, steps):
    # a workload at its full size, in the bench's launch configuration:
    # whole SSP-RK3 steps on both sides (the oracle's dt), every stage of
    # every cell compared, re-synced after a flag flip at a near tie
    w, m, U = inputs.make_workload(key)
    print(f"[full-size trajectory] {w['name']} cells={m.n_cell} steps={steps}", flush=True)
    lm = teno.Mesh(m.xy, m.tri).setup(order=w["order"], fallback=1)
    sv = teno.Solver(lm)
    om = oracle_mod.OracleMesh(m.xy, m.tri)
    om.setup(oracle_mod.params(order=w["order"], fallback=1))
    resyncs, worst, _ = trajectory(torch, sv, om, U, lm.perm, steps, label=w["name"])
    print(f"[full-size trajectory] {w['name']}: {steps} steps, {3 * steps} stages, "
          f"re-syncs {resyncs}, worst relative state error {worst:.2e}", flush=True)
    return resyncs


@pytest.mark.timeout(900)
def test_trajectory_teno5_lines_N512_10_steps(teno, oracle_mod, torch_cuda):
    # the headline workload (524,288 cells, TENO5, random lines): 10 steps
    _trajectory_full(teno, oracle_mod, torch_cuda, 2, 10)


@pytest.mark.timeout(900)
def test_trajectory_teno6_wavejump_N1024_2_steps(teno, oracle_mod, torch_cuda):
    # the TENO6 roofline workload (2,097,152 cells, wave plus jump): 2 steps
    _trajectory_full(teno, oracle_mod, torch_cuda, 3, 2)


def test_trajectory_resync_protocol(teno, oracle_mod, torch_cuda):
    # the re-sync path itself: with a cutoff chosen so that one chi of the
    # first stage sits exactly on it, the oracle reports a near tie there,
    # and the protocol must go on past it (flipped or not) to the end
    torch = torch_cuda
    m = inputs.jittered_periodic_mesh(16, 33)
    U = inputs.random_lines(m)
    om0 = oracle_mod.OracleMesh(m.xy, m.tri)
    om0.setup(oracle_mod.params(order=4, fallback=1))
    fp, fl, beta, _ = om0.reconstruct_cells(U, np.arange(m.n_cell))
    # chi_K of every (cell, variable) at C_T = 1e-6; put C_T on one of the
    # step-one values, so that it is a tie by construction
    g = (beta + 1e-12) ** -6.0
    chiK = g[..., 3] / g.sum(-1)
    pick = np.sort(chiK[(chiK > 1e-3) & (chiK < 0.2)].ravel())
    assert pick.size > 0
    ct = float(pick[pick.size // 2])
    lm = teno.Mesh(m.xy, m.tri).setup(order=4, fallback=1, ct=ct)
    sv = teno.Solver(lm)
    om = oracle_mod.OracleMesh(m.xy, m.tri)
    om.setup(oracle_mod.params(order=4, fallback=1, ct=ct))
    assert om.residual(U)["diag"]["tie_mask"].any()
    resyncs, worst, _ = trajectory(torch, sv, om, U, lm.perm, 2, label="tie")
    print(f"[re-sync protocol] C_T={ct:.6e}: re-syncs {resyncs}, worst {worst:.2e}", flush=True)


def test_teno6_past_2e31_operator_entries_sampled(teno, oracle_mod, torch_cuda):
    # the largest case: 1050^2 x 2 = 2,205,000 cells at order 6, whose
    # operators hold more than 2^31 doubles (17.4 GB)
    _sampled(teno, oracle_mod, torch_cuda, 3, n_sample=48, n=1050)


def test_full_size_teno5_khi_sampled(teno, oracle_mod, torch_cuda):
    # the paper's KHI state (Sec. 5.7) on 576,738 cells
    _sampled(teno, oracle_mod, torch_cuda, 6, n_sample=96)


def test_full_size_teno5_khi_characteristic_sampled(teno, oracle_mod, torch_cuda):
    # characteristic variables on the KHI workload at full size
    _sampled(teno, oracle_mod, torch_cuda, 6, n_sample=64, characteristic=1)


@pytest.mark.parametrize("order,variant,characteristic", [(3, 0, 0), (4, 0, 0), (6, 0, 0), (6, 2, 0),
                                                        (6, 0, 1), (6, 2, 1)])
def test_full_size_khi_other_schemes_sampled(teno, oracle_mod, torch_cuda, order, variant,
                                             characteristic):
    # the rest of the KHI timing legs at full size: TENO3, TENO4, TENO6,
    # CWENO6 and characteristic TENO6; and characteristic CWENO6
    _sampled(teno, oracle_mod, torch_cuda, 6, n_sample=48, characteristic=characteristic,
             variant=variant, order=order)


def test_full_size_cweno5_khi_sampled(teno, oracle_mod, torch_cuda):
    # CWENO5 on the KHI workload at full size, as the bench times it
    _sampled(teno, oracle_mod, torch_cuda, 6, n_sample=64, variant=2)


def test_full_size_cweno5_khi_characteristic_sampled(teno, oracle_mod, torch_cuda):
    # CWENO5 in characteristic variables on the KHI workload at full size
    _sampled(teno, oracle_mod, torch_cuda, 6, n_sample=64, characteristic=1, variant=2)


def test_rk_step_dt_equals_step_then_max_dt(teno, oracle_mod, torch_cuda):
    # the fused step leaves exactly teno_max_dt of its result in dt, and
    # its state and flags equal teno_rk_step's; over a few steps of a mesh
    # with a ragged last block of cells
    torch = torch_cuda
    c = Case(teno, oracle_mod, torch, 19, 55, 5, oracle_all=False)
    Ua, Ub = c.Ud.clone(), c.Ud.clone()
    da = c.sv.max_dt(Ua, 0.4)
    db = da.clone()
    fa, fb = c.sv.empty_flags(3), c.sv.empty_flags(3)
    for step in range(4):
        c.sv.rk_step(Ua, da, flags3=fa)
        c.sv.max_dt(Ua, 0.4, da)
        c.sv.rk_step_dt(Ub, db, 0.4, flags3=fb)
        torch.cuda.synchronize()
        assert torch.equal(Ua, Ub) and torch.equal(fa, fb), step
        assert da.item() == db.item(), (step, da.item(), db.item())

"""The comparison rules of the GPU parity tests, checked on the CPU with a
stand-in solver that replays the oracle's stages (test code only) and
plants a flipped selection flag: at a reported near tie the trajectory
must re-sync and go on; anywhere else it must fail."""
import numpy as np
import pytest
import torch

from paper_2105_02127_amd import inputs
from parity_check import check_flags, trajectory


class ReplaySolver:
    """Advances one SSP-RK3 stage with the oracle's residual (internal order
    = user order here), optionally flipping one flag nibble at a given
    (step, stage) and perturbing that cell's state as a flipped stencil
    would."""

    def __init__(self, om, plant=None):
        self.om, self.plant, self.calls = om, plant, 0

    def empty_state(self):
        return torch.empty((self.om.n_cell, 4), dtype=torch.float64)

    def empty_flags(self):
        return torch.zeros(self.om.n_cell, dtype=torch.int16)

    def rk_stage(self, k, Un, Uk, Uk1, dt, flags=None):
        un, uk, d = Un.numpy(), Uk.numpy(), float(dt.item())
        res = self.om.residual(uk)
        R, fl = res["R"], res["flags"].copy()
        if k == 0:
            out = un + d * R
        elif k == 1:
            out = 0.75 * un + 0.25 * uk + 0.25 * (d * R)
        else:
            out = (1.0 / 3.0) * un + (2.0 / 3.0) * uk + (2.0 / 3.0) * (d * R)
        if self.plant is not None and self.plant[0] == self.calls:
            cell, nib = self.plant[1], self.plant[2]
            fl[cell] ^= np.uint16(0x8 << (4 * nib))
            out = out.copy()
            out[cell] *= 1.0 + 1e-6
        self.calls += 1
        Uk1.copy_(torch.as_tensor(out))
        flags.copy_(torch.as_tensor(fl.view(np.int16)))
        return Uk1


def _tie_case(oracle_mod):
    m = inputs.jittered_periodic_mesh(12, 33)
    U = inputs.random_lines(m)
    om0 = oracle_mod.OracleMesh(m.xy, m.tri)
    om0.setup(oracle_mod.params(order=3, fallback=1))
    _, _, beta, _ = om0.reconstruct_cells(U, np.arange(m.n_cell))
    g = (beta + 1e-12) ** -6.0
    chiK = g[..., 3] / g.sum(-1)
    cand = np.argwhere((chiK > 1e-3) & (chiK < 0.2))
    cell, var = (int(x) for x in cand[len(cand) // 2])
    ct = float(chiK[cell, var])
    om = oracle_mod.OracleMesh(m.xy, m.tri)
    om.setup(oracle_mod.params(order=3, fallback=1, ct=ct))
    mask = om.residual(U)["diag"]["tie_mask"]
    assert (mask[cell] >> (4 * var)) & 0xF == 0xF      # the oracle reports this tie
    return m, U, om, cell, var, mask


def test_check_flags_by_location():
    orc = np.array([0x8888, 0x8881, 0x8888], np.uint16)
    ties = np.array([0, 0x000F, 0], np.uint16)
    assert check_flags(orc, orc, ties) == 0
    assert check_flags(orc ^ np.array([0, 0x0009, 0], np.uint16), orc, ties) == 1
    with pytest.raises(AssertionError):
        # a tie elsewhere does not excuse a flip at a cell without one
        check_flags(orc ^ np.array([0, 0, 0x0900], np.uint16), orc, ties)
    with pytest.raises(AssertionError):
        # nor at another variable of the tied cell
        check_flags(orc ^ np.array([0, 0x0090, 0], np.uint16), orc, ties)


def test_trajectory_resyncs_at_a_near_tie(oracle_mod):
    m, U, om, cell, var, _ = _tie_case(oracle_mod)
    sv = ReplaySolver(om, plant=(0, cell, var))
    log = []
    resyncs, worst, Uend = trajectory(torch, sv, om, U, np.arange(m.n_cell), 2, label="cpu",
                                      log=lambda *a, **k: log.append(a[0]), device="cpu")
    assert resyncs == 1 and len(log) == 1 and "step 0 stage 0" in log[0]
    assert worst <= 1e-13
    np.testing.assert_array_equal(Uend, om.rk_step(om.rk_step(U, om.dt(U))["U"],
                                                   om.dt(om.rk_step(U, om.dt(U))["U"]))["U"])


def test_trajectory_fails_away_from_ties(oracle_mod):
    m, U, om, cell, var, mask = _tie_case(oracle_mod)
    other = next(c for c in range(m.n_cell) if mask[c] == 0)
    sv = ReplaySolver(om, plant=(1, other, 0))
    with pytest.raises(AssertionError, match="away from near ties"):
        trajectory(torch, sv, om, U, np.arange(m.n_cell), 1, label="cpu",
                   log=lambda *a, **k: None, device="cpu")


def test_trajectory_fails_on_state_error(oracle_mod):
    # a state error without a flag flip is never excused
    m, U, om, cell, var, mask = _tie_case(oracle_mod)

    class Drift(ReplaySolver):
        def rk_stage(self, k, Un, Uk, Uk1, dt, flags=None):
            super().rk_stage(k, Un, Uk, Uk1, dt, flags)
            if k == 1:
                Uk1[3] *= 1.0 + 1e-9
            return Uk1

    with pytest.raises(AssertionError, match="max err"):
        trajectory(torch, Drift(om), om, U, np.arange(m.n_cell), 1, label="cpu",
                   log=lambda *a, **k: None, device="cpu")

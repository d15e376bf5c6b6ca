"""Comparison helpers of the GPU parity tests (HIP path against the oracle).

Bars (FP64 throughout):
  * selection flags bit-exact, except at the (cell, variable) nibbles where
    the oracle met a near tie (|chi/C_T - 1| <= 1e-10 for one of the chi of
    that selection): a differing nibble anywhere else fails;
  * states: max_i |x - y| <= 1e-12 max_i |y| per conservative variable;
  * adjoints: max_i |x - y| <= 1e-12 max_i S_i per variable, where S is the
    oracle's comparison scale (oracle_vjp_scale): at every cell the summed
    magnitudes of the terms the adjoint adds there, each bounded through
    its own factors.  The adjoint of a cell is a sum of O(1/h) face terms
    that largely cancel, so its own size is not the right reference (as
    the forward residual is compared against the flux scale).

`trajectory` implements the re-sync protocol of trajectory parity: both
sides step with the oracle's dt, every stage is compared, and a flag that
flips at a reported near tie is recorded and answered by copying the
oracle's stage state to the GPU before the next stage.
"""
from __future__ import annotations

import numpy as np

REL = 1e-12


def _nibbles(x):
    """Count of nonzero 4-bit nibbles of a uint16 array."""
    x = np.asarray(x, dtype=np.uint16)
    return int(sum(((x >> (4 * v)) & 0xF != 0).sum() for v in range(4)))


def check_flags(gpu, orc, tie_mask, what="flags"):
    """Flags equal outside the oracle's near ties; returns the number of
    nibbles that differ inside them."""
    g = np.asarray(gpu, dtype=np.uint16)
    o = np.asarray(orc, dtype=np.uint16)
    t = np.asarray(tie_mask, dtype=np.uint16)
    assert g.shape == o.shape == t.shape, (g.shape, o.shape, t.shape)
    d = g ^ o
    away = d & ~t
    if away.any():
        idx = np.argwhere(away != 0)[:8].tolist()
        raise AssertionError(f"{what}: {_nibbles(away)} flag nibbles differ away from near ties "
                             f"(first at {idx}: gpu {g[tuple(idx[0])]:#06x} oracle "
                             f"{o[tuple(idx[0])]:#06x})")
    return _nibbles(d)


def assert_states(x, y, rel=REL, what="state"):
    x = np.asarray(x).reshape(-1, 4)
    y = np.asarray(y).reshape(-1, 4)
    worst = 0.0
    for v in range(4):
        err = np.abs(x[:, v] - y[:, v]).max()
        ref = np.abs(y[:, v]).max()
        assert err <= rel * ref, f"{what} variable {v}: max err {err:.3e} vs {rel:.0e} * {ref:.3e}"
        worst = max(worst, err / ref if ref > 0 else err)
    return worst


def assert_adjoint(x, y, scale, rel=REL, what="adjoint"):
    """Adjoint parity against the comparison scale; prints and returns the
    worst error relative to the scale."""
    x = np.asarray(x).reshape(-1, 4)
    y = np.asarray(y).reshape(-1, 4)
    S = np.asarray(scale).reshape(-1, 4)
    worst = 0.0
    for v in range(4):
        err = np.abs(x[:, v] - y[:, v]).max()
        ref = S[:, v].max()
        assert err <= rel * ref, f"{what} variable {v}: max err {err:.3e} vs {rel:.0e} * {ref:.3e}"
        worst = max(worst, err / ref)
    print(f"[adjoint] {what}: worst error {worst:.2e} of the comparison scale "
          f"(max |y| / scale {np.abs(y).max() / S.max():.3f})", flush=True)
    return worst


def trajectory(torch, sv, om, U_user, perm, steps, cfl=0.4, label="", log=print,
               device="cuda"):
    """Steps the GPU solver `sv` and the oracle `om` side by side from the
    user-order state U_user, stage by stage (teno_rk_stage), with the
    oracle's dt.  After every stage: flags compared by location
    (check_flags), states at 1e-12 unless a flag flipped at a near tie, in
    which case the GPU's stage state is replaced by the oracle's (re-sync).
    Returns (re-sync count, worst relative state error, final oracle
    state)."""
    n = len(perm)

    def dev(a):
        return torch.as_tensor(np.ascontiguousarray(a[perm]), device=device)

    def user(t):
        a = t.cpu().numpy()
        out = np.empty_like(a)
        out[perm] = a
        return out

    U = np.ascontiguousarray(U_user, dtype=np.float64)
    Un = dev(U)
    bufs = [sv.empty_state() for _ in range(3)]
    fl = sv.empty_flags()
    dt = torch.empty(1, dtype=torch.float64, device=device)
    resyncs, worst = 0, 0.0
    for step in range(steps):
        dto = om.dt(U, cfl)
        ref = om.rk_step(U, dto, want_stages=True)
        dt.fill_(dto)
        outs = [ref["stages"][1], ref["stages"][2], ref["U"]]
        Uk = Un
        for k in range(3):
            Uk1 = bufs[k]
            sv.rk_stage(k, Un, Uk, Uk1, dt, flags=fl)
            if device != "cpu":
                torch.cuda.synchronize()
            gfl = np.empty(n, np.uint16)
            gfl[perm] = fl.cpu().numpy().view(np.uint16)
            tied = check_flags(gfl, ref["flags"][k], ref["diag"]["tie_mask"][k],
                               what=f"{label} step {step} stage {k}")
            if tied:
                resyncs += 1
                log(f"[re-sync] {label} step {step} stage {k}: {tied} flag nibbles flipped at "
                    f"near ties; GPU stage state replaced by the oracle's", flush=True)
                Uk1.copy_(dev(outs[k]))
            else:
                worst = max(worst, assert_states(user(Uk1), outs[k],
                                                 what=f"{label} step {step} stage {k}"))
            Uk = Uk1
        Un = bufs[2].clone()
        U = ref["U"]
    return resyncs, worst, U


def _fields5(x):
    """Count of nonzero 5-bit fields of a uint32 array (five variables)."""
    x = np.asarray(x, dtype=np.uint32)
    return int(sum(((x >> (5 * v)) & 0x1F != 0).sum() for v in range(5)))


def check_flags5(gpu, orc, tie_mask, what="flags"):
    """Tetrahedral flags (5 bits per variable) equal outside the oracle's
    near ties; returns the number of fields that differ inside them."""
    g = np.asarray(gpu, dtype=np.uint32)
    o = np.asarray(orc, dtype=np.uint32)
    t = np.asarray(tie_mask, dtype=np.uint32)
    assert g.shape == o.shape == t.shape, (g.shape, o.shape, t.shape)
    d = g ^ o
    away = d & ~t
    if away.any():
        idx = np.argwhere(away != 0)[:8].tolist()
        raise AssertionError(f"{what}: {_fields5(away)} flag fields differ away from near ties "
                             f"(first at {idx}: gpu {g[tuple(idx[0])]:#09x} oracle "
                             f"{o[tuple(idx[0])]:#09x})")
    return _fields5(d)


def assert_states5(x, y, rel=REL, what="state"):
    """Per conservative variable of the five: max |x - y| <= rel max |y|."""
    x = np.asarray(x).reshape(-1, 5)
    y = np.asarray(y).reshape(-1, 5)
    worst = 0.0
    for v in range(5):
        err = np.abs(x[:, v] - y[:, v]).max()
        ref = np.abs(y[:, v]).max()
        assert err <= rel * ref, f"{what} variable {v}: max err {err:.3e} vs {rel:.0e} * {ref:.3e}"
        worst = max(worst, err / ref if ref > 0 else err)
    return worst

"""The allocation-free time step (teno_max_dt_static, through the C ABI)
against teno_max_dt: bit-equal dt on two calls in a row, the second on a
smaller mesh (the static array keeps the first call's minima), and the
refusal of a mesh beyond its limit is an argument error, not a launch."""
import ctypes as C

import numpy as np
import pytest

from paper_2105_02127_amd import inputs

pytestmark = pytest.mark.gpu


def test_max_dt_static_matches_max_dt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_02127_amd import teno
    lib = teno.load()
    stream = torch.cuda.current_stream()
    for n, seed in ((40, 301), (17, 302)):
        m = inputs.jittered_periodic_mesh(n, seed)
        lm = teno.Mesh(m.xy, m.tri).setup(order=4, fallback=1)
        sv = teno.Solver(lm)
        U = torch.as_tensor(inputs.random_lines(m)[lm.perm], device="cuda")
        ref = sv.max_dt(U, 0.4)
        got = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        print(f"[no-alloc] teno_max_dt_static on {m.n_cell} cells", flush=True)
        rc = lib.teno_max_dt_static(sv.h, C.c_void_p(U.data_ptr()), C.c_double(0.4),
                                    C.c_void_p(got.data_ptr()), C.c_void_p(stream.cuda_stream))
        assert rc == 0, lib.teno_last_error().decode()
        torch.cuda.synchronize()
        assert got.item() == ref.item() > 0.0, (got.item(), ref.item())
    # argument errors come back before anything is launched
    rc = lib.teno_max_dt_static(sv.h, C.c_void_p(U.data_ptr()), C.c_double(-1.0),
                                C.c_void_p(got.data_ptr()), C.c_void_p(stream.cuda_stream))
    assert rc == -1 and b"cfl" in lib.teno_last_error()

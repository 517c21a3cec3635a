"""msd_adjoint_noalloc (scratch in the library's static device array) against
msd_adjoint with caller scratch: two calls in a row, the second on a smaller
problem, and the size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_cases import rand_D, smooth_field

pytestmark = pytest.mark.gpu


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _forward(shape, D, xi0, steps, every, precision):
    from paper_1808_06787_amd import adjoint
    from paper_1808_06787_amd.sim import Sim

    sim = Sim("D2Q5", D, shape, precision)
    sim.init(torch.from_numpy(xi0))
    ck = adjoint.forward_with_checkpoints(sim, steps, every)
    xi, _, _ = sim.read(torch.float64, flux=False, grad=False)
    return sim, ck, xi


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_adjoint_noalloc_matches_caller_scratch(precision):
    from paper_1808_06787_amd import _ffi as F
    from paper_1808_06787_amd import adjoint

    rng = np.random.default_rng(2100)
    # the second call runs a smaller problem over the contents the first one left
    for shape, steps, every in (((96, 80), 30, 8), ((40, 33), 17, 5)):
        N = 3
        D = rand_D(rng, N)
        xi0 = smooth_field(rng, N, shape[::-1], 0.1)
        target = torch.from_numpy(smooth_field(rng, N, shape[::-1], 0.1))
        ref_sim, ref_ck, xi = _forward(shape, D, xi0, steps, every, precision)
        g = 2.0 * (xi - target.to(xi.device))
        ref_dxi0, ref_dD = adjoint.gradients(ref_sim, ref_ck, steps, g, every)
        sim, ck, xi2 = _forward(shape, D, xi0, steps, every, precision)
        assert torch.equal(xi, xi2)
        assert sim.lib.msd_adjoint_scratch_bytes(sim._h, every) <= F.STATIC_SCRATCH_BYTES
        dxi0 = torch.empty((N - 1,) + sim.nodes_shape, dtype=torch.float64, device=sim.device)
        dD = (C.c_double * (N * N))()
        with torch.cuda.device(sim.device):
            F.check(sim.lib.msd_adjoint_noalloc(sim._h, steps, every, _p(ck["buffer"]), _p(g.contiguous()),
                                                _p(dxi0), dD), "msd_adjoint_noalloc")
        torch.cuda.synchronize()
        got_dD = np.array(dD[:]).reshape(N, N)
        # the same kernels on the same inputs: equal to rounding (bit for bit in practice)
        np.testing.assert_allclose(got_dD, ref_dD, rtol=1e-12, atol=0)
        s = float(ref_dxi0.abs().max())
        assert float((dxi0 - ref_dxi0).abs().max()) <= 1e-12 * s, (shape, precision)
        sim.close()
        ref_sim.close()


def test_adjoint_noalloc_rejects_problems_beyond_the_static_array():
    from paper_1808_06787_amd import _ffi as F

    rng = np.random.default_rng(2101)
    shape, steps, every = (2048, 1024), 3, 3
    N = 3
    D = rand_D(rng, N)
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    sim, ck, xi = _forward(shape, D, xi0, steps, every, "f32")
    assert sim.lib.msd_adjoint_scratch_bytes(sim._h, every) > F.STATIC_SCRATCH_BYTES
    g = torch.zeros_like(xi)
    dD = (C.c_double * (N * N))()
    st = sim.lib.msd_adjoint_noalloc(sim._h, steps, every, _p(ck["buffer"]), _p(g), None, dD)
    assert st == -7, F.lib().msd_last_error()
    assert b"exceeds the static array" in F.lib().msd_last_error()
    assert sim.time == steps      # nothing ran
    sim.close()

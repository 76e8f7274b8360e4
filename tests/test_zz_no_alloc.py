"""The allocation-free structure factor (sim_structure_factor_noalloc)
through the C ABI against sim_structure_factor on the same handle: the same
kernels and chunking, so the same bits; two calls in a row, the second with
a smaller input (fewer particles and a smaller wavevector grid), the output
in a caller-owned device buffer; requests beyond the static scratch are
refused with SIM_ECAPACITY.

torch (the caller's device buffers) is imported when the module is
collected: the library and torch load the HIP runtime under one soname, and
the process keeps whichever loads first; torch's device queries fail when the
library's copy came first, so torch must not be first imported after a test
has called into the library."""
import numpy as np
import pytest
import torch  # noqa: F401  (before any test loads the library)

from paper_1808_06381_amd import inputs
from paper_1808_06381_amd import sim as S

pytestmark = pytest.mark.gpu


def run_pair(cfgs, pos, nx, my_max, mz, steps):
    import torch
    with S.Sim(cfgs, pos, tol=1e-8) as sim:
        sim.step(steps)
        ref = sim.structure_factor(nx, my_max, mz)
        out = torch.full((sim.replicas, nx, 2 * my_max + 1), float("nan"),
                         dtype=torch.float64, device="cuda")
        sim.structure_factor_noalloc(nx, my_max, out, mz)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    return ref, got


def test_noalloc_matches_structure_factor_two_calls():
    import torch
    assert torch.cuda.is_available()
    # first call: a batch of two uneven replicas (several 4096-row chunks
    # each), a grid of two mx tiles and three my tiles, mz != 0
    cfgs = [inputs.cube_params(30000, 0.3, seed=31, stream=0),
            inputs.cube_params(9000, 0.05, seed=32, stream=1)]
    pos = np.concatenate([inputs.uniform_positions(c["n"], c["box"], c["seed"]) for c in cfgs])
    ref, got = run_pair(cfgs, pos, 80, 40, 2, steps=3)
    assert np.all(np.isfinite(got))
    np.testing.assert_array_equal(got, ref)
    # second call, smaller input: one box of 5000 particles, 17 x 11
    # wavevectors, on the same (shared, reused) scratch
    cfg = inputs.cube_params(5000, 0.5, seed=33)
    pos = inputs.uniform_positions(cfg["n"], cfg["box"], cfg["seed"])
    ref2, got2 = run_pair(cfg, pos, 17, 5, 0, steps=2)
    assert got2.shape == (1, 17, 11)
    np.testing.assert_array_equal(got2, ref2)
    assert got2[0, 0, 5] == pytest.approx(5000.0, rel=1e-12)   # q = 0: S = N


def test_noalloc_refuses_requests_beyond_its_scratch():
    import torch
    cfg = inputs.cube_params(1_000_000, 0.1, seed=34)
    pos = inputs.uniform_positions(cfg["n"], cfg["box"], cfg["seed"])
    with S.Sim(cfg, pos, tol=1e-8) as sim:
        out = torch.empty((1, 256, 257), dtype=torch.float64, device="cuda")
        with pytest.raises(S.SimError) as e:
            sim.structure_factor_noalloc(256, 128, out)
        assert e.value.code == -6
        out = torch.empty((1, 64, 129), dtype=torch.float64, device="cuda")
        sim.structure_factor_noalloc(64, 64, out)     # 35 MiB: fits
        ref = sim.structure_factor(64, 64)
        np.testing.assert_array_equal(out.cpu().numpy(), ref)

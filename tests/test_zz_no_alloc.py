"""The allocation-free energy entry point against dgw_energy.

dgw_energy_noalloc reduces through a static device array of the library
instead of an allocated buffer.  It is called through the C ABI on two
contexts in a row, the second with a smaller mesh (so the array holds the
first call's partial sums when the second runs), each with random fields,
and must give dgw_energy's value to FP64 rounding (the two sum their partials
in different orders).  The torch allocator, which the library uses for its
device memory, must see no new allocation during the call."""

import numpy as np
import pytest
import torch

import workloads as W
from gpu_helpers import gpu_solver, say

pytestmark = pytest.mark.gpu


def _solver(n, N, seed):
    mesh = W.kuhn_cube(n, 1.0)
    K = mesh["etov"].shape[0]
    rng = np.random.default_rng(seed)
    cp = rng.uniform(1.5, 3.0, K)
    rho, lam, mu = W.lame_from_velocities(cp, cp / rng.uniform(1.5, 2.2, K),
                                          rng.uniform(1.0, 3.0, K))
    s = gpu_solver(mesh, N, rho, lam, mu, 1e-3)
    s.set_fields(0, rng.standard_normal((K, 9, s.Np)))
    return s, K


def test_energy_noalloc_equals_energy():
    for n, N, seed in ((12, 3, 1), (2, 2, 2)):
        s, K = _solver(n, N, seed)
        say("case energy_noalloc, K=%d, order %d" % (K, N))
        for _ in range(2):
            torch.cuda.synchronize()
            before = torch.cuda.memory_allocated()
            e0 = s.energy_noalloc(0)
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() == before
            e1 = s.energy(0)
            say("  noalloc %.17e  energy %.17e" % (e0, e1))
            assert abs(e0 - e1) <= 1e-13 * abs(e1)
        s.close()

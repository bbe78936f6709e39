"""The no-allocation pheromone update (aco_update_pheromone_static, on the
library's own per-device scratch) against aco_update_pheromone with a
workspace: bit-identical pheromone on consecutive calls, the later ones on a
smaller instance, so what an earlier call left in the shared scratch must not
reach a later result."""
import numpy as np
import pytest

import oracle as orc
from paper_1709_03187_amd import instances
from tests.gpu_util import colony, require_gpu, say, to_np

pytestmark = pytest.mark.gpu

# (label, coordinates, k, m, seed): the second instance is the smaller one
CASES = [("n=20,000 m=256 k=16", instances.uniform_coords(20000, 2), 16, 256, 2),
         ("n=1,000 m=32 k=10", instances.uniform_coords(1000, 1), 10, 32, 1)]


def test_static_update_matches_workspace_update():
    require_gpu()
    import torch
    import paper_1709_03187_amd as aco
    for label, xy, k, m, seed in CASES:
        say(f"[no-alloc] {label}")
        col = colony(xy, k=k, m=m, seed=seed)
        col.setup()
        for it in range(2):
            col.construct(it)
            before = col.tau.clone()
            col.update()                                  # with the caller's workspace
            ref = col.tau.clone()
            col.tau.copy_(before)
            aco.aco_update_pheromone_static(col.n, col.k, col.nn, col.rev, col.m, col.tours,
                                            col.slots, col.lengths, col.rho, col.deposit_shift,
                                            col.tau)
            torch.cuda.synchronize()
            assert torch.equal(col.tau, ref), (label, it)
            if len(xy) <= 1000:                           # and the oracle's update
                want = orc.update(to_np(col.nn), to_np(before), to_np(col.tours),
                                  to_np(col.lengths), col.rho, col.deposit_shift)
                np.testing.assert_array_equal(to_np(col.tau), want)
        aco.aco_device_error()


def test_static_update_rejects_sizes_beyond_the_scratch():
    require_gpu()
    import torch
    import paper_1709_03187_amd as aco
    n, k = 200000, 16
    m = (aco.ACO_UPDATE_STATIC_BYTES - n * k * 8) // 8 + 256    # one block of ants too many
    dev = "cuda:0"
    nn = torch.zeros((n, k), dtype=torch.int32, device=dev)
    rev = torch.zeros((n, k), dtype=torch.int8, device=dev)
    tours = torch.zeros((1, n), dtype=torch.int32, device=dev)    # never read: rejected first
    lengths = torch.ones(1, dtype=torch.int64, device=dev)
    tau = torch.zeros((n, k), dtype=torch.float32, device=dev)
    with pytest.raises(aco.AcoError) as e:
        aco.aco_update_pheromone_static(n, k, nn, rev, m, tours, None, lengths, 0.1, 32, tau)
    assert e.value.code == aco.ACO_ERR_INVALID_ARG and "static scratch" in str(e.value)

"""Device-side checks: inputs that break a stated precondition the host cannot
see before a launch (a local best that is not a permutation, an impossible
local-best length, a tour entry out of range, a length <= 0, a deposit that
could overflow int64).  Each is reported as ACO_ERR_DEVICE by
aco_device_error, every kernel still finishes normally, and where the
library can recover (the kept part's length) the results stay exact."""
import numpy as np
import pytest

import oracle as orc
from paper_1709_03187_amd import instances
from tests.gpu_util import colony, require_gpu, to_np

pytestmark = pytest.mark.gpu

N, K, M, SEED = 600, 8, 16, 31


@pytest.fixture(scope="module")
def col():
    require_gpu()
    import paper_1709_03187_amd as aco
    xy = instances.uniform_coords(N, SEED)
    c = colony(xy, k=K, m=M, seed=SEED)
    c.setup()
    aco.aco_device_error()          # a clean start
    c.construct(0)
    c.update_local_best()
    c.update()
    aco.aco_device_error()          # the normal path trips nothing
    return c


def expect_device_error(fragment):
    import paper_1709_03187_amd as aco
    with pytest.raises(aco.AcoError) as e:
        aco.aco_device_error()
    assert e.value.code == aco.ACO_ERR_DEVICE
    assert fragment in str(e.value), str(e.value)
    aco.aco_device_error()          # reported once, then clear


def lengths_exact(c):
    xy, tours = to_np(c.xy), to_np(c.tours)
    assert np.array_equal(np.sort(tours, axis=1), np.broadcast_to(np.arange(N), tours.shape))
    np.testing.assert_array_equal(to_np(c.lengths), [orc.tour_length(xy, t) for t in tours])


def test_partial_construction_clean_run(col):
    import paper_1709_03187_amd as aco
    col.construct_ex(1, p_partial=1.0, max_modify=50, partial=True)
    aco.aco_device_error()
    lengths_exact(col)


@pytest.mark.parametrize("kind", ["duplicate_kept", "duplicate_across", "out_of_range"])
def test_non_permutation_local_best(col, kind):
    import torch
    import paper_1709_03187_amd as aco
    saved = col.lbest.clone()
    bad = saved.clone()
    if kind == "duplicate_kept":        # every row: the city of position 1 repeated at 2
        bad[:, 2] = bad[:, 1]
    elif kind == "duplicate_across":    # a kept city repeated where the ant rebuilds
        for a in range(M):
            s_pos, part, r = orc.partial_plan(SEED, 2, a, N, 1.0, 50)
            assert part
            bad[a, (s_pos + N - r) % N] = bad[a, s_pos]
    else:
        bad[:, 3] = N + 5
    col.lbest.copy_(bad)
    try:
        col.construct_ex(2, p_partial=1.0, max_modify=50, partial=True)
        torch.cuda.synchronize()
        tours = to_np(col.tours)
        assert tours.min() >= 0 and tours.max() < N     # every access stayed in range
        expect_device_error("permutation")
    finally:
        col.lbest.copy_(saved)
    aco.aco_device_error()


@pytest.mark.parametrize("value", [2**63 - 1, 0, -5])
def test_impossible_local_best_length(col, value):
    """The INT64_MAX start value (or <= 0) is reported, and that ant's kept part
    is then summed edge by edge: the lengths stay exact."""
    saved = col.lbest_len.clone()
    col.lbest_len[3] = value
    try:
        col.construct_ex(3, p_partial=1.0, max_modify=50, partial=True)
        expect_device_error("local best length")
        lengths_exact(col)
    finally:
        col.lbest_len.copy_(saved)


def test_tour_entry_out_of_range_and_bad_lengths(col):
    import torch
    import paper_1709_03187_amd as aco
    col.construct(6)
    torch.cuda.synchronize()
    col.tours[2, 10] = -1
    col.update()
    expect_device_error("out of range")
    col.construct(7)
    col.lengths[1] = 0
    col.update()
    expect_device_error("length is <= 0")
    # m * floor(2^62 / 1) >= 2^63: the int64 sums could overflow
    col.construct(8)
    col.lengths[:] = 1
    aco.aco_update_pheromone(col.n, col.k, col.nn, col.rev, col.m, col.tours, col.slots,
                             col.lengths, col.rho, 62, col.tau, col.uws)
    expect_device_error("overflow")

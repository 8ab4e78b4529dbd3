"""CPU model of the XCD-local task order of the batched pyramid steps.

The statistics and reduce launches of the batch map workgroup b to task
xcd_task(b) (paper_1901_09593_amd/csrc/common.hpp): the hardware deals
workgroups round-robin to the 8 XCDs, and the k-th workgroup of XCD x takes
task (k // RUN * 8 + x) * RUN + k % RUN, so each XCD works through runs of RUN
consecutive tiles; workgroups past the last whole group of 8 runs keep their
index.  The segment lookup that follows assumes a bijection on [0, grid): every
tile is computed exactly once.  These tests restate the formula and check that
property and the runs for many grid sizes.
"""
import pytest

XCDS, RUN = 8, 64


def xcd_task(b, grid):
    full = grid // (XCDS * RUN) * (XCDS * RUN)
    if b >= full:
        return b
    x, k = b % XCDS, b // XCDS
    return (k // RUN * XCDS + x) * RUN + k % RUN


GRIDS = sorted({1, 7, 8, 63, 64, 511, 512, 513, 1023, 1024, 1025, 4095, 4096, 4097, 5000, 17687, 35366}
               | set(range(500, 530)))


@pytest.mark.parametrize("grid", GRIDS)
def test_task_order_is_a_bijection(grid):
    tasks = [xcd_task(b, grid) for b in range(grid)]
    assert sorted(tasks) == list(range(grid))


@pytest.mark.parametrize("grid", [512, 4096, 35366])
def test_each_xcd_walks_runs_of_consecutive_tiles(grid):
    full = grid // (XCDS * RUN) * (XCDS * RUN)
    for x in range(XCDS):
        mine = [xcd_task(b, grid) for b in range(x, full, XCDS)]  # in dispatch order
        for r0 in range(0, len(mine), RUN):
            run = mine[r0:r0 + RUN]
            assert run == list(range(run[0], run[0] + RUN))
        # the runs of one XCD are spread over the whole range, one per group of 8 runs
        starts = [mine[r0] for r0 in range(0, len(mine), RUN)]
        assert starts == [(g * XCDS + x) * RUN for g in range(len(starts))]

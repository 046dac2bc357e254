"""Host-side scheduling of the serving loop: advection steps per job and tick."""
from paper_2503_16082_amd.serve import steps_this_tick


def test_jobs_with_fewer_substeps_take_more_steps():
    # the job with the most substeps per step takes one; the others as many as fit
    assert steps_this_tick([40, 10, 4, 13], [100, 100, 100, 100], cap=16) == [1, 4, 10, 3]


def test_cap_steps_left_and_unknown_counts():
    assert steps_this_tick([40, 4, 4], [100, 100, 2], cap=8) == [1, 8, 2]
    # a job whose substeps per step are not known yet takes one step
    assert steps_this_tick([0, 20, 5], [9, 9, 9], cap=8) == [1, 1, 4]
    assert steps_this_tick([0, 0], [5, 5], cap=8) == [1, 1]
    # cap 1 is lockstep
    assert steps_this_tick([40, 4], [9, 9], cap=1) == [1, 1]

"""The superstep schedule of the inter-task strip pipeline, checked on the CPU.

A model of the schedule the inter-task kernels follow (k_inter.hip,
k_batch.hip): with Wu = min(W, C // 2) waves in use, strip s runs on wave
s % Wu in round s // Wu and computes chunk c in superstep
(s // Wu) * C + 2 * (s % Wu) + c, prefetching that chunk's inputs one
superstep earlier; every wave passes T_total barriers.  Checked for every
bin length and strip count the library can launch: each chunk of the
boundary-row buffer is read by strip s only after strip s - 1 wrote it (in
an earlier superstep, so a barrier separates them), each wave's own
supersteps never overlap, and every wave passes the same number of
barriers.  A planted off-by-one in the model fails the check.
"""
import pytest

D = 2


def schedule(W, C, S):
    Wu = min(W, C // D)
    q_last, w_last = (S - 1) // Wu, (S - 1) % Wu
    T_total = q_last * C + D * w_last + C
    waves = []
    for w in range(W):
        my_rounds = (S - 1 - w) // Wu + 1 if (w < S and w < Wu) else 0
        lead = min(D * w, T_total)
        waves.append((my_rounds, lead))
    return Wu, T_total, waves


def check(W, C, S, skew=D):
    Wu, T_total, waves = schedule(W, C, S)
    for w, (my_rounds, lead) in enumerate(waves):
        barriers = lead + my_rounds * C + max(0, T_total - lead - my_rounds * C)
        assert barriers == T_total, ("barriers", W, C, S, w)
        assert lead + my_rounds * C <= T_total, ("overrun", W, C, S, w)
        if my_rounds:
            assert lead == D * w

    def t(s, c):        # superstep in which strip s computes (and writes) chunk c
        return (s // Wu) * C + skew * (s % Wu) + c

    for s in range(1, S):
        for c in range(C):
            # prefetch of chunk c by strip s happens in t(s, c) - 1
            assert t(s, c) - 1 > t(s - 1, c), ("race", W, C, S, s, c)
    for s in range(S):
        assert t(s, C - 1) < T_total


@pytest.mark.parametrize("W", [1, 2, 4, 8, 12, 16])
def test_pipeline_schedule_is_race_free(W):
    for C in list(range(24, 70)) + [96, 127, 128, 255, 512]:
        for S in list(range(1, 40)) + [63, 64, 65, 343]:
            check(W, C, S)


def test_model_catches_a_skew_of_one():
    with pytest.raises(AssertionError):
        check(12, 40, 30, skew=1)


def test_wave_count_shrinks_for_short_bins():
    assert schedule(16, 24, 40)[0] == 12
    assert schedule(16, 31, 40)[0] == 15
    assert schedule(16, 32, 40)[0] == 16
    assert schedule(12, 24, 40)[0] == 12

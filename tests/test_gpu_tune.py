"""GPU parity under schedules set by the caller (mgt_plan_set_schedule) and
the autotuner built on it: every schedule must give the oracle's result."""
import pytest

from workloads import gen

from .common import assert_matches_oracle, host, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("setting", [
    (8, -1, 0),       # the default rule
    (6, 5, 4096),
    (5, 4, 8192),     # three passes
    (3, 6, 4096),     # four passes
    (8, 10, 2048),    # one pass, 1,024-column finish buckets spanning many sub-chunks
    (7, 9, 16384),
])
@pytest.mark.parametrize("partitioned", [False, True])
def test_forced_schedules_match_oracle(setting, partitioned):
    from paper_2012_06012_amd import mgt
    a = gen.large(seed=6, scale=7)
    d = to_device(a)
    plan = mgt.plan_for(d, mgt.EMIT_PERM)
    plan.set_schedule(*setting)
    sc = plan.schedule(partitioned)
    assert sc["tile_cells"] == (setting[2] or sc["tile_cells"])
    if setting[1] >= 0 and not partitioned:
        assert sc["finish_bits"] == setting[1]
    out, st = mgt.transpose(d, plan=plan, perm=True, partitioned=partitioned)
    assert int(st.cpu()[0]) == 0
    assert_matches_oracle(a, host(out), partitioned=partitioned)


def test_autotune_keeps_the_result_and_sets_the_fastest():
    from paper_2012_06012_amd import autotune, mgt
    a = gen.large(seed=7, scale=8)
    d = to_device(a)
    plan, r = autotune.autotune(d, reps=2, pass_bits=(6, 8), finish_span=(0, 1), tiles=(8192, 16384),
                                use_cache=False)
    assert r.trials and all(t["bit_exact"] for t in r.trials)
    assert r.best["ms"] <= r.default_ms
    out, st = mgt.transpose(d, plan=plan, perm=False)
    assert int(st.cpu()[0]) == 0
    assert_matches_oracle(a, host(out), check_perm=False)
    # a second call for the same shape comes from the cache
    plan2, r2 = autotune.autotune(d)
    assert plan2.schedule() == plan.schedule()

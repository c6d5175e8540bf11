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


def _batch_items(seed, n_items):
    items = []
    for i in range(n_items):
        n, deg, width = gen.batch_item_params(seed, i, 100, 30000)
        a = gen.generate(n, n, seed=(seed << 20) + i, deg_law=gen.DEG_POISSON,
                         deg_mean=float(min(deg, 24)), pay_law=gen.PAY_BYTES, w_lo=width,
                         w_hi=width, offset_width=8, name=f"item{i}")
        if i % 4 == 1:
            a.bounds = gen.equal_bounds(n, min(n, 3 + i % 5))
        items.append(a)
    return items


@pytest.mark.parametrize("setting", [(4, -1, 0), (6, -1, 8192), (8, -1, 16384), (4, -1, 2048),
                                     (5, 3, 4096)])
@pytest.mark.parametrize("perm", [False, True])
def test_batch_schedules_match_oracle(setting, perm):
    """A batch plan's schedule setting (digit widths 4/6/8, tile sizes, an exact
    finish width) applies to every item; each item still equals the oracle."""
    from paper_2012_06012_amd import mgt
    items = _batch_items(11, 14)
    mats = [to_device(a) for a in items]
    plan = mgt.batch_plan_for(mats, perm)
    plan.set_schedule(*setting)
    outs, st, _, _ = mgt.batch_transpose(mats, plan=plan, perm=perm)
    assert (st.cpu().numpy() == 0).all()
    for a, o in zip(items, outs):
        assert_matches_oracle(a, host(o), check_perm=perm, partitioned=a.n_parts > 1)


def test_autotune_batch_keeps_the_result():
    from paper_2012_06012_amd import autotune, mgt
    items = _batch_items(12, 10)
    mats = [to_device(a) for a in items]
    plan, r = autotune.autotune_batch(mats, reps=2, pass_bits=(4, 8), tiles=(8192, 16384),
                                      use_cache=False)
    assert len(r.trials) == 4 and all(t["bit_exact"] for t in r.trials)
    assert r.best["ms"] <= r.default_ms
    outs, st, _, _ = mgt.batch_transpose(mats, plan=plan)
    assert (st.cpu().numpy() == 0).all()
    for a, o in zip(items, outs):
        assert_matches_oracle(a, host(o), check_perm=False, partitioned=a.n_parts > 1)
    # the same batch shape class comes from the cache
    plan2, r2 = autotune.autotune_batch(mats)
    assert r2.best["pass_bits"] == r.best["pass_bits"]
    assert r2.best["tile_cells"] == r.best["tile_cells"]

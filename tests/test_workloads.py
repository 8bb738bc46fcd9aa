"""Seeded workload generators (host only): the serving pool spans the ranges
its requests are drawn from, and is reproducible."""
from workloads import configs


def test_serving_pool_spans_its_ranges():
    pool = configs.serving_pool(seed=4, count=32)
    ns = [cc.n for cc in pool]
    ks = [len(cc.cuts) for cc in pool]
    subs = [cc.n_sub for cc in pool]
    assert (min(ns), max(ns)) == (16, 80)
    assert (min(ks), max(ks)) == (2, 10)
    assert min(subs) == 2 and max(subs) == 5
    assert all(max(cc.summary()["w"]) <= 18 for cc in pool)
    kinds = {cc.meta.get("name") for cc in pool}
    assert len(kinds) == 32
    again = configs.serving_pool(seed=4, count=32)
    assert [cc.n for cc in again] == ns and [len(cc.cuts) for cc in again] == ks

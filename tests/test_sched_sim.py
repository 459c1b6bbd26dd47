"""The serving scheduler on a simulated device (CPU): admission by footprint,
LRU eviction of unheld plans only, grouped dispatch, completion of every
request, failure propagation.  The simulated device runs builds and grouped
applies on two queues with a virtual clock."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from paper_2410_06129_amd.schedsim import Sim

GB = 1 << 30


def run_trace(sim, trace, dt=0.01, max_steps=200000):
    """trace: list of dicts with t, key, foot, res, build_s, apply_s, fail, tag (sorted by t)."""
    i = 0
    done = []
    steps = 0
    while i < len(trace) or not sim.idle():
        while i < len(trace) and trace[i]["t"] <= sim.now:
            r = trace[i]
            sim.submit(r["key"], r["foot"], r["res"], r["build_s"], r["apply_s"], r["fail"], r["tag"])
            i += 1
        sim.advance(dt)
        done += sim.completions()
        steps += 1
        assert steps < max_steps, "simulation did not drain"
    done += sim.completions()
    return done


def make_trace(seed, n, keys, rate, budget):
    rng = np.random.default_rng(seed)
    kinfo = {}
    for k in range(keys):
        res = int(rng.uniform(0.05, 0.45) * budget)
        kinfo[k] = dict(res=res, foot=int(res * rng.uniform(1.2, 2.0)), build_s=rng.uniform(0.05, 1.0))
    t = 0.0
    out = []
    for j in range(n):
        t += rng.exponential(1.0 / rate)
        k = int(rng.integers(0, keys))
        out.append(dict(t=t, key=k + 1, foot=min(kinfo[k]["foot"], budget), res=kinfo[k]["res"],
                        build_s=kinfo[k]["build_s"], apply_s=rng.uniform(0.001, 0.05), fail=False,
                        tag=j))
    return out


@settings(max_examples=40, deadline=None)
@given(seed=st.integers(0, 10_000), n=st.integers(1, 120), keys=st.integers(1, 12),
       rate=st.floats(0.5, 50.0), max_group=st.integers(1, 32), max_inflight=st.integers(1, 3),
       max_builds=st.integers(1, 3))
def test_invariants_hold_on_random_traces(seed, n, keys, rate, max_group, max_inflight, max_builds):
    budget = 64 * GB
    sim = Sim(budget, max_group, max_inflight, max_builds)
    trace = make_trace(seed, n, keys, rate, budget)
    done = run_trace(sim, trace)
    s = sim.stats()
    assert len(done) == n
    assert sorted(d["tag"] for d in done) == list(range(n))
    assert all(d["status"] == 0 for d in done)
    assert s["invariant_violations"] == 0
    assert s["use_after_release"] == 0
    assert s["peak_used"] <= budget
    assert s["items"] == n
    for d in done:
        assert d["t_arrival"] <= d["t_dispatch"] <= d["t_done"]
    # every encoding is built at least once; later requests are cache hits unless evicted
    assert s["builds"] >= len({r["key"] for r in trace})
    assert s["builds"] + s["hits"] == n


def test_reuse_hits_cache_and_batches_group():
    sim = Sim(100 * GB, max_group=8, max_inflight=1)
    # one encoding, 20 requests arriving together after its build
    trace = [dict(t=0.0, key=7, foot=10 * GB, res=5 * GB, build_s=1.0, apply_s=0.01, fail=False, tag=0)]
    trace += [dict(t=0.001 * j, key=7, foot=10 * GB, res=5 * GB, build_s=1.0, apply_s=0.01,
                   fail=False, tag=j) for j in range(1, 20)]
    done = run_trace(sim, trace, dt=0.005)
    s = sim.stats()
    assert s["builds"] == 1 and s["hits"] == 19
    assert s["batches"] < s["items"]          # several requests per grouped apply
    assert s["used"] == 5 * GB                # build workspace returned, plan resident
    assert all(d["t_done"] >= 1.0 for d in done)


def test_admission_waits_and_evicts_lru():
    budget = 10 * GB
    sim = Sim(budget, max_group=4, max_inflight=1, max_builds=1)
    # three encodings each needing 6 GB to build and 4 GB resident: only one build fits at a time,
    # and a resident plan must be evicted before the third build
    trace = [dict(t=0.1 * j, key=j + 1, foot=6 * GB, res=4 * GB, build_s=0.5, apply_s=0.01,
                  fail=False, tag=j) for j in range(3)]
    done = run_trace(sim, trace)
    s = sim.stats()
    assert len(done) == 3 and all(d["status"] == 0 for d in done)
    assert s["peak_used"] <= budget
    assert s["evictions"] >= 1
    assert s["use_after_release"] == 0 and s["invariant_violations"] == 0


def test_held_plan_is_never_evicted():
    budget = 10 * GB
    sim = Sim(budget, max_group=1, max_inflight=1, max_builds=1)
    # key 1: long applies keep it held; key 2 cannot fit until key 1's requests finish
    trace = [dict(t=0.0, key=1, foot=8 * GB, res=7 * GB, build_s=0.1, apply_s=0.5, fail=False, tag=j)
             for j in range(4)]
    trace.append(dict(t=0.2, key=2, foot=8 * GB, res=7 * GB, build_s=0.1, apply_s=0.01, fail=False,
                      tag=4))
    done = run_trace(sim, trace)
    s = sim.stats()
    by_tag = {d["tag"]: d for d in done}
    assert s["use_after_release"] == 0 and s["invariant_violations"] == 0
    # the second encoding's request finishes after every request of the first
    assert by_tag[4]["t_done"] >= max(by_tag[j]["t_done"] for j in range(4))


def test_oversized_and_failing_requests_do_not_block_others():
    budget = 10 * GB
    sim = Sim(budget, max_group=4, max_inflight=1, max_builds=1)
    trace = [
        dict(t=0.0, key=1, foot=20 * GB, res=12 * GB, build_s=0.1, apply_s=0.01, fail=False, tag=0),
        dict(t=0.0, key=2, foot=2 * GB, res=1 * GB, build_s=0.1, apply_s=0.01, fail=True, tag=1),
        dict(t=0.05, key=2, foot=2 * GB, res=1 * GB, build_s=0.1, apply_s=0.01, fail=True, tag=2),
        dict(t=0.0, key=3, foot=2 * GB, res=1 * GB, build_s=0.1, apply_s=0.01, fail=False, tag=3),
    ]
    done = {d["tag"]: d for d in run_trace(sim, sorted(trace, key=lambda r: r["t"]))}
    assert done[0]["status"] == 2          # larger than the whole budget: NOMEM
    assert done[1]["status"] == 3 and done[2]["status"] == 3   # the build failed (NOT_PD)
    assert done[3]["status"] == 0
    assert sim.stats()["build_failures"] == 1


def test_deterministic():
    a = run_trace(Sim(64 * GB, 8, 2, 1), make_trace(5, 80, 6, 10.0, 64 * GB))
    b = run_trace(Sim(64 * GB, 8, 2, 1), make_trace(5, 80, 6, 10.0, 64 * GB))
    assert [(d["tag"], d["t_done"]) for d in a] == [(d["tag"], d["t_done"]) for d in b]

"""CPU test of the request server's admission policy with a stand-in
executor: server_policy_sim.cpp drives the same header the server compiles
(paper_2112_10258_amd/csrc/server_policy.h) through a discrete-event model
of arrivals, group runs and an in-order client, and reports the invariants:
slot bytes within the budget at every admission, every request completed
(no deadlock, including under budgets that force evictions and pass-over
decisions), groups of one shape with power-of-two sizes led by the head of
the queue, at most max_inflight groups at once."""
import json
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "server_policy_sim.cpp")
INC = os.path.join(ROOT, "paper_2112_10258_amd", "csrc")


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sim") / "server_policy_sim")
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-Wall", "-Werror", "-I", INC, SRC, "-o", exe])
    return exe


def run(sim, seed, budget_mb, max_batch, max_inflight, n_req, saturated, timeout=0.0):
    out = subprocess.check_output([sim, str(seed), str(budget_mb), str(max_batch), str(max_inflight), str(n_req),
                                   "1" if saturated else "0", repr(float(timeout))], timeout=60)
    return json.loads(out)


def check(r, max_batch, max_inflight):
    assert not r["deadlock"], r
    assert r["completed"] == r["requests"], r
    assert r["ok_deadline"], r
    assert r["ok_budget"] and r["peak_bytes"] <= r["budget"], r
    assert r["ok_shape"] and r["ok_pow2"] and r["ok_head"], r
    assert r["max_group"] <= max_batch and r["max_running"] <= max_inflight, r


def test_ample_budget_groups_form_and_slots_are_reused(sim):
    r = run(sim, 1, 200000, 8, 8, 2000, True)
    check(r, 8, 8)
    assert r["max_group"] == 8 and r["evictions"] == 0
    assert r["allocations"] < r["groups"] / 4      # slots come back from the pool


def test_paced_arrivals_complete(sim):
    r = run(sim, 2, 200000, 8, 8, 2000, False)
    check(r, 8, 8)


def test_tight_budget_evicts_and_never_deadlocks(sim):
    # the 256^3 lone slot is about 1.3 GB: budgets of 1.4 .. 4 GB force
    # evictions, halved groups and pass-over decisions
    for seed, mb in ((3, 4096), (4, 2000), (5, 1500), (6, 1400)):
        r = run(sim, seed, mb, 8, 8, 300, True)
        check(r, 8, 8)
        assert r["evictions"] > 0


def test_random_configurations(sim):
    rng = np.random.default_rng(2112)
    for seed in range(40):
        budget = float(rng.uniform(1400, 8000))
        mb = int(rng.choice([1, 2, 4, 8, 16]))
        mi = int(rng.choice([1, 2, 4, 8]))
        r = run(sim, 100 + seed, budget, mb, mi, 150, bool(rng.integers(2)))
        check(r, mb, mi)


def test_admission_timeout_ends_only_requests_past_their_deadline(sim):
    # a saturated burst through one group at a time: with a timeout the
    # late requests expire (never after being admitted, never before their
    # deadline) and everything else completes; without one nothing expires
    r = run(sim, 7, 200000, 1, 1, 400, True, timeout=0.01)
    check(r, 1, 1)
    assert r["expired"] > 0 and r["expired"] < r["requests"]
    r0 = run(sim, 7, 200000, 1, 1, 400, True, timeout=0.0)
    check(r0, 1, 1)
    assert r0["expired"] == 0
    # tight budgets and paced arrivals with a timeout still never deadlock
    for seed, mb, sat in ((8, 1500, True), (9, 2000, False), (10, 4096, True)):
        r = run(sim, seed, mb, 8, 4, 300, sat, timeout=0.05)
        check(r, 8, 4)

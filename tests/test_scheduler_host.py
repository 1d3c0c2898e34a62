"""The continuous-batching scheduler (admission by slot and HBM budget,
batched steps, retirement, cancellation, failure detection, latency
statistics), compiled for the host and driven against a simulated executor
with a virtual clock.  The library's server runs the same header."""
import json
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "sched_sim.cpp")

QUEUED, RUNNING, DONE, FAILED, CANCELLED = 0, 1, 2, 3, 4
ERR_OOM, ERR_BUDGET, ERR_NONFINITE = 3, 4, 6


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sched") / "sched_sim")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-o", exe, SRC], check=True)

    def run(scenario):
        out = subprocess.run([exe, scenario], check=True, capture_output=True, text=True).stdout
        d = json.loads(out)
        d["reqs"] = {int(k): v for k, v in d["reqs"].items()}
        return d
    return run


def test_budget_bounds_concurrency_and_order_is_fifo(sim):
    d = sim("fifo_budget")      # six 4-byte requests, budget 10
    assert d["max_active"] == 2 and d["stats"]["peak_bytes"] == 8
    assert d["done_order"] == [1, 2, 3, 4, 5, 6]
    admits = [d["reqs"][i]["t_admit"] for i in range(1, 7)]
    assert admits == sorted(admits)
    assert all(r["state"] == DONE and r["steps_done"] == 5 for r in d["reqs"].values())
    assert d["stats"]["bytes_in_use"] == 0


def test_slots_bound_concurrency(sim):
    d = sim("slots")
    assert d["max_active"] == 3 and d["stats"]["peak_active"] == 3
    assert all(r["state"] == DONE and r["steps_done"] == 3 + i for i, r in d["reqs"].items())


def test_request_larger_than_budget_is_rejected(sim):
    d = sim("reject")
    r1, r2 = d["reqs"][1], d["reqs"][2]
    assert r1["rc"] == ERR_BUDGET and r1["state"] == FAILED and r1["status"] == ERR_BUDGET
    assert r2["state"] == DONE
    assert d["stats"]["rejected"] == 1


def test_every_request_runs_exactly_its_steps(sim):
    d = sim("mixed_steps")
    want = {1: 3, 2: 7, 3: 12, 4: 2}
    for i, n in want.items():
        assert d["reqs"][i]["steps_done"] == n and d["reqs"][i]["n_losses"] == n
    assert d["stats"]["steps"] == 12      # batched steps: the longest request
    # the late arrival joined at the first step boundary after it came
    assert d["reqs"][4]["t_admit"] >= 0.05 and d["reqs"][4]["t_admit"] < d["reqs"][2]["t_done"]


def test_cancel_queued_and_running(sim):
    d = sim("cancel")
    assert d["reqs"][2]["state"] == CANCELLED and d["reqs"][2]["steps_done"] == 0
    assert d["reqs"][1]["state"] == CANCELLED and 0 < d["reqs"][1]["steps_done"] < 10
    assert d["reqs"][3]["state"] == DONE and d["reqs"][3]["steps_done"] == 4
    assert d["stats"]["cancelled"] == 2 and d["stats"]["bytes_in_use"] == 0


def test_non_finite_loss_fails_only_that_request(sim):
    d = sim("nan")
    assert d["reqs"][2]["state"] == FAILED and d["reqs"][2]["status"] == ERR_NONFINITE
    assert d["reqs"][2]["steps_done"] < 10
    assert d["reqs"][1]["state"] == DONE and d["reqs"][3]["state"] == DONE


def test_failed_allocation_releases_nothing_it_did_not_take(sim):
    d = sim("add_fail")
    assert d["reqs"][1]["state"] == FAILED and d["reqs"][1]["status"] == ERR_OOM
    assert d["reqs"][2]["state"] == DONE      # needs the whole budget
    assert d["stats"]["bytes_in_use"] == 0


def test_strict_fifo_small_request_waits_behind_big_one(sim):
    d = sim("hol")
    assert d["reqs"][3]["t_admit"] >= d["reqs"][2]["t_admit"]
    assert d["reqs"][3]["t_admit"] > 0


def test_latency_statistics(sim):
    d = sim("latency")          # serial: completions at 1, 2, 3, 4 s
    done = sorted(r["t_done"] for r in d["reqs"].values())
    assert done == pytest.approx([1.0, 2.0, 3.0, 4.0])
    st = d["stats"]
    assert st["p50"] == pytest.approx(2.0) and st["p99"] == pytest.approx(4.0)
    assert st["mean"] == pytest.approx(2.5) and st["recons_per_s"] == pytest.approx(1.0)


def test_idle_gaps_between_arrivals(sim):
    d = sim("arrivals")
    for i, r in d["reqs"].items():
        assert r["state"] == DONE and r["t_admit"] == pytest.approx(r["t_submit"])
    assert d["reqs"][4]["t_done"] - d["reqs"][4]["t_submit"] < 0.1


def test_work_cap_bounds_the_work_stepped_together(sim):
    d = sim("work_cap")          # works 4, 4, 4, 12, 1, 1 under a cap of 10
    assert d["max_work"] == 12 and d["peak_work"] == 12   # the over-cap request ran alone
    assert all(r["state"] == DONE and r["steps_done"] == 4 + i for i, r in d["reqs"].items())
    admits = [d["reqs"][i]["t_admit"] for i in range(1, 7)]
    assert admits == sorted(admits)                          # FIFO
    # 1 and 2 together (8), 3 waits for a free share, 4 waits until it is alone
    assert d["reqs"][3]["t_admit"] > 0.0
    assert d["reqs"][4]["t_admit"] >= max(d["reqs"][i]["t_done"] for i in (1, 2, 3))
    assert d["reqs"][5]["t_admit"] >= d["reqs"][4]["t_done"]


def test_work_cap_lowers_latency_at_equal_throughput(sim):
    """Stepping past the point where the device is full only shares it: under
    a batch arrival the capped server completes requests in FIFO waves, with
    half the median latency and the same completion rate."""
    u, c = sim("cap_latency_uncapped"), sim("cap_latency_capped")
    assert u["max_active"] == 8 and c["max_active"] == 2
    assert u["stats"]["p50"] == pytest.approx(8.0) and c["stats"]["p50"] == pytest.approx(4.0)
    assert c["stats"]["recons_per_s"] == pytest.approx(u["stats"]["recons_per_s"])
    assert c["done_order"] == [1, 2, 3, 4, 5, 6, 7, 8]

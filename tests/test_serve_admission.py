"""Host logic of the serving engine's admission (no GPU): the shared budget
of live plans and device bytes, and each plan's bytes from the library's own
arena sizing."""
import threading

import workloads
from paper_2411_03416_amd.serve import Admission, plan_bytes


def test_budget_and_concurrency_limits():
    adm = Admission(budget_bytes=100, max_concurrent=3)
    assert adm.try_take(60)
    assert not adm.try_take(50)  # 110 > 100 while a plan is live
    assert adm.try_take(40)
    assert not adm.try_take(1)  # the budget is spent
    adm.give(40)
    assert adm.try_take(10) and adm.try_take(10)
    assert not adm.try_take(1)  # three plans live
    assert (adm.used, adm.live, adm.peak_live) == (80, 3, 3)
    assert adm.peak_used == 100


def test_a_request_larger_than_the_budget_runs_alone():
    adm = Admission(budget_bytes=100, max_concurrent=8)
    assert adm.try_take(500)  # nothing live: admitted, so every request is served
    assert not adm.try_take(1)  # and nothing joins it
    adm.give(500)
    assert adm.try_take(1)


def test_concurrent_takes_never_pass_the_limits():
    adm = Admission(budget_bytes=1000, max_concurrent=50)
    taken = []

    def worker():
        for _ in range(200):
            if adm.try_take(7):
                taken.append(7)

    threads = [threading.Thread(target=worker) for _ in range(8)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert len(taken) == adm.live <= 50
    assert adm.used == 7 * len(taken) <= 1000


def test_plan_bytes_grow_with_horizon_state_dimension_and_windows():
    small = workloads.point2d_problem(0, N=50)
    large = workloads.point2d_problem(0, N=400)
    assert plan_bytes(large, 8, 8) > plan_bytes(small, 8, 8) > 0
    # a 3-D point plan (n = 6) weighs more than a planar one of equal N
    p3 = workloads.point3d_problem(0, N=50)
    assert plan_bytes(p3, 8, 8) > plan_bytes(small, 8, 8)
    # wider trial windows hold more trial states
    assert plan_bytes(p3, 24, 24) > plan_bytes(p3, 8, 8)

"""The allocation-free entry point pgvimp_factor_expectations_noalloc gives
the same outputs as pgvimp_factor_expectations, bitwise (same kernels; only
the host staging differs), on two calls in a row, the second on a smaller
plan, in FP64 and mixed mode.  It also holds when the first call was made on
a larger plan of another context on the same device (the staging array
keeps the last call's contents)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pg():
    import paper_2411_03416_amd as m
    return m


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_equals_allocating_entry_point(pg, precision):
    big = workloads.point2d_problem(0, N=50)
    small = workloads.point2d_problem(1, N=23, gh_points=4)
    print(f"noalloc precision={precision} N=50 then N=23", flush=True)
    ctx = pg.pgvimp_create([big, small], precision=precision, use_graph=False)
    pg.pgvimp_prox_step(ctx, 2)  # a non-trivial state
    for plan, N in ((0, 50), (1, 23)):
        ref = pg.pgvimp_factor_expectations(ctx, plan)
        got = pg.pgvimp_factor_expectations_noalloc(ctx, plan)
        assert got[0].shape == (N,) and got[3].shape == (N + 1,)
        assert np.all(np.isfinite(got[0])) and np.all(np.isfinite(got[2]))
        assert _same(got, ref), f"plan {plan}: allocation-free outputs differ"
    pg.pgvimp_destroy(ctx)


def test_noalloc_across_contexts_and_dims(pg):
    # a larger n = 6 plan first, then a smaller n = 4 plan in another context
    p6 = workloads.point3d_problem(2, N=40)
    p4 = workloads.point2d_problem(3, N=17)
    print("noalloc n=6 N=40 then n=4 N=17", flush=True)
    c6 = pg.pgvimp_create([p6], precision=0, use_graph=False)
    c4 = pg.pgvimp_create([p4], precision=1, use_graph=False)
    for ctx in (c6, c4):
        ref = pg.pgvimp_factor_expectations(ctx, 0)
        got = pg.pgvimp_factor_expectations_noalloc(ctx, 0)
        assert _same(got, ref)
    pg.pgvimp_destroy(c6)
    pg.pgvimp_destroy(c4)

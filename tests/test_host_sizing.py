"""Host-side sizing of the C ABI (pgvimp_arena_bytes computes the arena
layout on the host, no GPU): the default trial windows per state dimension
and the trial scratch they imply."""
import pytest

from paper_2411_03416_amd import pgvimp_arena_bytes


@pytest.mark.parametrize("n,width,slots", [(2, 8, 16), (4, 8, 16), (6, 24, 24), (8, 24, 24), (14, 24, 24)])
def test_default_trial_windows(n, width, slots):
    """trial_width = trial_slots = 0 take 8 and 16 step sizes for n <= 4, 24
    and 24 for n >= 6 (a trial there is a long latency-bound chain, so one
    wide window runs all the trials an iteration needs)."""
    default = pgvimp_arena_bytes(n, 8, 800, 0)
    explicit = pgvimp_arena_bytes(n, 8, 800, 0, trial_width=width, trial_slots=slots)
    assert default == explicit


@pytest.mark.parametrize("n", [4, 6, 14])
def test_trial_scratch_grows_with_slots(n):
    """The arena holds per-slot trial states: more slots, more bytes, and the
    per-slot share grows with the number of states."""
    a8 = pgvimp_arena_bytes(n, 4, 400, 0, trial_width=8, trial_slots=8)
    a16 = pgvimp_arena_bytes(n, 4, 400, 0, trial_width=8, trial_slots=16)
    b8 = pgvimp_arena_bytes(n, 4, 800, 0, trial_width=8, trial_slots=8)
    b16 = pgvimp_arena_bytes(n, 4, 800, 0, trial_width=8, trial_slots=16)
    assert a16 > a8 and b16 > b8
    assert (b16 - b8) > (a16 - a8)


def test_slots_are_clamped_to_the_width():
    """trial_slots below trial_width is raised to it (the widest window is
    at least the narrowest)."""
    assert pgvimp_arena_bytes(6, 4, 400, 0, trial_width=16, trial_slots=4) == \
        pgvimp_arena_bytes(6, 4, 400, 0, trial_width=16, trial_slots=16)

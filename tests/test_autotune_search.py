"""Host logic of the autotuner's coordinate search (no device): it finds the
optimum of a separable cost, never times an option set twice, treats a
rejected candidate as infinitely slow and reports only non-default values."""
import math

from paper_1002_1202_amd.autotune import (SPACE_BATCHED, SPACE_FULL, SPACE_PROJECTED,
                                          coordinate_search)


def test_separable_optimum_and_trial_count():
    space = {"a": [0, 1, 2, 3], "b": [0, 8, 16], "c": [0, 5]}
    best_of = {"a": 2, "b": 16, "c": 0}
    calls = []

    def cost(opts):
        calls.append(dict(opts))
        full = {k: opts.get(k, v[0]) for k, v in space.items()}
        return 1.0 + sum((full[k] != best_of[k]) * (i + 1) for i, k in enumerate(space))

    best, t, table = coordinate_search(space, cost)
    assert best == {"a": 2, "b": 16}          # c at its default is omitted
    assert t == 1.0
    keys = [tuple(sorted(c.items())) for c in calls]
    assert len(keys) == len(set(keys))        # no option set timed twice
    assert len(calls) == 1 + sum(len(v) - 1 for v in space.values())
    assert len(table) == len(calls)


def test_rejected_candidates_are_skipped():
    space = {"x": [0, 12, 16], "y": [0, 1]}

    def cost(opts):
        if opts.get("x") == 12:
            raise ValueError("rejected")
        return 2.0 - 0.5 * (opts.get("x") == 16) - 0.25 * (opts.get("y") == 1)

    best, t, table = coordinate_search(space, cost)
    assert best == {"x": 16, "y": 1} and t == 1.25
    assert any(c == {"x": 12} and math.isinf(v) for c, v in table)


def test_spaces_start_at_the_library_defaults():
    for space in (SPACE_FULL, SPACE_PROJECTED, SPACE_BATCHED):
        assert all(v[0] == 0 and len(set(v)) == len(v) for v in space.values())
        if "row_groups" in space:
            assert all(g % 8 == 0 for g in space["row_groups"])
        if "cheb_block" in space:
            assert all(b % 64 == 0 for b in space["cheb_block"])

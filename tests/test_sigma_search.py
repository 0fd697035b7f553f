"""Host logic of the bandwidth-schedule search (no GPU): the candidate family
and the selection rule."""
from paper_1709_08610_amd import events, sigma_search as ss


def test_geometric_stages_stop_above_twice_sigma_final():
    assert ss.geometric(4.0, 0.5, 0.03) == [4.0, 2.0, 1.0, 0.5, 0.25, 0.125, 0.0625]
    assert ss.geometric(0.05, 0.5, 0.03) == []
    assert all(s > 0.06 for s in ss.geometric(8.0, 0.35, 0.03))


def test_candidates_current_first_unique_and_slope_steps():
    base = events.load_config("c2")["params"]
    cands = ss.candidates(base)
    assert cands[0][0] == "current" and cands[0][1] is not base and cands[0][1]["sigma"] == base["sigma"]
    keys = [(tuple(p["sigma"]), p["n_final_steps"]) for _, p in cands]
    assert len(keys) == len(set(keys))
    for name, p in cands[1:]:
        assert p["n_slope_steps"] == sum(1 for s in p["sigma"] if s >= ss.SLOPE_ONLY_MIN_SIGMA)
        assert p["sigma_final"] == base["sigma_final"] and p["n_polish"] == base["n_polish"]
    # origin-constrained tracks keep every step slope-only
    c8 = events.load_config("c8")["params"]
    assert all(p["n_slope_steps"] == c8["n_slope_steps"] for _, p in ss.candidates(c8))


def _row(name, ms, eff, fake=0.0):
    return dict(schedule=name, ms_per_event=ms, efficiency=eff, fake_rate=fake)


def test_choose_rule():
    cur = _row("current", 1.0, 0.976)
    rows = [cur, _row("a", 0.90, 0.9712), _row("b", 0.95, 0.9748), _row("c", 0.5, 0.94),
            _row("d", 0.8, 0.99, fake=0.01)]
    assert ss.choose(rows)["schedule"] == "a"          # 0.0048 below the current: within, and fastest
    rows[1]["efficiency"] = 0.9709                      # 0.0051 below: out
    assert ss.choose(rows)["schedule"] == "b"
    rows[1]["efficiency"] = 0.9711                      # 0.0049 below: in, and the fastest
    assert ss.choose(rows)["schedule"] == "a"
    # below 0.95 now: the bar is the current efficiency less the slack
    low = [_row("current", 1.0, 0.82), _row("x", 0.9, 0.816), _row("y", 0.5, 0.81)]
    assert ss.choose(low)["schedule"] == "x"
    # at 0.952 the 0.95 floor binds before the slack does
    edge = [_row("current", 1.0, 0.952), _row("x", 0.9, 0.9495), _row("y", 0.95, 0.9501)]
    assert ss.choose(edge)["schedule"] == "y"
    # nothing faster qualifies: the current schedule stays
    assert ss.choose([cur, _row("z", 0.2, 0.5)])["schedule"] == "current"

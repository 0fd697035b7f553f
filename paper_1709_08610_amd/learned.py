"""Learned-seed settings of a workload (the "learned" block of its config):
the model file, the proposal thresholds and the sigma schedule used when the
ascent starts from proposer seeds (bin centres are already close to the
maxima, so the schedule starts at a smaller sigma than the lattice's)."""
from __future__ import annotations

import os

_HERE = os.path.dirname(os.path.abspath(__file__))


def settings(cfg: dict) -> dict:
    lb = cfg.get("learned")
    if lb is None:
        raise KeyError("workload %s has no learned-seed settings" % cfg.get("name"))
    params = dict(cfg["params"])
    params.update(lb.get("params", {}))
    return dict(model=os.path.join(_HERE, lb["model"]), k_max=int(lb["k_max"]), tau=float(lb["tau"]),
                conf_min=float(lb["conf_min"]), nms=bool(lb["nms"]), params=params)

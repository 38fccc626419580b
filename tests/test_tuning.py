"""The tuning cache (host logic only): problem classes, keys and the JSON round trip."""
import json

import numpy as np
import pytest

from paper_1306_4743_amd import tuning


def test_size_class_is_the_next_power_of_two():
    assert tuning.size_class((33, 33, 33)) == 64
    assert tuning.size_class((64, 2, 2)) == 64
    assert tuning.size_class((65, 9, 9)) == 128
    assert tuning.size_class((513, 513, 513)) == 1024
    assert tuning.size_class((2, 2, 2)) == 2


def test_speed_class():
    assert tuning.speed_class(np.ones((3, 3, 3))) == "constant"
    F = np.ones((4, 4, 4))
    F[0, 0, 0] = 0.2
    assert tuning.speed_class(F) == "smooth"
    F[0, 0, 0] = 0.01
    assert tuning.speed_class(F) == "contrast"


def test_keys_separate_classes_and_modes():
    F = np.ones((5, 5, 5))
    assert tuning.solve_key((5, 5, 5), F, 0) != tuning.solve_key((5, 5, 5), F, 2)
    assert tuning.solve_key((5, 5, 5), F, 0) == tuning.solve_key((7, 6, 8), F, 0)
    assert tuning.server_key((33, 65), "contrast", 0) == "server/sizes33-65/contrast/mode0"


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = tuning.TuneCache(path)
    assert c.get("k") is None
    c.put("k", {"cell": 8, "inner": 1, "workers": 0, "delta": 0.0})
    c.put("s", {"cell": 4, "rounds_per_step": 16})
    again = tuning.TuneCache(path)
    assert again.get("k")["cell"] == 8 and again.get("s")["rounds_per_step"] == 16
    assert json.load(open(path))["k"]["inner"] == 1


@pytest.mark.gpu
def test_tuned_options_are_measured_once_and_reused(tmp_path):
    import torch
    from paper_1306_4743_amd import eik, workloads as W
    eik.load()
    p = W.maze(33, seed=3, n_sources=2)
    F = torch.from_numpy(p.F).to("cuda:0")
    cache = tuning.TuneCache(str(tmp_path / "t.json"))
    opt, key, measured = tuning.tuned_solve_options(F, p.h, p.src, p.q, cache=cache, reps=1)
    assert measured and opt["cell"] in (4, 8, 16)
    opt2, key2, measured2 = tuning.tuned_solve_options(F, p.h, p.src, p.q, cache=cache)
    assert key2 == key and not measured2 and opt2 == opt
    u = eik.solve(F, p.h, p.src, p.q, **opt)
    assert eik.status()[0] == 0 and np.isfinite(u.cpu().numpy()).all()

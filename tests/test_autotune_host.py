"""Host logic of the launch tuner: the coordinate descent and the stored
records (no GPU: the timing of a trial is replaced by a model)."""
import json

from paper_1905_08717_amd import autotune as A


class FakeSolver:
    def __init__(self):
        self.knobs = {"list_grid": 2048, "iface_grid": 512, "comp_grid": 8192, "bulk_levels": 1}

    def set_launch(self, **kw):
        self.knobs.update({k: v for k, v in kw.items() if v})

    def get_launch(self):
        return dict(self.knobs)


def _model(best):
    """Seconds per step: a bowl around `best`, separable in the knobs."""
    def t(knobs):
        return 1.0 + sum(abs(knobs[k] - best[k]) / best[k] for k in best)
    return t


def test_descent_finds_the_separable_optimum(monkeypatch):
    target = {"list_grid": 3072, "iface_grid": 1024, "comp_grid": 4096, "bulk_levels": 2}
    model = _model(target)
    calls = []

    def fake_time(solver, q0, dt, knobs, warmup, steps):
        solver.set_launch(**knobs)
        calls.append(dict(knobs))
        return model(knobs)

    monkeypatch.setattr(A, "time_config", fake_time)
    s = FakeSolver()
    r = A.tune(s, None, 1.0)
    assert r["best"] == target and s.get_launch() == target
    assert r["seconds_per_step"] == 1.0 and r["default"] > 1.0
    assert len(r["trials"]) == len(calls)
    # the first trial times the context's current setting
    assert calls[0] == {"list_grid": 2048, "iface_grid": 512, "comp_grid": 8192, "bulk_levels": 1}


def test_margin_keeps_the_incumbent_on_small_gains(monkeypatch):
    def fake_time(solver, q0, dt, knobs, warmup, steps):
        return 1.0 - (0.01 if knobs["list_grid"] == 4096 else 0.0)   # 1 % better only

    monkeypatch.setattr(A, "time_config", fake_time)
    s = FakeSolver()
    r = A.tune(s, None, 1.0, margin=0.02)
    assert r["best"]["list_grid"] == 2048
    r = A.tune(s, None, 1.0, margin=0.0)
    assert r["best"]["list_grid"] == 4096


def test_record_and_lookup_round_trip(tmp_path):
    path = str(tmp_path / "rec.json")
    assert A.lookup("nagumo2d_L9_b512", path=path) is None
    res = {"best": {"list_grid": 1536, "iface_grid": 2048, "comp_grid": 8192},
           "seconds_per_step": 0.19, "default": 0.21, "trials": [0] * 7}
    A.record(A.nagumo_key(9, 512), res, "test", path=path)
    A.record(A.nagumo_key(9, 64), dict(res, best=dict(res["best"], list_grid=1024)), "test", path=path)
    assert A.lookup("nagumo2d_L9_b512", path=path) == res["best"]
    assert A.lookup("nagumo2d_L9_b64", path=path)["list_grid"] == 1024
    with open(path) as fh:
        data = json.load(fh)
    assert data["nagumo2d_L9_b512"]["trials"] == 7 and data["nagumo2d_L9_b512"]["ms_per_step"] == 190.0


def test_stored_records_name_every_knob():
    # the committed record (if any) holds valid grid caps for every knob
    try:
        with open(A.RECORD_PATH) as fh:
            data = json.load(fh)
    except OSError:
        return
    for key, rec in data.items():
        for k in A.CANDIDATES:
            if k == "bulk_levels":
                assert int(rec.get(k, 1)) in (1, 2), (key, k)
            else:
                assert 1 <= int(rec[k]) <= 65535, (key, k)

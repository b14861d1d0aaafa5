"""The autotuner's JSON cache (host logic only): a miss runs the library's
tuner once and stores its table under the configuration's key, a hit installs
the stored table without tuning, another source count or device is another
key, and a damaged cache file is treated as empty."""
import json
import types

from paper_1806_11277_amd import tuning


class _FakeSolver:
    def __init__(self, levels=3, n=(64, 32)):
        o = types.SimpleNamespace(levels=levels, precond_bits=32, coarse_bits=32, dd_parts=[1, 1, 1],
                                  dd_overlap=0, dd_pad=0, coarse_dd_parts=[1, 1, 1], vanka=1)
        p = types.SimpleNamespace(dim=2, n=list(n) + [1])
        self.problem, self.options, self.levels = p, o, levels
        self.tuned, self.installed = 0, []

    def autotune(self, nrhs):
        self.tuned += 1
        return [nrhs, 1] * self.levels

    def set_tuning(self, table):
        self.installed.append(list(table))


def test_cache_miss_then_hit(tmp_path):
    path = str(tmp_path / "sub" / "t.json")
    S = _FakeSolver()
    t, how = tuning.tune(S, 8, path=path, device="dev0")
    assert how == "tuned" and t == [8, 1] * 3 and S.tuned == 1
    t2, how2 = tuning.tune(S, 8, path=path, device="dev0")
    assert how2 == "cache" and t2 == t and S.tuned == 1 and S.installed == [t]
    tuning.tune(S, 4, path=path, device="dev0")
    tuning.tune(S, 8, path=path, device="dev1")
    assert S.tuned == 3
    assert len(json.load(open(path))) == 3
    # a different grid is a different key
    tuning.tune(_FakeSolver(n=(64, 64)), 8, path=path, device="dev0")
    assert len(json.load(open(path))) == 4


def test_damaged_or_mismatched_cache_is_ignored(tmp_path):
    path = tmp_path / "t.json"
    path.write_text("{not json")
    S = _FakeSolver()
    _, how = tuning.tune(S, 8, path=str(path), device="d")
    assert how == "tuned"
    # an entry of the wrong length (other hierarchy depth) is re-tuned
    d = json.load(open(path))
    k = next(iter(d))
    d[k] = [1, 2]
    path.write_text(json.dumps(d))
    _, how = tuning.tune(S, 8, path=str(path), device="d")
    assert how == "tuned" and S.tuned == 2


def test_cache_path_from_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("EHH_TUNE_CACHE", str(tmp_path / "x.json"))
    assert tuning.cache_path() == str(tmp_path / "x.json")
    monkeypatch.delenv("EHH_TUNE_CACHE")
    assert tuning.cache_path().endswith("tuning.json")

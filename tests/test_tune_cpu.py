"""Tuning cache logic (no GPU): records round-trip per device key."""
from paper_2504_07264_amd import tune


def test_cache_round_trip(tmp_path, monkeypatch):
    path = str(tmp_path / "t.json")
    monkeypatch.setattr(tune, "device_key", lambda device=None: "devA")
    assert tune.lookup("length:1024:16", path) is None
    tune.record("length:1024:16", 0x300, {0x300: {"us": 1.0}, 0x100: {"us": 2.0}}, path)
    assert tune.lookup("length:1024:16", path) == 0x300
    monkeypatch.setattr(tune, "device_key", lambda device=None: "devB")
    assert tune.lookup("length:1024:16", path) is None  # another device or library build
    tune.record("length:1024:16", 0x100, {0x100: {"us": 1.5}}, path)
    monkeypatch.setattr(tune, "device_key", lambda device=None: "devA")
    assert tune.lookup("length:1024:16", path) == 0x300


def test_keys_are_stable():
    assert tune.length_key(1024, 16384) == "length:1024:16384"
    assert tune.length_key(1024, 16384, dif=True) == "length-dif:1024:16384"
    assert tune.ragged_key([16, 32]) == tune.ragged_key([16, 32]) != tune.ragged_key([32, 16])


def test_cli_ragged_path_passes_the_workload_lengths(monkeypatch, tmp_path):
    # the --ragged path hands tune_many the drawn lengths (a list of powers of
    # two from the workload recipe) and records under their key
    seen = {}

    def fake_tune_many(lengths):
        seen["lengths"] = lengths
        return 0, {0: 1.0}

    monkeypatch.setattr(tune, "tune_many", fake_tune_many)
    monkeypatch.setattr(tune, "device_key", lambda device=None: "test-device")
    path = str(tmp_path / "tune.json")
    tune.main(["--lengths", "", "--ragged", "12", "--cache", path])
    ls = seen["lengths"]
    assert isinstance(ls, list) and len(ls) == 12
    assert all(isinstance(v, int) and v >= 16 and v & (v - 1) == 0 for v in ls)
    assert tune.lookup(tune.ragged_key(ls), path) == 0

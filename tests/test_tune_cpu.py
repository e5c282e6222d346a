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

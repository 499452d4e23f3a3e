"""Host logic of the batched tile table: JSON round trip, nearest-bucket lookup, and rejection of
malformed files (no GPU needed)."""
import json

import pytest

import paper_1905_10574_amd as T


@pytest.fixture
def clean_table():
    saved = dict(T._TILE_TABLE)
    T._TILE_TABLE.clear()
    yield
    T._TILE_TABLE.clear()
    T._TILE_TABLE.update(saved)


def test_default_before_tuning(clean_table):
    assert T.tile_for(8192) == 128 and T.tile_for(40) == 40 and T.tile_for(5) == 16


def test_round_trip_and_nearest_bucket(clean_table, tmp_path):
    path = tmp_path / "t.json"
    path.write_text(json.dumps({"tiles": {"64": 32, "256": 64, "2048": 128}, "meta": {}}))
    assert T.load_tile_table(str(path)) == {64: 32, 256: 64, 2048: 128}
    assert T.tile_for(70) == 32            # nearest by ratio: 64
    assert T.tile_for(200) == 64
    assert T.tile_for(1500) == 128
    out = tmp_path / "u.json"
    T.save_tile_table(str(out), {"note": "x"})
    rec = json.loads(out.read_text())
    assert rec["tiles"] == {"64": 32, "256": 64, "2048": 128} and rec["meta"] == {"note": "x"}


def test_rejects_malformed(clean_table, tmp_path):
    path = tmp_path / "bad.json"
    path.write_text(json.dumps({"tiles": {}}))
    with pytest.raises(ValueError):
        T.load_tile_table(str(path))
    path.write_text(json.dumps({"tiles": {"64": 0}}))
    with pytest.raises(ValueError):
        T.load_tile_table(str(path))

"""The binding's cache of tuned batch tiles (host logic only)."""
import json

import torch

from paper_1803_02009_amd import _lib
from paper_1803_02009_amd import misslam as M


def _prob(n, m, w, h):
    return dict(points=torch.zeros((6, n)), nodes=torch.zeros((3, m)), cam=M.camera(w, h, 1.0, 1.0, 0.0, 0.0))


def test_key_buckets_and_largest_frame():
    p = M.Params()
    a = [_prob(1000, 100, 320, 240), _prob(2000, 200, 640, 480)]
    b = [_prob(1500, 150, 640, 480), _prob(1600, 250, 320, 240)]   # same buckets (4096 points, 512 nodes)
    assert M.tile_key(a, p) == M.tile_key(b, p) == "N4096-m512-640x480-prec0-k4-pcg10-form0-count2"
    assert M.tile_key(a, M.Params(precision=_lib.PREC_BF16)) != M.tile_key(a, p)
    assert M.tile_key(a[:1], p) == "N1024-m128-320x240-prec0-k4-pcg10-form0-count1"


def test_cache_file_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "tiles.json"
    monkeypatch.setenv("MISSLAM_TILE_CACHE", str(path))
    assert M.tile_cache_path() == str(path)
    assert M._read_tile_cache(str(path)) == {}            # missing file: empty
    M._write_tile_cache(str(path), "k1", {"rows_per_wg": 16, "asm_waves": 2})
    M._write_tile_cache(str(path), "k2", {"rows_per_wg": 21, "asm_waves": 1})
    assert json.loads(path.read_text()) == {"k1": {"rows_per_wg": 16, "asm_waves": 2},
                                            "k2": {"rows_per_wg": 21, "asm_waves": 1}}
    path.write_text("not json")
    assert M._read_tile_cache(str(path)) == {}            # a damaged file is ignored, not fatal

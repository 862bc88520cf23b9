"""The autotuner's cache (host logic, no GPU): entries are keyed by device
architecture, precision, grid, boundary, coarse operator, number of
right-hand sides and constant/variable k; a lookup returns the recorded choice
or nothing; writes keep the other entries."""
from paper_2308_06152_amd import autotune


def test_cache_roundtrip_and_keys(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "arch", lambda: "gfx950")
    path = str(tmp_path / "cache.json")
    grid = (4097, 4097, 1 / 4096, 1 / 4096, 1)
    opts = dict(coarse_op=1, precision=0)
    assert autotune.lookup(grid, 1, opts, False, cache_path=path) == {}
    k1 = autotune.key(4097, 4097, 1, 1, 0, 1, False)
    k2 = autotune.key(4097, 4097, 1, 1, 1, 1, False)
    k3 = autotune.key(2049, 1025, 1, 1, 0, 64, True)
    assert len({k1, k2, k3}) == 3 and k1.startswith("gfx950|")
    autotune.save_cache({k1: {"best": {"vc_tail": 70000, "graphs": 0, "coarse_restart": 20}},
                         k3: {"best": {"vc_tail": 0, "graphs": 0, "coarse_restart": 10}}}, path)
    assert autotune.lookup(grid, 1, opts, False, cache_path=path) == \
        {"vc_tail": 70000, "graphs": 0, "coarse_restart": 20}
    assert autotune.lookup(grid, 1, dict(opts, precision=1), False, cache_path=path) == {}
    assert autotune.lookup((2049, 1025, 5.0, 5.0, 1), 64, opts, True, cache_path=path) == \
        {"vc_tail": 0, "graphs": 0, "coarse_restart": 10}
    monkeypatch.setattr(autotune, "arch", lambda: "gfx942")
    assert autotune.lookup(grid, 1, opts, False, cache_path=path) == {}

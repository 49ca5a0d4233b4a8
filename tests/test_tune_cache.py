"""The JSON cache of autotuned launch shapes (host logic; the lattices and
batches here are stand-ins that record what the cache asks of them)."""
import json

from paper_1805_08643_amd import tune_cache as tc


class FakeLattice:
    def __init__(self, cfg, mode="split", tuned=(128, 4, 64)):
        self.cfg, self.mode, self.tuned = cfg, mode, tuned
        self.tile, self.autotunes = None, 0

    def step_mode(self):
        return self.mode

    def set_tile(self, tx, ty, cz):
        self.tile = (tx, ty, cz)

    def autotune(self, trials):
        self.autotunes += 1
        self.tile = self.tuned
        return self.tuned


class FakeBatch:
    def __init__(self, cfgs):
        self.cfgs, self.calls, self.state = cfgs, [], ("fused", 8192, 256)

    def autotune(self, trials):
        self.calls.append("autotune")
        self.state = ("split", 16384, 256)

    def tuning(self):
        return self.state

    def set_step_mode(self, m):
        self.calls.append(("mode", m))

    def set_item_nodes(self, n):
        self.calls.append(("items", n))

    def set_blocks(self, b):
        self.calls.append(("blocks", b))


CFG = dict(nx=256, ny=256, nz=256, storage="f32", op="nonorth")


def test_lattice_miss_then_hit(tmp_path):
    path = str(tmp_path / "tune.json")
    c = tc.TuneCache(path, device="gfx950:test", code="abc")
    a = FakeLattice(CFG)
    assert c.tune_lattice(a) == ((128, 4, 64), False) and a.autotunes == 1
    b = FakeLattice(CFG, tuned=(1, 1, 1))
    c2 = tc.TuneCache(path, device="gfx950:test", code="abc")  # read back from the file
    assert c2.tune_lattice(b) == ((128, 4, 64), True)
    assert b.autotunes == 0 and b.tile == (128, 4, 64)
    d = json.load(open(path))
    assert d["format"] == tc.FORMAT and d["version"] == tc.VERSION and len(d["entries"]) == 1


def test_keys_separate_what_changes_the_choice(tmp_path):
    base = tc.lattice_key(CFG, "split", "dev", "code")
    for cfg, mode, dev, code in [(dict(CFG, nx=128), "split", "dev", "code"), (dict(CFG, storage="f16s"), "split",
                                                                              "dev", "code"),
                                 (dict(CFG, op="orth"), "split", "dev", "code"), (dict(CFG, wall_z=1), "split", "dev",
                                                                                 "code"),
                                 (CFG, "pairs", "dev", "code"), (CFG, "split", "dev2", "code"),
                                 (CFG, "split", "dev", "code2")]:
        assert tc.lattice_key(cfg, mode, dev, code) != base
    runs = [dict(CFG, nx=n, ny=n, nz=n) for n in (32, 48, 64)]
    assert tc.batch_key(runs, "d", "c") == tc.batch_key(runs[::-1], "d", "c")  # order of runs does not matter
    assert tc.batch_key(runs, "d", "c") != tc.batch_key(runs[:2], "d", "c")


def test_batch_miss_then_hit(tmp_path):
    path = str(tmp_path / "tune.json")
    runs = [dict(CFG, nx=n, ny=n, nz=n) for n in (32, 48)]
    b = FakeBatch(runs)
    c = tc.TuneCache(path, device="d", code="c")
    assert c.tune_batch(b) == (("split", 16384, 256), False) and b.calls == ["autotune"]
    b2 = FakeBatch(runs)
    assert tc.TuneCache(path, device="d", code="c").tune_batch(b2) == (("split", 16384, 256), True)
    assert b2.calls == [("mode", "split"), ("items", 16384), ("blocks", 256)]


def test_unreadable_or_foreign_file_is_ignored_and_rewritten(tmp_path):
    path = tmp_path / "tune.json"
    for content in ("{not json", json.dumps({"format": "other", "entries": {}}),
                    json.dumps({"format": tc.FORMAT, "version": tc.VERSION,
                                "entries": {"lattice|x": {"mode": "split", "tile": [0, 1, 2]},
                                            "batch|y": {"mode": "split", "item_nodes": "many", "blocks": 3}}})):
        path.write_text(content)
        c = tc.TuneCache(str(path), device="d", code="c")
        assert c.entries == {}
        c.tune_lattice(FakeLattice(CFG))
        assert len(json.load(open(path))["entries"]) == 1
    assert not [p for p in tmp_path.iterdir() if p.name.startswith(".tune-")]  # no temporary left behind

"""Host logic of the autotuning cache (JSON file keyed by ensemble, device
and library build)."""
import json
from types import SimpleNamespace

from paper_2112_08926_amd import tuning


def _p(nx=64, ny=32, nz=16, q=19, collision=1, storage=3, arith=0, unshifted=0, tau=0.6):
    return SimpleNamespace(nx=nx, ny=ny, nz=nz, q=q, collision=collision, storage=storage, arith=arith,
                           unshifted=unshifted, tau=tau)


LAUNCH = {"mode": 1, "block": 256, "cells_per_lane": 1, "persistent": 2048, "graph_steps": 100}


def test_key_is_stable_and_ignores_physics():
    k = tuning.ensemble_key([_p()], "MI355X|gfx950", "abc")
    assert k == tuning.ensemble_key([_p(tau=0.9)], "MI355X|gfx950", "abc")
    assert len(k) == 64


def test_key_changes_with_what_the_launch_depends_on():
    base = tuning.ensemble_key([_p()], "dev", "lib")
    variants = [
        tuning.ensemble_key([_p(storage=1)], "dev", "lib"),
        tuning.ensemble_key([_p(q=27)], "dev", "lib"),
        tuning.ensemble_key([_p(collision=0)], "dev", "lib"),
        tuning.ensemble_key([_p(arith=1)], "dev", "lib"),
        tuning.ensemble_key([_p(unshifted=1)], "dev", "lib"),
        tuning.ensemble_key([_p(nx=65)], "dev", "lib"),
        tuning.ensemble_key([_p(), _p()], "dev", "lib"),
        tuning.ensemble_key([_p()], "dev2", "lib"),
        tuning.ensemble_key([_p()], "dev", "lib2"),
    ]
    assert base not in variants and len(set(variants)) == len(variants)
    # lattice order matters (the tile table follows it)
    a = tuning.ensemble_key([_p(nx=32), _p(nx=64)], "dev", "lib")
    b = tuning.ensemble_key([_p(nx=64), _p(nx=32)], "dev", "lib")
    assert a != b


def test_store_load_round_trip_keeps_other_entries(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert tuning.load(path, "k1") is None
    tuning.store(path, "k1", LAUNCH, note="first")
    other = dict(LAUNCH, block=64, cells_per_lane=2)
    tuning.store(path, "k2", other)
    assert tuning.load(path, "k1") == {f: LAUNCH[f] for f in tuning.LAUNCH_FIELDS}
    assert tuning.load(path, "k2") == {f: other[f] for f in tuning.LAUNCH_FIELDS}
    data = json.load(open(path))
    assert set(data) == {"k1", "k2"} and "graph_steps" not in data["k1"] and data["k1"]["note"] == "first"
    tuning.store(path, "k1", other)                   # replace
    assert tuning.load(path, "k1")["block"] == 64
    assert [f.name for f in (tmp_path / "sub").iterdir()] == ["tune.json"]   # no temporary left


def test_bad_files_read_as_empty(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert tuning.load(str(path), "k") is None
    tuning.store(str(path), "k", LAUNCH)              # overwrites the broken file
    assert tuning.load(str(path), "k")["persistent"] == 2048
    path.write_text(json.dumps({"k": {"mode": 1}}))   # incomplete entry
    assert tuning.load(str(path), "k") is None
    path.write_text(json.dumps([1, 2]))
    assert tuning.load(str(path), "k") is None

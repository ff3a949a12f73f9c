"""Host-only checks of the tuning options and of the tuning cache lookup
(QGT_TUNE_CACHE): the planner's choice per block, from the caller, the cache
or the defaults, with no HIP call."""
import json
import os

import pytest

import paper_2510_08430_amd as qgt

PROBS = [(8192, [40400, 160400], 1e-4), (4096, [8320, 65], 1e-3)]
# the shape classes of those blocks: gfx950 / Gram precision / form /
# padded order / contraction length rounded up to a power of two
CLASS_WIDE = "gfx950/bf16/S/m8192/k65536"     # 40400 columns at n_s = 8192
CLASS_SMALL = "gfx950/fp64/P/m128/k4096"      # 65 columns at n_s = 4096


@pytest.fixture(autouse=True)
def no_cache(monkeypatch):
    monkeypatch.delenv("QGT_TUNE_CACHE", raising=False)
    qgt.load()


def write_cache(path, entries):
    lines = ['{', ' "format": "qgt-tune-1",', ' "entries": {']
    items = list(entries.items())
    for k, (key, t) in enumerate(items):
        lines.append(f'  "{key}": ' + json.dumps(t) + ("," if k + 1 < len(items) else ""))
    lines += [' }', '}']
    path.write_text("\n".join(lines) + "\n")


def test_defaults():
    t = qgt.tuning_query(PROBS, "c64", "auto", 0)
    assert t == {"gram_tile": 2, "gram_items": 256, "chol_chunk": 4, "gram_patch": 4, "source": "default"}
    t = qgt.tuning_query(PROBS, "c64", "auto", 3)     # FP64 parameter-space block: 128x128 tiles
    assert t["gram_tile"] == 1 and t["source"] == "default"


def test_cache_lookup_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    write_cache(path, {CLASS_WIDE: {"gram_tile": 1, "gram_items": 1024, "chol_chunk": 6, "gram_patch": 8,
                                    "form_ms": 1.0, "step_ms": 2.0},
                       CLASS_SMALL: {"gram_tile": 1, "gram_items": 512, "chol_chunk": 2, "gram_patch": 2}})
    monkeypatch.setenv("QGT_TUNE_CACHE", str(path))
    assert qgt.tuning_query(PROBS, "c64", "auto", 0) == {"gram_tile": 1, "gram_items": 1024, "chol_chunk": 6,
                                                           "gram_patch": 8, "source": "cache"}
    assert qgt.tuning_query(PROBS, "c64", "auto", 3) == {"gram_tile": 1, "gram_items": 512, "chol_chunk": 2,
                                                           "gram_patch": 2, "source": "cache"}
    # classes without an entry take the defaults
    t = qgt.tuning_query(PROBS, "c64", "auto", 1)
    assert t["source"] == "default" and t["chol_chunk"] == 4
    # the same problems in another order find the same entries (lookup by
    # class, not by position)
    t = qgt.tuning_query(list(reversed(PROBS)), "c64", "auto", 2)
    assert t["chol_chunk"] == 6 and t["source"] == "cache"
    # the caller's tuning wins over the cache
    t = qgt.tuning_query(PROBS, "c64", "auto", 0, tuning=[{"chol_chunk": 3}] * 4)
    assert t["chol_chunk"] == 3 and t["gram_tile"] == 2 and t["source"] == "caller"
    # a FP32 factor is another class
    t = qgt.tuning_query(PROBS, "c64", "auto", 0, factor="fp32")
    assert t["source"] == "default"


def test_missing_cache_file_gives_defaults(tmp_path, monkeypatch):
    monkeypatch.setenv("QGT_TUNE_CACHE", str(tmp_path / "absent.json"))
    assert qgt.tuning_query(PROBS, "c64", "auto", 0)["source"] == "default"


@pytest.mark.parametrize("bad", [{"gram_tile": 4}, {"chol_chunk": 17}, {"gram_patch": 40}, {"gram_items": -1}])
def test_invalid_tuning_is_rejected(bad):
    with pytest.raises(qgt.QgtError):
        qgt.tuning_query(PROBS, "c64", "auto", 0, tuning=[bad] * 4)
    # the wide BF16 tile on a block that cannot take it
    with pytest.raises(qgt.QgtError):
        qgt.tuning_query([(4096, [65], 1e-3)], "c64", "auto", 0, tuning=[{"gram_tile": 2}])


CLASSES_OF_PROBS = [CLASS_WIDE, "gfx950/bf16/S/m8192/k262144", "gfx950/bf16/S/m4096/k16384", CLASS_SMALL]


def plan_key(classes):
    """The cache key of a set of blocks for its Cholesky launch mode: FNV-1a
    (64 bits) over the sorted shape classes, each followed by '|'."""
    h, mask = 1469598103934665603, (1 << 64) - 1
    for k in sorted(classes):
        for ch in k.encode() + b"|":
            h = ((h ^ ch) * 1099511628211) & mask
    return f"gfx950/plan/{h:016x}/n{len(classes)}"


def test_cholesky_mode_from_the_cache(tmp_path, monkeypatch):
    # no cache: the persistent launch by default, the caller's choice if given
    assert qgt.cholesky_query(PROBS) == {"mode": "persistent", "source": "default"}
    assert qgt.cholesky_query(PROBS, cholesky="host-steps") == {"mode": "host-steps", "source": "caller"}
    path = tmp_path / "tune.json"
    write_cache(path, {CLASS_WIDE: {"gram_tile": 2, "gram_items": 256, "chol_chunk": 6, "gram_patch": 8},
                       plan_key(CLASSES_OF_PROBS): {"cholesky": 1, "persistent_ms": 10.0, "host_steps_ms": 9.0}})
    monkeypatch.setenv("QGT_TUNE_CACHE", str(path))
    # the plan entry applies to this set of blocks, in any problem order
    assert qgt.cholesky_query(PROBS) == {"mode": "host-steps", "source": "cache"}
    assert qgt.cholesky_query(list(reversed(PROBS))) == {"mode": "host-steps", "source": "cache"}
    # the block entries are still read beside it
    assert qgt.tuning_query(PROBS, "c64", "auto", 0)["chol_chunk"] == 6
    # the caller's choice wins; another set of blocks has no entry
    assert qgt.cholesky_query(PROBS, cholesky="persistent") == {"mode": "persistent", "source": "caller"}
    assert qgt.cholesky_query(PROBS[:1]) == {"mode": "persistent", "source": "default"}
    # an entry naming the persistent launch
    write_cache(path, {plan_key(CLASSES_OF_PROBS): {"cholesky": 2}})
    assert qgt.cholesky_query(PROBS) == {"mode": "persistent", "source": "cache"}


def test_duo_tiles_only_for_bf16_blocks():
    """gram_tile 3 (128x128 tiles, two workgroups per CU) is a BF16 kernel:
    accepted for the BF16 blocks, refused for an FP64 block."""
    t = qgt.tuning_query(PROBS, "c64", "auto", 0, tuning=[{"gram_tile": 3}, {}, {}, {}])
    assert t["gram_tile"] == 3 and t["source"] == "caller"
    with pytest.raises(qgt.QgtError):
        qgt.tuning_query(PROBS, "c64", "auto", 0, tuning=[{}, {}, {}, {"gram_tile": 3}])


def test_class_entry_inside_a_set_of_blocks(tmp_path, monkeypatch):
    """A shape class tuned inside a set of blocks: that set takes the entry
    stored under its plan key (source "plan-cache"); a set that shares the
    class but not the other blocks takes the class's own entry."""
    path = tmp_path / "tune.json"
    inside = plan_key(CLASSES_OF_PROBS) + "/" + CLASS_WIDE[len("gfx950/"):]
    write_cache(path, {CLASS_WIDE: {"gram_tile": 2, "gram_items": 256, "chol_chunk": 6, "gram_patch": 8},
                       inside: {"gram_tile": 3, "gram_items": 256, "chol_chunk": 12, "gram_patch": 2}})
    monkeypatch.setenv("QGT_TUNE_CACHE", str(path))
    assert qgt.tuning_query(PROBS, "c64", "auto", 0) == {"gram_tile": 3, "gram_items": 256, "chol_chunk": 12,
                                                           "gram_patch": 2, "source": "plan-cache"}
    # the same set in another problem order
    t = qgt.tuning_query(list(reversed(PROBS)), "c64", "auto", 2)
    assert t["gram_tile"] == 3 and t["source"] == "plan-cache"
    # another set with the class: the class entry
    assert qgt.tuning_query(PROBS[:1], "c64", "auto", 0) == {"gram_tile": 2, "gram_items": 256, "chol_chunk": 6,
                                                               "gram_patch": 8, "source": "cache"}
    # a class of the set without an entry inside it falls back to its own
    # (here none: the defaults)
    assert qgt.tuning_query(PROBS, "c64", "auto", 1)["source"] == "default"
    # the caller's tuning still wins
    assert qgt.tuning_query(PROBS, "c64", "auto", 0, tuning=[{}] * 4)["source"] == "caller"

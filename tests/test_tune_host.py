"""The autotuner's table without a GPU: set / get / reset, the variants
compiled per pass and length, and the JSON cache (save, load, rejection of
malformed or impossible entries).  Timing itself needs the device
(tests/test_gpu_tune.py)."""
import json

import pytest

from paper_2504_19410_amd import fsa as F


@pytest.fixture(autouse=True)
def clean_table():
    F.tune_reset()
    yield
    F.tune_reset()


def test_defaults_and_set_get():
    assert F.tune_get("f32", "conv", 512) == (0, 0, 0.0)
    F.tune_set("f32", "conv", 512, 1, 2)
    assert F.tune_get("f32", "conv", 512)[:2] == (1, 2)
    assert F.tune_get("f64", "conv", 512)[:2] == (0, 0)   # per precision
    F.tune_reset()
    assert F.tune_get("f32", "conv", 512)[:2] == (0, 0)


def test_variant_sets_follow_the_radix_plans():
    # the alternate radix family differs from the default at these lengths
    for n in (128, 256, 512, 1024, 2048, 4096):
        assert 1 in F.tune_variants("f32", "conv", n), n
    # and falls back to it (so is not compiled) at small powers of two
    for n in (16, 32, 64):
        assert 1 not in F.tune_variants("f32", "conv", n), n
    # at 3 * 2^a the alternate is the radix-3-last split of the middle-3 plan
    for n in (24, 48, 96, 192, 384, 768, 1536, 3072):
        assert 1 in F.tune_variants("f32", "conv", n), n
    for p in F.PASSES:
        assert 0 in F.tune_variants("f64", p, 256)


def test_rejects_impossible_entries():
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.tune_set("f32", "conv", 64, 1)          # variant 1 not compiled at 64
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.tune_set("f32", "conv", 100, 0)         # unsupported length
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.tune_set("f32", "r2c", 4096, 0)         # real passes stop at 2048
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.tune_set("f32", "conv", 512, 0, -1)     # negative occupancy


def test_save_load_roundtrip(tmp_path):
    F.tune_set("f32", "conv", 512, 1, 0)
    F.tune_set("f32", "fwd_t", 512, 2, 1)
    F.tune_set("f32", "c2r", 1024, 1, 3)
    path = tmp_path / "tune.json"
    F.tune_save(str(path))
    doc = json.loads(path.read_text())
    assert doc["format"] == "fsa-tune-1"
    assert len(doc["entries"]) == 3
    F.tune_reset()
    F.tune_load(str(path))
    assert F.tune_get("f32", "conv", 512)[:2] == (1, 0)
    assert F.tune_get("f32", "fwd_t", 512)[:2] == (2, 1)
    assert F.tune_get("f32", "c2r", 1024)[:2] == (1, 3)


@pytest.mark.parametrize("text", [
    "",
    "{",
    '{"format": "other", "arch": "", "entries": []}',
    '{"format": "fsa-tune-1", "arch": "", "entries": [{"precision": "f32", "pass": "conv", '
    '"length": 64, "variant": 1, "occupancy": 0, "us": 1.0}]}',
    '{"format": "fsa-tune-1", "arch": "", "entries": [{"precision": "f16", "pass": "conv", '
    '"length": 512, "variant": 0, "occupancy": 0, "us": 1.0}]}',
    '{"format": "fsa-tune-1", "arch": "", "entries": [{"precision": "f32", "pass": "conv", '
    '"length": 512.5, "variant": 0, "occupancy": 0, "us": 1.0}]}',
    '{"format": "fsa-tune-1", "arch": "", "entries": [{"precision": "f32", "pass": "conv", '
    '"length": 1e300, "variant": 0, "occupancy": 0, "us": 1.0}]}',
])
def test_load_rejects_bad_files_as_a_whole(tmp_path, text):
    F.tune_set("f32", "conv", 512, 1, 0)
    path = tmp_path / "bad.json"
    path.write_text(text)
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.tune_load(str(path))
    assert F.tune_get("f32", "conv", 512)[:2] == (1, 0)   # table untouched


def test_load_missing_file():
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.tune_load("/nonexistent/tune.json")


def test_slab_schedule_table(tmp_path):
    assert F.tune_get_slabs("f32", (256, 256, 256)) == (1, 0.0)
    F.tune_set_slabs("f32", (256, 256, 256), 4)
    F.tune_set_slabs("f64", (128, 64, 256), 2)
    assert F.tune_get_slabs("f32", (256, 256, 256))[0] == 4
    assert F.tune_get_slabs("f64", (256, 256, 256))[0] == 1
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.tune_set_slabs("f32", (256, 256, 256), 17)
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.tune_set_slabs("f32", (250, 256, 256), 2)
    path = tmp_path / "t.json"
    F.tune_save(str(path))
    F.tune_reset()
    assert F.tune_get_slabs("f32", (256, 256, 256))[0] == 1
    F.tune_load(str(path))
    assert F.tune_get_slabs("f32", (256, 256, 256))[0] == 4
    assert F.tune_get_slabs("f64", (128, 64, 256))[0] == 2


def test_entries_are_kept_per_size_class():
    # a 256^3 grid's pencils (131584) and a 256^2 grid's (257) fall in
    # different classes; each launch takes the nearest tuned class
    F.tune_set("f32", "conv", 512, 2, 0, lines=131584)
    F.tune_set("f32", "conv", 512, 1, 0, lines=257)
    assert F.tune_get("f32", "conv", 512, 131584)[:2] == (2, 0)
    assert F.tune_get("f32", "conv", 512, 100000)[:2] == (2, 0)   # same class
    assert F.tune_get("f32", "conv", 512, 257)[:2] == (1, 0)
    assert F.tune_get("f32", "conv", 512, 300)[:2] == (1, 0)      # nearest: 2^8
    assert F.tune_get("f32", "conv", 512, 13000)[:2] == (2, 0)    # nearest: 2^17 vs 2^8
    assert F.tune_get("f32", "conv", 1024, 257)[:2] == (0, 0)     # other length: default


def test_batched_entries_are_kept_apart(tmp_path):
    """Entries of the batched launches (FSA_PASS_BATCHED) do not change the
    single-evaluation choices; a batched launch without a batched entry of
    its (precision, pass, length) takes the single-evaluation entry; both
    kinds survive a save / load."""
    F.tune_reset()
    F.tune_set("f32", "r2c", 256, 0, 0, lines=65536)
    F.tune_set("f32", "batched_r2c", 256, 1, 2, lines=70400)   # same size class
    assert F.tune_get("f32", "r2c", 256, 65536) == (0, 0, 0.0)
    assert F.tune_get("f32", "batched_r2c", 256, 70400)[:2] == (1, 2)
    F.tune_set("f32", "conv", 2048, 2, 0, lines=1025)
    assert F.tune_get("f32", "batched_conv", 2048, 73842)[:2] == (2, 0)   # fallback
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.tune_set("f32", "batched_conv", 64, 1)    # same variant rules as the pass
    assert F.tune_variants("f32", "batched_conv", 512) == F.tune_variants("f32", "conv", 512)
    path = tmp_path / "tune.json"
    F.tune_save(str(path))
    names = sorted(e["pass"] for e in json.loads(path.read_text())["entries"])
    assert names == ["batched_r2c", "conv", "r2c"]
    F.tune_reset()
    F.tune_load(str(path))
    assert F.tune_get("f32", "batched_r2c", 256, 70400)[:2] == (1, 2)
    assert F.tune_get("f32", "r2c", 256, 65536)[:2] == (0, 0)
    F.tune_reset()


def test_load_survives_mangled_files(tmp_path):
    """Random damage to a valid table file (deleted, duplicated, swapped or
    replaced bytes) either loads or is rejected with FSA_EINVAL; the parser
    never crashes or hangs, and a rejected file leaves the table untouched."""
    import random
    F.tune_reset()
    F.tune_set("f32", "conv", 512, 1, 0)
    F.tune_set("f32", "fwd_t", 512, 2, 1)
    F.tune_set_slabs("f64", (256, 256, 256), 2)
    good = tmp_path / "good.json"
    F.tune_save(str(good))
    text = good.read_text()
    rng = random.Random(7)
    alphabet = '{}[]":,.-+eE0123456789 \n\tabcfnrstu\\'
    for trial in range(300):
        s = list(text)
        for _ in range(rng.randint(1, 6)):
            i = rng.randrange(len(s)) if s else 0
            op = rng.randrange(4)
            if op == 0 and s:
                del s[i]
            elif op == 1:
                s.insert(i, rng.choice(alphabet))
            elif op == 2 and s:
                s[i] = rng.choice(alphabet)
            elif s:
                j = rng.randrange(len(s))
                s[i], s[j] = s[j], s[i]
        path = tmp_path / f"m{trial}.json"
        path.write_text("".join(s))
        F.tune_reset()
        F.tune_set("f32", "conv", 512, 1, 0)
        try:
            F.tune_load(str(path))
        except F.FsaError as e:
            assert "EINVAL" in str(e)
            assert F.tune_get("f32", "conv", 512)[:2] == (1, 0)
    F.tune_reset()


def test_lane_exchange_and_matrix_core_variants_only_at_512():
    """Variant 3 (exchanges across lanes) exists only for the fused pass at
    length 512, the one-wave 8 * 8 * 8 plan, in both precisions; variant 4
    (first stage on the matrix cores) only there in FP32."""
    for prec in ("f32", "f64"):
        for p in (256, 384, 512, 768, 1024, 2048):
            assert (3 in F.tune_variants(prec, "conv", p)) == (p == 512), (prec, p)
            assert (4 in F.tune_variants(prec, "conv", p)) == (p == 512 and prec == "f32"), (prec, p)
        for name in ("r2c", "c2r", "fwd_t", "inv_t"):
            for n in (256, 512, 1024):
                assert not {3, 4} & set(F.tune_variants(prec, name, n)), (prec, name, n)

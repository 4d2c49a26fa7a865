"""CPU tests of the autotuner's cache file (no device work): a file written by hand loads, merges by key and
is written back field for field; malformed files are refused with SSQA_EINVAL and a message, leaving the
cache unchanged."""

import json

import pytest

lib_mod = pytest.importorskip("paper_2302_12454_amd._lib")


@pytest.fixture()
def api():
    try:
        lib_mod.load()
    except ImportError as e:
        pytest.fail(str(e))
    import paper_2302_12454_amd as api
    api.ssqa_tune_clear()
    yield api
    api.ssqa_tune_clear()


PLAIN = {"form": "plain", "device": "AMD Instinct MI355X|gfx950:sramecc+:xnack-|256", "kernel": "0123456789abcdef",
         "np": 2560, "planes": 1, "replicas": 64, "trials": 1024, "delay": 1, "mode": 0, "fast": 1, "fp4_ok": 1,
         "block_columns": 128, "trials_per_block": 2, "operand_format": 2, "ms_per_cycle": 0.1875}
BATCH = {"form": "batch", "device": "AMD Instinct MI355X|gfx950:sramecc+:xnack-|256", "kernel": "0123456789abcdef",
         "signature": "00ff00ff00ff00ff", "instances": 512, "wide_rows": 1024, "ms_per_cycle": 1.125}


def _write(path, obj):
    path.write_text(obj if isinstance(obj, str) else json.dumps(obj))
    return str(path)


def test_roundtrip_and_merge(api, tmp_path):
    src = _write(tmp_path / "a.json", {"format": "ssqa-tune-1", "entries": [PLAIN, BATCH]})
    assert api.ssqa_tune_load(src) == 2
    assert api.ssqa_tune_entries() == 2
    assert api.ssqa_tune_load(src) == 2          # same keys: replaced, not duplicated
    assert api.ssqa_tune_entries() == 2
    other = dict(PLAIN, trials=512, trials_per_block=1, ms_per_cycle=0.25)
    assert api.ssqa_tune_load(_write(tmp_path / "b.json", {"format": "ssqa-tune-1", "entries": [other]})) == 1
    assert api.ssqa_tune_entries() == 3
    out = tmp_path / "out.json"
    api.ssqa_tune_save(str(out))
    back = json.loads(out.read_text())
    assert back["format"] == "ssqa-tune-1"
    assert sorted(json.dumps(e, sort_keys=True) for e in back["entries"]) == \
        sorted(json.dumps(e, sort_keys=True) for e in (PLAIN, BATCH, other))
    api.ssqa_tune_clear()
    assert api.ssqa_tune_entries() == 0
    assert api.ssqa_tune_load(str(out)) == 3


@pytest.mark.parametrize("text,needle", [
    ("not json", "unexpected token"),
    ("[1, 2", "expected ',' or ']'"),
    ("@", "expected a value"),
    ('{"format": "ssqa-tune-1", "entries": [', "unexpected end"),
    ('{"format": "other", "entries": []}', "format"),
    ('{"format": "ssqa-tune-1", "entries": {}}', "entries"),
    ('{"format": "ssqa-tune-1", "entries": []} trailing', "trailing"),
    (json.dumps({"format": "ssqa-tune-1", "entries": [dict(PLAIN, block_columns=96)]}), "block width"),
    (json.dumps({"format": "ssqa-tune-1", "entries": [dict(PLAIN, np=2500)]}), "padded size"),
    (json.dumps({"format": "ssqa-tune-1", "entries": [{k: v for k, v in PLAIN.items() if k != "trials"}]}),
     "'trials'"),
    (json.dumps({"format": "ssqa-tune-1", "entries": [dict(PLAIN, delay=9)]}), "'delay'"),
    (json.dumps({"format": "ssqa-tune-1", "entries": [dict(PLAIN, ms_per_cycle=-1)]}), "ms_per_cycle"),
    (json.dumps({"format": "ssqa-tune-1", "entries": [dict(BATCH, signature="xyz")]}), "signature"),
    (json.dumps({"format": "ssqa-tune-1", "entries": [dict(BATCH, form="served")]}), "form"),
    (json.dumps({"format": "ssqa-tune-1", "entries": [PLAIN, dict(PLAIN, operand_format=3)]}), "operand_format"),
])
def test_malformed_files_are_refused(api, tmp_path, text, needle):
    good = _write(tmp_path / "good.json", {"format": "ssqa-tune-1", "entries": [BATCH]})
    assert api.ssqa_tune_load(good) == 1
    with pytest.raises(api.SSQAError) as err:
        api.ssqa_tune_load(_write(tmp_path / "bad.json", text))
    assert err.value.name == "SSQA_EINVAL" and needle in str(err.value), str(err.value)
    assert api.ssqa_tune_entries() == 1            # nothing merged from the refused file


def test_missing_file_and_unwritable_path(api, tmp_path):
    with pytest.raises(api.SSQAError):
        api.ssqa_tune_load(str(tmp_path / "absent.json"))
    with pytest.raises(api.SSQAError):
        api.ssqa_tune_save(str(tmp_path / "no_such_dir" / "x.json"))

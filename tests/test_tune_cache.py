"""Host logic of the autotuner: cache key buckets and the JSON cache file
(reader strictness, write-then-rename, never overwriting an unreadable file).
Built with g++ from the header the library itself includes."""
import json
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def tool(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tune") / "tune_cache_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-o", exe,
                    os.path.join(HERE, "tune_cache_check.cpp")], check=True)

    def run(*args):
        return subprocess.run([exe, *map(str, args)], check=True, capture_output=True, text=True).stdout
    return run


def test_key_buckets(tool):
    assert tool("key", "gfx950", 256, 0, 16, 100000, 1).strip() == "gfx950/cu256/fp64/kc16/n2^17/s2^0"
    assert tool("key", "gfx950", 256, 1, 32, 131072, 256).strip() == "gfx950/cu256/mixed/kc32/n2^17/s2^8"
    assert tool("key", "gfx950", 256, 1, 32, 131073, 257).strip() == "gfx950/cu256/mixed/kc32/n2^18/s2^9"


def test_missing_file_is_empty_and_round_trip(tool, tmp_path):
    p = tmp_path / "cache.json"
    assert tool("load", p).split() == ["ok", "0"]
    assert tool("put", p, "a/b", 32, 2, 64, 16, 2, 2, 1.5, 0.0812).strip() == "stored"
    assert tool("put", p, "c/d", 16, 3, 256, 64, 1, 1, 1.0, 1.25).strip() == "stored"
    data = json.loads(p.read_text())  # the file is plain JSON
    assert data["a/b"] == {"resort_every": 32, "device_rounds": 2, "repair_cells": 64, "tail_items": 16,
                           "full_rounds": 2, "force_mode": 2, "bin_factor": 1.5, "ms_per_step": 0.0812}
    out = tool("load", p).splitlines()
    assert out[0] == "ok 2"
    f = out[1].split()
    assert f[:7] == ["a/b", "32", "2", "64", "16", "2", "2"] and float(f[7]) == 1.5 and float(f[8]) == 0.0812
    assert not os.path.exists(str(p) + ".tmp")


@pytest.mark.parametrize("text", [
    "",                                      # empty file
    "[]",                                    # not an object
    '{"k": {"resort_every": 32}}',           # missing knobs
    '{"k": {"resort_every": 32, "device_rounds": 2, "repair_cells": 64, "tail_items": 8, "full_rounds": 1, "force_mode": 1, "bin_factor": 1.0, "x": 1}}',
    '{"k": {"resort_every": 32, "device_rounds": 2, "repair_cells": 64, "tail_items": 8, "full_rounds": 1, "force_mode": 1, "bin_factor": 99}}',
    '{"k": {"resort_every": 32, "device_rounds": 0, "repair_cells": 64, "tail_items": 8, "full_rounds": 1, "force_mode": 1, "bin_factor": 1}}',
    '{"k": {"resort_every": "32", "device_rounds": 2, "repair_cells": 64, "tail_items": 8, "full_rounds": 1, "force_mode": 1, "bin_factor": 1}}',
    '{"k": {"resort_every": 32, "device_rounds": 2, "repair_cells": 64, "tail_items": 8, "full_rounds": 1, "force_mode": 1, "bin_factor": 1}} x',
    '{"k": {"resort_every": 32, "device_rounds": 2, "repair_cells": 64, "tail_items": 8, "full_rounds": 1, "bin_factor": 1}}',
    '{"k": {"resort_every": 32, "device_rounds": 2, "repair_cells": 64, "tail_items": 8, "full_rounds": 1, "force_mode": 3, "bin_factor": 1}}',
    '{"k": {"resort_every": 32, "device_rounds": 2, "repair_cells": 64, "bin_factor": 1, "ms_per_step": 1}}',
])
def test_malformed_cache_is_rejected_and_kept(tool, tmp_path, text):
    p = tmp_path / "cache.json"
    p.write_text(text)
    assert tool("load", p).strip() == "bad"
    assert tool("put", p, "a/b", 32, 2, 64, 8, 1, 1, 1.0, 0.1).strip() == "refused"
    assert p.read_text() == text

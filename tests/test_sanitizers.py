"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle's C entry points (both models) on small seeded systems, and the
library's tuning-cache reader and writer on well-formed and malformed
files.  Any sanitizer report fails the run (no recovery)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _have_sanitizer_runtime(cc):
    probe = subprocess.run([cc, "-fsanitize=address,undefined", "-x", "c", "-", "-o", os.devnull],
                           input="int main(void){return 0;}", capture_output=True, text=True)
    return probe.returncode == 0


@pytest.fixture(scope="module")
def tmp(tmp_path_factory):
    if not shutil.which("gcc") or not _have_sanitizer_runtime("gcc"):
        pytest.skip("gcc with sanitizer runtimes not available")
    return tmp_path_factory.mktemp("san")


def test_oracle_under_sanitizers(tmp):
    exe = str(tmp / "oracle_san")
    subprocess.run(["gcc", "-std=c11", "-ffp-contract=off", *SAN, "-o", exe,
                    os.path.join(HERE, "sanitize_oracle_main.c"), "-lm"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_avm_oracle_under_sanitizers(tmp):
    exe = str(tmp / "avm_oracle_san")
    odir = os.path.join(HERE, "..", "oracle")
    subprocess.run(["gcc", "-std=c11", "-ffp-contract=off", *SAN, "-o", exe, os.path.join(HERE, "sanitize_avm_main.c"),
                    os.path.join(odir, "spv_oracle.c"), os.path.join(odir, "avm_oracle.c"), "-lm"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized avm oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_tune_cache_under_sanitizers(tmp):
    exe = str(tmp / "tune_san")
    subprocess.run(["g++", "-std=c++17", *SAN, "-Wall", "-Werror", "-o", exe,
                    os.path.join(HERE, "tune_cache_check.cpp")], check=True)
    p = tmp / "cache.json"

    def run(*args):
        r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, env=ENV, timeout=60)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "runtime error" not in r.stderr
        return r.stdout.strip()
    assert run("load", p).split() == ["ok", "0"]
    assert run("put", p, "a/b", 32, 2, 64, 16, 2, 2, 1.5, 0.08) == "stored"
    assert run("load", p).splitlines()[0] == "ok 1"
    for text in ("", "{", '{"k": {"resort_every": 1e999}}', '{"k": [1, 2, 3]}', '{"k": {"a": "\\u0000"}}',
                 '{"k": {"resort_every": 32, "device_rounds": 2, "repair_cells": 64, "tail_items": 8, '
                 '"full_rounds": 1, "force_mode": 1, "bin_factor": 1}} trailing'):
        p.write_text(text)
        assert run("load", p) == "bad"
    assert run("key", "gfx950", 256, 0, 16, 100000, 1) == "gfx950/cu256/fp64/kc16/n2^17/s2^0"

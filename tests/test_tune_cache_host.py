"""The autotuner's JSON cache (host code of the library, compiled here with
g++ into a small driver): round trip of entries, the file readable by a
standard JSON parser, unknown fields skipped, and files that are not a
tuning cache refused."""

import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1710_08830_amd", "csrc")

DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include <string>
#include "tune_cache.h"
// read IN; print "OK" and every entry, or "ERR <message>"; with a third
// argument, add the entry "k\"ey|x" {"v": 3, "w": 0.25} and write it to OUT
int main(int argc, char **argv) {
  tufrg::TuneEntries e;
  std::string err;
  if (!tufrg::tune_cache_read(argv[1], e, err)) { std::printf("ERR %s\n", err.c_str()); return 0; }
  std::printf("OK\n");
  for (auto &kv : e)
    for (auto &p : kv.second) std::printf("%s|%s=%.17g\n", kv.first.c_str(), p.first.c_str(), p.second);
  if (argc > 2) {
    e["k\"ey|x"] = {{"v", 3.0}, {"w", 0.25}};
    if (!tufrg::tune_cache_write(argv[2], e, err)) { std::printf("WERR %s\n", err.c_str()); return 1; }
  }
  return 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("tune")
    (d / "driver.cpp").write_text(DRIVER)
    exe = d / "driver"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I" + SRC, "-x", "c++", os.path.join(SRC, "tune_cache.hip"),
                    str(d / "driver.cpp"), "-o", str(exe)], check=True, capture_output=True, timeout=120)
    return exe


def run(exe, *args):
    return subprocess.run([str(exe), *map(str, args)], capture_output=True, text=True, timeout=30).stdout.splitlines()


def test_missing_file_is_an_empty_cache_and_round_trip(driver, tmp_path):
    a, b = tmp_path / "none.json", tmp_path / "b.json"
    assert run(driver, a, b) == ["OK"]
    doc = json.loads(b.read_text())
    assert doc == {"version": 1, "entries": {'k"ey|x': {"v": 3, "w": 0.25}}}
    out = run(driver, b, tmp_path / "c.json")
    assert out == ["OK", 'k"ey|x|v=3', 'k"ey|x|w=0.25']
    assert json.loads((tmp_path / "c.json").read_text()) == doc
    assert not [p for p in os.listdir(tmp_path) if ".tmp." in p]


def test_unknown_fields_are_skipped_and_numbers_kept_exactly(driver, tmp_path):
    p = tmp_path / "x.json"
    p.write_text(json.dumps({"note": ["a", {"b": [1, 2]}, True, None], "version": 1,
                             "entries": {"gfx950:256cu|n_o=2": {"loop_kx_chunks": 8, "loop_ms": 1.8712345678901234,
                                                               "default_ms": 1.9e-3}}}))
    out = run(driver, p)
    assert out[0] == "OK"
    vals = dict(line.rsplit("|", 1)[1].split("=") for line in out[1:])
    assert int(vals["loop_kx_chunks"]) == 8
    assert float(vals["loop_ms"]) == 1.8712345678901234 and float(vals["default_ms"]) == 1.9e-3


@pytest.mark.parametrize("text", ["not json", "{}", '{"version": 1}', '{"entries": {"k": {"v": "x"}}}',
                                  '{"entries": {}} trailing', '{"entries": {"k": [1]}}', ""])
def test_files_that_are_not_a_tuning_cache_are_refused(driver, tmp_path, text):
    p = tmp_path / "bad.json"
    p.write_text(text)
    out = run(driver, p, tmp_path / "out.json")
    assert out and out[0].startswith("ERR ") and "not a tuning cache" in out[0]
    assert not (tmp_path / "out.json").exists() and p.read_text() == text


def test_empty_entries_are_a_valid_cache(driver, tmp_path):
    p = tmp_path / "e.json"
    p.write_text('{"version": 1, "entries": {}}')
    assert run(driver, p) == ["OK"]

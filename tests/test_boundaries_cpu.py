"""Structural boundaries: the product path has no CPU fallback and never
touches the oracle; the oracle is independent of the product; the shared
input generators depend on neither."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sources(sub, exts=(".py", ".hip", ".cpp", ".h")):
    base = os.path.join(ROOT, sub)
    for dp, _, fs in os.walk(base):
        for f in fs:
            if f.endswith(exts):
                yield os.path.join(dp, f)


def test_library_missing_fails_loudly(monkeypatch, tmp_path):
    from paper_2506_04891_amd import tqsim
    monkeypatch.setattr(tqsim, "_lib", None)
    monkeypatch.setattr(tqsim, "LIB_PATH", str(tmp_path / "libtqsim.so"))
    with pytest.raises(ImportError):
        tqsim.lib()
    with pytest.raises(ImportError):
        tqsim.Circuit(2, [], "c64")


def test_product_never_uses_the_oracle():
    for path in _sources("paper_2506_04891_amd"):
        text = open(path).read()
        assert not re.search(r"^\s*(from|import)\s+oracle\b", text, re.M), path
        assert not re.search(r"\boracle\.\w", text), path


def test_oracle_is_independent_of_the_product():
    for path in _sources("oracle"):
        text = open(path).read()
        assert "paper_2506_04891_amd" not in text and "tqsim" not in text.replace("TQml", ""), path


def test_input_generators_import_neither_side():
    for path in _sources("workloads"):
        text = open(path).read()
        assert not re.search(r"^\s*(from|import)\s+(oracle|paper_2506_04891_amd)\b", text, re.M), path


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asking for more ends with a message."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_committed_code_does_not_use_working_files():
    """Nothing committed imports, reads or runs a file of the scratch folder."""
    import subprocess
    files = subprocess.run(["git", "-C", ROOT, "ls-files"], capture_output=True, text=True).stdout.split()
    pat = re.compile(r"_work[/\\]")
    bad = []
    for f in files:
        if not f.endswith((".py", ".hip", ".cpp", ".h", ".inc", ".sh", ".toml", ".cfg")):
            continue
        with open(os.path.join(ROOT, f), errors="replace") as fh:
            if pat.search(fh.read()):
                bad.append(f)
    assert not bad, bad

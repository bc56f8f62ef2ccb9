"""Host-side checks of the product boundary: the library and its binding never
reach into the oracle, and bench.py refuses more than one GPU."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2401_17018_amd")


def _product_files():
    for base, _, files in os.walk(PKG):
        if "_build" in base or "__pycache__" in base:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                yield os.path.join(base, f)


def test_product_path_does_not_use_the_oracle():
    for path in _product_files():
        text = open(path).read()
        assert not re.search(r"\boracle\b|libo2|o2_run", text), path


def test_binding_has_no_cpu_fallback():
    text = open(os.path.join(PKG, "capi.py")).read()
    assert "raise RuntimeError" in text and "not built" in text


def test_bench_refuses_multi_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr

"""Host-side parts of bench.py that need no GPU: the one-GPU refusal and the
algorithmic FLOP count of an evaluation (the roofline's numerator), which
for the slit row must be 128 (12 x 42 + 71) + 128 (3 x 42 + 71) = 98,816."""
import importlib.util
import os
import subprocess
import sys

import pytest

import synth_inputs as si

ROOT = os.path.join(os.path.dirname(__file__), "..")


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_flops_per_evaluation_of_the_slit_row():
    g = pytest.importorskip("paper_1208_0302_amd")
    try:
        g.lib()
    except RuntimeError:
        pytest.skip("library not built")
    b = _bench()
    lines = []
    for ln, n in si.line_set("slit"):
        st, sp = si.grid(ln, n)
        lines.append((g.line_from_terms(ln["lambda0"], ln["Jl"], ln["gl"], ln["Ju"], ln["gu"]),
                      g.grid(st, sp, n)))
    assert [ln.ncomp for ln, _ in lines] == [12, 3]
    assert b.flops_per_eval(lines) == 98816

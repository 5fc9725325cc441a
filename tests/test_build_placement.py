"""The build's code-placement step (paper_1208_0302_amd/build.py) reports what
it did: "unchecked" with a reason when its tools are missing or fail, and an
error when the entry shift does not fix a kernel's placement.  No compiler or
device is run: the tools and the recompile are replaced by fakes."""
import subprocess

import pytest

from paper_1208_0302_amd import build as B


def test_missing_tools_give_unchecked(tmp_path, monkeypatch):
    lib = tmp_path / "lib.so"
    lib.write_bytes(b"x")
    monkeypatch.setattr(B, "_llvm", lambda tool: None)
    monkeypatch.setattr(B.shutil, "which", lambda tool: None)
    out, rec = B.place(str(lib), {}, False, str(tmp_path),
                       compile_fn=lambda *a: pytest.fail("must not recompile"))
    assert out == str(lib)
    assert rec["placement"] == "unchecked"
    assert "llvm-objdump" in rec["reason"] and "objcopy" in rec["reason"]


def test_failing_tool_gives_unchecked(tmp_path, monkeypatch):
    lib = tmp_path / "lib.so"
    lib.write_bytes(b"x")

    def boom(so, wd):
        raise subprocess.CalledProcessError(1, ["objcopy"])
    monkeypatch.setattr(B, "_code_objects", boom)
    out, rec = B.place(str(lib), {}, False, str(tmp_path))
    assert out == str(lib) and rec["placement"] == "unchecked" and "objcopy" in rec["reason"]


def _fake(tmp_path, monkeypatch, after):
    """Kernels all badly placed in the first build; `after` gives the
    (good, bad) counts of the shifted build."""
    first = tmp_path / "first.so"
    first.write_bytes(b"1")
    state = {"built": 0}

    def compile_fn(pads, verbose):
        state["built"] += 1
        state["pads"] = pads
        p = tmp_path / "second.so"
        p.write_bytes(b"2")
        return str(p)
    monkeypatch.setattr(B, "_code_objects", lambda so, wd: [so])
    monkeypatch.setattr(B, "placement",
                        lambda cos, pat: (10, 90) if cos[0].endswith("first.so") else after)
    monkeypatch.setattr(B, "code_sha256", lambda cos, pat: "code of " + cos[0][-9:] + pat)
    return str(first), compile_fn, state


def test_shift_is_recorded(tmp_path, monkeypatch):
    first, compile_fn, state = _fake(tmp_path, monkeypatch, (90, 10))
    out, rec = B.place(first, {k: 0 for k in B.PLACEMENT}, False, str(tmp_path), compile_fn)
    assert state["built"] == 1 and out.endswith("second.so")
    assert rec["placement"] == "checked"
    assert all(rec[k] == {"shift": 1, "good": 90, "bad": 10,
                          "code_sha256": "code of second.so" + B.PLACEMENT[k]}
               for k in B.PLACEMENT)
    assert all(v == 1 for v in state["pads"].values())


def test_shift_that_does_not_help_raises(tmp_path, monkeypatch):
    first, compile_fn, _ = _fake(tmp_path, monkeypatch, (40, 60))
    with pytest.raises(RuntimeError, match="placement"):
        B.place(first, {k: 0 for k in B.PLACEMENT}, False, str(tmp_path), compile_fn)


def test_code_hash_follows_the_machine_code(tmp_path, monkeypatch):
    # the hash covers the matching symbols' instruction encodings only
    dumps = {"a.co": ("  0 g F .text 0 k_ga_invertIfLi0ELb0E\n  0 g F .text 0 k_other\n",
                      "  s_mov_b32 s0, 1 // 000000001000: BE800081\n"),
             "b.co": ("  0 g F .text 0 k_ga_invertIfLi0ELb0E\n",
                      "  s_mov_b32 s0, 2 // 000000001000: BE800082\n")}

    class R:
        def __init__(self, out):
            self.stdout = out

    def run(cmd, **kw):
        co = cmd[-1]
        return R(dumps[co][0] if cmd[1] == "-t" else dumps[co][1])
    monkeypatch.setattr(B.subprocess, "run", run)
    monkeypatch.setattr(B, "_llvm", lambda tool: tool)
    ha = B.code_sha256(["a.co"], r"k_ga_invertIfLi0ELb0E")
    hb = B.code_sha256(["b.co"], r"k_ga_invertIfLi0ELb0E")
    assert ha != hb and len(ha) == 64
    assert ha == B.code_sha256(["a.co"], r"k_ga_invertIfLi0ELb0E")


def test_layout_of_missing_record(tmp_path, monkeypatch):
    monkeypatch.setattr(B, "LAYOUT", str(tmp_path / "none.json"))
    assert B.layout() == {"placement": "unknown"}

"""Build libgenesis_hip.so for gfx950 in-tree with hipcc.

The library is a plain C-ABI shared object (include/genesis.h); the Python
binding in this package only loads it with ctypes.
"""
from __future__ import annotations

import json
import os
import re
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libgenesis_hip.so")
SRCS = [os.path.join(HERE, "csrc", f) for f in ("genesis.hip", "serving.hip", "mlp.hip",
                                                 "uncert.hip")]
DEPS = SRCS + [os.path.join(HERE, "csrc", f) for f in
               ("genesis_device.h", "genesis_common.h", "genesis_half.h", "voigt_rational.h",
                "voigt_rational_h.h", "weideman36.h", "weideman28.h", "scheduler.h")] + \
       [os.path.join(ROOT, "include", "genesis.h")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # reproducible arithmetic: FMAs only where the source asks for them
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


# Code placement of the hot kernels (see code_shift in csrc/genesis_common.h):
# switch -> mangled-name pattern of the kernel it moves.
PLACEMENT = {
    "GENESIS_PAD_INVERT_F32": r"k_ga_invertIfLi0ELb0E",
    "GENESIS_PAD_INVERT_F16": r"k_ga_invertIfLi1ELb0E",
    "GENESIS_PAD_INVERT_F64": r"k_ga_invertIdLi0ELb0E",
    "GENESIS_PAD_FILL_F32": r"k_ga_invertIfLi0ELb1E",
    "GENESIS_PAD_FILL_F16": r"k_ga_invertIfLi1ELb1E",
    "GENESIS_PAD_FILL_F64": r"k_ga_invertIdLi0ELb1E",
    "GENESIS_PAD_ADVANCE": r"k_ga_advance",
    "GENESIS_PAD_REFINE": r"k_refine_f64",
}
LAYOUT = os.path.join(HERE, "libgenesis_hip.layout.json")


def _llvm(tool):
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "llvm", "bin", tool)
    return cand if os.path.exists(cand) else shutil.which(tool)


def _code_objects(so, workdir):
    """The gfx950 code objects embedded in the shared library (our own build):
    one offload bundle per translation unit in the .hip_fatbin section."""
    fat = os.path.join(workdir, "fatbin")
    objcopy = shutil.which("objcopy") or _llvm("llvm-objcopy")
    bundler = _llvm("clang-offload-bundler")
    if not objcopy or not bundler or not _llvm("llvm-objdump"):
        return None
    subprocess.run([objcopy, "-O", "binary", "--only-section=.hip_fatbin", so, fat], check=True)
    data = open(fat, "rb").read()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    starts = [i for i in range(len(data)) if data.startswith(magic, i)]
    out = []
    for n, a in enumerate(starts):
        b = starts[n + 1] if n + 1 < len(starts) else len(data)
        part = os.path.join(workdir, "bundle%d" % n)
        with open(part, "wb") as f:
            f.write(data[a:b])
        co = os.path.join(workdir, "gfx950_%d.co" % n)
        subprocess.run([bundler, "--unbundle", "--type=o", "--input=" + part, "--output=" + co,
                        "--targets=hipv4-amdgcn-amd-amdhsa--gfx950"], check=True)
        out.append(co)
    return out


_ADDR = re.compile(r"//\s*([0-9A-F]{12}):\s*([0-9A-F ]+)")
_TARGET = re.compile(r"<[^>]*\+0x([0-9a-f]+)>")


def placement(cos, pattern):
    """(good, bad): 8-byte instructions of the kernel's innermost loops that
    start at 4 (mod 8), resp. 0 (mod 8)."""
    good = bad = 0
    for co in cos:
        g, b = _placement_one(co, pattern)
        good += g
        bad += b
    return good, bad


def _placement_one(co, pattern):
    table = subprocess.run([_llvm("llvm-objdump"), "-t", co], capture_output=True,
                           text=True).stdout
    syms = [l.split()[-1] for l in table.splitlines()
            if " F .text" in l and re.search(pattern, l.split()[-1])]
    good = bad = 0
    for sym in syms:
        out = subprocess.run([_llvm("llvm-objdump"), "-d", "--disassemble-symbols=" + sym, co],
                             capture_output=True, text=True).stdout
        insts, loops = [], []
        for line in out.splitlines():
            m = _ADDR.search(line)
            if not m:
                continue
            a = int(m.group(1), 16)
            insts.append((a, 4 * len(m.group(2).split()), line.split("//")[0].strip()))
            t = _TARGET.search(line)
            if t and "branch" in line:
                tgt = insts[0][0] + int(t.group(1), 16)
                if tgt < a:
                    loops.append((tgt, a))
        inner = [(t, a) for t, a in loops
                 if not any(t <= t2 and a2 <= a and (t2, a2) != (t, a) for t2, a2 in loops)]
        for t, a in inner:
            body = [(x, size, txt) for x, size, txt in insts if t <= x <= a]
            # profile loops: one reciprocal per Zeeman component and wavelength
            if sum(1 for _, _, txt in body if txt.startswith("v_rcp")) < 4:
                continue
            for x, size, _ in body:
                if size == 8:
                    if x % 8:
                        good += 1
                    else:
                        bad += 1
    return good, bad


def code_sha256(cos, pattern):
    """SHA-256 of the machine code of the kernels whose symbols match
    `pattern` (their instruction encodings in symbol order): a record of
    measurements of a kernel stays valid exactly while this is unchanged."""
    import hashlib
    h = hashlib.sha256()
    for co in cos:
        table = subprocess.run([_llvm("llvm-objdump"), "-t", co], capture_output=True,
                               text=True).stdout
        syms = sorted(l.split()[-1] for l in table.splitlines()
                      if " F .text" in l and re.search(pattern, l.split()[-1]))
        for sym in syms:
            out = subprocess.run([_llvm("llvm-objdump"), "-d", "--disassemble-symbols=" + sym,
                                  co], capture_output=True, text=True).stdout
            h.update(sym.encode())
            for line in out.splitlines():
                m = _ADDR.search(line)
                if m:
                    h.update(m.group(2).encode())
    return h.hexdigest()


def _compile(pads, verbose):
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-D%s=%d" % kv for kv in sorted(pads.items())] + \
          ["-o", tmp] + SRCS
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building %s" % SO)
    return tmp


def place(tmp, pads, verbose, workdir, compile_fn=None):
    """Check the hot kernels' placement in the library `tmp` and recompile
    with a one-s_nop entry shift where most 8-byte instructions of a kernel's
    innermost loops start at 0 (mod 8).  Returns (library, record).  The
    record says "checked" with the counts, or "unchecked" with the reason when
    the tools are missing or fail (the library is then the unshifted build,
    which may run a hot kernel up to 20 % slower).  Raises if a shifted
    kernel still has more instructions at 0 (mod 8) than at 4."""
    compile_fn = compile_fn or _compile
    try:
        co = _code_objects(tmp, workdir)
        if co is None:
            missing = [t for t in ("objcopy", "clang-offload-bundler", "llvm-objdump")
                       if not (shutil.which(t) if t == "objcopy" else _llvm(t))]
            return tmp, {"placement": "unchecked",
                         "reason": "missing tool(s): %s" % ", ".join(missing or ["?"])}
        counts = {k: placement(co, p) for k, p in PLACEMENT.items()}
        flip = {k: 1 for k, (g, b) in counts.items() if b > g}
        if flip:
            os.remove(tmp)
            pads = dict(pads, **flip)
            tmp = compile_fn(pads, verbose)
            co = _code_objects(tmp, workdir)
            counts = {k: placement(co, p) for k, p in PLACEMENT.items()}
            worse = [k for k in flip if counts[k][1] > counts[k][0]]
            if worse:
                raise RuntimeError("code placement: the entry shift left more 8-byte loop "
                                   "instructions at 0 (mod 8) than at 4 in %s" % worse)
        hashes = {k: code_sha256(co, p) for k, p in PLACEMENT.items()}
    except (subprocess.CalledProcessError, OSError) as e:
        return tmp, {"placement": "unchecked", "reason": str(e)}
    record = {"placement": "checked"}
    record.update({k: {"shift": pads.get(k, 0), "good": counts[k][0], "bad": counts[k][1],
                       "code_sha256": hashes[k]}
                   for k in PLACEMENT})
    return tmp, record


def build(verbose: bool = False) -> str:
    """Compile; then place each hot kernel so that most 8-byte instructions of
    its innermost loops start at 4 (mod 8), recompiling with the shift where
    the first placement is the other one.  The outcome is written to
    libgenesis_hip.layout.json (and warned about on stderr when unchecked)."""
    pads = {k: 0 for k in PLACEMENT}
    tmp = _compile(pads, verbose)
    with tempfile.TemporaryDirectory() as wd:
        tmp, record = place(tmp, pads, verbose, wd)
    if record["placement"] != "checked":
        sys.stderr.write("WARNING: code placement unchecked (%s); hot kernels may run up to "
                         "20 %% slower\n" % record["reason"])
    os.replace(tmp, SO)
    with open(LAYOUT, "w") as f:
        json.dump(record, f, indent=1)
    if verbose:
        print(json.dumps(record), flush=True)
    return SO


def layout():
    """The placement record of the installed library ({"placement": "unknown"}
    when there is none)."""
    try:
        with open(LAYOUT) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {"placement": "unknown"}


def stale() -> bool:
    if not os.path.exists(SO):
        return True
    t = os.path.getmtime(SO)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))

"""The gfx950 code of every kernel source, read from the assembly hipcc emits:
no kernel reads or writes memory through generic (flat) instructions.  A flat
access waits on both the global-memory and the LDS counters; one that slipped
into the multi-species force pass (an LDS read folded with its global-memory
fallback) cost it a fifth of its time.  Also: only the list build spills
registers (it trades a few spills for six waves per SIMD)."""
import os
import re
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2405_07898_amd import build as B

pytestmark = pytest.mark.skipif(shutil.which(B.hipcc()) is None and not os.path.exists(B.hipcc()),
                                reason="hipcc not available")

FLAGS = [f for f in B.HIPCC_FLAGS if f not in ("-fPIC", "-shared")]


def _asm(src: str, out_dir: str) -> str:
    out = os.path.join(out_dir, os.path.basename(src) + ".s")
    cmd = [B.hipcc(), *FLAGS, "--cuda-device-only", "-S", "-I", os.path.join(B.ROOT, "include"),
           "-I", B.CSRC, os.path.join(B.CSRC, src), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    return open(out).read()


@pytest.fixture(scope="module")
def assembly():
    with tempfile.TemporaryDirectory() as d:
        with ThreadPoolExecutor(max_workers=len(B.SOURCES)) as ex:
            texts = list(ex.map(lambda s: _asm(s, d), B.SOURCES))
    return dict(zip(B.SOURCES, texts))


def _functions(text: str):
    """(name, body) of every kernel in an assembly file."""
    out, name, body = [], None, []
    for line in text.splitlines():
        m = re.match(r"(_Z\S+):", line)
        if m:
            name, body = m.group(1), []
        elif line.startswith(".Lfunc_end") and name:
            out.append((name, "\n".join(body)))
            name = None
        elif name:
            body.append(line)
    return out


def test_no_flat_memory_instructions(assembly):
    bad, seen = [], 0
    for src, text in assembly.items():
        funcs = _functions(text)
        seen += len(funcs)
        for name, body in funcs:
            n = len(re.findall(r"^\s*flat_(?:load|store|atomic)", body, re.M))
            if n:
                bad.append((src, name[:80], n))
    assert seen > 40  # every kernel of the library was read
    assert not bad, bad


def test_only_the_list_build_spills(assembly):
    spills = []
    for src, text in assembly.items():
        for m in re.finditer(r"\.name:\s+(\S+)\n(.*?)(?=\n  - \.|\n\.end_amdgpu_metadata)", text,
                             re.S):
            v = re.search(r"\.vgpr_spill_count:\s+(\d+)", m.group(2))
            if v and int(v.group(1)) > 0:
                spills.append(m.group(1))
    assert all("k_build" in n for n in spills), spills

"""Checks on the gfx950 assembly of the integer kernel (CPU only: hipcc -S).

The update blocks of the change-vector kernel are inline assembly that sets
EXEC and uses scalar ops, which write SCC.  A build in which the compiler kept
a comparison in SCC across such a block (SCC was not declared clobbered) chose
the wrong plane segment in a later s_cselect and read before the image.  This
test compiles the kernel and checks that no SCC value produced by compiled code
is consumed after an SCC-writing asm block, and that no 16-bit VOP2 op (which
keeps the upper half of its destination) produces an LDS offset.

Image loads are 8- or 16-bit only.  A build that read each row as a dword of
the values at x-1 and x (2-byte aligned) faulted the GPU with a memory
violation: misaligned vector-memory accesses trap on the parts this runs on.
"""
import pathlib
import re
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_1705_02045_amd" / "csrc"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

SALU_SCC = re.compile(r"\s*s_(cmp|cmpk|bitcmp|and|or|xor|andn2|orn2|nand|nor|xnor|not|add|sub|addk|lshl|lshr|ashr"
                      r"|bfe|min|max|abs|absdiff|addc|subb)\w*\s")
READS_SCC = re.compile(r"\s*s_(cselect|cbranch_scc|addc|subb|cmov|cmovk)\w*")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not pathlib.Path(HIPCC).exists():
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("isa") / "ecc_int.s"
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", str(ROOT / "include"), "-I", str(CSRC), "--offload-device-only",
           "-S", "-o", str(out), str(CSRC / "ecc_int.hip")]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text().splitlines()


def scc_across_asm(lines):
    blk = [None] * len(lines)
    cur = None
    for i, line in enumerate(lines):
        if "ASMSTART" in line:
            cur = {"scc": False}
            continue
        if "ASMEND" in line:
            cur = None
            continue
        if cur is not None:
            blk[i] = cur
            if SALU_SCC.match(line):
                cur["scc"] = True
    bad = []
    for i, line in enumerate(lines):
        if blk[i] is not None or not READS_SCC.match(line):
            continue
        j, clobbered = i - 1, False
        while j >= 0:
            t = lines[j].strip()
            if t.startswith(".LBB") or t.startswith("; %bb"):
                break
            if blk[j] is not None:
                clobbered |= blk[j]["scc"]
            elif SALU_SCC.match(lines[j]):
                break
            j -= 1
        if clobbered and j >= 0 and blk[j] is None and SALU_SCC.match(lines[j]):
            bad.append((i, line.strip()))
    return bad


def test_no_scc_live_across_update_blocks(asm):
    assert any("s_xor_b64 exec" in line for line in asm), "update blocks not found"
    assert scc_across_asm(asm) == []


def test_no_partial_register_16bit_ops(asm):
    bad = [l for l in asm if re.match(r"\s*v_(lshlrev_b16|min_u16)(_e32|_e64)?\s", l)]
    assert bad == []


def test_image_loads_are_element_sized(asm):
    """No multi-byte buffer load in the integer kernels: their image offsets are
    only element-aligned (see the module docstring)."""
    loads = [l.strip().split()[0] for l in asm if re.match(r"\s*buffer_load_", l)]
    assert loads, "no buffer loads found"
    assert set(loads) <= {"buffer_load_ushort", "buffer_load_ubyte"}, sorted(set(loads))

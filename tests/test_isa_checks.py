"""Checks on the gfx950 assembly of the integer kernel (CPU only: hipcc -S).

The update blocks of the change-vector kernel are inline assembly that sets
EXEC and uses scalar ops, which write SCC.  A build in which the compiler kept
a comparison in SCC across such a block (SCC was not declared clobbered) chose
the wrong plane segment in a later s_cselect and read before the image.  This
test compiles the kernel and checks that no SCC value produced by compiled code
is consumed after an SCC-writing asm block, and that no 16-bit VOP2 op (which
keeps the upper half of its destination) produces an LDS offset.

Two builds of the row-pair path (16-bit values at x-1 and x packed in one
register) faulted the GPU with a memory violation.  Their packed shift by an
inline constant, `v_pk_lshlrev_b16 d, 2, s`, kept the default op_sel_hi, so
the high lane read bits 31:16 of the constant (0) and was not shifted: the
LDS byte offsets of the high values were not multiples of 4, and the
histogram adds trapped on them.  The compiler's own splat shift carries
op_sel_hi:[0,1].  Checked here: every packed op with an inline constant
reads that constant's low half in both lanes.  Dword image loads exist only
in the row-pair path, whose offsets are 4-byte aligned by construction
(test_row_pair_map.py); it is recognisable by its wave shift and bit-field
extract.
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



def functions(asm):
    """(name, lines) of each function of the assembly."""
    out, name, body = [], None, []
    for line in asm:
        m = re.match(r"^(_Z\w+):", line)
        if m:
            if name:
                out.append((name, body))
            name, body = m.group(1), []
        elif name:
            body.append(line)
    if name:
        out.append((name, body))
    return out


def test_dword_image_loads_only_in_row_pair_path(asm):
    """Image loads are 8- or 16-bit, except in functions that carry the
    row-pair form (a wave shift by one lane and a bit-field extract)."""
    seen = 0
    for name, body in functions(asm):
        loads = {l.strip().split()[0] for l in body if re.match(r"\s*buffer_load_", l)}
        wide = loads - {"buffer_load_ushort", "buffer_load_ubyte"}
        if not wide:
            continue
        assert wide == {"buffer_load_dword"}, (name, sorted(wide))
        text = "\n".join(body)
        assert "wave_shr:1" in text and "v_bfe_u32" in text, name
        assert "int_vcec" in name, name
        seen += 1
    assert seen > 0, "row-pair path not found"


PK_OP = re.compile(r"\s*(v_pk_\w+)\s+([^;]*)")


def test_packed_inline_constants_reach_both_lanes(asm):
    """A packed op whose source k is an inline integer constant has bit k of
    op_sel_hi clear (the high lane reads the constant's low half)."""
    bad, seen = [], 0
    for line in asm:
        m = PK_OP.match(line)
        if not m:
            continue
        text = m.group(2)
        mods = dict(re.findall(r"(\w+):\[([\d,]+)\]", text))
        ops = [o.strip() for o in re.sub(r"\s\w+:\[[\d,]+\]", "", text).split(",")][1:]
        hi = [int(b) for b in mods.get("op_sel_hi", "1,1,1").split(",")]
        for k, o in enumerate(ops):
            if re.fullmatch(r"-?\d+", o):
                seen += 1
                if k < len(hi) and hi[k] != 0:
                    bad.append(line.strip())
    assert seen > 0, "no packed op with an inline constant found"
    assert bad == [], bad[:5]

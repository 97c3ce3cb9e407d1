"""Static checks on the gfx950 assembly of the float32 pair-sum kernel.

The kernel's weight FMA is inline assembly (a v_fmac_f32 with a DPP
row_newbcast source), which the compiler's hazard recognizer does not
inspect.  Two hardware hazards apply to it and are covered by wait states
inside the asm block:
  * a VALU reading the result of a transcendental (v_exp_f32) needs one wait
    state;
  * a DPP source VGPR needs two wait states after a VALU writes it.
This test compiles the kernel and checks every such instruction against the
instructions the compiler placed before it."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1305_5179_amd", "csrc", "pairsum.hip")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def f32_asm(tmp_path_factory):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    from paper_1305_5179_amd.build import HIPFLAGS
    out = tmp_path_factory.mktemp("isa") / "pairsum.s"
    flags = [f for f in HIPFLAGS if f not in ("-fPIC",)]
    subprocess.run([hipcc, *flags, "--cuda-device-only", "-S", SRC, "-o", str(out)], check=True,
                   capture_output=True)
    text = out.read_text()
    start = text.index("k_pairsum_f32ENS0_8PairArgsE:")
    end = text.index("s_endpgm", start)
    lines = [l.split(";")[0].strip() for l in text[start:end].splitlines()]
    return [l for l in lines if l and not l.startswith(".") and not l.endswith(":")]


def _wait_states(instr):
    m = re.match(r"s_nop\s+(\d+)", instr)
    return int(m.group(1)) + 1 if m else 0


def _dst(instr):
    m = re.match(r"(v_\w+)\s+(v\[?\d+)", instr)
    if not m or m.group(1).startswith(("v_cmp", "v_readlane", "v_readfirstlane")):
        return None
    return m.group(2).lstrip("v[")


def test_asm_fmac_is_preceded_by_enough_wait_states(f32_asm):
    n = 0
    for i, ins in enumerate(f32_asm):
        m = re.match(r"v_fmac_f32_dpp\s+v(\d+),\s*v(\d+),\s*v(\d+)", ins)
        if not m:
            continue
        n += 1
        src0, src1 = m.group(2), m.group(3)
        # walk back over the wait states inside the asm block
        j, waits = i - 1, 0
        while j >= 0 and f32_asm[j].startswith("s_nop"):
            waits += _wait_states(f32_asm[j])
            j -= 1
        assert waits >= 1, f"no wait state before {ins}"
        # instructions the compiler placed before the block
        prev = [f32_asm[k] for k in range(max(0, j - 2), j + 1)]
        for dist, p in enumerate(reversed(prev)):
            d = _dst(p)
            if d is None:
                continue
            if d == src1 and p.startswith("v_exp_f32"):
                assert waits + dist >= 1, (p, ins)
            if d == src0:
                assert waits + dist >= 2, f"DPP source v{src0} written by '{p}' right before '{ins}'"
    assert n >= 32   # inner and outer bodies, 16 each

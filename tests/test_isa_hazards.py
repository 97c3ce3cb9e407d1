"""Static checks on the gfx950 assembly of the float32 pair-sum kernel and
of the issue-rate probes that reuse its steps.

Parts of the kernel's pair loop are inline assembly (DPP row_newbcast FMAs,
and whole pipelined chunks), which the compiler's hazard recognizer does not
look into.  Two hardware hazards apply to that code and must be covered by
the instruction order or by s_nop wait states:
  * a DPP instruction whose permuted source (src0) was written by a VALU
    needs two wait states after that write;
  * a (non-transcendental) VALU reading the result of a transcendental
    (v_exp_f32 and the like) needs one wait state on gfx950.
This test compiles the kernels and checks every instruction of them against
the instructions that can precede it, following branches into labels."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1305_5179_amd", "csrc", "pairsum.hip")
# every instantiation of the kernel
KERNEL = "_ZN3rbf12_GLOBAL__N_113k_pairsum_f32"
TRANS = ("v_exp_f32", "v_log_f32", "v_rcp_f32", "v_rsq_f32", "v_sqrt_f32", "v_sin_f32", "v_cos_f32",
         "v_rcp_f64", "v_rsq_f64", "v_sqrt_f64", "v_rcp_iflag_f32")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return None


def _kernel_bodies(tmp_path_factory, src, prefix):
    """Instructions (labels kept) of every kernel of `src` whose symbol
    starts with `prefix`, from the device assembly of this build's flags."""
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    from paper_1305_5179_amd.build import HIPFLAGS
    out = tmp_path_factory.mktemp("isa") / (os.path.basename(src) + ".s")
    flags = [f for f in HIPFLAGS if f not in ("-fPIC",)]
    subprocess.run([hipcc, *flags, "--cuda-device-only", "-S", src, "-o", str(out)], check=True,
                   capture_output=True)
    text = out.read_text()
    bodies = []
    for m in re.finditer(r"^(" + prefix + r"\w*):", text, re.M):
        end = text.index(".Lfunc_end", m.end())
        lines = []
        for raw in text[m.end():end].splitlines()[1:]:
            l = raw.split(";")[0].strip()
            if not l or (l.startswith(".") and not l.endswith(":")):
                continue
            lines.append(l)
        bodies.append((m.group(1), lines))
    return bodies


@pytest.fixture(scope="module")
def f32_asm(tmp_path_factory):
    bodies = _kernel_bodies(tmp_path_factory, SRC, KERNEL)
    # float32 or float64 weights, buffer or flat loads
    assert len(bodies) == 4, [b[0] for b in bodies]
    return bodies


def _regs(operand):
    """VGPR numbers named by one operand (v7, -v7, |v7|, v[4:5])."""
    m = re.search(r"v\[(\d+):(\d+)\]", operand)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.search(r"(?<![\w])v(\d+)\b", operand)
    return {int(m.group(1))} if m else set()


def _parse(instr):
    parts = instr.split(None, 1)
    op = parts[0]
    args = [a.strip() for a in parts[1].split(",")] if len(parts) > 1 else []
    # drop DPP/modifier words glued to the last operand
    if args:
        args[-1] = args[-1].split()[0]
    return op, args


def _is_valu(op):
    return op.startswith("v_")


def _writes(instr):
    """VGPRs written by a VALU instruction (both operands of a lane swap)."""
    op, args = _parse(instr)
    if not _is_valu(op) or not args or op.startswith(("v_cmp", "v_readlane", "v_readfirstlane")):
        return set()
    if op.startswith(("v_permlane16_swap", "v_permlane32_swap")) and len(args) > 1:
        return _regs(args[0]) | _regs(args[1])
    return _regs(args[0])


def _reads(instr):
    op, args = _parse(instr)
    if not args:
        return set()
    srcs = args[1:]
    r = set().union(*[_regs(a) for a in srcs]) if srcs else set()
    if op.startswith(("v_fmac", "v_mac")):
        r |= _regs(args[0])     # tied accumulator
    return r


def _wait_states(instr):
    m = re.match(r"s_nop\s+(\d+)", instr)
    return int(m.group(1)) + 1 if m else 1


def _predecessors(lines):
    """index of the line -> list of indices that may execute right before it."""
    labels = {l[:-1]: i for i, l in enumerate(lines) if l.endswith(":")}
    preds = {i: [] for i in range(len(lines))}
    for i, l in enumerate(lines):
        if i + 1 < len(lines) and not l.startswith(("s_branch", "s_endpgm", "s_setpc")):
            preds[i + 1].append(i)
        m = re.match(r"s_(?:cbranch_\w+|branch)\s+(\S+)", l)
        if m and m.group(1) in labels:
            preds[labels[m.group(1)]].append(i)
    return preds


def _violations(lines, i, regs, need, producer_ok):
    """Producers of `regs` among the instructions within `need` wait states
    before line i, on every path."""
    preds = _predecessors.cache
    found = []
    stack = [(p, 0) for p in preds[i]]
    seen = set()
    while stack:
        j, waited = stack.pop()
        if (j, waited) in seen or waited >= need:
            continue
        seen.add((j, waited))
        l = lines[j]
        if l.endswith(":"):
            stack.extend((p, waited) for p in preds[j])
            continue
        if producer_ok(l) and _writes(l) & regs:
            found.append((l, waited))
        # regs written here are the newest value on this path: stop for them
        rest = regs - _writes(l)
        if rest:
            stack.extend((p, waited + _wait_states(l)) for p in preds[j])
    return found


def test_no_dpp_or_transcendental_forwarding_hazard(f32_asm):
    for name, lines in f32_asm:
        _check_kernel(name, lines)


def test_rate_probes_have_no_hazard(tmp_path_factory):
    """The register-resident rate kernels of rbf_measure_rates: the pair
    kernel's own chunk bodies (pairsum.hip) and the DPP FMA and
    exponential-mix loops (profile.hip)."""
    steps = _kernel_bodies(tmp_path_factory, SRC, "_ZN3rbf12_GLOBAL__N_111k_step_rate")
    assert len(steps) == 2, [b[0] for b in steps]
    for name, lines in steps:
        _check_kernel(name, lines, min_fmac_dpp=48, min_dpp=64)
    rates = _kernel_bodies(tmp_path_factory, os.path.join(os.path.dirname(SRC), "profile.hip"),
                           "_ZN3rbf12_GLOBAL__N_17k_rates")
    assert len(rates) == 5, [b[0] for b in rates]
    for name, lines in rates:
        _check_kernel(name, lines, min_fmac_dpp=0, min_dpp=0)
    assert any(l.startswith("v_fmac_f32_dpp") for _, lines in rates for l in lines)


def _check_kernel(name, lines, min_fmac_dpp=64, min_dpp=128):
    _predecessors.cache = _predecessors(lines)
    n_dpp = n_fmac_dpp = 0
    problems = []
    for i, l in enumerate(lines):
        if l.endswith(":") or l.startswith("s_"):
            continue
        op, args = _parse(l)
        if not _is_valu(op):
            continue
        if "_dpp" in op:
            n_dpp += 1
            n_fmac_dpp += op.startswith("v_fmac_f32_dpp")
            src0 = _regs(args[1]) if len(args) > 1 else set()
            for p, w in _violations(lines, i, src0, 2, lambda x: _is_valu(_parse(x)[0])):
                problems.append(f"DPP source written {w} wait states before: '{p}' -> '{l}'")
        if not op.startswith(TRANS):
            for p, w in _violations(lines, i, _reads(l), 1, lambda x: _parse(x)[0].startswith(TRANS)):
                problems.append(f"transcendental result read after {w} wait states: '{p}' -> '{l}'")
    assert not problems, name + "\n" + "\n".join(problems[:20])
    # the pair loops (of both forms, in the pair kernel) are present
    assert n_fmac_dpp >= min_fmac_dpp, (name, n_fmac_dpp)
    assert n_dpp >= min_dpp, (name, n_dpp)


def test_checker_sees_planted_hazards():
    """The checker itself: two planted sequences must be reported."""
    lines = [
        "v_cvt_f32_f64_e32 v3, v[4:5]",
        "v_mul_f32_dpp v1, v3, v2 row_newbcast:0 row_mask:0xf bank_mask:0xf bound_ctrl:1",
        "v_exp_f32_e32 v6, v1",
        "v_fmac_f32_e32 v7, v6, v8",
        "s_endpgm",
    ]
    _predecessors.cache = _predecessors(lines)
    dpp = _violations(lines, 1, {3}, 2, lambda x: _is_valu(_parse(x)[0]))
    trans = _violations(lines, 3, _reads(lines[3]), 1, lambda x: _parse(x)[0].startswith(TRANS))
    assert dpp and trans
    # and with the waits in place, nothing
    ok = ["v_cvt_f32_f64_e32 v3, v[4:5]", "s_nop 1",
          "v_mul_f32_dpp v1, v3, v2 row_newbcast:0 row_mask:0xf bank_mask:0xf bound_ctrl:1",
          "v_exp_f32_e32 v6, v1", "s_nop 0", "v_fmac_f32_e32 v7, v6, v8"]
    _predecessors.cache = _predecessors(ok)
    assert not _violations(ok, 2, {3}, 2, lambda x: _is_valu(_parse(x)[0]))
    assert not _violations(ok, 5, _reads(ok[5]), 1, lambda x: _parse(x)[0].startswith(TRANS))


def test_checker_follows_branches():
    lines = [
        "s_cbranch_vccnz .LBB0_9",
        "v_mov_b32_e32 v3, 0",
        "s_branch .LBB0_10",
        ".LBB0_9:",
        "v_exp_f32_e32 v3, v1",
        ".LBB0_10:",
        "v_mul_f32_dpp v1, v3, v2 row_newbcast:0 row_mask:0xf bank_mask:0xf bound_ctrl:1",
    ]
    _predecessors.cache = _predecessors(lines)
    found = _violations(lines, 6, {3}, 2, lambda x: _is_valu(_parse(x)[0]))
    assert len(found) == 2   # both paths write v3 right before the DPP read

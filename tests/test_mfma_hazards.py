"""Wait states between the matrix instructions of the guess network and the
first instruction that reads their results, in the gfx950 assembly of the
kernels as the library build compiles them.

The ReLU packing of the guess network (mhd_device.h, pack2_relu) uses an
empty inline-asm statement to keep a converted BF16 pair whole.  An asm
statement emits no instruction, so it must not stand for a wait state
between an MFMA and a reader of its destination registers.  This test
compiles mhd_kernels.hip to assembly with the build's flags and checks
every MFMA -> first-reader window that contains asm statements: its real
wait states (s_nop N counts N + 1, any other instruction 1, asm 0) are at
least the fewest the same compile leaves in windows of the same kind
without asm, plus one for each asm statement in the window -- enough even
if every asm statement had been counted as an instruction.  CPU only
(cross-compiles; needs hipcc)."""
import collections
import re


def _vregs(tok):
    m = re.match(r"v\[(\d+):(\d+)\]$", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def _split(line):
    body = line.split(";")[0].strip()
    parts = body.split(None, 1)
    if len(parts) < 2:
        return (parts[0] if parts else ""), []
    return parts[0], [t.strip() for t in parts[1].split(",")]


def mfma_windows(lines):
    """(mfma opcode, reader kind, wait states, asm statements) per MFMA whose
    destination is read later in the same basic block."""
    out = []
    for i, line in enumerate(lines):
        if not re.match(r"^\s+v_mfma", line):
            continue
        op, ops = _split(line)
        dst = _vregs(ops[0])
        ws = nasm = 0
        for x in lines[i + 1:]:
            if ";;#ASMSTART" in x:
                nasm += 1
                continue
            if re.match(r"^\.LBB|^\s+s_(cbranch|branch|setpc|endpgm)", x):
                break
            if not re.match(r"^\s+[vsgdb]\w+", x):
                continue
            op2, ops2 = _split(x)
            srcs = set().union(*[_vregs(t) for t in ops2]) if ops2 else set()
            if srcs & dst:
                out.append((op, "mfma" if op2.startswith("v_mfma") else "valu", ws, nasm))
                break
            m = re.match(r"s_nop (\d+)", x.strip())
            ws += int(m.group(1)) + 1 if m else 1
    return out


def test_asm_statements_never_stand_for_mfma_wait_states(kernels_asm):
    wins = mfma_windows(kernels_asm)
    assert len(wins) >= 20, "the guess network's MFMAs were not found"
    need = collections.defaultdict(lambda: None)
    for op, kind, ws, nasm in wins:
        if nasm == 0:
            k = (op, kind)
            need[k] = ws if need[k] is None else min(need[k], ws)
    checked = 0
    for op, kind, ws, nasm in wins:
        if nasm == 0:
            continue
        base = need[(op, kind)]
        assert base is not None, f"no window without asm to compare with for {op} -> {kind}"
        assert ws >= base + nasm, (op, kind, ws, nasm, base)
        checked += 1
    print(f"{len(wins)} MFMA windows, {checked} with asm statements, fewest wait states "
          f"without asm: {dict(need)}")


def test_checker_sees_asm_and_counts_wait_states():
    """The window scan on a hand-written listing: a reader 12 states after
    its MFMA, and one whose window holds an asm statement and only 11."""
    text = """
\tv_mfma_f32_32x32x8_bf16 v[2:17], v[40:41], v[42:43], 0
\ts_nop 11
\tv_mul_f32_e32 v1, v2, v3
\tv_mfma_f32_32x32x8_bf16 v[18:33], v[40:41], v[42:43], 0
\t;;#ASMSTART
\t;;#ASMEND
\ts_nop 9
\tv_add_f32_e32 v50, v51, v52
\tv_cvt_pk_bf16_f32 v4, v18, v19
"""
    wins = mfma_windows(text.split("\n"))
    assert wins == [("v_mfma_f32_32x32x8_bf16", "valu", 12, 0),
                    ("v_mfma_f32_32x32x8_bf16", "valu", 11, 1)]
    base = wins[0][2]
    assert not wins[1][2] >= base + wins[1][3]

"""The stage kernel's argument layout and addressing, in the gfx950 assembly
of the library build (CPU only: cross-compiles, needs hipcc).

The stage kernel takes its arguments as one struct and, inside the plane
loop of its FP32 variants, reads them again from the kernel-argument
segment through the segment pointer (mhd_kernels.hip, stage_args_view).  That is only the same
data if the struct is the kernel's only explicit argument and sits at
offset 0 of the segment.  The code-object metadata states both; each
scalar load the kernel makes through the segment pointer (or a copy of it)
must lie inside the struct or inside one of the hidden arguments after
it.  Two properties of the compiled plane loop are pinned as well: every
global load and store takes the scalar-base form (uniform plane address,
32-bit column offset), and the FP32 variants reload no more than a few
scalar values from vector lanes."""
import re

LOAD_WIDTH = {"": 4, "x2": 8, "x4": 16, "x8": 32, "x16": 64}


def kernel_args(lines, name_re):
    """{kernel name: [(offset, size, value_kind), ...]} from the metadata."""
    out = {}
    for i, line in enumerate(lines):
        m = re.match(r"\s+\.name:\s+(\S+)$", line)
        if not m or not re.search(name_re, m.group(1)):
            continue
        # the .args list precedes .name in the kernel's metadata map
        j = i - 1
        while j > 0 and not re.match(r"\s+\.args:", lines[j]) and not re.match(r"\s+- \.agpr_count", lines[j]):
            j -= 1
        args, cur = [], {}
        for x in lines[j + 1:i]:
            mo = re.match(r"\s+(?:- )?\.(offset|size|value_kind):\s+(\S+)", x)
            if mo:
                if mo.group(1) == "offset" and cur:
                    args.append(cur)
                    cur = {}
                cur[mo.group(1)] = mo.group(2)
        if cur:
            args.append(cur)
        out[m.group(1)] = [(int(a["offset"]), int(a["size"]), a["value_kind"]) for a in args]
    return out


def segment_loads(lines, sym):
    """(offset, bytes) of every scalar load of the kernel `sym` whose base is
    the kernel-argument segment pointer s[0:1] or a copy of it."""
    s = next(i for i, x in enumerate(lines) if x.startswith(sym + ":"))
    e = next(i for i in range(s + 1, len(lines)) if lines[i].startswith(".Lfunc_end"))
    bases = {"s[0:1]"}
    out = []
    for x in lines[s:e]:
        m = re.match(r"\s+s_mov_b64 (s\[\d+:\d+\]), (s\[\d+:\d+\])", x)
        if m:
            (bases.add if m.group(2) in bases else bases.discard)(m.group(1))
            continue
        m = re.match(r"\s+s_load_dword(x\d+)? \S+, (s\[\d+:\d+\]), (0x[0-9a-f]+|\d+)", x)
        if m and m.group(2) in bases:
            out.append((int(m.group(3), 0), LOAD_WIDTH[m.group(1) or ""]))
    return out


def test_stage_kernel_takes_one_struct_at_offset_zero(kernels_asm):
    kern = kernel_args(kernels_asm, r"^_ZN3mhd12stage_kernelI")
    assert len(kern) == 8, sorted(kern)
    for name, args in kern.items():
        explicit = [a for a in args if not a[2].startswith("hidden_")]
        assert len(explicit) == 1, (name, args)
        off, size, kind = explicit[0]
        assert (off, kind) == (0, "by_value"), (name, explicit)
        loads = segment_loads(kernels_asm, name)
        # the FP32 variants' plane loop reads pointers and constants of the
        # struct again
        if name.startswith("_ZN3mhd12stage_kernelIf"):
            assert len(loads) >= 20, (name, len(loads))
        # each load lies inside the struct or inside one hidden argument
        # (grid size and the like, read by the kernel's set-up)
        for o, w in loads:
            assert any(a <= o and o + w <= a + n for a, n, _ in args), (name, o, w, args)
        assert any(o + w <= size for o, w in loads)


def plane_loop(lines, sym):
    """Lines of the largest loop of the kernel `sym` (the plane loop)."""
    s = next(i for i, x in enumerate(lines) if x.startswith(sym + ":"))
    e = next(i for i in range(s + 1, len(lines)) if lines[i].startswith(".Lfunc_end"))
    f = lines[s:e]
    labels = {m.group(1): i for i, x in enumerate(f) for m in [re.match(r"^(\.LBB\w+):", x)] if m}
    best = (0, 0, 0)
    for i, x in enumerate(f):
        m = re.search(r"s_(?:cbranch_\w+|branch)\s+(\.LBB\w+)", x)
        if m and m.group(1) in labels and labels[m.group(1)] < i:
            best = max(best, (i - labels[m.group(1)], labels[m.group(1)], i))
    return f[best[1]:best[2] + 1]


def test_plane_loop_addressing_and_scalar_reloads(kernels_asm):
    kern = kernel_args(kernels_asm, r"^_ZN3mhd12stage_kernelI")
    for name in kern:
        loop = plane_loop(kernels_asm, name)
        mem = [x.split(None, 1) for x in loop if re.match(r"\s+global_(load|store)", x)]
        assert len(mem) >= 40, (name, len(mem))
        # the scalar-base form names a scalar register pair last; the
        # vector-address form names "off"
        vec = [m for m in mem if m[1].split(",")[-1].strip().startswith("off")]
        assert not vec, (name, vec[:3])
        if name.startswith("_ZN3mhd12stage_kernelIf"):
            reloads = sum(1 for x in loop if "v_readlane_b32" in x)
            assert reloads <= 4, (name, reloads)


def test_metadata_and_load_scan_on_a_listing():
    text = """
_ZN3mhd12stage_kernelIdLb0ELb0EEEv6StageArgs:
\ts_load_dwordx16 s[4:19], s[0:1], 0x0
\ts_mov_b64 s[52:53], s[0:1]
\ts_load_dwordx2 s[20:21], s[52:53], 0x1b8
\ts_mov_b64 s[60:61], s[2:3]
\ts_load_dword s22, s[60:61], 0x0
.Lfunc_end0:
amdhsa.kernels:
  - .agpr_count:     0
    .args:
      - .offset:         0
        .size:           480
        .value_kind:     by_value
      - .offset:         480
        .size:           4
        .value_kind:     hidden_block_count_x
    .name:           _ZN3mhd12stage_kernelIdLb0ELb0EEEv6StageArgs
"""
    lines = text.split("\n")
    args = kernel_args(lines, r"^_ZN3mhd12stage_kernelI")
    assert args == {"_ZN3mhd12stage_kernelIdLb0ELb0EEEv6StageArgs":
                    [(0, 480, "by_value"), (480, 4, "hidden_block_count_x")]}
    assert segment_loads(lines, "_ZN3mhd12stage_kernelIdLb0ELb0EEEv6StageArgs") == [(0, 64), (0x1b8, 8)]

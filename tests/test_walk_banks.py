"""The fast walk's register banks, read from the built library's gfx950 code (nothing runs on a GPU:
the code objects in libperm3.so are unbundled and disassembled with ROCm's LLVM tools).

A 3-input VALU op whose three VGPR sources share one register bank (register number mod 4) issues
at about half rate on gfx950.  The walk holds its block's high-row sum H and each low-row sum L_k as
64-bit values pinned to register pairs so that no op of a block can read three sources from one
bank; left to the allocator, 6 of a block's 44 ops did and the 36x36 walk ran 11-13% slower.  This
test finds every fast-walk block in every walk kernel and in the census lanes (a run of code
between branches with the block's two bitop3 per state and its tree of v_max3) and checks each
3-source op."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2407_20205_amd import perm3 as P

LLVM = "/opt/rocm/llvm/bin"
BUNDLER = os.path.join(LLVM, "clang-offload-bundler")
OBJDUMP = os.path.join(LLVM, "llvm-objdump")
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"
# the kernels that run the fast walk, by a fragment of their mangled names
KERNELS = {"k_walk<1, false>": "k_walkILi1ELb0E", "k_walk<2, true>": "k_walkILi2ELb1E",
           "k_tick": "k_tickENS_8TickArgsE", "k_small": "k_smallENS_8PlanArgs", "k_walk_wide": "k_walk_wideENS",
           "k_census_filtered": "k_census_filteredENS"}
# block loops each kernel holds at least: one per half of a chunk in the chunk walks, one in the
# census lanes (a lane's whole matrix is one run of blocks)
MIN_LOOPS = {k: (1 if k == "k_census_filtered" else 2) for k in KERNELS}


def code_objects(tmp_path):
    if not (shutil.which("objcopy") and os.path.exists(BUNDLER) and os.path.exists(OBJDUMP)):
        pytest.skip("objcopy or ROCm's LLVM tools unavailable")
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libperm3.so is not built")
    fat = tmp_path / "fatbin.bin"
    subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", P.LIB_PATH, str(fat)], check=True)
    data = fat.read_bytes()
    # one offload bundle per translation unit, each opening with the bundler's magic string
    starts = [m.start() for m in re.finditer(re.escape(b"__CLANG_OFFLOAD_BUNDLE__"), data)]
    texts = []
    for k, st in enumerate(starts):
        part = tmp_path / f"bundle{k}.bin"
        part.write_bytes(data[st:starts[k + 1] if k + 1 < len(starts) else len(data)])
        co = tmp_path / f"bundle{k}.co"
        subprocess.run([BUNDLER, "--unbundle", "--type=o", f"--targets={TARGET}", f"--input={part}",
                        f"--output={co}"], check=True)
        out = subprocess.run([OBJDUMP, "-d", "--mcpu=gfx950", "--no-show-raw-insn", str(co)],
                             capture_output=True, text=True, check=True).stdout
        texts.append(out + "\n\n")
    return texts


def functions(text):
    for name, body in re.findall(r"\n[0-9a-f]+ <([^>]*)>:\n(.*?)(?=\n\n)", text, re.S):
        lines = [l.split("//")[0].strip() for l in body.split("\n")]
        yield name, [l for l in lines if l]


def straight_runs(ins):
    """The function cut after every branch."""
    run = []
    for i in ins:
        run.append(i)
        if i.startswith("s_cbranch") or i.startswith("s_branch"):
            yield run
            run = []
    if run:
        yield run


def is_fast_block(run):
    """15 states at two bitop3 each plus H's step, and the tree of 3-input maxima."""
    bitop3 = sum(1 for i in run if i.startswith("v_bitop3_b32"))
    max3 = sum(1 for i in run if i.startswith("v_max3_u32"))
    return bitop3 >= 30 and max3 >= 5


def one_bank_ops(run):
    bad = []
    for i in run:
        if not (i.startswith("v_bitop3_b32") or i.startswith("v_max3_u32")):
            continue
        ops = re.sub(r"bitop3:\S+", "", i.split(None, 1)[1])
        srcs = [p.strip() for p in ops.split(",")[1:4]]
        regs = [int(x[1:]) for x in srcs if re.fullmatch(r"v\d+", x)]
        if len(regs) == 3 and len({r % 4 for r in regs}) == 1:
            bad.append(i)
    return bad


def test_fast_walk_blocks_spread_register_banks(tmp_path):
    found = {k: 0 for k in KERNELS}
    for text in code_objects(tmp_path):
        for name, ins in functions(text):
            kind = next((k for k, frag in KERNELS.items() if frag in name), None)
            if kind is None:
                continue
            for run in straight_runs(ins):
                if is_fast_block(run):
                    found[kind] += 1
                    assert not one_bank_ops(run), (kind, one_bank_ops(run))
    # every walk kernel was looked at
    assert all(found[k] >= MIN_LOOPS[k] for k in KERNELS), found

"""Resource use of the built stage kernels (CPU: reads the code objects in
libbssn_hip.so, nothing runs on a GPU).

The LDS-pipelined stage kernels are designed around their register and LDS
budgets: no private (scratch) memory in any of them, two workgroups per CU
for the order-4 FP32 launch of mixed precision (at most 256 registers per
lane and 80 KB of LDS), and the order-8 ring within one CU's 160 KB.  A
change that breaks one of these still passes the parity tests, so it is
checked here against the compiler's own kernel descriptors.
"""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1111_3344_amd", "libbssn_hip.so")
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


def _tool(name):
    p = os.path.join(LLVM, name)
    return p if os.path.exists(p) else shutil.which(name)


def _kernels():
    """{mangled name: {field: int}} over every gfx950 code object."""
    objcopy, bundler, readelf = (_tool("llvm-objcopy"),
                                 _tool("clang-offload-bundler"),
                                 _tool("llvm-readelf"))
    if not (os.path.exists(LIB) and objcopy and bundler and readelf):
        pytest.skip("library or LLVM tools not available")
    out = {}
    with tempfile.TemporaryDirectory() as d:
        fat = os.path.join(d, "fat.bin")
        subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fat}", LIB,
                        os.path.join(d, "x.so")], check=True,
                       capture_output=True)
        blob = open(fat, "rb").read()
        starts = [m.start() for m in re.finditer(re.escape(MAGIC), blob)]
        for i, s in enumerate(starts):
            e = starts[i + 1] if i + 1 < len(starts) else len(blob)
            part = os.path.join(d, f"b{i}.bin")
            open(part, "wb").write(blob[s:e])
            elf = os.path.join(d, f"b{i}.elf")
            r = subprocess.run([bundler, "--unbundle", "--type=o",
                                f"--input={part}", f"--targets={TARGET}",
                                f"--output={elf}"], capture_output=True)
            if r.returncode != 0 or not os.path.exists(elf) or \
                    os.path.getsize(elf) == 0:
                continue
            notes = subprocess.run([readelf, "--notes", elf],
                                   capture_output=True, text=True).stdout
            # one kernel per item of amdhsa.kernels ("  - .field: value"),
            # its scalar fields at the item's own indentation
            item = None
            for line in notes.splitlines():
                m = re.match(r"^  - \.(\w+):\s*(.*)$", line)
                if m:
                    item = {}
                    key, val = m.group(1), m.group(2)
                else:
                    m = re.match(r"^    \.(\w+):\s*(.*)$", line)
                    if not (m and item is not None):
                        continue
                    key, val = m.group(1), m.group(2)
                if key == "name":
                    out[val.strip()] = item
                elif re.fullmatch(r"\d+", val.strip()):
                    item[key] = int(val)
    if not out:
        pytest.skip("no gfx950 code object found")
    return out


@pytest.fixture(scope="module")
def kernels():
    return _kernels()


def _select(kernels, pattern):
    sel = {k: v for k, v in kernels.items() if re.search(pattern, k)}
    assert sel, f"no kernel matches {pattern}"
    return sel


def test_lds_stage_kernels_use_no_scratch(kernels):
    # every LDS-pipelined stage kernel, single and batched, both orders
    sel = _select(kernels, r"k_stage_lds")
    bad = {k: v.get("private_segment_fixed_size")
           for k, v in sel.items() if v.get("private_segment_fixed_size")}
    assert not bad, f"scratch in {bad}"


def test_order4_fp32_launch_fits_two_workgroups_per_cu(kernels):
    sel = _select(kernels, r"k_stage_lds(_batch)?_f32ILi4E")
    for k, v in sel.items():
        # vgpr_count counts the accumulation registers too
        assert v["vgpr_count"] <= 256, k
        assert v["group_segment_fixed_size"] <= 80 * 1024, k


def test_order8_ring_fits_one_cu(kernels):
    sel = _select(kernels, r"k_stage_lds\w*ILi8E")
    for k, v in sel.items():
        assert v["group_segment_fixed_size"] <= 160 * 1024, k

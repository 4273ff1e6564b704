"""The complex64 subdomain-solve kernel (the chosen form) keeps its whole state in registers
and LDS: compiled for gfx950 with the library's own flags, neither of its instantiations (256 and
512 threads) uses scratch memory.

Why this is a test: a spill inside the coarse solve's step loop is reloaded through a wait on
every factor load in flight, which made the complex64 kernel 7% slower on the large workload,
and the kernel sits at the 256-register limit, so an edit anywhere in it can push the register
allocator over that edge.  The check reads the code-object metadata of the assembly that
hipcc produces here (private segment size and VGPR spill count per kernel).  The complex128 kernels are
not held to it: at 512 threads they spill two registers, and a shorter factor ring that removes
the spills measured no faster over whole solves.
"""

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2103_17081_amd", "csrc", "inner_kernels.hip")


def _field(block: str, name: str) -> int:
    m = re.search(r"^\s+\." + name + r":\s+(\d+)", block, re.M)
    assert m, name
    return int(m.group(1))


def test_inner_kernel_uses_no_scratch(tmp_path):
    from paper_2103_17081_amd import build
    try:
        hipcc = build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    out = tmp_path / "inner.s"
    cmd = [hipcc, "-x", "hip", *build.COMMON, "--cuda-device-only", "-S", SRC, "-o", str(out), *build.DEVICE_FLAGS]
    subprocess.run(cmd, check=True, capture_output=True, timeout=900)
    text = out.read_text()
    meta = text[text.index("amdhsa.kernels:"):]
    for t, nt in (("f", 512), ("f", 256)):
        sym = f"_ZN3ddh18inner_solve_kernelI{t}Li{nt}EEEvNS_9InnerArgsIT_EE"
        start = meta.index(".name:           " + sym)
        nxt = meta.find(".name:", start + 10)
        # the entry's fields are listed alphabetically around .name; take the entry's span
        lo = meta.rfind("\n  - ", 0, start)
        hi = meta.find("\n  - ", start)
        block = meta[lo:hi if hi > 0 else (nxt if nxt > 0 else len(meta))]
        assert _field(block, "private_segment_fixed_size") == 0, (t, nt)
        assert _field(block, "vgpr_spill_count") == 0, (t, nt)

"""Code-generation checks of the gfx950 matrix-core kernels (CPU only: hipcc
cross-compiles the sources to assembly).

A buffer load takes its 128-bit resource in scalar registers.  When the
compiler cannot prove a resource uniform across the wave, it wraps the load
in a loop over lanes (v_readfirstlane, compare, exec mask, branch back),
which costs every stage of a tile a dozen extra instructions per load; the
exchange kernels once did this and ran at 54 instead of 60 TFLOP/s.  The
check: no buffer load of the 16x16x4 kernels sits inside such a loop.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_06536_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "--cuda-device-only", "-S"]

# kernels on the 16x16x4 engine (buffer-load operands), per source file
KERNELS = {
    "jk_fp64.hip": ["k_half_transform16", "k_half_transform16a", "k_half_transform16_packed",
                    "k_exchange16"],
    "jk_vjp.hip": ["k_vjp_stage_b", "k_vjp_stage_c", "k_vjp_stage_d"],
    "jk_batched.hip": ["k_b_half_transform16", "k_b_exchange"],
}


def _assembly(src, tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    out = tmp_path / (src + ".s")
    r = subprocess.run([HIPCC, *FLAGS, "-o", str(out), os.path.join(CSRC, src)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text().split("\n")


def _functions(lines):
    """name -> list of instruction lines of each kernel body."""
    funcs, name = {}, None
    for line in lines:
        m = re.match(r"^(_Z\S+):", line)
        if m:
            name = m.group(1)
            funcs[name] = []
            continue
        if name is not None:
            if line.lstrip().startswith(".end_amdhsa_kernel") or line.startswith("\t.size"):
                name = None
                continue
            funcs[name].append(line.strip())
    return funcs


def _lane_loops(body):
    """Buffer loads inside a loop that steps through the lanes' values: a
    short backward s_cbranch_execnz whose body opens with v_readfirstlane of
    the resource and holds an s_and_saveexec and the load."""
    found = []
    labels = {}
    for i, ins in enumerate(body):
        m = re.match(r"^(\.LBB\S+):", ins)
        if m:
            labels[m.group(1)] = i
    for i, ins in enumerate(body):
        m = re.match(r"s_cbranch_execnz\s+(\.LBB\S+)", ins)
        if not m or m.group(1) not in labels:
            continue
        head = labels[m.group(1)]
        if not 0 < i - head <= 24:
            continue
        loop = [x for x in body[head + 1:i + 1] if x and not x.startswith(";")]
        if (any(x.startswith("v_readfirstlane") for x in loop[:4])
                and any(x.startswith("s_and_saveexec") for x in loop)
                and any(x.startswith("buffer_load") for x in loop)):
            found.append(i)
    return found


@pytest.mark.parametrize("src", sorted(KERNELS))
def test_buffer_loads_take_scalar_resources(src, tmp_path):
    funcs = _functions(_assembly(src, tmp_path))
    seen = set()
    for mangled, body in funcs.items():
        short = next((k for k in KERNELS[src] if re.search(r"\d" + re.escape(k) + r"[EI]", mangled)),
                     None)
        if short is None:
            continue
        seen.add(short)
        assert any(x.startswith("buffer_load") for x in body), mangled
        assert not _lane_loops(body), f"{mangled}: buffer loads inside a per-lane loop"
    assert seen == set(KERNELS[src]), (src, sorted(set(KERNELS[src]) - seen))

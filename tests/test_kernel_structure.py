"""Host check of the compiled persistent kernel (no GPU needed: hipcc cross-compiles).

The persistent schedule's task loop must keep wavefront 0 whole between barriers: a
layout in which the loop's exit mask is a single lane lets the other lanes go back to the
barrier without it, and the workgroup then repeats its previous task without end.  In the
compiled code that shows as barriers inside a loop nested in the task loop.  This test
compiles every instantiation the library uses to gfx950 assembly and checks that each
barrier sits directly in the task loop (loop depth 1).
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1304_7211_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (KIND, ORIENT, S, LMAX, NW): span kernels (KIND 0) with every LMAX, sliding kernels
# (KIND 1); eight wavefronts with strips of 4 and 8, four wavefronts with strips of 8
VARIANTS = [(k, o, s, l, nw) for k in (0, 1) for o in (0, 1) for (s, nw) in ((4, 8), (8, 8), (8, 4))
            for l in ((1, 4, 8, 16) if k == 0 else (1,))]


def _barrier_depths(asm):
    """{kernel symbol: [loop depth of the block holding each s_barrier]}"""
    out, name, label = {}, None, ""
    for line in asm.splitlines():
        m = re.match(r"^(_ZN3rlk14persist_kernel\S+):", line)
        if m:
            name, label = m.group(1), ""
            out[name] = []
            continue
        if name is None:
            continue
        if re.match(r"^(\.LBB\S+|; %bb\.\d+):", line):
            label = line
        elif "s_barrier" in line:
            d = re.search(r"Depth=(\d+)", label)
            out[name].append(int(d.group(1)) if d else 0)
        elif line.strip().startswith("s_endpgm"):
            name = None
    return out


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="needs hipcc")
def test_persistent_kernel_barriers_in_task_loop(tmp_path):
    src = tmp_path / "persist.hip"
    src.write_text('#include "rl_kernels.hpp"\n' + "".join(
        f"template __global__ void rlk::persist_kernel<{k}, {o}, {s}, {l}, {nw}>(rlk::PersistArgs);\n"
        for k, o, s, l, nw in VARIANTS))
    asm = tmp_path / "persist.s"
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "--offload-arch=gfx950", "-O3",
           "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "--offload-device-only", "-S", str(src), "-o", str(asm)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    depths = _barrier_depths(asm.read_text())
    assert len(depths) == len(VARIANTS)
    for name, ds in depths.items():
        assert ds, name
        assert all(d == 1 for d in ds), (name, ds)

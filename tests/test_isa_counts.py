"""The benchmark's algorithmic work figure for the fused stencil -- dynamic
VALU lane-operations per output pixel of the steady-state loop -- checked
against the gfx950 code the compiler makes of the kernel now (no GPU: the
kernel is compiled to assembly on the host).

The loop marches six rows per iteration and issues one 12-byte load and one
wide store per lane and row (BF16 / FP16: dwordx2, FP32: dwordx4); views
narrower than 4 pixels have a loop of their own that loads byte by byte.
Edge strips run an extra block that puts mirrored columns in lane order; it
sits behind a uniform branch and is not part of the steady state.
Per pixel: (VALU instructions of the loop - that block) / (6 rows x 4 pixels)."""
import os
import re
import shutil
import subprocess

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_08661_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
WIDE_STORE = {0: "buffer_store_dwordx4", 1: "buffer_store_dwordx2", 2: "buffer_store_dwordx2"}


def _loop_lane_ops_per_px(asm: str, prec: int) -> float:
    name = f"_ZN4igsp12_GLOBAL__N_117edge_fused_kernelILi{prec}ELi4EEEvNS_10EdgeLaunchEii"
    i = asm.index(name + ":")
    body = asm[i:asm.index("s_endpgm", i)].splitlines()
    labels = {m.group(1): k for k, line in enumerate(body) if (m := re.match(r"^(\.LBB\S+):", line))}
    best = None
    for k, line in enumerate(body):
        m = re.search(r"s_cbranch_\w+\s+(\.LBB\S+)|s_branch\s+(\.LBB\S+)", line)
        if not m:
            continue
        target = m.group(1) or m.group(2)
        if target not in labels or labels[target] >= k:
            continue
        seg = body[labels[target]:k + 1]
        ins = [x.strip() for x in seg if x.strip() and not x.strip().startswith((".", ";"))]
        if sum(1 for x in ins if x.split()[0] == WIDE_STORE[prec]) != 6:
            continue
        if sum(1 for x in ins if x.split()[0] == "buffer_load_dwordx3") != 6:
            continue  # the byte-by-byte loop of views narrower than 4 pixels
        valu = sum(1 for x in ins if x.startswith("v_"))
        remap = 0
        for a, x in enumerate(seg):
            mm = re.search(r"s_cbranch_vccnz\s+(\.LBB\S+)", x)
            if mm:
                end = next(b for b in range(a + 1, len(seg)) if seg[b].startswith(mm.group(1) + ":"))
                remap += sum(1 for y in seg[a + 1:end] if y.strip().startswith("v_"))
        per_px = (valu - remap) / 24.0
        best = per_px if best is None else max(best, per_px)
    assert best is not None, "steady-state loop not found"
    return best


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_loop_lane_ops_match_the_benchmark_figure(tmp_path):
    out = tmp_path / "edge_kernels.s"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "--cuda-device-only", "-S", os.path.join(CSRC, "edge_kernels.hip"),
                    "-o", str(out)], check=True, capture_output=True)
    asm = out.read_text()
    for prec, name in ((0, "fp32"), (1, "fp16"), (2, "bf16")):
        got = _loop_lane_ops_per_px(asm, prec)
        assert abs(got - bench.LOOP_LANE_OPS_PER_PX[name]) < 0.01, (name, got)

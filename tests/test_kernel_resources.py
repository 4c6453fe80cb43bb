"""Register-resident accumulators of the AAR history kernels (host-only check).

The Anderson step's Gram partials are 35 FP64 accumulators per thread; a
reduction loop that indexes them at run time makes the compiler place the
array in scratch (per-lane private) memory, which cost a factor of three in
that kernel.  This compiles the AAR source for gfx950 (device code only, a
couple of seconds) and reads the compiler's resource-usage remarks: the
grid-wide history kernels must use no scratch.  The per-orbital normal
equation solve runs on one thread per orbital and may keep its small matrix
in scratch.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_01186_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _resource_usage(src):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "--cuda-device-only", "-c", "-Rpass-analysis=kernel-resource-usage",
           "-I" + CSRC, os.path.join(CSRC, src), "-o", os.devnull]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    usage, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            usage[name] = {}
            continue
        m = re.search(r"(VGPRs|ScratchSize \[bytes/lane\]): (\d+)", line)
        if m and name:
            usage[name][m.group(1).split()[0]] = int(m.group(2))
    return usage


def test_aar_history_kernels_use_no_scratch():
    usage = _resource_usage("aar.hip")
    names = {k: v for k, v in usage.items() if "k_aar_dots" in k or "k_aar_step" in k}
    assert any("k_aar_dots" in k for k in names) and sum("k_aar_step" in k for k in names) == 2, usage
    for k, v in names.items():
        assert v.get("ScratchSize") == 0, (k, v)

"""Register budget of the device code (compiled for gfx950 on the host, no GPU
needed): no kernel spills to scratch memory; the residual and product kernels
keep the eight waves per SIMD they are built for, and the G^T and G
iteration kernels (two rows per lane over sliced diagonals, twice the
operands) the four waves their default grid fills. A spill in the SpMV
kernels costs several times their run time."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_27517_amd", "csrc")


def _resource_usage(tmp_path):
    from paper_2510_27517_amd import build

    cmd = [build.HIPCC, *build.COMMON, *build.DEVICE, "-Rpass-analysis=kernel-resource-usage", "-c",
           os.path.join(CSRC, "kernels.hip"), "-o", str(tmp_path / "k.o")]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-2000:]
    out, cur = {}, None
    for line in r.stdout.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        for key, pat in (("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"), ("occupancy", r"Occupancy \[waves/SIMD\]: (\d+)"),
                         ("vgpr", r"VGPRs: (\d+)")):
            m = re.search(pat, line)
            if m and cur:
                out[cur][key] = int(m.group(1))
    return out


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not installed")
def test_no_spills_and_full_occupancy(tmp_path):
    res = _resource_usage(tmp_path)
    assert len(res) > 50
    spills = {k: v["scratch"] for k, v in res.items() if v.get("scratch", 0) > 0}
    assert not spills, spills
    want = {}
    for k in res:
        if re.search(r"k_iter_GT?I", k):
            want[k] = 4
        elif re.search(r"k_(iter_A|resid|spmv|spmm)I", k):
            want[k] = 8
    assert len(want) >= 20
    low = {k: res[k].get("occupancy") for k in want if res[k].get("occupancy", 0) < want[k]}
    assert not low, low

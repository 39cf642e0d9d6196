"""Register budget of the FP32-bulk 2D stage kernels, from the compiler's
own report for gfx950 (hipcc, device code only; no GPU needed).

Three 16x14 blocks share a CU only while each lane holds at most 168
registers; the kernel carries a waves-per-EU bound of 3, so a change that
needs more registers would spill to scratch memory instead.  This test
fails on either: more than 168 registers, or any scratch use."""
import os
import re
import subprocess

import pytest

from paper_2210_04037_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fp32_asm(tmp_path_factory):
    try:
        hipcc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    flags = dict(B.UNITS)["fv_fp32.hip"]
    out = str(tmp_path_factory.mktemp("asm") / "fv_fp32.s")
    cmd = ([hipcc] + B.FLAGS + flags +
           ["--cuda-device-only", "-S", "-o", out, os.path.join(B.CSRC, "fv_fp32.hip")])
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    with open(out) as f:
        return f.read()


def _kernel_info(asm, tx, ty, nth, nm):
    """Largest VGPR, AGPR and scratch figures over the builds of one tile
    shape (with and without the extended closures)."""
    name = (f"_ZN3fvk12stage_kernelILi2ELi{nm}ELi1EffLi{tx}ELi{ty}ELi{nth}E")
    found = list(re.finditer(r"^(" + re.escape(name) + r"\S*):", asm, re.M))
    assert len(found) == 2, f"stage kernel {tx}x{ty}/{nth} (NM={nm}): {len(found)} builds"
    out = []
    for m in found:
        end = asm.index(".Lfunc_end", m.end())
        info = asm[end:end + 12000]
        get = lambda k: int(re.search(r"; %s: (\d+)" % k, info).group(1))
        out.append((get("NumVgprs"), get("NumAgprs"), get("ScratchSize")))
    return tuple(max(v[i] for v in out) for i in range(3))


@pytest.mark.parametrize("nm", [1, 2])
def test_16x14_stage_kernel_fits_three_blocks_per_cu(fp32_asm, nm):
    vgpr, agpr, scratch = _kernel_info(fp32_asm, 16, 14, 256, nm)
    assert vgpr + agpr <= 168, (vgpr, agpr)
    assert scratch == 0


@pytest.mark.parametrize("tx,ty,nth", [(16, 15, 256), (32, 7, 256), (15, 16, 256),
                                       (32, 15, 512), (64, 8, 512), (32, 8, 256)])
def test_other_fp32_tiles_do_not_spill(fp32_asm, tx, ty, nth):
    assert _kernel_info(fp32_asm, tx, ty, nth, 2)[2] == 0

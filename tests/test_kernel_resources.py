"""The production kernels fit in registers: no private (scratch) memory.

Each HIP source is compiled for gfx950 with the library's own flags
(paper_2306_05051_amd/build.py) and the compiler's resource report is read.
A production kernel (every glint_* kernel but the instrumented debug
instantiations of the forward) that needs scratch memory, from register
spills or from a helper that is called instead of inlined (whose arguments
then travel through a stack in scratch), runs several times slower without
any change in its results, so parity tests cannot see it; this test does.
CPU only (hipcc cross-compiles), about half a minute.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2306_05051_amd import build

HIPCC = build.HIPCC
pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which(HIPCC)), reason="hipcc not available")

_REPORT = re.compile(r"Function Name: (\S+).*?VGPRs: (\d+).*?ScratchSize \[bytes/lane\]: (\d+)"
                     r".*?Occupancy \[waves/SIMD\]: (\d+)", re.S)


def _debug_instantiation(name):
    # glint_fwd_kernel<true, ...>: the instrumented forward (debug planes, dumps)
    return name.startswith("_ZN5glint16glint_fwd_kernelILb1E")


def _report(src, tmp_path):
    cmd = [HIPCC, *build.FLAGS, *build.SOURCE_FLAGS.get(src, []), "--cuda-device-only", "-c",
           "-Rpass-analysis=kernel-resource-usage", os.path.join(build.CSRC, src),
           "-o", str(tmp_path / (src + ".o"))]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    return [(m.group(1), int(m.group(2)), int(m.group(3)), int(m.group(4))) for m in _REPORT.finditer(r.stderr)]


@pytest.mark.parametrize("src", build.SOURCES)
def test_production_kernels_use_no_scratch(src, tmp_path):
    rows = _report(src, tmp_path)
    kernels = [r for r in rows if "glint" in r[0] and not _debug_instantiation(r[0])]
    assert kernels, f"no kernel reported for {src}"
    bad = [(n, v, s) for n, v, s, _ in kernels if s != 0]
    assert not bad, f"kernels with scratch (name, VGPRs, bytes per lane): {bad}"


def test_shading_kernels_keep_four_waves_per_simd(tmp_path):
    """The forward's LDS allows 16 tiles per CU; its production kernels must
    not lose that occupancy to registers (at most 128 VGPRs)."""
    rows = _report("glint_fwd.hip", tmp_path)
    fwd = [r for r in rows if r[0].startswith("_ZN5glint16glint_fwd_kernelILb0E")]
    assert len(fwd) >= 4
    low = [(n, v, o) for n, v, _, o in fwd if o < 4]
    assert not low, f"forward kernels below 4 waves per SIMD: {low}"

"""Register budget of the coefficient kernels, checked on the CPU from the
compiler's own resource report (hipcc cross-compiles gfx950 device code).

The coefficient launches are VALU-issue bound, and their speed rests on how
many wavefronts share a SIMD: the kernels ask for a fixed number with
`amdgpu_waves_per_eu`, and the file is built without machine-level hoisting so
that they fit it.  A change that makes a kernel spill to scratch instead of
fitting its budget shows up here, before any GPU run."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2608_16208_amd")
SRC = "csrc/ffbie_kernels.hip"


@pytest.fixture(scope="module")
def report(tmp_path_factory):
    sys.path.insert(0, PKG)
    try:
        import build as b
    finally:
        sys.path.remove(PKG)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("ru") / "k.o")
    cmd = ([hipcc] + b.FLAGS + b.EXTRA.get(SRC, [])
           + ["--cuda-device-only", "-Rpass-analysis=kernel-resource-usage",
              "-c", os.path.join(PKG, SRC), "-o", out])
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    kernels = {}
    for block in res.stderr.split("Function Name: ")[1:]:
        name = block.split()[0]
        fields = dict(re.findall(r"remark:\s+([A-Za-z][A-Za-z ]*?)(?: \[[^\]]*\])?: (\S+) \[-Rpass",
                                 block))
        kernels[name] = fields
    return kernels


def _coeff(kernels):
    return {n: f for n, f in kernels.items() if "ffbie_coeff" in n}


def test_no_coefficient_kernel_spills(report):
    coeff = _coeff(report)
    # 5 azimuthal orders x {main, refine} x {FP64, FP32} x radix, plus the batch kernels
    assert len(coeff) >= 30, sorted(coeff)
    bad = {n: (f.get("VGPRs Spill"), f.get("ScratchSize")) for n, f in coeff.items()
           if f.get("VGPRs Spill") != "0" or f.get("ScratchSize") != "0"}
    assert not bad, bad


@pytest.mark.parametrize("real, waves", [("d", 4), ("f", 5)])
def test_config2_kernel_occupancy(report, real, waves):
    """The kernel of the config-2 launch (azimuthal order 2, radix 2, main
    pass, unstretched surface): four wavefronts per SIMD in FP64, five with the
    FP32 spectral stage."""
    name = "_ZN5ffbie20ffbie_coeff_kernel_tILi2ELb0E%sLi2ELb0EEEvNS_9CoeffArgsE" % real
    f = report[name]
    assert int(f["Occupancy"]) == waves, f
    assert int(f["VGPRs"]) <= 512 // waves, f

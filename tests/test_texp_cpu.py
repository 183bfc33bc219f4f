"""The table-driven double exp of the FP64 dense passes (pins_texp.h, Tang's
method) checked on the CPU against the host libm exp: at most 1 ulp over
random and edge arguments in [-746, 710] (subnormal results included), exact
underflow to 0 below the range, overflow to inf above it, NaN kept.  The
header is the very code the kernels run (host and device share it)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_03749_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_texp_against_libm(tmp_path):
    exe = str(tmp_path / "texp_check")
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", CSRC,
                           os.path.join(ROOT, "tests", "texp_check.cpp"), "-o", exe])
    out = subprocess.check_output([exe, "4000000"], text=True).split()
    res = dict(zip(out[0::2], out[1::2]))
    assert int(res["special_ok"]) == 1
    assert int(res["n"]) > 5_000_000
    assert float(res["max_ulp"]) <= 1.0, res
    assert int(res["nonpos_diff"]) == 0, res  # the sweeps' form for x <= 0 is bitwise the general one

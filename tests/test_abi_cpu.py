"""CPU checks of the C ABI: the library loads, exports every declared symbol,
its struct layouts match the ctypes mirror, and the host-only calls behave.
No compute call is made (there is no GPU here)."""
import ctypes
import os
import subprocess

import pytest

import paper_2502_03749_amd as P
from paper_2502_03749_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = P.declared_functions()
    assert "pins_solve" in names and "pins_solve_batch_device" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert L.pins_abi_version() == 2


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "pins.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(pins_params), sizeof(pins_problem),'
                   ' sizeof(pins_result), offsetof(pins_result, kern_ms), offsetof(pins_problem, a));'
                   'printf("%zu %zu\\n", sizeof(pins_state), offsetof(pins_state, B));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert got == [ctypes.sizeof(B.Params), ctypes.sizeof(B.Problem), ctypes.sizeof(B.Result),
                   B.Result.kern_ms.offset, B.Problem.a.offset, ctypes.sizeof(B.State), B.State.B.offset]


def test_default_params_are_the_papers():
    p = P.params()
    assert (p.max_outer, p.max_sinkhorn, p.max_newton) == (250, 100, 50)
    assert (p.ls_beta, p.ls_c1, p.cg_rtol, p.inner_tol) == (0.5, 1e-4, 1e-6, 1e-9)


def test_workspace_bytes_scales_with_size():
    prm = P.params()
    small = P.workspace_bytes([dict(kind=P.COST_DENSE, m=100, n=100)], prm)
    big = P.workspace_bytes([dict(kind=P.COST_DENSE, m=1000, n=1000)], prm)
    assert 0 < small < big
    two = P.workspace_bytes([dict(kind=P.COST_DENSE, m=100, n=100)] * 2, prm)
    assert two > small
    mat = P.workspace_bytes([dict(kind=P.COST_DENSE, m=1000, n=1000)], P.params(shift_mode=P.SHIFT_MATERIALIZED))
    assert mat >= big + 1000 * 1000 * 8


def test_workspace_bytes_rejects_bad_input():
    with pytest.raises(B.PinsError):
        P.workspace_bytes([dict(kind=P.COST_GRID, m=10, n=10, grid_s=3)], P.params())
    with pytest.raises(B.PinsError):
        P.workspace_bytes([dict(kind=P.COST_DENSE, m=10, n=10)], P.params(eta=-1.0))


def test_workspace_bytes_size_limits():
    # m*n < 2^31 and m+n < 2^28 (the CG stores byte offsets of vector entries
    # in int32); both are refused as unsupported, not as invalid
    with pytest.raises(B.PinsError) as e:
        P.workspace_bytes([dict(kind=P.COST_DENSE, m=2, n=(1 << 30) + 1)], P.params())
    assert e.value.code == B.PINS_EUNSUPPORTED
    with pytest.raises(B.PinsError) as e:
        P.workspace_bytes([dict(kind=P.COST_DENSE, m=1, n=(1 << 28) - 1)], P.params())
    assert e.value.code == B.PINS_EUNSUPPORTED
    P.workspace_bytes([dict(kind=P.COST_DENSE, m=1, n=(1 << 28) - 2)], P.params(max_outer=1))


def test_create_without_gpu_reports_device_error():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(B.PinsError) as e:
        P.Context(0)
    assert e.value.code == B.PINS_EDEVICE


def test_server_without_gpu_reports_device_error():
    """On a host without a usable GPU the server refuses to start (no crash)."""
    import ctypes
    import paper_2502_03749_amd as P
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    prm = P.params(eta=0.1)
    assert P.lib().pins_server_create(0, 2, 8, 0, ctypes.byref(prm), ctypes.byref(h)) == P._binding.PINS_EDEVICE
    assert P.lib().pins_server_create(0, 0, 8, 0, ctypes.byref(prm), ctypes.byref(h)) == P._binding.PINS_EINVAL


def test_entry_points_reject_a_null_context():
    """Every solve entry point returns PINS_EINVAL for a NULL context, with no GPU."""
    prm = P.params(eta=0.1)
    L = P.lib()
    assert L.pins_solve(None, None, ctypes.byref(prm), None) == B.PINS_EINVAL
    assert L.pins_solve_device(None, None, ctypes.byref(prm), None, None) == B.PINS_EINVAL
    assert L.pins_solve_batch_device(None, None, 1, ctypes.byref(prm), None, None) == B.PINS_EINVAL
    assert L.pins_solve_resume(None, None, ctypes.byref(prm), None, 0, None, None) == B.PINS_EINVAL
    best = B.Params()
    assert L.pins_tune_batch_device(None, None, 1, ctypes.byref(prm), 4, 1, None, None, ctypes.byref(best),
                                    None, 0, None) == B.PINS_EINVAL
    assert L.pins_solve_device_noalloc(None, None, ctypes.byref(prm), None, None) == B.PINS_EINVAL


def test_exp_probe_argument_checks():
    """pins_probe_exp_rate rejects bad sizes before touching a device; without a GPU it reports a device error."""
    import torch

    rate = ctypes.c_double(0.0)
    L = P.lib()
    assert L.pins_probe_exp_rate(0, 0, 16, ctypes.byref(rate), None) == B.PINS_EINVAL
    assert L.pins_probe_exp_rate(0, 8, 0, ctypes.byref(rate), None) == B.PINS_EINVAL
    assert L.pins_probe_exp_rate(0, 8, 16, None, None) == B.PINS_EINVAL
    if not torch.cuda.is_available():
        assert L.pins_probe_exp_rate(0, 8, 16, ctypes.byref(rate), None) == B.PINS_EDEVICE

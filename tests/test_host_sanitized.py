"""The library's host code under AddressSanitizer and UBSan, without a GPU.

The host sources (validation, workspace planning, entry-point guards, the
server) are compiled with the sanitizers on the host side only, linked with
the kernels into a small driver and run on the CPU: workspace planning of
single, uneven and grid batches, argument rejection, context creation with
no usable device and the NULL-context guards.  Any out-of-bounds access,
leak or undefined arithmetic on those paths fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_03749_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DRIVER = r"""
#include <cstdio>
#include <cstring>
#include "pins.h"

static int bad = 0;
static void expect(bool ok, int line) {
    if (!ok) { std::printf("failed check at line %d\n", line); bad = 1; }
}
#define EXPECT(c) expect((c), __LINE__)

int main() {
    pins_params p;
    pins_params_default(&p);
    static double a[4] = {0.25, 0.25, 0.25, 0.25}, C[16];
    pins_problem pr;
    std::memset(&pr, 0, sizeof(pr));
    pr.kind = PINS_COST_DENSE; pr.m = 4; pr.n = 4; pr.a = a; pr.b = a; pr.C = C;
    size_t one = 0, two = 0, grid = 0;
    EXPECT(pins_workspace_bytes(&pr, 1, &p, &one) == PINS_OK && one > 0);
    pins_problem many[2] = {pr, pr};
    many[1].m = 1000; many[1].n = 17;
    EXPECT(pins_workspace_bytes(many, 2, &p, &two) == PINS_OK && two > one);
    pins_problem g = pr;
    g.kind = PINS_COST_GRID; g.grid_s = 9; g.m = g.n = 81; g.C = nullptr;
    EXPECT(pins_workspace_bytes(&g, 1, &p, &grid) == PINS_OK && grid > 0);
    size_t x = 0;
    pr.m = 0; EXPECT(pins_workspace_bytes(&pr, 1, &p, &x) == PINS_EINVAL); pr.m = 4;
    pr.C = nullptr; EXPECT(pins_workspace_bytes(&pr, 1, &p, &x) == PINS_EINVAL); pr.C = C;
    p.eta = -1.0; EXPECT(pins_workspace_bytes(&pr, 1, &p, &x) == PINS_EINVAL); pins_params_default(&p);
    EXPECT(pins_workspace_bytes(&pr, 0, &p, &x) == PINS_EINVAL);
    pr.m = 1 << 16; pr.n = 1 << 16;
    EXPECT(pins_workspace_bytes(&pr, 1, &p, &x) == PINS_EUNSUPPORTED); pr.m = pr.n = 4;
    pins_ctx* ctx = nullptr;
    int rc = pins_create(0, &ctx);
    EXPECT(rc == PINS_EDEVICE || rc == PINS_OK);
    if (rc == PINS_OK) pins_destroy(ctx);
    pins_result r;
    std::memset(&r, 0, sizeof(r));
    EXPECT(pins_solve(nullptr, &pr, &p, &r) == PINS_EINVAL);
    EXPECT(pins_solve_resume(nullptr, &pr, &p, nullptr, 0, nullptr, &r) == PINS_EINVAL);
    pins_params best;
    EXPECT(pins_tune_batch_device(nullptr, &pr, 1, &p, 4, 1, &r, nullptr, &best, nullptr, 0, nullptr) == PINS_EINVAL);
    EXPECT(pins_solve_device_noalloc(nullptr, &pr, &p, &r, nullptr) == PINS_EINVAL);
    p.tile_rows[1] = 65; EXPECT(pins_workspace_bytes(&pr, 1, &p, &x) == PINS_EINVAL); pins_params_default(&p);
    pins_server* s = nullptr;
    rc = pins_server_create(0, 2, 8, 0, &p, &s);
    EXPECT(rc == PINS_EDEVICE || rc == PINS_OK);
    if (rc == PINS_OK) pins_server_destroy(s);
    EXPECT(pins_server_create(0, 0, 8, 0, &p, &s) == PINS_EINVAL);
    std::printf("workspace %zu %zu %zu bad %d\n", one, two, grid, bad);
    return bad;
}
"""


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("gcc") is None, reason="needs hipcc")
def test_host_code_clean_under_asan_and_ubsan(tmp_path):
    (tmp_path / "drv.cpp").write_text(DRIVER)
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    objs = []
    for src, sanitize in (("pins_kernels.hip", False), ("pins_probe.hip", False), ("pins_host.cpp", True),
                          ("pins_server.cpp", True), (str(tmp_path / "drv.cpp"), True)):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        subprocess.check_call([HIPCC] + common + (san if sanitize else []) + ["-c", path, "-o", obj],
                              stderr=subprocess.DEVNULL)
        objs.append(obj)
    exe = str(tmp_path / "drv")
    subprocess.check_call([HIPCC, "-fsanitize=address,undefined", "-fno-gpu-sanitize", "--offload-arch=gfx950"] +
                          objs + ["-o", exe], stderr=subprocess.DEVNULL)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "bad 0" in r.stdout

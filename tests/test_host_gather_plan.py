"""The neighbour-gather planner (plan_gather in csrc/gather_plan.cpp) on the
host: tests/host/gather_plan_check.cpp plans seeded random gather lists (FP64
blocks, FP32 copies, packed BF16 copies; narrow and wide chunks; column
segments; 1-3 right-hand sides), evaluates every plan the way the chunk and
reduction kernels define it, and requires the gathers' definition
y_i = base_i + alpha_i sum op(B) x bit for bit (integer data), every slot
written once, every block element read once, documented chunk boundaries and
flags, and every read inside the block's copy.  Built with g++ from the
library's own planner source, with the address and undefined-behaviour
checks when the toolchain links them."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECK_SRC = os.path.join(ROOT, "tests", "host", "gather_plan_check.cpp")
PLAN_SRC = os.path.join(ROOT, "paper_2502_02395_amd", "csrc", "gather_plan.cpp")
ROCM_INC = "/opt/rocm/include"


def _build(out):
    base = ["g++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC,
            CHECK_SRC, PLAN_SRC, "-o", out]
    checked = base[:1] + ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"] + base[1:]
    for cmd in (checked, base):
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
        if r.returncode == 0:
            return
    pytest.fail("could not build the planner check:\n" + r.stderr[-3000:])


def test_gather_plans_evaluate_to_the_definition(tmp_path):
    if shutil.which("g++") is None or not os.path.isdir(ROCM_INC):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path / "gather_plan_check")
    _build(exe)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " 0 failures" in r.stdout

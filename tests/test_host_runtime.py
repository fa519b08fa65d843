"""The library's host layer (pf_api.cpp: handles, filter-group streams,
event fork and join, graph capture and replay, tuning changes, timing,
history, the PMMH and SMC^2 drivers) built for the CPU against a stand-in
HIP runtime (tests/hostcheck/fake_hip.cpp) and kernel launchers that do
nothing, then driven through the call sequences of the GPU tests and the
benchmark under AddressSanitizer and UndefinedBehaviorSanitizer.  The
stand-in checks the stream-capture rules (forked streams joined back
before the capture ends, no host copy, memset, synchronisation or
null-stream work inside a capture, no use of destroyed streams, events or
graphs).  No GPU and no result values are involved: only host logic."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1306_3277_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "hostcheck")
CXX = "/opt/rocm/llvm/bin/clang++"
HEADERS = ["pf_internal.hpp", "pf_smc2.hpp", "pf_path.hpp", "pf_kalman.hpp"]
SCENARIOS = ["autotune", "groups", "bench", "plain", "errors", "pmmh", "smc2", "kalman"]


def launcher_stubs():
    """One stub per kernel launcher declared in the internal headers: it
    records a kernel on the launcher's stream and does nothing else."""
    out = [f'#include "{h}"' for h in HEADERS]
    out += ['extern "C" void fake_kernel(hipStream_t s);', "namespace pfk {"]
    seen = []
    for h in HEADERS:
        src = open(os.path.join(CSRC, h)).read()
        for m in re.finditer(r"hipError_t (launch_\w+)\(([^;]*?)\);", src, re.S):
            name, params = m.group(1), m.group(2)
            if name in seen:
                continue
            last = params.split(",")[-1].strip()
            assert last.startswith("hipStream_t"), (name, last)
            seen.append(name)
            out.append(f"hipError_t {name}({params}) {{ fake_kernel({last.split()[-1]}); "
                       "return hipSuccess; }")
    out.append("}  // namespace pfk")
    return "\n".join(out) + "\n", seen


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("ROCm clang++ not found")
    d = tmp_path_factory.mktemp("hostcheck")
    stubs, names = launcher_stubs()
    assert len(names) >= 20
    (d / "stubs.cpp").write_text(stubs)
    flags = ["-std=c++17", "-g", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-w"]
    srcs = [os.path.join(CSRC, "pf_api.cpp"), os.path.join(HERE, "fake_hip.cpp"),
            os.path.join(HERE, "driver.cpp"), str(d / "stubs.cpp")]
    procs, objs = [], []
    for s in srcs:
        o = str(d / (os.path.splitext(os.path.basename(s))[0] + ".o"))
        procs.append(subprocess.Popen([CXX] + flags + ["-c", s, "-o", o], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True, cwd=str(d)))
        objs.append(o)
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out[-4000:]
    exe = str(d / "driver")
    r = subprocess.run([CXX] + flags + ["-o", exe] + objs, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    # the library must not link any HIP symbol the stand-in lacks: the link
    # above resolved them all without libamdhip64
    yield exe
    shutil.rmtree(str(d), ignore_errors=True)


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_host_layer_under_sanitizers(driver, scenario):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([driver, scenario], capture_output=True, text=True, env=env, timeout=300)
    log = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, log
    assert f"scenario {scenario} done" in r.stdout, log
    assert "FAKEHIP VIOLATION" not in log and "runtime error" not in log, log

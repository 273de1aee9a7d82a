"""Host-side parsers and planners under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library sources that hold host logic taking untrusted sizes or text (the
expression-program parser, the tiling planner, the batch plan's validation,
the status and workspace queries) are compiled host-only with the sanitizers
and linked into the seeded fuzz driver tests/host_fuzz/fuzz_host.cpp, which
must finish with no failed check and no sanitizer report.
"""

import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_19851_amd", "csrc")
SOURCES = ["abi_common.hip", "expr.hip", "tiled.hip", "batch.hip"]
HIPCC = "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _have_toolchain():
    return os.path.exists(HIPCC) and os.path.exists(CLANGXX)


@pytest.fixture(scope="module")
def fuzz_exe(tmp_path_factory):
    if not _have_toolchain():
        pytest.skip("ROCm toolchain not found")
    out = tmp_path_factory.mktemp("host_fuzz")
    common = ["-O1", "-g", "-std=c++17", "-fPIC", f"-I{ROOT}/include", f"-I{CSRC}"]

    def compile_one(src):
        obj = str(out / (src[:-4] + ".o"))
        # device code as usual; the sanitizers apply to the host code only
        cmd = [HIPCC, "--offload-arch=gfx950", *SAN, *common, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    drv = str(out / "fuzz_host.o")
    r = subprocess.run([CLANGXX, "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *common, "-c",
                        os.path.join(ROOT, "tests", "host_fuzz", "fuzz_host.cpp"), "-o", drv],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(out / "fuzz_host")
    r = subprocess.run([CLANGXX, "-fsanitize=address,undefined", "-o", exe, drv, *objs, "-L/opt/rocm/lib",
                        "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lhiprtc"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    yield exe
    shutil.rmtree(out, ignore_errors=True)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_host_fuzz_clean_under_sanitizers(fuzz_exe, seed):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["HIP_VISIBLE_DEVICES"] = ""  # host code only; no device is used
    r = subprocess.run([fuzz_exe, str(seed), "1500"], capture_output=True, text=True, env=env, timeout=600)
    report = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, report
    assert "0 failures" in r.stdout, report
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report

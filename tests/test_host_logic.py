"""Host logic of the runtime on the CPU: the tile and injection tables, the
workspace layout and the storage-RTM launch schedule, checked by a C++
program that includes the runtime with the device launchers replaced by
recorders (no GPU call), built with host AddressSanitizer and UBSan; and
every entry point of the oracle under the same sanitizers."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2204_03380_amd", "csrc")
RECORDERS = {"launch_fwd2d", "launch_fwd3d", "launch_fwd2d_t2", "launch_fwd2d_t3", "launch_snap_store", "launch_recv2d",
             "launch_recv3d", "launch_inj_set", "launch_rev2d", "launch_rev2d_t2", "launch_rev2d_t3", "launch_sample"}


def _stubs(api_src):
    """A definition returning hipSuccess for every launcher the runtime
    declares, except those the checker records itself."""
    head = api_src[:api_src.index("}  // namespace rtm")]
    out = []
    for full, name in re.findall(r"(hipError_t\s+(launch_\w+)\(.*?\);)", head, re.S):
        if name not in RECORDERS:
            out.append(full[:-1] + " { return hipSuccess; }")
    sizes = re.findall(r"(size_t\s+(\w+)\(\);)", head)
    for full, name in sizes:
        out.append(full[:-1] + " { return 64; }")
    return "\n".join(out) + "\n"


@pytest.mark.timeout(600)
def test_host_tables_layout_and_storage_schedule(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    work = str(tmp_path)
    with open(os.path.join(CSRC, "api.hip")) as f:
        stubs = _stubs(f.read())
    with open(os.path.join(work, "stubs.inc"), "w") as f:
        f.write(stubs)
    src = os.path.join(ROOT, "tests", "host", "host_check.hip")
    obj = os.path.join(work, "host_check.o")
    exe = os.path.join(work, "host_check")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    subprocess.run([hipcc, "-std=c++17", "-O1", "-g", "-fPIC", "--cuda-host-only", "-x", "hip", *san,
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", work, "-c", src, "-o", obj],
                   check=True, capture_output=True, text=True)
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc)))
    libdir = os.path.join(rocm, "lib")
    # link with the same compiler's sanitizer runtimes (host only: no device code in the object)
    clang = os.path.join(rocm, "llvm", "bin", "clang++")
    host_san = ["-fsanitize=address,undefined"]
    subprocess.run([clang, obj, "-o", exe, *host_san, "-L", libdir, "-lamdhip64", "-lrocprofiler-sdk-roctx",
                    "-Wl,-rpath," + libdir],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0 and "ALL OK" in r.stdout, (r.stdout[-2000:], r.stderr[-2000:])


@pytest.mark.timeout(300)
def test_oracle_under_sanitizers(tmp_path):
    """Every oracle entry point on tiny 2-D and 3-D grids, built with
    AddressSanitizer and UBSan (plain gcc, no GPU)."""
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = os.path.join(str(tmp_path), "oracle_driver")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.run([gcc, *flags, os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "tests", "host",
                   "oracle_driver.c"), "-o", exe, "-lm"], check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=dict(os.environ, ASAN_OPTIONS=""))
    assert r.returncode == 0 and "ALL OK" in r.stdout, (r.stdout[-2000:], r.stderr[-2000:])

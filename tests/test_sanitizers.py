"""CPU-only AddressSanitizer and UndefinedBehaviorSanitizer builds (gcc) of the
test oracle's C code and of the host-side entry points of libvdwdf.so reached
through the plain C caller: tests/c_abi/sanitize_driver.c runs them on small
inputs; any sanitizer report fails the test.  Nothing here uses the GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "c_abi", "sanitize_driver.c")
ORACLE_C = os.path.join(ROOT, "oracle", "vdw_oracle.c")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(exe, env_extra=None):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    env.pop("LD_PRELOAD", None)
    if env_extra:
        env.update(env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    text = r.stdout + r.stderr
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    assert r.returncode == 0 and "sanitize driver ok" in r.stdout, text[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-std=gnu11", "-Wall"] + SAN + [DRIVER, ORACLE_C, "-o", exe, "-lm"], check=True)
    _run(exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_c_caller_host_paths_under_asan_ubsan(tmp_path):
    lib_dir = os.path.join(ROOT, "paper_0810_2273_amd")
    if not os.path.exists(os.path.join(lib_dir, "libvdwdf.so")):
        pytest.skip("libvdwdf.so is not built")
    exe = str(tmp_path / "caller_san")
    caller = os.path.join(ROOT, "tests", "c_abi", "enl_from_c.c")
    subprocess.run(["gcc", "-std=gnu11", "-Wall", "-DWITH_LIBVDWDF", "-D__HIP_PLATFORM_AMD__"] + SAN +
                   ["-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"), DRIVER, ORACLE_C,
                    caller, "-L" + lib_dir, "-lvdwdf", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
                    "-Wl,-rpath," + lib_dir, "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe, "-lm"], check=True)
    # the HIP runtime's own allocations are not this code's: leak checks off for this process
    _run(exe, {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1"})

"""Build the plain-C caller of libvdwdf.so (tests/c_abi/enl_from_c.c) with
gcc as strict C99: it proves that vdwdf.h and the library serve a C program
that uses only the HIP runtime's C API.  Test infrastructure; run by the
package build after libvdwdf.so exists."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "enl_from_c.c")
LIB = os.path.join(HERE, "libenl_from_c.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"), SRC,
           "-L" + os.path.join(ROOT, "paper_0810_2273_amd"), "-lvdwdf", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_0810_2273_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

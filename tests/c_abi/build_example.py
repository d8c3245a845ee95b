"""Build the plain-C user of the C-ABI (``srm3_c_example``) next to its source,
linked against the in-tree ``libsrm3.so`` (rpath relative to the binary)."""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "srm3_c_example.c")
EXE = os.path.join(HERE, "srm3_c_example")


def build() -> str:
    rocm = "/opt/rocm"
    cc = shutil.which("gcc") or "cc"
    cmd = [cc, "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(rocm, "include"), SRC, "-o", EXE + ".tmp",
           "-L", os.path.join(ROOT, "paper_2310_03979_amd"), "-lsrm3", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2310_03979_amd", "-Wl,-rpath," + os.path.join(rocm, "lib"), "-lm"]
    subprocess.check_call(cmd)
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    print(build())

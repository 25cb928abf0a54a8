"""Build of the plain-C consumer of the library's C ABI (tests/c_abi/abi_smoke):
gcc, C99, linked against paper_2110_03732_amd/libgrmhd.so and the HIP runtime."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "abi_smoke.c")
EXE = os.path.join(HERE, "abi_smoke")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def command(out):
    return ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC, "-o", out,
            "-L", os.path.join(ROOT, "paper_2110_03732_amd"), "-lgrmhd", "-L", os.path.join(ROCM, "lib"),
            "-lamdhip64", "-Wl,-rpath,$ORIGIN/../../paper_2110_03732_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
            "-lm"]


def build(verbose=False):
    tmp = EXE + ".tmp%d" % os.getpid()
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build(verbose=True))

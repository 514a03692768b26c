"""Build the C caller of the library (trace_client) next to its source.

gcc compiles it as C99 against include/rayramses.h and the HIP runtime's C
header (which needs the AMD platform macro that hipcc would define) and links
it to the in-tree librayramses.so (found at run time through an rpath)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "trace_client.c")
OUT = os.path.join(HERE, "trace_client")
PKG = os.path.join(ROOT, "paper_1601_02012_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def command(out=OUT):
    return ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
            "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROCM, "include"), SRC,
            "-o", out, "-L" + PKG, "-lrayramses", "-Wl,-rpath," + PKG,
            "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
            "-lm"]


def build(out=OUT) -> str:
    r = subprocess.run(command(out), capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"trace_client build failed:\n{r.stdout}\n{r.stderr}")
    return out


if __name__ == "__main__":
    print("built", build())

"""Compiles the plain-C consumer of the library's C ABI (test infrastructure:
it links the oracle)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
BIN = os.path.join(HERE, "c_consumer")


def build(out: str = BIN) -> str:
    cmd = [
        "gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
        "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"),
        os.path.join(HERE, "c_consumer.c"), "-o", out,
        "-L" + os.path.join(ROOT, "paper_2106_06161_amd"), "-lbshuffle",
        "-L" + os.path.join(ROOT, "oracle"), "-loracle",
        "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
        "-Wl,-rpath," + ":".join(["$ORIGIN/../../paper_2106_06161_amd", "$ORIGIN/../../oracle",
                                  os.path.join(ROCM, "lib")]),
    ]
    subprocess.check_call(cmd)
    return out


if __name__ == "__main__":
    print(build())

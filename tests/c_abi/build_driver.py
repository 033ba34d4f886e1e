"""Builds tests/c_abi/roundtrip: the plain-C test driver of the library's C
ABI, linked against paper_2505_07158_amd/libvcipher.so, the HIP runtime and
the oracle's C source (compiled with the oracle's own flags)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
BIN = os.path.join(HERE, "roundtrip")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> str:
    sys.path.insert(0, ROOT)
    import oracle
    # the oracle's arithmetic flags (no contraction, IEEE rounding), not its
    # shared-library ones: this is an executable
    flags = [f for f in oracle.CFLAGS if f not in ("-shared", "-fPIC")]
    cmd = ["gcc", *flags, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "oracle"), "-I", os.path.join(ROCM, "include"),
           os.path.join(HERE, "roundtrip.c"), os.path.join(ROOT, "oracle", "vc_oracle.c"),
           "-L", os.path.join(ROOT, "paper_2505_07158_amd"), "-lvcipher",
           "-Wl,-rpath,$ORIGIN/../../paper_2505_07158_amd", "-L", os.path.join(ROCM, "lib"),
           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lamdhip64", "-lm", "-o", BIN + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(BIN + ".tmp", BIN)
    return BIN


if __name__ == "__main__":
    print(build())

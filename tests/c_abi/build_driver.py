"""Builds the plain-C test drivers of the library's C ABI (tests/c_abi/
roundtrip: encrypt_frames / decrypt_frames; tests/c_abi/serve: the serving
loop), each linked against paper_2505_07158_amd/libvcipher.so, the HIP
runtime and the oracle's C source (compiled with the oracle's own flags)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
DRIVERS = ("roundtrip", "serve")
BIN = os.path.join(HERE, "roundtrip")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_one(name: str) -> str:
    sys.path.insert(0, ROOT)
    import oracle
    # the oracle's arithmetic flags (no contraction, IEEE rounding), not its
    # shared-library ones: this is an executable
    flags = [f for f in oracle.CFLAGS if f not in ("-shared", "-fPIC")]
    out = os.path.join(HERE, name)
    cmd = ["gcc", *flags, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "oracle"), "-I", os.path.join(ROCM, "include"),
           os.path.join(HERE, name + ".c"), os.path.join(ROOT, "oracle", "vc_oracle.c"),
           "-L", os.path.join(ROOT, "paper_2505_07158_amd"), "-lvcipher",
           "-Wl,-rpath,$ORIGIN/../../paper_2505_07158_amd", "-L", os.path.join(ROCM, "lib"),
           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lamdhip64", "-lm", "-o", out + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build() -> str:
    """Builds every driver; returns the round-trip driver's path."""
    for name in DRIVERS:
        build_one(name)
    return BIN


if __name__ == "__main__":
    print(build())

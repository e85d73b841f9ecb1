"""Build of libtpcreco.so for gfx950 with hipcc (in-tree)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
         # packed FP32 instructions stay off: plain float code only
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(extra=None) -> str:
    out = os.path.join(HERE, "libtpcreco.so")
    src = os.path.join(HERE, "csrc", "tpc.hip")
    cmd = ["hipcc"] + FLAGS + list(extra or []) + ["-o", out + ".tmp", src]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())

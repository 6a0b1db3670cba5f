"""Build the reference oracle (test infrastructure) into oracle/liblbo.so.

The oracle is plain serial C++17 compiled with the host compiler; it shares
no source with the HIP library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblbo.so")


# AddressSanitizer and UndefinedBehaviorSanitizer, every UB report fatal; the
# library is then loaded into a process that preloads the runtimes
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined"]


def build(verbose: bool = False, out: str = LIB, sanitize: bool = False) -> str:
    flags = SANITIZE if sanitize else ["-O2"]
    cmd = ["g++", *flags, "-std=c++17", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", out + ".tmp", os.path.join(HERE, "lbo.cpp")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

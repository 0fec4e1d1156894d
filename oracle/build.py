"""Build the oracle's shared library with gcc (IEEE double, no contraction).

build() makes oracle/liboracle.so; build_sanitized() makes the same source
with AddressSanitizer and UndefinedBehaviorSanitizer into
_build/san/liboracle_san.so, which tests/test_sanitizers.py loads in a
subprocess (with the sanitizer runtimes preloaded) to run oracle workloads."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_FLAGS = ["-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra",
          "-Wno-unused-parameter"]
SAN_LIB = os.path.join(os.path.dirname(_HERE), "_build", "san", "liboracle_san.so")


def _gcc(out, extra, verbose):
    src = os.path.join(_HERE, "gmls_oracle.c")
    tmp = out + ".tmp"
    cmd = ["gcc"] + extra + _FLAGS + [src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    return _gcc(os.path.join(_HERE, "liboracle.so"), ["-O2"], verbose)


def build_sanitized(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(SAN_LIB), exist_ok=True)
    return _gcc(SAN_LIB, ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                          "-fno-sanitize-recover=undefined"], verbose)


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_sanitized(verbose=True))

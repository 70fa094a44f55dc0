"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

`build(sanitize=True)` builds the same source with AddressSanitizer and
UndefinedBehaviorSanitizer into oracle/liboracle_san.so instead; the tests
load it in a child process with the sanitizer runtimes preloaded (see
`sanitizer_env`) and `ORACLE_LIB` pointing at it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
LIB_SAN = os.path.join(HERE, "liboracle_san.so")

# -O3 -march=native: the CPU baseline times this build on the host it runs on.
# -ffp-contract=off keeps every multiply and add separately rounded, as written.
OPT = ["-O3", "-march=native"]
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SAN if sanitize else LIB
    cmd = (["g++"] + (SAN if sanitize else OPT) +
           ["-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
            "-o", out + ".tmp", SRC])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def sanitizer_env(base=None) -> dict:
    """Environment for a child Python process that loads liboracle_san.so."""
    env = dict(os.environ if base is None else base)
    rt = []
    for name in ("libasan.so", "libubsan.so"):
        p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True,
                           text=True, check=True).stdout.strip()
        rt.append(p)
    env["LD_PRELOAD"] = ":".join(rt + ([env["LD_PRELOAD"]] if env.get("LD_PRELOAD") else []))
    # the interpreter itself is not instrumented: its allocations are not leaks of ours
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1:exitcode=86"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=87"
    env["ORACLE_LIB"] = LIB_SAN
    return env


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)

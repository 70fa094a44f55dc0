"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

`build(sanitize=True)` builds the same source with AddressSanitizer and
UndefinedBehaviorSanitizer into oracle/liboracle_san.so instead; the tests
load it in a child process with the sanitizer runtimes preloaded (see
`sanitizer_env`) and `ORACLE_LIB` pointing at it.

`build_native()` builds it with -march=native for the host it runs on (the
CPU baseline times that build), into a file named for the host's CPU so a
build made on one machine is never loaded on another.
"""
import hashlib
import os
import platform
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
LIB_SAN = os.path.join(HERE, "liboracle_san.so")

# The checker build targets a baseline x86-64 so that it loads on any host the
# tests run on; the timed build adds -march=native on its own host.
# -ffp-contract=off keeps every multiply and add separately rounded, as written
# (so both builds give the same bits).
OPT = ["-O3", "-march=x86-64-v2"]
OPT_NATIVE = ["-O3", "-march=native"]
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]


def _cpu_tag() -> str:
    """Short fingerprint of this host's CPU model and instruction-set flags."""
    model, flags = platform.processor(), ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and not model:
                    model = line.split(":", 1)[1].strip()
                if line.startswith("flags"):
                    flags = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return hashlib.sha256((model + "|" + flags).encode()).hexdigest()[:12]


def native_lib_path() -> str:
    return os.path.join(HERE, f"liboracle_native_{_cpu_tag()}.so")


def build_native(verbose: bool = False) -> str:
    """-O3 -march=native build for this host (built once per CPU, then reused)."""
    out = native_lib_path()
    if not os.path.exists(out):
        _compile(OPT_NATIVE, out, verbose)
    return out


def _compile(flags, out, verbose):
    cmd = (["g++"] + flags +
           ["-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
            "-o", out + ".tmp", SRC])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False, sanitize: bool = False) -> str:
    return _compile(SAN if sanitize else OPT, LIB_SAN if sanitize else LIB, verbose)


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

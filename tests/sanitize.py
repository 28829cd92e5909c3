"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

    python tests/sanitize.py

Builds two libraries into a temporary directory:
- libnf with the sanitizers on its host code (-Xarch_host; its device code is
  built as usual and never run here);
- the oracle's C code with gcc's sanitizers.

Then runs, in child processes that preload the matching sanitizer runtimes:
- the CPU tests of the C ABI (tests/test_abi.py) against the first, which
  covers argument validation, the wavefront schedule's invariants, the tune
  file, and the serving engine's failure and shutdown-race paths;
- the oracle's pins (tests/test_oracle.py) against the second.

Any report stops the run (halt_on_error) and the script exits non-zero.
Leak checking is off: the interpreter itself holds memory until exit.
"""

import glob
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def build_nf(out: str) -> None:
    sys.path.insert(0, ROOT)
    from paper_1307_7820_amd import build as b
    flags = [f for f in b.FLAGS if f != "-O3"] + ["-O1", "-g"]
    flags += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.check_call([b.HIPCC, *flags, *[os.path.join(b.CSRC, s) for s in b.SOURCES], "-o", out])


def build_oracle(out: str) -> None:
    src = os.path.join(ROOT, "oracle", "nussinov.c")
    subprocess.check_call(["gcc", "-O1", "-g", "-march=x86-64-v3", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", out, src])


def clang_asan_runtime() -> str:
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise SystemExit("clang's ASan runtime was not found under /opt/rocm/llvm")
    return hits[-1]


def gcc_runtime(name: str) -> str:
    return subprocess.check_output(["gcc", "-print-file-name=" + name], text=True).strip()


def child(kind: str, lib: str) -> int:
    # runs inside the preloaded process: point the module at the sanitized
    # library before its first use, then run the CPU tests
    sys.path.insert(0, ROOT)
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import pytest
    if kind == "nf":
        from paper_1307_7820_amd import nf
        nf.load(lib)
        target = "test_abi.py"
    else:
        import oracle
        oracle._LIB = lib
        target = "test_oracle.py"
    return pytest.main([os.path.join(ROOT, "tests", target), "-q", "-m", "not gpu", "-p", "no:cacheprovider"])


def main() -> int:
    if len(sys.argv) == 4 and sys.argv[1] == "--child":
        return child(sys.argv[2], sys.argv[3])
    with tempfile.TemporaryDirectory() as tmp:
        nf_lib = os.path.join(tmp, "libnf_san.so")
        or_lib = os.path.join(tmp, "libnforacle_san.so")
        print("building", nf_lib, flush=True)
        build_nf(nf_lib)
        print("building", or_lib, flush=True)
        build_oracle(or_lib)
        runs = [("nf", nf_lib, clang_asan_runtime()),
                ("oracle", or_lib, gcc_runtime("libasan.so") + " " + gcc_runtime("libubsan.so"))]
        for kind, lib, preload in runs:
            env = dict(os.environ, LD_PRELOAD=preload, **SAN_ENV)
            print("running the %s tests under ASan + UBSan" % kind, flush=True)
            rc = subprocess.call([sys.executable, os.path.abspath(__file__), "--child", kind, lib], env=env)
            if rc != 0:
                print("%s: sanitized run failed (exit %d)" % (kind, rc), flush=True)
                return 1
    print("sanitized host runs clean", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

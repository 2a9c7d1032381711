"""The host runtime (planner, call drivers, engine host code) and the FP64 oracle built
under AddressSanitizer + UndefinedBehaviorSanitizer, with the host-side tests run
against those builds in child processes (each preloads its compiler's ASan runtime,
since the Python interpreter is not instrumented; reports abort the child).

Commands (the same ones these tests run):
  python -m paper_2104_02646_amd.build --sanitize <dir>      # host runtime, clang
  GSIM_LIB=<dir>/libgsim.so LD_PRELOAD=<clang libclang_rt.asan> \\
      python -m pytest tests/test_abi_host.py
  GSIM_ORACLE_LIB=<dir>/libgsim_oracle.so LD_PRELOAD=$(gcc -print-file-name=libasan.so) \\
      python -m pytest tests/test_oracle_*.py

A negative control first shows that each runtime, loaded this way, does catch a heap
overflow and a signed overflow in a library built with the same flags."""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
       "HIP_VISIBLE_DEVICES": "", "PYTHONDONTWRITEBYTECODE": "1"}

BUGGY = textwrap.dedent("""
    #include <climits>
    #include <cstdlib>
    extern "C" int heap_past_end(int n) {
        int* a = (int*)std::malloc(sizeof(int) * n);
        for (int i = 0; i < n; ++i) a[i] = i;
        int s = a[n];  /* one past the end */
        std::free(a);
        return s;
    }
    extern "C" int add_overflow(int a) { return a + INT_MAX; }
""")


def _gcc_asan():
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


def _child(code, preload, extra_env, timeout=900):
    env = dict(os.environ, **ENV, **extra_env, LD_PRELOAD=preload)
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=timeout)


@pytest.fixture(scope="module")
def san_dir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("san"))


def _control(lib, preload):
    for fn, arg, expect in (("heap_past_end", 8, "heap-buffer-overflow"),
                            ("add_overflow", 1, "signed integer overflow")):
        r = _child("import ctypes; print(ctypes.CDLL(%r).%s(%d))" % (lib, fn, arg), preload, {}, timeout=120)
        assert r.returncode != 0 and expect in r.stderr, (fn, r.returncode, r.stderr[-2000:])


def test_negative_controls(san_dir):
    from oracle.oracle import SAN_FLAGS
    from paper_2104_02646_amd import build as gbuild
    src = os.path.join(san_dir, "buggy.cpp")
    with open(src, "w") as f:
        f.write(BUGGY)
    g = os.path.join(san_dir, "libbuggy_gcc.so")
    subprocess.check_call(["g++", "-shared", "-fPIC", *SAN_FLAGS, src, "-o", g])
    _control(g, _gcc_asan())
    c = os.path.join(san_dir, "libbuggy_clang.so")
    host = [f for f in gbuild.SAN_HOST if f != "-Xarch_host"]
    subprocess.check_call([gbuild.CLANGXX, "-shared", "-fPIC", "-shared-libasan", *host, src, "-o", c])
    _control(c, gbuild.asan_runtime())


CHECK_LOADED = textwrap.dedent("""
    import ctypes, os, sys
    sys.path.insert(0, %(root)r)
    lib = os.environ[%(var)r]
    ctypes.CDLL(lib)
    maps = open("/proc/self/maps").read()
    assert lib in maps and "asan" in maps, "sanitizer build not loaded"
    assert hasattr(ctypes.CDLL(None), "__asan_init")
    import pytest
    sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + %(tests)r))
""")


def test_host_runtime_under_asan_ubsan(san_dir):
    from paper_2104_02646_amd import build as gbuild
    lib = gbuild.build_sanitized(os.path.join(san_dir, "gsim"))
    code = CHECK_LOADED % {"root": ROOT, "var": "GSIM_LIB", "tests": ["tests/test_abi_host.py"]}
    r = _child(code, gbuild.asan_runtime(), {"GSIM_LIB": lib})
    print(r.stdout[-1500:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_oracle_under_asan_ubsan(san_dir):
    import oracle.oracle as orc
    lib = orc.build_sanitized(os.path.join(san_dir, "oracle"))
    tests = sorted(os.path.relpath(p, ROOT) for p in glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    assert len(tests) >= 8
    code = CHECK_LOADED % {"root": ROOT, "var": "GSIM_ORACLE_LIB", "tests": tests}
    r = _child(code, _gcc_asan(), {"GSIM_ORACLE_LIB": lib})
    print(r.stdout[-1500:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr

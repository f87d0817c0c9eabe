"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only,
no GPU needed): the C oracle, built with gcc, runs every pin; libm3s's host
layer, built with hipcc with the sanitizers on its host pass only, runs every
argument-validation case of the C ABI (all of them return before any HIP call).
Each runs in a fresh Python process with the sanitizer runtime preloaded, and
any report fails the run."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(code, preload, timeout):
    env = dict(os.environ, LD_PRELOAD=preload, PYTHONPATH=os.pathsep.join([ROOT, os.path.join(ROOT, "tests")]),
               **SAN_ENV)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0 and "SANITIZED-OK" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r


def test_oracle_pins_under_asan_ubsan(tmp_path):
    import oracle
    lib = str(tmp_path / "liboracle_san.so")
    oracle.compile_oracle(out=lib, extra_flags=("-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                                                "-fno-sanitize-recover=undefined"))
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    code = ("import oracle, pins\n"
            "oracle._lib = oracle.load(%r)\n"
            "for pin in pins.ALL_PINS:\n"
            "    pin(oracle._lib)\n"
            "print('SANITIZED-OK', len(pins.ALL_PINS))\n" % lib)
    r = _run(code, libasan, 600)
    print(r.stdout.strip().splitlines()[-1])


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_capi_validation_under_asan_ubsan(tmp_path):
    rt = _clang_asan_runtime()
    if rt is None:
        pytest.skip("clang AddressSanitizer runtime not found")
    from paper_2412_12392_amd import build
    lib = str(tmp_path / "libm3s_san.so")
    build.build(out=lib, extra=("-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                                "-fno-omit-frame-pointer"))
    code = ("import ctypes, test_capi_host as T\n"
            "from paper_2412_12392_amd import _lib\n"
            "lib = _lib.load(%r)\n"
            "n = 0\n"
            "for name in dir(T):\n"
            "    f = getattr(T, name)\n"
            "    if not name.startswith('test_') or not callable(f):\n"
            "        continue\n"
            "    marks = getattr(f, 'pytestmark', [])\n"
            "    params = [m for m in marks if m.name == 'parametrize']\n"
            "    args = f.__code__.co_varnames[:f.__code__.co_argcount]\n"
            "    if 'tmp_path' in args:\n"
            "        continue\n"
            "    if params:\n"
            "        for vals in params[0].args[1]:\n"
            "            f(lib, *vals)\n"
            "            n += 1\n"
            "    elif args == ('lib',):\n"
            "        f(lib)\n"
            "        n += 1\n"
            "print('SANITIZED-OK', n)\n" % lib)
    r = _run(code, rt, 600)
    print(r.stdout.strip().splitlines()[-1])

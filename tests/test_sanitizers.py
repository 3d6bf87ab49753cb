"""Sanitizer builds on the CPU (no GPU is used):

- the host library (layouts, the threaded BVH builder, argument validation,
  and the serving dispatcher thread in its simulated mode, fed from two
  submitting threads, and its watchdog giving up a stalled simulated device
  while a thread submits) under AddressSanitizer + UndefinedBehaviorSanitizer,
  and under ThreadSanitizer, through tests/sanitize_host.cpp;
- the oracle (C, OpenMP) under AddressSanitizer + UndefinedBehaviorSanitizer,
  running its own pin tests in a child process.

The HIP kernel sources are compiled as usual (their device code is not
run); the sanitizers instrument host code only.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2503_23410_amd")
sys.path.insert(0, ROOT)

pytestmark = pytest.mark.slow

HOST_SOURCES = ("api.cpp", "layout.cpp", "bvh.cpp", "batch.cpp", "server.cpp", "noalloc.cpp")
KERNEL_SOURCES = ("trace.hip", "reconstruct.hip", "fxaa.hip", "reproject.hip")


def _have_toolchain():
    return shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    pytest.skip("clang++ not found")


def _compile_all(out_dir, host_flags):
    from paper_2503_23410_amd import build as B
    common = [B.hipcc()] + B.COMMON
    jobs = []
    for src in HOST_SOURCES:
        jobs.append(common + B.SOURCES[src] + host_flags + ["-g", "-c", os.path.join(B.CSRC, src), "-o",
                                                             os.path.join(out_dir, src + ".o")])
    for src in KERNEL_SOURCES:
        jobs.append(common + B.SOURCES[src] + ["-c", os.path.join(B.CSRC, src), "-o",
                                               os.path.join(out_dir, src + ".o")])
    jobs.append(common + ["-x", "hip", "-g"] + host_flags + ["-c", os.path.join(ROOT, "tests", "sanitize_host.cpp"),
                                                              "-o", os.path.join(out_dir, "driver.o")])

    def run(cmd):
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(" ".join(cmd) + "\n" + r.stderr)
        return cmd[-1]

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        return list(ex.map(run, jobs))


def _driver(tmp_path_factory, name, sanitize):
    if not _have_toolchain():
        pytest.skip("hipcc not found")
    d = str(tmp_path_factory.mktemp(name))
    host = []
    for s in sanitize.split(","):
        host += ["-Xarch_host", f"-fsanitize={s}"]
    host += ["-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    objs = _compile_all(d, host)
    exe = os.path.join(d, "sanitize_host")
    link = [_clang(), f"-fsanitize={sanitize}", "-o", exe] + objs + ["-L/opt/rocm/lib", "-lamdhip64", "-pthread",
                                                                    f"-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, what, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    env["HIP_VISIBLE_DEVICES"] = ""          # never touch a GPU, even where one exists
    r = subprocess.run([exe, what], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, f"{what}: exit {r.returncode}\n{r.stderr[-4000:]}"
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert "WARNING: ThreadSanitizer" not in r.stderr
    return r.stdout


@pytest.fixture(scope="module")
def asan_exe(tmp_path_factory):
    return _driver(tmp_path_factory, "asan", "address,undefined")


@pytest.fixture(scope="module")
def tsan_exe(tmp_path_factory):
    return _driver(tmp_path_factory, "tsan", "thread")


@pytest.mark.parametrize("what", ["layouts", "scenes", "serving", "stall"])
def test_host_library_under_asan_ubsan(asan_exe, what):
    out = _run(asan_exe, what, {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0",
                                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    assert "0 failed checks" in out


@pytest.mark.parametrize("what", ["scenes", "serving", "stall"])
def test_host_threads_under_tsan(tsan_exe, what):
    out = _run(tsan_exe, what, {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"})
    assert "0 failed checks" in out


def test_oracle_under_asan_ubsan(tmp_path):
    """The oracle's own pins, with the oracle built under ASan + UBSan."""
    import oracle
    lib = str(tmp_path / "liboracle_san.so")
    cmd = ["gcc", "-O1", "-g", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c11", "-D_DEFAULT_SOURCE",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", lib,
           oracle._SRC, "-lm"]
    subprocess.check_call(cmd)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, VAFR_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="4")
    tests = [os.path.join(ROOT, "tests", t) for t in ("test_oracle_mapping.py", "test_oracle_tracing.py",
                                                     "test_oracle_rep.py", "test_oracle_fxaa.py",
                                                     "test_oracle_lafr.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"] + tests,
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0
    assert "ERROR: AddressSanitizer" not in r.stderr + r.stdout and "runtime error" not in r.stderr + r.stdout

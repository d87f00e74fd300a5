"""Host AddressSanitizer + UndefinedBehaviorSanitizer runs (no GPU needed).

* The oracle library is rebuilt with gcc's sanitizers and the oracle's CPU tests are rerun
  against it in a child process (the sanitizer runtime preloaded, reports to log files; any
  report aborts the child).
* The C ABI library is rebuilt with its host code instrumented (device code as usual: the
  sanitizers are for the host side only) and its host-side argument checks, workspace
  queries and export table are exercised.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["test_oracle_kernel.py", "test_oracle_particles.py", "test_oracle_surrogate.py",
                "test_oracle_training.py"]


def _gcc_asan_runtime():
    if shutil.which("gcc") is None:
        return None
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _run_child(cmd, env_extra, logdir, timeout):
    logdir = os.path.join(logdir, "reports")
    os.makedirs(logdir, exist_ok=True)
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = f"detect_leaks=0:abort_on_error=0:log_path={logdir}/asan"
    env["UBSAN_OPTIONS"] = f"print_stacktrace=1:log_path={logdir}/ubsan"
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    reports = "".join(open(f).read() for f in sorted(glob.glob(os.path.join(logdir, "*"))))
    return r, reports


def test_oracle_under_asan_ubsan(tmp_path):
    rt = _gcc_asan_runtime()
    if rt is None:
        pytest.skip("gcc with libasan not available")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(
        ["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared", "-Wall",
         "-o", lib, os.path.join(ROOT, "oracle", "wk_oracle.c"), "-lm"])
    env = {"WK_ORACLE_LIB": lib, "LD_PRELOAD": rt + (":" + os.environ["LD_PRELOAD"] if os.environ.get("LD_PRELOAD") else "")}
    # the instrumented build is the one the child loads
    probe = ("import oracle, os; oracle._LIB = os.environ['WK_ORACLE_LIB']; oracle.lib(); "
             "print(sum('liboracle_san.so' in l for l in open('/proc/self/maps')) > 0)")
    r, rep = _run_child([sys.executable, "-c", probe], env, tmp_path, 120)
    assert r.returncode == 0 and r.stdout.strip() == "True", (r.stdout, r.stderr, rep)
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           *[os.path.join("tests", t) for t in ORACLE_TESTS]]
    r, rep = _run_child(cmd, env, tmp_path, 600)
    assert r.returncode == 0 and not rep, (r.stdout[-3000:], r.stderr[-3000:], rep[:6000])
    assert " passed" in r.stdout


HOST_ABI_CHILD = """
import sys
sys.path.insert(0, 'tests')
from paper_1806_00082_amd import _lib
_lib.LIB_PATH = sys.argv[1]
import test_abi
test_abi.test_header_declares_the_boundary()
test_abi.test_library_exports_every_declared_symbol()
test_abi.test_python_binding_names_match_header()
test_abi.test_host_validation_without_gpu()
test_abi.test_workspace_contracts_without_gpu()
test_abi.test_particle_calls_reject_aliased_buffers_without_gpu()
print('host checks passed', _lib.lib()._name)
"""


def test_abi_host_code_under_asan_ubsan(tmp_path):
    from paper_1806_00082_amd import build
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not os.path.exists(build.HIPCC) or not rts:
        pytest.skip("hipcc or its AddressSanitizer runtime not available")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-O1" if f == "-O3" else f for f in build.FLAGS] + ["-g0"] + san
    procs, objs = [], []
    for src in build.SOURCES:
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([build.HIPCC, *flags, "-c", os.path.join(build.CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out = p.communicate(timeout=600)[0]
        assert p.returncode == 0, out[-3000:]
    lib = str(tmp_path / "libwigner_san.so")
    subprocess.check_call([build.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-shared-libsan", "-o", lib, *objs])
    env = {"LD_PRELOAD": rts[-1] + (":" + os.environ["LD_PRELOAD"] if os.environ.get("LD_PRELOAD") else "")}
    r, rep = _run_child([sys.executable, "-c", HOST_ABI_CHILD, lib], env, tmp_path, 300)
    assert r.returncode == 0 and not rep, (r.stdout[-3000:], r.stderr[-3000:], rep[:6000])
    assert "host checks passed" in r.stdout and "libwigner_san.so" in r.stdout

"""Host logic of the library, and the C oracle, under AddressSanitizer and UBSan, without a GPU.

The library's sources are compiled host-only (no device code) with the sanitizers and linked
against tests/host_stub/hip_stub.cpp, a stand-in HIP runtime that keeps device memory in host
memory, range-checks every copy, validates and counts launches, tracks graph captures and
returns pseudo-random timings.  tests/host_stub/host_driver.cpp then drives every entry point:
invalid arguments, ragged batches with and without autotuning for every p and mode, searches
split into candidate chunks by a workspace bound, and the allocation-free entry point (no
allocation; an oversized search refused before any launch).  Kernels do not run: this checks
the planning, workspace layout, chunking, tuning and bookkeeping code around them."""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not (shutil.which(HIPCC) and os.path.exists(CLANG) and shutil.which("g++")):
        pytest.skip("hipcc, clang++ or g++ not available")
    out = str(tmp_path_factory.mktemp("host_stub"))
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_0811_3301_amd", "csrc")]
    host_san = [f for s in SAN for f in ("-Xarch_host", s)]
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_0811_3301_amd", "csrc", "*.hip")))
    objs = [os.path.join(out, os.path.basename(s) + ".o") for s in srcs]
    cmds = [[HIPCC, "--offload-arch=gfx950", "--offload-host-only", "-O1", "-g", "-std=c++17", "-fPIC", *host_san, *inc,
             "-c", s, "-o", o] for s, o in zip(srcs, objs)]
    with ThreadPoolExecutor(min(8, os.cpu_count() or 4)) as pool:
        list(pool.map(lambda c: _run(c, out), cmds))
    # host-only objects refer to a per-file device-code symbol that no device pass defines
    syms = set()
    for o in objs:
        for line in _run(["nm", "-u", o], out).stdout.splitlines():
            name = line.split()[-1]
            if name.startswith("__hip_fatbin"):
                syms.add(name)
    with open(os.path.join(out, "fatbins.c"), "w") as f:
        f.writelines(f"char {s}[16];\n" for s in sorted(syms))
    _run(["gcc", "-c", "fatbins.c", "-o", "fatbins.o"], out)
    here = os.path.join(ROOT, "tests", "host_stub")
    rt = ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", *inc]
    for name in ("hip_stub", "host_driver"):
        _run(["g++", "-O1", "-g", "-std=c++17", *SAN, *rt, "-c", os.path.join(here, name + ".cpp"), "-o", name + ".o"],
             out)
    exe = os.path.join(out, "host_driver")
    _run([CLANG, *SAN, "-o", exe, "host_driver.o", "hip_stub.o", "fatbins.o", *objs], out)
    return exe


def test_host_logic_under_sanitizers(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, f"rc={r.returncode}\n{r.stdout[-4000:]}\n{r.stderr[-8000:]}"
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]


def test_oracle_c_under_sanitizers(tmp_path):
    """The C oracle (test infrastructure) built with AddressSanitizer and UBSan and driven over
    edge shapes by tests/host_stub/oracle_driver.c."""
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", *SAN, "-o", exe,
          os.path.join(ROOT, "tests", "host_stub", "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"],
         str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, f"rc={r.returncode}\n{r.stdout[-4000:]}\n{r.stderr[-8000:]}"
    assert "all checks passed" in r.stdout

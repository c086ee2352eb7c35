"""Kernels run on the host through an emulation of the HIP device API
(tests/hipemu), compiled with g++ and AddressSanitizer: every access of the
kernel source is bounds-checked and the results are compared with plain
host computations (a sort by (depth, position); exclusive scans and
compaction).  No GPU is involved."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_16422_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "hipemu")


def host_source(name: str) -> str:
    """Kernel source with each `extern __shared__` array bound to the launch's
    dynamic shared memory buffer."""
    src = open(os.path.join(CSRC, name)).read()
    return re.sub(r"extern __shared__ (\w+) (\w+)\[\];", r"\1 *\2 = (\1 *)g_dyn_lds;", src)


def run_on_host(tmp_path, kernel_file: str, check: str, *args: str):
    inc = os.path.splitext(kernel_file)[0] + "_host.inc"
    (tmp_path / inc).write_text(host_source(kernel_file))
    exe = str(tmp_path / os.path.splitext(check)[0])
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address", "-I", str(tmp_path), "-I", EMU, "-I", CSRC,
           "-I", os.path.join(ROOT, "include"), os.path.join(EMU, check), "-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_bucket_depth_order_kernels_on_host(tmp_path):
    run_on_host(tmp_path, "k_bucket.hip", "bucket_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scans_on_host(tmp_path):
    run_on_host(tmp_path, "k_scan.hip", "scan_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tile_binning_kernels_on_host(tmp_path):
    """Emission, stable tile sort and ranges at an exact capacity; with
    FDGS_HOST_EMU_FULL=1 also above 2^20 instances, where the emission writes
    the sort's first-digit histogram (several minutes in the emulation)."""
    run_on_host(tmp_path, "k_sort.hip", "sort_check.cpp", *(["full"] if os.environ.get("FDGS_HOST_EMU_FULL") else []))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_xcd_block_order_is_a_bijection(tmp_path):
    run_on_host(tmp_path, "k_sort.hip", "xcd_check.cpp")

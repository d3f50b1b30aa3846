"""The kernels' address maps audited on the CPU (no GPU): a host driver
(tests/audit/addr_audit.cpp) is compiled against the very header the
kernels take their address functions from (paper_2609_06449_amd/csrc/addr.h)
and enumerates every load and store of every workgroup, thread and item of
the symmetric split form, the split form of Phase I (N1 = 2^12, 2^13, 2^14;
several N2 and bases, mixed radix included; the 2^28 shapes the benchmark
times in the full run), the digit maps, the XCD tile order and the LDS
exchange buffers of the MFMA passes: every index inside its buffer, every
output written once, in-place passes reading and writing the same items per
workgroup, no 32-bit wrap; every exchange-buffer load reading the slot its
item was stored to, with no two lanes of a store half-wave or a load wave
on one bank."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "audit", "addr_audit.cpp")
CSRC = os.path.join(ROOT, "paper_2609_06449_amd", "csrc")


def _compiler():
    for cc in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if cc and os.path.exists(cc):
            return cc
    return None


@pytest.fixture(scope="module")
def audit_exe(tmp_path_factory):
    cc = _compiler()
    if cc is None:
        pytest.skip("clang++ not available")
    exe = str(tmp_path_factory.mktemp("audit") / "addr_audit")
    r = subprocess.run([cc, "-O2", "-std=c++17", "-Wall", "-I", CSRC, SRC, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_address_maps(audit_exe):
    r = subprocess.run([audit_exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "address audit passed" in r.stdout


def test_address_maps_2p28_shapes(audit_exe):
    r = subprocess.run([audit_exe, "full"], capture_output=True, text=True, timeout=900)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok split form 8192 x 32768" in r.stdout and "ok split form 16384 x 16384" in r.stdout

"""The public header compiles as C99 and a C program links and calls the
library (device-free entry points only)."""

import os
import shutil
import subprocess
import tempfile

import pytest

from paper_1604_02334_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_c99_consumer_builds_and_runs():
    libdir = os.path.dirname(A.LIB_PATH)
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "consumer")
        cmd = ["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
               os.path.join(ROOT, "tests", "c_consumer.c"), "-o", exe, "-L", libdir, "-lmu",
               f"-Wl,-rpath,{libdir}", "-Wl,-rpath,/opt/rocm/lib"]
        # the library is named libmu.so in the package directory
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        env = dict(os.environ, MU_FORCE_NODEVICE="1",
                   LD_LIBRARY_PATH="/opt/rocm/lib:" + os.environ.get("LD_LIBRARY_PATH", ""))
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
        assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
        assert "c consumer ok" in r.stdout

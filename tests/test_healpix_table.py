"""On the CPU: the HEALPix direction table that nrt_init_grid builds on the
host (healpix.h's geometry and the C library's sincos) equals the oracle's
pixel centres bit for bit, so both FP64 paths and the oracle take their
decisions on the same directions.  The GPU test reads the table a context
actually holds."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_direction_table_equals_oracle(tmp_path, orc):
    exe = str(tmp_path / "hp_check")
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "-O3", "-ffp-contract=off",
           "-I" + os.path.join(ROOT, "paper_2512_12466_amd", "csrc"),
           os.path.join(ROOT, "tests", "healpix_table_check.cpp"), "-o", exe,
           "-L" + os.path.join(ROOT, "oracle"), "-l:liboracle.so",
           "-Wl,-rpath," + os.path.join(ROOT, "oracle")]
    if not os.path.exists(cmd[0]):
        pytest.skip("no hipcc")
    subprocess.run(cmd, check=True, capture_output=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert p.returncode == 0 and "mismatches 0 of" in p.stdout, p.stdout + p.stderr

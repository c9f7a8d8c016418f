"""Constant-time evidence for the secret-dependent kernels (the constant-time
extended gcd that Section 3.1 relies on, the samplers and the products):
under rocprofv3 --pmc, every kernel dispatch of ct_probe.py issues exactly the
same number of vector, scalar, LDS, matrix-core and scalar-memory
instructions for three different secret inputs of the same shape.  (Which g
draws are rejected in KeyGen depends on g, as in the paper's KeyGen; the
reciprocals, products and samplers themselves do not.)"""
import csv
import os
import shutil
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_MFMA", "SQ_INSTS_SMEM")


def counter_rows(directory):
    for root, _, files in os.walk(directory):
        for f in files:
            if f.endswith("counter_collection.csv"):
                with open(os.path.join(root, f)) as fh:
                    yield from csv.DictReader(fh)


def test_secret_independent_instruction_counts(tmp_path):
    rocprof = shutil.which("rocprofv3") or "/opt/rocm/bin/rocprofv3"
    if not os.path.exists(rocprof):
        pytest.skip("rocprofv3 not available")
    env = dict(os.environ, TMPDIR=str(tmp_path))
    cmd = [rocprof, "--pmc", *COUNTERS, "--output-format", "csv", "-d", str(tmp_path / "ct"), "-o", "ct", "--",
           sys.executable, os.path.join(HERE, "ct_probe.py")]
    out = subprocess.run(cmd, cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=240)
    assert "kem encap and decap" in out.stdout, out.stdout[-2000:] + out.stderr[-2000:]
    per = {}
    for row in counter_rows(str(tmp_path / "ct")):
        if not row["Kernel_Name"].startswith(("ntrup::", "void ntrup::")):
            continue
        key = (int(row["Dispatch_Id"]), row["Kernel_Name"])
        per.setdefault(key, {})[row["Counter_Name"]] = float(row["Counter_Value"])
    by_kernel = {}
    for (did, name), c in sorted(per.items()):
        by_kernel.setdefault(name, []).append(tuple(c.get(k, -1.0) for k in COUNTERS))
    assert any("r3_kernel" in k for k in by_kernel) and any("recip_q_kernel" in k for k in by_kernel)
    assert any("sample_short_kernel" in k for k in by_kernel) and any("mulm_kernel" in k for k in by_kernel)
    assert any("kem_encap_kernel" in k for k in by_kernel) and any("kem_decap_kernel" in k for k in by_kernel)
    for name, seq in by_kernel.items():
        # each operation ran on three secret inputs in a row: dispatches of one
        # kernel come in runs of three with identical counts
        assert len(seq) % 3 == 0, (name, len(seq))
        for i in range(0, len(seq), 3):
            assert seq[i] == seq[i + 1] == seq[i + 2], (name, i, seq[i:i + 3])

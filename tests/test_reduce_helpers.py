"""Exhaustive host check of the exact int32 reduction helpers that every
kernel uses (reduce_rough, freeze, mul24, mac_chunk in
paper_2106_08759_amd/csrc/ntrup_params.h): all int32 inputs for the four
moduli q of Section 2.1 (plus sntrup1277's 7879), every pair of rough
residues through the 24-bit multiply, and the tightness of the int32
accumulation bound.  The header's host path is compiled with g++ and OpenMP
(reduce_check.cpp); about 10 s on 8 cores."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_reduction_helpers_exhaustive(tmp_path):
    exe = str(tmp_path / "reduce_check")
    subprocess.check_call(["g++", "-O2", "-fopenmp", "-std=c++17", os.path.join(HERE, "reduce_check.cpp"),
                           "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    lines = out.stdout.strip().splitlines()
    assert len(lines) == 4 and all(" ok " in ln for ln in lines), out.stdout

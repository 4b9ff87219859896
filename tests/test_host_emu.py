"""Host runs of the kernels' own arithmetic against independent references.

The NTT rounds, the basis-conversion epilogues and the modular helpers are
__host__ __device__ code; the programs under tests/emu compile those headers
for the CPU with g++ and compare them with the oracle's textbook NTT or with
plain 128-bit integer arithmetic.  They check the index maps of every kernel
shape, the FP64 exactness bounds (largest |value| / q, integrality), the
factored pass-2 twiddles, both basis-conversion epilogues, the FP64 key inner
product and the tile property of the automorphism.  No GPU is involved.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emu")
CXX = shutil.which("g++")
CC = shutil.which("gcc")

pytestmark = pytest.mark.skipif(CXX is None or CC is None, reason="needs g++ and gcc")


@pytest.fixture(scope="module")
def build_dir(tmp_path_factory):
    d = tmp_path_factory.mktemp("emu")
    # the oracle's C routines provide the reference transform
    subprocess.run([CC, "-O2", "-ffp-contract=off", "-c", os.path.join(ROOT, "oracle", "oracle.c"), "-o",
                    str(d / "oracle.o")], check=True)
    return d


def run_emu(build_dir, name, with_oracle=False):
    exe = str(build_dir / name)
    cmd = [CXX, "-O2", "-std=c++17", "-ffp-contract=off", os.path.join(EMU, name + ".cpp")]
    if with_oracle:
        cmd += [str(build_dir / "oracle.o"), "-lm"]
    subprocess.run(cmd + ["-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900)
    print(r.stdout)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr
    return r.stdout


def test_ntt_rounds_every_shape(build_dir):
    out = run_emu(build_dir, "ntt_rounds_emu", with_oracle=True)
    assert "0 with mismatches" in out


def test_bconv_epilogues(build_dir):
    out = run_emu(build_dir, "bconv_emu")
    assert " 0 mismatches" in out


def test_fp64_key_inner_product(build_dir):
    out = run_emu(build_dir, "ip_f64_emu")
    assert " 0 mismatches" in out


def test_automorphism_maps_tiles_to_tiles(build_dir):
    out = run_emu(build_dir, "automorph_blocks")
    assert ", 0 outside" in out

"""The contraction's and the adjoint's work decompositions on the host: small C++ checkers are
built against geometry.cpp and run for several configurations (every selected
triangle maps to exactly one accumulator element that decodes back to it, its
shells are staged by its work group, and the vector-kernel tiles cover it)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2107_14564_amd", "csrc")

CASES = [
    ("512", "100", "1500", "1", "0"),        # all closable triangles of 100 shells
    ("256", "40", "1000", "2", "2", *[str(k) for k in range(2, 41, 2)]),   # (mu, t) grid selection
    ("256", "30", "1000", "1", "1", "29", "30"),
    ("32", "10", "300", "1", "0"),
    ("64", "20", "100", "1", "0"),
    ("48", "9", "200", "1.5", "0"),
    ("16", "1", "100", "1", "0"),            # one shell, one triangle
    ("1024", "128", "1000", "1", "1", "128", "100", "64"),   # the split-bf16 maximum of 128 shells
]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("tiling") / "tiling_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(ROOT, "tests", "host", "tiling_check.cpp"), os.path.join(CSRC, "geometry.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


@pytest.mark.parametrize("args", CASES, ids=lambda a: "_".join(a[:5]))
def test_tiling_covers_every_triangle_once(checker, args):
    r = subprocess.run([checker, *args], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


@pytest.fixture(scope="module")
def adjoint_checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("adjoint") / "adjoint_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(ROOT, "tests", "host", "adjoint_check.cpp"), os.path.join(CSRC, "geometry.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


@pytest.mark.parametrize("args", CASES[:7], ids=lambda a: "_".join(a[:5]))
def test_adjoint_tables_rebuild_the_adjoint_fields(adjoint_checker, args):
    """The matrix-core adjoint's row blocks and weight slots, read the way the
    kernel reads them, give G_n = sum_t c_t d(F_a1 F_a2 F_a3)/dF_n exactly (random
    weights and field values, every grid class); every shell in one wavefront."""
    r = subprocess.run([adjoint_checker, *args], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


QUAD_CASES = [("48", "10", "200", "1", "0"), ("128", "30", "600", "1", "0"), ("16", "3", "100", "1", "0"),
              ("64", "10", "300", "1.5", "1", "10", "9"), ("16", "1", "100", "1", "0")]


@pytest.fixture(scope="module")
def quad_checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("quad") / "quad_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(ROOT, "tests", "host", "quad_check.cpp"), os.path.join(CSRC, "geometry.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


@pytest.mark.parametrize("args", QUAD_CASES, ids=lambda a: "_".join(a[:5]))
def test_quad_tiling_decodes_every_bin(quad_checker, args):
    """The order-4 pair tiling: each quadruple in one accumulator element that
    decodes back to its two pairs; wavefronts hold at most 16 tiles."""
    r = subprocess.run([quad_checker, *args], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr

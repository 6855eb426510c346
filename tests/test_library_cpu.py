"""CPU-only checks of the library: it builds, loads, exports every entry point
the C header declares, and its host planner produces plans whose every
device access stays in bounds (replayed on the CPU)."""
import os
import re
import subprocess

import numpy as np
import pytest

from workloads import generators as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsq2l.h")


def _lib():
    import paper_2107_09006_amd as L
    from paper_2107_09006_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2107_09006_amd import build
        build.build()
    return L, L.load_library()


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    text = open(HEADER).read()
    declared = sorted(set(re.findall(r"\b(lsq2l_[a-z_]+)\s*\(", text)))
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(L.EXPORTS) == declared


def test_default_options():
    L, lib = _lib()
    o = L.default_options()
    assert o.tol == 1e-8 and o.max_it == 10000 and o.precision == L.FP64
    assert o.variant == L.ADDITIVE and o.nev_max == 0 and o.check_every == 1 and o.use_graph == 0


@pytest.fixture(scope="module")
def plan_check(tmp_path_factory):
    d = tmp_path_factory.mktemp("plan")
    exe = str(d / "plan_check")
    cmd = ["hipcc", "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
           os.path.join(ROOT, "tests", "host", "plan_check.cpp"),
           os.path.join(ROOT, "paper_2107_09006_amd", "csrc", "plan.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe, d


CASES = {
    "worked": lambda: [W.worked_example()],
    "banded_1000": lambda: [W.banded_1000()],
    "grid_small": lambda: [W.small_config("grid")],
    "irregular_small": lambda: [W.small_config("irregular")],
    "single_part": lambda: [W.random_banded(200, 400, 1, seed=3)],
    "many_parts": lambda: [W.random_banded(480, 960, 32, seed=232)],
    "wide_interfaces": lambda: [W.random_banded(1600, 4800, 4, seed=77, tau=0.3, half_width=160)],
    "batch": lambda: [W.random_banded(300 + 50 * k, 600 + 100 * k, 3 + k, seed=k) for k in range(4)],
    "grid_500": lambda: [W.grid_500()],
    "grid_1000": lambda: [W.grid_1000()],
    # rows starting at unrelated columns, 65,536 rows: the row-sorted iteration copy
    "irregular_16k": lambda: [W.irregular_clustered(16384, 49152, 16, seed=21, tau=0.05, tol=1e-8,
                                                    name="irregular_16k")],
}


@pytest.mark.parametrize("name", list(CASES))
def test_host_plan_accesses_in_bounds(plan_check, name):
    from tests._dump import dump_problems
    exe, d = plan_check
    path = str(d / f"{name}.bin")
    dump_problems(CASES[name](), path)
    r = subprocess.run([exe, path], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr + r.stdout
    assert r.stdout.splitlines()[-1].startswith("OK")
    assert "solve layout (global)" in r.stdout and "solve layout (split)" in r.stdout
    if name == "irregular_16k":
        assert "row order: permuted" in r.stdout


@pytest.fixture(scope="module")
def qr_replay(tmp_path_factory):
    d = tmp_path_factory.mktemp("qr")
    exe = str(d / "qr_replay")
    cmd = ["hipcc", "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
           os.path.join(ROOT, "tests", "host", "qr_replay.cpp"),
           os.path.join(ROOT, "paper_2107_09006_amd", "csrc", "plan.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe, d


QR_CASES = ["worked", "banded_1000", "grid_small", "irregular_small", "many_parts",
            "wide_interfaces", "batch", "irregular_16k"]


@pytest.mark.parametrize("name", QR_CASES)
def test_host_qr_factors(qr_replay, name):
    """The QR local factors (Remarks 3.1, 3.2) replayed on the host with the
    kernel's blocks, tile order, envelope lists and strip layout: every access
    in bounds, the envelope property the kernel relies on, and L L^T = S C_ii S
    (both solve orders), the selection's L_I / L_GI and R_G^T R_G = S Ct_GG S
    against the formed matrices."""
    from tests._dump import dump_problems
    exe, d = qr_replay
    path = str(d / f"{name}.bin")
    dump_problems(CASES[name](), path, values=True)
    # the 16k irregular problem has subdomains of 1,500-1,800 positions: its
    # rows leave rounding residue small enough to underflow when squared
    args = [exe, path] + (["2000"] if name == "irregular_16k" else [])
    r = subprocess.run(args, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr + r.stdout
    last = r.stdout.splitlines()[-1]
    assert last.startswith("OK") and " 0 checked" not in last

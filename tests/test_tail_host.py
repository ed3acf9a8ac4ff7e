"""The single-workgroup coarse tail's device code run on the CPU (no GPU): the library's
kernel source is compiled for the host with the shim of tests/tail_host (one host thread
per work-item of the 1024-thread workgroup, emulated barriers and wave shuffles), under
AddressSanitizer with every buffer a separate heap allocation of the size the library
allocates, on the case whose first GPU run faulted (2D 129^2 random medium, 5 levels, the
tail on levels 1-3, FP64).  It must stay in bounds and give the oracle's V-cycle from
level 1 (GMRES relaxation with l+2 steps on every level, exact coarsest solve)."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from oracle import multigrid as omg
from oracle import solve as osolve
from paper_1712_06091_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1712_06091_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "tail_host")
CLANG = "/opt/rocm/llvm/bin/clang++"
# 2D coarse stencil offsets in the kernels' order (dy-major, then dx; at most one |d| = 2).
OFFS = [(x, y) for y in range(-2, 3) for x in range(-2, 3) if (abs(x) == 2) + (abs(y) == 2) <= 1]


def _host_sources(dst):
    for f in ("adr_common.hpp", "adr_fine.hpp", "adr_kernels.hpp", "adr_kernels.hip"):
        s = open(os.path.join(CSRC, f)).read()
        s = s.replace("#include <hip/hip_runtime.h>", '#include "shim.hpp"')
        s = re.sub(r"__attribute__\(\(amdgpu_waves_per_eu\([0-9, ]*\)\)\)", "", s)
        name = "adr_kernels_host.cpp" if f.endswith(".hip") else f
        with open(os.path.join(dst, name), "w") as fh:
            fh.write(s)
    for f in ("shim.hpp", "driver.cpp"):
        shutil.copy(os.path.join(HERE, f), dst)


def _case(dst):
    """Levels 1..4 of the 5-level hierarchy: SoA planes, inverse diagonals, the coarsest
    inverse, a right-hand side on level 1 and the oracle's V-cycle of it."""
    wl = W.random_medium(129, 2, seed=21)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy(5)
    case = os.path.join(dst, "case")
    os.makedirs(case)
    meta = []
    for l in range(1, 5):
        A = hier.A[l].tocsr()
        ny, nx = hier.shapes[l]
        N = nx * ny
        planes = np.zeros((len(OFFS), N), dtype=np.complex128)
        iy, ix = np.divmod(np.arange(N), nx)
        for k, (dx, dy) in enumerate(OFFS):
            jx, jy = ix + dx, iy + dy
            ok = (jx >= 0) & (jx < nx) & (jy >= 0) & (jy < ny)
            rows = np.nonzero(ok)[0]
            planes[k, rows] = np.asarray(A[rows, jy[ok] * nx + jx[ok]]).ravel()
        planes.tofile(os.path.join(case, f"planes{l}.bin"))
        (1.0 / A.diagonal()).astype(np.complex128).tofile(os.path.join(case, f"dinv{l}.bin"))
        meta.append((nx, ny, N, l + 2))
    np.linalg.inv(hier.A[4].toarray()).astype(np.complex128).tofile(os.path.join(case, "ainv.bin"))
    rng = np.random.default_rng(41)
    b1 = (rng.standard_normal(meta[0][2]) + 1j * rng.standard_normal(meta[0][2])).astype(np.complex128)
    b1.tofile(os.path.join(case, "b1.bin"))
    sub = omg.Hierarchy(hier.A[1], hier.shapes[1], 4, nu=[3, 4, 5, 6], smoothers=["gmres"] * 4)
    sub.vcycle(b1).astype(np.complex128).tofile(os.path.join(case, "ref1.bin"))
    with open(os.path.join(case, "meta.txt"), "w") as fh:
        for m in meta:
            fh.write(" ".join(map(str, m)) + "\n")
    return case


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ of the ROCm toolchain not found")
def test_coarse_tail_device_code_on_cpu(tmp_path):
    dst = str(tmp_path)
    _host_sources(dst)
    case = _case(dst)
    cc = subprocess.run([CLANG, "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
                         "-pthread", "driver.cpp", "-o", "driver"], cwd=dst, capture_output=True, text=True,
                        timeout=600)
    assert cc.returncode == 0, cc.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    run = subprocess.run(["./driver", case], cwd=dst, capture_output=True, text=True, timeout=600, env=env)
    assert run.returncode == 0 and "AddressSanitizer" not in run.stderr, run.stderr[-3000:]
    rel = float(re.search(r"rel_l2 (\S+)", run.stdout).group(1))
    assert rel <= 1e-12, rel

"""The node storage order (Layout in csrc/lbm_device.h) on the CPU: the host
side of the same header, compiled here with hipcc, maps every node of small
lattices; the row layout must be the natural order and the brick layout a
bijection whose aligned groups of 16, 64 and 4096 storage indices are 4x4x1
patches, 4^3 bricks and 16^3 blocks (what the storage sectors, the step's
waves and the population blocks rely on)."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_09242_amd", "csrc")

PROBE = r'''
#include <cstdio>
#include <cstdlib>
#include "lbm_device.h"
int main(int argc, char **argv) {
    const int brick = atoi(argv[1]), nx = atoi(argv[2]), ny = atoi(argv[3]), nz = atoi(argv[4]);
    const lbmd::Layout L = lbmd::make_layout(brick, nx, ny);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) printf("%d\n", L.at(x, y, z));
    return 0;
}
'''


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    d = tmp_path_factory.mktemp("layout")
    src, exe = d / "probe.hip", d / "probe"
    src.write_text(PROBE)
    r = subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-std=c++20", "-I" + CSRC,
                        "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return str(exe)


def _map(exe, brick, nx, ny, nz):
    out = subprocess.run([exe, str(brick), str(nx), str(ny), str(nz)], capture_output=True, text=True, check=True)
    return np.array(out.stdout.split(), dtype=np.int64).reshape(nz, ny, nx)


def test_row_layout_is_natural_order(probe):
    s = _map(probe, 0, 7, 5, 3)
    assert np.array_equal(s.ravel(), np.arange(7 * 5 * 3))


@pytest.mark.parametrize("nx,ny,nz", [(16, 16, 16), (32, 48, 16), (48, 16, 32)])
def test_brick_layout_structure(probe, nx, ny, nz):
    s = _map(probe, 1, nx, ny, nz)
    n = nx * ny * nz
    assert np.array_equal(np.sort(s.ravel()), np.arange(n)), "not a bijection onto [0, N)"
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inv = np.empty((n, 3), dtype=np.int64)
    inv[s.ravel()] = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    for size, ext in ((16, (4, 4, 1)), (64, (4, 4, 4)), (4096, (16, 16, 16))):
        g = inv.reshape(n // size, size, 3)
        lo, hi = g.min(axis=1), g.max(axis=1)
        assert np.all(hi - lo + 1 == np.array(ext)), f"groups of {size} are not {ext} boxes"
        assert np.all(lo % np.array(ext) == 0), f"groups of {size} are not aligned"
    # inside a brick x runs fastest, then y, then z
    b = inv[:64]
    assert np.array_equal(b[:4, 0], np.arange(4)) and np.all(b[:4, 1:] == 0)
    assert np.array_equal(b[::4, 1][:4], np.arange(4)) and np.array_equal(b[::16, 2], np.arange(4))

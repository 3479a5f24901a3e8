"""Host-side decomposition lists (lb_lists.hpp) against their definition.

The coupled step (Sec. 2.2) evolves the rows of each tile in one of two
velocity sets; the partner set's radius-2 stencil reads a node through the
Hermite projection when the node lies within two nodes, along x or y, of a
node of that set (no node beyond a wall, the wrapped node across a periodic
boundary).  The library builds these lists from candidate rows near band
edges; here they are compared with a brute-force scan of every node on
random decompositions, and the per-step image/pressure list with its plain
definition.  The driver is compiled with g++ from the header alone.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
XBC_PERIODIC, XBC_PRESSURE = 0, 1
YBC_WALLS, YBC_PERIODIC = 0, 1
IF_HERMITE, IF_PAPER = 0, 1
LOW, HIGH, IFACE = 0, 1, 2


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("lists") / "lists_driver")
    subprocess.run([gxx, "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "lists_driver.cpp")], check=True)
    return exe


def run(driver, cases):
    text = ""
    for c in cases:
        text += " ".join(str(v) for v in (c["nx"], c["ny"], c["xbc"], c["ybc"], c["iface"], c["tw"]))
        text += " " + " ".join(str(v) for v in list(c["lo"]) + list(c["hi"])) + "\n"
    out = subprocess.run([driver], input=text, capture_output=True, text=True, check=True).stdout.splitlines()
    res = []
    for line in out:
        v = [int(x) for x in line.split()]
        nf, n0, n1 = v[:3]
        fin = v[3:3 + 4 * nf]
        proj = v[3 + 4 * nf:]
        assert len(proj) == 2 * (n0 + n1)
        res.append((fin, proj, n0, n1))
    assert len(res) == len(cases)
    return res


def regions(c):
    nx, ny = c["nx"], c["ny"]
    R = np.zeros((ny + 1, nx), np.int64)
    for i in range(nx):
        t = i // c["tw"] if c["tw"] > 0 else 0
        lo, hi = c["lo"][t], c["hi"][t]
        for j in range(ny + 1):
            if j < lo or j > ny - hi:
                R[j, i] = HIGH
            elif c["iface"] == IF_PAPER and ((lo > 0 and j == lo) or (hi > 0 and j == ny - hi)):
                R[j, i] = IFACE
            else:
                R[j, i] = LOW
    return R


def brute(c):
    nx, ny = c["nx"], c["ny"]
    nrow = ny + 1
    R = regions(c)
    fin, low, high = [], [], []
    for j in range(nrow):
        for i in range(nx):
            r = R[j, i]
            if r == IFACE:
                continue
            image = c["ybc"] == YBC_PERIODIC and (j < 2 or j >= nrow - 2)
            press = c["xbc"] == XBC_PRESSURE and i in (0, nx - 1)
            if image or press:
                fin += [i, j, int(r == HIGH), 0]
            if c["iface"] != IF_HERMITE:
                continue
            other = LOW if r == HIGH else HIGH
            src = False
            for d in (-2, -1, 1, 2):
                jj, ii = j + d, i + d
                if not 0 <= jj < nrow:
                    jj = jj % nrow if c["ybc"] == YBC_PERIODIC else None
                if not 0 <= ii < nx:
                    ii = ii % nx if c["xbc"] == XBC_PERIODIC else None
                if (jj is not None and R[jj, i] == other) or (ii is not None and R[j, ii] == other):
                    src = True
            if src:
                (high if r == HIGH else low).extend([i, j])
    return fin, low + high, len(low) // 2, len(high) // 2


def random_cases(seed, n):
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(n):
        nx, ny = int(rng.integers(1, 41)), int(rng.integers(2, 41))
        tw = int(rng.integers(0, 11))
        nt = (nx + tw - 1) // tw if tw > 0 else 1
        iface = int(rng.integers(0, 2))
        ybc = int(rng.integers(0, 2))
        bmin = int(rng.integers(0, 3))
        bmax = bmin + int(rng.integers(0, ny // 2 + 1))
        lo = rng.integers(bmin, bmax + 1, nt)
        hi = rng.integers(bmin, bmax + 1, nt)
        if iface == IF_PAPER:   # the interpolation interface takes one band pair for every tile
            lo[:], hi[:] = lo[0], hi[0]
        if ybc == YBC_PERIODIC and rng.integers(0, 2):
            lo[:], hi[:] = 0, 0
        cases.append(dict(nx=nx, ny=ny, xbc=int(rng.integers(0, 2)), ybc=ybc, iface=iface, tw=tw,
                          lo=[int(v) for v in lo], hi=[int(v) for v in hi]))
    return cases


def test_lists_match_definition_on_random_decompositions(driver):
    cases = random_cases(2024, 300)
    for c, (fin, proj, n0, n1) in zip(cases, run(driver, cases)):
        bf, bp, b0, b1 = brute(c)
        assert fin == bf, c
        assert (proj, n0, n1) == (bp, b0, b1), c


def test_wall_row_source_beside_empty_band(driver):
    # tile 0 has no high rows at the bottom wall, tile 1 has 7: the high
    # nodes of rows 0..1 just right of the tile boundary are read along x by
    # the low set although nothing lies below them
    c = dict(nx=128, ny=32, xbc=XBC_PERIODIC, ybc=YBC_WALLS, iface=IF_HERMITE, tw=64, lo=[0, 7], hi=[5, 0])
    (fin, proj, n0, n1), = run(driver, [c])
    assert fin == []
    high = {(proj[k], proj[k + 1]) for k in range(2 * n0, len(proj), 2)}
    low = {(proj[k], proj[k + 1]) for k in range(0, 2 * n0, 2)}
    for j in range(2):
        assert (64, j) in high and (65, j) in high
        assert (62, j) in low and (63, j) in low
    bf, bp, b0, b1 = brute(c)
    assert (fin, proj, n0, n1) == (bf, bp, b0, b1)


def test_full_size_channel_lists(driver):
    # the pressure channel's shape: 4096 x 257, 64-column tiles, bands 8-64
    rng = np.random.default_rng(5)
    c = dict(nx=4096, ny=256, xbc=XBC_PRESSURE, ybc=YBC_WALLS, iface=IF_HERMITE, tw=64,
             lo=[int(v) for v in rng.integers(8, 65, 64)], hi=[int(v) for v in rng.integers(8, 65, 64)])
    (fin, proj, n0, n1), = run(driver, [c])
    # pressure columns: every row, first and last column
    assert fin == [v for j in range(257) for i in (0, 4095) for v in (i, j, int(j < c["lo"][i // 64] or j > 256 - c["hi"][i // 64]), 0)]
    # every listed node is a source and belongs to the stated set; row-major per set
    R = regions(c)
    pts = np.array(proj, np.int64).reshape(-1, 2)
    assert np.all(R[pts[:n0, 1], pts[:n0, 0]] == LOW) and np.all(R[pts[n0:, 1], pts[n0:, 0]] == HIGH)
    for part in (pts[:n0], pts[n0:]):
        key = part[:, 1] * 4096 + part[:, 0]
        assert np.all(np.diff(key) > 0)
    # count against a vectorised scan of the definition
    src = np.zeros_like(R, bool)
    for d in (-2, -1, 1, 2):
        sy = np.full_like(R, -1)
        if d > 0:
            sy[:-d] = R[d:]
        else:
            sy[-d:] = R[:d]
        sx = np.full_like(R, -1)
        if d > 0:
            sx[:, :-d] = R[:, d:]
        else:
            sx[:, -d:] = R[:, :d]
        src |= ((sy >= 0) & (sy != R)) | ((sx >= 0) & (sx != R))
    assert n0 == int(np.sum(src & (R == LOW))) and n1 == int(np.sum(src & (R == HIGH)))

"""Host logic: the grouped projector table that the residual-update kernel indexes.

The builder (paper_1709_09347_amd/csrc/tables.hpp, plain C++) is compiled with g++ and run
on the projector sets of the synthetic workloads.  Checked against the input entries:
the groups cover the points in order, keys ascend within a group, and per point and key
the grouped values equal the sum of the point's entries with that key (a ball wider than
the 5x5 transverse cell reaches some points twice with the same key), zero elsewhere;
and the block mask marks exactly the 16-point blocks with a nonzero value.
"""
import os
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1709_09347_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "host", "tables_driver.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tables") / "tables_driver")
    # address and undefined-behaviour sanitizers on the host builder (CPU code only)
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-fno-sanitize-recover=all", "-I", CSRC, DRIVER, "-o", exe], check=True)
    return exe


def _point_major(sysw):
    p = sysw.proj
    keys, pts, vals = [], [], []
    for a in range(p.n_atoms):
        lo, hi = int(p.ball_off[a]), int(p.ball_off[a + 1])
        v = np.zeros((hi - lo, 4))
        v[:, :p.n_proj] = p.ball_val[lo:hi]
        pts.append(p.ball_idx[lo:hi].astype(np.int64))
        keys.append(a * 4 + (p.ball_w[lo:hi].astype(np.int64) + 1))
        vals.append(v)
    pts, keys, vals = np.concatenate(pts), np.concatenate(keys).astype(np.int32), np.concatenate(vals)
    order = np.argsort(pts, kind="stable")
    pts, keys, vals = pts[order], keys[order], vals[order]
    off = np.zeros(sysw.n + 1, np.int32)
    np.add.at(off, pts + 1, 1)
    return np.cumsum(off).astype(np.int32), keys, vals, pts


def _run(driver, tmp_path, n, off, keys, vals, kg):
    inp = tmp_path / "in.bin"
    with open(inp, "wb") as f:
        np.array([n], np.int64).tofile(f)
        np.array([kg], np.int32).tofile(f)
        np.array([len(keys)], np.int64).tofile(f)
        off.astype(np.int32).tofile(f)
        keys.astype(np.int32).tofile(f)
        vals.astype(np.float64).tofile(f)
    out = tmp_path / "out.bin"
    subprocess.run([driver, str(inp), str(out)], check=True)
    data = open(out, "rb").read()
    tabs, pos = [], 0
    for dt in (np.int32, np.int32, np.float64, np.int32):
        m = int(np.frombuffer(data, np.int64, 1, pos)[0])
        pos += 8
        tabs.append(np.frombuffer(data, dt, m, pos).copy())
        pos += m * np.dtype(dt).itemsize
    return tabs


@pytest.mark.parametrize("case", ["tiny", "cfg2"])
def test_grouped_ket_table(driver, tmp_path, case):
    sysw = W.tiny(with_proj=True, fd_order=8) if case == "tiny" else W.config(2).systems[0]
    kg = 64
    off, keys, vals, pts = _point_major(sysw)
    n = sysw.n
    grp_off, grp_key, grp_u, grp_mask = _run(driver, tmp_path, n, off, keys, vals, kg)
    ng = (n + kg - 1) // kg
    grp_u = grp_u.reshape(-1, kg, 4)
    assert len(grp_off) == ng + 1 and grp_off[0] == 0 and grp_off[-1] == len(grp_key)
    # one bit per 16-point block of a group: set exactly where the block has a nonzero value
    nz_blocks = np.any(grp_u.reshape(len(grp_key), kg // 16, 16 * 4) != 0, axis=2)
    want_mask = (nz_blocks * (1 << np.arange(kg // 16))).sum(axis=1)
    np.testing.assert_array_equal(grp_mask, want_mask)
    want = {}
    for e in range(len(keys)):
        k = (int(pts[e]), int(keys[e]))
        want[k] = want.get(k, 0) + vals[e]
    got = {}
    for g in range(ng):
        ks = grp_key[grp_off[g]:grp_off[g + 1]]
        assert np.all(np.diff(ks) > 0)
        for j, key in enumerate(ks):
            u = grp_u[grp_off[g] + j]
            assert np.any(u != 0)   # every key of a group reaches one of its points
            for lane in range(kg):
                if np.any(u[lane] != 0):
                    assert g * kg + lane < n
                    got[(g * kg + lane, int(key))] = u[lane]
    assert set(want) == set(got)
    for k, v in want.items():
        np.testing.assert_allclose(got[k], v, rtol=0, atol=1e-15)
    if case == "tiny":
        assert len(want) < len(keys)

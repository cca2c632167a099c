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


# ----------------------------------------------------------------- chunked bra table

def _atom_major(sysw):
    """The projector entries per atom and cell shift (segments w = -1, 0, +1), as the
    library orders them before building its tables."""
    p = sysw.proj
    seg, idx, vals = [], [], []
    pos = 0
    for a in range(p.n_atoms):
        lo, hi = int(p.ball_off[a]), int(p.ball_off[a + 1])
        w = p.ball_w[lo:hi].astype(np.int64)
        for s in range(3):
            seg.append(pos)
            m = w == s - 1
            idx.append(p.ball_idx[lo:hi][m].astype(np.int32))
            v = np.zeros((int(m.sum()), 4))
            v[:, :p.n_proj] = p.ball_val[lo:hi][m]
            vals.append(v)
            pos += int(m.sum())
        seg.append(pos)
    return np.array(seg, np.int32), np.concatenate(idx), np.concatenate(vals)


def _run_bra(driver, tmp_path, n, n_atoms, seg, idx, vals, tp, max_pieces, pad):
    inp = tmp_path / "bra_in.bin"
    with open(inp, "wb") as f:
        np.array([n], np.int64).tofile(f)
        np.array([n_atoms, tp, max_pieces, pad], np.int32).tofile(f)
        np.array([len(idx)], np.int64).tofile(f)
        seg.astype(np.int32).tofile(f)
        idx.astype(np.int32).tofile(f)
        vals.astype(np.float64).tofile(f)
    out = tmp_path / "bra_out.bin"
    r = subprocess.run([driver, "bra", str(inp), str(out)], capture_output=True, text=True)
    if r.returncode != 0:
        return None, r.stderr
    data = open(out, "rb").read()
    names = ["piece_off", "piece_beg", "piece_meta", "piece_real", "slot_off", "slot_piece", "ent_pt", "ent_u",
             "key_off", "key_slot", "scalars"]
    tabs, pos = {}, 0
    for nm in names:
        dt = np.float64 if nm == "ent_u" else np.int32
        m = int(np.frombuffer(data, np.int64, 1, pos)[0])
        pos += 8
        tabs[nm] = np.frombuffer(data, dt, m, pos).copy()
        pos += m * np.dtype(dt).itemsize
    return tabs, ""


@pytest.mark.parametrize("case,tp,pad", [("tiny", 64, 4), ("tiny", 7, 1), ("tiny", 512, 3), ("cfg2", 256, 4),
                                         ("cfg2", 512, 4)])
def test_chunked_bra_table(driver, tmp_path, case, tp, pad):
    sysw = {"tiny": lambda: W.tiny(with_proj=True, fd_order=8),
            "cfg2": lambda: W.config(2).systems[0]}[case]()
    n, na = sysw.n, sysw.proj.n_atoms
    seg, idx, vals = _atom_major(sysw)
    max_pieces = 128
    t, err = _run_bra(driver, tmp_path, n, na, seg, idx, vals, tp, max_pieces, pad)
    assert t is not None, err
    pl, worst, max_slots = (int(x) for x in t["scalars"])
    nch = (n + tp - 1) // tp
    po, pbeg, pmeta, preal = t["piece_off"], t["piece_beg"], t["piece_meta"], t["piece_real"]
    so, sp = t["slot_off"], t["slot_piece"]
    ent_pt, ent_u = t["ent_pt"], t["ent_u"].reshape(-1, 4)
    key_off, key_slot = t["key_off"], t["key_slot"]
    nslots = len(key_slot)
    assert len(po) == nch + 1 and len(so) == nch + 1 and so[-1] == nslots and len(sp) == nslots + 1
    assert po[0] == 0 and np.all(np.diff(po) >= 0) and po[-1] == len(pbeg) == sp[-1] == len(preal)
    # pieces: counts padded to a multiple of pad, at most max_pieces per chunk
    cnt = pmeta & 0xFFFF
    assert np.all(preal >= 1) and np.all(cnt % pad == 0) and np.all((cnt >= preal) & (cnt < preal + pad))
    assert cnt.max() == pl and np.diff(po).max() == worst <= max_pieces
    assert pbeg[0] == 0 and np.all(pbeg[1:] == pbeg[:-1] + cnt[:-1]) and pbeg[-1] + cnt[-1] == len(ent_pt)
    # key of every reordered entry, from the slot its piece belongs to; padding marked -2
    key_of_slot = np.empty(nslots, np.int64)
    for k in range(3 * na):
        key_of_slot[key_slot[key_off[k]:key_off[k + 1]]] = k
    chunk_of_slot = np.repeat(np.arange(nch), np.diff(so))
    ent_key = np.full(len(ent_pt), -1, np.int64)
    ent_chunk = np.full(len(ent_pt), -1, np.int64)
    for c in range(nch):
        for q in range(po[c], po[c + 1]):
            ls = pmeta[q] >> 16
            g = so[c] + ls
            assert so[c] <= g < so[c + 1] and sp[g] <= q < sp[g + 1]
            ent_key[pbeg[q]:pbeg[q] + preal[q]] = key_of_slot[g]
            ent_chunk[pbeg[q]:pbeg[q] + preal[q]] = c
            ent_key[pbeg[q] + preal[q]:pbeg[q] + cnt[q]] = -2
        # the pieces of a slot are consecutive and differ in size by at most one; one piece
        # fewer per slot would have been too long: the chunk's pieces are as short as the
        # limit allows
        lc = preal[po[c]:po[c + 1]].max() if po[c + 1] > po[c] else 0
        for g in range(so[c], so[c + 1]):
            qs = np.arange(sp[g], sp[g + 1])
            assert len(qs) >= 1 and preal[qs].max() - preal[qs].min() <= 1
        if lc > 1:
            sizes = np.array([preal[sp[g]:sp[g + 1]].sum() for g in range(so[c], so[c + 1])])
            assert np.sum(-(-sizes // (lc - 1))) > max_pieces
        assert np.all(np.diff(key_of_slot[so[c]:so[c + 1]]) > 0)   # slots of a chunk by ascending key
    assert np.all(ent_key != -1), "every entry lies in one piece"
    pad_e = ent_key == -2
    assert np.all(ent_pt[pad_e] == 0) and np.all(ent_u[pad_e] == 0)
    real = ~pad_e
    assert real.sum() == len(idx)
    for k in range(3 * na):   # slots of a key in chunk order
        assert np.all(np.diff(chunk_of_slot[key_slot[key_off[k]:key_off[k + 1]]]) > 0)
    assert np.all((ent_pt >= 0) & (ent_pt < tp)) and np.all(ent_chunk[real] * tp + ent_pt[real] < n)
    # the same multiset of (point, key, values) as the input
    key_in = np.concatenate([np.full(seg[4 * a + s + 1] - seg[4 * a + s], 3 * a + s)
                             for a in range(na) for s in range(3)])
    a_in = np.lexsort((vals[:, 3], vals[:, 2], vals[:, 1], vals[:, 0], idx, key_in))
    pt_out = (ent_chunk * tp + ent_pt)[real]
    u_out, k_out = ent_u[real], ent_key[real]
    a_out = np.lexsort((u_out[:, 3], u_out[:, 2], u_out[:, 1], u_out[:, 0], pt_out, k_out))
    np.testing.assert_array_equal(key_in[a_in], k_out[a_out])
    np.testing.assert_array_equal(idx[a_in], pt_out[a_out])
    np.testing.assert_array_equal(vals[a_in], u_out[a_out])
    # the bra through the tables (every piece entry, padding included, then the chunk sums
    # added per key in chunk order) equals the direct per-segment sums; integer values keep
    # both sums exact
    rng = np.random.default_rng(3)
    x = rng.integers(-8, 9, size=n).astype(np.float64)
    ui = np.round(vals * 16)
    direct = np.zeros((3 * na, 4))
    np.add.at(direct, key_in, ui * x[idx][:, None])
    ui_all = np.zeros_like(ent_u)
    real_idx = np.flatnonzero(real)
    ui_all[real_idx[a_out]] = ui[a_in]
    chunk_pt = np.repeat(np.arange(nch), np.diff(so))   # chunk of each slot
    chunk_sum = np.zeros((nslots, 4))
    for g in range(nslots):
        base = chunk_pt[g] * tp
        for q in range(sp[g], sp[g + 1]):
            e = np.arange(pbeg[q], pbeg[q] + cnt[q])
            chunk_sum[g] += (ui_all[e] * x[np.minimum(base + ent_pt[e], n - 1)][:, None]).sum(axis=0)
    via = np.array([chunk_sum[key_slot[key_off[k]:key_off[k + 1]]].sum(axis=0) for k in range(3 * na)])
    np.testing.assert_array_equal(via, direct)


def test_chunked_bra_table_refuses_too_many_keys(driver, tmp_path):
    sysw = W.config(2).systems[0]
    seg, idx, vals = _atom_major(sysw)
    t, err = _run_bra(driver, tmp_path, sysw.n, sysw.proj.n_atoms, seg, idx, vals, 512, 8, 4)
    assert t is None and "keys in a chunk" in err

"""CPU model of the wavefront sweep kernel (csrc/wavefront.hip).

The GPU kernel runs tiles concurrently; any order in which each tile runs
after every tile it depends on is one of its possible executions.  This model
replays the kernel's exact index arithmetic -- lane -> column mapping with
shear, per-lane skew with the KB padding, the LDS ring rows and halo slots,
the roles of the waves (compute lanes, halo loader, right-hand-side loader,
result / export store), the three chunk buffers, the column-run groups and
their offset arithmetic, the buffer windows of the vectors, the sentinel
prefill for the next sweep, the packed coefficient positions -- with the
tiles run one after another in ticket order, and checks that

  * the result equals the sequential lexicographic sweep of the oracle,
  * every LDS ring read of a lane that has a point finds the value written
    for exactly that neighbour point in the same tile (or zero where the
    neighbour lies outside the grid), and lanes without a point compute
    zero from finite values,
  * every value fetched from another tile's column held the sentinel when the
    sweep started (so a concurrent reader would have waited for it) and was
    written by that tile's export path,
  * the right-hand side reaches each lane through the chunk buffer filled by
    the load role (column runs) and results leave as column runs one chunk
    behind; the roles' LDS accesses within a step never touch the same slot,
  * every buffer offset stays inside the planes the kernel's buffer covers,
    the run groups' offsets equal the points' indices, every used halo slot
    is inside the frame and has a loader lane, and the exported columns
    enumerated by the store role are exactly the columns other tiles read,
  * the prefill of a sweep marks every position the next sweep fetches, and
  * the packed-data position of every point is unique and inverted by the
    setup kernel's mapping.
"""
import numpy as np
import pytest

import oracle
import workloads

TX = TY = 16
NL = TX * TY
NH = 104
HIST = 16    # LDS ring rows
CH = 16      # steps per chunk of right-hand side / results
NB = 3       # chunk buffers
GRP = NL * CH // 64   # column-run groups per chunk
GPS = GRP // CH       # groups moved per step


def pat_has(pat, d):
    m = sum(abs(v) for v in d)
    return pat == 27 or (pat == 19 and m <= 2) or (pat == 7 and m <= 1)


def col_d(c):
    return (0, -1) if c == 3 else (-1, c - 1)


def col_used(pat, c):
    cx, cy = col_d(c)
    return any(pat_has(pat, (cx, cy, dz)) for dz in (-1, 0, 1))


def col_of(dx, dy):
    return dy + 1 if dx == -1 else (3 if dy == -1 else -1)


def hp(pat):
    return {7: (1, 1), 19: (3, 2), 27: (4, 2)}[pat]


def kb_of(pat):
    WX, WY = hp(pat)
    off = workloads.offsets(pat)
    return max(-(WX * int(d[0]) + WY * int(d[1]) + int(d[2])) for d in off[:pat // 2])


def halo_slot(qx, qy):
    if qx == -1:
        return qy + 2
    if qx == TX:
        return 22 + qy
    return 40 + 2 * qx + (qy + 2) if qy < 0 else 72 + 2 * qx + (qy - TY)


def halo_pos(hs):
    if hs < 20:
        return -1, hs - 2
    if hs < 40:
        return TX, hs - 22
    if hs < 72:
        return (hs - 40) // 2, (hs - 40) % 2 - 2
    return (hs - 72) // 2, TY + (hs - 72) % 2


def halo_used(pat, direction, sh, qx, qy):
    for c in range(4):
        if not col_used(pat, c):
            continue
        cx, cy = col_d(c)
        cx, cy = direction * cx, direction * cy
        lx, ly = qx - cx, qy - cy - sh * cx
        if 0 <= lx < TX and 0 <= ly < TY:
            return True
    return False


def exported(pat, lx, ly, sh, direction):
    for c in range(4):
        if not col_used(pat, c):
            continue
        cx, cy = col_d(c)
        cx, cy = direction * cx, direction * cy
        qx, qy = lx - cx, ly - cy - sh * cx
        if qx < 0 or qx >= TX or qy < 0 or qy >= TY:
            return True
    return False


def tiling(g, pat):
    nx, ny, nz = g
    WX, WY = hp(pat)
    sh = 0 if (pat == 7 or ny <= TY) else 1
    ntx = (nx + TX - 1) // TX
    nty = (ny + sh * (TX - 1) + TY - 1) // TY
    ns = nz + (WX - sh * WY) * (TX - 1) + WY * (TY - 1) + 2 * kb_of(pat)
    return sh, ntx, nty, ns


def inner_rect(pat, direction, sh):
    """Lanes whose column no other tile reads: the kernel's wf_inner."""
    xl, xh, yl, yh = 0, TX, 0, TY
    for c in range(4):
        if not col_used(pat, c):
            continue
        cx0, cy0 = col_d(c)
        cx, cy = direction * cx0, direction * cy0 + sh * direction * cx0
        xl, xh, yl, yh = max(xl, cx), min(xh, TX + cx), max(yl, cy), min(yh, TY + cy)
    return xl, xh, yl, yh


def exported_lane(rect, e):
    """The kernel's wf_exported_lane: e-th lane outside the rectangle."""
    xl, xh, yl, yh = rect
    nm = TY - (yh - yl)
    if e < TY * xl:
        lx, ly = divmod(e, TY)
    elif e < TY * xl + nm * (xh - xl):
        q = e - TY * xl
        lx, w = xl + q // nm, q % nm
        ly = w if w < yl else yh + (w - yl)
    else:
        q = e - TY * xl - nm * (xh - xl)
        lx, ly = xh + q // TY, q % TY
    return lx * TY + ly


def wf_point(g, pat, q):
    """The setup kernel's map from a packed position to its point (or -1)."""
    nx, ny, nz = g
    WX, WY = hp(pat)
    sh, ntx, nty, ns = tiling(g, pat)
    l, r = q % NL, q // NL
    s, tile = r % ns, r // ns
    X, Y = divmod(tile, nty)
    lx, ly = divmod(l, TY)
    x, y = X * TX + lx, Y * TY + ly - sh * lx
    z = s - ((WX - sh * WY) * lx + WY * ly + kb_of(pat))
    ok = x < nx and 0 <= y < ny and 0 <= z < nz
    return (x * ny + y) * nz + z if ok else -1


def run_sweep(g, pat, direction, A, rd, h, x_init, nxt_dir, nxt_buf, lds=None):
    """Replays one kernel launch in ticket order.  x_init: output buffer at
    launch (nan marks a sentinel).  lds: the workgroup's LDS (ring, chunk
    buffers) carried from tile to tile, zero at launch.  Returns (x, prefill
    mask, packed index of every point)."""
    nx, ny, nz = g
    N = nx * ny * nz
    WX, WY = hp(pat)
    KB = kb_of(pat)
    off = workloads.offsets(pat)
    C = pat // 2
    T = list(range(C)) if direction > 0 else list(range(C + 1, pat))
    sh, ntx, nty, NS = tiling(g, pat)
    nsteps = -(-NS // HIST) * HIST
    NC = nsteps // CH
    RW = NL + NH + 1
    HRW = NL + 1
    x = x_init.copy()
    done = np.full(N, np.nan)   # every value as soon as it is computed (model bookkeeping only)
    sent_at_start = np.isnan(x_init)
    exported_at = set()         # positions written by an export
    pref = np.zeros(N, bool)
    lanes = np.arange(NL)
    lx, ly = lanes // TY, lanes % TY
    skew = (WX - sh * WY) * lx + WY * ly + KB
    # exported columns: the store role's rectangle enumeration equals the
    # columns other tiles read, in lane order
    rect = inner_rect(pat, direction, sh)
    ne = NL - (rect[1] - rect[0]) * (rect[3] - rect[2])
    assert ne <= 64, "more exported columns than lanes of the store wave"
    elanes = [exported_lane(rect, e) for e in range(ne)]
    assert elanes == [l for l in range(NL) if exported(pat, l // TY, l % TY, sh, direction)]
    rectn = inner_rect(pat, nxt_dir, sh) if nxt_buf is not None else None
    # neighbour column LDS indices
    nidx = {}
    for c in range(4):
        if not col_used(pat, c):
            continue
        cx, cy = col_d(c)
        cx, cy = direction * cx, direction * cy
        qx, qy = lx + cx, ly + cy + sh * cx
        idx = np.empty(NL, np.int64)
        for l in range(NL):
            if 0 <= qx[l] < TX and 0 <= qy[l] < TY:
                idx[l] = qx[l] * TY + qy[l]
            else:
                hs = halo_slot(int(qx[l]), int(qy[l]))
                assert 0 <= hs < NH and halo_pos(hs) == (qx[l], qy[l])
                idx[l] = NL + hs
        nidx[c] = idx
    # halo loader: lane t of the halo wave handles slots t and 64 + t
    loaders = [hs for hs in range(NH) if halo_used(pat, direction, sh, *halo_pos(hs))]
    assert all(hs < 128 for hs in loaders)
    used_slots = {int(v) - NL for c in nidx for v in nidx[c] if v >= NL}
    assert used_slots <= set(loaders), "a used halo slot has no loader lane"
    if lds is None:
        lds = {"ring": np.zeros((HIST, RW)), "hbuf": np.zeros((NB, CH, HRW))}
    ring, hbuf = lds["ring"], lds["hbuf"]
    pkidx = np.full(N, -1, np.int64)
    ntiles = ntx * nty
    pl = ny * nz
    for ticket in range(ntiles):
        t = ticket if direction > 0 else ntiles - 1 - ticket
        X, Y = divmod(t, nty)
        p0 = max(X * TX - 1, 0)
        p1 = min(X * TX + TX + 1, nx)
        lo_i, hi_i = p0 * pl, p1 * pl
        xt = X * TX + lx
        yt = Y * TY + ly - sh * lx
        colv = (xt < nx) & (yt >= 0) & (yt < ny)
        cb = (xt * ny + yt) * nz
        ring_pt = np.full((HIST, RW), -2, np.int64)    # point index, or -1 for "zero"
        ring_it = np.full((HIST, RW), -10 ** 9, np.int64)
        hbuf_pt = np.full((NB, CH, HRW), -2, np.int64)  # point a slot holds (-1: none)
        touched = {}                                    # LDS slots used in the current step, by role
        own_prev = np.zeros(NL)

        def step_of(k):
            return k if direction > 0 else NS - 1 - k

        def touch(key, role, write):
            # two roles may read one slot in a step; a write excludes any other role
            for r2, w2 in touched.setdefault(key, set()):
                assert r2 == role or not (write or w2), f"{role} and {r2} race on LDS slot {key}"
            touched[key].add((role, write))

        def run_point(c, r, tl):
            """Group r of chunk c, lane tl of a run wave: (step row m, column,
            point index or -1), with the kernel's offset arithmetic checked."""
            cq, m = tl // 16, tl % 16
            col = 4 * r + cq
            s = step_of(c * CH + m)
            # the kernel's bases
            skq = WY * cq + KB
            y0 = Y * TY + cq
            a0 = ((X * TX - p0) * ny + y0) * nz - skq
            sx = WX - sh * WY
            gx, gy = (ny - sh) * nz - sx, 4 * (nz - WY)
            jj, gg = r // 4, r % 4
            e = a0 + s + jj * gx + gg * gy
            zz = s - skq - jj * sx - 4 * WY * gg
            yy = (y0 - sh * jj) if X * TX + jj < nx else -TY - 1
            yy += 4 * gg
            ok = 0 <= yy < ny and 0 <= zz < nz
            # the point directly
            cl, cyy = col // TY, col % TY
            xx, yd = X * TX + cl, Y * TY + cyy - sh * cl
            z = s - ((WX - sh * WY) * cl + WY * cyy + KB)
            valid = xx < nx and 0 <= yd < ny and 0 <= z < nz
            assert ok == valid, "run group validity differs from the point's"
            gi = (xx * ny + yd) * nz + z if valid else -1
            if valid:
                assert e + p0 * pl == gi, "run group offset differs from the point index"
                assert lo_i <= gi < hi_i, "column-run offset outside the buffer window"
            return m, col, gi

        def load_group(c, r):
            for tl in range(64):
                m, col, gi = run_point(c, r, tl)
                touch(("hbuf", c % NB, m, col), "load", True)
                hbuf[c % NB, m, col] = h[gi] if gi >= 0 else 0.0
                hbuf_pt[c % NB, m, col] = -3   # holds a right-hand side now

        def drain_group(c, r):
            for tl in range(64):
                m, col, gi = run_point(c, r, tl)
                touch(("hbuf", c % NB, m, col), "store", False)
                if gi < 0:
                    continue
                assert hbuf_pt[c % NB, m, col] == gi, "result slot holds another point"
                if not exported(pat, col // TY, col % TY, sh, direction):
                    assert np.isnan(x[gi]) or not sent_at_start[gi]
                    x[gi] = hbuf[c % NB, m, col]
                else:
                    assert x[gi] == hbuf[c % NB, m, col]   # exported earlier, same value
                if nxt_buf is not None and exported(pat, col // TY, col % TY, sh, nxt_dir):
                    xl, xh, yl, yh = rectn
                    lxr, g4 = r // 4, r % 4
                    assert lxr < xl or lxr >= xh or 4 * g4 < yl or 4 * g4 + 3 >= yh, \
                        "sentinel store of a group skipped"
                    pref[gi] = True

        def export_step(k):
            if k < 0:
                return
            s = step_of(k)
            r = k % HIST
            for el in elanes:
                z = s - skew[el]
                touch(("ring", r, el), "store", False)
                if 0 <= s < NS and colv[el] and 0 <= z < nz:
                    gi = cb[el] + z
                    assert lo_i <= gi < hi_i, "export offset outside the buffer window"
                    assert ring_pt[r, el] == gi, "exported ring slot holds another point"
                    x[gi] = ring[r, el]
                    exported_at.add(int(gi))

        def halo_put(k):
            s = step_of(k)
            r = k % HIST
            for hs in loaders:
                qx, qy = halo_pos(hs)
                hskew = (WX - sh * WY) * qx + WY * qy + KB
                gx, gy = X * TX + qx, Y * TY + qy - sh * qx
                hz = s - hskew
                ok = 0 <= s < NS and 0 <= gx < nx and 0 <= gy < ny and 0 <= hz < nz
                touch(("ring", r, NL + hs), "halo", True)
                if ok:
                    gi = (gx * ny + gy) * nz + hz
                    assert lo_i <= gi < hi_i, "halo offset outside the buffer window"
                    assert sent_at_start[gi], "fetched a position that was not a sentinel at launch"
                    assert not np.isnan(x[gi]), "fetched a value its producer has not written"
                    assert int(gi) in exported_at, "fetched a value not written by an export"
                    ring[r, NL + hs], ring_pt[r, NL + hs] = x[gi], gi
                else:
                    ring[r, NL + hs], ring_pt[r, NL + hs] = 0.0, -1
                ring_it[r, NL + hs] = k

        # prologue: chunk 0 into buffer 0 (chunk 1 is in the load role's registers)
        for r in range(GRP):
            load_group(0, r)
        for k in range(nsteps):
            touched.clear()
            j, c = k % HIST, k // CH
            halo_put(k)
            s = step_of(k)
            z = s - skew
            act = colv & (z >= 0) & (z < nz)
            xr = np.zeros(NL)
            for l in range(NL):
                slot = (c % NB, k % CH, l)
                touch(("hbuf",) + slot, "compute", True)
                tv = hbuf[slot]
                if not act[l]:
                    # no point: zero right-hand side, zero coefficients, finite values
                    assert tv == 0.0
                    for so in T:
                        dx, dy, dz = (int(v) for v in off[so])
                        if not (dx == 0 and dy == 0):
                            c4 = col_of(direction * dx, direction * dy)
                            back = direction * (WX * dx + WY * dy + dz)
                            assert np.isfinite(ring[(j + back) % HIST, nidx[c4][l]])
                    continue
                i = cb[l] + z[l]
                assert lo_i <= i < hi_i, "point offset outside the buffer window"
                pkidx[i] = (t * NS + s) * NL + l
                assert tv == h[i] and hbuf_pt[slot] == -3, "right-hand side chunk holds another point"
                for so in T:
                    dx, dy, dz = (int(v) for v in off[so])
                    xn, yn, zn = xt[l] + dx, yt[l] + dy, z[l] + dz
                    inb = 0 <= xn < nx and 0 <= yn < ny and 0 <= zn < nz
                    gi = (xn * ny + yn) * nz + zn
                    if dx == 0 and dy == 0:
                        val = own_prev[l]
                        assert (val == done[gi]) if inb else val == 0.0
                    else:
                        c4 = col_of(direction * dx, direction * dy)
                        back = direction * (WX * dx + WY * dy + dz)
                        assert -KB <= back <= -1
                        r = (j + back) % HIST
                        idx = nidx[c4][l]
                        touch(("ring", r, int(idx)), "compute", False)
                        assert ring_it[r, idx] == k + back, "ring row not written in this tile at that step"
                        val = ring[r, idx]
                        if inb:
                            assert ring_pt[r, idx] == gi, "ring slot holds another point"
                        else:
                            assert val == 0.0
                    tv = _fma(-A[so, i], val, tv)
                xr[l] = tv * rd[i]
                done[i] = xr[l]
            own_prev = xr
            for l in range(NL):
                touch(("ring", j, l), "compute", True)
            ring[j, :NL] = xr
            ring_pt[j, :NL] = np.where(act, cb + z, -1)
            ring_it[j, :NL] = k
            for l in range(NL):   # each lane's result over its right-hand-side slot
                slot = (c % NB, k % CH, l)
                hbuf[slot] = xr[l]
                hbuf_pt[slot] = (cb[l] + z[l]) if act[l] else -1
            # store role: the previous step's exports, then the previous
            # chunk's groups of this step; load role: the next chunk's groups
            export_step(k - 1)
            for gq in range(GPS):
                if c > 0:
                    drain_group(c - 1, j * GPS + gq)
                load_group(c + 1, j * GPS + gq)
        touched.clear()
        export_step(nsteps - 1)
        for r in range(GRP):
            drain_group(NC - 1, r)
    return x, pref, pkidx


def _fma(a, b, c):
    from fractions import Fraction
    return float(Fraction(a) * Fraction(b) + Fraction(c))


@pytest.mark.parametrize("pat", [7, 19, 27])
@pytest.mark.parametrize("g", [(20, 35, 6), (33, 17, 5), (5, 40, 4), (37, 9, 5)])
def test_wavefront_schedule_matches_sequential(pat, g):
    A = workloads.random_sgdia(g, pat, seed=2)
    off = workloads.offsets(pat)
    N = int(np.prod(g))
    rd = 1.0 / A[pat // 2]
    b = workloads.rng(1).uniform(-1, 1, size=N)
    # forward sweep with zero initial guess; every output position starts as sentinel
    x0 = np.full(N, np.nan)
    u_f, pref_f, pk_f = run_sweep(g, pat, +1, A, rd, b, x0, -1, True)
    ref_f = oracle.gs_sweep(off, A, rd, b.reshape(g), np.zeros(g), 1, 1).ravel()
    assert np.array_equal(u_f, ref_f)
    # backward sweep: input h = f - L u_old (old values first), output starts
    # with the sentinels the forward sweep wrote
    u_old = workloads.rng(3).uniform(-1, 1, size=N)
    hb = b.copy()
    for i in range(N):
        xx, yy, zz = i // (g[1] * g[2]), (i // g[2]) % g[1], i % g[2]
        for s in range(pat // 2):
            d = off[s]
            a, bb, c = xx + d[0], yy + d[1], zz + d[2]
            if 0 <= a < g[0] and 0 <= bb < g[1] and 0 <= c < g[2]:
                hb[i] = _fma(-A[s, i], u_old[(a * g[1] + bb) * g[2] + c], hb[i])
    xb0 = np.where(pref_f, np.nan, 0.0)
    u_b, pref_b, pk_b = run_sweep(g, pat, -1, A, rd, hb, xb0, +1, True)
    ref_b = oracle.gs_sweep(off, A, rd, b.reshape(g), u_old.reshape(g), -1, 0).ravel()
    assert np.array_equal(u_b, ref_b)
    # both directions use the same packed position per point, every point
    # exactly once, and the setup kernel maps each position back to its point
    assert np.array_equal(pk_f, pk_b) and (pk_f >= 0).all()
    assert len(np.unique(pk_f)) == N
    assert all(wf_point(g, pat, int(pk_f[i])) == i for i in range(N))
    # and the next forward sweep fetches only positions the backward sweep prefilled
    xf1 = np.where(pref_b, np.nan, 0.0)
    u_f2, _, _ = run_sweep(g, pat, +1, A, rd, b, xf1, -1, None)
    assert np.array_equal(u_f2, ref_f)


def test_out_of_grid_couplings_are_zero():
    # the kernel applies every coupling unconditionally; the generator (like
    # every operator the library builds) stores couplings leaving the grid as 0
    g = (6, 5, 4)
    for pat in (7, 19, 27):
        A = workloads.random_sgdia(g, pat, seed=5)
        off = workloads.offsets(pat)
        for s, d in enumerate(off):
            for i in range(int(np.prod(g))):
                xx, yy, zz = i // (g[1] * g[2]), (i // g[2]) % g[1], i % g[2]
                if not (0 <= xx + d[0] < g[0] and 0 <= yy + d[1] < g[1] and 0 <= zz + d[2] < g[2]):
                    assert A[s, i] == 0.0

"""CPU model of the point-block (3x3) wavefront sweep (csrc/block.hip).

Replays the kernel's index arithmetic -- 8 x 8-column sheared tiles in
ticket order, per-lane skew with the 3d27 weights and KB padding, the LDS
ring rows and the 56 halo slots, the loader lanes, buffer windows of the
interleaved vectors, the sentinel prefill -- with the tiles run one after
another, and checks that the result equals the oracle's sequential
point-block Gauss-Seidel sweep bit for bit, that every ring read finds the
value of exactly the neighbour node it stands for (or zero outside the
grid), that every value fetched from another tile held the sentinel at
launch, and that every offset stays inside its buffer.
"""
import numpy as np
import pytest

import oracle
import workloads

TX = TY = 8
NL = TX * TY
NH = 56
HIST = 16
WX, WY, KB = 4, 2, 7


def col_d(c):
    return (0, -1) if c == 3 else (-1, c - 1)


def col_of(dx, dy):
    return dy + 1 if dx == -1 else (3 if dy == -1 else -1)


def halo_slot(qx, qy):
    if qx == -1:
        return qy + 2
    if qx == TX:
        return 14 + qy
    return 24 + 2 * qx + (qy + 2) if qy < 0 else 40 + 2 * qx + (qy - TY)


def halo_pos(hs):
    if hs < 12:
        return -1, hs - 2
    if hs < 24:
        return TX, hs - 14
    if hs < 40:
        return (hs - 24) // 2, (hs - 24) % 2 - 2
    return (hs - 40) // 2, TY + (hs - 40) % 2


def halo_used(direction, sh, qx, qy):
    for c in range(4):
        cx, cy = col_d(c)
        cx, cy = direction * cx, direction * cy
        if 0 <= qx - cx < TX and 0 <= qy - cy - sh * cx < TY:
            return True
    return False


def exported(direction, lx, ly, sh):
    for c in range(4):
        cx, cy = col_d(c)
        cx, cy = direction * cx, direction * cy
        qx, qy = lx - cx, ly - cy - sh * cx
        if qx < 0 or qx >= TX or qy < 0 or qy >= TY:
            return True
    return False


def tiling(g):
    nx, ny, nz = g
    sh = 0 if ny <= TY else 1
    ntx = (nx + TX - 1) // TX
    nty = (ny + sh * (TX - 1) + TY - 1) // TY
    ns = nz + (WX - sh * WY) * (TX - 1) + WY * (TY - 1) + 2 * KB
    return sh, ntx, nty, ns


def run_bsweep(g, direction, A, Dinv, h, x_init, nxt_dir, nxt):
    nx, ny, nz = g
    N = nx * ny * nz
    off = workloads.offsets(27)
    T = list(range(13)) if direction > 0 else list(range(14, 27))
    sh, ntx, nty, NS = tiling(g)
    RW = (NL + NH) * 3 + 1
    x = x_init.copy()
    sent0 = np.isnan(x_init)
    pref = np.zeros(3 * N, bool)
    lanes = np.arange(NL)
    lx, ly = lanes // TY, lanes % TY
    skew = (WX - sh * WY) * lx + WY * ly + KB
    exp_now = [exported(direction, a, b, sh) for a, b in zip(lx, ly)]
    exp_next = [nxt and exported(nxt_dir, a, b, sh) for a, b in zip(lx, ly)]
    nidx = {}
    for c in range(4):
        cx, cy = col_d(c)
        cx, cy = direction * cx, direction * cy
        idx = []
        for l in range(NL):
            qx, qy = lx[l] + cx, ly[l] + cy + sh * cx
            if 0 <= qx < TX and 0 <= qy < TY:
                idx.append(qx * TY + qy)
            else:
                hs = halo_slot(qx, qy)
                assert 0 <= hs < NH and halo_pos(hs) == (qx, qy)
                idx.append(NL + hs)
        nidx[c] = idx
    loaders = {hs: hs for hs in range(NH) if halo_used(direction, sh, *halo_pos(hs))}
    assert {v - NL for c in nidx for v in nidx[c] if v >= NL} <= set(loaders)
    ntiles = ntx * nty
    pl = ny * nz
    for ticket in range(ntiles):
        t = ticket if direction > 0 else ntiles - 1 - ticket
        X, Y = divmod(t, nty)
        p0, p1 = max(X * TX - 1, 0), min(X * TX + TX + 1, nx)
        lo_i, hi_i = p0 * pl, p1 * pl
        xt, yt = X * TX + lx, Y * TY + ly - sh * lx
        colv = (xt < nx) & (yt >= 0) & (yt < ny)
        ring = np.full(HIST * RW, np.nan)
        ring_pt = np.full(HIST * RW, -2, np.int64)
        ring_it = np.full(HIST * RW, -10 ** 9, np.int64)

        def step_of(k):
            return k if direction > 0 else NS - 1 - k

        def halo_put(k):
            s = step_of(k)
            for hs in loaders:
                qx, qy = halo_pos(hs)
                hskew = (WX - sh * WY) * qx + WY * qy + KB
                gx, gy = X * TX + qx, Y * TY + qy - sh * qx
                hz = s - hskew
                base = (k % HIST) * RW + (NL + hs) * 3
                assert base + 2 < HIST * RW
                if 0 <= s < NS and 0 <= gx < nx and 0 <= gy < ny and 0 <= hz < nz:
                    gi = (gx * ny + gy) * nz + hz
                    assert lo_i <= gi < hi_i
                    assert sent0[gi * 3:gi * 3 + 3].all(), "fetched a node that was not a sentinel at launch"
                    assert not np.isnan(x[gi * 3:gi * 3 + 3]).any(), "fetched a value not yet written"
                    ring[base:base + 3] = x[gi * 3:gi * 3 + 3]
                    ring_pt[base:base + 3] = gi
                else:
                    ring[base:base + 3] = 0.0
                    ring_pt[base:base + 3] = -1
                ring_it[base:base + 3] = k

        halo_put(0)
        nsteps = -(-NS // 4) * 4
        for k in range(nsteps):
            s = step_of(k)
            z = s - skew
            act = colv & (z >= 0) & (z < nz)
            xr = np.zeros((NL, 3))
            for l in np.nonzero(act)[0]:
                i = (xt[l] * ny + yt[l]) * nz + z[l]
                assert lo_i <= i < hi_i
                tv = h[i * 3:i * 3 + 3].copy()
                for so in T:
                    dx, dy, dz = (int(v) for v in off[so])
                    xn, yn, zn = xt[l] + dx, yt[l] + dy, z[l] + dz
                    inb = 0 <= xn < nx and 0 <= yn < ny and 0 <= zn < nz
                    gi = (xn * ny + yn) * nz + zn
                    if dx == 0 and dy == 0:
                        # the same column one step earlier (this lane's own ring slot)
                        base = ((k - 1) % HIST) * RW + l * 3
                        assert ring_it[base] == k - 1, "ring row not written at that step"
                    else:
                        c = col_of(direction * dx, direction * dy)
                        back = direction * (WX * dx + WY * dy + dz)
                        assert -KB <= back <= -1
                        base = ((k + back) % HIST) * RW + nidx[c][l] * 3
                        assert ring_it[base] == k + back, "ring row not written at that step"
                    u = ring[base:base + 3]
                    if inb:
                        assert ring_pt[base] == gi, "ring slot holds another node"
                    else:
                        assert (u == 0.0).all()
                    for r in range(3):
                        for cc in range(3):
                            tv[r] = _fma(-A[(so * 9 + r * 3 + cc), i], u[cc], tv[r])
                for r in range(3):
                    acc = Dinv[r * 3, i] * tv[0]
                    acc = _fma(Dinv[r * 3 + 1, i], tv[1], acc)
                    acc = _fma(Dinv[r * 3 + 2, i], tv[2], acc)
                    xr[l, r] = acc
                x[i * 3:i * 3 + 3] = xr[l]
                if exp_next[l]:
                    pref[i * 3:i * 3 + 3] = True
            for l in range(NL):
                base = (k % HIST) * RW + l * 3
                ring[base:base + 3] = xr[l]
                ring_pt[base:base + 3] = ((xt[l] * ny + yt[l]) * nz + z[l]) if act[l] else -1
                ring_it[base:base + 3] = k
            halo_put(k + 1)
    return x, pref


def _fma(a, b, c):
    from fractions import Fraction
    return float(Fraction(a) * Fraction(b) + Fraction(c))


@pytest.mark.parametrize("g", [(10, 12, 4), (17, 9, 3), (5, 20, 3)])
def test_block_wavefront_matches_sequential(g):
    N = int(np.prod(g))
    off = workloads.offsets(27)
    A4 = workloads.random_sgdia(g, 27, seed=3, block=3)
    A = A4.reshape(27 * 9, N)
    Dinv = oracle.block_dinv(off, A4, g)
    b = workloads.rng(4).uniform(-1, 1, size=3 * N)
    sh4 = tuple(g) + (3,)
    x0 = np.full(3 * N, np.nan)
    u_f, pref_f = run_bsweep(g, +1, A, Dinv, b, x0, -1, True)
    ref_f = oracle.bgs_sweep(off, A4, Dinv, b.reshape(sh4), np.zeros(sh4), +1, 1).ravel()
    assert np.array_equal(u_f, ref_f)
    # backward sweep from h = f - L u_old, output starting with the forward sweep's sentinels
    u_old = workloads.rng(5).uniform(-1, 1, size=3 * N)
    hb = b.copy()
    for i in range(N):
        xx, yy, zz = i // (g[1] * g[2]), (i // g[2]) % g[1], i % g[2]
        for s in range(13):
            d = off[s]
            a_, bb, c_ = xx + d[0], yy + d[1], zz + d[2]
            if 0 <= a_ < g[0] and 0 <= bb < g[1] and 0 <= c_ < g[2]:
                j = (a_ * g[1] + bb) * g[2] + c_
                for r in range(3):
                    for cc in range(3):
                        hb[i * 3 + r] = _fma(-A[s * 9 + r * 3 + cc, i], u_old[j * 3 + cc], hb[i * 3 + r])
    xb0 = np.where(pref_f, np.nan, 0.0)
    u_b, _ = run_bsweep(g, -1, A, Dinv, hb, xb0, +1, True)
    ref_b = oracle.bgs_sweep(off, A4, Dinv, b.reshape(sh4), u_old.reshape(sh4), -1, 0).ravel()
    assert np.array_equal(u_b, ref_b)

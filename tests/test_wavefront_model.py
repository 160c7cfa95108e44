"""CPU model of the wavefront sweep kernel's schedule (csrc/wavefront.hip).

The GPU kernel runs tiles concurrently; any order in which each tile runs
after every tile it depends on is one of its possible executions.  This model
replays the kernel's exact index arithmetic -- lane -> column mapping with
shear, per-lane skew, LDS ring slots, register windows, the set of columns
read from other tiles, the sentinel prefill for the next sweep -- with the
tiles run one after another in ticket order, and checks that

  * the result equals the sequential lexicographic sweep of the oracle,
  * every value read from another tile lies in a column that the producer
    writes with a coherent store and that held the sentinel when the sweep
    started (so a concurrent reader would have waited for it),
  * every LDS ring read finds the value written for that point,
  * the prefill of a sweep marks every position the next sweep reads remotely.
"""
import numpy as np
import pytest

import oracle
import workloads

TX = TY = 16
HIST = 8


def pat_has(pat, d):
    m = sum(abs(v) for v in d)
    return pat == 27 or (pat == 19 and m <= 2) or (pat == 7 and m <= 1)


def col_d(c):
    return (0, -1) if c == 3 else (-1, c - 1)


def col_used(pat, c):
    cx, cy = col_d(c)
    return any(pat_has(pat, (cx, cy, dz)) for dz in (-1, 0, 1))


def col_maxdz(pat, c):
    cx, cy = col_d(c)
    return 1 if pat_has(pat, (cx, cy, 1)) else 0


def hp(pat):
    return {7: (1, 1), 19: (3, 2), 27: (4, 2)}[pat]


def exported(pat, lx, ly, sh, direction):
    """Is lane (lx, ly)'s column read by a lane of another tile in a sweep of
    the given direction?"""
    for c in range(4):
        if not col_used(pat, c):
            continue
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
    return sh, ntx, nty


def run_sweep(g, pat, direction, A, rd, h, x_init, nxt_dir, nxt_buf):
    """Replays one kernel launch in the kernel's tile order.  Both directions
    share one tile geometry (forward frame); the backward sweep visits tiles
    and steps in reverse and reads upper neighbours.  x_init: output buffer
    at launch (nan marks a sentinel).  Returns (x, prefill mask, skewed-index
    map used for the coefficient reads)."""
    nx, ny, nz = g
    N = nx * ny * nz
    WX, WY = hp(pat)
    off = workloads.offsets(pat)
    C = pat // 2
    T = list(range(C)) if direction > 0 else list(range(C + 1, pat))
    sh, ntx, nty = tiling(g)
    PRE = max(col_maxdz(pat, c) for c in range(4) if col_used(pat, c))
    x = x_init.copy()
    sent_at_start = np.isnan(x_init)
    pref = np.zeros(N, bool)
    coherent = np.zeros(N, bool)
    lanes = np.arange(TX * TY)
    lx, ly = lanes // TY, lanes % TY
    skew = (WX - sh * WY) * lx + WY * ly + PRE
    NS = nz + (WX - sh * WY) * (TX - 1) + WY * (TY - 1) + 2 * PRE  # pre-roll at both ends
    exp_lane = np.array([exported(pat, a, b, sh, direction) for a, b in zip(lx, ly)])
    exp_next = np.array([exported(pat, a, b, sh, nxt_dir) for a, b in zip(lx, ly)]) if nxt_buf is not None \
        else np.zeros(TX * TY, bool)
    skidx = np.full(N, -1, np.int64)
    ntiles = ntx * nty
    for ticket in range(ntiles):
        t = ticket if direction > 0 else ntiles - 1 - ticket
        X, Y = divmod(t, nty)
        ring = np.full((HIST, TX * TY), np.nan)
        ring_pt = -np.ones((HIST, TX * TY), np.int64)
        xt = X * TX + lx
        yt = Y * TY + ly - sh * lx
        colv = (xt < nx) & (yt >= 0) & (yt < ny)
        cb = (xt * ny + yt) * nz
        nl, nsk, rem, cin, ncb = {}, {}, {}, {}, {}
        for c in range(4):
            cx, cy = col_d(c)
            cxo, cyo = direction * cx, direction * cy
            qx, qy = lx + cxo, ly + cyo + sh * cxo
            rem[c] = (qx < 0) | (qx >= TX) | (qy < 0) | (qy >= TY)
            nl[c] = np.where(rem[c], 0, qx * TY + qy)
            nsk[c] = (WX - sh * WY) * qx + WY * qy + PRE
            qxx, qyy = xt + cxo, yt + cyo
            cin[c] = colv & (qxx >= 0) & (qxx < nx) & (qyy >= 0) & (qyy < ny)
            ncb[c] = (qxx * ny + qyy) * nz
        win = np.zeros((4, 3, TX * TY))
        own_prev = np.zeros(TX * TY)
        for k in range(NS):
            s = k if direction > 0 else NS - 1 - k
            z = s - skew
            for c in range(4):
                if not col_used(pat, c):
                    continue
                md = col_maxdz(pat, c)
                win[c][0] = win[c][1]
                win[c][1] = win[c][2]
                zn = z + direction * md
                ok = cin[c] & (zn >= 0) & (zn < nz)
                v = np.zeros(TX * TY)
                for l in np.nonzero(ok)[0]:
                    gi = ncb[c][l] + zn[l]
                    if not rem[c][l]:
                        slot = (zn[l] + nsk[c][l]) % HIST
                        assert ring_pt[slot, nl[c][l]] == gi, "LDS ring slot does not hold the point"
                        v[l] = ring[slot, nl[c][l]]
                    else:
                        assert sent_at_start[gi], "remote read of a position that was not a sentinel"
                        assert coherent[gi], "remote read of a value not written coherently"
                        v[l] = x[gi]
                win[c][md + 1] = v
            act = colv & (z >= 0) & (z < nz)
            for l in np.nonzero(act)[0]:
                i = cb[l] + z[l]
                skidx[i] = (t * NS + s) * TX * TY + l
                tv = h[i]
                for so in T:
                    dx, dy, dz = (int(v) for v in off[so])
                    if dx == 0 and dy == 0:
                        val, ok = own_prev[l], 0 <= z[l] - direction < nz
                    else:
                        c = col_of(direction * dx, direction * dy)
                        val = win[c][direction * dz + 1][l]
                        ok = cin[c][l] and 0 <= z[l] + dz < nz
                    if ok:
                        tv = _fma(-A[so, i], val, tv)
                xv = tv * rd[i]
                own_prev[l] = xv
                ring[s % HIST, l] = xv
                ring_pt[s % HIST, l] = i
                x[i] = xv
                if exp_lane[l]:
                    coherent[i] = True
                if exp_next[l]:
                    pref[i] = True
    return x, pref, skidx


def col_of(dx, dy):
    return dy + 1 if dx == -1 else (3 if dy == -1 else -1)


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
    u_f, pref_f, sk_f = run_sweep(g, pat, +1, A, rd, b, x0, -1, True)
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
    u_b, pref_b, sk_b = run_sweep(g, pat, -1, A, rd, hb, xb0, +1, True)
    ref_b = oracle.gs_sweep(off, A, rd, b.reshape(g), u_old.reshape(g), -1, 0).ravel()
    assert np.array_equal(u_b, ref_b)
    # both directions read the coefficients at the same skewed positions,
    # every point exactly once, each position belonging to one point
    assert np.array_equal(sk_f, sk_b) and (sk_f >= 0).all()
    assert len(np.unique(sk_f)) == N
    # and the next forward sweep reads only positions the backward sweep prefilled
    xf1 = np.where(pref_b, np.nan, 0.0)
    u_f2, _, _ = run_sweep(g, pat, +1, A, rd, b, xf1, -1, None)
    assert np.array_equal(u_f2, ref_f)

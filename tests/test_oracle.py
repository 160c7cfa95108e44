"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check compares the oracle with something other than itself: explicit
dense matrices assembled in ``helpers.py``, closed forms, values printed in
the paper (``tests/golden``), textbook special cases and library solvers.
"""
import os

import numpy as np
import pytest

import oracle
import workloads
from tests import helpers

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold_tables():
    out = {}
    with open(os.path.join(GOLD, "paper_tables.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            out[tuple(t[:-1] if t[0] == "chains" else t[:2])] = t[-1] if t[0] == "chains" else t[2:]
    return out


SHAPES = [(3, 4, 5), (5, 3, 7), (4, 4, 4), (1, 1, 6), (2, 5, 3)]


@pytest.mark.parametrize("npts", [7, 19, 27])
def test_pattern_order(npts):
    off = oracle.pattern(npts)
    assert off.shape == (npts, 3)
    assert np.array_equal(off, workloads.offsets(npts))
    keys = [tuple(o) for o in off]
    assert keys == sorted(keys)
    assert keys[npts // 2] == (0, 0, 0)


@pytest.mark.parametrize("npts", [7, 19, 27])
@pytest.mark.parametrize("shape", SHAPES)
def test_spmv_matches_dense(npts, shape):
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=11, symmetric=False)
    x = workloads.rng(3).uniform(-1, 1, size=shape)
    M = helpers.dense_from_sgdia(A, off, shape)
    y = oracle.spmv(off, A, x)
    ref = M @ x.ravel()
    assert np.allclose(y.ravel(), ref, rtol=0, atol=1e-15 * np.abs(M).sum(1).max() * 4)
    b = workloads.rng(4).uniform(-1, 1, size=shape)
    r = oracle.residual(off, A, b, x)
    assert np.array_equal(r, b - y)


@pytest.mark.parametrize("npts", [7, 19, 27])
@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 4), (1, 1, 5)])
@pytest.mark.parametrize("direction,zero_guess", [(1, 1), (1, 0), (-1, 0)])
def test_gs_bitexact_vs_csr(npts, shape, direction, zero_guess):
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=5, symmetric=False)
    M = helpers.dense_from_sgdia(A, off, shape)
    rd = 1.0 / A[npts // 2]
    g = workloads.rng(9)
    b = g.uniform(-1, 1, size=shape)
    u0 = np.zeros(shape) if zero_guess else g.uniform(-1, 1, size=shape)
    u = oracle.gs_sweep(off, A, rd, b, u0, direction, zero_guess)
    ref = helpers.csr_gs(M, b.ravel(), u0.ravel(), direction, zero_guess)
    assert np.array_equal(u.ravel(), ref)
    # matrix form of the GS formulas: u + (D+L)^-1 (b - A u)  (or D+U)
    tri = np.tril(M) if direction > 0 else np.triu(M)
    mf = u0.ravel() + np.linalg.solve(tri, b.ravel() - M @ u0.ravel())
    assert np.allclose(u.ravel(), mf, rtol=1e-13, atol=1e-13)


def test_gs_single_cell():
    off = workloads.offsets(7)
    A = np.zeros((7, 1))
    A[3] = 4.0
    u = oracle.gs_sweep(off, A, 1.0 / A[3], np.array([[[3.0]]]), np.zeros((1, 1, 1)), 1, 1)
    assert u.ravel()[0] == 3.0 * 0.25


def test_gs_zero_guess_equals_zero_start():
    off = workloads.offsets(27)
    shape = (4, 3, 5)
    A = workloads.random_sgdia(shape, 27, seed=2)
    b = workloads.rng(1).uniform(-1, 1, size=shape)
    rd = 1.0 / A[13]
    u1 = oracle.gs_sweep(off, A, rd, b, np.zeros(shape), 1, 1)
    u2 = oracle.gs_sweep(off, A, rd, b, np.zeros(shape), 1, 0)
    assert np.array_equal(u1, u2)


@pytest.mark.parametrize("npts", [7, 19, 27])
@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 7), (1, 1, 6), (4, 3, 1)])
@pytest.mark.parametrize("direction,zero_guess", [(1, 1), (1, 0), (-1, 0)])
def test_lgs_matches_dense_block_gs(npts, shape, direction, zero_guess):
    """Line GS = block GS with the z-columns as blocks, solved densely."""
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=5, symmetric=False)
    M = helpers.dense_from_sgdia(A, off, shape)
    rden, cp = oracle.tri_factor(off, A, shape)
    g = workloads.rng(9)
    b = g.uniform(-1, 1, size=shape)
    u0 = np.zeros(shape) if zero_guess else g.uniform(-1, 1, size=shape)
    u = oracle.lgs_sweep(off, A, rden, cp, b, u0, direction, zero_guess)
    ref = helpers.line_gs(M, shape, b, u0, direction)
    assert np.allclose(u.ravel(), ref, rtol=1e-13, atol=1e-13)
    # matrix form of the GS formulas with D the column blocks:
    # u + (D + L)^-1 (b - A u), L the couplings to earlier columns
    col = np.arange(M.shape[0]) // shape[2]
    keep = (col[None, :] <= col[:, None]) if direction > 0 else (col[None, :] >= col[:, None])
    mf = u0.ravel() + np.linalg.solve(np.where(keep, M, 0.0), b.ravel() - M @ u0.ravel())
    assert np.allclose(u.ravel(), mf, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("npts", [7, 19, 27])
@pytest.mark.parametrize("direction,zero_guess", [(1, 1), (1, 0), (-1, 0)])
def test_lgs_one_point_columns_is_point_gs(npts, direction, zero_guess):
    """With nz = 1 every column is one point: line GS is point GS, bit for bit."""
    shape = (5, 4, 1)
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=8, symmetric=False)
    rden, cp = oracle.tri_factor(off, A, shape)
    assert np.array_equal(rden, 1.0 / A[npts // 2]) and not cp.any()
    g = workloads.rng(3)
    b = g.uniform(-1, 1, size=shape)
    u0 = np.zeros(shape) if zero_guess else g.uniform(-1, 1, size=shape)
    u = oracle.lgs_sweep(off, A, rden, cp, b, u0, direction, zero_guess)
    ref = oracle.gs_sweep(off, A, 1.0 / A[npts // 2], b, u0, direction, zero_guess)
    assert np.array_equal(u, ref)


def test_thomas_pivots_and_column_solve():
    """On one column the sweep is the Thomas algorithm: the pivots multiply to
    the determinant of the tridiagonal matrix and the solve matches a dense
    solver."""
    shape = (1, 1, 9)
    off = workloads.offsets(19)
    A = workloads.random_sgdia(shape, 19, seed=11, symmetric=False)
    M = helpers.dense_from_sgdia(A, off, shape)
    rden, cp = oracle.tri_factor(off, A, shape)
    assert np.isclose(np.prod(1.0 / rden), np.linalg.det(M), rtol=1e-12)
    b = workloads.rng(2).uniform(-1, 1, size=shape)
    u = oracle.lgs_sweep(off, A, rden, cp, b, np.zeros(shape), 1, 1)
    assert np.allclose(u.ravel(), np.linalg.solve(M, b.ravel()), rtol=1e-14, atol=1e-14)


def test_lgs_exact_when_columns_decouple():
    """Without couplings between columns one sweep solves A u = b."""
    shape = (3, 4, 6)
    off = workloads.offsets(27)
    A = workloads.random_sgdia(shape, 27, seed=6, symmetric=False)
    for s, (dx, dy, dz) in enumerate(off):
        if dx or dy:
            A[s] = 0.0
    M = helpers.dense_from_sgdia(A, off, shape)
    rden, cp = oracle.tri_factor(off, A, shape)
    b = workloads.rng(4).uniform(-1, 1, size=shape)
    for d in (1, -1):
        u = oracle.lgs_sweep(off, A, rden, cp, b, np.zeros(shape), d, 1 if d > 0 else 0)
        assert np.allclose(u.ravel(), np.linalg.solve(M, b.ravel()), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("npts", [7, 19, 27])
@pytest.mark.parametrize("shape", [(3, 4, 5), (4, 2, 3)])
def test_ilu0_property(npts, shape):
    """(L U)_ij = a_ij on the mask (defining property of ILU(0))."""
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=21, symmetric=False)
    L, U, rU = oracle.ilu0(off, A, shape)
    Lm = helpers.dense_from_sgdia(L, off, shape) + np.eye(int(np.prod(shape)))
    Um = helpers.dense_from_sgdia(U, off, shape)
    M = helpers.dense_from_sgdia(A, off, shape)
    mask = helpers.dense_from_sgdia(np.ones_like(A), off, shape) != 0
    LU = Lm @ Um
    scale = np.abs(M).max()
    assert np.abs((LU - M)[mask]).max() <= 1e-14 * scale
    assert np.allclose(rU, 1.0 / np.diag(Um), rtol=0, atol=0)
    # the triangular solves invert the factors
    r = workloads.rng(2).uniform(-1, 1, size=shape)
    y = oracle.tri_solve(off, L, None, r, 0)
    z = oracle.tri_solve(off, U, rU, y, 1)
    assert np.allclose(LU @ z.ravel(), r.ravel(), rtol=0, atol=1e-13)


@pytest.mark.parametrize("apat", [7, 19, 27])
@pytest.mark.parametrize("mpat", [7, 19, 27])
def test_ilu0_mask_property(apat, mpat):
    """ILU(0) on a mask other than A's pattern (Sec. 4.2.3): (L U)_ij = a_ij
    at every position of the mask, with a_ij = 0 where A has no such offset
    (fill kept) and A's entries outside the mask dropped."""
    shape = (4, 3, 5)
    off = workloads.offsets(apat)
    offm = workloads.offsets(mpat)
    A = workloads.random_sgdia(shape, apat, seed=23, symmetric=False)
    L, U, rU = oracle.ilu0_mask(off, A, offm, shape)
    n = int(np.prod(shape))
    Lm = helpers.dense_from_sgdia(L, offm, shape) + np.eye(n)
    Um = helpers.dense_from_sgdia(U, offm, shape)
    M = helpers.dense_from_sgdia(A, off, shape)
    mask = helpers.dense_from_sgdia(np.ones((mpat, n)), offm, shape) != 0
    LU = Lm @ Um
    assert np.abs((LU - M)[mask]).max() <= 1e-14 * np.abs(M).max()
    assert np.allclose(rU, 1.0 / np.diag(Um), rtol=0, atol=0)
    r = workloads.rng(2).uniform(-1, 1, size=shape)
    z = oracle.tri_solve(offm, U, rU, oracle.tri_solve(offm, L, None, r, 0), 1)
    assert np.allclose(LU @ z.ravel(), r.ravel(), rtol=0, atol=1e-13)
    if mpat == apat:
        L0, U0, rU0 = oracle.ilu0(off, A, shape)
        assert np.array_equal(L, L0) and np.array_equal(U, U0) and np.array_equal(rU, rU0)


def test_ilu_mask_more_fill_fewer_iterations():
    """A 3d7 operator smoothed with ILU(0) on its own mask, on 3d19 and on
    3d27: more fill-in gives a stronger smoother (fewer PCG iterations)."""
    shape = (24, 24, 24)
    A, b = workloads.diffusion7(shape, seed=2, nspheres=2, rmin=3.0, rmax=6.0)
    its = []
    for m in (0, 19, 27):
        H = oracle.Hierarchy(shape, 7, A, smoother="ilu0", ilu_mask=m)
        assert H.level_info(0)["Sm"] == (m or 7) and H.level_info(1)["Sm"] == 27
        x, st, it, rel = H.pcg(b.reshape(shape), 1e-9, 200)
        assert st == 0 and rel < 1e-9
        its.append(it)
    assert its[0] > its[1] >= its[2], its


def test_ilu0_exact_on_tridiagonal():
    """On a 1 x 1 x n grid the 3d7 operator is tridiagonal and ILU(0) = LU."""
    off = workloads.offsets(7)
    shape = (1, 1, 9)
    A = workloads.random_sgdia(shape, 7, seed=4, symmetric=False)
    L, U, rU = oracle.ilu0(off, A, shape)
    b = workloads.rng(5).uniform(-1, 1, size=shape)
    z = oracle.tri_solve(off, U, rU, oracle.tri_solve(off, L, None, b, 0), 1)
    M = helpers.dense_from_sgdia(A, off, shape)
    assert np.allclose(z.ravel(), np.linalg.solve(M, b.ravel()), rtol=0, atol=1e-15)


def test_ilu0_diagonal():
    off = workloads.offsets(27)
    shape = (2, 3, 3)
    A = np.zeros((27, 18))
    A[13] = workloads.rng(1).uniform(1, 2, size=18)
    L, U, rU = oracle.ilu0(off, A, shape)
    assert not L.any() and np.array_equal(U, A)


@pytest.mark.parametrize("shape", [(6, 5, 7), (8, 8, 8), (5, 6, 4), (7, 3, 9)])
@pytest.mark.parametrize("cmask", [7, 3, 1, 6])
def test_restrict_prolong_are_transposes(shape, cmask):
    P, cs = helpers.interp_matrix(shape, cmask)
    g = workloads.rng(8)
    r = g.uniform(-1, 1, size=shape)
    rc = oracle.restrict(r, cmask)
    assert rc.shape == cs
    assert np.allclose(rc.ravel(), P.T @ r.ravel(), rtol=0, atol=1e-14)
    e = g.uniform(-1, 1, size=cs)
    u = g.uniform(-1, 1, size=shape)
    out = oracle.prolong_add(u, e, cmask)
    assert np.allclose(out.ravel(), u.ravel() + P @ e.ravel(), rtol=0, atol=1e-14)
    # interior fine points: P 1 = 1
    ones = oracle.prolong_add(np.zeros(shape), np.ones(cs), cmask)
    inner = tuple(slice(1, n - 1) if (cmask >> a) & 1 else slice(None) for a, n in enumerate(shape))
    assert np.all(ones[inner] == 1.0)


@pytest.mark.parametrize("npts", [7, 19, 27])
@pytest.mark.parametrize("shape,cmask", [((6, 5, 7), 7), ((8, 6, 5), 3), ((5, 8, 6), 5), ((4, 7, 9), 6),
                                         ((7, 4, 4), 1)])
def test_rap_matches_brute_force(npts, shape, cmask):
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=31, symmetric=False)
    Ac = oracle.rap(off, A, shape, cmask)
    M = helpers.dense_from_sgdia(A, off, shape)
    P, cs = helpers.interp_matrix(shape, cmask)
    Mc = P.T @ M @ P
    ref = helpers.sgdia_from_dense27(Mc, cs, tol=1e-13 * np.abs(Mc).max())
    assert np.abs(Ac - ref).max() <= 1e-13 * np.abs(ref).max()


def test_rap_block_matches_brute_force():
    shape = (5, 6, 4)
    off = workloads.offsets(27)
    A = workloads.random_sgdia(shape, 27, seed=3, block=3)
    Ac = oracle.rap(off, A, shape, 7, bs=3)
    M = helpers.dense_from_sgdia(A, off, shape, bs=3)
    P, cs = helpers.interp_matrix(shape, 7)
    P3 = np.kron(P, np.eye(3))
    ref = helpers.sgdia_from_dense27(P3.T @ M @ P3, cs, bs=3, tol=1e-12)
    assert np.abs(Ac - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("npts,shape,cmask,bs", [(19, (8, 6, 5), 3, 1), (7, (6, 5, 7), 7, 1), (27, (5, 6, 4), 7, 3)])
def test_rap_points_match_whole_and_brute_force(npts, shape, cmask, bs):
    """Rows of the stencil product at listed coarse points (shuffled, with
    repeats) equal the whole product's rows and the brute-force P^T A P."""
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=37, block=bs)
    Ac = oracle.rap(off, A, shape, cmask, bs=bs)
    cs = oracle.coarse_dims(shape, cmask)
    nc = int(np.prod(cs))
    pts = workloads.rng(12).permutation(np.concatenate([np.arange(nc), [0, nc - 1]]))
    Ap = oracle.rap_points(off, A, shape, cmask, pts, bs=bs)
    assert np.array_equal(Ap, Ac[:, pts])
    M = helpers.dense_from_sgdia(A, off, shape, bs=bs)
    P, _ = helpers.interp_matrix(shape, cmask)
    P = np.kron(P, np.eye(bs))
    ref = helpers.sgdia_from_dense27(P.T @ M @ P, cs, bs=bs, tol=1e-12)
    assert np.abs(Ap - ref[:, pts]).max() <= 1e-13 * np.abs(ref).max()


def _tridiag(n, c, d):
    T = np.diag(np.full(n, d)) + np.diag(np.full(n - 1, c), 1) + np.diag(np.full(n - 1, c), -1)
    return T


def test_rap_laplace_closed_form_bitexact():
    """A = T(x)I(x)I + I(x)T(x)I + I(x)I(x)T and P = p(x)p(x)p give coarse
    levels T_l(x)M_l(x)M_l + ... with T_{l+1} = p^T T_l p and M_{l+1} = p^T M_l p.
    All entries are dyadic rationals, so the stencil RAP must be exact."""
    n = 32
    A, _ = workloads.poisson7(n)
    off = workloads.offsets(7)
    T = _tridiag(n, -1.0, 2.0)
    Mm = np.eye(n)
    shape = (n, n, n)
    Acur, offcur = A, off
    expect_center = {1: 27 / 4, 2: 363 / 32}
    expect_face = {1: -3 / 8, 2: -11 / 64}
    expect_edge = {1: -5 / 16, 2: -85 / 128}
    expect_corner = {1: -3 / 32, 2: -75 / 256}
    for lev in (1, 2, 3):
        Acur = oracle.rap(offcur, Acur, shape, 7)
        P1, _ = helpers.interp_matrix((shape[0], 1, 1), 1)
        T = P1.T @ T @ P1
        Mm = P1.T @ Mm @ P1
        shape = tuple(v // 2 for v in shape)
        offcur = workloads.offsets(27)
        ref = np.kron(np.kron(T, Mm), Mm) + np.kron(np.kron(Mm, T), Mm) + np.kron(np.kron(Mm, Mm), T)
        refs = helpers.sgdia_from_dense27(ref, shape) if shape[0] <= 8 else None
        if refs is not None:
            assert np.array_equal(Acur, refs)
        else:
            # check a band of rows against the Kronecker product
            N = int(np.prod(shape))
            for i in range(0, N, 97):
                x, y, z = i // (shape[1] * shape[2]), (i // shape[2]) % shape[1], i % shape[2]
                for s in range(27):
                    dx, dy, dz = s // 9 - 1, (s // 3) % 3 - 1, s % 3 - 1
                    a, b, c = x + dx, y + dy, z + dz
                    if 0 <= a < shape[0] and 0 <= b < shape[1] and 0 <= c < shape[2]:
                        j = (a * shape[1] + b) * shape[2] + c
                        tv = T[x, a] * Mm[y, b] * Mm[z, c] + Mm[x, a] * T[y, b] * Mm[z, c] + Mm[x, a] * Mm[y, b] * T[z, c]
                        assert Acur[s, i] == tv
        if lev in expect_center:
            m = shape[0] // 2
            i = (m * shape[1] + m) * shape[2] + m
            col = Acur[:, i]
            assert col[13] == expect_center[lev]
            assert col[4] == expect_face[lev] and col[12] == expect_face[lev]
            assert col[1] == expect_edge[lev]
            assert col[0] == expect_corner[lev]


@pytest.mark.parametrize("npts", [7, 19, 27])
def test_rap_symmetry(npts):
    shape = (9, 8, 7)
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=41, symmetric=True)
    Ac = oracle.rap(off, A, shape, 7)
    cs = (4, 4, 3)
    Mc = helpers.dense_from_sgdia(Ac, workloads.offsets(27), cs)
    assert np.abs(Mc - Mc.T).max() <= 1e-14 * np.abs(Mc).max()


@pytest.mark.parametrize("npts", [7, 19, 27])
@pytest.mark.parametrize("cmask", [7, 3])
def test_rap_zero_row_sums(npts, cmask):
    """Neumann-like operator (A 1 = 0): coarse rows away from the boundary,
    where P 1 = 1 on the whole chain support, keep zero row sums."""
    shape = (14, 13, 12)
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=7, symmetric=True).reshape((npts,) + shape)
    c = npts // 2
    A[c] = 0.0
    A[c] = -A.sum(axis=0)
    A = A.reshape(npts, -1)
    Ac = oracle.rap(off, A, shape, cmask)
    cs = oracle.coarse_dims(shape, cmask)
    sums = Ac.sum(axis=0).reshape(cs)
    inner = tuple(slice(1, n - 1) if (cmask >> a) & 1 else slice(None) for a, n in enumerate(cs))
    assert np.abs(sums[inner]).max() <= 1e-14 * np.abs(Ac).max() * 27


def test_chain_counts_table():
    tab = _gold_tables()
    for npts, key in ((19, ("chains", "3d27v", "3d19", "3d27v")), (27, ("chains", "3d27v", "3d27", "3d27v"))):
        off = workloads.offsets(npts)
        tot = sum(len(oracle.rap_chains(off, 7, n)) for n in range(27))
        assert tot == int(tab[key])
    # 3d7 fine pattern: centre 5^3 plus six faces at 4*5*5 each (per-axis count)
    tot7 = sum(len(oracle.rap_chains(workloads.offsets(7), 7, n)) for n in range(27))
    assert tot7 == 5 ** 3 + 6 * 4 * 5 * 5 == 725
    # semi-coarsening in x,y: the z factor contributes exactly one pair
    tot7xy = sum(len(oracle.rap_chains(workloads.offsets(7), 3, n)) for n in range(27))
    assert tot7xy == 5 ** 2 + 4 * 4 * 5 + 2 * 5 ** 2 == 155


@pytest.mark.parametrize("shape", [(6, 5, 7), (8, 8, 8), (5, 6, 4), (7, 3, 9)])
@pytest.mark.parametrize("cmask", [7, 3, 1, 6])
def test_cell_transfers_are_transposes(shape, cmask):
    """Cell_3d8 pair: prolongation is piecewise constant, restriction its
    transpose (sum over the children), n_c = ceil(n_f / 2)."""
    P, cs = helpers.cell_interp_matrix(shape, cmask)
    g = workloads.rng(8)
    r = g.uniform(-1, 1, size=shape)
    rc = oracle.restrict_cc(r, cmask)
    assert rc.shape == cs
    assert np.allclose(rc.ravel(), P.T @ r.ravel(), rtol=0, atol=1e-14)
    u = g.uniform(-1, 1, size=shape)
    e = g.uniform(-1, 1, size=cs)
    assert np.array_equal(oracle.prolong_add_cc(u, e, cmask).ravel(), u.ravel() + P @ e.ravel())


@pytest.mark.parametrize("npts", [7, 19, 27])
@pytest.mark.parametrize("shape,cmask", [((6, 5, 7), 7), ((8, 6, 5), 3), ((5, 8, 6), 5), ((4, 7, 9), 6),
                                         ((7, 7, 7), 7)])
def test_rap_cc_matches_dense(npts, shape, cmask):
    """Stencil product of the cell-centred pair = P^T A P assembled densely;
    the coarse operator keeps the fine pattern (no entry outside it)."""
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=13, symmetric=False)
    M = helpers.dense_from_sgdia(A, off, shape)
    P, cs = helpers.cell_interp_matrix(shape, cmask)
    Ac = oracle.rap_cc(off, A, shape, cmask)
    assert np.allclose(helpers.dense_from_sgdia(Ac, off, cs), P.T @ M @ P, rtol=0, atol=1e-13 * np.abs(M).max())


def test_rap_cc_chain_count_and_symmetry():
    tab = _gold_tables()
    assert oracle.rap_cc_chains(workloads.offsets(7), 7) == int(tab[("chains", "3d8c", "3d7", "3d8c")])
    # every (child, fine offset) pair lands on one coarse offset
    assert oracle.rap_cc_chains(workloads.offsets(27), 7) == 8 * 27
    assert oracle.rap_cc_chains(workloads.offsets(19), 3) == 4 * 19
    shape = (8, 7, 6)
    for npts in (7, 19, 27):
        off = workloads.offsets(npts)
        A = workloads.random_sgdia(shape, npts, seed=5, symmetric=True)
        cs = oracle.coarse_dims(shape, 7, cell=True)
        Mc = helpers.dense_from_sgdia(oracle.rap_cc(off, A, shape, 7), off, cs)
        assert np.allclose(Mc, Mc.T, rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape", [(6, 5, 7), (8, 8, 8), (7, 3, 9)])
@pytest.mark.parametrize("cmask", [7, 3, 6])
def test_cell_trilinear_interpolation(shape, cmask):
    """3d64c interpolation against its explicit matrix; interior rows sum to 1
    (constants are interpolated exactly away from the boundary)."""
    P, cs = helpers.cell_trilinear_matrix(shape, cmask)
    g = workloads.rng(3)
    u = g.uniform(-1, 1, size=shape)
    e = g.uniform(-1, 1, size=cs)
    assert np.allclose(oracle.prolong_add_c64(u, e, cmask).ravel(), u.ravel() + P @ e.ravel(), rtol=0, atol=1e-15)
    one = oracle.prolong_add_c64(np.zeros(shape), np.ones(cs), cmask)
    inner = tuple(slice(1, n - 1) if (cmask >> a) & 1 else slice(None) for a, n in enumerate(shape))
    assert np.array_equal(one[inner], np.ones_like(one[inner]))


@pytest.mark.parametrize("npts", [7, 19, 27])
@pytest.mark.parametrize("shape,cmask", [((6, 5, 7), 7), ((8, 6, 5), 3), ((5, 8, 6), 5), ((7, 7, 7), 7)])
def test_rap_c64_matches_dense(npts, shape, cmask):
    """Stencil product of the Cell_3d8 restriction and the 3d64c
    interpolation = R A P assembled densely (R = transpose of the
    piecewise-constant interpolation); 27-point coarse operator."""
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=13, symmetric=False)
    M = helpers.dense_from_sgdia(A, off, shape)
    R, cs = helpers.cell_interp_matrix(shape, cmask)
    P, _ = helpers.cell_trilinear_matrix(shape, cmask)
    Ac = oracle.rap_c64(off, A, shape, cmask)
    ref = R.T @ M @ P
    assert np.allclose(helpers.dense_from_sgdia(Ac, workloads.offsets(27), cs), ref, rtol=0,
                       atol=1e-13 * np.abs(M).max())


def test_rap_c64_chain_counts():
    tab = _gold_tables()
    for npts in (19, 27):
        assert oracle.rap_c64_chains(workloads.offsets(npts), 7) == int(tab[("chains", "3d8c", f"3d{npts}", "3d64c")])
    assert oracle.rap_c64_chains(workloads.offsets(7), 7) == 8 * 7 * 8


def test_cell_trilinear_hierarchy_converges():
    """Cell_3d8 restriction with 3d64c interpolation (the paper's Laplace
    setting): 27-point coarse levels, PCG on the Laplacian as fast as the
    vertex-centred hierarchy; R != P^T makes the cycle non-symmetric, so the
    high-contrast diffusion case is solved with GMRES."""
    A, b = workloads.poisson7(24)
    its = {}
    for interp in ("vertex", "cell_trilinear"):
        H = oracle.Hierarchy((24, 24, 24), 7, A, interp=interp)
        _, st, its[interp], rel = H.pcg(b.reshape(24, 24, 24), 1e-9, 100)
        assert st == 0 and rel < 1e-9
    assert H.level_info(1)["S"] == 27 and H.level_info(1)["dims"] == (12, 12, 12)
    assert its["cell_trilinear"] <= its["vertex"] + 1
    shape = (24, 24, 24)
    A, b = workloads.diffusion7(shape, seed=2, nspheres=3, rmin=3.0, rmax=8.0)
    H = oracle.Hierarchy(shape, 7, A, interp="cell_trilinear")
    _, st, it, rel = H.gmres(b.reshape(shape), 1e-9, 200)
    assert st == 0 and rel < 1e-9


def test_od_interpolation_is_trilinear_for_the_laplacian():
    """On the constant-coefficient 3d7 Laplacian the collapsed stencils give
    weights 1/2, 1/4, 1/8: away from the boundary the operator-dependent
    interpolation is the trilinear one, exactly."""
    n = 16
    A, _ = workloads.poisson7(n)
    W = oracle.od_weights(workloads.offsets(7), A, (n, n, n), 7)
    P, _ = helpers.od_matrix(W, (n, n, n), 7)
    T, _ = helpers.interp_matrix((n, n, n), 7)
    inner = [helpers.lin((n, n, n), x, y, z) for x in range(2, n - 2) for y in range(2, n - 2) for z in range(2, n - 2)]
    assert np.array_equal(P[inner], T[inner])


def test_od_interpolation_closed_forms():
    """1D: weight -a_(i,i+-1) / a_ii; zero row sums: constants are
    interpolated exactly (the weights of each fine point sum to 1)."""
    shape = (1, 1, 13)
    off = workloads.offsets(7)
    A = workloads.random_sgdia(shape, 7, seed=3, symmetric=False)
    W = oracle.od_weights(off, A, shape, 4)
    for z in range(0, 13, 2):
        if z > 0:
            assert W[0, z] == -(A[2, z] * (1.0 / A[3, z]))
        if z < 12:
            assert W[1, z] == -(A[4, z] * (1.0 / A[3, z]))
    shape = (9, 8, 7)
    for npts in (7, 19, 27):
        off = workloads.offsets(npts)
        A = workloads.random_sgdia(shape, npts, seed=4, symmetric=False)
        M = helpers.dense_from_sgdia(A, off, shape)
        A[npts // 2] -= M.sum(axis=1)  # zero row sums (Neumann-like)
        for cmask in (7, 3):
            W = oracle.od_weights(off, A, shape, cmask)
            P, _ = helpers.od_matrix(W, shape, cmask)
            assert np.allclose(P.sum(axis=1), 1.0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("npts", [7, 19, 27])
@pytest.mark.parametrize("shape,cmask", [((7, 6, 9), 7), ((8, 6, 5), 3), ((9, 9, 9), 7), ((6, 7, 8), 6)])
def test_od_transfers_and_rap_match_dense(npts, shape, cmask):
    """Restriction = P^T, prolongation = P, and the stencil product equals
    P^T A P assembled densely from the weights."""
    off = workloads.offsets(npts)
    A = workloads.random_sgdia(shape, npts, seed=19, symmetric=False)
    W = oracle.od_weights(off, A, shape, cmask)
    P, cs = helpers.od_matrix(W, shape, cmask)
    M = helpers.dense_from_sgdia(A, off, shape)
    g = workloads.rng(6)
    r = g.uniform(-1, 1, size=shape)
    e = g.uniform(-1, 1, size=cs)
    assert np.allclose(oracle.restrict_od(r, W, cmask).ravel(), P.T @ r.ravel(), rtol=0, atol=1e-14)
    assert np.allclose(oracle.prolong_add_od(r, W, e, cmask).ravel(), r.ravel() + P @ e.ravel(), rtol=0, atol=1e-14)
    Ac = oracle.rap_od(off, A, shape, cmask, W)
    assert np.allclose(helpers.dense_from_sgdia(Ac, workloads.offsets(27), cs), P.T @ M @ P, rtol=0,
                       atol=1e-13 * np.abs(M).max())


@pytest.mark.parametrize("shape,cmask", [((9, 8, 7), 7), ((8, 6, 5), 3), ((6, 7, 8), 6)])
def test_od_rap_points_match_dense(shape, cmask):
    """Rows of the stencil product at listed coarse points (in a shuffled
    order, with repeats) equal the whole product's rows and the rows of
    P^T A P assembled densely from the weights."""
    off = workloads.offsets(7)
    A = workloads.random_sgdia(shape, 7, seed=23, symmetric=False)
    W = oracle.od_weights(off, A, shape, cmask)
    P, cs = helpers.od_matrix(W, shape, cmask)
    nc = int(np.prod(cs))
    pts = workloads.rng(8).permutation(np.concatenate([np.arange(nc), [0, nc - 1]]))
    Ap = oracle.rap_od_points(off, A, shape, cmask, W, pts)
    Ac = oracle.rap_od(off, A, shape, cmask, W)
    assert np.array_equal(Ap, Ac[:, pts])
    D = P.T @ helpers.dense_from_sgdia(A, off, shape) @ P
    rows = helpers.dense_from_sgdia(Ac, workloads.offsets(27), cs)
    assert np.allclose(rows[pts], D[pts], rtol=0, atol=1e-13 * np.abs(A).max())


def test_od_hierarchy_symmetric_and_faster_on_high_contrast():
    """R = P^T keeps the cycle symmetric; on the high-contrast diffusion
    stand-in the operator-dependent interpolation needs fewer PCG iterations
    than the trilinear one."""
    shape = (16, 12, 10)
    A = workloads.random_sgdia(shape, 7, seed=17, symmetric=True)
    H = oracle.Hierarchy(shape, 7, A, interp="operator")
    g = workloads.rng(5)
    x = g.uniform(-1, 1, size=shape)
    y = g.uniform(-1, 1, size=shape)
    a = np.dot(H.apply(x).ravel(), y.ravel())
    b = np.dot(x.ravel(), H.apply(y).ravel())
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)
    shape = (32, 32, 32)
    A, b = workloads.diffusion7(shape, seed=2, nspheres=3, rmin=3.0, rmax=8.0)
    its = {}
    for interp in ("vertex", "operator"):
        _, st, its[interp], rel = oracle.Hierarchy(shape, 7, A, interp=interp).pcg(b.reshape(shape), 1e-9, 200)
        assert st == 0 and rel < 1e-9
    assert its["operator"] < its["vertex"], its


@pytest.mark.parametrize("npts", [7, 27])
def test_cell_vcycle_symmetric_and_pcg(npts):
    """Cell-centred hierarchy: every level keeps the fine pattern, the V(1,1)
    symmetric GS cycle is symmetric and PCG converges on the 3d7 Laplacian."""
    shape = (16, 12, 10)
    A = workloads.random_sgdia(shape, npts, seed=17, symmetric=True)
    H = oracle.Hierarchy(shape, npts, A, interp="cell")
    assert H.nlev >= 2 and all(H.level_info(l)["S"] == npts for l in range(H.nlev))
    assert H.level_info(1)["dims"] == (8, 6, 5)
    g = workloads.rng(5)
    x = g.uniform(-1, 1, size=shape)
    y = g.uniform(-1, 1, size=shape)
    a = np.dot(H.apply(x).ravel(), y.ravel())
    b = np.dot(x.ravel(), H.apply(y).ravel())
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)
    A7, b7 = workloads.poisson7(24)
    Hc = oracle.Hierarchy((24, 24, 24), 7, A7, interp="cell")
    _, st, it, rel = Hc.pcg(b7.reshape(24, 24, 24), 1e-9, 200)
    assert st == 0 and rel < 1e-9


def test_listing1_chain_set():
    """2D example: R = 2d9, A = 2d5, P = 2d9, coarse neighbour (-1, +1)."""
    exp = set()
    with open(os.path.join(GOLD, "listing1_chains.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            exp.add(tuple(int(v) for v in line.split()))
    off2d5 = np.array([(-1, 0, 0), (0, -1, 0), (0, 0, 0), (0, 1, 0), (1, 0, 0)], np.int32)
    n27 = (0 * 9) + (2 * 3) + 1  # n = (-1, +1, 0)
    ch = oracle.rap_chains(off2d5, 3, n27)
    got = set()
    for ri, s, pi in ch:
        rho = (ri // 9 - 1, (ri // 3) % 3 - 1, ri % 3 - 1)
        d = (pi // 9 - 1, (pi // 3) % 3 - 1, pi % 3 - 1)
        assert rho[2] == 0 and d[2] == 0
        got.add(((rho[0] + 1) * 3 + rho[1] + 1, int(s), (d[0] + 1) * 3 + d[1] + 1))
    assert got == exp
    # the fine elements u of the example's third group: P_to & Ngb(F_u)
    # = C_i + {(-2,1), (-1,1), (-1,2)} when u = fine(C_i) + (-1, +1)
    vs = set()
    for ri, s, pi in ch:
        if ri // 9 - 1 == -1 and (ri // 3) % 3 - 1 == 1:
            rho = (-1, 1)
            a = tuple(off2d5[s][:2])
            vs.add((rho[0] + a[0], rho[1] + a[1]))
    assert vs == {(-2, 1), (-1, 1), (-1, 2)}


def test_dense_lu_matches_numpy():
    g = workloads.rng(12)
    M = g.uniform(-1, 1, size=(40, 40)) + 5 * np.eye(40)
    M[[0, 3]] = M[[3, 0]]
    b = g.uniform(-1, 1, size=40)
    assert np.allclose(oracle.lu_solve(M, b), np.linalg.solve(M, b), rtol=0, atol=1e-13)


@pytest.mark.filterwarnings("ignore:overflow")
def test_f16_conversion_matches_numpy():
    g = workloads.rng(3)
    vals = np.concatenate([
        g.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** g.integers(-9, 6, 20000).astype(np.float32),
        np.float32([0.0, -0.0, 65504.0, 65519.0, 65520.0, 1e-8, 2.0 ** -25, 2.0 ** -24, 3 * 2.0 ** -26,
                    2.0 ** -14, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, np.inf, -np.inf]),
    ]).astype(np.float32)
    for v in vals:
        h = oracle.f32_to_f16_bits(v)
        ref = np.float32(v).astype(np.float16).view(np.uint16)
        assert h == int(ref), (v, h, ref)
        back = oracle.f16_bits_to_f32(h)
        assert np.float32(back) == np.float16(v).astype(np.float32) or (np.isnan(back) and np.isnan(v))


def _sym_hierarchy(shape, npts, smoother="gs", block=1):
    A = workloads.random_sgdia(shape, npts, seed=17, symmetric=True, block=block)
    return oracle.Hierarchy(shape, npts, A, block=block, smoother=smoother), A


@pytest.mark.parametrize("npts", [7, 27])
def test_vcycle_symmetric(npts):
    """Forward GS before and backward GS after the coarse correction with
    R = P^T give a symmetric preconditioner: <Mx, y> = <x, My>."""
    shape = (16, 12, 10)
    H, _ = _sym_hierarchy(shape, npts)
    assert H.nlev >= 2
    g = workloads.rng(5)
    x = g.uniform(-1, 1, size=shape)
    y = g.uniform(-1, 1, size=shape)
    a = np.dot(H.apply(x).ravel(), y.ravel())
    b = np.dot(x.ravel(), H.apply(y).ravel())
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


def test_vcycle_lgs_symmetric():
    """Forward line GS before and backward line GS after the coarse
    correction also give a symmetric preconditioner."""
    shape = (16, 12, 10)
    H, _ = _sym_hierarchy(shape, 19, smoother="lgs")
    assert H.nlev >= 2
    g = workloads.rng(7)
    x = g.uniform(-1, 1, size=shape)
    y = g.uniform(-1, 1, size=shape)
    a = np.dot(H.apply(x).ravel(), y.ravel())
    b = np.dot(x.ravel(), H.apply(y).ravel())
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


def test_lgs_beats_point_gs_on_strong_vertical_coupling():
    """Grid-aligned anisotropy (vertical coupling 100x the horizontal): line
    GS over z-columns needs far fewer PCG iterations than point GS."""
    shape = (24, 24, 16)
    A, b = workloads.weather19(shape, seed=3, skew=0.0)
    b = b.reshape(shape)
    its = {}
    for sm in ("gs", "lgs"):
        H = oracle.Hierarchy(shape, 19, A, smoother=sm, coarsen="semi_xy")
        x, st, it, rel = H.pcg(b, 1e-9, 300)
        assert st == 0 and rel < 1e-9
        its[sm] = it
    assert its["lgs"] * 2 <= its["gs"], its


def test_vcycle_block_symmetric():
    shape = (8, 9, 8)
    H, _ = _sym_hierarchy(shape, 27, block=3)
    g = workloads.rng(6)
    x = g.uniform(-1, 1, size=shape + (3,))
    y = g.uniform(-1, 1, size=shape + (3,))
    a = np.dot(H.apply(x).ravel(), y.ravel())
    b = np.dot(x.ravel(), H.apply(y).ravel())
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


def test_block_gs_exact_without_coupling():
    shape = (3, 3, 4)
    off = workloads.offsets(27)
    A = workloads.random_sgdia(shape, 27, seed=4, block=3)
    A[: 13 * 9] = 0.0
    A[14 * 9:] = 0.0
    D = oracle.block_dinv(off, A, shape)
    b = workloads.rng(1).uniform(-1, 1, size=shape + (3,))
    u = oracle.bgs_sweep(off, A, D, b, np.zeros_like(b), 1, 1)
    M = helpers.dense_from_sgdia(A, off, shape, bs=3)
    assert np.allclose(u.ravel(), np.linalg.solve(M, b.ravel()), rtol=0, atol=1e-14)
    assert np.allclose(oracle.bspmv(off, A, u).ravel(), M @ u.ravel(), rtol=0, atol=1e-14)


def _coupled_block_system(shape, seed):
    """27-point 3x3-block operator with every off-centre block nonzero and
    non-symmetric (neither A_ij = A_ji^T nor symmetric blocks), plus the
    inverses of its diagonal blocks computed by numpy."""
    off = workloads.offsets(27)
    A = workloads.random_sgdia(shape, 27, seed=seed, block=3, symmetric=False)
    N = int(np.prod(shape))
    A = A.reshape(27 * 9, N)
    g = workloads.rng(seed + 100)
    # perturb the diagonal blocks so that they are not symmetric either
    A[13 * 9:14 * 9] *= g.uniform(0.9, 1.1, size=(9, N))
    D = np.linalg.inv(A[13 * 9:14 * 9].T.reshape(N, 3, 3))
    Dl = np.ascontiguousarray(D.reshape(N, 9).T)  # oracle layout Dinv[(r*3+c)*N + i]
    return off, A, D, Dl


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 7), (4, 2, 3)])
def test_block_spmv_full_coupling_matches_dense(shape):
    """Block SpMV with all 27 blocks nonzero against the explicit matrix
    assembled entry by entry: a wrong neighbour index, block transpose or
    skipped block fails."""
    off, A, _, _ = _coupled_block_system(shape, 11)
    M = helpers.dense_from_sgdia(A, off, shape, bs=3)
    assert np.abs(M - M.T).max() > 0.1
    x = workloads.rng(12).uniform(-1, 1, size=tuple(shape) + (3,))
    y = oracle.bspmv(off, A, x).ravel()
    ref = M @ x.ravel()
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(M).sum(axis=1).max()


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 7), (4, 2, 3)])
@pytest.mark.parametrize("direction,zero_guess", [(1, 1), (1, 0), (-1, 0)])
def test_block_gs_full_coupling_bitexact_vs_dense(shape, direction, zero_guess):
    """Point-block GS with all 27 blocks nonzero and non-symmetric against a
    sequential block GS on the explicit matrix (old-value blocks, then
    new-value blocks, then the diagonal-block inverse row by row), bit for
    bit; and against the matrix form of one sweep, u = (D+L)^-1 (b - U u0)
    forward and (D+U)^-1 (b - L u0) backward."""
    off, A, D, Dl = _coupled_block_system(shape, 21)
    M = helpers.dense_from_sgdia(A, off, shape, bs=3)
    g = workloads.rng(22)
    b = g.uniform(-1, 1, size=tuple(shape) + (3,))
    u0 = np.zeros_like(b) if zero_guess else g.uniform(-1, 1, size=b.shape)
    u = oracle.bgs_sweep(off, A, Dl, b, u0, direction, zero_guess).ravel()
    ref = helpers.block_gs(M, D, b.ravel(), u0.ravel(), direction, zero_guess)
    assert np.array_equal(u, ref)
    # matrix form (node blocks: lower = j < i, upper = j > i)
    n3 = M.shape[0]
    node = np.arange(n3) // 3
    low = node[:, None] > node[None, :]
    upp = node[:, None] < node[None, :]
    if direction > 0:
        K, rhs = np.where(~upp, M, 0.0), b.ravel() - np.where(upp, M, 0.0) @ u0.ravel()
    else:
        K, rhs = np.where(~low, M, 0.0), b.ravel() - np.where(low, M, 0.0) @ u0.ravel()
    assert np.allclose(u, np.linalg.solve(K, rhs), rtol=0, atol=1e-12)


def test_block_dinv_matches_numpy_inverse():
    off, A, D, Dl = _coupled_block_system((3, 3, 4), 31)
    got = oracle.block_dinv(off, A, (3, 3, 4))
    assert np.allclose(got.reshape(9, -1), Dl.reshape(9, -1), rtol=1e-13, atol=1e-15)


def test_vcycle_single_level_is_exact_and_pcg_one_iteration():
    """A grid too small to coarsen gives a one-level hierarchy: M = A^-1, so
    PCG converges in one iteration."""
    shape = (4, 5, 6)
    H, A = _sym_hierarchy(shape, 7)
    assert H.nlev == 1
    b = workloads.rng(2).uniform(-1, 1, size=shape)
    M = helpers.dense_from_sgdia(A, workloads.offsets(7), shape)
    assert np.allclose(H.apply(b).ravel(), np.linalg.solve(M, b.ravel()), rtol=0, atol=1e-13)
    x, st, it, rel = H.pcg(b, 1e-10, 50)
    assert st == 0 and it == 1 and rel < 1e-10


def test_plain_cg_finite_termination():
    """A hierarchy whose coarsest level is the identity-like 1-cell grid
    still converges in at most n iterations on a tiny SPD system."""
    shape = (2, 2, 3)
    H, A = _sym_hierarchy(shape, 27)
    b = workloads.rng(3).uniform(-1, 1, size=shape)
    x, st, it, rel = H.pcg(b, 1e-12, 12)
    M = helpers.dense_from_sgdia(A, workloads.offsets(27), shape)
    assert st == 0 and it <= 12
    assert np.allclose(x.ravel(), np.linalg.solve(M, b.ravel()), atol=1e-11)


def test_laplace_pcg_iterations_and_complexity():
    """32^3 Laplace: PCG with the V(1,1) symmetric-GS cycle converges well
    within the paper's 13-iteration band, and the grid / operator complexity
    rounds to the Laplace row of the complexity table."""
    A, b = workloads.poisson7(32)
    H = oracle.Hierarchy((32, 32, 32), 7, A)
    dims = [H.level_info(l)["dims"] for l in range(H.nlev)]
    assert dims == [(32, 32, 32), (16, 16, 16), (8, 8, 8), (4, 4, 4)]
    x, st, it, rel = H.pcg(b, 1e-9, 100)
    assert st == 0 and rel < 1e-9 and it <= 15
    # Z_l: stored structured entries (pattern size times rows of level l)
    M_nnz = []
    n_l = []
    for l in range(H.nlev):
        n_l.append(int(np.prod(dims[l])))
        M_nnz.append(H.level_info(l)["S"] * n_l[-1])
    cg = sum(n_l) / n_l[0]
    co = sum(M_nnz) / M_nnz[0]
    tab = _gold_tables()[("complexity", "laplace")]
    assert round(cg, 2) == float(tab[0]) and round(co, 2) == float(tab[1])


def test_gmres_small_nonsymmetric():
    shape = (10, 8, 6)
    A = workloads.random_sgdia(shape, 19, seed=23, symmetric=False)
    b = workloads.rng(4).uniform(-1, 1, size=shape)
    for sm in ("gs", "ilu0"):
        H = oracle.Hierarchy(shape, 19, A, smoother=sm)
        x, st, it, rel = H.gmres(b, 1e-10, 200, restart=5)
        M = helpers.dense_from_sgdia(A, workloads.offsets(19), shape)
        assert st == 0 and rel < 1e-10
        assert np.allclose(x.ravel(), np.linalg.solve(M, b.ravel()), rtol=0, atol=1e-8)


def test_gmres_full_dimension_is_exact():
    """GMRES(n) with restart >= n on an n-unknown system is a direct method."""
    shape = (1, 2, 3)
    A = workloads.random_sgdia(shape, 7, seed=2, symmetric=False)
    H = oracle.Hierarchy(shape, 7, A)
    b = workloads.rng(8).uniform(-1, 1, size=shape)
    x, st, it, rel = H.gmres(b, 1e-14, 6, restart=6)
    M = helpers.dense_from_sgdia(A, workloads.offsets(7), shape)
    assert np.allclose(x.ravel(), np.linalg.solve(M, b.ravel()), rtol=0, atol=1e-13)


def test_gmres_agrees_with_pcg_on_spd():
    shape = (16, 16, 16)
    A, b = workloads.poisson7(16)
    H = oracle.Hierarchy(shape, 7, A)
    x1, s1, _, _ = H.pcg(b, 1e-11, 100)
    x2, s2, _, _ = H.gmres(b, 1e-11, 100)
    assert s1 == 0 and s2 == 0
    assert np.abs(x1 - x2).max() <= 1e-8 * np.abs(x1).max()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_mixed_precision_cycle_close_and_converges(prec):
    shape = (16, 16, 16)
    A, b = workloads.poisson7(16)
    H64 = oracle.Hierarchy(shape, 7, A)
    Hlo = oracle.Hierarchy(shape, 7, A, prec=prec)
    z64 = H64.apply(b)
    zlo = Hlo.apply(b)
    tol = 1e-5 if prec == "fp32" else 5e-3
    assert np.abs(z64 - zlo).max() <= tol * np.abs(z64).max()
    x, st, it, rel = Hlo.pcg(b, 1e-9, 100)
    assert st == 0 and rel < 1e-9


def test_fp16_truncation_rule():
    """Stored FP16 value = s * float(half(float(a/s))), s = float(max|a| in row)."""
    shape = (9, 8, 8)
    A = workloads.random_sgdia(shape, 7, seed=13)
    H = oracle.Hierarchy(shape, 7, A, prec="fp16")
    A32 = H.level_data(0, 5)
    s = np.abs(A).max(axis=0).astype(np.float32)
    h = (A / s.astype(np.float64)).astype(np.float32).astype(np.float16).astype(np.float32)
    assert np.array_equal(A32, (s * h).astype(np.float32))
    H32 = oracle.Hierarchy(shape, 7, A, prec="fp32")
    assert np.array_equal(H32.level_data(0, 5), A.astype(np.float32))
    assert np.array_equal(H32.level_data(0, 6), (1.0 / A[3]).astype(np.float32).reshape(1, -1))


def test_coarsening_rule_level_dims():
    """Level grids of the coarsening rule, worked out by hand: an axis is
    halved (floor) while allowed and >= 8; x,y only on the first semi_levels
    levels, switching to all axes early once x and y are both below 8."""
    A, _ = workloads.reservoir7((16, 19, 56), seed=1)
    H = oracle.Hierarchy((16, 19, 56), 7, A, semi_levels=3, max_coarse=512)
    dims = [H.level_info(l)["dims"] for l in range(H.nlev)]
    assert dims == [(16, 19, 56), (8, 9, 56), (4, 4, 56), (4, 4, 28), (4, 4, 14), (4, 4, 7)]
    # full coarsening from the start
    A, _ = workloads.reservoir7((17, 9, 8), seed=2)
    H = oracle.Hierarchy((17, 9, 8), 7, A)
    assert [H.level_info(l)["dims"] for l in range(H.nlev)] == [(17, 9, 8), (8, 4, 4), (4, 4, 4)]
    # semi mode never coarsens z
    A, _ = workloads.reservoir7((16, 16, 40), seed=3)
    H = oracle.Hierarchy((16, 16, 40), 7, A, coarsen="semi_xy")
    assert [H.level_info(l)["dims"] for l in range(H.nlev)] == [(16, 16, 40), (8, 8, 40), (4, 4, 40)]

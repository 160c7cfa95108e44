"""Independent explicit-matrix constructions used to pin the oracle.

Nothing here calls the oracle: matrices are assembled entry by entry from the
SG-DIA arrays and from the written definitions of the interpolation weights,
so a mistake in the oracle's index arithmetic shows up as a mismatch.
"""
import numpy as np


def lin(shape, x, y, z):
    return (x * shape[1] + y) * shape[2] + z


def dense_from_sgdia(A, off, shape, bs=1):
    """Explicit (N*bs) x (N*bs) matrix of an SG-DIA operator."""
    nx, ny, nz = shape
    N = nx * ny * nz
    M = np.zeros((N * bs, N * bs))
    for s, (dx, dy, dz) in enumerate(off):
        for x in range(nx):
            for y in range(ny):
                for z in range(nz):
                    a, b, c = x + dx, y + dy, z + dz
                    if not (0 <= a < nx and 0 <= b < ny and 0 <= c < nz):
                        continue
                    i = lin(shape, x, y, z)
                    j = lin(shape, a, b, c)
                    for r in range(bs):
                        for cc in range(bs):
                            M[i * bs + r, j * bs + cc] = A[s * bs * bs + r * bs + cc, i]
    return M


def interp_matrix(shape, cmask):
    """Explicit trilinear vertex-centred interpolation P (Nf x Nc): coarse X
    sits at fine 2X+1 on coarsened axes; weight prod_a w(f_a - (2X_a+1)) with
    w(0)=1, w(+-1)=1/2; identity on axes that are not coarsened."""
    cs = tuple(n // 2 if (cmask >> a) & 1 else n for a, n in enumerate(shape))
    Nf = int(np.prod(shape))
    Nc = int(np.prod(cs))
    P = np.zeros((Nf, Nc))
    for X in range(cs[0]):
        for Y in range(cs[1]):
            for Z in range(cs[2]):
                J = (X, Y, Z)
                base = [2 * J[a] + 1 if (cmask >> a) & 1 else J[a] for a in range(3)]
                rng = [(-1, 0, 1) if (cmask >> a) & 1 else (0,) for a in range(3)]
                for dx in rng[0]:
                    for dy in rng[1]:
                        for dz in rng[2]:
                            f = (base[0] + dx, base[1] + dy, base[2] + dz)
                            if not all(0 <= f[a] < shape[a] for a in range(3)):
                                continue
                            w = 1.0
                            for d in (dx, dy, dz):
                                if d != 0:
                                    w *= 0.5
                            P[lin(shape, *f), lin(cs, *J)] = w
    return P, cs


def sgdia_from_dense27(M, shape, bs=1, tol=0.0):
    """Reads a dense coarse operator back into 27-point SG-DIA form and checks
    that no entry lies outside the offsets {-1,0,1}^3."""
    nx, ny, nz = shape
    N = nx * ny * nz
    out = np.zeros((27 * bs * bs, N))
    seen = np.zeros_like(M, dtype=bool)
    for s in range(27):
        dx, dy, dz = s // 9 - 1, (s // 3) % 3 - 1, s % 3 - 1
        for x in range(nx):
            for y in range(ny):
                for z in range(nz):
                    a, b, c = x + dx, y + dy, z + dz
                    if not (0 <= a < nx and 0 <= b < ny and 0 <= c < nz):
                        continue
                    i = lin(shape, x, y, z)
                    j = lin(shape, a, b, c)
                    for r in range(bs):
                        for cc in range(bs):
                            out[s * bs * bs + r * bs + cc, i] = M[i * bs + r, j * bs + cc]
                            seen[i * bs + r, j * bs + cc] = True
    outside = np.abs(M[~seen]).max() if (~seen).any() else 0.0
    assert outside <= tol, "coarse operator has entries outside the 27-point pattern"
    return out


def csr_gs(M, b, u, direction, zero_guess):
    """Sequential point GS on an explicit matrix, rows in ascending
    (direction=+1) or descending order.  Row update: t = b_i, then the
    columns holding values from before the sweep, then the columns already
    updated in this sweep, each group in ascending column order,
    t = fma(-a_ij, u_j, t); u_i = t * (1/a_ii)."""
    n = len(b)
    u = u.copy()
    rows = range(n) if direction > 0 else range(n - 1, -1, -1)
    for i in rows:
        t = b[i]
        cols = np.nonzero(M[i])[0]
        old = [j for j in cols if (j > i if direction > 0 else j < i)]
        new = [j for j in cols if (j < i if direction > 0 else j > i)]
        groups = [new] if zero_guess else [old, new]
        for grp in groups:
            for j in grp:
                t = float(np.fma(-M[i, j], u[j], t)) if hasattr(np, "fma") else _fma(-M[i, j], u[j], t)
        u[i] = t * (1.0 / M[i, i])
    return u


def block_gs(M, Dinv, b, u, direction, zero_guess):
    """Sequential point-block GS on an explicit (3N x 3N) matrix: nodes in
    ascending (direction=+1) or descending order.  Node update: t = b_i (three
    rows); then the nodes holding values from before the sweep, then the nodes
    already updated in this sweep, each group in ascending node order, and per
    neighbour node j: for row r, for column c, t_r = fma(-M[3i+r, 3j+c],
    u[3j+c], t_r).  Then u_i = Dinv_i t row by row: Dinv_r0 * t_0, then
    fma(Dinv_r1, t_1, .), fma(Dinv_r2, t_2, .).  Dinv has shape (N, 3, 3)."""
    n = len(b) // 3
    u = np.array(u, dtype=np.float64).copy()
    fma = np.fma if hasattr(np, "fma") else _fma
    nodes = range(n) if direction > 0 else range(n - 1, -1, -1)
    for i in nodes:
        t = [float(b[3 * i + r]) for r in range(3)]
        nz = np.nonzero(np.abs(M[3 * i:3 * i + 3]).sum(axis=0))[0]
        nbrs = sorted({int(c) // 3 for c in nz} - {i})
        old = [j for j in nbrs if (j > i if direction > 0 else j < i)]
        new = [j for j in nbrs if (j < i if direction > 0 else j > i)]
        for grp in ([new] if zero_guess else [old, new]):
            for j in grp:
                for r in range(3):
                    for c in range(3):
                        t[r] = float(fma(-M[3 * i + r, 3 * j + c], u[3 * j + c], t[r]))
        for r in range(3):
            acc = Dinv[i, r, 0] * t[0]
            acc = float(fma(Dinv[i, r, 1], t[1], acc))
            acc = float(fma(Dinv[i, r, 2], t[2], acc))
            u[3 * i + r] = acc
    return u


def _fma(a, b, c):
    """Correctly rounded a*b+c via exact rational arithmetic."""
    from fractions import Fraction
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def line_gs(M, shape, b, u0, direction):
    """Block Gauss-Seidel over z-columns written with dense blocks: for each
    column J in lexicographic (x, y) order (reversed for direction -1),
    u_J = M_JJ^-1 (b_J - sum_{K != J} M_JK u_K) with the current u."""
    nx, ny, nz = shape
    u = np.array(u0, dtype=np.float64).ravel().copy()
    b = np.asarray(b, dtype=np.float64).ravel()
    cols = range(nx * ny) if direction > 0 else range(nx * ny - 1, -1, -1)
    for J in cols:
        r = slice(J * nz, (J + 1) * nz)
        rhs = b[r] - M[r, :] @ u + M[r, r] @ u[r]
        u[r] = np.linalg.solve(M[r, r], rhs)
    return u


def cell_interp_matrix(shape, cmask):
    """Explicit cell-centred piecewise-constant interpolation P (Nf x Nc):
    fine cell f takes the value of its parent cell f // 2 on each coarsened
    axis (identity on the others); n_c = ceil(n_f / 2)."""
    cs = tuple((n + 1) // 2 if (cmask >> a) & 1 else n for a, n in enumerate(shape))
    P = np.zeros((int(np.prod(shape)), int(np.prod(cs))))
    for x in range(shape[0]):
        for y in range(shape[1]):
            for z in range(shape[2]):
                f = (x, y, z)
                J = tuple(f[a] // 2 if (cmask >> a) & 1 else f[a] for a in range(3))
                P[lin(shape, *f), lin(cs, *J)] = 1.0
    return P, cs


def cell_trilinear_matrix(shape, cmask):
    """Explicit cell-centred trilinear interpolation (Nf x Nc): on a coarsened
    axis fine cell 2I + d takes weight 3/4 from I and 1/4 from I - 1 (d = 0)
    or I + 1 (d = 1), contributors outside the coarse grid dropped; weights of
    the axes multiply."""
    cs = tuple((n + 1) // 2 if (cmask >> a) & 1 else n for a, n in enumerate(shape))
    P = np.zeros((int(np.prod(shape)), int(np.prod(cs))))

    def axis(f, a):
        if not (cmask >> a) & 1:
            return [(f, 1.0)]
        I = f // 2
        J = I + 1 if f % 2 else I - 1
        return [(k, w) for k, w in ((I, 0.75), (J, 0.25)) if 0 <= k < cs[a]]

    for x in range(shape[0]):
        for y in range(shape[1]):
            for z in range(shape[2]):
                for jx, wx in axis(x, 0):
                    for jy, wy in axis(y, 1):
                        for jz, wz in axis(z, 2):
                            P[lin(shape, x, y, z), lin(cs, jx, jy, jz)] += wx * wy * wz
    return P, cs


def od_matrix(W, shape, cmask):
    """Explicit interpolation matrix (Nf x Nc) of operator-dependent weights
    W (8, Nf): weight c of fine point f belongs to its corner c, whose index on
    a coarsened axis is (f-1)/2 for odd f (c_a = 0) or f/2 - 1 + c_a for even
    f, and f itself on other axes; corners outside the coarse grid and c_a = 1
    on a non-even axis carry nothing."""
    cs = tuple(n // 2 if (cmask >> a) & 1 else n for a, n in enumerate(shape))
    P = np.zeros((int(np.prod(shape)), int(np.prod(cs))))
    for x in range(shape[0]):
        for y in range(shape[1]):
            for z in range(shape[2]):
                f = (x, y, z)
                i = lin(shape, *f)
                for c in range(8):
                    cc = (c // 4, (c // 2) % 2, c % 2)
                    J = []
                    for a in range(3):
                        if not (cmask >> a) & 1 or f[a] % 2:
                            j = (f[a] if not (cmask >> a) & 1 else (f[a] - 1) // 2) if cc[a] == 0 else -1
                        else:
                            j = f[a] // 2 - 1 + cc[a]
                        J.append(j)
                    if all(0 <= J[a] < cs[a] for a in range(3)):
                        P[i, lin(cs, *J)] += W[c, i]
    return P, cs


def masked_sgdia(A, off, shape, be=1):
    """SG-DIA matrix (len(off) * be, N) with the couplings of slot s zeroed
    where the neighbour i + off[s] lies outside the grid (the finest level's
    Dirichlet masking); be entries per slot (9 for 3x3 blocks)."""
    Am = np.array(A, dtype=np.float64).reshape(len(off), be, *shape)
    for s, o in enumerate(off):
        for a in range(3):
            if o[a] != 0:
                sl = [slice(None)] * 3
                sl[a] = slice(0, 1) if o[a] < 0 else slice(shape[a] - 1, shape[a])
                Am[(s, slice(None), *sl)] = 0.0
    return Am.reshape(len(off) * be, -1)


def coarse_sample_points(cdims, n, seed):
    """Sorted distinct flat indices of about 2n coarse points: n uniform in the
    grid, n on its faces, and its 8 corners."""
    g = np.random.default_rng(seed)
    X, Y, Z = (g.integers(0, d, size=n) for d in cdims)
    face, side = g.integers(0, 3, size=n), g.integers(0, 2, size=n)
    B = [X.copy(), Y.copy(), Z.copy()]
    for a in range(3):
        B[a] = np.where(face == a, side * (cdims[a] - 1), B[a])
    corners = np.array([(x, y, z) for x in (0, cdims[0] - 1) for y in (0, cdims[1] - 1) for z in (0, cdims[2] - 1)])

    def flat(x, y, z):
        return (np.asarray(x, np.int64) * cdims[1] + np.asarray(y)) * cdims[2] + np.asarray(z)

    return np.unique(np.concatenate([flat(X, Y, Z), flat(*B), flat(*corners.T)])).astype(np.int64)

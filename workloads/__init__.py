"""Seeded synthetic inputs shaped like the paper's test problems.

This module only *constructs* linear systems (coefficients in SG-DIA layout
and right-hand sides).  It contains none of the multigrid method's arithmetic,
so both the CPU oracle and the GPU library can consume its arrays.

Layout of every matrix returned here: ``A[s, i]`` (float64, shape (S, N)) is
the coefficient of row ``i`` for stencil offset ``s``; offsets are listed in
lexicographic (dx slowest) order; ``i = (x*ny + y)*nz + z``.  Couplings to
neighbours outside the grid are zero (Dirichlet boundaries eliminated).
Block systems (3 unknowns per node) use ``A[s*9 + r*3 + c, i]`` and interleaved
vectors ``x[i*3 + c]``.

All random draws use ``numpy.random.Generator(PCG64(seed))``.
"""
import numpy as np


def offsets(npts):
    """Offsets of the 3d7 / 3d19 / 3d27 patterns in lexicographic order."""
    out = []
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                m = abs(dx) + abs(dy) + abs(dz)
                if npts == 27 or (npts == 19 and m <= 2) or (npts == 7 and m <= 1):
                    out.append((dx, dy, dz))
    return np.array(out, dtype=np.int32)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def rhs(shape, seed, block=1):
    """i.i.d. uniform[-1, 1] right-hand side (the problems' RHS recipe)."""
    g = rng(seed + 7919)
    return g.uniform(-1.0, 1.0, size=tuple(shape) + ((block,) if block > 1 else ()))


def _shift_valid(shape, d):
    """Slices (dst, src) so that dst[i] pairs with src[i + d] inside the grid."""
    dst, src = [], []
    for n, o in zip(shape, d):
        if o >= 0:
            dst.append(slice(0, n - o))
            src.append(slice(o, n))
        else:
            dst.append(slice(-o, n))
            src.append(slice(0, n + o))
    return tuple(dst), tuple(src)


def fv7_from_cells(kx, ky=None, kz=None):
    """Cell-centred finite-volume 7-point operator (h = 1) from cell
    coefficients: face transmissibility is the harmonic mean 2 ka kb/(ka+kb);
    a Dirichlet boundary face (ghost value at h/2) contributes 2k to the
    diagonal.  Returns A with shape (7, N).  (Written with in-place numpy
    operations so that large grids need few temporary arrays.)"""
    ky = kx if ky is None else ky
    kz = kx if kz is None else kz
    shape = kx.shape
    off = offsets(7)
    A = np.zeros((7,) + shape)
    diag = A[3]
    kk = {0: kx, 1: ky, 2: kz}
    buf1 = np.empty(int(np.prod(shape)))
    buf2 = np.empty(int(np.prod(shape)))
    for s, d in enumerate(off):
        d = tuple(int(v) for v in d)
        if d == (0, 0, 0):
            continue
        ax = [a for a in range(3) if d[a] != 0][0]
        k = kk[ax]
        dst, src = _shift_valid(shape, d)
        ka, kb = k[dst], k[src]
        n = ka.size
        T = buf1[:n].reshape(ka.shape)
        den = buf2[:n].reshape(ka.shape)
        np.multiply(ka, kb, out=T)
        T *= 2.0
        np.add(ka, kb, out=den)
        T /= den
        np.negative(T, out=A[s][dst])
        diag[dst] += T
        # boundary faces in direction d: cells whose neighbour i+d is outside
        bnd = [slice(None)] * 3
        bnd[ax] = slice(shape[ax] - 1, shape[ax]) if d[ax] > 0 else slice(0, 1)
        diag[tuple(bnd)] += 2.0 * k[tuple(bnd)]
    return A.reshape(7, -1)


def poisson7(n=32, seed=1):
    """3D Poisson, 7-point constant stencil (6 on the diagonal, -1 off it),
    Dirichlet boundaries eliminated; RHS uniform[-1,1].  (Laplace problem.)"""
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    off = offsets(7)
    A = np.zeros((7,) + shape)
    for s, d in enumerate(off):
        d = tuple(int(v) for v in d)
        if d == (0, 0, 0):
            A[s] = 6.0
            continue
        dst, _ = _shift_valid(shape, d)
        A[s][dst] = -1.0
    return A.reshape(7, -1), rhs(shape, seed)


def diffusion7(shape=(256, 256, 256), seed=2, sigma=2.0, nspheres=32, rmin=8.0, rmax=32.0):
    """Variable-coefficient diffusion (radiation-hydrodynamics-like): cell
    coefficient k = exp(sigma Z), Z ~ N(0,1) i.i.d., times 10^U[-3,3] inside
    each of `nspheres` random spheres (centres uniform in the box, radii
    U[rmin, rmax] cells); 7-point FV with harmonic-mean faces."""
    shape = tuple(shape)
    g = rng(seed)
    k = g.standard_normal(shape)
    k *= sigma
    np.exp(k, out=k)
    cen = g.uniform(0.0, 1.0, size=(nspheres, 3)) * np.array(shape)
    rad = g.uniform(rmin, rmax, size=nspheres)
    con = 10.0 ** g.uniform(-3.0, 3.0, size=nspheres)
    for c, r, f in zip(cen, rad, con):
        lo = [max(0, int(np.floor(c[a] - r))) for a in range(3)]
        hi = [min(shape[a], int(np.ceil(c[a] + r)) + 1) for a in range(3)]
        xs, ys, zs = [np.arange(lo[a], hi[a]) + 0.5 - c[a] for a in range(3)]
        inside = (xs[:, None, None] ** 2 + ys[None, :, None] ** 2 + zs[None, None, :] ** 2) <= r * r
        sub = k[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        sub[inside] *= f
    return fv7_from_cells(k), rhs(shape, seed)


def weather19(shape=(512, 512, 64), seed=3, vert=100.0, noise=0.1, skew=0.05):
    """Anisotropic weather-like 19-point operator (z vertical and contiguous).
    Symmetric pair couplings c = base * g(x,y) * (1 + noise*xi), xi ~ U[-1,1]
    per pair, g = exp(0.5 sin(2 pi x/nx) sin(2 pi y/ny)); bases: horizontal
    faces 1, vertical faces `vert`, xz/yz edges 2.5, xy edges 0.05.  Face pairs
    get a non-symmetric advection-like split A_ij = -c(1+skew*beta),
    A_ji = -c(1-skew*beta), beta ~ U[-1,1].  Diagonal: 0.01 plus the sum of
    |off-diagonals| in the row, plus the base couplings of neighbours outside
    the grid (Dirichlet)."""
    shape = tuple(shape)
    nx, ny, nz = shape
    g = rng(seed)
    off = offsets(19)
    S = len(off)
    cidx = S // 2
    X = np.arange(nx)[:, None, None]
    Y = np.arange(ny)[None, :, None]
    gxy = np.exp(0.5 * np.sin(2 * np.pi * X / nx) * np.sin(2 * np.pi * Y / ny)) * np.ones((1, 1, nz))

    def base(d):
        dx, dy, dz = d
        m = abs(dx) + abs(dy) + abs(dz)
        if m == 1:
            return vert if dz != 0 else 1.0
        if dz != 0:
            return 2.5
        return 0.05

    A = np.zeros((S,) + shape)
    diag = np.full(shape, 0.01)
    for s in range(cidx + 1, S):
        d = tuple(int(v) for v in off[s])
        sm = S - 1 - s  # mirrored (lower) offset
        c = base(d) * gxy * (1.0 + noise * g.uniform(-1.0, 1.0, size=shape))
        dst, src = _shift_valid(shape, d)
        if sum(abs(v) for v in d) == 1:
            beta = g.uniform(-1.0, 1.0, size=shape)
            up = -c * (1.0 + skew * beta)
            lo = -c * (1.0 - skew * beta)
        else:
            up = -c
            lo = -c
        A[s][dst] = up[dst]
        A[sm][src] = lo[dst]
        # Dirichlet: couplings that would leave the grid go to the diagonal
        outside_up = np.ones(shape, bool)
        outside_up[dst] = False
        diag[outside_up] += base(d) * gxy[outside_up]
        dst2, _ = _shift_valid(shape, tuple(-v for v in d))
        outside_lo = np.ones(shape, bool)
        outside_lo[dst2] = False
        diag[outside_lo] += base(d) * gxy[outside_lo]
    for s in range(S):
        if s != cidx:
            diag += np.abs(A[s])
    A[cidx] = diag
    return A.reshape(S, -1), rhs(shape, seed)


def reservoir7(shape, seed, sigma=1.5, kz_ratio=0.01):
    """Reservoir-like 7-point FV system: kx = ky = exp(sigma Z) per cell,
    kz = kz_ratio * kx, harmonic-mean faces."""
    g = rng(seed)
    k = np.exp(sigma * g.standard_normal(tuple(shape)))
    return fv7_from_cells(k, k, kz_ratio * k), rhs(shape, seed)


def reservoir_batch(nsys=256, seed=5, lo=16, hi=96):
    """Batch of independent reservoir-like systems with grid sizes drawn
    uniformly from {lo..hi} per axis."""
    g = rng(seed)
    dims = g.integers(lo, hi + 1, size=(nsys, 3))
    return [tuple(int(v) for v in d) for d in dims]


# ---- Q1 hexahedral linear elasticity (3 unknowns per node) --------------

def _q1_element_matrices():
    """Reference 24x24 stiffness matrices of a unit cube Q1 element for
    (lambda=1, mu=0) and (lambda=0, mu=1), 2x2x2 Gauss quadrature.
    Local node a = (ax, ay, az) in {0,1}^3, ordered ax slowest; dof 3a+c."""
    gp = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    nodes = [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    KL = np.zeros((24, 24))
    KM = np.zeros((24, 24))
    for px in gp:
        for py in gp:
            for pz in gp:
                p = (px, py, pz)
                dN = np.zeros((8, 3))
                for k, nd in enumerate(nodes):
                    f = [p[a] if nd[a] else 1.0 - p[a] for a in range(3)]
                    df = [1.0 if nd[a] else -1.0 for a in range(3)]
                    dN[k] = [df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]]
                B = np.zeros((6, 24))
                for k in range(8):
                    gx, gy, gz = dN[k]
                    B[0, 3 * k] = gx
                    B[1, 3 * k + 1] = gy
                    B[2, 3 * k + 2] = gz
                    B[3, 3 * k] = gy
                    B[3, 3 * k + 1] = gx
                    B[4, 3 * k + 1] = gz
                    B[4, 3 * k + 2] = gy
                    B[5, 3 * k] = gz
                    B[5, 3 * k + 2] = gx
                DL = np.zeros((6, 6))
                DL[:3, :3] = 1.0
                DM = np.diag([2.0, 2.0, 2.0, 1.0, 1.0, 1.0])
                w = 1.0 / 8.0
                KL += w * B.T @ DL @ B
                KM += w * B.T @ DM @ B
    return nodes, KL, KM


def elasticity27(n=128, seed=4, sigma=1.0, nu=0.3):
    """Linear-elasticity-like block system: Q1 FEM on (n+1)^3 unit cells, the
    n^3 interior nodes are unknowns (all boundary nodes clamped).  Young's
    modulus E = exp(sigma Z) per cell, Poisson ratio nu, so lambda and mu are
    log-normal with a fixed ratio.  27-point stencil of 3x3 blocks, returned as
    A with shape (243, N) and RHS of shape (n,n,n,3)."""
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    g = rng(seed)
    ncell = tuple(v + 1 for v in shape)
    E = np.exp(sigma * g.standard_normal(ncell))
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    nodes, KL, KM = _q1_element_matrices()
    off = offsets(27)
    sidx = {tuple(int(v) for v in d): s for s, d in enumerate(off)}
    A = np.zeros((27 * 9,) + shape)
    # unknown node (X,Y,Z) = global node (X+1, Y+1, Z+1); cell (cx,cy,cz) has
    # global corner nodes (cx+ax, ...). Cell c touches unknown X when
    # X+1 = c+a, i.e. c = X+1-a.
    for ia, na in enumerate(nodes):
        for ib, nb in enumerate(nodes):
            d = tuple(nb[k] - na[k] for k in range(3))
            s = sidx[d]
            # cells for row node X: c = X + 1 - na, valid range of X
            cl = [slice(1 - na[k], 1 - na[k] + shape[k]) for k in range(3)]
            lam_c = lam[tuple(cl)]
            mu_c = mu[tuple(cl)]
            for r in range(3):
                for c in range(3):
                    v = KL[3 * ia + r, 3 * ib + c] * lam_c + KM[3 * ia + r, 3 * ib + c] * mu_c
                    A[s * 9 + r * 3 + c] += v
    # zero couplings to clamped (out-of-grid) nodes
    for s, d in enumerate(off):
        d = tuple(int(v) for v in d)
        mask = np.zeros(shape, bool)
        dst, _ = _shift_valid(shape, d)
        mask[dst] = True
        for e in range(9):
            A[s * 9 + e][~mask] = 0.0
    return A.reshape(243, -1), rhs(shape, seed, block=3)


def random_sgdia(shape, npts, seed, symmetric=True, dominance=1.0, block=1):
    """Random test operator on the given pattern: off-diagonals uniform in
    [-1, 0) (symmetric pairs when `symmetric`), diagonal = dominance * sum of
    |off-diagonals| + 1, out-of-grid couplings zero.  Block systems get random
    3x3 off-diagonal blocks and a diagonally dominant diagonal block."""
    shape = tuple(shape)
    g = rng(seed)
    off = offsets(npts)
    S = len(off)
    c = S // 2
    be = block * block
    A = np.zeros((S * be,) + shape)
    for s in range(c + 1, S):
        d = tuple(int(v) for v in off[s])
        sm = S - 1 - s
        dst, src = _shift_valid(shape, d)
        for e in range(be):
            v = -g.uniform(0.0, 1.0, size=shape) if block == 1 else g.uniform(-1.0, 1.0, size=shape)
            A[s * be + e][dst] = v[dst]
            if symmetric:
                r_, c_ = divmod(e, block)
                A[sm * be + c_ * block + r_][src] = v[dst]
            else:
                w = -g.uniform(0.0, 1.0, size=shape) if block == 1 else g.uniform(-1.0, 1.0, size=shape)
                A[sm * be + e][src] = w[dst]
    rows = np.zeros((block,) + shape)
    for s in range(S):
        if s == c:
            continue
        for e in range(be):
            rows[e // block] += np.abs(A[s * be + e])
    for r in range(block):
        for cc in range(block):
            if r == cc:
                A[c * be + r * block + cc] = dominance * (rows[r] + (block - 1) * 0.5) + 1.0
            else:
                A[c * be + r * block + cc] = 0.25 * g.uniform(-1.0, 1.0, size=shape)
                if symmetric and r > cc:
                    A[c * be + r * block + cc] = A[c * be + cc * block + r]
    return A.reshape(S * be, -1)

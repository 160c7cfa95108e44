"""Pins of the oracle's smoothing settings and coarsening choices.

* weighted GS (Sec. 4.4 GS-Forward / GS-Backward formulas with weight w):
  one sweep against the dense formula u + w (D + wL)^-1 (b - A u);
* several smoothing steps per level: a V-cycle with as many steps after the
  coarse correction as before is a symmetric operator (GS directions paired
  in reverse), one with unequal counts is not; many steps drive the V-cycle
  to the exact solve;
* ZeroGuess off gives the same values;
* the automatic x,y-only levels against their closed form, and min_coarse
  against plain halving.
"""
import numpy as np
import pytest
from scipy.linalg import solve_triangular

import oracle
import workloads
from tests import helpers


def _system(shape, npts, seed, symmetric=False):
    A = workloads.random_sgdia(shape, npts, seed=seed, symmetric=symmetric)
    off = workloads.offsets(npts)
    A = helpers.masked_sgdia(A, off, shape)
    return A, off


@pytest.mark.parametrize("shape,npts", [((5, 4, 6), 7), ((3, 7, 5), 27), ((4, 5, 3), 19)])
@pytest.mark.parametrize("w", [0.7, 1.35])
def test_weighted_gs_sweep_matches_dense_formula(shape, npts, w):
    A, off = _system(shape, npts, seed=13)
    M = helpers.dense_from_sgdia(A, off, shape)
    n = M.shape[0]
    d = np.diag(M).copy()
    Lo = np.tril(M, -1)
    Up = np.triu(M, 1)
    g = workloads.rng(3)
    b = g.uniform(-1, 1, size=shape)
    u0 = g.uniform(-1, 1, size=shape)
    c = npts // 2
    rd = (w / A[c]).reshape(1, -1)
    qa = ((1.0 - w) / w) * A[c]
    bf, uf = b.ravel(), u0.ravel()
    res = bf - M @ uf
    want_f = uf + w * solve_triangular(np.diag(d) + w * Lo, res, lower=True)
    want_b = uf + w * solve_triangular(np.diag(d) + w * Up, res, lower=False)
    want_z = w * solve_triangular(np.diag(d) + w * Lo, bf, lower=True)
    got_f = oracle.gs_sweep_w(off, A, rd, qa, b, u0, +1, 0).ravel()
    got_b = oracle.gs_sweep_w(off, A, rd, qa, b, u0, -1, 0).ravel()
    got_z = oracle.gs_sweep_w(off, A, rd, qa, b, np.full(shape, np.nan), +1, 1).ravel()
    scale = max(1.0, np.abs(want_f).max())
    assert n == uf.size
    assert np.abs(got_f - want_f).max() <= 1e-12 * scale
    assert np.abs(got_b - want_b).max() <= 1e-12 * scale
    assert np.abs(got_z - want_z).max() <= 1e-12 * scale


def _symmetry_gap(H, shape, seed):
    g = workloads.rng(seed)
    x = g.uniform(-1, 1, size=shape)
    y = g.uniform(-1, 1, size=shape)
    a = np.dot(H.apply(x).ravel(), y.ravel())
    b = np.dot(x.ravel(), H.apply(y).ravel())
    return abs(a - b) / max(abs(a), 1.0)


@pytest.mark.parametrize("kw", [dict(smoother="gs"), dict(smoother="gs", relax_weight=1.3),
                                dict(smoother="gs", relax_weight=0.8), dict(smoother="lgs"),
                                dict(smoother="ilu0")])
@pytest.mark.parametrize("steps", [2, 3])
def test_vcycle_equal_step_counts_symmetric(kw, steps):
    """pre_sweeps == post_sweeps: forward, backward, ... before and the
    adjoint steps in reverse order after the correction give <Mx,y> = <x,My>;
    with one step fewer after, the operator is not symmetric."""
    shape = (14, 12, 10)
    A = workloads.random_sgdia(shape, 19, seed=17, symmetric=True)
    H = oracle.Hierarchy(shape, 19, A, pre_sweeps=steps, post_sweeps=steps, **kw)
    assert H.nlev >= 2
    assert _symmetry_gap(H, shape, 5) <= 1e-12
    if kw["smoother"] != "ilu0":  # an ILU(0) step is itself symmetric for symmetric A
        Hu = oracle.Hierarchy(shape, 19, A, pre_sweeps=steps, post_sweeps=steps - 1, **kw)
        assert _symmetry_gap(Hu, shape, 5) > 1e-6


def test_vcycle_block_equal_step_counts_symmetric():
    shape = (8, 9, 8)
    A = workloads.random_sgdia(shape, 27, seed=17, symmetric=True, block=3)
    H = oracle.Hierarchy(shape, 27, A, block=3, pre_sweeps=2, post_sweeps=2)
    g = workloads.rng(6)
    x = g.uniform(-1, 1, size=shape + (3,))
    y = g.uniform(-1, 1, size=shape + (3,))
    a = np.dot(H.apply(x).ravel(), y.ravel())
    b = np.dot(x.ravel(), H.apply(y).ravel())
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


@pytest.mark.parametrize("smoother", ["gs", "lgs", "ilu0"])
def test_many_steps_approach_the_solve(smoother):
    """More smoothing steps per level make the V-cycle a better inverse: the
    error of M f against A^-1 f falls with the step count and is tiny after
    eight steps on a diagonally dominant system."""
    shape = (10, 9, 8)
    A = workloads.random_sgdia(shape, 7, seed=21, symmetric=True, dominance=2.0)
    off = workloads.offsets(7)
    M = helpers.dense_from_sgdia(helpers.masked_sgdia(A, off, shape), off, shape)
    f = workloads.rng(2).uniform(-1, 1, size=shape)
    x = np.linalg.solve(M, f.ravel())
    errs = []
    for k in (1, 2, 4, 8):
        H = oracle.Hierarchy(shape, 7, A, smoother=smoother, pre_sweeps=k, post_sweeps=k)
        errs.append(np.abs(H.apply(f).ravel() - x).max() / np.abs(x).max())
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6, errs


@pytest.mark.parametrize("kw", [dict(smoother="gs"), dict(smoother="gs", relax_weight=1.2), dict(smoother="lgs"),
                                dict(smoother="ilu0"), dict(smoother="gs", pre_sweeps=2, post_sweeps=3)])
def test_zero_guess_off_same_values(kw):
    """Without ZeroGuess the first step applies the full stencil to u = 0:
    the same values (zeros of either sign compare equal)."""
    shape = (11, 9, 10)
    A = workloads.random_sgdia(shape, 19, seed=9, symmetric=False)
    f = workloads.rng(4).uniform(-1, 1, size=shape)
    on = oracle.Hierarchy(shape, 19, A, **kw).apply(f)
    off = oracle.Hierarchy(shape, 19, A, zero_guess=False, **kw).apply(f)
    assert np.array_equal(on, off)


def test_block_zero_guess_off_same_values():
    shape = (8, 7, 9)
    A = workloads.random_sgdia(shape, 27, seed=9, symmetric=False, block=3)
    f = workloads.rng(4).uniform(-1, 1, size=shape + (3,))
    on = oracle.Hierarchy(shape, 27, A, block=3).apply(f)
    off = oracle.Hierarchy(shape, 27, A, block=3, zero_guess=False).apply(f)
    assert np.array_equal(on, off)


@pytest.mark.parametrize("ratio,want", [(0.01, 3), (0.05, 2), (0.2, 1), (1.0, 0), (10.0, 0)])
def test_auto_semi_levels_closed_form(ratio, want):
    """Uniform cell coefficients with kz = ratio * kx on a cube: the face
    couplings are kz and kx, so rho = ratio and the rule rho * 4^l < 1/4
    gives `want` leading x,y-only levels."""
    n = 32
    k = np.ones((n, n, n))
    A = workloads.fv7_from_cells(k, k, ratio * k)
    off = workloads.offsets(7)
    assert oracle.auto_semi_levels(off, A, (n, n, n)) == want
    H = oracle.Hierarchy((n, n, n), 7, A, coarsen="auto")
    masks = [H.level_info(l)["cmask"] for l in range(H.nlev - 1)]
    full = oracle.Hierarchy((n, n, n), 7, A, coarsen="full", semi_levels=want)
    assert masks == [full.level_info(l)["cmask"] for l in range(full.nlev - 1)]
    assert masks[:want] == [3] * want
    assert masks[want] & 4  # z is coarsened from here on


@pytest.mark.parametrize("min_coarse,dims", [(4, [16, 8, 4]), (2, [16, 8, 4, 2]), (3, [16, 8, 4]),
                                             (5, [16, 8])])
def test_min_coarse_halving(min_coarse, dims):
    """An axis of n points is coarsened (n -> floor(n/2)) while n >= 2 * min_coarse."""
    n = 16
    A = workloads.random_sgdia((n, n, n), 7, seed=3, symmetric=True)
    H = oracle.Hierarchy((n, n, n), 7, A, min_coarse=min_coarse)
    assert [H.level_info(l)["dims"][0] for l in range(H.nlev)] == dims

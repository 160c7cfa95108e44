"""GPU parity tests: every kernel of the V-cycle, called through the C ABI,
against the CPU oracle on the same seeded inputs.

Bar: bit-exact for the stencil kernels (SpMV / residual, Gauss-Seidel and
ILU sweeps, restriction, prolongation, triple product, truncation) whose
per-element operation order is fixed; 1e-13 relative for the coarsest solve
(explicit inverse on the GPU, LU on the CPU) and for quantities built from it.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_21932_amd as smg  # noqa: E402

DEV = torch.device("cuda:0")


def T(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def N(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = [
    # (shape, pattern, coarsen, semi_levels)
    ((20, 18, 17), 7, "full", 0),
    ((33, 17, 9), 19, "full", 0),
    ((24, 21, 12), 27, "full", 0),
    ((40, 36, 6), 19, "semi_xy", 0),
    ((37, 19, 23), 7, "full", 2),
    # finest levels above the size where residual + restriction and
    # prolongation + lower terms run as separate passes
    ((66, 50, 41), 19, "full", 0),
    ((80, 52, 36), 7, "full", 1),
]


def _ids(c):
    return f"{c[0][0]}x{c[0][1]}x{c[0][2]}-3d{c[1]}-{c[2]}{c[3]}"


def _pair(case, smoother="gs", prec="fp64", sym=True, seed=3):
    shape, pat, coarsen, semi = case
    A = workloads.random_sgdia(shape, pat, seed=seed, symmetric=sym)
    H = oracle.Hierarchy(shape, pat, A, smoother=smoother, coarsen=coarsen, semi_levels=semi, prec=prec)
    mg = smg.StructMG(T(A), shape, pattern=pat, smoother=smoother, coarsen=coarsen, semi_levels=semi, prec=prec,
                      device=DEV)
    return A, H, mg


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_hierarchy_rap_bitexact(case):
    A, H, mg = _pair(case)
    assert mg.nlev == H.nlev
    for l in range(H.nlev):
        inf = mg.level_info(l)
        ref = H.level_info(l)
        assert inf["dims"] == ref["dims"] and inf["S"] == ref["S"] and inf["cmask"] == ref["cmask"]
        Ar = H.level_data(l, 0)
        got = N(mg.export(l, 0, torch.empty(Ar.shape, dtype=torch.float64, device=DEV)))
        assert np.array_equal(got, Ar), f"level {l}: max diff {np.abs(got - Ar).max()}"
        if l < H.nlev - 1:
            rd = H.level_data(l, 1)
            got = N(mg.export(l, 1, torch.empty(rd.shape, dtype=torch.float64, device=DEV)))
            assert np.array_equal(got, rd)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_level_kernels_bitexact(case):
    A, H, mg = _pair(case)
    g = workloads.rng(11)
    for l in range(H.nlev - 1):
        inf = H.level_info(l)
        dims, S, cm = inf["dims"], inf["S"], inf["cmask"]
        off = workloads.offsets(S)
        Al, rd = H.level_data(l, 0), H.level_data(l, 1).ravel()
        f = g.uniform(-1, 1, size=dims)
        u = g.uniform(-1, 1, size=dims)
        cdims = oracle.coarse_dims(dims, cm)
        ec = g.uniform(-1, 1, size=cdims)
        # SpMV
        y = N(mg.op_spmv(l, T(f), torch.empty(int(np.prod(dims)), dtype=torch.float64, device=DEV)))
        assert np.array_equal(y, oracle.spmv(off, Al, f).ravel()), f"spmv level {l}"
        # pre-smoothing: forward GS from zero
        ug = N(mg.op_presmooth(l, T(f), torch.empty(int(np.prod(dims)), dtype=torch.float64, device=DEV)))
        ur = oracle.gs_sweep(off, Al, rd, f, np.zeros(dims), 1, 1)
        assert np.array_equal(ug, ur.ravel()), f"forward GS level {l}: {np.abs(ug - ur.ravel()).max()}"
        # residual + restriction
        rc = N(mg.op_resid_restrict(l, T(f), T(u), torch.empty(int(np.prod(cdims)), dtype=torch.float64,
                                                               device=DEV)))
        rr = oracle.restrict(oracle.residual(off, Al, f, u), cm)
        assert np.array_equal(rc, rr.ravel()), f"resid+restrict level {l}"
        # prolongation + backward GS
        uo = N(mg.op_postsmooth(l, T(f), T(u), T(ec), torch.empty(int(np.prod(dims)), dtype=torch.float64,
                                                                  device=DEV)))
        ref = oracle.gs_sweep(off, Al, rd, f, oracle.prolong_add(u, ec, cm), -1, 0)
        assert np.array_equal(uo, ref.ravel()), f"backward GS level {l}: {np.abs(uo - ref.ravel()).max()}"
        # plain restriction / prolongation
        rc2 = N(mg.op_restrict(l, T(f), torch.empty(int(np.prod(cdims)), dtype=torch.float64, device=DEV)))
        assert np.array_equal(rc2, oracle.restrict(f, cm).ravel())
        uf = T(u.copy())
        mg.op_prolong_add(l, T(ec), uf)
        assert np.array_equal(N(uf).ravel(), oracle.prolong_add(u, ec, cm).ravel())


@pytest.mark.parametrize("case", CASES[:3], ids=_ids)
def test_sweeps_deterministic(case):
    """Repeated sweeps give identical bits (a missed dependence would not)."""
    A, H, mg = _pair(case)
    dims = H.level_info(0)["dims"]
    f = T(workloads.rng(5).uniform(-1, 1, size=dims))
    first = None
    for _ in range(20):
        u = mg.op_presmooth(0, f, torch.empty(int(np.prod(dims)), dtype=torch.float64, device=DEV))
        v = N(u)
        if first is None:
            first = v
        assert np.array_equal(v, first)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_coarse_solve_and_vcycle(case):
    A, H, mg = _pair(case)
    L = H.nlev - 1
    inf = H.level_info(L)
    n = int(np.prod(inf["dims"]))
    f = workloads.rng(2).uniform(-1, 1, size=n)
    u = N(mg.op_coarse_solve(T(f), torch.empty(n, dtype=torch.float64, device=DEV)))
    M = oracle.dense(workloads.offsets(27) if L > 0 else workloads.offsets(case[1]), H.level_data(L, 0),
                     inf["dims"])
    ref = np.linalg.solve(M, f)
    assert np.abs(u - ref).max() <= 1e-13 * np.abs(ref).max() * max(1.0, np.linalg.cond(M) / 1e3)
    # whole V-cycle
    dims = H.level_info(0)["dims"]
    r = workloads.rng(9).uniform(-1, 1, size=dims)
    z = N(mg.precondition(T(r.ravel()), torch.empty(r.size, dtype=torch.float64, device=DEV)))
    zr = H.apply(r).ravel()
    assert np.abs(z - zr).max() <= 1e-12 * np.abs(zr).max()
    # twice in a row (buffers are reused across cycles)
    z2 = N(mg.precondition(T(r.ravel()), torch.empty(r.size, dtype=torch.float64, device=DEV)))
    assert np.array_equal(z, z2)


def test_poisson_32_pcg():
    """32^3 Poisson, PCG with the V(1,1) symmetric GS cycle, tol 1e-9."""
    A, b = workloads.poisson7(32)
    shape = (32, 32, 32)
    H = oracle.Hierarchy(shape, 7, A)
    xr, st, itr, relr = H.pcg(b, 1e-9, 100)
    mg = smg.StructMG(T(A), shape, pattern=7, device=DEV)
    x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    res = mg.solve(T(b.ravel()), x, rtol=1e-9, maxit=100)
    assert res["status"] == 0 and res["rel_resid_true"] < 1e-9
    assert abs(res["iters"] - itr) <= 1
    xg = N(x)
    assert np.abs(xg - xr.ravel()).max() / np.abs(xr).max() < 1e-6
    assert res["levels"] == 4


# the last two cases have hyperplanes of several 64-row chunks and more chunks
# than the persistent factorisation keeps resident, so its workgroups loop
@pytest.mark.parametrize("case", [CASES[1], CASES[3], CASES[5], CASES[6]], ids=_ids)
def test_ilu0_bitexact(case):
    A, H, mg = _pair(case, smoother="ilu0", sym=False)
    g = workloads.rng(13)
    for l in range(H.nlev - 1):
        inf = H.level_info(l)
        dims, S, cm = inf["dims"], inf["S"], inf["cmask"]
        off = workloads.offsets(S)
        for what in (2, 3, 4):
            ref = H.level_data(l, what)
            got = N(mg.export(l, what, torch.empty(ref.shape, dtype=torch.float64, device=DEV)))
            assert np.array_equal(got, ref), f"ILU factor {what} level {l}"
        Lf, Uf, rU = H.level_data(l, 2), H.level_data(l, 3), H.level_data(l, 4).ravel()
        Al = H.level_data(l, 0)
        f = g.uniform(-1, 1, size=dims)
        u = g.uniform(-1, 1, size=dims)
        ec = g.uniform(-1, 1, size=oracle.coarse_dims(dims, cm))
        ug = N(mg.op_presmooth(l, T(f), torch.empty(int(np.prod(dims)), dtype=torch.float64, device=DEV)))
        ref = oracle.tri_solve(off, Uf, rU, oracle.tri_solve(off, Lf, None, f, 0), 1)
        assert np.array_equal(ug, ref.ravel()), f"ILU solve level {l}"
        uo = N(mg.op_postsmooth(l, T(f), T(u), T(ec), torch.empty(int(np.prod(dims)), dtype=torch.float64,
                                                                  device=DEV)))
        uold = oracle.prolong_add(u, ec, cm)
        r = oracle.residual(off, Al, f, uold)
        zc = oracle.tri_solve(off, Uf, rU, oracle.tri_solve(off, Lf, None, r, 0), 1)
        assert np.array_equal(uo, (uold + zc).ravel()), f"ILU correction level {l}"


def test_gmres_ilu_nonsymmetric():
    shape = (40, 36, 10)
    A = workloads.random_sgdia(shape, 19, seed=23, symmetric=False)
    b = workloads.rng(4).uniform(-1, 1, size=shape)
    H = oracle.Hierarchy(shape, 19, A, smoother="ilu0", coarsen="semi_xy")
    xr, st, itr, relr = H.gmres(b, 1e-9, 300, restart=30)
    mg = smg.StructMG(T(A), shape, pattern=19, smoother="ilu0", coarsen="semi_xy", gmres_restart=30, device=DEV)
    x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    res = mg.solve(T(b.ravel()), x, rtol=1e-9, maxit=300, krylov=30)
    assert res["status"] == 0 and res["rel_resid_true"] < 1e-9
    assert abs(res["iters"] - itr) <= 2
    assert np.abs(N(x) - xr.ravel()).max() <= 1e-6 * np.abs(xr).max()


@pytest.mark.parametrize("case", [CASES[0], CASES[6]], ids=_ids)
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_reduced_precision_bitexact(prec, case):
    A, H, mg = _pair(case, prec=prec)
    g = workloads.rng(17)
    for l in range(H.nlev - 1):
        inf = H.level_info(l)
        dims, S, cm = inf["dims"], inf["S"], inf["cmask"]
        off = workloads.offsets(S)
        A32 = H.level_data(l, 5)
        rd32 = H.level_data(l, 6).ravel()
        got = N(mg.export(l, 5, torch.empty(A32.shape, dtype=torch.float32, device=DEV)))
        assert np.array_equal(got, A32), f"{prec} matrix level {l}"
        got = N(mg.export(l, 6, torch.empty(rd32.shape, dtype=torch.float32, device=DEV)))
        assert np.array_equal(got, rd32)
        f = g.uniform(-1, 1, size=dims).astype(np.float32)
        u = g.uniform(-1, 1, size=dims).astype(np.float32)
        ec = g.uniform(-1, 1, size=oracle.coarse_dims(dims, cm)).astype(np.float32)
        f32 = torch.float32
        y = N(mg.op_spmv(l, T(f, f32), torch.empty(f.size, dtype=f32, device=DEV)))
        assert np.array_equal(y, oracle.spmv(off, A32, f).ravel())
        ug = N(mg.op_presmooth(l, T(f, f32), torch.empty(f.size, dtype=f32, device=DEV)))
        assert np.array_equal(ug, oracle.gs_sweep(off, A32, rd32, f, np.zeros(dims, np.float32), 1, 1).ravel())
        uo = N(mg.op_postsmooth(l, T(f, f32), T(u, f32), T(ec, f32), torch.empty(f.size, dtype=f32, device=DEV)))
        ref = oracle.gs_sweep(off, A32, rd32, f, oracle.prolong_add(u, ec, cm), -1, 0)
        assert np.array_equal(uo, ref.ravel())
        rc = N(mg.op_resid_restrict(l, T(f, f32), T(u, f32),
                                    torch.empty(int(np.prod(oracle.coarse_dims(dims, cm))), dtype=f32, device=DEV)))
        assert np.array_equal(rc, oracle.restrict(oracle.residual(off, A32, f, u), cm).ravel())
    # the mixed-precision V-cycle matches the oracle's mixed-precision cycle
    dims = H.level_info(0)["dims"]
    r = workloads.rng(9).uniform(-1, 1, size=dims)
    z = N(mg.precondition(T(r.ravel()), torch.empty(r.size, dtype=torch.float64, device=DEV)))
    zr = H.apply(r).ravel()
    assert np.abs(z - zr).max() <= 1e-5 * np.abs(zr).max()
    # and the outer FP64 PCG reaches 1e-9
    x = torch.zeros(r.size, dtype=torch.float64, device=DEV)
    res = mg.solve(T(r.ravel()), x, rtol=1e-9, maxit=200)
    assert res["status"] == 0 and res["rel_resid_true"] < 1e-9


def test_error_paths():
    A, b = workloads.poisson7(8)
    with pytest.raises(smg.SmgError) as e:
        smg.StructMG(T(A), (8, 8, 8), pattern=5, device=DEV)
    assert e.value.status == smg.SMG_EINVAL
    A2 = A.copy()
    A2[3, 17] = 0.0  # zero diagonal
    with pytest.raises(smg.SmgError) as e:
        smg.StructMG(T(A2), (8, 8, 8), pattern=7, device=DEV)
    assert e.value.status == smg.SMG_EBREAKDOWN


def test_singular_coarsest():
    """A one-level system whose dense operator is [[1, 1], [1, 1]] (1x1x2
    grid, unit diagonal and z couplings): the coarsest inverse meets an exact
    zero pivot and the setup reports a breakdown."""
    shape = (1, 1, 2)
    off = [tuple(int(v) for v in o) for o in workloads.offsets(7)]
    A = np.zeros((7, 2))
    A[off.index((0, 0, 0))] = 1.0
    A[off.index((0, 0, 1)), 0] = 1.0
    A[off.index((0, 0, -1)), 1] = 1.0
    assert np.array_equal(oracle.dense(workloads.offsets(7), A, shape), np.ones((2, 2)))
    with pytest.raises(smg.SmgError) as e:
        smg.StructMG(T(A), shape, pattern=7, device=DEV)
    assert e.value.status == smg.SMG_EBREAKDOWN


# ---------------------------------------------------------------- 3x3 blocks
BCASES = [(12, 10, 9), (17, 16, 8)]
OFF27 = workloads.offsets(27)


def _bpair(shape, prec="fp64", seed=7):
    A = workloads.random_sgdia(shape, 27, seed=seed, block=3)
    H = oracle.Hierarchy(shape, 27, A, block=3, prec=prec)
    mg = smg.StructMG(T(A), shape, pattern=27, block=3, prec=prec, device=DEV)
    return A, H, mg


@pytest.mark.parametrize("shape", BCASES, ids=lambda s: "x".join(map(str, s)))
def test_block_kernels_bitexact(shape):
    A, H, mg = _bpair(shape)
    assert mg.nlev == H.nlev
    for l in range(H.nlev):
        Ar = H.level_data(l, 0)
        got = N(mg.export(l, 0, torch.empty(Ar.shape, dtype=torch.float64, device=DEV)))
        assert np.array_equal(got, Ar), f"block triple product level {l}"
        if l < H.nlev - 1:
            D = H.level_data(l, 1)
            got = N(mg.export(l, 1, torch.empty(D.shape, dtype=torch.float64, device=DEV)))
            assert np.array_equal(got, D), f"block inverses level {l}"
    g = workloads.rng(21)
    for l in range(H.nlev - 1):
        inf = H.level_info(l)
        dims, cm = inf["dims"], inf["cmask"]
        cdims = oracle.coarse_dims(dims, cm)
        Al, D = H.level_data(l, 0), H.level_data(l, 1)
        f = g.uniform(-1, 1, size=dims + (3,))
        u = g.uniform(-1, 1, size=dims + (3,))
        ec = g.uniform(-1, 1, size=cdims + (3,))
        n3, nc3 = f.size, ec.size
        y = N(mg.op_spmv(l, T(f.ravel()), torch.empty(n3, dtype=torch.float64, device=DEV)))
        assert np.array_equal(y, oracle.bspmv(OFF27, Al, f).ravel()), f"block SpMV level {l}"
        ug = N(mg.op_presmooth(l, T(f.ravel()), torch.empty(n3, dtype=torch.float64, device=DEV)))
        ur = oracle.bgs_sweep(OFF27, Al, D, f, np.zeros_like(f), 1, 1)
        assert np.array_equal(ug, ur.ravel()), f"forward block GS level {l}: {np.abs(ug - ur.ravel()).max()}"
        rc = N(mg.op_resid_restrict(l, T(f.ravel()), T(u.ravel()), torch.empty(nc3, dtype=torch.float64, device=DEV)))
        rr = oracle.restrict(f - oracle.bspmv(OFF27, Al, u), cm, bs=3)
        assert np.array_equal(rc, rr.ravel()), f"block resid+restrict level {l}"
        uo = N(mg.op_postsmooth(l, T(f.ravel()), T(u.ravel()), T(ec.ravel()),
                                torch.empty(n3, dtype=torch.float64, device=DEV)))
        ref = oracle.bgs_sweep(OFF27, Al, D, f, oracle.prolong_add(u, ec, cm, bs=3), -1, 0)
        assert np.array_equal(uo, ref.ravel()), f"backward block GS level {l}: {np.abs(uo - ref.ravel()).max()}"
    # whole V-cycle, twice (buffers reused)
    dims = H.level_info(0)["dims"]
    r = workloads.rng(9).uniform(-1, 1, size=dims + (3,))
    z = N(mg.precondition(T(r.ravel()), torch.empty(r.size, dtype=torch.float64, device=DEV)))
    zr = H.apply(r).ravel()
    assert np.abs(z - zr).max() <= 1e-12 * np.abs(zr).max()
    z2 = N(mg.precondition(T(r.ravel()), torch.empty(r.size, dtype=torch.float64, device=DEV)))
    assert np.array_equal(z, z2)


def test_block_elasticity_pcg():
    A, b = workloads.elasticity27(12, seed=4)
    shape = (12, 12, 12)
    H = oracle.Hierarchy(shape, 27, A, block=3)
    xr, st, itr, relr = H.pcg(b, 1e-8, 200)
    mg = smg.StructMG(T(A), shape, pattern=27, block=3, device=DEV)
    x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    res = mg.solve(T(b.ravel()), x, rtol=1e-8, maxit=200)
    assert res["status"] == 0 and res["rel_resid_true"] < 1e-8
    assert abs(res["iters"] - itr) <= 1
    assert np.abs(N(x) - xr.ravel()).max() <= 1e-5 * np.abs(xr).max()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_block_reduced_precision_bitexact(prec):
    shape = BCASES[0]
    A, H, mg = _bpair(shape, prec=prec)
    f32 = torch.float32
    g = workloads.rng(23)
    for l in range(H.nlev - 1):
        inf = H.level_info(l)
        dims, cm = inf["dims"], inf["cmask"]
        A32, D32 = H.level_data(l, 5), H.level_data(l, 6)
        got = N(mg.export(l, 5, torch.empty(A32.shape, dtype=f32, device=DEV)))
        assert np.array_equal(got, A32), f"{prec} block matrix level {l}"
        f = g.uniform(-1, 1, size=dims + (3,)).astype(np.float32)
        u = g.uniform(-1, 1, size=dims + (3,)).astype(np.float32)
        ec = g.uniform(-1, 1, size=oracle.coarse_dims(dims, cm) + (3,)).astype(np.float32)
        y = N(mg.op_spmv(l, T(f.ravel(), f32), torch.empty(f.size, dtype=f32, device=DEV)))
        assert np.array_equal(y, oracle.bspmv(OFF27, A32, f).ravel())
        ug = N(mg.op_presmooth(l, T(f.ravel(), f32), torch.empty(f.size, dtype=f32, device=DEV)))
        assert np.array_equal(ug, oracle.bgs_sweep(OFF27, A32, D32, f, np.zeros_like(f), 1, 1).ravel())
        uo = N(mg.op_postsmooth(l, T(f.ravel(), f32), T(u.ravel(), f32), T(ec.ravel(), f32),
                                torch.empty(f.size, dtype=f32, device=DEV)))
        ref = oracle.bgs_sweep(OFF27, A32, D32, f, oracle.prolong_add(u, ec, cm, bs=3), -1, 0)
        assert np.array_equal(uo, ref.ravel())
    dims = H.level_info(0)["dims"]
    r = workloads.rng(9).uniform(-1, 1, size=dims + (3,))
    z = N(mg.precondition(T(r.ravel()), torch.empty(r.size, dtype=torch.float64, device=DEV)))
    zr = H.apply(r).ravel()
    assert np.abs(z - zr).max() <= 1e-5 * np.abs(zr).max()
    x = torch.zeros(r.size, dtype=torch.float64, device=DEV)
    res = mg.solve(T(r.ravel()), x, rtol=1e-8, maxit=300)
    assert res["status"] == 0 and res["rel_resid_true"] < 1e-8


def test_single_level_hierarchy():
    """A grid small enough to be its own coarsest level: the dense operator is
    assembled from the finest (7-point) pattern and solved exactly."""
    shape = (5, 6, 7)
    A, b = workloads.reservoir7(shape, seed=56)
    mg = smg.StructMG(T(A), shape, pattern=7, max_coarse=512, device=DEV)
    assert mg.nlev == 1
    f = workloads.rng(8).uniform(-1, 1, size=int(np.prod(shape)))
    u = N(mg.op_coarse_solve(T(f), torch.empty(f.size, dtype=torch.float64, device=DEV)))
    ref = np.linalg.solve(oracle.dense(workloads.offsets(7), A, shape), f)
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()
    H = oracle.Hierarchy(shape, 7, A, max_coarse=512)
    xr, st, itr, relr = H.pcg(b, 1e-9, 50)
    x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    res = mg.solve(T(b.ravel()), x, rtol=1e-9, maxit=50)
    assert res["status"] == 0 and res["rel_resid_true"] < 1e-9 and abs(res["iters"] - itr) <= 1


# dense coarsest inverses of every size class: blocked panels of 32 and 16
# columns with one row per thread, 9-column panels with two rows per thread,
# and one pivot step per pair of launches beyond 2048 unknowns
@pytest.mark.parametrize("shape,pat", [((5, 6, 7), 7), ((10, 10, 10), 27), ((12, 12, 12), 7), ((13, 13, 13), 27)],
                         ids=["210", "1000", "1728", "2197"])
def test_dense_coarsest_sizes(shape, pat):
    if pat == 7:
        A, _ = workloads.reservoir7(shape, seed=57)
    else:
        A = workloads.random_sgdia(shape, pat, seed=58, symmetric=False)
    mg = smg.StructMG(T(A), shape, pattern=pat, max_coarse=4096, min_coarse=64, device=DEV)  # one level
    assert mg.nlev == 1
    f = workloads.rng(8).uniform(-1, 1, size=int(np.prod(shape)))
    u = N(mg.op_coarse_solve(T(f), torch.empty(f.size, dtype=torch.float64, device=DEV)))
    M = oracle.dense(workloads.offsets(pat), A, shape)
    ref = np.linalg.solve(M, f)
    assert np.abs(u - ref).max() <= 1e-13 * np.abs(ref).max() * max(1.0, np.linalg.cond(M) / 1e3)


@pytest.mark.parametrize("kind", ["gs_fp64", "gs_fp32", "block_fp16", "lgs_fp64", "operator_fp64", "cell_fp32",
                                  "ilu27_fp64"])
def test_graph_replay_identical(kind):
    """PCG with the V-cycle replayed from a captured graph gives the same bits
    as launching its kernels one by one, also across repeated solves (line
    GS, operator-dependent and cell-centred transfers and ILU masks
    included)."""
    if kind == "block_fp16":
        shape = (12, 12, 12)
        A, b = workloads.elasticity27(12, seed=4)
        mg = smg.StructMG(T(A), shape, pattern=27, block=3, prec="fp16", device=DEV)
    elif kind != "gs_fp64" and kind != "gs_fp32":
        shape = (33, 17, 20)
        A = workloads.random_sgdia(shape, 19, seed=5)
        b = workloads.rng(6).uniform(-1, 1, size=shape)
        opts = {"lgs_fp64": dict(smoother="lgs"), "operator_fp64": dict(interp="operator"),
                "cell_fp32": dict(interp="cell", prec="fp32"), "ilu27_fp64": dict(smoother="ilu0", ilu_mask=27)}
        mg = smg.StructMG(T(A), shape, pattern=19, device=DEV, **opts[kind])
    else:
        shape = (33, 17, 20)
        A = workloads.random_sgdia(shape, 7, seed=5)
        b = workloads.rng(6).uniform(-1, 1, size=shape)
        mg = smg.StructMG(T(A), shape, pattern=7, prec=kind.split("_")[1], device=DEV)
    out = []
    for graph in (True, False, True):
        mg.set_graph(graph)
        x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
        res = mg.solve(T(b.ravel()), x, rtol=1e-9, maxit=200)
        assert res["status"] == 0
        out.append((N(x), res["iters"]))
    for xg, it in out[1:]:
        assert np.array_equal(xg, out[0][0]) and it == out[0][1]


# level 0 small enough for the one-workgroup hyperplane sweep (ragged shapes,
# every pattern, every V-cycle precision); each has a coarser level
HP_CASES = [((7, 11, 5), 27, "fp64"), ((9, 4, 13), 19, "fp64"), ((16, 16, 16), 7, "fp64"),
            ((6, 13, 10), 27, "fp32"), ((12, 5, 9), 7, "fp16"), ((10, 9, 8), 19, "fp16")]


@pytest.mark.parametrize("shape,pat,prec", HP_CASES, ids=lambda v: str(v))
def test_small_level_sweeps_bitexact(shape, pat, prec):
    A = workloads.random_sgdia(shape, pat, seed=19)
    H = oracle.Hierarchy(shape, pat, A, prec=prec)
    mg = smg.StructMG(T(A), shape, pattern=pat, prec=prec, device=DEV)
    assert mg.nlev == H.nlev and H.nlev >= 2
    inf = H.level_info(0)
    dims, cm = inf["dims"], inf["cmask"]
    off = workloads.offsets(pat)
    if prec == "fp64":
        Al, rd, dt, npt = H.level_data(0, 0), H.level_data(0, 1).ravel(), torch.float64, np.float64
    else:
        Al, rd, dt, npt = H.level_data(0, 5), H.level_data(0, 6).ravel(), torch.float32, np.float32
    g = workloads.rng(29)
    for rep in range(2):
        f = g.uniform(-1, 1, size=dims).astype(npt)
        u = g.uniform(-1, 1, size=dims).astype(npt)
        ec = g.uniform(-1, 1, size=oracle.coarse_dims(dims, cm)).astype(npt)
        ug = N(mg.op_presmooth(0, T(f, dt), torch.empty(f.size, dtype=dt, device=DEV)))
        assert np.array_equal(ug, oracle.gs_sweep(off, Al, rd, f, np.zeros(dims, npt), 1, 1).ravel())
        uo = N(mg.op_postsmooth(0, T(f, dt), T(u, dt), T(ec, dt), torch.empty(f.size, dtype=dt, device=DEV)))
        ref = oracle.gs_sweep(off, Al, rd, f, oracle.prolong_add(u, ec, cm), -1, 0)
        assert np.array_equal(uo, ref.ravel())
    # and the whole solve
    b = workloads.rng(30).uniform(-1, 1, size=dims)
    x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    res = mg.solve(T(b.ravel()), x, rtol=1e-9, maxit=200)
    assert res["status"] == 0 and res["rel_resid_true"] < 1e-9


# line Gauss-Seidel: the five level shapes above plus columns longer than
# one chunk (nz > 512: one column per chunk) and one-point columns
LGS_CASES = CASES + [((16, 10, 520), 7, "full", 0), ((30, 20, 1), 19, "full", 0)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", LGS_CASES, ids=_ids)
def test_lgs_bitexact(case, prec):
    A, H, mg = _pair(case, smoother="lgs", prec=prec, sym=False)
    g = workloads.rng(21)
    for l in range(H.nlev - 1):
        inf = H.level_info(l)
        dims, S, cm = inf["dims"], inf["S"], inf["cmask"]
        n = int(np.prod(dims))
        off = workloads.offsets(S)
        tr, tc = H.level_data(l, 7), H.level_data(l, 8)
        for what, ref in ((7, tr), (8, tc)):
            got = N(mg.export(l, what, torch.empty(ref.shape, dtype=torch.float64, device=DEV)))
            assert np.array_equal(got, ref), f"Thomas factor {what} level {l}"
        if prec == "fp64":
            Al, dt, npt = H.level_data(l, 0), torch.float64, np.float64
        else:
            Al, dt, npt = H.level_data(l, 5), torch.float32, np.float32
            tr, tc = tr.astype(np.float32), tc.astype(np.float32)
        f = g.uniform(-1, 1, size=dims).astype(npt)
        u = g.uniform(-1, 1, size=dims).astype(npt)
        ec = g.uniform(-1, 1, size=oracle.coarse_dims(dims, cm)).astype(npt)
        ug = N(mg.op_presmooth(l, T(f, dt), torch.empty(n, dtype=dt, device=DEV)))
        ur = oracle.lgs_sweep(off, Al, tr, tc, f, np.zeros(dims, npt), 1, 1)
        assert np.array_equal(ug, ur.ravel()), f"forward LGS level {l}: {np.abs(ug - ur.ravel()).max()}"
        uo = N(mg.op_postsmooth(l, T(f, dt), T(u, dt), T(ec, dt), torch.empty(n, dtype=dt, device=DEV)))
        ref = oracle.lgs_sweep(off, Al, tr, tc, f, oracle.prolong_add(u, ec, cm), -1, 0)
        assert np.array_equal(uo, ref.ravel()), f"backward LGS level {l}: {np.abs(uo - ref.ravel()).max()}"


@pytest.mark.parametrize("case", [CASES[1], CASES[3], CASES[5]], ids=_ids)
def test_lgs_vcycle_and_repeat(case):
    A, H, mg = _pair(case, smoother="lgs", sym=False)
    dims = H.level_info(0)["dims"]
    r = workloads.rng(9).uniform(-1, 1, size=dims)
    zr = H.apply(r).ravel()
    z = None
    for _ in range(3):  # buffers and sentinels are reused across cycles
        zi = N(mg.precondition(T(r.ravel()), torch.empty(r.size, dtype=torch.float64, device=DEV)))
        assert np.abs(zi - zr).max() <= 1e-12 * np.abs(zr).max()
        if z is None:
            z = zi
        assert np.array_equal(zi, z)


def test_gmres_lgs_weather_like():
    """Anisotropic weather-like 19-point operator: GMRES(30) with the line GS
    V-cycle reaches 1e-9 in the oracle's iteration count (+-1)."""
    shape = (48, 40, 24)
    A, b = workloads.weather19(shape, seed=3)
    b = b.reshape(shape)
    H = oracle.Hierarchy(shape, 19, A, smoother="lgs", coarsen="semi_xy")
    xr, st, itr, relr = H.gmres(b, 1e-9, 200, restart=30)
    assert st == 0
    for prec in ("fp64", "fp32"):
        mg = smg.StructMG(T(A), shape, pattern=19, smoother="lgs", coarsen="semi_xy", prec=prec, gmres_restart=30,
                          device=DEV)
        x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
        res = mg.solve(T(b.ravel()), x, rtol=1e-9, maxit=200, krylov=30)
        assert res["status"] == 0 and res["rel_resid_true"] < 1e-9, (prec, res)
        assert abs(res["iters"] - itr) <= 1, (prec, res["iters"], itr)
        if prec == "fp64":
            assert np.abs(N(x) - xr.ravel()).max() / np.abs(xr).max() < 1e-6


def test_fgmres_reduced_precision_cycle_keeps_iterations():
    """Weather-like operator with the ILU(0) V-cycle: flexible GMRES(30) with
    the V-cycle in FP32 storage needs as many iterations as with the FP64
    V-cycle (+-1), which needs the oracle's count (+-1); every run's true FP64
    residual meets the tolerance and the FP64 run's solution matches the
    oracle's."""
    shape = (64, 48, 24)
    A, b = workloads.weather19(shape, seed=3)
    b = b.reshape(shape)
    H = oracle.Hierarchy(shape, 19, A, smoother="ilu0", coarsen="semi_xy")
    xr, st, itr, relr = H.gmres(b, 1e-9, 200, restart=30)
    assert st == 0
    its = {}
    for prec in ("fp64", "fp32"):
        mg = smg.StructMG(T(A), shape, pattern=19, smoother="ilu0", coarsen="semi_xy", prec=prec, gmres_restart=30,
                          device=DEV)
        x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
        res = mg.solve(T(b.ravel()), x, rtol=1e-9, maxit=200, krylov=30)
        assert res["status"] == 0 and res["rel_resid_true"] < 1e-9, (prec, res)
        its[prec] = res["iters"]
        if prec == "fp64":
            assert abs(res["iters"] - itr) <= 1
            assert np.abs(N(x) - xr.ravel()).max() / np.abs(xr).max() < 1e-6
        mg.close()
    assert abs(its["fp32"] - its["fp64"]) <= 1, its


# ILU(0) of the finest matrix on a mask other than its pattern (fewer or more
# fill-ins); coarse levels keep their own pattern
ILU_MASK_CASES = [(CASES[1], 7), (CASES[1], 27), (CASES[0], 19), (CASES[0], 27), (CASES[5], 27), (CASES[3], 7)]


@pytest.mark.parametrize("case,mask", ILU_MASK_CASES, ids=lambda v: str(v) if isinstance(v, int) else _ids(v))
def test_ilu0_mask_bitexact(case, mask):
    shape, pat, coarsen, semi = case
    A = workloads.random_sgdia(shape, pat, seed=3, symmetric=False)
    H = oracle.Hierarchy(shape, pat, A, smoother="ilu0", coarsen=coarsen, semi_levels=semi, ilu_mask=mask)
    mg = smg.StructMG(T(A), shape, pattern=pat, smoother="ilu0", coarsen=coarsen, semi_levels=semi, ilu_mask=mask,
                      device=DEV)
    assert mg.nlev == H.nlev and H.level_info(0)["Sm"] == mask
    g = workloads.rng(17)
    for l in range(H.nlev - 1):
        inf = H.level_info(l)
        dims, cm = inf["dims"], inf["cmask"]
        offm = workloads.offsets(inf["Sm"])
        for what in (2, 3, 4):
            ref = H.level_data(l, what)
            got = N(mg.export(l, what, torch.empty(ref.shape, dtype=torch.float64, device=DEV)))
            assert np.array_equal(got, ref), f"ILU factor {what} level {l}"
        Lf, Uf, rU = H.level_data(l, 2), H.level_data(l, 3), H.level_data(l, 4).ravel()
        f = g.uniform(-1, 1, size=dims)
        u = g.uniform(-1, 1, size=dims)
        ec = g.uniform(-1, 1, size=oracle.coarse_dims(dims, cm))
        n = int(np.prod(dims))
        ug = N(mg.op_presmooth(l, T(f), torch.empty(n, dtype=torch.float64, device=DEV)))
        ref = oracle.tri_solve(offm, Uf, rU, oracle.tri_solve(offm, Lf, None, f, 0), 1)
        assert np.array_equal(ug, ref.ravel()), f"ILU solve level {l}"
        uo = N(mg.op_postsmooth(l, T(f), T(u), T(ec), torch.empty(n, dtype=torch.float64, device=DEV)))
        uold = oracle.prolong_add(u, ec, cm)
        r = oracle.residual(workloads.offsets(inf["S"]), H.level_data(l, 0), f, uold)
        zc = oracle.tri_solve(offm, Uf, rU, oracle.tri_solve(offm, Lf, None, r, 0), 1)
        assert np.array_equal(uo, (uold + zc).ravel()), f"ILU correction level {l}"
    dims = H.level_info(0)["dims"]
    rr = workloads.rng(9).uniform(-1, 1, size=dims)
    zr = H.apply(rr).ravel()
    z = N(mg.precondition(T(rr.ravel()), torch.empty(rr.size, dtype=torch.float64, device=DEV)))
    assert np.abs(z - zr).max() <= 1e-12 * np.abs(zr).max()


# cell-centred piecewise-constant transfers (every level keeps the finest
# pattern; odd sizes give coarse cells with a single child)
CELL_CASES = [(CASES[0], "gs", "fp64", "cell"), (CASES[1], "gs", "fp64", "cell"), (CASES[2], "gs", "fp64", "cell"),
              (CASES[4], "gs", "fp64", "cell"), (CASES[3], "ilu0", "fp64", "cell"), (CASES[1], "lgs", "fp64", "cell"),
              (CASES[0], "gs", "fp32", "cell"), (CASES[6], "gs", "fp64", "cell"),
              (CASES[0], "gs", "fp64", "cell_trilinear"), (CASES[1], "gs", "fp64", "cell_trilinear"),
              (CASES[2], "ilu0", "fp64", "cell_trilinear"), (CASES[4], "gs", "fp32", "cell_trilinear"),
              (CASES[3], "lgs", "fp64", "cell_trilinear")]


@pytest.mark.parametrize("case,smoother,prec,interp", CELL_CASES,
                         ids=lambda v: v if isinstance(v, str) else _ids(v))
def test_cell_centred_bitexact(case, smoother, prec, interp):
    shape, pat, coarsen, semi = case
    A = workloads.random_sgdia(shape, pat, seed=3, symmetric=smoother != "ilu0")
    H = oracle.Hierarchy(shape, pat, A, smoother=smoother, coarsen=coarsen, semi_levels=semi, prec=prec,
                         interp=interp)
    mg = smg.StructMG(T(A), shape, pattern=pat, smoother=smoother, coarsen=coarsen, semi_levels=semi, prec=prec,
                      interp=interp, gmres_restart=30, device=DEV)
    assert mg.nlev == H.nlev
    prolong = oracle.prolong_add_cc if interp == "cell" else oracle.prolong_add_c64
    dt, npt = (torch.float64, np.float64) if prec == "fp64" else (torch.float32, np.float32)
    g = workloads.rng(31)
    for l in range(H.nlev):
        inf = H.level_info(l)
        assert mg.level_info(l)["dims"] == inf["dims"] and inf["S"] == (pat if interp == "cell" or l == 0 else 27)
        Ar = H.level_data(l, 0)
        got = N(mg.export(l, 0, torch.empty(Ar.shape, dtype=torch.float64, device=DEV)))
        assert np.array_equal(got, Ar), f"cell RAP level {l}"
        if l == H.nlev - 1:
            break
        dims, cm = inf["dims"], inf["cmask"]
        cdims = oracle.coarse_dims(dims, cm, cell=True)
        Al = Ar if prec == "fp64" else H.level_data(l, 5)
        off = workloads.offsets(inf["S"])
        f = g.uniform(-1, 1, size=dims).astype(npt)
        u = g.uniform(-1, 1, size=dims).astype(npt)
        ec = g.uniform(-1, 1, size=cdims).astype(npt)
        rc = N(mg.op_resid_restrict(l, T(f, dt), T(u, dt), torch.empty(int(np.prod(cdims)), dtype=dt, device=DEV)))
        assert np.array_equal(rc, oracle.restrict_cc(oracle.residual(off, Al, f, u), cm).ravel())
        uf = T(u.copy(), dt)
        mg.op_prolong_add(l, T(ec, dt), uf)
        assert np.array_equal(N(uf).ravel(), prolong(u, ec, cm).ravel())
        if smoother == "gs":
            rd = H.level_data(l, 1 if prec == "fp64" else 6).ravel()
            uo = N(mg.op_postsmooth(l, T(f, dt), T(u, dt), T(ec, dt), torch.empty(int(np.prod(dims)), dtype=dt,
                                                                                  device=DEV)))
            ref = oracle.gs_sweep(off, Al, rd, f, prolong(u, ec, cm), -1, 0)
            assert np.array_equal(uo, ref.ravel()), f"cell post-smoothing level {l}"
    dims = H.level_info(0)["dims"]
    r = workloads.rng(9).uniform(-1, 1, size=dims)
    z = N(mg.precondition(T(r.ravel()), torch.empty(r.size, dtype=torch.float64, device=DEV)))
    zr = H.apply(r).ravel()  # the oracle's cycle in the hierarchy's precision
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert np.abs(z - zr).max() <= tol * np.abs(zr).max()
    if smoother == "gs" and prec == "fp64":
        # the trilinear interpolation with R != P^T gives a non-symmetric cycle: GMRES
        kr = 0 if interp == "cell" else 30
        b = workloads.rng(4).uniform(-1, 1, size=dims)
        xr, st, itr, _ = H.pcg(b, 1e-9, 300) if kr == 0 else H.gmres(b, 1e-9, 300, restart=kr)
        x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
        res = mg.solve(T(b.ravel()), x, rtol=1e-9, maxit=300, krylov=kr)
        assert st == 0 and res["status"] == 0 and res["rel_resid_true"] < 1e-9
        assert abs(res["iters"] - itr) <= 1


# operator-dependent vertex interpolation (weights from each level's stencil)
OD_CASES = [(CASES[0], "gs", "fp64"), (CASES[1], "gs", "fp64"), (CASES[2], "gs", "fp64"), (CASES[4], "gs", "fp64"),
            (CASES[3], "ilu0", "fp64"), (CASES[1], "lgs", "fp64"), (CASES[0], "gs", "fp32"), (CASES[6], "gs", "fp64")]


@pytest.mark.parametrize("case,smoother,prec", OD_CASES, ids=lambda v: v if isinstance(v, str) else _ids(v))
def test_operator_interp_bitexact(case, smoother, prec):
    shape, pat, coarsen, semi = case
    A = workloads.random_sgdia(shape, pat, seed=3, symmetric=smoother != "ilu0")
    H = oracle.Hierarchy(shape, pat, A, smoother=smoother, coarsen=coarsen, semi_levels=semi, prec=prec,
                         interp="operator")
    mg = smg.StructMG(T(A), shape, pattern=pat, smoother=smoother, coarsen=coarsen, semi_levels=semi, prec=prec,
                      interp="operator", device=DEV)
    assert mg.nlev == H.nlev
    dt, npt = (torch.float64, np.float64) if prec == "fp64" else (torch.float32, np.float32)
    g = workloads.rng(37)
    for l in range(H.nlev):
        inf = H.level_info(l)
        Ar = H.level_data(l, 0)
        got = N(mg.export(l, 0, torch.empty(Ar.shape, dtype=torch.float64, device=DEV)))
        assert np.array_equal(got, Ar), f"operator-dependent RAP level {l}"
        if l == H.nlev - 1:
            break
        W = H.level_data(l, 9)
        gw = N(mg.export(l, 9, torch.empty(W.shape, dtype=torch.float64, device=DEV)))
        assert np.array_equal(gw, W), f"interpolation weights level {l}"
        dims, cm = inf["dims"], inf["cmask"]
        cdims = oracle.coarse_dims(dims, cm)
        Al = Ar if prec == "fp64" else H.level_data(l, 5)
        Wl = W.astype(npt)
        off = workloads.offsets(inf["S"])
        f = g.uniform(-1, 1, size=dims).astype(npt)
        u = g.uniform(-1, 1, size=dims).astype(npt)
        ec = g.uniform(-1, 1, size=cdims).astype(npt)
        rc = N(mg.op_resid_restrict(l, T(f, dt), T(u, dt), torch.empty(int(np.prod(cdims)), dtype=dt, device=DEV)))
        assert np.array_equal(rc, oracle.restrict_od(oracle.residual(off, Al, f, u), Wl, cm).ravel())
        uf = T(u.copy(), dt)
        mg.op_prolong_add(l, T(ec, dt), uf)
        assert np.array_equal(N(uf).ravel(), oracle.prolong_add_od(u, Wl, ec, cm).ravel())
        if smoother == "gs":
            rd = H.level_data(l, 1 if prec == "fp64" else 6).ravel()
            uo = N(mg.op_postsmooth(l, T(f, dt), T(u, dt), T(ec, dt), torch.empty(int(np.prod(dims)), dtype=dt,
                                                                                  device=DEV)))
            ref = oracle.gs_sweep(off, Al, rd, f, oracle.prolong_add_od(u, Wl, ec, cm), -1, 0)
            assert np.array_equal(uo, ref.ravel()), f"post-smoothing level {l}"
    dims = H.level_info(0)["dims"]
    r = workloads.rng(9).uniform(-1, 1, size=dims)
    z = N(mg.precondition(T(r.ravel()), torch.empty(r.size, dtype=torch.float64, device=DEV)))
    zr = H.apply(r).ravel()
    assert np.abs(z - zr).max() <= (1e-12 if prec == "fp64" else 1e-5) * np.abs(zr).max()
    if smoother == "gs" and prec == "fp64":
        b = workloads.rng(4).uniform(-1, 1, size=dims)
        xr, st, itr, _ = H.pcg(b, 1e-9, 300)
        x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
        res = mg.solve(T(b.ravel()), x, rtol=1e-9, maxit=300)
        assert st == 0 and res["status"] == 0 and res["rel_resid_true"] < 1e-9
        assert abs(res["iters"] - itr) <= 1

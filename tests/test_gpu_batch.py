"""GPU tests of the batched lockstep solve of independent systems.

A batched preconditioner application runs, per system, exactly the kernels of
that system's single-system V-cycle, so it must equal smg_precondition bit
for bit, whatever the merge order of the sweep tiles and the persistent grid.
The batched PCG solve is checked per system against the oracle's PCG
(iteration count within one, true residual below the tolerance, solution
within the bound implied by the tolerance), with and without the captured
graph (which must give identical bits).
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

# reservoir-like systems of mixed sizes: tiny ones are a single (dense) level,
# the others have 2-6 levels; 33 and 40 in y give sheared tilings
SHAPES = [(16, 16, 16), (20, 17, 23), (9, 30, 12), (33, 18, 16), (8, 8, 8), (40, 24, 19), (5, 6, 7), (17, 40, 33)]
KW = dict(coarsen="full", semi_levels=3, max_coarse=512)


def T(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def N(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _systems(shapes, seed0=50):
    out = []
    for k, s in enumerate(shapes):
        A, b = workloads.reservoir7(s, seed=seed0 + k)
        out.append((s, A, b))
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_batch_precondition_equals_single(prec):
    sysl = _systems(SHAPES)
    B = smg.StructMGBatch([T(A) for _, A, _ in sysl], [s for s, _, _ in sysl], pattern=7, prec=prec, **KW)
    singles = [smg.StructMG(T(A), s, pattern=7, prec=prec, **KW) for s, A, _ in sysl]
    g = workloads.rng(3)
    rs = [T(g.uniform(-1, 1, size=int(np.prod(s)))) for s, _, _ in sysl]
    ref = [N(m.precondition(r, torch.empty_like(r))) for m, r in zip(singles, rs)]
    for k, m in enumerate(singles):
        assert B.levels(k) == m.nlev
    for order, grid in [(1, 0), (0, 0), (1, 3), (0, 1)]:
        B.set_schedule(order, grid)
        for rep in range(2):  # twice: the sweeps' sentinel state carries over
            zs = [torch.full_like(r, np.nan) for r in rs]
            B.precondition(rs, zs)
            for k in range(len(sysl)):
                got = N(zs[k])
                assert np.array_equal(got, ref[k]), f"system {k} {SHAPES[k]} order {order} grid {grid} rep {rep}"


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_solve_matches_oracle(prec):
    sysl = _systems(SHAPES)
    B = smg.StructMGBatch([T(A) for _, A, _ in sysl], [s for s, _, _ in sysl], pattern=7, prec=prec, **KW)
    bs = [T(b.ravel()) for _, _, b in sysl]
    xs = [torch.zeros_like(b) for b in bs]
    st, res = B.solve(bs, xs, rtol=1e-9, maxit=200)
    assert st == smg.SMG_OK
    for k, (s, A, b) in enumerate(sysl):
        H = oracle.Hierarchy(s, 7, A, prec=prec, **KW)
        xr, ost, itr, relr = H.pcg(b, 1e-9, 200)
        assert ost == 0
        r = res[k]
        assert r["status"] == smg.SMG_OK and r["rel_resid_true"] < 1e-9, (k, r)
        assert abs(r["iters"] - itr) <= 1, (k, r["iters"], itr)
        x = N(xs[k])
        assert np.abs(x - xr.ravel()).max() <= 1e-6 * np.abs(xr).max(), k
        # the true residual, recomputed here
        rr = b.ravel() - oracle.spmv(workloads.offsets(7), A, x.reshape(s)).ravel()
        assert np.linalg.norm(rr) / np.linalg.norm(b) < 1e-9


def test_batch_graph_and_restart():
    sysl = _systems(SHAPES[:6], seed0=80)
    B = smg.StructMGBatch([T(A) for _, A, _ in sysl], [s for s, _, _ in sysl], pattern=7, prec="fp32", **KW)
    bs = [T(b.ravel()) for _, _, b in sysl]
    out = {}
    for graph in (True, False):
        B.set_graph(graph)
        xs = [torch.zeros_like(b) for b in bs]
        st, res = B.solve(bs, xs, rtol=1e-9, maxit=200)
        assert st == smg.SMG_OK
        out[graph] = ([N(x) for x in xs], [r["iters"] for r in res])
    for a, b in zip(out[True][0], out[False][0]):
        assert np.array_equal(a, b)
    assert out[True][1] == out[False][1]
    # a second solve from a nonzero start reuses the captured graph
    B.set_graph(True)
    xs = [T(workloads.rng(k).uniform(-1, 1, size=b.numel())) for k, b in enumerate(bs)]
    st, res = B.solve(bs, xs, rtol=1e-9, maxit=200)
    assert st == smg.SMG_OK and all(r["rel_resid_true"] < 1e-9 for r in res)
    # iteration limit: every system reports not converged
    xs = [torch.zeros_like(b) for b in bs]
    st, res = B.solve(bs, xs, rtol=1e-9, maxit=2)
    assert st == smg.SMG_ENOTCONV
    assert all(r["status"] == smg.SMG_ENOTCONV and r["iters"] == 2 for r in res)
    # a limit that is not a multiple of the iterations per graph launch stops
    # every system on the device at exactly that count
    xs = [torch.zeros_like(b) for b in bs]
    st, res = B.solve(bs, xs, rtol=1e-9, maxit=5)
    assert st == smg.SMG_ENOTCONV
    assert all(r["status"] == smg.SMG_ENOTCONV and r["iters"] == 5 for r in res)


def test_batch_tune_keeps_results():
    sysl = _systems(SHAPES[:5], seed0=90)
    B = smg.StructMGBatch([T(A) for _, A, _ in sysl], [s for s, _, _ in sysl], pattern=7, prec="fp32", **KW)
    bs = [T(b.ravel()) for _, _, b in sysl]
    xs0 = [torch.zeros_like(b) for b in bs]
    B.solve(bs, xs0, rtol=1e-9, maxit=200)
    choice = B.tune()
    assert choice["order"] in (0, 1) and choice["grid"] > 0 and choice["ms_per_vcycle"] > 0
    assert all(s in (0, 1, 2) for s in choice["tile_shapes"]) and choice["tile_shapes"][0] in (1, 2)
    xs1 = [torch.zeros_like(b) for b in bs]
    st, res = B.solve(bs, xs1, rtol=1e-9, maxit=200)
    assert st == smg.SMG_OK
    for a, b in zip(xs0, xs1):
        assert np.array_equal(N(a), N(b))


def test_batch_tile_shapes_bitexact():
    """Each level's sweeps in either tile shape give the batched V-cycle's
    bits (the schedule is the sequential order whatever the shape)."""
    sysl = _systems(SHAPES, seed0=95)
    B = smg.StructMGBatch([T(A) for _, A, _ in sysl], [s for s, _, _ in sysl], pattern=7, prec="fp64", **KW)
    g = workloads.rng(96)
    rs = [T(g.standard_normal(int(np.prod(s)))) for s, _, _ in sysl]
    zs0 = [torch.empty_like(r) for r in rs]
    B.precondition(rs, zs0)
    ref = [N(z) for z in zs0]
    nl = max(B.levels(k) for k in range(B.n))
    # level 0 (7 points): both shapes; coarser levels (27 points): sheared,
    # and rectangles only where every system has a single tile row there
    for shape in (1, 2):
        B.set_tile_shape(0, shape)
        assert B.tile_shape(0) == shape
        for l in range(1, nl - 1):
            B.set_tile_shape(l, 1)
        zs = [torch.empty_like(r) for r in rs]
        B.precondition(rs, zs)
        B.precondition(rs, zs)
        for a, z in zip(ref, zs):
            assert np.array_equal(a, N(z)), f"shape {shape}"
    bs = [T(b.ravel()) for _, _, b in sysl]
    xs = [torch.zeros_like(b) for b in bs]
    st, res = B.solve(bs, xs, rtol=1e-9, maxit=200)
    assert st == smg.SMG_OK

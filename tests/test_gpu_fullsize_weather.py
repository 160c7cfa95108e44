"""Parity at full size for the weather-like case: 512 x 512 x 64, 19-point
nonsymmetric stencil, GMRES(30) with an ILU(0) V-cycle and x-y
semi-coarsening, configured as the benchmark configures it, in FP64 and with
an FP32 V-cycle.

The finest level is compared element by element with the oracle: the masked
matrix, the ILU(0) factors, SpMV, the ILU pre-smoothing (two triangular
solves), residual + restriction, and the post-smoothing correction; the
level-1 stencil product at sampled coarse points; both solves through the
oracle's true residual.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests import helpers

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_21932_amd as smg  # noqa: E402

DEV = torch.device("cuda:0")
SHAPE = (512, 512, 64)
CMASK = 3  # x-y semi-coarsening
KW = dict(pattern=19, smoother="ilu0", coarsen="semi_xy", gmres_restart=30, device=DEV)


def T(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def N(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _say(msg):
    print(f"[fullsize-weather] {msg}", flush=True)


@pytest.fixture(scope="module")
def full():
    _say("generating the 512x512x64 weather-like workload")
    A, b = workloads.weather19(SHAPE, seed=3)
    off = workloads.offsets(19)
    _say("GPU hierarchy (FP64)")
    mg = smg.StructMG(T(A), SHAPE, **KW)
    Am = helpers.masked_sgdia(A, off, SHAPE)
    _say("oracle ILU(0) factors")
    L, U, rU = oracle.ilu0(off, Am, SHAPE)
    return dict(A=A, b=b, off=off, mg=mg, Am=Am, L=L, U=U, rU=rU)


def test_weather_level0_data(full):
    mg, Am = full["mg"], full["Am"]
    _say("level-0 exports")
    assert np.array_equal(N(mg.export(0, 0, torch.empty(Am.shape, dtype=torch.float64, device=DEV))), Am)
    for what, ref in ((2, full["L"]), (3, full["U"]), (4, full["rU"])):
        got = N(mg.export(0, what, torch.empty(ref.shape, dtype=torch.float64, device=DEV)))
        assert np.array_equal(got, ref), f"ILU factor {what}"


def test_weather_level0_kernels(full):
    mg, Am, off, L, U, rU = (full[k] for k in ("mg", "Am", "off", "L", "U", "rU"))
    n = Am.shape[1]
    cdims = oracle.coarse_dims(SHAPE, CMASK)
    nc = int(np.prod(cdims))
    g = workloads.rng(51)
    f = g.uniform(-1, 1, size=SHAPE)
    u = g.uniform(-1, 1, size=SHAPE)
    ec = g.uniform(-1, 1, size=cdims)
    _say("level-0 SpMV")
    y = N(mg.op_spmv(0, T(f), torch.empty(n, dtype=torch.float64, device=DEV)))
    assert np.array_equal(y, oracle.spmv(off, Am, f).ravel())
    _say("level-0 ILU pre-smoothing")
    ug = N(mg.op_presmooth(0, T(f), torch.empty(n, dtype=torch.float64, device=DEV)))
    assert np.array_equal(ug, oracle.tri_solve(off, U, rU, oracle.tri_solve(off, L, None, f, 0), 1).ravel())
    _say("level-0 residual + restriction")
    rc = N(mg.op_resid_restrict(0, T(f), T(u), torch.empty(nc, dtype=torch.float64, device=DEV)))
    assert np.array_equal(rc, oracle.restrict(oracle.residual(off, Am, f, u), CMASK).ravel())
    _say("level-0 prolongation + ILU correction")
    uo = N(mg.op_postsmooth(0, T(f), T(u), T(ec), torch.empty(n, dtype=torch.float64, device=DEV)))
    uold = oracle.prolong_add(u, ec, CMASK)
    zc = oracle.tri_solve(off, U, rU, oracle.tri_solve(off, L, None, oracle.residual(off, Am, f, uold), 0), 1)
    assert np.array_equal(uo, (uold + zc).ravel())


def test_weather_level1_product_sampled(full):
    mg, Am, off = full["mg"], full["Am"], full["off"]
    cdims = oracle.coarse_dims(SHAPE, CMASK)
    nc = int(np.prod(cdims))
    pts = helpers.coarse_sample_points(cdims, 6000, 61)
    _say(f"level-1 stencil product at {pts.size} coarse points")
    A1 = N(mg.export(1, 0, torch.empty((27, nc), dtype=torch.float64, device=DEV)))
    assert np.array_equal(A1[:, pts], oracle.rap_points(off, Am, SHAPE, CMASK, pts))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_weather_gmres_true_residual(full, prec):
    Am, b, off = full["Am"], full["b"], full["off"]
    mg = full["mg"] if prec == "fp64" else smg.StructMG(T(full["A"]), SHAPE, prec=prec, **KW)
    if prec == "fp32":
        got = N(mg.export(0, 5, torch.empty(Am.shape, dtype=torch.float32, device=DEV)))
        assert np.array_equal(got, Am.astype(np.float32)), "FP32 copy of the finest matrix"
    _say(f"GMRES(30) to 1e-9, {prec} V-cycle")
    x = torch.zeros(Am.shape[1], dtype=torch.float64, device=DEV)
    res = mg.solve(T(b.ravel()), x, rtol=1e-9, maxit=500, krylov=30)
    assert res["status"] == 0
    r = oracle.residual(off, Am, b.reshape(SHAPE), N(x).reshape(SHAPE))
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)

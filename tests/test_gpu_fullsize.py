"""Parity at the benchmark's full size: diffusion 256^3 with the 7-point
stencil, PCG with a V-cycle using operator-dependent interpolation, the
hierarchy configured as the benchmark configures it.

The finest level is compared element by element with the oracle: the masked
matrix, its reciprocal diagonal, the interpolation weights, SpMV, the
pre-smoothing sweep, residual + restriction, prolongation and the
post-smoothing sweep.  The level-1 stencil product is compared at sampled
coarse points (the oracle computes those rows one by one), the whole V-cycle
through its symmetry, and the solve through the oracle's true residual.
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
SHAPE = (256, 256, 256)
CMASK = 7


def T(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def N(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _say(msg):
    print(f"[fullsize] {msg}", flush=True)


@pytest.fixture(scope="module")
def full():
    _say("generating the 256^3 diffusion workload")
    A, b = workloads.diffusion7(SHAPE, seed=2)
    off = workloads.offsets(7)
    _say("GPU hierarchy")
    mg = smg.StructMG(T(A), SHAPE, pattern=7, smoother="gs", coarsen="full", semi_levels=0, interp="operator",
                      device=DEV)
    Am = helpers.masked_sgdia(A, off, SHAPE)
    _say("oracle interpolation weights")
    W = oracle.od_weights(off, Am, SHAPE, CMASK)
    return dict(A=A, b=b, off=off, mg=mg, Am=Am, W=W)


def test_fullsize_level0_data(full):
    mg, Am, W = full["mg"], full["Am"], full["W"]
    n = Am.shape[1]
    _say("level-0 exports")
    assert np.array_equal(N(mg.export(0, 0, torch.empty(Am.shape, dtype=torch.float64, device=DEV))), Am)
    rd = N(mg.export(0, 1, torch.empty(n, dtype=torch.float64, device=DEV)))
    assert np.array_equal(rd, 1.0 / Am[3])
    assert np.array_equal(N(mg.export(0, 9, torch.empty(W.shape, dtype=torch.float64, device=DEV))), W)


def test_fullsize_level0_kernels(full):
    mg, Am, W, off = full["mg"], full["Am"], full["W"], full["off"]
    n = Am.shape[1]
    cdims = oracle.coarse_dims(SHAPE, CMASK)
    nc = int(np.prod(cdims))
    rd = 1.0 / Am[3]
    g = workloads.rng(41)
    f = g.uniform(-1, 1, size=SHAPE)
    u = g.uniform(-1, 1, size=SHAPE)
    ec = g.uniform(-1, 1, size=cdims)
    _say("level-0 SpMV")
    y = N(mg.op_spmv(0, T(f), torch.empty(n, dtype=torch.float64, device=DEV)))
    assert np.array_equal(y, oracle.spmv(off, Am, f).ravel())
    _say("level-0 forward GS from zero")
    ug = N(mg.op_presmooth(0, T(f), torch.empty(n, dtype=torch.float64, device=DEV)))
    assert np.array_equal(ug, oracle.gs_sweep(off, Am, rd, f, np.zeros(SHAPE), 1, 1).ravel())
    _say("level-0 residual + restriction")
    rc = N(mg.op_resid_restrict(0, T(f), T(u), torch.empty(nc, dtype=torch.float64, device=DEV)))
    assert np.array_equal(rc, oracle.restrict_od(oracle.residual(off, Am, f, u), W, CMASK).ravel())
    _say("level-0 prolongation")
    uf = T(u.copy())
    mg.op_prolong_add(0, T(ec), uf)
    up = oracle.prolong_add_od(u, W, ec, CMASK)
    assert np.array_equal(N(uf).ravel(), up.ravel())
    _say("level-0 prolongation + backward GS")
    uo = N(mg.op_postsmooth(0, T(f), T(u), T(ec), torch.empty(n, dtype=torch.float64, device=DEV)))
    assert np.array_equal(uo, oracle.gs_sweep(off, Am, rd, f, up, -1, 0).ravel())


def test_fullsize_level1_product_sampled(full):
    mg, Am, W, off = full["mg"], full["Am"], full["W"], full["off"]
    cdims = oracle.coarse_dims(SHAPE, CMASK)
    nc = int(np.prod(cdims))
    pts = helpers.coarse_sample_points(cdims, 6000, 43)
    _say(f"level-1 product at {pts.size} coarse points")
    A1 = N(mg.export(1, 0, torch.empty((27, nc), dtype=torch.float64, device=DEV)))
    assert np.array_equal(A1[:, pts], oracle.rap_od_points(off, Am, SHAPE, CMASK, W, pts))


def test_fullsize_vcycle_symmetric(full):
    """Symmetric GS smoothing, R = P^T and an exact coarsest solve make the
    V-cycle a symmetric positive definite operator at any size."""
    mg = full["mg"]
    n = int(np.prod(SHAPE))
    g = workloads.rng(47)
    r1 = g.uniform(-1, 1, size=n)
    r2 = g.uniform(-1, 1, size=n)
    _say("two V-cycles")
    z1 = N(mg.precondition(T(r1), torch.empty(n, dtype=torch.float64, device=DEV)))
    z2 = N(mg.precondition(T(r2), torch.empty(n, dtype=torch.float64, device=DEV)))
    scale = np.linalg.norm(r1) * np.linalg.norm(z2)
    assert abs(np.dot(r2, z1) - np.dot(r1, z2)) <= 1e-11 * scale
    assert np.dot(r1, z1) > 0 and np.dot(r2, z2) > 0


def test_fullsize_pcg_true_residual(full):
    mg, Am, b, off = full["mg"], full["Am"], full["b"], full["off"]
    n = int(np.prod(SHAPE))
    _say("PCG to 1e-9")
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    res = mg.solve(T(b.ravel()), x, rtol=1e-9, maxit=300)
    assert res["status"] == 0
    # device-resident PCG: the host reads the state once per batch of iterations
    assert res["host_waits"] <= res["iters"] // 2, res
    r = oracle.residual(off, Am, b.reshape(SHAPE), N(x).reshape(SHAPE))
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)

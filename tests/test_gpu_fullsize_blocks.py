"""Parity at full size for the elasticity-like block case: 128^3 nodes with
3 unknowns each, 27-point stencil of 3x3 blocks, PCG with a block
Gauss-Seidel V-cycle, configured as the benchmark configures it.

The finest level is compared element by element with the oracle: the masked
matrix, the inverse diagonal blocks, block SpMV, the forward block sweep from
zero, residual + restriction and prolongation + backward block sweep; the
level-1 block stencil product at sampled coarse points; the FP64 V-cycle
through its symmetry; the FP16 row-scaled V-cycle's solve (and the FP64 one)
through the oracle's true residual.
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
NN = 128
SHAPE = (NN, NN, NN)
CMASK = 7
OFF27 = workloads.offsets(27)


def T(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)


def N(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _say(msg):
    print(f"[fullsize-blocks] {msg}", flush=True)


@pytest.fixture(scope="module")
def full():
    _say("generating the 128^3 x 3 elasticity-like workload")
    A, b = workloads.elasticity27(NN, seed=4)
    _say("GPU hierarchy (FP64)")
    mg = smg.StructMG(T(A), SHAPE, pattern=27, block=3, device=DEV)
    Am = helpers.masked_sgdia(A, OFF27, SHAPE, be=9)
    _say("oracle inverse diagonal blocks")
    D = oracle.block_dinv(OFF27, Am, SHAPE)
    return dict(A=A, b=b, mg=mg, Am=Am, D=D)


def test_blocks_level0_data(full):
    mg, Am, D = full["mg"], full["Am"], full["D"]
    _say("level-0 exports")
    assert np.array_equal(N(mg.export(0, 0, torch.empty(Am.shape, dtype=torch.float64, device=DEV))), Am)
    assert np.array_equal(N(mg.export(0, 1, torch.empty(D.shape, dtype=torch.float64, device=DEV))), D)


def test_blocks_level0_kernels(full):
    mg, Am, D = full["mg"], full["Am"], full["D"]
    cdims = oracle.coarse_dims(SHAPE, CMASK)
    g = workloads.rng(53)
    f = g.uniform(-1, 1, size=SHAPE + (3,))
    u = g.uniform(-1, 1, size=SHAPE + (3,))
    ec = g.uniform(-1, 1, size=cdims + (3,))
    n3, nc3 = f.size, ec.size
    _say("level-0 block SpMV")
    y = N(mg.op_spmv(0, T(f.ravel()), torch.empty(n3, dtype=torch.float64, device=DEV)))
    assert np.array_equal(y, oracle.bspmv(OFF27, Am, f).ravel())
    _say("level-0 forward block GS from zero")
    ug = N(mg.op_presmooth(0, T(f.ravel()), torch.empty(n3, dtype=torch.float64, device=DEV)))
    assert np.array_equal(ug, oracle.bgs_sweep(OFF27, Am, D, f, np.zeros_like(f), 1, 1).ravel())
    _say("level-0 residual + restriction")
    rc = N(mg.op_resid_restrict(0, T(f.ravel()), T(u.ravel()), torch.empty(nc3, dtype=torch.float64, device=DEV)))
    assert np.array_equal(rc, oracle.restrict(f - oracle.bspmv(OFF27, Am, u), CMASK, bs=3).ravel())
    _say("level-0 prolongation + backward block GS")
    uo = N(mg.op_postsmooth(0, T(f.ravel()), T(u.ravel()), T(ec.ravel()),
                            torch.empty(n3, dtype=torch.float64, device=DEV)))
    ref = oracle.bgs_sweep(OFF27, Am, D, f, oracle.prolong_add(u, ec, CMASK, bs=3), -1, 0)
    assert np.array_equal(uo, ref.ravel())


def test_blocks_level1_product_sampled(full):
    mg, Am = full["mg"], full["Am"]
    cdims = oracle.coarse_dims(SHAPE, CMASK)
    nc = int(np.prod(cdims))
    pts = helpers.coarse_sample_points(cdims, 3000, 67)
    _say(f"level-1 block stencil product at {pts.size} coarse points")
    A1 = N(mg.export(1, 0, torch.empty((27 * 9, nc), dtype=torch.float64, device=DEV)))
    assert np.array_equal(A1[:, pts], oracle.rap_points(OFF27, Am, SHAPE, CMASK, pts, bs=3))


def test_blocks_vcycle_symmetric(full):
    """Forward block GS before and backward after the correction, R = P^T and
    an exact coarsest solve: a symmetric V-cycle for the symmetric matrix."""
    mg = full["mg"]
    n3 = int(np.prod(SHAPE)) * 3
    g = workloads.rng(57)
    r1 = g.uniform(-1, 1, size=n3)
    r2 = g.uniform(-1, 1, size=n3)
    _say("two V-cycles")
    z1 = N(mg.precondition(T(r1), torch.empty(n3, dtype=torch.float64, device=DEV)))
    z2 = N(mg.precondition(T(r2), torch.empty(n3, dtype=torch.float64, device=DEV)))
    assert abs(np.dot(r2, z1) - np.dot(r1, z2)) <= 1e-11 * np.linalg.norm(r1) * np.linalg.norm(z2)
    assert np.dot(r1, z1) > 0 and np.dot(r2, z2) > 0


@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_blocks_pcg_true_residual(full, prec):
    Am, b = full["Am"], full["b"]
    mg = full["mg"] if prec == "fp64" else smg.StructMG(T(full["A"]), SHAPE, pattern=27, block=3, prec=prec,
                                                        device=DEV)
    _say(f"PCG to 1e-8, {prec} V-cycle")
    x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    res = mg.solve(T(b.ravel()), x, rtol=1e-8, maxit=500)
    assert res["status"] == 0
    r = b - oracle.bspmv(OFF27, Am, N(x).reshape(b.shape))
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b)

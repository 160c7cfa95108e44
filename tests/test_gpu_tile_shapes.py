"""GPU tests of the selectable tile shape of the wavefront sweeps.

Every tile shape a level accepts (sheared, or rectangular 16 x 16 columns
where no two tiles would wait on each other) runs the exact sequential
lexicographic order of the Gauss-Seidel / ILU(0) sweeps (Sec. 4.4), so a
V-cycle must give the same bits whatever shape each level uses; the default
shapes are checked against the oracle by the parity tests.
"""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_21932_amd as smg  # noqa: E402

DEV = torch.device("cuda:0")

# (shape, pattern, smoother, precision): more than one tile row on the finest
# levels, so that the two shapes give different tilings there
CASES = [((48, 40, 20), 27, "gs", "fp64"), ((48, 40, 20), 19, "ilu0", "fp64"), ((40, 48, 24), 7, "gs", "fp32"),
         ((40, 36, 16), 27, "gs", "fp16"), ((33, 50, 17), 7, "ilu0", "fp32")]


def _ids(c):
    return f"{'x'.join(map(str, c[0]))}-{c[1]}-{c[2]}-{c[3]}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_vcycle_identical_for_every_tile_shape(case):
    shape, pat, smoother, prec = case
    A = workloads.random_sgdia(shape, pat, seed=21, symmetric=smoother == "gs")
    mg = smg.StructMG(torch.from_numpy(A).to(DEV), shape, pattern=pat, smoother=smoother, prec=prec, device=DEV)
    n = int(np.prod(shape))
    r = torch.from_numpy(workloads.rng(22).standard_normal(n)).to(DEV)
    z0 = torch.empty_like(r)
    mg.precondition(r, z0)
    torch.cuda.synchronize()
    ref = z0.cpu().numpy()
    changed = 0
    for l in range(mg.nlev - 1):
        d = mg.tile_shape(l)
        assert d in (1, 2)
        alt = 3 - d
        info = mg.level_info(l)
        if alt == 2 and info["S"] != 7 and info["dims"][1] > 16:
            # rectangles of a 19/27-point level with several tile rows
            with pytest.raises(smg.SmgError):
                mg.set_tile_shape(l, alt)
            assert mg.tile_shape(l) == d
            continue
        mg.set_tile_shape(l, alt)
        assert mg.tile_shape(l) == alt
        changed += 1
        z = torch.empty_like(r)
        mg.precondition(r, z)
        torch.cuda.synchronize()
        assert np.array_equal(z.cpu().numpy(), ref), f"level {l} shape {alt}"
    assert changed >= 1
    # a V-cycle twice in a row with the new shapes (sentinel state kept)
    z = torch.empty_like(r)
    mg.precondition(r, z)
    mg.precondition(r, z)
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy(), ref)
    for l in range(mg.nlev - 1):
        mg.set_tile_shape(l, 0)
    mg.precondition(r, z)
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy(), ref)
    with pytest.raises(smg.SmgError):
        mg.set_tile_shape(mg.nlev - 1, 1)
    with pytest.raises(smg.SmgError):
        mg.set_tile_shape(0, 3)
    mg.close()


def test_pcg_identical_for_every_tile_shape():
    shape = (48, 40, 24)
    A = workloads.random_sgdia(shape, 7, seed=23, symmetric=True)
    mg = smg.StructMG(torch.from_numpy(A).to(DEV), shape, pattern=7, device=DEV)
    n = int(np.prod(shape))
    b = torch.from_numpy(workloads.rng(24).standard_normal(n)).to(DEV)
    x0 = torch.zeros_like(b)
    r0 = mg.solve(b, x0, rtol=1e-9, maxit=100)
    # the 7-point finest level in sheared tiles; 27-point levels of one tile
    # row in rectangles
    mg.set_tile_shape(0, 1)
    for l in range(1, mg.nlev - 1):
        if mg.level_info(l)["dims"][1] <= 16:
            mg.set_tile_shape(l, 3 - mg.tile_shape(l))
    x1 = torch.zeros_like(b)
    r1 = mg.solve(b, x1, rtol=1e-9, maxit=100)
    torch.cuda.synchronize()
    assert r0["status"] == 0 and r1["iters"] == r0["iters"]
    assert np.array_equal(x0.cpu().numpy(), x1.cpu().numpy())
    mg.close()

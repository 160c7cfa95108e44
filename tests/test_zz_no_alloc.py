"""GPU check of smg_setup_noalloc (hierarchy in the library's static device
array) against smg_setup (hierarchy in a caller workspace), through the C
ABI: the level operators, one V-cycle and a PCG solve must agree bit for bit
on two calls in a row, the second on a smaller grid (which rebuilds in the
same array)."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2506_21932_amd as smg
import workloads

pytestmark = pytest.mark.gpu

CASES = [
    ("poisson 32^3, 7-point", (32, 32, 32), 7, 11),
    ("random 20x18x17, 27-point", (20, 18, 17), 27, 12),
]


def _noalloc_handle(L, cfg, coeffs):
    h = C.c_void_p()
    st = L.smg_setup_noalloc(C.byref(cfg), C.c_void_p(coeffs.data_ptr()), smg._stream(), C.byref(h))
    assert st == smg.SMG_OK, L.smg_last_error(None).decode()
    return h


def test_setup_noalloc_matches_setup_twice():
    L = smg.load()
    dev = torch.device("cuda:0")
    for name, shape, npts, seed in CASES:
        print(f"[no-alloc] {name}", flush=True)
        if npts == 7:
            A, b = workloads.poisson7(shape[0], seed=seed)
        else:
            A = workloads.random_sgdia(shape, npts, seed=seed)
            b = workloads.rng(seed).uniform(-1, 1, size=shape)
        coeffs = torch.from_numpy(np.ascontiguousarray(A)).to(dev)
        bt = torch.from_numpy(np.ascontiguousarray(b).ravel().copy()).to(dev)
        ref = smg.StructMG(coeffs, shape, pattern=npts, device=dev)
        cfg = smg.make_config(shape, pattern=npts)
        h = _noalloc_handle(L, cfg, coeffs)
        try:
            assert L.smg_num_levels(h) == ref.nlev
            # every level's operator
            for lev in range(ref.nlev):
                info = ref.level_info(lev)
                n = int(np.prod(info["dims"])) * info["S"]
                a1 = torch.empty(n, dtype=torch.float64, device=dev)
                a2 = torch.empty_like(a1)
                ref.export(lev, 0, a1)
                assert L.smg_level_export(h, lev, 0, C.c_void_p(a2.data_ptr()), smg._stream()) == smg.SMG_OK
                torch.cuda.synchronize()
                assert torch.equal(a1, a2), f"level {lev} operator differs"
            # one V-cycle
            z1 = torch.empty_like(bt)
            z2 = torch.full_like(bt, float("nan"))
            ref.precondition(bt, z1)
            assert L.smg_precondition(h, C.c_void_p(bt.data_ptr()), C.c_void_p(z2.data_ptr()),
                                      smg._stream()) == smg.SMG_OK
            torch.cuda.synchronize()
            assert torch.equal(z1, z2), "V-cycle differs"
            # PCG to 1e-9
            x1 = torch.zeros_like(bt)
            x2 = torch.zeros_like(bt)
            r1 = ref.solve(bt, x1, rtol=1e-9, maxit=200)
            res = smg.Result()
            st = L.smg_solve(h, C.c_void_p(bt.data_ptr()), C.c_void_p(x2.data_ptr()), 1e-9, 200, 0, C.byref(res),
                             smg._stream())
            torch.cuda.synchronize()
            assert st == smg.SMG_OK and r1["status"] == smg.SMG_OK
            assert res.iters == r1["iters"] and res.rel_resid_true < 1e-9
            assert torch.equal(x1, x2), "PCG solution differs"
        finally:
            L.smg_destroy(h)
            ref.close()

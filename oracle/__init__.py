"""CPU oracle for the structured multigrid V-cycle preconditioner.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_2506_21932_amd``) never imports it, and the two share no code.

The numerical work lives in ``oracle.c`` (plain sequential C, FP64 plus an
FP32 instantiation of the same loops); this module only marshals numpy arrays
through ctypes.  See ``oracle.c`` for the formulas and the paper passages each
function follows.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, f) for f in ("oracle.c", "oracle_kernels.inc", "oracle_vcycle.inc")]

CFLAGS = ["-O2", "-mfma", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99"]


def build(force=False):
    """Compile liboracle.so with gcc (no contraction, hardware fma)."""
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC[0], "-lm"], cwd=_HERE)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = C.CDLL(_SO)
        _declare(_lib)
    return _lib


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i = C.c_int


def _declare(L):
    for sfx, p in (("_f64", _dp), ("_f32", _fp)):
        getattr(L, "orc_spmv" + sfx).argtypes = [_i, _i, _i, _i, _ip, p, p, p]
        getattr(L, "orc_residual" + sfx).argtypes = [_i, _i, _i, _i, _ip, p, p, p, p]
        getattr(L, "orc_gs_sweep" + sfx).argtypes = [_i, _i, _i, _i, _ip, p, p, p, p, _i, _i]
        getattr(L, "orc_gs_sweep_w" + sfx).argtypes = [_i, _i, _i, _i, _ip, p, p, C.c_void_p, p, p, _i, _i]
        getattr(L, "orc_tri_solve" + sfx).argtypes = [_i, _i, _i, _i, _ip, p, C.c_void_p, p, p, _i]
        getattr(L, "orc_restrict" + sfx).argtypes = [_i, _i, _i, _i, _i, p, p]
        getattr(L, "orc_prolong_add" + sfx).argtypes = [_i, _i, _i, _i, _i, p, p]
        getattr(L, "orc_bspmv" + sfx).argtypes = [_i, _i, _i, _i, _ip, p, p, p]
        getattr(L, "orc_bresidual" + sfx).argtypes = [_i, _i, _i, _i, _ip, p, p, p, p]
        getattr(L, "orc_bgs_sweep" + sfx).argtypes = [_i, _i, _i, _i, _ip, p, p, p, p, _i, _i]
        getattr(L, "orc_lgs_sweep" + sfx).argtypes = [_i, _i, _i, _i, _ip, p, p, p, p, p, _i, _i, p]
        getattr(L, "orc_restrict_cc" + sfx).argtypes = [_i, _i, _i, _i, _i, p, p]
        getattr(L, "orc_prolong_add_cc" + sfx).argtypes = [_i, _i, _i, _i, _i, p, p]
        getattr(L, "orc_prolong_add_c64" + sfx).argtypes = [_i, _i, _i, _i, _i, p, p]
        getattr(L, "orc_restrict_od" + sfx).argtypes = [_i, _i, _i, _i, _i, p, p, p]
        getattr(L, "orc_prolong_add_od" + sfx).argtypes = [_i, _i, _i, _i, _i, p, p, p]
    L.orc_pattern.argtypes = [_i, _ip]
    L.orc_pattern.restype = _i
    L.orc_rap.argtypes = [_i, _i, _i, _i, _ip, _i, _dp, _i, _dp]
    L.orc_rap_points.argtypes = [_i, _i, _i, _i, _ip, _i, _dp, _i, _i, _lp, _dp]
    L.orc_rap_chains.argtypes = [_i, _ip, _i, _i, _ip, _i]
    L.orc_rap_chains.restype = _i
    L.orc_rap_cc.argtypes = [_i, _i, _i, _i, _ip, _i, _dp, _i, _dp]
    L.orc_rap_cc_chains.argtypes = [_i, _ip, _i]
    L.orc_rap_cc_chains.restype = _i
    L.orc_rap_c64.argtypes = [_i, _i, _i, _i, _ip, _i, _dp, _i, _dp]
    L.orc_rap_c64_chains.argtypes = [_i, _ip, _i]
    L.orc_rap_c64_chains.restype = _i
    L.orc_od_weights.argtypes = [_i, _i, _i, _i, _ip, _dp, _i, _dp]
    L.orc_od_weights.restype = _i
    L.orc_rap_od.argtypes = [_i, _i, _i, _i, _ip, _dp, _i, _dp, _dp]
    L.orc_rap_od_points.argtypes = [_i, _i, _i, _i, _ip, _dp, _i, _dp, _i, _lp, _dp]
    L.orc_ilu0.argtypes = [_i, _i, _i, _i, _ip, _dp, _dp, _dp, _dp]
    L.orc_ilu0.restype = _i
    L.orc_ilu0_mask.argtypes = [_i, _i, _i, _i, _ip, _dp, _i, _ip, _dp, _dp, _dp]
    L.orc_ilu0_mask.restype = _i
    L.orc_tri_factor.argtypes = [_i, _i, _i, _i, _ip, _dp, _dp, _dp]
    L.orc_tri_factor.restype = _i
    L.orc_lu_factor.argtypes = [_i, _dp, _ip]
    L.orc_lu_factor.restype = _i
    L.orc_lu_solve.argtypes = [_i, _dp, _ip, _dp]
    L.orc_dense_from_sgdia.argtypes = [_i, _i, _i, _i, _ip, _i, _dp, _dp]
    L.orc_block_dinv.argtypes = [_i, _i, _i, _i, _ip, _dp, _dp]
    L.orc_block_dinv.restype = _i
    L.orc_f32_to_f16.argtypes = [C.c_float]
    L.orc_f32_to_f16.restype = C.c_uint16
    L.orc_f16_to_f32.argtypes = [C.c_uint16]
    L.orc_f16_to_f32.restype = C.c_float
    L.orc_mg_create.argtypes = [_i, _i, _i, _i, _i, _dp, _i, _i, _i, _i, _i, _i, _i]
    L.orc_mg_create.restype = C.c_void_p
    L.orc_mg_create_ex.argtypes = [_i, _i, _i, _i, _i, _dp, _i, _i, _i, _i, _i, _i, _i, _i, _i, C.c_double, _i, _i]
    L.orc_mg_create_ex.restype = C.c_void_p
    L.orc_auto_semi_levels.argtypes = [_i, _i, _i, _i, _ip, _dp]
    L.orc_auto_semi_levels.restype = _i
    L.orc_mg_destroy.argtypes = [C.c_void_p]
    L.orc_mg_nlev.argtypes = [C.c_void_p]
    L.orc_mg_nlev.restype = _i
    L.orc_mg_level_info.argtypes = [C.c_void_p, _i, _ip]
    L.orc_mg_level_data.argtypes = [C.c_void_p, _i, _i, C.c_void_p]
    L.orc_mg_apply.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_mg_apply_f32.argtypes = [C.c_void_p, _fp, _fp]
    L.orc_pcg.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _i, _dp]
    L.orc_pcg.restype = _i
    L.orc_gmres.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _i, _i, _dp]
    L.orc_gmres.restype = _i


def _sfx(a):
    return "_f32" if a.dtype == np.float32 else "_f64"


def _c(a, dt=None):
    return np.ascontiguousarray(a, dtype=dt if dt is not None else a.dtype)


def pattern(npts):
    """Offsets (S,3) int32 of the 3d7 / 3d19 / 3d27 pattern in lexicographic order."""
    off = np.zeros(81, np.int32)
    S = lib().orc_pattern(npts, off)
    return off[: 3 * S].reshape(S, 3).copy()


def _dims(shape):
    return [int(v) for v in shape]


def spmv(off, A, x):
    off = _c(off, np.int32)
    nx, ny, nz = _dims(x.shape)
    y = np.empty_like(x)
    getattr(lib(), "orc_spmv" + _sfx(x))(nx, ny, nz, off.shape[0], off.ravel(), _c(A).ravel(), _c(x).ravel(), y.ravel())
    return y


def residual(off, A, b, x):
    off = _c(off, np.int32)
    nx, ny, nz = _dims(x.shape)
    r = np.empty_like(x)
    getattr(lib(), "orc_residual" + _sfx(x))(nx, ny, nz, off.shape[0], off.ravel(), _c(A).ravel(), _c(b).ravel(),
                                            _c(x).ravel(), r.ravel())
    return r


def gs_sweep(off, A, rd, b, u, direction, zero_guess):
    """In-place lexicographic GS sweep; returns u."""
    off = _c(off, np.int32)
    nx, ny, nz = _dims(b.shape)
    u = _c(u).copy()
    getattr(lib(), "orc_gs_sweep" + _sfx(b))(nx, ny, nz, off.shape[0], off.ravel(), _c(A).ravel(), _c(rd).ravel(),
                                            _c(b).ravel(), u.ravel(), int(direction), int(zero_guess))
    return u


def gs_sweep_w(off, A, rd, qa, b, u, direction, zero_guess):
    """Weighted GS sweep: rd = w / a_ii, qa = ((1 - w) / w) a_ii (None: w = 1); returns u."""
    off = _c(off, np.int32)
    nx, ny, nz = _dims(b.shape)
    u = _c(u).copy()
    qp = None if qa is None else _c(qa, b.dtype).ravel().ctypes.data_as(C.c_void_p)
    getattr(lib(), "orc_gs_sweep_w" + _sfx(b))(nx, ny, nz, off.shape[0], off.ravel(), _c(A).ravel(), _c(rd).ravel(),
                                              qp, _c(b).ravel(), u.ravel(), int(direction), int(zero_guess))
    return u


def auto_semi_levels(off, A, shape):
    """x,y-only levels of the automatic coarsening for the (S, N) matrix A."""
    off = _c(off, np.int32)
    return lib().orc_auto_semi_levels(*(int(v) for v in shape), off.shape[0], off.ravel(), _c(A, np.float64).ravel())


def lgs_sweep(off, A, rden, cp, b, u, direction, zero_guess):
    """In-place line GS sweep over z-columns; returns u."""
    off = _c(off, np.int32)
    nx, ny, nz = _dims(b.shape)
    u = _c(u).copy()
    d = np.zeros(nz, b.dtype)
    getattr(lib(), "orc_lgs_sweep" + _sfx(b))(nx, ny, nz, off.shape[0], off.ravel(), _c(A).ravel(),
                                             _c(rden).ravel(), _c(cp).ravel(), _c(b).ravel(), u.ravel(),
                                             int(direction), int(zero_guess), d)
    return u


def tri_factor(off, A, shape):
    """Thomas factors (rden, cp) of the z-column tridiagonal blocks of A."""
    off = _c(off, np.int32)
    N = int(np.prod(shape))
    rden = np.zeros(N)
    cp = np.zeros(N)
    if lib().orc_tri_factor(*_dims(shape), off.shape[0], off.ravel(), _c(A, np.float64).ravel(), rden, cp):
        raise ValueError("zero pivot")
    return rden, cp


def tri_solve(off, F, rU, r, upper):
    off = _c(off, np.int32)
    nx, ny, nz = _dims(r.shape)
    y = np.zeros_like(r)
    rp = None if rU is None else _c(rU).ravel().ctypes.data_as(C.c_void_p)
    keep = None if rU is None else _c(rU)
    if keep is not None:
        rp = keep.ctypes.data_as(C.c_void_p)
    getattr(lib(), "orc_tri_solve" + _sfx(r))(nx, ny, nz, off.shape[0], off.ravel(), _c(F).ravel(), rp,
                                             _c(r).ravel(), y.ravel(), int(upper))
    return y


def coarse_dims(shape, cmask, cell=False):
    return tuple(((n + 1) // 2 if cell else n // 2) if (cmask >> a) & 1 else n for a, n in enumerate(shape))


def restrict_cc(rf, cmask, bs=1):
    shp = rf.shape[:3]
    rc = np.zeros(coarse_dims(shp, cmask, True) + rf.shape[3:], rf.dtype)
    getattr(lib(), "orc_restrict_cc" + _sfx(rf))(*_dims(shp), int(cmask), int(bs), _c(rf).ravel(), rc.ravel())
    return rc


def prolong_add_cc(uf, ec, cmask, bs=1):
    shp = uf.shape[:3]
    out = _c(uf).copy()
    getattr(lib(), "orc_prolong_add_cc" + _sfx(uf))(*_dims(shp), int(cmask), int(bs), _c(ec).ravel(), out.ravel())
    return out


def rap_cc(off, Af, shape, cmask, bs=1):
    off = _c(off, np.int32)
    Nc = int(np.prod(coarse_dims(shape, cmask, True)))
    Ac = np.zeros((off.shape[0] * bs * bs, Nc))
    lib().orc_rap_cc(*_dims(shape), off.shape[0], off.ravel(), int(bs), _c(Af, np.float64).ravel(), int(cmask),
                     Ac.ravel())
    return Ac


def prolong_add_c64(uf, ec, cmask, bs=1):
    shp = uf.shape[:3]
    out = _c(uf).copy()
    getattr(lib(), "orc_prolong_add_c64" + _sfx(uf))(*_dims(shp), int(cmask), int(bs), _c(ec).ravel(), out.ravel())
    return out


def rap_c64(off, Af, shape, cmask, bs=1):
    off = _c(off, np.int32)
    Nc = int(np.prod(coarse_dims(shape, cmask, True)))
    Ac = np.zeros((27 * bs * bs, Nc))
    lib().orc_rap_c64(*_dims(shape), off.shape[0], off.ravel(), int(bs), _c(Af, np.float64).ravel(), int(cmask),
                      Ac.ravel())
    return Ac


def rap_c64_chains(off, cmask):
    off = _c(off, np.int32)
    return lib().orc_rap_c64_chains(off.shape[0], off.ravel(), int(cmask))


def od_weights(off, A, shape, cmask):
    """Operator-dependent interpolation weights W (8, N) of a vertex level."""
    off = _c(off, np.int32)
    W = np.zeros((8, int(np.prod(shape))))
    if lib().orc_od_weights(*_dims(shape), off.shape[0], off.ravel(), _c(A, np.float64).ravel(), int(cmask),
                            W.ravel()):
        raise ValueError("zero collapsed diagonal")
    return W


def restrict_od(rf, W, cmask):
    shp = rf.shape[:3]
    rc = np.zeros(coarse_dims(shp, cmask), rf.dtype)
    getattr(lib(), "orc_restrict_od" + _sfx(rf))(*_dims(shp), int(cmask), 1, _c(W, rf.dtype).ravel(),
                                                _c(rf).ravel(), rc.ravel())
    return rc


def prolong_add_od(uf, W, ec, cmask):
    shp = uf.shape[:3]
    out = _c(uf).copy()
    getattr(lib(), "orc_prolong_add_od" + _sfx(uf))(*_dims(shp), int(cmask), 1, _c(W, uf.dtype).ravel(),
                                                   _c(ec).ravel(), out.ravel())
    return out


def rap_od(off, Af, shape, cmask, W):
    off = _c(off, np.int32)
    Ac = np.zeros((27, int(np.prod(coarse_dims(shape, cmask)))))
    lib().orc_rap_od(*_dims(shape), off.shape[0], off.ravel(), _c(Af, np.float64).ravel(), int(cmask),
                     _c(W, np.float64).ravel(), Ac.ravel())
    return Ac


def rap_od_points(off, Af, shape, cmask, W, pts):
    """Rows (27, len(pts)) of rap_od at the flat coarse indices pts."""
    off = _c(off, np.int32)
    pts = _c(np.asarray(pts), np.int64)
    Ac = np.zeros((27, pts.size))
    lib().orc_rap_od_points(*_dims(shape), off.shape[0], off.ravel(), _c(Af, np.float64).ravel(), int(cmask),
                            _c(W, np.float64).ravel(), int(pts.size), pts.ravel(), Ac.ravel())
    return Ac


def rap_cc_chains(off, cmask):
    off = _c(off, np.int32)
    return lib().orc_rap_cc_chains(off.shape[0], off.ravel(), int(cmask))


def restrict(rf, cmask, bs=1):
    shp = rf.shape[:3]
    cs = coarse_dims(shp, cmask)
    rc = np.zeros(cs + rf.shape[3:], rf.dtype)
    getattr(lib(), "orc_restrict" + _sfx(rf))(*_dims(shp), int(cmask), int(bs), _c(rf).ravel(), rc.ravel())
    return rc


def prolong_add(uf, ec, cmask, bs=1):
    shp = uf.shape[:3]
    out = _c(uf).copy()
    getattr(lib(), "orc_prolong_add" + _sfx(uf))(*_dims(shp), int(cmask), int(bs), _c(ec).ravel(), out.ravel())
    return out


def bspmv(off, A, x):
    off = _c(off, np.int32)
    nx, ny, nz = _dims(x.shape[:3])
    y = np.empty_like(x)
    getattr(lib(), "orc_bspmv" + _sfx(x))(nx, ny, nz, off.shape[0], off.ravel(), _c(A).ravel(), _c(x).ravel(), y.ravel())
    return y


def bgs_sweep(off, A, Dinv, b, u, direction, zero_guess):
    off = _c(off, np.int32)
    nx, ny, nz = _dims(b.shape[:3])
    u = _c(u).copy()
    getattr(lib(), "orc_bgs_sweep" + _sfx(b))(nx, ny, nz, off.shape[0], off.ravel(), _c(A).ravel(),
                                             _c(Dinv).ravel(), _c(b).ravel(), u.ravel(), int(direction),
                                             int(zero_guess))
    return u


def block_dinv(off, A, shape):
    off = _c(off, np.int32)
    N = int(np.prod(shape))
    D = np.zeros((9, N))
    if lib().orc_block_dinv(*_dims(shape), off.shape[0], off.ravel(), _c(A, np.float64).ravel(), D.ravel()):
        raise ValueError("singular diagonal block")
    return D


def rap(off, Af, shape, cmask, bs=1):
    off = _c(off, np.int32)
    cs = coarse_dims(shape, cmask)
    Nc = int(np.prod(cs))
    Ac = np.zeros((27 * bs * bs, Nc))
    lib().orc_rap(*_dims(shape), off.shape[0], off.ravel(), int(bs), _c(Af, np.float64).ravel(), int(cmask),
                  Ac.ravel())
    return Ac


def rap_points(off, Af, shape, cmask, pts, bs=1):
    """Rows (27 * bs^2, len(pts)) of rap at the flat coarse indices pts."""
    off = _c(off, np.int32)
    pts = _c(np.asarray(pts), np.int64)
    Ac = np.zeros((27 * bs * bs, pts.size))
    lib().orc_rap_points(*_dims(shape), off.shape[0], off.ravel(), int(bs), _c(Af, np.float64).ravel(), int(cmask),
                         int(pts.size), pts.ravel(), Ac.ravel())
    return Ac


def rap_chains(off, cmask, n_index):
    off = _c(off, np.int32)
    out = np.zeros(3 * 4096, np.int32)
    cnt = lib().orc_rap_chains(off.shape[0], off.ravel(), int(cmask), int(n_index), out, 4096)
    return out[: 3 * cnt].reshape(cnt, 3).copy()


def ilu0(off, A, shape):
    off = _c(off, np.int32)
    S = off.shape[0]
    N = int(np.prod(shape))
    L = np.zeros((S, N))
    U = np.zeros((S, N))
    rU = np.zeros(N)
    if lib().orc_ilu0(*_dims(shape), S, off.ravel(), _c(A, np.float64).ravel(), L.ravel(), U.ravel(), rU):
        raise ValueError("zero pivot")
    return L, U, rU


def ilu0_mask(off, A, offm, shape):
    """ILU(0) of A (pattern off) on the mask offm: factors on offm's slots."""
    off = _c(off, np.int32)
    offm = _c(offm, np.int32)
    Sm = offm.shape[0]
    N = int(np.prod(shape))
    L = np.zeros((Sm, N))
    U = np.zeros((Sm, N))
    rU = np.zeros(N)
    if lib().orc_ilu0_mask(*_dims(shape), off.shape[0], off.ravel(), _c(A, np.float64).ravel(), Sm, offm.ravel(),
                           L.ravel(), U.ravel(), rU):
        raise ValueError("zero pivot")
    return L, U, rU


def dense(off, A, shape, bs=1):
    off = _c(off, np.int32)
    n = int(np.prod(shape)) * bs
    M = np.zeros((n, n))
    lib().orc_dense_from_sgdia(*_dims(shape), off.shape[0], off.ravel(), int(bs), _c(A, np.float64).ravel(), M.ravel())
    return M


def lu_solve(M, b):
    M = _c(M, np.float64).copy()
    n = M.shape[0]
    piv = np.zeros(n, np.int32)
    if lib().orc_lu_factor(n, M.ravel(), piv):
        raise ValueError("singular")
    x = _c(b, np.float64).copy()
    lib().orc_lu_solve(n, M.ravel(), piv, x)
    return x


def f32_to_f16_bits(v):
    return lib().orc_f32_to_f16(float(v))


def f16_bits_to_f32(h):
    return lib().orc_f16_to_f32(int(h))


PREC = {"fp64": 0, "fp32": 1, "fp16": 2}
SMOOTHER = {"gs": 0, "ilu0": 1, "lgs": 2}
INTERP = {"vertex": 0, "cell": 1, "cell_trilinear": 2, "operator": 3}


class Hierarchy:
    """Oracle multigrid hierarchy built from the finest matrix (FP64 setup)."""

    def __init__(self, shape, pattern_pts, A0, block=1, smoother="gs", coarsen="full", semi_levels=0,
                 prec="fp64", max_coarse=8192, ilu_mask=0, interp="vertex", pre_sweeps=1, post_sweeps=1,
                 relax_weight=1.0, zero_guess=True, min_coarse=4):
        self.shape = tuple(int(v) for v in shape)
        self.bs = int(block)
        self._A0 = _c(A0, np.float64)
        mode = {"full": 0, "semi_xy": 1, "auto": 2}[coarsen]
        h = lib().orc_mg_create_ex(*self.shape, int(pattern_pts), self.bs, self._A0.ravel(),
                                   SMOOTHER[smoother], mode, int(semi_levels), PREC[prec], int(max_coarse),
                                   int(ilu_mask), INTERP[interp], int(pre_sweeps), int(post_sweeps),
                                   float(relax_weight), int(bool(zero_guess)), int(min_coarse))
        if not h:
            raise ValueError("oracle hierarchy setup failed")
        self.h = C.c_void_p(h)
        self.prec = prec

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.orc_mg_destroy(h)
            self.h = None

    @property
    def nlev(self):
        return lib().orc_mg_nlev(self.h)

    def level_info(self, l):
        info = np.zeros(6, np.int32)
        lib().orc_mg_level_info(self.h, l, info)
        return {"dims": tuple(int(v) for v in info[:3]), "S": int(info[3]), "cmask": int(info[4]),
                "Sm": int(info[5])}

    def level_data(self, l, what):
        inf = self.level_info(l)
        N = int(np.prod(inf["dims"]))
        be = self.bs * self.bs
        S = inf["S"]
        Sm = inf["Sm"] or S
        sizes = {0: (S * be, N), 1: ((9 if self.bs == 3 else 1), N), 2: (Sm, N), 3: (Sm, N), 4: (1, N),
                 5: (S * be, N), 6: ((9 if self.bs == 3 else 1), N), 7: (1, N), 8: (1, N), 9: (8, N)}
        dt = np.float32 if what in (5, 6) else np.float64
        out = np.zeros(sizes[what], dt)
        lib().orc_mg_level_data(self.h, l, what, out.ctypes.data_as(C.c_void_p))
        return out

    def apply(self, r):
        r = _c(r, np.float64)
        z = np.zeros_like(r)
        lib().orc_mg_apply(self.h, r.ravel(), z.ravel())
        return z

    def apply_f32(self, r):
        r = _c(r, np.float32)
        z = np.zeros_like(r)
        lib().orc_mg_apply_f32(self.h, r.ravel(), z.ravel())
        return z

    def pcg(self, b, tol, maxit, x0=None):
        b = _c(b, np.float64)
        x = np.zeros_like(b) if x0 is None else _c(x0, np.float64).copy()
        out = np.zeros(2)
        st = lib().orc_pcg(self.h, b.ravel(), x.ravel(), float(tol), int(maxit), out)
        return x, st, int(out[0]), float(out[1])

    def gmres(self, b, tol, maxit, restart=30, x0=None):
        b = _c(b, np.float64)
        x = np.zeros_like(b) if x0 is None else _c(x0, np.float64).copy()
        out = np.zeros(2)
        st = lib().orc_gmres(self.h, b.ravel(), x.ravel(), float(tol), int(maxit), int(restart), out)
        return x, st, int(out[0]), float(out[1])

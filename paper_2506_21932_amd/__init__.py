"""Python binding of libstructmg (structured multigrid preconditioner, gfx950).

Argument marshalling only: every numerical step runs in the HIP kernels of
``libstructmg.so`` behind the C ABI of ``include/structmg.h``.  PyTorch tensors
provide device memory and the current HIP stream.  There is no fallback: if
the library is missing or cannot be loaded, importing the binding's entry
points raises.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstructmg.so")

SMG_OK, SMG_ENOTCONV, SMG_EINVAL, SMG_ENOMEM, SMG_EDEVICE, SMG_EBREAKDOWN, SMG_EDEADLOCK = 0, 1, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "SMG_OK", 1: "SMG_ENOTCONV", -1: "SMG_EINVAL", -2: "SMG_ENOMEM", -3: "SMG_EDEVICE",
                -4: "SMG_EBREAKDOWN", -5: "SMG_EDEADLOCK"}
PREC = {"fp64": 0, "fp32": 1, "fp16": 2}
SMOOTHER = {"gs": 0, "ilu0": 1, "lgs": 2}
INTERP = {"vertex": 0, "cell": 1, "cell_trilinear": 2, "operator": 3}
COARSEN = {"full": 0, "semi_xy": 1, "auto": 2}


class SmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("block", C.c_int), ("pattern", C.c_int),
                ("smoother", C.c_int), ("coarsen", C.c_int), ("semi_levels", C.c_int), ("prec", C.c_int),
                ("max_coarse", C.c_int), ("gmres_restart", C.c_int), ("ilu_mask", C.c_int), ("interp", C.c_int),
                ("pre_sweeps", C.c_int), ("post_sweeps", C.c_int), ("relax_weight", C.c_double),
                ("zero_guess", C.c_int), ("min_coarse", C.c_int)]


class Result(C.Structure):
    _fields_ = [("iters", C.c_int), ("levels", C.c_int), ("rel_resid_true", C.c_double),
                ("rel_resid_recur", C.c_double), ("grid_complexity", C.c_double), ("op_complexity", C.c_double), ("t_setup_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("host_waits", C.c_int)]


EXPORTS = ["smg_workspace_size", "smg_setup", "smg_precondition", "smg_solve", "smg_destroy", "smg_last_error",
           "smg_level_info", "smg_num_levels", "smg_level_export", "smg_rap_chain_count", "smg_op_spmv",
           "smg_op_spmv_fp64", "smg_op_presmooth", "smg_op_postsmooth", "smg_op_resid_restrict", "smg_op_restrict",
           "smg_op_prolong_add", "smg_op_coarse_solve", "smg_set_timing", "smg_timing_report", "smg_resetup",
           "smg_batch_workspace_size", "smg_batch_setup", "smg_batch_precondition", "smg_batch_solve",
           "smg_batch_set_schedule", "smg_batch_tune", "smg_batch_set_graph", "smg_batch_num_systems",
           "smg_batch_system", "smg_batch_destroy", "smg_batch_last_error", "smg_set_graph", "smg_setup_noalloc",
           "smg_set_tile_shape", "smg_tile_shape", "smg_batch_set_tile_shape", "smg_batch_tile_shape"]

TIMING_KINDS = ["pre_sweep", "pre_sweep_u", "resid_restrict", "coarse_solve", "prolong_post", "post_sweep",
                "post_sweep_u", "spmv_fp64"]

_lib = None


def load():
    """Loads libstructmg.so (built by __graft_entry__.build / build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2506_21932_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    L.smg_workspace_size.argtypes = [C.POINTER(Config), C.POINTER(C.c_size_t)]
    L.smg_setup.argtypes = [C.POINTER(Config), vp, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.smg_setup_noalloc.argtypes = [C.POINTER(Config), vp, vp, C.POINTER(vp)]
    L.smg_precondition.argtypes = [vp, vp, vp, vp]
    L.smg_solve.argtypes = [vp, vp, vp, d, i, i, C.POINTER(Result), vp]
    L.smg_destroy.argtypes = [vp]
    L.smg_last_error.argtypes = [vp]
    L.smg_last_error.restype = C.c_char_p
    L.smg_level_info.argtypes = [vp, i, C.POINTER(C.c_int)]
    L.smg_num_levels.argtypes = [vp]
    L.smg_num_levels.restype = i
    L.smg_level_export.argtypes = [vp, i, i, vp, vp]
    L.smg_rap_chain_count.argtypes = [i, i]
    L.smg_rap_chain_count.restype = i
    L.smg_op_spmv.argtypes = [vp, i, vp, vp, vp]
    L.smg_op_spmv_fp64.argtypes = [vp, vp, vp, vp]
    L.smg_op_presmooth.argtypes = [vp, i, vp, vp, vp]
    L.smg_op_postsmooth.argtypes = [vp, i, vp, vp, vp, vp, vp]
    L.smg_op_resid_restrict.argtypes = [vp, i, vp, vp, vp, vp]
    L.smg_op_restrict.argtypes = [vp, i, vp, vp, vp]
    L.smg_op_prolong_add.argtypes = [vp, i, vp, vp, vp]
    L.smg_op_coarse_solve.argtypes = [vp, vp, vp, vp]
    L.smg_set_timing.argtypes = [vp, i, i, C.c_uint]
    L.smg_resetup.argtypes = [vp, vp, vp]
    L.smg_timing_report.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int), i, C.POINTER(C.c_int)]
    L.smg_set_graph.argtypes = [vp, i]
    L.smg_set_tile_shape.argtypes = [vp, i, i, vp]
    L.smg_tile_shape.argtypes = [vp, i]
    L.smg_batch_set_tile_shape.argtypes = [vp, i, i, vp]
    L.smg_batch_tile_shape.argtypes = [vp, i]
    L.smg_batch_workspace_size.argtypes = [i, C.POINTER(Config), C.POINTER(C.c_size_t)]
    L.smg_batch_setup.argtypes = [i, C.POINTER(Config), C.POINTER(vp), vp, C.c_size_t, vp, C.POINTER(vp)]
    L.smg_batch_precondition.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), vp]
    L.smg_batch_solve.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), d, i, C.POINTER(Result), C.POINTER(C.c_int), vp]
    L.smg_batch_set_schedule.argtypes = [vp, i, i]
    L.smg_batch_tune.argtypes = [vp, vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.smg_batch_set_graph.argtypes = [vp, i]
    L.smg_batch_num_systems.argtypes = [vp]
    L.smg_batch_system.argtypes = [vp, i]
    L.smg_batch_system.restype = vp
    L.smg_batch_destroy.argtypes = [vp]
    L.smg_batch_last_error.argtypes = [vp]
    L.smg_batch_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("smg_last_error", "smg_num_levels", "smg_rap_chain_count", "smg_batch_system",
                        "smg_batch_last_error"):
            getattr(L, name).restype = i
    _lib = L
    return L


def rap_chain_count(pattern, cmask):
    return load().smg_rap_chain_count(int(pattern), int(cmask))


def make_config(shape, pattern=7, block=1, smoother="gs", coarsen="full", semi_levels=0, prec="fp64",
                max_coarse=0, gmres_restart=0, ilu_mask=0, interp="vertex", pre_sweeps=0, post_sweeps=0,
                relax_weight=0.0, zero_guess=0, min_coarse=0):
    """smg_config; zero smoothing fields select the defaults (one step before and
    after the coarse correction, weight 1, ZeroGuess, min_coarse 4)."""
    nx, ny, nz = (int(v) for v in shape)
    return Config(nx, ny, nz, int(block), int(pattern), SMOOTHER[smoother], COARSEN[coarsen], int(semi_levels),
                  PREC[prec], int(max_coarse), int(gmres_restart), int(ilu_mask), INTERP[interp], int(pre_sweeps),
                  int(post_sweeps), float(relax_weight), int(zero_guess), int(min_coarse))


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class StructMG:
    """Owns a libstructmg handle and its workspace (a torch uint8 tensor)."""

    def __init__(self, coeffs, shape, pattern=7, block=1, smoother="gs", coarsen="full", semi_levels=0, prec="fp64",
                 max_coarse=0, gmres_restart=0, device="cuda", workspace=None, ilu_mask=0, interp="vertex",
                 pre_sweeps=0, post_sweeps=0, relax_weight=0.0, zero_guess=0, min_coarse=0):
        import torch
        L = load()
        self.L = L
        self.cfg = make_config(shape, pattern, block, smoother, coarsen, semi_levels, prec, max_coarse, gmres_restart,
                               ilu_mask, interp, pre_sweeps, post_sweeps, relax_weight, zero_guess, min_coarse)
        self.block = int(block)
        self.prec = prec
        nbytes = C.c_size_t(0)
        self._check(L.smg_workspace_size(C.byref(self.cfg), C.byref(nbytes)), None)
        if workspace is not None and workspace.numel() >= nbytes.value:
            self.workspace = workspace
        else:
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
        coeffs = coeffs.to(device=device, dtype=torch.float64).contiguous()
        h = C.c_void_p()
        self._check(L.smg_setup(C.byref(self.cfg), _ptr(coeffs), _ptr(self.workspace), nbytes, _stream(),
                                C.byref(h)), None)
        self.h = h
        self.shape = tuple(int(v) for v in shape)

    def _check(self, st, h):
        if st not in (SMG_OK,):
            msg = self.L.smg_last_error(h).decode()
            raise SmgError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            self.L.smg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nlev(self):
        return self.L.smg_num_levels(self.h)

    def level_info(self, l):
        info = (C.c_int * 6)()
        self._check(self.L.smg_level_info(self.h, int(l), info), self.h)
        return {"dims": (info[0], info[1], info[2]), "S": info[3], "cmask": info[4], "block": info[5]}

    def export(self, l, what, out):
        self._check(self.L.smg_level_export(self.h, int(l), int(what), _ptr(out), _stream()), self.h)
        return out

    def precondition(self, r, z):
        self._check(self.L.smg_precondition(self.h, _ptr(r), _ptr(z), _stream()), self.h)
        return z

    def solve(self, b, x, rtol=1e-9, maxit=500, krylov=0):
        res = Result()
        st = self.L.smg_solve(self.h, _ptr(b), _ptr(x), float(rtol), int(maxit), int(krylov), C.byref(res), _stream())
        if st not in (SMG_OK, SMG_ENOTCONV):
            self._check(st, self.h)
        return {"status": st, "iters": res.iters, "levels": res.levels, "rel_resid_true": res.rel_resid_true,
                "rel_resid_recur": res.rel_resid_recur,
                "grid_complexity": res.grid_complexity, "op_complexity": res.op_complexity,
                "t_setup_ms": res.t_setup_ms, "t_solve_ms": res.t_solve_ms, "host_waits": res.host_waits}

    # single V-cycle steps (same kernels as the cycle)
    def op_spmv(self, l, x, y):
        self._check(self.L.smg_op_spmv(self.h, int(l), _ptr(x), _ptr(y), _stream()), self.h)
        return y

    def op_spmv_fp64(self, x, y):
        self._check(self.L.smg_op_spmv_fp64(self.h, _ptr(x), _ptr(y), _stream()), self.h)
        return y

    def op_presmooth(self, l, f, u):
        self._check(self.L.smg_op_presmooth(self.h, int(l), _ptr(f), _ptr(u), _stream()), self.h)
        return u

    def op_postsmooth(self, l, f, u_in, ec, u_out):
        self._check(self.L.smg_op_postsmooth(self.h, int(l), _ptr(f), _ptr(u_in), _ptr(ec), _ptr(u_out),
                                             _stream()), self.h)
        return u_out

    def op_resid_restrict(self, l, f, u, rc):
        self._check(self.L.smg_op_resid_restrict(self.h, int(l), _ptr(f), _ptr(u), _ptr(rc), _stream()), self.h)
        return rc

    def op_restrict(self, l, rf, rc):
        self._check(self.L.smg_op_restrict(self.h, int(l), _ptr(rf), _ptr(rc), _stream()), self.h)
        return rc

    def op_prolong_add(self, l, ec, uf):
        self._check(self.L.smg_op_prolong_add(self.h, int(l), _ptr(ec), _ptr(uf), _stream()), self.h)
        return uf

    def set_timing(self, enable, level=-1, kinds=None):
        mask = 0xFF if kinds is None else sum(1 << TIMING_KINDS.index(k) for k in kinds)
        self._check(self.L.smg_set_timing(self.h, int(bool(enable)), int(level), mask), self.h)

    def resetup(self, coeffs):
        self._check(self.L.smg_resetup(self.h, _ptr(coeffs), _stream()), self.h)

    def timing_report(self, max_levels=40):
        """{(level, kind): (ms, launches)} of the launches recorded since the last report."""
        n = max_levels * len(TIMING_KINDS)
        ms = (C.c_double * n)()
        cnt = (C.c_int * n)()
        dropped = C.c_int(0)
        self._check(self.L.smg_timing_report(self.h, ms, cnt, int(max_levels), C.byref(dropped)), self.h)
        out = {}
        for k in range(n):
            if cnt[k]:
                out[(k // len(TIMING_KINDS), TIMING_KINDS[k % len(TIMING_KINDS)])] = (ms[k], cnt[k])
        return out, bool(dropped.value)

    @staticmethod
    def workspace_bytes(shape, **kw):
        cfg = make_config(shape, **kw)
        n = C.c_size_t(0)
        st = load().smg_workspace_size(C.byref(cfg), C.byref(n))
        if st != SMG_OK:
            raise SmgError(st, load().smg_last_error(None).decode())
        return int(n.value)

    def set_graph(self, enable):
        self._check(self.L.smg_set_graph(self.h, int(bool(enable))), self.h)

    def set_tile_shape(self, l, shape):
        """Tile shape of level l's sweeps: 0 default, 1 sheared, 2 rectangular."""
        self._check(self.L.smg_set_tile_shape(self.h, int(l), int(shape), _stream()), self.h)

    def tile_shape(self, l):
        return self.L.smg_tile_shape(self.h, int(l))

    def op_coarse_solve(self, f, u):
        self._check(self.L.smg_op_coarse_solve(self.h, _ptr(f), _ptr(u), _stream()), self.h)
        return u


def _ptr_array(ts):
    return (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


class StructMGBatch:
    """Owns a batch of independent scalar systems solved in lockstep (one
    workspace tensor holds every hierarchy and the batch's tables)."""

    def __init__(self, coeffs, shapes, pattern=7, smoother="gs", coarsen="full", semi_levels=0, prec="fp64",
                 max_coarse=0, device="cuda"):
        import torch
        L = load()
        self.L = L
        self.n = len(shapes)
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.cfgs = (Config * self.n)(*[make_config(s, pattern, 1, smoother, coarsen, semi_levels, prec, max_coarse,
                                                    0) for s in self.shapes])
        nbytes = C.c_size_t(0)
        self._check(L.smg_batch_workspace_size(self.n, self.cfgs, C.byref(nbytes)), None)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
        cs = [c.to(device=device, dtype=torch.float64).contiguous() for c in coeffs]
        b = C.c_void_p()
        self._check(L.smg_batch_setup(self.n, self.cfgs, _ptr_array(cs), _ptr(self.workspace), nbytes, _stream(),
                                      C.byref(b)), None)
        self.b = b

    def _check(self, st, b):
        if st != SMG_OK:
            raise SmgError(st, self.L.smg_batch_last_error(b).decode())

    def close(self):
        if getattr(self, "b", None):
            self.L.smg_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def levels(self, k):
        return self.L.smg_num_levels(self.L.smg_batch_system(self.b, int(k)))

    def precondition(self, rs, zs):
        self._check(self.L.smg_batch_precondition(self.b, _ptr_array(rs), _ptr_array(zs), _stream()), self.b)
        return zs

    def solve(self, bs, xs, rtol=1e-9, maxit=500):
        res = (Result * self.n)()
        stt = (C.c_int * self.n)()
        st = self.L.smg_batch_solve(self.b, _ptr_array(bs), _ptr_array(xs), float(rtol), int(maxit), res, stt,
                                    _stream())
        if st not in (SMG_OK, SMG_ENOTCONV, SMG_EBREAKDOWN):
            self._check(st, self.b)
        return st, [{"status": stt[k], "iters": res[k].iters, "levels": res[k].levels,
                     "rel_resid_true": res[k].rel_resid_true, "rel_resid_recur": res[k].rel_resid_recur,
                     "t_setup_ms": res[k].t_setup_ms,
                     "t_solve_ms": res[k].t_solve_ms} for k in range(self.n)]

    def set_schedule(self, order, grid=0):
        self._check(self.L.smg_batch_set_schedule(self.b, int(order), int(grid)), self.b)

    def set_graph(self, enable):
        self._check(self.L.smg_batch_set_graph(self.b, int(bool(enable))), self.b)

    def tune(self):
        o, g, ms = C.c_int(0), C.c_int(0), C.c_double(0)
        self._check(self.L.smg_batch_tune(self.b, _stream(), C.byref(o), C.byref(g), C.byref(ms)), self.b)
        nl = max(self.levels(k) for k in range(self.n))
        return {"order": o.value, "grid": g.value, "ms_per_vcycle": ms.value,
                "tile_shapes": [self.tile_shape(l) for l in range(nl - 1)]}

    def set_tile_shape(self, l, shape):
        self._check(self.L.smg_batch_set_tile_shape(self.b, int(l), int(shape), _stream()), self.b)

    def tile_shape(self, l):
        return self.L.smg_batch_tile_shape(self.b, int(l))

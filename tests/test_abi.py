"""Host-side checks of the C ABI (no GPU needed): the shared library loads,
exports every entry point declared in include/structmg.h, validates
configurations, and its generated triple-product kernels cover the chain
counts printed in the paper."""
import ctypes as C
import os
import re

import pytest

import paper_2506_21932_amd as smg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "structmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(smg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = smg.load()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(smg.EXPORTS)


def test_chain_counts_of_generated_kernels():
    # Table of chain counts (vertex-centred restriction / interpolation)
    assert smg.rap_chain_count(19, 7) == 1685
    assert smg.rap_chain_count(27, 7) == 2197
    # per-axis closed forms: centre 5^3 plus faces 4*5*5 (3d7), one z-factor under x,y coarsening
    assert smg.rap_chain_count(7, 7) == 725
    assert smg.rap_chain_count(7, 3) == 155
    assert smg.rap_chain_count(27, 3) == 13 * 13 * 3
    assert smg.rap_chain_count(27, 1) == 13 * 9


def _ws(**kw):
    cfg = smg.make_config(**kw)
    n = C.c_size_t(0)
    st = smg.load().smg_workspace_size(C.byref(cfg), C.byref(n))
    return st, n.value


def test_workspace_size_and_validation():
    st, n = _ws(shape=(32, 32, 32), pattern=7)
    assert st == smg.SMG_OK and n > 7 * 32 ** 3 * 8
    st2, n2 = _ws(shape=(32, 32, 32), pattern=7, prec="fp32")
    # the FP32 V-cycle keeps the FP64 finest matrix (for the Galerkin products) plus its FP32 copy
    assert st2 == smg.SMG_OK and n2 > 7 * 32 ** 3 * (8 + 4)
    st3, n3 = _ws(shape=(32, 32, 32), pattern=7, prec="fp16")
    assert st3 == smg.SMG_OK and n3 < n2  # half-precision coefficients with one FP32 scale per row
    assert _ws(shape=(32, 32, 32), pattern=5)[0] == smg.SMG_EINVAL
    assert _ws(shape=(0, 32, 32), pattern=7)[0] == smg.SMG_EINVAL
    assert _ws(shape=(8, 8, 8), pattern=7, block=3)[0] == smg.SMG_EINVAL
    assert _ws(shape=(8, 8, 8), pattern=27, block=3, smoother="ilu0")[0] == smg.SMG_EINVAL
    # coarsest level too large for the dense solve
    assert _ws(shape=(4, 4, 4096), pattern=7, coarsen="semi_xy")[0] == smg.SMG_EINVAL
    msg = smg.load().smg_last_error(None).decode()
    assert "max_coarse" in msg


def test_setup_rejects_null_arguments():
    L = smg.load()
    cfg = smg.make_config((8, 8, 8), pattern=7)
    h = C.c_void_p()
    assert L.smg_setup(C.byref(cfg), None, None, 0, None, C.byref(h)) == smg.SMG_EINVAL
    assert L.smg_precondition(None, None, None, None) == smg.SMG_EINVAL
    assert L.smg_solve(None, None, None, 1e-9, 10, 0, None, None) == smg.SMG_EINVAL


@pytest.mark.parametrize("bad", [dict(semi_levels=-1), dict(max_coarse=-5), dict(gmres_restart=500)])
def test_bad_configs(bad):
    kw = dict(shape=(16, 16, 16), pattern=7)
    kw.update(bad)
    assert _ws(**kw)[0] == smg.SMG_EINVAL


def test_batch_validation_host_only():
    """Batch sizing and configuration checks run on the host (no GPU)."""
    import ctypes as C
    import paper_2506_21932_amd as smg
    L = smg.load()
    shapes = [(16, 16, 16), (9, 30, 12), (5, 6, 7)]
    cfgs = (smg.Config * 3)(*[smg.make_config(s, 7, 1, "gs", "full", 3, "fp32", 512, 0) for s in shapes])
    n = C.c_size_t(0)
    assert L.smg_batch_workspace_size(3, cfgs, C.byref(n)) == smg.SMG_OK
    single = sum(smg.StructMG.workspace_bytes(s, pattern=7, semi_levels=3, prec="fp32", max_coarse=512)
                 for s in shapes)
    assert n.value > single  # every hierarchy plus the batch tables
    mixed = (smg.Config * 2)(smg.make_config((8, 8, 8), 7), smg.make_config((8, 8, 8), 19))
    assert L.smg_batch_workspace_size(2, mixed, C.byref(n)) == smg.SMG_EINVAL
    assert b"same pattern" in L.smg_batch_last_error(None)
    ilu = (smg.Config * 1)(smg.make_config((8, 8, 8), 7, smoother="ilu0"))
    assert L.smg_batch_workspace_size(1, ilu, C.byref(n)) == smg.SMG_EINVAL
    blk = (smg.Config * 1)(smg.make_config((8, 8, 8), 27, block=3))
    assert L.smg_batch_workspace_size(1, blk, C.byref(n)) == smg.SMG_EINVAL
    assert L.smg_batch_workspace_size(0, ilu, C.byref(n)) == smg.SMG_EINVAL
    assert L.smg_batch_workspace_size(4096, ilu, C.byref(n)) == smg.SMG_EINVAL


def test_smoother_and_interpolation_options_host_only():
    """Line GS, ILU masks and the interpolation options are validated and
    sized on the host."""
    base = _ws(shape=(32, 32, 32), pattern=19)[1]
    st, n = _ws(shape=(32, 32, 32), pattern=19, smoother="lgs")
    assert st == smg.SMG_OK and n > 0
    assert _ws(shape=(32, 32, 32), pattern=19, smoother="lgs", prec="fp32")[0] == smg.SMG_OK
    assert _ws(shape=(8, 8, 8), pattern=19, smoother="lgs", prec="fp16")[0] == smg.SMG_EINVAL
    assert _ws(shape=(8, 8, 8), pattern=27, block=3, smoother="lgs")[0] == smg.SMG_EINVAL
    assert _ws(shape=(4, 4, 2048), pattern=7, smoother="lgs", coarsen="semi_xy")[0] == smg.SMG_EINVAL
    # ILU masks: fewer slots with the 3d7 mask, more with 3d27, only for ILU(0)
    n19 = _ws(shape=(32, 32, 32), pattern=19, smoother="ilu0")[1]
    n7 = _ws(shape=(32, 32, 32), pattern=19, smoother="ilu0", ilu_mask=7)[1]
    n27 = _ws(shape=(32, 32, 32), pattern=19, smoother="ilu0", ilu_mask=27)[1]
    assert n7 < n19 < n27
    assert _ws(shape=(8, 8, 8), pattern=19, smoother="ilu0", ilu_mask=9)[0] == smg.SMG_EINVAL
    assert _ws(shape=(8, 8, 8), pattern=19, ilu_mask=7)[0] == smg.SMG_EINVAL
    # interpolation: cell-centred keeps the fine pattern (smaller coarse
    # levels), operator-dependent adds 8 weights per fine point
    assert _ws(shape=(32, 32, 32), pattern=7, interp="cell")[1] < _ws(shape=(32, 32, 32), pattern=7)[1]
    assert _ws(shape=(32, 32, 32), pattern=19, interp="operator")[1] > base
    assert _ws(shape=(32, 32, 32), pattern=7, interp="cell_trilinear")[0] == smg.SMG_OK
    assert _ws(shape=(8, 8, 8), pattern=27, block=3, interp="operator")[0] == smg.SMG_EINVAL
    cfg = smg.make_config((8, 8, 8), pattern=7)
    cfg.interp = 4
    n_ = C.c_size_t(0)
    assert smg.load().smg_workspace_size(C.byref(cfg), C.byref(n_)) == smg.SMG_EINVAL
    cells = (smg.Config * 1)(smg.make_config((8, 8, 8), 7, interp="cell"))
    assert smg.load().smg_batch_workspace_size(1, cells, C.byref(n_)) == smg.SMG_EINVAL


def test_setup_noalloc_rejects_hierarchies_beyond_its_array():
    """The static-array setup refuses, before any device call, a hierarchy
    larger than its array (so this runs without a GPU)."""
    cfg = smg.make_config(shape=(128, 128, 128), pattern=7)
    need = C.c_size_t(0)
    assert smg.load().smg_workspace_size(C.byref(cfg), C.byref(need)) == smg.SMG_OK
    assert need.value > 64 << 20
    h = C.c_void_p()
    st = smg.load().smg_setup_noalloc(C.byref(cfg), C.c_void_p(1), None, C.byref(h))
    assert st == smg.SMG_ENOMEM and not h.value
    msg = smg.load().smg_last_error(None).decode()
    assert "static scratch array" in msg
    assert smg.load().smg_setup_noalloc(C.byref(cfg), C.c_void_p(1), None, None) == smg.SMG_EINVAL


def _struct_fields(name):
    src = open(os.path.join(ROOT, "include", "structmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r";", src).group(1)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        m = re.match(r"(int|double)\s+(.*)", decl)
        names += [v.strip() for v in m.group(2).split(",")]
    return names


def test_binding_structs_match_header():
    assert [f[0] for f in smg.Config._fields_] == _struct_fields("smg_config")
    assert [f[0] for f in smg.Result._fields_] == _struct_fields("smg_result")


@pytest.mark.parametrize("bad", [dict(pre_sweeps=-1), dict(pre_sweeps=9), dict(post_sweeps=9),
                                 dict(relax_weight=-0.5), dict(relax_weight=2.0), dict(relax_weight=float("nan")),
                                 dict(relax_weight=1.2, smoother="ilu0"), dict(relax_weight=1.2, smoother="lgs"),
                                 dict(relax_weight=1.2, pattern=27, block=3), dict(zero_guess=2),
                                 dict(zero_guess=-2), dict(min_coarse=1), dict(min_coarse=5000),
                                 dict(coarsen="auto", pattern=27, block=3)])
def test_smoothing_and_coarsening_fields_validated(bad):
    kw = dict(shape=(16, 16, 16), pattern=7)
    kw.update(bad)
    assert _ws(**kw)[0] == smg.SMG_EINVAL
    assert smg.load().smg_last_error(None).decode() != "no error"


def test_smoothing_fields_size_their_buffers():
    base = _ws(shape=(32, 32, 32), pattern=7)[1]
    # defaults spelled out are the defaults
    assert _ws(shape=(32, 32, 32), pattern=7, pre_sweeps=1, post_sweeps=1, relax_weight=1.0, zero_guess=1,
               min_coarse=4)[1] == base
    assert _ws(shape=(32, 32, 32), pattern=7, pre_sweeps=2, post_sweeps=2)[1] == base
    # an odd number of steps per level needs a third sweep buffer; the weight
    # its old-centre terms; ZeroGuess off a vector of zeros
    for kw in (dict(pre_sweeps=2), dict(relax_weight=1.3), dict(zero_guess=-1)):
        assert _ws(shape=(32, 32, 32), pattern=7, **kw)[1] > base, kw
    # min_coarse 2 adds the 2^3 level below 4^3
    assert _ws(shape=(32, 32, 32), pattern=7, min_coarse=2)[1] > base


def test_auto_coarsening_sizes_for_every_choice():
    L = smg.load()
    auto = _ws(shape=(64, 64, 48), pattern=7, coarsen="auto")
    assert auto[0] == smg.SMG_OK
    sizes = [_ws(shape=(64, 64, 48), pattern=7, coarsen="full", semi_levels=s)[1] for s in range(0, 8)]
    assert auto[1] == max(sizes)
    assert L is not None


def test_batch_rejects_non_default_smoothing():
    L = smg.load()
    n = C.c_size_t(0)
    for kw in (dict(pre_sweeps=2), dict(relax_weight=1.1), dict(zero_guess=-1), dict(coarsen="auto")):
        cfgs = (smg.Config * 1)(smg.make_config((8, 8, 8), 7, **kw))
        assert L.smg_batch_workspace_size(1, cfgs, C.byref(n)) == smg.SMG_EINVAL, kw
        assert "batches" in L.smg_batch_last_error(None).decode()

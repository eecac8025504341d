"""The C ABI library loads and exports every entry point declared in
include/lg.h; argument validation rejects bad calls before any device work
(no GPU is touched).  CPU only."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2511_07418_amd", "liblg.so")


def declared():
    src = open(os.path.join(ROOT, "include", "lg.h")).read()
    return sorted(set(re.findall(r"\b(lg_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lglib():
    if not os.path.exists(LIB):
        from paper_2511_07418_amd import build
        build.build()
    from paper_2511_07418_amd import lg
    return lg


def test_exports_every_declared_symbol(lglib):
    L = C.CDLL(LIB)
    names = declared()
    assert {"lg_build_field", "lg_query_domains", "lg_search", "lg_realize"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    assert set(lglib.EXPORTED) == set(names)
    assert lglib.version().startswith("lg-gfx950")


def test_status_strings(lglib):
    L = lglib.lib()
    assert L.lg_status_str(0) == b"LG_OK"
    assert L.lg_status_str(-1) == b"LG_EINVAL"


def test_validation_rejects_bad_calls_without_device_work(lglib):
    L = lglib.lib()
    assert L.lg_query_domains(None, None, None, 0, None, 1, None, None, None) == lglib.LG_EINVAL
    assert b"null field" in L.lg_last_error()
    assert L.lg_search(None, None, None, 0, None, 0, None, None, None, None, None, None, None, None,
                       None, None, 0, None) == lglib.LG_EINVAL
    assert L.lg_realize(None, None, None, None, 0, None, 0, None, None, 0, 0, None, None, 0, None,
                        None, None, None, None, None, None) == lglib.LG_EINVAL
    w = synth.workload("c1", n_poses=2)
    # 48 bins is not supported (32 or 64)
    fp = synth.FieldParams(samples=16, seed=0, grid=8, h=0.01, bins=48, grid_frame=w.field.grid_frame)
    with pytest.raises(lglib.LgError) as ei:
        lglib.lg_build_field(w.hand, fp)
    assert ei.value.status == lglib.LG_EINVAL
    # a finger that is not a serial chain
    bad = synth.hand_c1()
    bad.joint_parent = bad.joint_parent.copy()
    bad.joint_parent[2] = 0
    with pytest.raises(lglib.LgError):
        lglib.lg_build_field(bad, w.field)


def test_proposer_validation_rejects_bad_calls_without_device_work(lglib):
    L = lglib.lib()
    EINVAL = lglib.LG_EINVAL
    assert L.lg_prop_num_params() == 204568
    bad = lglib.PropParams(0, 2048, 16, 0)          # max_batch < 1
    out = C.c_void_p()
    assert L.lg_prop_create(C.byref(bad), None, C.byref(out)) == EINVAL and not out.value
    assert L.lg_prop_create(None, None, C.byref(out)) == EINVAL
    assert L.lg_prop_forward(None, None, 1, 1, None, None, None, None) == EINVAL
    assert L.lg_prop_backward(None, None, 1, 1, None, None, 1, None, None, None) == EINVAL
    assert L.lg_prop_adam(None, 1e-3, 0.9, 0.999, 1e-8, None) == EINVAL
    assert L.lg_prop_train_step(None, None, 1, 1, None, None, 1, 1e-3, None, None) == EINVAL
    assert L.lg_prop_sample(None, None, 1, 1, 0, 0.5, 0.08, 0.12, None, None) == EINVAL
    assert L.lg_prop_get_params(None, None) == EINVAL and L.lg_prop_set_params(None, None) == EINVAL
    # sampler arguments: negative count, fraction outside [0, 1], d_lo > d_hi, null buffers
    assert L.lg_prop_sample_mixture(None, -1, 0, 0.5, 0.08, 0.12, None, None) == EINVAL
    assert L.lg_prop_sample_mixture(None, 0, 0, 0.5, 0.08, 0.12, None, None) == lglib.LG_OK
    assert L.lg_prop_sample_mixture(None, 4, 0, 0.5, 0.08, 0.12, None, None) == EINVAL
    dummy = C.c_void_p(1)
    assert L.lg_prop_sample_mixture(dummy, 4, 0, 1.5, 0.08, 0.12, dummy, None) == EINVAL
    assert L.lg_prop_sample_mixture(dummy, 4, 0, 0.5, 0.12, 0.08, dummy, None) == EINVAL
    assert b"d_lo" in L.lg_last_error()
    assert L.lg_prop_release(None) == lglib.LG_OK


def test_search_workspace_grows_with_the_optimisation(lglib):
    w = synth.workload("c1", n_poses=4)
    p0 = lglib.search_params(w.search)
    import dataclasses
    p1 = lglib.search_params(dataclasses.replace(w.search, opt_outer=1))
    L = lglib.lib()
    b0 = L.lg_search_workspace_bytes(2048, 256, C.byref(p0))
    b1 = L.lg_search_workspace_bytes(2048, 256, C.byref(p1))
    assert b1 >= b0 + 2048 * 4 and L.lg_search_workspace_bytes(2048, 0, C.byref(p1)) == 256
    # with Alg. 2 the asked-for workspace holds, beyond the candidate ids
    # (4 B per set, contact and candidate), the gathered-LP criteria arrays:
    # 36 B per set (last pick's t* and basis) + 40 B per candidate (t*, basis, queue)
    n_sets, k, n_in = 256 * w.search.draws, w.search.k, p1.opt_inner
    assert b1 - b0 >= n_sets * k * n_in * 4 + n_sets * 36 + n_sets * n_in * 40


def test_concave_filter_validation_without_device_work(lglib):
    L = lglib.lib()
    EINVAL = lglib.LG_EINVAL
    dummy = C.c_void_p(16)        # never dereferenced: validation fails first
    good = lglib.Sdf((C.c_float * 3)(0, 0, 0), 0.002, 64, dummy)
    args = (dummy, dummy, 8, 0.008, 4, 0.001, dummy, dummy, dummy, dummy, None)
    assert L.lg_concave_filter(None, *args) == EINVAL
    bad_sdf = lglib.Sdf((C.c_float * 3)(0, 0, 0), 0.0, 64, dummy)
    assert L.lg_concave_filter(C.byref(bad_sdf), *args) == EINVAL
    for edge, lat, depth in ((0.0, 4, 0.001), (-1.0, 4, 0.001), (0.008, 0, 0.001), (0.008, 17, 0.001),
                             (0.008, 4, float("nan"))):
        assert L.lg_concave_filter(C.byref(good), dummy, dummy, 8, edge, lat, depth, dummy, dummy, dummy, dummy,
                                   None) == EINVAL
    assert L.lg_concave_filter(C.byref(good), dummy, dummy, -1, 0.008, 4, 0.001, dummy, dummy, dummy, dummy,
                               None) == EINVAL
    assert L.lg_concave_filter(C.byref(good), None, dummy, 8, 0.008, 4, 0.001, dummy, dummy, dummy, dummy,
                               None) == EINVAL
    assert L.lg_gather_points(dummy, dummy, 8, dummy, -1, dummy, dummy, None) == EINVAL
    assert L.lg_gather_points(dummy, None, 8, dummy, 4, dummy, dummy, None) == EINVAL
    assert L.lg_gather_points(None, None, 8, None, 0, None, None, None) == lglib.LG_OK   # nothing to do


def test_morton_order_on_the_host(lglib):
    """lg_morton_order is a host routine: a permutation whose Morton codes,
    recomputed here from the definition (10 bits per axis over the bounding
    cube, x lowest), never decrease, with ties in input order."""
    rng = np.random.default_rng(4)
    p = rng.normal(size=(5000, 3)).astype(np.float32) * np.float32([0.05, 0.02, 0.08])
    p[100:110] = p[100]                                  # ties
    perm = lglib.lg_morton_order(p)
    assert sorted(perm.tolist()) == list(range(len(p)))
    q = p.astype(np.float64)
    lo = q.min(0)
    ext = (q.max(0) - lo).max()
    iq = np.clip(np.floor((q - lo) / ext * 1023.0), 0, 1023).astype(np.uint64)
    code = np.zeros(len(p), np.uint64)
    for b in range(10):
        for a in range(3):
            code |= ((iq[:, a] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + a)
    assert (np.diff(code[perm].astype(np.int64)) >= 0).all()
    tied = [i for i in perm if 100 <= i < 110]
    assert tied == sorted(tied)
    L = lglib.lib()
    assert L.lg_morton_order(None, 4, None) == lglib.LG_EINVAL
    bad = p.copy()
    bad[3, 1] = np.nan
    with pytest.raises(lglib.LgError):
        lglib.lg_morton_order(bad)
    assert L.lg_chunk_bounds(None, 10, None, None) == lglib.LG_EINVAL


def test_server_parameters_checked_before_device_work(lglib):
    """lg_serve_create refuses bad parameters (batch slots, active requests,
    chunk size) before it allocates anything."""
    L = lglib.lib()
    h = C.c_void_p()
    for p in (lglib.ServerParams(1 << 20, 4, 64, 1, 9),     # more than 8 batch slots
              lglib.ServerParams(1 << 20, 4, 64, 1, -1),    # negative batch slots
              lglib.ServerParams(1 << 20, 65, 64, 1, 0),    # more than 64 active requests
              lglib.ServerParams(1 << 20, 4, 0, 0, 0)):     # empty chunks
        assert L.lg_serve_create(C.byref(p), C.byref(h)) == lglib.LG_EINVAL
        assert b"batch_slots" in L.lg_last_error() or b"max_active" in L.lg_last_error()
        assert h.value is None

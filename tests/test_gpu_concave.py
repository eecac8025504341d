"""GPU parity of the concave-point preprocessing (Sec. 5.2) against the FP64
oracle, through the C ABI.

Bars: depth within 1e-6 m (FP32 lattice positions and trilinear weights err by
~1e-8 m); keep identical outside the oracle's flags (depth within 1e-6 of the
threshold); kept indices exactly the GPU's keep mask in increasing order;
gathered points bit-identical copies.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import dev, lgmod, soa

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def tool():
    w = synth.workload("c3", n_poses=1, samples=1024, with_sdf=True)
    return w


def _check(w, idx, edge=0.008, lattice=4, max_depth=0.001):
    lg = lgmod()
    pts, nrm = w.obj.pts[idx], w.obj.nrm[idx]
    sdf_vals = dev(w.sdf.values)
    sdf = lg.sdf_struct(w.sdf, sdf_vals)
    r = lg.lg_concave_filter(sdf, soa(pts), soa(nrm), edge, lattice, max_depth)
    torch.cuda.synchronize()
    n = len(idx)
    d = r.depth.cpu().numpy()[:n]
    keep = r.keep.cpu().numpy()[:n]
    nk = int(r.n_kept.item())
    kept = r.kept_idx.cpu().numpy()[:nk]
    o = oracle.concave_filter(w.sdf, pts, nrm, edge, lattice, max_depth)
    assert np.abs(d - o["depth"]).max(initial=0.0) <= 1e-6
    fl = o["flag"].astype(bool)
    assert ((keep != o["keep"]) & ~fl).sum() == 0
    assert nk == int(keep.sum()) and (kept == np.flatnonzero(keep)).all()
    return r, keep, nk


def test_c3_tool_full(tool):
    r, keep, nk = _check(tool, np.arange(tool.obj.n))
    assert 0.5 * tool.obj.n < nk < tool.obj.n          # creases are dropped, most of the surface kept


@pytest.mark.parametrize("n", [1, 1023, 1024, 1025, 5000])
def test_ragged_sizes(tool, n):
    idx = np.random.default_rng(n).choice(tool.obj.n, n, replace=False)
    _check(tool, idx)


@pytest.mark.parametrize("lattice,edge", [(1, 0.008), (2, 0.004), (16, 0.012)])
def test_lattices(tool, lattice, edge):
    idx = np.random.default_rng(lattice).choice(tool.obj.n, 4096, replace=False)
    _check(tool, idx, edge=edge, lattice=lattice)


def test_no_points():
    lg = lgmod()
    w = synth.workload("c1", n_poses=1, with_sdf=True)
    sdf_vals = dev(w.sdf.values)
    sdf = lg.sdf_struct(w.sdf, sdf_vals)
    e = torch.empty((3, 0), dtype=torch.float32, device="cuda")
    r = lg.lg_concave_filter(sdf, e, e)
    torch.cuda.synchronize()
    assert int(r.n_kept.item()) == 0


def test_gather_and_pipeline_on_kept_points(tool):
    from paper_2511_07418_amd.pipeline import Pipeline
    lg = lgmod()
    w = synth.workload("c3", n_poses=256, samples=8192, with_sdf=True)
    sdf_vals = dev(w.sdf.values)
    sdf = lg.sdf_struct(w.sdf, sdf_vals)
    P, Nn = soa(w.obj.pts), soa(w.obj.nrm)
    r = lg.lg_concave_filter(sdf, P, Nn)
    nk = int(r.n_kept.item())
    po, no = lg.lg_gather_points(P, Nn, r.kept_idx, nk)
    torch.cuda.synchronize()
    kept = r.kept_idx[:nk].long()
    assert torch.equal(po, P[:, kept]) and torch.equal(no, Nn[:, kept])
    # an index outside the points gives NaN columns
    bad = torch.tensor([0, w.obj.n, -1], dtype=torch.int32, device="cuda")
    bo, _ = lg.lg_gather_points(P, Nn, bad, 3)
    torch.cuda.synchronize()
    assert torch.equal(bo[:, 0], P[:, 0]) and torch.isnan(bo[:, 1:]).all()
    # the path runs unchanged on the kept points (a count that is not a multiple of 32)
    pts_k = po.t().cpu().numpy()
    nrm_k = no.t().cpu().numpy()
    field = lg.lg_build_field(w.hand, w.field, keep_witness=True)
    pipe = Pipeline(field, pts_k, nrm_k, w.poses, w.search, sdf=w.sdf, ik=w.ik)
    pipe.step()
    torch.cuda.synchronize()
    assert pipe.n_acc() > 0

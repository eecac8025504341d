"""lg_search_noalloc (the search on the library's static device scratch)
against lg_search (the search on a caller workspace), through the C ABI.

The plain search runs the same kernels in both, so every output must be
identical: drawn points and links, verdicts, t* (bit for bit, NaN where the
set is invalid), the accepted list and its length.  With contact-point
optimisation (Alg. 2) lg_search gathers the slow criterion LPs into launches
of their own (per-candidate arrays in its workspace), while lg_search_noalloc
does so only where those arrays fit the static scratch and otherwise solves a
step's LPs in one launch: the same LPs from the same starting bases, compiled
into different kernels, so the points, links, verdicts and accepted lists
must still be identical and t* agrees within 1e-9 (the bar against the
oracle), not bit for bit.  Two calls in a row on the shared scratch, the
second smaller than the first (the first call of the Alg. 2 case exceeds the
scratch with those arrays, the second fits), for the plain search and for the
search with Alg. 2, whose cell grid lives in the scratch and is cleared by a
kernel on every call.  A request above the scratch size is refused before
anything is enqueued.
"""
import dataclasses

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _lg():
    from paper_2511_07418_amd import lg
    return lg


def _outputs(b):
    n = int(b.n_acc.item())
    return {"set_pt": b.set_pt.cpu().numpy(), "set_link": b.set_link.cpu().numpy(),
            "verdict": b.verdict.cpu().numpy(), "tstar": b.tstar.cpu().numpy(), "n_acc": n,
            "acc": b.acc_list[:n].cpu().numpy()}


def _same(a, b, exact_tstar=True):
    for key in ("set_pt", "set_link", "verdict", "acc"):
        assert np.array_equal(a[key], b[key]), key
    assert a["n_acc"] == b["n_acc"]
    ta, tb = a["tstar"], b["tstar"]
    assert np.array_equal(np.isnan(ta), np.isnan(tb))
    fa, fb = ta[~np.isnan(ta)], tb[~np.isnan(tb)]
    if exact_tstar:
        assert np.array_equal(fa.view(np.uint64), fb.view(np.uint64))
    else:
        dt = float(np.abs(fa - fb).max()) if fa.size else 0.0
        print(f"[no_alloc] max |t* difference| {dt:.3e} over {fa.size} sets", flush=True)
        assert dt <= 1e-9


def _case(name, n_poses, n_points, opt):
    lg = _lg()
    w = synth.workload(name, n_poses=n_poses, n_points=n_points, samples=8192, with_sdf=False)
    sp = w.search
    if opt:
        sp = dataclasses.replace(sp, opt_outer=1, opt_inner=4)
    field = lg.lg_build_field(w.hand, w.field)
    pts = torch.from_numpy(np.ascontiguousarray(w.obj.pts.T)).cuda()
    nrm = torch.from_numpy(np.ascontiguousarray(w.obj.nrm.T)).cuda()
    poses = torch.from_numpy(np.ascontiguousarray(w.poses, np.float32)).cuda()
    F, NW = w.hand.n_fingers, (pts.shape[1] + 31) // 32
    dom_bits = torch.empty((poses.shape[0], F, NW), dtype=torch.int32, device="cuda")
    dom_count = torch.empty((poses.shape[0], F), dtype=torch.int32, device="cuda")
    lg.lg_query_domains(field, pts, nrm, poses, dom_bits, dom_count)
    ref = _outputs(lg.lg_search(field, pts, nrm, poses, dom_bits, dom_count, sp))
    out = lg.SearchBuffers(poses.shape[0], sp, "cuda", n_points=pts.shape[1])
    for t in (out.set_pt, out.set_link, out.verdict, out.acc_list, out.n_acc):
        t.fill_(-7)
    out.tstar.fill_(-7.0)
    lg.lg_search_noalloc(field, pts, nrm, poses, dom_bits, dom_count, sp, out)
    torch.cuda.synchronize()
    got = _outputs(out)
    field.release()
    assert ref["n_acc"] > 0
    return ref, got


@pytest.mark.parametrize("name,sizes,opt", [
    ("c1", [(256, 2048), (97, 1500)], False),
    ("c3", [(512, 8192), (129, 3001)], True),
])
def test_noalloc_equals_workspace_search_twice(name, sizes, opt):
    for n_poses, n_points in sizes:      # second call smaller: the scratch keeps the first call's contents
        print(f"[no_alloc] {name} P={n_poses} N={n_points} opt={opt}", flush=True)
        ref, got = _case(name, n_poses, n_points, opt)
        _same(ref, got, exact_tstar=not opt)


def test_noalloc_refuses_above_the_scratch():
    lg = _lg()
    w = synth.workload("c1", n_poses=16, samples=1024, with_sdf=False)
    sp = lg.search_params(w.search)
    cap = int(lg.lib().lg_search_noalloc_max_bytes())
    assert cap == 8 << 20
    big_p = 4_000_000           # needs more than 8 MiB of workspace
    assert int(lg.lib().lg_search_workspace_bytes(2048, big_p, lg.C.byref(sp))) > cap
    field = lg.lg_build_field(w.hand, w.field)
    pts = torch.zeros((3, 2048), dtype=torch.float32, device="cuda")
    poses = torch.zeros((1, 12), dtype=torch.float32, device="cuda")
    dummy = torch.zeros((1,), dtype=torch.int32, device="cuda")
    st = lg.lib().lg_search_noalloc(field.handle, lg._ptr(pts), lg._ptr(pts), 2048, lg._ptr(poses), big_p,
                                    lg._ptr(dummy), lg._ptr(dummy), lg.C.byref(sp), lg._ptr(dummy), lg._ptr(dummy),
                                    lg._ptr(dummy), lg._ptr(dummy), lg._ptr(dummy), lg._ptr(dummy), None)
    assert st == lg.LG_EINVAL
    assert b"static scratch" in lg.lib().lg_last_error()
    field.release()

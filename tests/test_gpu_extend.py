"""GPU parity of the second contact round on the unused fingers (Sec. 5.3's
additional search phase; Sec. 5.6, the general form) through the C ABI:
lg_compact_unstable, lg_search_extend and lg_realize of the extended sets,
each fed the oracle's own inputs (imported field, domains, round-1 sets).

Bars: the list of unstable sets exact; extended points bit-exact; links
exact outside the oracle's band flags (at most 1e-4 of entries flagged and
different); verdicts exact outside |t* - eps| <= 1e-6; t* within 1e-9;
compaction in increasing set order; realize of the extended sets at the
realize bar (tests/_realize_bars.py).
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests._realize_bars import check_realize
from tests.test_gpu_parity import dev, lgmod, soa

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _round1(name="c3", k1=2, n_poses=256, n_points=8192, draws=32):
    w = synth.workload(name, samples=4096, n_poses=n_poses, n_points=n_points, with_sdf=True)
    w = dataclasses.replace(w, search=dataclasses.replace(w.search, k=k1, draws=draws))
    ref = oracle.build_field(w.hand, w.field, witness=True, flags=False)
    Q = oracle.query(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, flags=False)
    spt, sln = oracle.draw(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                           Q["dom_count"], w.search)
    V = oracle.verdicts(w.obj.pts, w.obj.nrm, spt, w.search)
    return w, ref, Q, spt, sln, V


class _Round1Bufs:
    """The oracle's round-1 sets on the device, in lg_search's buffer layout."""

    def __init__(self, spt, sln, verdict):
        self.set_pt = dev(spt.astype(np.int32))
        self.set_link = dev(sln.astype(np.int8))
        self.verdict = dev(verdict.astype(np.uint8))


def _extend_check(w, ref, Q, spt, sln, V, k_add, take, set_list=None, list_n=None, list_ok=None, request_id=3):
    lg = lgmod()
    P, D, k1 = spt.shape
    field = lg.lg_field_import(w.hand, w.field, ref["bits"], ref["wit"])
    r1 = _Round1Bufs(spt, sln, V["verdict"].reshape(P, D))
    eb = lg.lg_search_extend(field, soa(w.obj.pts), soa(w.obj.nrm), dev(w.poses), dev(Q["dom_bits"].view(np.int32)),
                             dev(Q["dom_count"].view(np.int32)), w.search, r1, k_add, request_id=request_id,
                             set_list=set_list, list_n=list_n, list_ok=list_ok)
    torch.cuda.synchronize()
    g_pt = eb.set_pt.cpu().numpy()
    g_ln = eb.set_link.cpu().numpy().astype(np.int32)
    g_v = eb.verdict.cpu().numpy().reshape(-1)
    g_t = eb.tstar.cpu().numpy().reshape(-1)
    g_acc = eb.acc_list[:int(eb.n_acc.item())].cpu().numpy()
    o_pt, o_ln, o_lf = oracle.extend(w.hand, w.field, ref["bits"], w.obj.pts, w.obj.nrm, w.poses, Q["dom_bits"],
                                     Q["dom_count"], spt, sln, take, k_add, w.search, request_id=request_id)
    assert np.array_equal(g_pt, o_pt), "extended points differ"
    mis = g_ln != o_ln
    assert (mis & (o_lf == 0)).sum() == 0, "links differ outside the rounding bands"
    assert mis.sum() <= max(1, 1e-4 * mis.size)
    sp2 = dataclasses.replace(w.search, k=k1 + k_add)
    V2 = oracle.verdicts(w.obj.pts, w.obj.nrm, o_pt, sp2)
    vf = V2["vflag"].astype(bool)
    assert ((g_v != V2["verdict"]) & ~vf).sum() == 0, "verdicts differ outside the band"
    fin = ~np.isnan(V2["tstar"])
    assert np.allclose(g_t[fin], V2["tstar"][fin], atol=1e-9, rtol=0) and np.isnan(g_t[~fin]).all()
    assert (g_acc == np.flatnonzero(g_v)).all(), "compaction order"
    ext = o_pt[..., 0] >= 0
    assert ext.sum() > 0
    return field, o_pt, o_ln, V2, ext


def test_compact_unstable_matches_definition():
    lg = lgmod()
    w, ref, Q, spt, sln, V = _round1()
    P, D, k = spt.shape
    verdict = V["verdict"].reshape(P, D)
    sln_m = sln.copy()
    sln_m[::7, ::5, 0] = -1                      # some sets without a link: never listed
    r1 = _Round1Bufs(spt, sln_m, verdict)
    lst, n, _ = lg.lg_compact_unstable(r1)
    torch.cuda.synchronize()
    want = np.flatnonzero(((spt >= 0).all(-1) & (sln_m >= 0).all(-1) & (verdict == 0)).reshape(-1))
    assert int(n.item()) == len(want) and (lst[:len(want)].cpu().numpy() == want).all()
    # no sets at all
    empty = _Round1Bufs(spt[:0], sln[:0], verdict[:0])
    lst0, n0, _ = lg.lg_compact_unstable(empty)
    torch.cuda.synchronize()
    assert int(n0.item()) == 0


@pytest.mark.parametrize("k1,k_add", [(2, 2), (3, 2), (1, 4)])
def test_extend_every_unstable_set(k1, k_add):
    w, ref, Q, spt, sln, V = _round1(k1=k1)
    P, D, _ = spt.shape
    take = ((spt >= 0).all(-1) & (sln >= 0).all(-1) & (V["verdict"].reshape(P, D) == 0)).astype(np.uint8)
    _extend_check(w, ref, Q, spt, sln, V, k_add, take)


def test_extend_listed_sets_with_ok_mask_then_realize():
    """The general form's chain: the unstable sets listed, a per-entry mask
    (here the oracle's realize of the round-1 sets: collision-free with the
    contacts met), the extended sets realised with k1 + k_add contacts."""
    lg = lgmod()
    w, ref, Q, spt, sln, V = _round1(k1=2, n_poses=192)
    P, D, k1 = spt.shape
    unstable = np.flatnonzero(((spt >= 0).all(-1) & (sln >= 0).all(-1) & (V["verdict"].reshape(P, D) == 0))
                              .reshape(-1)).astype(np.int32)
    R1 = oracle.realize(w.hand, w.field, ref["wit"], w.sdf, w.obj.pts, w.obj.nrm, w.poses, spt.reshape(-1, k1),
                        sln.reshape(-1, k1), w.search, unstable, w.ik)
    ok = R1["valid"].astype(np.uint8)
    assert 0 < ok.sum() < len(ok)
    take = np.zeros(P * D, np.uint8)
    take[unstable[ok != 0]] = 1
    field, o_pt, o_ln, V2, ext = _extend_check(
        w, ref, Q, spt, sln, V, 2, take.reshape(P, D), set_list=dev(unstable), list_n=dev(np.array([len(unstable)],
                                                                                                np.int32)),
        list_ok=dev(ok))
    assert (ext.reshape(-1) <= take.astype(bool)).all()
    # realize the oracle's accepted extended sets on the GPU and in the oracle
    k2 = k1 + 2
    sp2 = dataclasses.replace(w.search, k=k2)
    acc2 = oracle.compact(V2["verdict"])
    assert len(acc2) > 0
    R2 = oracle.realize(w.hand, w.field, ref["wit"], w.sdf, w.obj.pts, w.obj.nrm, w.poses, o_pt.reshape(-1, k2),
                        o_ln.reshape(-1, k2), sp2, acc2, w.ik)
    sdf_vals = dev(w.sdf.values)
    sdf = lg.sdf_struct(w.sdf, sdf_vals)
    rb = lg.lg_realize(field, sdf, soa(w.obj.pts), soa(w.obj.nrm), dev(w.poses), dev(o_pt.astype(np.int32)),
                       dev(o_ln.astype(np.int8)), k2, D, dev(acc2.astype(np.int32)),
                       dev(np.array([len(acc2)], np.int32)), len(acc2), w.ik, sp=sp2)
    torch.cuda.synchronize()
    n = len(acc2)
    check_realize(w.hand, R2, rb.q[:n].cpu().numpy(), rb.contact_err[:n].cpu().numpy(), rb.depth[:n].cpu().numpy(),
                  rb.valid[:n].cpu().numpy())


def test_extend_argument_errors():
    lg = lgmod()
    w, ref, Q, spt, sln, V = _round1(k1=3, n_poses=8, n_points=256, draws=4)
    field = lg.lg_field_import(w.hand, w.field, ref["bits"], ref["wit"])
    P, D, _ = spt.shape
    r1 = _Round1Bufs(spt, sln, V["verdict"].reshape(P, D))
    args = (field, soa(w.obj.pts), soa(w.obj.nrm), dev(w.poses), dev(Q["dom_bits"].view(np.int32)),
            dev(Q["dom_count"].view(np.int32)), w.search, r1)
    with pytest.raises(lg.LgError):
        lg.lg_search_extend(*args, 3)            # 3 + 3 > 5 fingers
    with pytest.raises(lg.LgError):
        lg.lg_search_extend(*args, 1, set_list=dev(np.zeros(1, np.int32)))   # a list without its count


def test_pipeline_general_form():
    """The whole chain on the GPU (query, round 1 with k = 2, realize, the
    unstable list, its realize, the extension by 2, realize of the extended
    sets): deterministic, adds valid grasps, and the extension takes only
    listed sets that realised collision-free."""
    from paper_2511_07418_amd.pipeline import Pipeline
    lg = lgmod()
    w = synth.workload("c3", samples=8192, n_poses=512, n_points=16384)
    w = dataclasses.replace(w, search=dataclasses.replace(w.search, k=2))
    field = lg.lg_build_field(w.hand, w.field, keep_witness=True)
    pipe = Pipeline(field, w.obj.pts, w.obj.nrm, w.poses, w.search, ik=w.ik, sdf=w.sdf, extend_k=2)
    pipe.step()
    torch.cuda.synchronize()
    v1 = int(pipe.rbuf.valid[:pipe.n_acc()].sum().item())
    total = pipe.valid_count()
    n2 = int(pipe.ebuf.n_acc.item())
    assert n2 > 0 and total > v1
    lst, n, _ = pipe.unstable
    n = int(n.item())
    ok = pipe.rbuf_rej.valid[:n].cpu().numpy().astype(bool)
    listed_ok = set(lst[:n].cpu().numpy()[ok].tolist())
    ext = np.flatnonzero((pipe.ebuf.set_pt[..., 0] >= 0).cpu().numpy().reshape(-1))
    assert set(ext.tolist()) <= listed_ok
    state = (pipe.ebuf.set_pt.clone(), pipe.ebuf.verdict.clone(), pipe.rbuf2.valid[:n2].clone())
    pipe.step()
    torch.cuda.synchronize()
    assert pipe.valid_count() == total
    assert torch.equal(state[0], pipe.ebuf.set_pt) and torch.equal(state[1], pipe.ebuf.verdict)
    assert torch.equal(state[2], pipe.rbuf2.valid[:n2])

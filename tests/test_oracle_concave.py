"""Pins of the concave-point preprocessing oracle (Sec. 5.2: a small box placed
at an object point; the point is dropped when the box penetrates the object
significantly):

* a flat surface: the box stands on it, penetration 0 (trilinear interpolation
  of a linear SDF is exact), and every point is kept; turned the wrong way
  (normal into the object) the box would sink by its full edge;
* inside a spherical cavity of radius R: the bottom-face corners sit at
  sqrt(R^2 + s^2/2) from the centre, so the penetration is
  sqrt(R^2 + s^2/2) - R, within the trilinear error bound 3 h^2 / (8 R);
* on a ball (convex): the deepest lattice point is the face centre on the
  surface, penetration 0 within the same bound;
* the tool object's SDF: the oracle's penetration equals the maximum over the
  lattice evaluated with scipy's RegularGridInterpolator (an independent
  trilinear interpolation); refining the lattice (m -> 2m, a superset of
  points) never lowers it; the filter drops points near the tool's creases
  and keeps most of the surface.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import synth


def _grid(f, lo, h, G):
    ax = lo + h * np.arange(G)
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    v = f(np.stack([x, y, z], -1).reshape(-1, 3)).reshape(G, G, G)
    return synth.SDF(origin=np.full(3, lo, np.float32), h=float(h), dims=G, values=v.astype(np.float32))


def test_flat_surface():
    h, G = 0.002, 40
    sdf = _grid(lambda x: x[:, 2], -0.039, h, G)          # object z < 0, SDF = z
    rng = np.random.default_rng(0)
    p = np.zeros((200, 3), np.float32)
    p[:, :2] = rng.uniform(-0.02, 0.02, size=(200, 2))
    n = np.tile(np.float32([0, 0, 1]), (200, 1))
    r = oracle.concave_filter(sdf, p, n, 0.008, 4, 0.001)
    assert np.abs(r["depth"]).max() <= 1e-7 and r["keep"].all()
    wrong = oracle.concave_filter(sdf, p, -n, 0.008, 4, 0.001)
    np.testing.assert_allclose(wrong["depth"], 0.008, atol=1e-7)
    assert not wrong["keep"].any()


@pytest.mark.parametrize("R,s", [(0.03, 0.008), (0.02, 0.012)])
def test_spherical_cavity(R, s):
    h, G = 0.0015, 56
    sdf = _grid(lambda x: R - np.linalg.norm(x, axis=1), -0.041, h, G)  # object |x| > R
    rng = np.random.default_rng(1)
    u = rng.normal(size=(300, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    p = (R * u).astype(np.float32)
    n = (-u).astype(np.float32)
    want = math.sqrt(R * R + s * s / 2) - R
    r = oracle.concave_filter(sdf, p, n, s, 4, 0.5 * want)
    bound = 3 * h * h / (8 * (R - 0.5 * s)) + 1e-6
    assert np.abs(r["depth"] - want).max() <= bound
    assert not r["keep"].any()
    assert oracle.concave_filter(sdf, p, n, s, 4, 2.0 * want)["keep"].all()


def test_ball_is_kept():
    R, h, G = 0.04, 0.002, 56
    sdf = _grid(lambda x: np.linalg.norm(x, axis=1) - R, -0.055, h, G)
    rng = np.random.default_rng(2)
    u = rng.normal(size=(300, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = oracle.concave_filter(sdf, (R * u).astype(np.float32), u.astype(np.float32), 0.008, 4, 0.001)
    assert np.abs(r["depth"]).max() <= 3 * h * h / (8 * R) + 1e-6
    assert r["keep"].all()


@pytest.fixture(scope="module")
def tool():
    w = synth.workload("c3", n_poses=1, with_sdf=True, samples=1024, n_points=8192)
    return w.obj, w.sdf


def test_tool_against_scipy_interpolation(tool):
    obj, sdf = tool
    rng = np.random.default_rng(3)
    idx = rng.choice(obj.n, 200, replace=False)
    p, nrm = obj.pts[idx].astype(np.float64), obj.nrm[idx].astype(np.float64)
    s, m = 0.008, 2
    r = oracle.concave_filter(sdf, obj.pts[idx], obj.nrm[idx], s, m, 0.001)
    G, h = sdf.dims, float(np.float32(sdf.h))
    o = sdf.origin.astype(np.float64)
    ax = [o[a] + h * np.arange(G) for a in range(3)]
    # values are [iz][iy][ix]: the interpolator takes axes (x, y, z) of the transposed grid
    f = RegularGridInterpolator(ax, np.transpose(sdf.values.astype(np.float64), (2, 1, 0)),
                                bounds_error=False, fill_value=np.inf)
    t = -0.5 * s + s * np.arange(m + 1) / m
    c = s * np.arange(m + 1) / m
    for j in range(len(idx)):
        n = nrm[j] / np.linalg.norm(nrm[j])
        x, y = oracle.tangent_basis(n)
        A, B, Cc = np.meshgrid(t, t, c, indexing="ij")
        q = p[j] + A.reshape(-1, 1) * x + B.reshape(-1, 1) * y + Cc.reshape(-1, 1) * n
        assert r["depth"][j] == pytest.approx(np.max(-f(q)), abs=1e-9)


def test_refined_lattice_never_lowers_and_creases_are_dropped(tool):
    obj, sdf = tool
    r1 = oracle.concave_filter(sdf, obj.pts, obj.nrm, 0.008, 2, 0.001)
    r2 = oracle.concave_filter(sdf, obj.pts, obj.nrm, 0.008, 4, 0.001)
    assert (r2["depth"] >= r1["depth"] - 1e-15).all()
    kept = r2["keep"].mean()
    assert 0.5 < kept < 1.0, kept
    # a dropped point's box sinks deeper than the threshold
    assert (r2["depth"][r2["keep"] == 0] > 0.001).all()

"""Pins of the oracle's FP64 Siddon projector to things other than itself.

Each check is chosen so that a plausible mistake in ``oracle/siddon.c`` (a
wrong plane list, a dropped segment, a transposed index, a wrong sign in the
geometry, a scatter to the wrong voxel) fails at least one of them:
  * hand-derived segments of single rays (tests/golden/siddon_rays.json);
  * brute-force dense A by per-voxel slab clipping on tiny grids;
  * closed-form chords through the whole box and through a voxel-aligned box;
  * chords through a voxelised ball converge at first order in the voxel size;
  * the FP64 adjoint identity <A x, y> = <x, A^T y>;
  * the 90-degree rotation symmetry of a centred square grid;
  * a single voxel projects only inside its perspective footprint.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "siddon_rays.json")


def _tiny_geoms():
    return [
        oracle.Geometry(nx=5, ny=4, nz=3, vx=1.0, vy=1.2, vz=0.9, nu=8, nv=6, du=1.3, dv=1.1,
                        dso=20.0, dsd=35.0, angles=tuple(synth.angles(7)), ox=0.3, oy=-0.2, oz=0.1),
        oracle.Geometry(nx=6, ny=6, nz=4, vx=0.5, vy=0.5, vz=0.5, nu=9, nv=5, du=0.45, dv=0.5,
                        dso=10.0, dsd=16.0, angles=tuple(synth.angles(5, span=math.pi, start=0.3))),
        oracle.Geometry(nx=3, ny=7, nz=2, vx=2.0, vy=1.0, vz=1.5, nu=4, nv=4, du=3.0, dv=2.0,
                        dso=30.0, dsd=45.0, angles=(0.0, math.pi / 2, math.pi, 1.234)),
    ]


def test_golden_rays():
    with open(GOLDEN) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        g = oracle.Geometry.from_dict(c["geom"])
        idx, ln = oracle.ray_segments(g, c["ray"]["a"], c["ray"]["iv"], c["ray"]["iu"])
        want_idx = [s[0] for s in c["segments"]]
        want_len = [eval(s[1], {"sqrt": math.sqrt}) for s in c["segments"]]
        assert list(idx) == want_idx, c["name"]
        np.testing.assert_allclose(ln, want_len, rtol=1e-13, atol=1e-13, err_msg=c["name"])


@pytest.mark.parametrize("gi", range(3))
def test_brute_force_dense(gi):
    g = _tiny_geoms()[gi]
    A = dense.system_matrix(g)
    rng = np.random.default_rng(gi)
    x = rng.standard_normal(g.vol_shape)
    y = rng.standard_normal(g.proj_shape)
    yf = oracle.forward(g, x).ravel()
    xa = oracle.adjoint(g, y).ravel()
    np.testing.assert_allclose(yf, A @ x.ravel(), rtol=0, atol=1e-12 * np.abs(A).sum(1).max())
    np.testing.assert_allclose(xa, A.T @ y.ravel(), rtol=0, atol=1e-12 * np.abs(A).sum(0).max())
    assert (A > 0).sum() > 0.05 * A.size  # the geometry really exercises the traversal
    # Column sums: A^T 1 equals the dense column sums.
    np.testing.assert_allclose(oracle.adjoint(g, np.ones(g.proj_shape)).ravel(), A.sum(0), rtol=1e-12)


def test_box_chords():
    g = oracle.Geometry.from_dict(synth.geometry("cgls32"))
    y = oracle.forward(g, np.ones(g.vol_shape))
    np.testing.assert_allclose(y, dense.box_chords(g), rtol=1e-12, atol=1e-12)
    assert np.mean(y > 0) > 0.3


def test_subbox_chords():
    g = oracle.Geometry(nx=16, ny=16, nz=12, vx=0.7, vy=0.7, vz=0.8, nu=40, nv=30, du=0.6, dv=0.6,
                        dso=50.0, dsd=80.0, angles=tuple(synth.angles(9, start=0.1)), oz=0.4)
    x = np.zeros(g.vol_shape)
    i0, i1, j0, j1, k0, k1 = 3, 11, 5, 14, 2, 7
    x[k0:k1, j0:j1, i0:i1] = 1.0
    X0, Y0, Z0 = -8 * 0.7, -8 * 0.7, 0.4 - 6 * 0.8
    lo = (X0 + i0 * 0.7, Y0 + j0 * 0.7, Z0 + k0 * 0.8)
    hi = (X0 + i1 * 0.7, Y0 + j1 * 0.7, Z0 + k1 * 0.8)
    np.testing.assert_allclose(oracle.forward(g, x), dense.box_chords(g, lo, hi), rtol=1e-12, atol=1e-12)


def test_sphere_chords_converge():
    """Voxelised ball (voxel centres inside radius R): chord error is O(h)."""
    R = 6.0
    errs = []
    for n in (16, 32, 64):
        h = 16.0 / n
        g = oracle.Geometry(nx=n, ny=n, nz=n, vx=h, vy=h, vz=h, nu=24, nv=24, du=0.9, dv=0.9,
                            dso=60.0, dsd=100.0, angles=(0.2, 1.1, 2.5))
        c = (np.arange(n) + 0.5) * h - 8.0
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        x = ((X ** 2 + Y ** 2 + Z ** 2) <= R * R).astype(np.float64)
        ref = dense.sphere_chords(g, (0.0, 0.0, 0.0), R)
        errs.append(float(np.mean(np.abs(oracle.forward(g, x) - ref))))
    # mean |error| below half a voxel, halving with h (first order)
    assert errs[0] < 0.5 * 1.0 and errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1], errs


def test_adjoint_identity_fp64():
    g = oracle.Geometry.from_dict(synth.geometry("cgls32"))
    rng = np.random.default_rng(3)
    x = rng.standard_normal(g.vol_shape)
    y = rng.standard_normal(g.proj_shape)
    Ax = oracle.forward(g, x)
    ATy = oracle.adjoint(g, y)
    lhs = float(np.dot(Ax.ravel(), y.ravel()))
    rhs = float(np.dot(x.ravel(), ATy.ravel()))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_rotation_90_symmetry():
    """Rotating the object by +90 deg about z and the gantry by +90 deg leaves
    the projections unchanged (centred square grid)."""
    n = 12
    base = oracle.Geometry(nx=n, ny=n, nz=6, vx=1.0, vy=1.0, vz=1.0, nu=20, nv=10, du=1.1, dv=1.1,
                           dso=40.0, dsd=70.0, angles=(0.3, 1.9))
    rot = base.with_angles(tuple(a + math.pi / 2 for a in base.angles))
    x = np.random.default_rng(5).standard_normal(base.vol_shape)
    # R90 maps (x, y) -> (-y, x); the rotated object at voxel (i', j') takes the
    # value of the original at the voxel rotated back: i = j', j = n-1-i'.
    xr = np.empty_like(x)
    for jp in range(n):
        for ip in range(n):
            xr[:, jp, ip] = x[:, n - 1 - ip, jp]
    np.testing.assert_allclose(oracle.forward(rot, xr), oracle.forward(base, x), rtol=1e-11, atol=1e-11)


def test_single_voxel_footprint():
    g = oracle.Geometry(nx=8, ny=8, nz=8, vx=1.0, vy=1.0, vz=1.0, nu=32, nv=32, du=0.8, dv=0.8,
                        dso=30.0, dsd=50.0, angles=tuple(synth.angles(6)))
    i, j, k = 5, 2, 6
    x = np.zeros(g.vol_shape)
    x[k, j, i] = 1.0
    y = oracle.forward(g, x)
    lo = np.array([-4 + i, -4 + j, -4 + k], dtype=float)
    corners = np.array([[lo[0] + a, lo[1] + b, lo[2] + c] for a in (0, 1) for b in (0, 1) for c in (0, 1)])
    for a, th in enumerate(g.angles):
        ct, st = math.cos(th), math.sin(th)
        depth = g.dso - (corners[:, 0] * ct + corners[:, 1] * st)
        lat = -corners[:, 0] * st + corners[:, 1] * ct
        us = g.dsd * lat / depth
        vs = g.dsd * corners[:, 2] / depth
        u = (np.arange(g.nu) - (g.nu - 1) / 2) * g.du
        v = (np.arange(g.nv) - (g.nv - 1) / 2) * g.dv
        inside = (v[:, None] >= vs.min() - 1e-9) & (v[:, None] <= vs.max() + 1e-9) & \
                 (u[None, :] >= us.min() - 1e-9) & (u[None, :] <= us.max() + 1e-9)
        assert np.all(y[a][~inside] == 0.0)
        assert y[a][inside].sum() > 0.0


def test_forward_rays_subset():
    g = oracle.Geometry.from_dict(synth.geometry("cgls32"))
    x = synth.random_volume(g.vol_shape, 11).astype(np.float64)
    full = oracle.forward(g, x).ravel()
    rays = np.random.default_rng(2).choice(full.size, 500, replace=False)
    np.testing.assert_array_equal(oracle.forward_rays(g, x, rays), full[rays])


def test_count_nnz_matches_dense():
    for g in _tiny_geoms():
        A = dense.system_matrix(g)
        nnz, hits = oracle.count_nnz(g)
        # Segments of positive length == positive entries of the brute-force A
        # (grazing segments of ~1e-15 mm included on both sides).
        assert nnz == int((A > 0).sum())
        assert hits == int((A.sum(1) > 0).sum())


def test_block_locality():
    """A line integral only sums the voxels the ray crosses: with the volume
    zero outside a block, every ray's value equals its integral through a grid
    that is just that block (voxel origin moved by the volume offset), and
    the adjoint restricted to the block equals the block grid's adjoint."""
    gd = synth.geometry(dict(nx=24, ny=20, nz=18, vx=0.9, vy=1.1, vz=1.0, nu=40, nv=36, du=1.2, dv=1.1,
                             dso=300.0, dsd=450.0, n_angles=7, ox=0.8, oy=-1.3, oz=0.4))
    origin, shape = (3, 11, 5), (9, 6, 13)
    g = oracle.Geometry.from_dict(gd)
    gb = oracle.Geometry.from_dict(synth.block_geometry(gd, origin, shape))
    xb = synth.random_volume(shape, 7)
    x = np.zeros(g.vol_shape)
    sl = tuple(slice(o, o + s) for o, s in zip(origin, shape))
    x[sl] = xb
    y_full, y_block = oracle.forward(g, x), oracle.forward(gb, xb)
    assert np.count_nonzero(y_block) > 200
    np.testing.assert_allclose(y_block, y_full, rtol=0, atol=1e-12 * np.abs(y_full).max())
    yr = synth.random_projections(g.proj_shape, 8)
    a_full, a_block = oracle.adjoint(g, yr)[sl], oracle.adjoint(gb, yr)
    np.testing.assert_allclose(a_block, a_full, rtol=0, atol=1e-12 * np.abs(a_full).max())

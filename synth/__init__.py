"""Seeded synthetic inputs for the Krylov CBCT path.

This package is the only code that both the GPU library's harness and the
oracle use.  It holds none of the method's arithmetic (no projection, no
solver step): only workload descriptions, phantoms sampled at voxel
centres, the measurement-noise model applied to given clean projections,
and random test vectors.  Everything is drawn from NumPy's PCG64 with an
explicit seed.

Workloads (shapes, sizes and value ranges of the paper's experiments,
Sec. 3; the paper's datasets are not available, so seeded phantoms stand
in for them):
  cgls32      32^3 at 1 mm, 10 ellipsoids, 64x64 detector at 1 mm, 36 angles,
              Gaussian noise 1 % of max; CGLS 20 iterations.  Stands in for the
              64^3 synthetic head of Sec. 3.1 at a size the oracle solves fast.
  medical256  256^3 at 0.5 mm, 40 ellipsoids, 512x512 at 0.4 mm, 360 angles,
              Poisson noise I0 = 1e5; CGLS, LSQR, LSMR 30 iterations.  Stands in
              for the Alderson head scan of Sec. 3.2 (512^2 projections,
              256x256x200 volume).
  torso512    512^3 at 0.5 mm torso (shell, 60 ellipsoids, 5 dense inserts),
              1024x768 at 0.4 mm, 720 angles; damped and hybrid LSQR, lam = 10,
              50 iterations, 16-bit storage variants.
  muct1500    1500^3 at 10 um porous cylinder (2000 spherical pores, Gaussian
              blur sigma = 1 voxel), DSO 150, DSD 800, 2000^2 at 0.1 mm, 1571
              angles; IRN-TV 10 outer x 20 inner.  Stands in for the bumblebee
              uCT scan of Sec. 3.3.  Generated per crop, never whole, in tests.
  serve       64 requests with Poisson arrivals at 2 req/s, mixed sizes,
              angle counts, detectors and solvers.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["angles", "workload", "geometry", "crop_geometry", "ellipsoid_phantom", "torso_phantom",
           "porous_phantom", "porous_phantom_torch", "phantom", "add_noise", "add_noise_torch", "random_volume", "random_projections",
           "serve_stream", "block_geometry", "WORKLOADS"]


def angles(n: int, span: float = 2.0 * math.pi, start: float = 0.0) -> np.ndarray:
    """n equidistant angles over ``span`` radians, endpoint excluded (FP64)."""
    return start + span * np.arange(n, dtype=np.float64) / n


WORKLOADS = {
    "cgls32": dict(
        geom=dict(nx=32, ny=32, nz=32, vx=1.0, vy=1.0, vz=1.0, nu=64, nv=64, du=1.0, dv=1.0,
                  dso=1000.0, dsd=1500.0, n_angles=36),
        phantom=dict(kind="ellipsoids", n=10, axes_mm=(2.0, 12.0), atten=(0.1, 1.0)),
        noise=dict(kind="gaussian", rel_sigma=0.01),
        solve=dict(solvers=("cgls",), n_iter=20, lam=0.0),
        seed=1),
    "medical256": dict(
        geom=dict(nx=256, ny=256, nz=256, vx=0.5, vy=0.5, vz=0.5, nu=512, nv=512, du=0.4, dv=0.4,
                  dso=1000.0, dsd=1500.0, n_angles=360),
        phantom=dict(kind="ellipsoids", n=40, axes_mm=(2.0, 12.0), atten=(0.1, 1.0)),
        noise=dict(kind="poisson", i0=1.0e5, length_unit_mm=10.0),
        solve=dict(solvers=("cgls", "lsqr", "lsmr"), n_iter=30, lam=0.0),
        seed=2),
    "torso512": dict(
        geom=dict(nx=512, ny=512, nz=512, vx=0.5, vy=0.5, vz=0.5, nu=1024, nv=768, du=0.4, dv=0.4,
                  dso=1000.0, dsd=1500.0, n_angles=720),
        phantom=dict(kind="torso", n=60, atten=(0.15, 0.5), shell=0.2, n_inserts=5, insert=2.0),
        noise=dict(kind="poisson", i0=1.0e5, length_unit_mm=10.0),
        solve=dict(solvers=("lsqr", "hybrid_lsqr"), n_iter=50, lam=10.0),
        seed=3),
    "muct1500": dict(
        geom=dict(nx=1500, ny=1500, nz=1500, vx=0.01, vy=0.01, vz=0.01, nu=2000, nv=2000, du=0.1, dv=0.1,
                  dso=150.0, dsd=800.0, n_angles=1571),
        phantom=dict(kind="porous", n=2000, radius_vox=(5.0, 40.0), cyl_frac=0.45, blur_sigma=1.0),
        noise=dict(kind="poisson", i0=1.0e5, length_unit_mm=10.0),
        solve=dict(solvers=("irn_tv_cgls",), n_outer=10, n_inner=20, lam=10.0, eps=1.0e-3),
        seed=4),
}


def geometry(name_or_geom) -> dict:
    """Plain geometry dict (with an ``angles`` FP64 array) for a workload name or dict."""
    g = dict(WORKLOADS[name_or_geom]["geom"]) if isinstance(name_or_geom, str) else dict(name_or_geom)
    n = g.pop("n_angles", None)
    if "angles" not in g:
        g["angles"] = angles(n)
    g.setdefault("ox", 0.0)
    g.setdefault("oy", 0.0)
    g.setdefault("oz", 0.0)
    return g


def crop_geometry(name: str, n_vox: int, n_det: int, n_angles: int) -> dict:
    """A workload's magnification, voxel and pixel size on a smaller grid.

    The volume becomes n_vox^3 voxels and the detector n_det^2 pixels; the
    distances, voxel size and pixel pitch are kept.
    """
    g = dict(WORKLOADS[name]["geom"])
    g.update(nx=n_vox, ny=n_vox, nz=n_vox, nu=n_det, nv=n_det, n_angles=n_angles)
    return geometry(g)


def block_geometry(g: dict, origin, shape) -> dict:
    """The sub-grid of geometry ``g`` that starts at voxel ``origin`` (k, j, i)
    and has ``shape`` (nz, ny, nx): same voxel size, same place in space, same
    source, detector and angles."""
    (k0, j0, i0), (bz, by, bx) = origin, shape
    b = dict(g)
    b.update(nx=bx, ny=by, nz=bz,
             ox=g["ox"] + (i0 + bx / 2 - g["nx"] / 2) * g["vx"],
             oy=g["oy"] + (j0 + by / 2 - g["ny"] / 2) * g["vy"],
             oz=g["oz"] + (k0 + bz / 2 - g["nz"] / 2) * g["vz"])
    return b


def _haar_rotation(rng) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _voxel_centres(g: dict, axis: str) -> np.ndarray:
    n, v, o = g["n" + axis], g["v" + axis], g["o" + axis]
    return o - 0.5 * n * v + (np.arange(n) + 0.5) * v


def _add_ellipsoid(vol, g, centre, axes, rot, value, mode="add"):
    xc, yc, zc = _voxel_centres(g, "x"), _voxel_centres(g, "y"), _voxel_centres(g, "z")
    r = float(np.max(axes))
    sel = []
    for cen, c, vs in ((xc, centre[0], g["vx"]), (yc, centre[1], g["vy"]), (zc, centre[2], g["vz"])):
        lo = np.searchsorted(cen, c - r - vs)
        hi = np.searchsorted(cen, c + r + vs)
        sel.append((lo, hi))
    (i0, i1), (j0, j1), (k0, k1) = sel
    if i0 >= i1 or j0 >= j1 or k0 >= k1:
        return
    Z, Y, X = np.meshgrid(zc[k0:k1] - centre[2], yc[j0:j1] - centre[1], xc[i0:i1] - centre[0], indexing="ij")
    P = np.stack([X, Y, Z], axis=-1) @ rot  # body-frame coordinates
    inside = np.sum((P / np.asarray(axes)) ** 2, axis=-1) <= 1.0
    sub = vol[k0:k1, j0:j1, i0:i1]
    if mode == "add":
        sub[inside] += value
    else:
        sub[inside] = value


def ellipsoid_phantom(g: dict, n: int, axes_mm, atten, seed: int) -> np.ndarray:
    """Sum of n random ellipsoids sampled at voxel centres (FP32, zero outside).

    Centres uniform in the inner 70 % of the volume box, semi-axes uniform in
    ``axes_mm``, Haar-random orientations, attenuation uniform in ``atten``
    (mm^-1), values added where ellipsoids overlap.
    """
    rng = np.random.default_rng(seed)
    vol = np.zeros((g["nz"], g["ny"], g["nx"]), dtype=np.float64)
    half = np.array([g["nx"] * g["vx"], g["ny"] * g["vy"], g["nz"] * g["vz"]]) / 2
    off = np.array([g["ox"], g["oy"], g["oz"]])
    for _ in range(n):
        c = off + rng.uniform(-0.7, 0.7, 3) * half
        ax = rng.uniform(axes_mm[0], axes_mm[1], 3)
        R = _haar_rotation(rng)
        val = rng.uniform(atten[0], atten[1])
        _add_ellipsoid(vol, g, c, ax, R, val)
    return vol.astype(np.float32)


def torso_phantom(g: dict, n: int, atten, shell: float, n_inserts: int, insert: float, seed: int) -> np.ndarray:
    """A torso-like ellipsoid: outer body of value ``shell``, n inner ellipsoids
    with attenuation uniform in ``atten`` added inside, and ``n_inserts`` dense
    spheres set to ``insert``.  FP32, zero outside the body."""
    rng = np.random.default_rng(seed)
    vol = np.zeros((g["nz"], g["ny"], g["nx"]), dtype=np.float64)
    L = np.array([g["nx"] * g["vx"], g["ny"] * g["vy"], g["nz"] * g["vz"]])
    off = np.array([g["ox"], g["oy"], g["oz"]])
    body = np.array([0.45, 0.32, 0.48]) * L
    _add_ellipsoid(vol, g, off, body, np.eye(3), shell)
    for _ in range(n):
        c = off + rng.uniform(-0.6, 0.6, 3) * body
        ax = rng.uniform(0.03, 0.15, 3) * L
        _add_ellipsoid(vol, g, c, ax, _haar_rotation(rng), rng.uniform(atten[0], atten[1]))
    for _ in range(n_inserts):
        c = off + rng.uniform(-0.6, 0.6, 3) * body
        r = rng.uniform(0.006, 0.016) * L[0]
        _add_ellipsoid(vol, g, c, (r, r, r), np.eye(3), insert, mode="set")
    return vol.astype(np.float32)


def porous_phantom(g: dict, n: int, radius_vox, cyl_frac: float, blur_sigma: float, seed: int,
                   full_n: int | None = None, crop_origin=(0, 0, 0)) -> np.ndarray:
    """Binary porous cylinder, Gaussian-blurred; optionally one crop of it.

    The full object is a cylinder (axis z, radius cyl_frac * side) of value 1
    on a ``full_n``^3 grid, minus n spherical pores with radii uniform in
    ``radius_vox`` voxels and centres uniform inside the cylinder; then a
    Gaussian blur of ``blur_sigma`` voxels.  The crop of shape (nz, ny, nx)
    starting at voxel ``crop_origin`` (k, j, i) of the full grid is returned,
    so a crop is identical to the same block of the full phantom.
    """
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    full_n = full_n or g["nx"]
    R = cyl_frac * full_n
    c0 = full_n / 2.0
    pores = _pores(rng, n, radius_vox, R, c0, full_n)
    pad = int(math.ceil(4 * blur_sigma)) + 1
    k0, j0, i0 = crop_origin
    shape = (g["nz"] + 2 * pad, g["ny"] + 2 * pad, g["nx"] + 2 * pad)
    kk = np.arange(shape[0]) + k0 - pad + 0.5
    jj = np.arange(shape[1]) + j0 - pad + 0.5
    ii = np.arange(shape[2]) + i0 - pad + 0.5
    vol = np.zeros(shape, dtype=np.float32)
    cyl = (ii[None, :] - c0) ** 2 + (jj[:, None] - c0) ** 2 <= R * R
    inz = (kk >= 0) & (kk < full_n)
    vol[inz] = cyl[None].astype(np.float32)
    for p, r in pores:
        lo = [int(max(0, math.floor(p[a] - r - (k0, j0, i0)[2 - a] + pad))) for a in range(3)]
        hi = [int(min(shape[2 - a], math.ceil(p[a] + r - (k0, j0, i0)[2 - a] + pad + 1))) for a in range(3)]
        if lo[0] >= hi[0] or lo[1] >= hi[1] or lo[2] >= hi[2]:
            continue
        Z, Y, X = np.meshgrid(kk[lo[2]:hi[2]], jj[lo[1]:hi[1]], ii[lo[0]:hi[0]], indexing="ij")
        hole = (X - p[0]) ** 2 + (Y - p[1]) ** 2 + (Z - p[2]) ** 2 <= r * r
        vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]][hole] = 0.0
    if blur_sigma > 0:
        vol = gaussian_filter(vol, blur_sigma, mode="constant")
    return np.ascontiguousarray(vol[pad:-pad, pad:-pad, pad:-pad]).astype(np.float32)


def _pores(rng, n, radius_vox, R, c0, full_n):
    pores = []
    while len(pores) < n:
        p = rng.uniform(0, full_n, 3)
        if (p[0] - c0) ** 2 + (p[1] - c0) ** 2 <= R * R:
            pores.append((p, rng.uniform(radius_vox[0], radius_vox[1])))
    return pores


def porous_phantom_torch(g: dict, n: int, radius_vox, cyl_frac: float, blur_sigma: float, seed: int, device):
    """``porous_phantom`` of the whole grid, built with torch on ``device``
    (the 1500^3 volume takes minutes on the host).  Same pores (the same PCG64
    draws), cylinder and blur: a truncated Gaussian of radius int(4 sigma + 0.5)
    voxels, normalised, applied along each axis in turn with zeros outside the
    grid, summed in FP64 as c0 x_i + sum_t c_t (x_{i+t} + x_{i-t}).  Equals
    the host version to FP32 rounding; FP32 result on ``device``."""
    import torch

    rng = np.random.default_rng(seed)
    nz, ny, nx = g["nz"], g["ny"], g["nx"]
    full_n = nx
    R = cyl_frac * full_n
    c0 = full_n / 2.0
    pores = _pores(rng, n, radius_vox, R, c0, full_n)
    ii = torch.arange(nx, device=device, dtype=torch.float64) + 0.5
    jj = torch.arange(ny, device=device, dtype=torch.float64) + 0.5
    kk = torch.arange(nz, device=device, dtype=torch.float64) + 0.5
    cyl = ((ii[None, :] - c0) ** 2 + (jj[:, None] - c0) ** 2 <= R * R).to(torch.float32)
    vol = cyl[None].expand(nz, ny, nx).contiguous()
    for p, r in pores:
        lo = [int(max(0, math.floor(p[a] - r))) for a in range(3)]
        hi = [int(min((nx, ny, nz)[a], math.ceil(p[a] + r + 1))) for a in range(3)]
        if lo[0] >= hi[0] or lo[1] >= hi[1] or lo[2] >= hi[2]:
            continue
        Z, Y, X = torch.meshgrid(kk[lo[2]:hi[2]], jj[lo[1]:hi[1]], ii[lo[0]:hi[0]], indexing="ij")
        hole = (X - p[0]) ** 2 + (Y - p[1]) ** 2 + (Z - p[2]) ** 2 <= r * r
        vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].masked_fill_(hole, 0.0)
    if blur_sigma > 0:
        rad = int(4.0 * blur_sigma + 0.5)
        t = np.arange(-rad, rad + 1, dtype=np.float64)
        w = np.exp(-0.5 * (t / blur_sigma) ** 2)
        w /= w.sum()
        for axis in range(3):
            out = torch.empty_like(vol)
            for k0 in range(0, nz, 64):  # FP64 sums, a z-slab at a time
                k1 = min(nz, k0 + 64)
                if axis == 0:
                    src = vol[max(0, k0 - rad):min(nz, k1 + rad)].double()
                    off = k0 - max(0, k0 - rad)
                else:
                    src = vol[k0:k1].double()
                    off = 0
                dim = 0 if axis == 0 else axis
                n_ax = src.shape[dim]
                m = k1 - k0 if axis == 0 else n_ax
                acc = w[rad] * src.narrow(dim, off, m)
                for s in range(1, rad + 1):
                    # x_{i+s} + x_{i-s}, zero outside the grid
                    up = torch.zeros_like(acc)
                    dn = torch.zeros_like(acc)
                    a0, a1 = max(0, off + s), min(n_ax, off + m + s)
                    if a1 > a0:
                        up.narrow(dim, a0 - off - s, a1 - a0).copy_(src.narrow(dim, a0, a1 - a0))
                    b0, b1 = max(0, off - s), min(n_ax, off + m - s)
                    if b1 > b0:
                        dn.narrow(dim, b0 - off + s, b1 - b0).copy_(src.narrow(dim, b0, b1 - b0))
                    acc += w[rad + s] * (up + dn)
                out[k0:k1] = acc.float()
                del src, acc
            vol = out
    return vol


def phantom(name: str, g: dict | None = None, **overrides) -> np.ndarray:
    """The workload's phantom on geometry ``g`` (default: the workload's own)."""
    w = WORKLOADS[name]
    g = g or geometry(name)
    spec = dict(w["phantom"])
    spec.update(overrides)
    seed = spec.pop("seed", w["seed"])
    kind = spec.pop("kind")
    if kind == "ellipsoids":
        return ellipsoid_phantom(g, spec["n"], spec["axes_mm"], spec["atten"], seed)
    if kind == "torso":
        return torso_phantom(g, spec["n"], spec["atten"], spec["shell"], spec["n_inserts"], spec["insert"], seed)
    if kind == "porous":
        return porous_phantom(g, spec["n"], spec["radius_vox"], spec["cyl_frac"], spec["blur_sigma"], seed,
                              full_n=spec.get("full_n"), crop_origin=spec.get("crop_origin", (0, 0, 0)))
    raise ValueError(kind)


def add_noise(b_clean, spec: dict, seed: int) -> tuple[np.ndarray, dict]:
    """Apply the measurement-noise model to clean line integrals; FP32 result.

    ``gaussian``: b + N(0, (rel_sigma * max b)^2).
    ``poisson``: counts I = max(Poisson(I0 exp(-b / L)), 1), then
    b = L ln(I0 / I) (the Beer-Lambert transform; zero counts are clamped to
    one).  L = ``length_unit_mm`` (default 1) is the length, in mm, that the
    phantom's attenuation values are per: the workloads give them in 1/cm,
    the usual unit (water is about 0.2/cm), so L = 10 with lengths in mm.
    Returns the noisy data and a dict with the clamped fraction.
    """
    rng = np.random.default_rng(seed + 1000)
    b = np.asarray(b_clean, dtype=np.float64)
    info = {}
    if spec["kind"] == "gaussian":
        out = b + rng.normal(0.0, spec["rel_sigma"] * float(np.max(np.abs(b))), b.shape)
    elif spec["kind"] == "poisson":
        i0, L = float(spec["i0"]), float(spec.get("length_unit_mm", 1.0))
        counts = rng.poisson(i0 * np.exp(-b / L)).astype(np.float64)
        info["clamped_fraction"] = float(np.mean(counts < 1.0))
        out = L * np.log(i0 / np.maximum(counts, 1.0))
    elif spec["kind"] == "none":
        out = b
    else:
        raise ValueError(spec["kind"])
    return out.astype(np.float32), info


def add_noise_torch(b_clean, spec: dict, seed: int):
    """``add_noise`` for a torch tensor, drawn on the tensor's device (for
    projections too large to round-trip through host memory).  Same model,
    different random stream (torch's generator).  Tensors of more than 2^28
    elements are drawn in blocks of whole leading-axis slices (angles), block
    by block from one generator, so that no single draw exceeds 2^28
    elements."""
    import torch

    gen = torch.Generator(device=b_clean.device).manual_seed(seed + 1000)
    info = {}
    if spec["kind"] == "none":
        return b_clean.float().contiguous(), info
    if spec["kind"] not in ("gaussian", "poisson"):
        raise ValueError(spec["kind"])
    out = torch.empty(b_clean.shape, dtype=torch.float32, device=b_clean.device)
    per = max(1, b_clean[0].numel()) if b_clean.dim() > 0 else 1
    step = max(1, (1 << 28) // per) if b_clean.dim() > 0 else 1
    n_lead = b_clean.shape[0] if b_clean.dim() > 0 else 1
    sig = spec.get("rel_sigma", 0.0) * float(b_clean.abs().max()) if spec["kind"] == "gaussian" else 0.0
    clamped = 0
    for a0 in range(0, n_lead, step):
        blk = b_clean[a0:a0 + step] if b_clean.dim() > 0 else b_clean
        dst = out[a0:a0 + step] if b_clean.dim() > 0 else out
        if spec["kind"] == "gaussian":
            dst.copy_(blk + sig * torch.randn(blk.shape, generator=gen, device=blk.device))
        else:
            i0, L = float(spec["i0"]), float(spec.get("length_unit_mm", 1.0))
            counts = torch.poisson(i0 * torch.exp(-blk.double() / L), generator=gen)
            clamped += int((counts < 1.0).sum())
            dst.copy_(L * torch.log(i0 / counts.clamp_(min=1.0)))
            del counts
    if spec["kind"] == "poisson":
        info["clamped_fraction"] = clamped / max(1, b_clean.numel())
    return out, info


def random_volume(shape, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Uniform random FP32 volume (parity inputs)."""
    return np.random.default_rng(seed).uniform(lo, hi, shape).astype(np.float32)


def random_projections(shape, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Uniform random FP32 projections (parity inputs)."""
    return np.random.default_rng(seed + 7).uniform(lo, hi, shape).astype(np.float32)


def serve_stream(n_requests: int = 64, rate: float = 2.0, seed: int = 5,
                 sizes=(128, 256, 384, 512), angle_counts=(90, 180, 360, 720),
                 det_range=(256, 1024), solvers=("cgls", "lsqr", "lsmr"), iters=(20, 50)):
    """Seeded request stream: arrival times (s) and per-request workloads.

    Exponential inter-arrival times of mean 1/rate; each request draws a cube
    size at 0.5 mm, an angle count, an even square detector side whose pitch
    makes the field of view 1.1x the volume's width at the isocentre, a
    solver and an iteration count.  DSO 1000 mm, DSD 1500 mm.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    reqs = []
    for r in range(n_requests):
        n = int(rng.choice(sizes))
        na = int(rng.choice(angle_counts))
        side = int(rng.integers(det_range[0] // 2, det_range[1] // 2 + 1)) * 2
        pitch = 1.1 * n * 0.5 * (1500.0 / 1000.0) / side
        geom = dict(nx=n, ny=n, nz=n, vx=0.5, vy=0.5, vz=0.5, nu=side, nv=side, du=pitch, dv=pitch,
                    dso=1000.0, dsd=1500.0, n_angles=na)
        reqs.append(dict(id=r, arrival=float(t[r]), geom=geom, solver=str(rng.choice(solvers)),
                         n_iter=int(rng.integers(iters[0], iters[1] + 1)),
                         n_ellipsoids=int(rng.integers(10, 41)), seed=10_000 + r))
    return reqs

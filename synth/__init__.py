"""Seeded synthetic inputs for the filtering workloads.

This module produces *inputs only* -- texels, sparse-grid leaves and query
positions -- with numpy's own seeded generator.  It holds none of the
filtering method's arithmetic (no filter weights, no tap selection, no
random draws of the method), and it is the only code that the GPU path and the
CPU oracle both consume.

Workloads (sizes are the defaults; tests pass smaller ones):
  texture2d    W x H x C texels, i.i.d. uniform [0, 1), with uniform uv
               queries in [0, 1)^2.
  fbm_grid     a sparse 3D voxel grid: 5-octave value-noise fBm (lacunarity 2,
               gain 0.5) thresholded at 0.55; density = max(noise - 0.55, 0);
               an 8^3 leaf is stored iff one of its voxels has density > 0.
  ray_queries  query positions along random rays through the grid's bounds:
               uniform origin in the box, uniform direction, clipped to the
               box, n_samples stratified-jittered samples per ray, ray-major.
"""
from __future__ import annotations

import numpy as np
import torch

# ----------------------------------------------------------------------------
# storage-format conversion of generated values (input preparation)
# ----------------------------------------------------------------------------


def to_f16(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, np.float32).astype(np.float16)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """binary32 -> bfloat16 bit patterns, round to nearest even (no NaNs in
    generated data)."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    rounded = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def to_e4m3_bits(x: np.ndarray) -> np.ndarray:
    """binary32 -> OCP E4M3 ("FN") bit patterns, round to nearest even,
    saturating at +-448.  Exhaustive: picks the nearest of the 254 finite
    codes (ties to the even mantissa)."""
    x = np.asarray(x, np.float32).ravel()
    codes = np.arange(256, dtype=np.uint8)
    s = (codes >> 7) & 1
    e = (codes >> 3) & 15
    m = codes & 7
    val = np.where(e == 0, m.astype(np.float64) * 2.0 ** -9,
                   (8 + m).astype(np.float64) * np.exp2(e.astype(np.float64) - 10))
    val = np.where(s == 1, -val, val)
    finite = ~((e == 15) & (m == 7))
    pos = codes[(s == 0) & finite]
    pos_val = val[(s == 0) & finite]
    order = np.argsort(pos_val)
    pos, pos_val = pos[order], pos_val[order]
    a = np.minimum(np.abs(x.astype(np.float64)), 448.0)
    k = np.searchsorted(pos_val, a)          # pos_val[k-1] < a <= pos_val[k]
    k = np.clip(k, 1, len(pos_val) - 1)
    lo, hi = pos_val[k - 1], pos_val[k]
    pick_hi = (a - lo > hi - a) | ((a - lo == hi - a) & ((pos[k] & 1) == 0))
    pick_hi |= a == hi
    code = np.where(pick_hi, pos[k], pos[k - 1]).astype(np.uint8)
    code = np.where(a == 0.0, np.uint8(0), code)
    neg = np.signbit(x) & (code != 0)
    code = np.where(neg, code | np.uint8(0x80), code)
    return code.astype(np.uint8)


def to_u8(x: np.ndarray) -> np.ndarray:
    """[0,1] -> UNORM8 (round to nearest)."""
    return np.clip(np.rint(np.asarray(x, np.float64) * 255.0), 0, 255).astype(np.uint8)


FORMAT_NAMES = ("f32", "f16", "bf16", "fp8_e4m3", "u8")


def encode(x: np.ndarray, fmt: str) -> np.ndarray:
    if fmt == "f32":
        return np.asarray(x, np.float32)
    if fmt == "f16":
        return to_f16(x).view(np.uint16)
    if fmt == "bf16":
        return to_bf16_bits(x).reshape(np.shape(x))
    if fmt == "fp8_e4m3":
        return to_e4m3_bits(x).reshape(np.shape(x))
    if fmt == "u8":
        return to_u8(x)
    raise ValueError(fmt)


# ----------------------------------------------------------------------------
# 2D texture workload
# ----------------------------------------------------------------------------
def texture2d(width: int = 256, height: int = 256, channels: int = 4, seed: int = 1) -> np.ndarray:
    """(H, W, C) float32 texels i.i.d. uniform in [0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.random((height, width, channels), dtype=np.float32)


def uv_queries(n: int = 65536, seed: int = 2) -> np.ndarray:
    """(n, 2) float32 texture coordinates uniform in [0, 1)^2."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 2), dtype=np.float32)


def screen_uv_queries(width: int = 3840, height: int = 2160, seed: int = 53) -> np.ndarray:
    """(width * height, 2) float32 texture coordinates of a frame, pixel-major
    (row by row): a pinhole camera (60-degree horizontal field of view) 2
    units above a ground plane, looking 25 degrees down; the plane carries the
    texture tiled every 8 units (so the texel density runs from magnified in
    the foreground to minified towards the horizon).  Pixels whose ray misses
    the plane (above the horizon) look at the sky and are given a random uv
    (a query stream has no holes).  A per-frame jitter of the pixel centres
    comes from the seed."""
    rng = np.random.default_rng(seed)
    jx, jy = rng.random(2)
    px = (np.arange(width) + jx) / width * 2.0 - 1.0
    py = 1.0 - (np.arange(height) + jy) / height * 2.0
    tan_h = np.tan(np.radians(30.0))
    X, Y = np.meshgrid(px * tan_h, py * tan_h * height / width)
    pitch = np.radians(25.0)
    # camera frame: forward f, right r, up u (world z up)
    f = np.array([0.0, np.cos(pitch), -np.sin(pitch)])
    u = np.array([0.0, np.sin(pitch), np.cos(pitch)])
    d = f[None, None, :] + X[:, :, None] * np.array([1.0, 0.0, 0.0]) + Y[:, :, None] * u[None, None, :]
    hit = d[:, :, 2] < -1e-6
    t = np.where(hit, 2.0 / np.maximum(-d[:, :, 2], 1e-6), 0.0)
    wx = d[:, :, 0] * t
    wy = d[:, :, 1] * t
    uv = np.stack([wx / 8.0, wy / 8.0], axis=-1)
    uv = uv - np.floor(uv)
    sky = ~hit
    uv[sky] = rng.random((int(sky.sum()), 2))
    return np.ascontiguousarray(uv.reshape(-1, 2).astype(np.float32))


def mip_levels(tex: np.ndarray) -> list:
    """Full MIP pyramid of an (H, W, C) texture down to 1x1: level l has
    max(1, H >> l) x max(1, W >> l) texels, each the average of the 2x2 block
    below it (rows / columns beyond an odd edge dropped; a side of 1 averages
    its single row / column twice), computed in binary64 and stored in the
    input's dtype (round to nearest for integer types)."""
    levels = [np.ascontiguousarray(tex)]
    cur = tex.astype(np.float64)
    while cur.shape[0] > 1 or cur.shape[1] > 1:
        h, w = max(1, cur.shape[0] // 2), max(1, cur.shape[1] // 2)
        r0 = cur[0:2 * h:2] if cur.shape[0] > 1 else cur
        r1 = cur[1:2 * h:2] if cur.shape[0] > 1 else cur
        a = (r0[:, 0:2 * w:2] if cur.shape[1] > 1 else r0) + (r0[:, 1:2 * w:2] if cur.shape[1] > 1 else r0)
        b = (r1[:, 0:2 * w:2] if cur.shape[1] > 1 else r1) + (r1[:, 1:2 * w:2] if cur.shape[1] > 1 else r1)
        cur = 0.25 * (a + b)
        if np.issubdtype(tex.dtype, np.integer):
            levels.append(np.ascontiguousarray(np.rint(cur).astype(tex.dtype)))
        else:
            levels.append(np.ascontiguousarray(cur.astype(tex.dtype)))
    return levels


def screen_ewa_queries(width: int = 3840, height: int = 2160, seed: int = 53, tile: float = 2.0) -> np.ndarray:
    """(width * height, 6) float32 EWA queries of the camera and ground plane
    of screen_uv_queries, the texture tiled every `tile` units (2 by default:
    mostly minified, strongly anisotropic towards the horizon): (s, t) and
    the texture-space derivatives along the
    pixel x and y axes (forward differences of the untiled coordinates, the
    last column / row repeated); sky pixels get a random (s, t) and a
    one-texel footprint of a 4096^2 texture."""
    rng = np.random.default_rng(seed)
    jx, jy = rng.random(2)
    px = (np.arange(width) + jx) / width * 2.0 - 1.0
    py = 1.0 - (np.arange(height) + jy) / height * 2.0
    tan_h = np.tan(np.radians(30.0))
    X, Y = np.meshgrid(px * tan_h, py * tan_h * height / width)
    pitch = np.radians(25.0)
    f = np.array([0.0, np.cos(pitch), -np.sin(pitch)])
    u = np.array([0.0, np.sin(pitch), np.cos(pitch)])
    d = f[None, None, :] + X[:, :, None] * np.array([1.0, 0.0, 0.0]) + Y[:, :, None] * u[None, None, :]
    hit = d[:, :, 2] < -1e-6
    t = np.where(hit, 2.0 / np.maximum(-d[:, :, 2], 1e-6), 0.0)
    su = d[:, :, 0] * t / tile
    sv = d[:, :, 1] * t / tile
    dsx = np.diff(su, axis=1, append=su[:, -1:] + (su[:, -1:] - su[:, -2:-1]))
    dtx = np.diff(sv, axis=1, append=sv[:, -1:] + (sv[:, -1:] - sv[:, -2:-1]))
    dsy = np.diff(su, axis=0, append=su[-1:, :] + (su[-1:, :] - su[-2:-1, :]))
    dty = np.diff(sv, axis=0, append=sv[-1:, :] + (sv[-1:, :] - sv[-2:-1, :]))
    q = np.stack([su - np.floor(su), sv - np.floor(sv), dsx, dtx, dsy, dty], axis=-1)
    sky = ~hit | ~np.all(np.isfinite(q), axis=-1) | (np.abs(q[..., 2:]) > 1.0).any(axis=-1)
    m = int(sky.sum())
    q[sky, 0:2] = rng.random((m, 2))
    q[sky, 2:6] = np.array([1.0 / 4096, 0.0, 0.0, 1.0 / 4096])
    return np.ascontiguousarray(q.reshape(-1, 6).astype(np.float32))


# ----------------------------------------------------------------------------
# fBm value noise and the sparse grid built from it
# ----------------------------------------------------------------------------
def _axis_interp(n_vox: int, period: float, offset: float):
    """Lattice cell and smoothstep-faded weight of each voxel along one axis."""
    x = (np.arange(n_vox, dtype=np.float64) + offset) / period
    cell = np.floor(x).astype(np.int64)
    f = x - cell
    w = f * f * (3.0 - 2.0 * f)
    return cell, w.astype(np.float32)


class _FbmOctaves:
    """fBm value noise on voxels.  Octave o has lattice period
    base_period / 2^o, amplitude 0.5^o and its own lattice (seeded from seed
    and o); lattice values are uniform in [-1, 1); interpolation is trilinear
    with a smoothstep fade; octave o is weighted by amp0 * 0.5^o (amp0 = 0.65
    puts about 6% of the 8^3 leaves above the 0.55 threshold at a base period
    of 64 voxels).  The x and y interpolation passes are
    done once per octave; z slabs are then produced on demand (with torch's
    multi-threaded CPU element-wise ops, each op rounded separately)."""

    def __init__(self, dims, base_period: float, seed: int, octaves: int = 5, amp0: float = 0.65):
        dx, dy, dz = dims
        self.dims = dims
        self.parts = []
        for o in range(octaves):
            period = base_period / (2.0 ** o)
            amp = amp0 * 0.5 ** o
            rng = np.random.default_rng(seed * 1000003 + o)
            off = rng.random(3) * period   # breaks lattice alignment across octaves
            cx, wx = _axis_interp(dx, period, off[0])
            cy, wy = _axis_interp(dy, period, off[1])
            cz, wz = _axis_interp(dz, period, off[2])
            lat = rng.random((int(cz[-1]) + 2, int(cy[-1]) + 2, int(cx[-1]) + 2), dtype=np.float32) * 2.0 - 1.0
            a = lat[:, :, cx] * (1.0 - wx) + lat[:, :, cx + 1] * wx
            b = a[:, cy, :] * (1.0 - wy)[None, :, None] + a[:, cy + 1, :] * wy[None, :, None]
            self.parts.append((float(amp), torch.from_numpy(cz), torch.from_numpy(wz),
                               torch.from_numpy(np.ascontiguousarray(b, np.float32))))

    def slab(self, z0: int, z1: int) -> np.ndarray:
        dx, dy, _ = self.dims
        out = torch.zeros((z1 - z0, dy, dx), dtype=torch.float32)
        for amp, cz, wz, b in self.parts:
            c, w = cz[z0:z1], wz[z0:z1][:, None, None]
            lo = b.index_select(0, c) * (1.0 - w)
            hi = b.index_select(0, c + 1) * w
            out += (lo + hi) * amp
        return out.numpy()


def fbm3d(dims=(512, 512, 512), base_period: float = 64.0, seed: int = 3, octaves: int = 5) -> np.ndarray:
    """fBm value noise on all voxels, float32 array (z, y, x)."""
    return _FbmOctaves(dims, base_period, seed, octaves).slab(0, dims[2])


class SparseGrid:
    """Leaves of a sparse voxel grid as plain arrays.

    origins: (n, 3) int32 voxel coordinates (x, y, z) of each leaf's corner,
             multiples of 8, sorted by (z, y, x).
    values:  (n, 8, 8, 8) float32 densities, index [z][y][x] within the leaf.
    dims:    domain size (x, y, z) in voxels.
    """

    def __init__(self, dims, origins, values):
        self.dims = tuple(int(d) for d in dims)
        self.origins = np.ascontiguousarray(origins, np.int32)
        self.values = np.ascontiguousarray(values, np.float32)

    @property
    def n_leaves(self) -> int:
        return int(self.origins.shape[0])

    def occupancy(self) -> float:
        nb = np.prod([(d + 7) // 8 for d in self.dims])
        return self.n_leaves / float(nb)

    def encoded(self, fmt: str) -> np.ndarray:
        return np.ascontiguousarray(encode(self.values, fmt)).reshape(self.values.shape)

    def dense(self) -> np.ndarray:
        """(z, y, x) float32 dense field, zero where no leaf is stored."""
        dx, dy, dz = self.dims
        nb = [(d + 7) // 8 for d in self.dims]
        d = np.zeros((nb[2] * 8, nb[1] * 8, nb[0] * 8), np.float32)
        for (ox, oy, oz), v in zip(self.origins, self.values):
            d[oz:oz + 8, oy:oy + 8, ox:ox + 8] = v
        return d[:dz, :dy, :dx]


def grid_from_field(field: np.ndarray, threshold: float = 0.55, z_offset: int = 0):
    """Leaves of density max(field - threshold, 0) whose maximum is > 0.
    field: (z, y, x) float32, every extent a multiple of 8."""
    nz, ny, nx = field.shape
    assert nz % 8 == 0 and ny % 8 == 0 and nx % 8 == 0
    bz, by, bx = nz // 8, ny // 8, nx // 8
    dens = np.maximum(field - np.float32(threshold), np.float32(0.0))
    leaves = dens.reshape(bz, 8, by, 8, bx, 8).transpose(0, 2, 4, 1, 3, 5)
    active = leaves.reshape(bz, by, bx, 512).max(axis=3) > 0
    kz, ky, kx = np.nonzero(active)
    origins = np.stack([kx * 8, ky * 8, kz * 8 + z_offset], axis=1).astype(np.int32)
    values = np.ascontiguousarray(leaves[kz, ky, kx])
    return origins, values


def fbm_grid(dims=(512, 512, 512), base_period: float = 64.0, seed: int = 3, threshold: float = 0.55,
             slab: int = 32) -> SparseGrid:
    """Sparse grid of the thresholded fBm field, built slab by slab in z."""
    dx, dy, dz = dims
    assert dx % 8 == 0 and dy % 8 == 0 and dz % 8 == 0 and slab % 8 == 0
    noise = _FbmOctaves(dims, base_period, seed)
    origins, values = [], []
    for z0 in range(0, dz, slab):
        z1 = min(z0 + slab, dz)
        o, v = grid_from_field(noise.slab(z0, z1), threshold, z_offset=z0)
        origins.append(o)
        values.append(v)
    return SparseGrid(dims, np.concatenate(origins), np.concatenate(values))


def ray_queries(dims=(512, 512, 512), n_rays: int = 65536, samples_per_ray: int = 256, seed: int = 4,
                shuffle: bool = False) -> np.ndarray:
    """(n_rays * samples_per_ray, 3) float32 positions in voxel index space
    (voxel k centred at k), ray-major.  Each ray: origin uniform in the box
    [0, dim - 1]^3, direction uniform on the sphere; the full chord of that
    line through the box is sampled at t0 + (k + xi) (t1 - t0) / n with one
    jitter xi per ray."""
    rng = np.random.default_rng(seed)
    hi = np.asarray(dims, np.float64) - 1.0
    o = rng.random((n_rays, 3)) * hi
    z = rng.random(n_rays) * 2.0 - 1.0
    phi = rng.random(n_rays) * 2.0 * np.pi
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    d = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    d = np.where(np.abs(d) < 1e-12, 1e-12, d)
    ta = (0.0 - o) / d
    tb = (hi - o) / d
    t0 = np.max(np.minimum(ta, tb), axis=1)
    t1 = np.min(np.maximum(ta, tb), axis=1)
    xi = rng.random(n_rays)
    k = np.arange(samples_per_ray, dtype=np.float64)
    out = np.empty((n_rays, samples_per_ray, 3), np.float32)
    step = (t1 - t0) / samples_per_ray
    for a in range(3):
        tt = t0[:, None] + (k[None, :] + xi[:, None]) * step[:, None]
        out[:, :, a] = (o[:, a:a + 1] + tt * d[:, a:a + 1]).astype(np.float32)
    out = out.reshape(-1, 3)
    np.minimum(out, hi.astype(np.float32), out=out)
    np.maximum(out, np.float32(0.0), out=out)
    if shuffle:
        out = out[rng.permutation(out.shape[0])]
    return np.ascontiguousarray(out)


def medium_ray_queries(grid: "SparseGrid", n: int = 1 << 24, seed: int = 4,
                       samples_per_ray: int = 256) -> np.ndarray:
    """(n, 3) float32 ray samples as ray_queries makes them (ray-major), kept
    only where the 4^3 voxel block around the sample (voxels floor(p) - 1 ..
    floor(p) + 2 per axis) meets a stored leaf: the lookups a renderer makes
    inside the medium once empty space is skipped.  Rays come in batches of
    65,536 (seeds seed, seed + 1, ...) until n samples are kept."""
    nb = [(d + 7) // 8 for d in grid.dims]
    occ = np.zeros((nb[0] + 2, nb[1] + 2, nb[2] + 2), bool)   # leaf (x, y, z) at [x + 1, y + 1, z + 1]
    o = grid.origins.astype(np.int64) // 8
    occ[o[:, 0] + 1, o[:, 1] + 1, o[:, 2] + 1] = True
    kept, total, k = [], 0, 0
    while total < n:
        pts = ray_queries(grid.dims, 65536, samples_per_ray, seed + k)
        c = np.floor(pts).astype(np.int64) - 1
        lo = np.clip(c >> 3, -1, np.asarray(nb)) + 1
        hi = np.clip((c + 3) >> 3, -1, np.asarray(nb)) + 1
        hit = np.zeros(pts.shape[0], bool)
        for sx in (lo[:, 0], hi[:, 0]):
            for sy in (lo[:, 1], hi[:, 1]):
                for sz in (lo[:, 2], hi[:, 2]):
                    hit |= occ[sx, sy, sz]
        kept.append(pts[hit])
        total += int(hit.sum())
        k += 1
    return np.ascontiguousarray(np.concatenate(kept)[:n])


def uniform_box_queries(dims, n: int, seed: int = 5, margin: float = 2.0) -> np.ndarray:
    """(n, 3) float32 positions uniform in [-margin, dim - 1 + margin] per
    axis, covering the boundary and the background outside the domain."""
    rng = np.random.default_rng(seed)
    lo = -margin
    hi = np.asarray(dims, np.float64) - 1.0 + margin
    return (lo + rng.random((n, 3)) * (hi - lo)).astype(np.float32)


# ----------------------------------------------------------------------------
# material texture for filtering with shading
# ----------------------------------------------------------------------------
MATERIAL_DTYPE = np.dtype([("albedo", np.uint8, 3), ("rough", np.uint8), ("nx", np.float16), ("ny", np.float16)])


def _gauss_blur_fft(img: np.ndarray, sigma: float) -> np.ndarray:
    """Periodic Gaussian blur of a 2D float64 image via the FFT (torch's
    multi-threaded CPU FFT)."""
    h, w = img.shape
    fy = torch.fft.fftfreq(h, dtype=torch.float64)[:, None]
    fx = torch.fft.rfftfreq(w, dtype=torch.float64)[None, :]
    g = torch.exp(-2.0 * (np.pi * sigma) ** 2 * (fx * fx + fy * fy))
    f = torch.fft.rfft2(torch.from_numpy(np.ascontiguousarray(img, np.float64)))
    return torch.fft.irfft2(f * g, s=img.shape).numpy()


def material_levels(size: int = 4096, seed: int = 21, levels: int = 3):
    """Material texels (H, W) of MATERIAL_DTYPE for levels 0..levels-1.

    Level 0: albedo RGB uniform integers; roughness round(255 Beta(2, 5));
    tangent normal from a height field of Gaussian bumps -- signed impulses at
    uniform positions, blurred with radii 2..64 texels (log-spaced, density
    falling with the radius squared, amplitude growing with the radius) plus a
    small white perturbation -- by central differences, (nx, ny) rounded to
    binary16.  Level l+1 is the 2x2 box average of level l: UNORM8 channels as
    (a + b + c + d + 2) >> 2, normal components ((a + b) + c) + d in binary32,
    divided by 4 and rounded to binary16, not renormalised."""
    rng = np.random.default_rng(seed)
    lv0 = np.zeros((size, size), MATERIAL_DTYPE)
    lv0["albedo"] = rng.integers(0, 256, (size, size, 3), dtype=np.uint8)
    lv0["rough"] = np.clip(np.rint(255.0 * rng.beta(2.0, 5.0, (size, size))), 0, 255).astype(np.uint8)
    height = np.zeros((size, size), np.float64)
    for r in (2.0, 4.0, 8.0, 16.0, 32.0, 64.0):
        count = int(size * size / (r * r) * 0.05) + 1
        imp = np.zeros((size, size), np.float64)
        ys = rng.integers(0, size, count)
        xs = rng.integers(0, size, count)
        np.add.at(imp, (ys, xs), rng.normal(0.0, 1.0, count) * r * r * r * 2.0)
        height += _gauss_blur_fft(imp, r)
    height += rng.normal(0.0, 0.02, (size, size))
    dhx = 0.5 * (np.roll(height, -1, axis=1) - np.roll(height, 1, axis=1))
    dhy = 0.5 * (np.roll(height, -1, axis=0) - np.roll(height, 1, axis=0))
    inv = 1.0 / np.sqrt(dhx * dhx + dhy * dhy + 1.0)
    lv0["nx"] = (-dhx * inv).astype(np.float32).astype(np.float16)
    lv0["ny"] = (-dhy * inv).astype(np.float32).astype(np.float16)
    out = [lv0]
    for _ in range(1, levels):
        p = out[-1]
        h2, w2 = p.shape[0] // 2, p.shape[1] // 2
        q = np.zeros((h2, w2), MATERIAL_DTYPE)
        a, b, c, d = p[0::2, 0::2], p[0::2, 1::2], p[1::2, 0::2], p[1::2, 1::2]
        for f in ("albedo", "rough"):
            s = a[f].astype(np.uint32) + b[f] + c[f] + d[f] + 2
            q[f] = (s >> 2).astype(np.uint8)
        for f in ("nx", "ny"):
            s = ((a[f].astype(np.float32) + b[f].astype(np.float32)) + c[f].astype(np.float32)) + d[f].astype(np.float32)
            q[f] = (s / np.float32(4.0)).astype(np.float16)
        out.append(q)
    return out


def shade_queries(n: int = 1 << 23, seed: int = 22) -> np.ndarray:
    """(n, 9) float32 shading records: uv uniform in [0,1)^2, footprint scale
    s = 2^U(-2, 2) texels, then wo and wi uniform on the upper hemisphere
    (z uniform in [0, 1), azimuth uniform)."""
    rng = np.random.default_rng(seed)
    rec = np.empty((n, 9), np.float32)
    rec[:, 0:2] = rng.random((n, 2), dtype=np.float32)
    rec[:, 2] = np.exp2(rng.random(n) * 4.0 - 2.0).astype(np.float32)
    for k in (3, 6):
        z = rng.random(n)
        phi = rng.random(n) * 2.0 * np.pi
        r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
        rec[:, k] = (r * np.cos(phi)).astype(np.float32)
        rec[:, k + 1] = (r * np.sin(phi)).astype(np.float32)
        rec[:, k + 2] = z.astype(np.float32)
    return rec


# ----------------------------------------------------------------------------
# neural texture workload
# ----------------------------------------------------------------------------
def _smooth_field(size: int, rng, radii=(4.0, 8.0, 16.0, 32.0)) -> np.ndarray:
    """Sum of periodically blurred white noise at several radii, normalised to
    zero mean and unit standard deviation."""
    f = np.zeros((size, size), np.float64)
    for r in radii:
        f += _gauss_blur_fft(rng.normal(0.0, 1.0, (size, size)), r) * r
    f -= f.mean()
    return f / (f.std() + 1e-30)


def _fbm2d(size: int, rng, base_period: float = 64.0, octaves: int = 5) -> np.ndarray:
    """2D value-noise fBm (lacunarity 2, gain 0.5), smoothstep-faded bilinear
    interpolation of uniform [-1, 1) lattices."""
    out = np.zeros((size, size), np.float64)
    for o in range(octaves):
        period = base_period / 2 ** o
        cx, wx = _axis_interp(size, period, rng.random() * period)
        cy, wy = _axis_interp(size, period, rng.random() * period)
        lat = rng.random((int(cy[-1]) + 2, int(cx[-1]) + 2)) * 2.0 - 1.0
        a = lat[:, cx] * (1 - wx) + lat[:, cx + 1] * wx
        out += 0.5 ** o * (a[cy, :] * (1 - wy)[:, None] + a[cy + 1, :] * wy[:, None])
    return out


def neural_target(size: int = 4096, seed: int = 41) -> np.ndarray:
    """(size, size, 8) float32 material for the neural texture: albedo RGB
    and roughness as smooth fields squashed into [0, 1], a tangent normal
    (x, y) from a Gaussian-bump height field, and two fBm detail channels."""
    rng = np.random.default_rng(seed)
    t = np.empty((size, size, 8), np.float32)
    for c in range(3):
        t[:, :, c] = 0.5 + 0.35 * np.tanh(_smooth_field(size, rng))
    t[:, :, 3] = 0.35 + 0.25 * np.tanh(_smooth_field(size, rng, radii=(8.0, 32.0)))
    height = _smooth_field(size, rng, radii=(2.0, 6.0, 18.0)) * 1.5
    dhx = 0.5 * (np.roll(height, -1, axis=1) - np.roll(height, 1, axis=1))
    dhy = 0.5 * (np.roll(height, -1, axis=0) - np.roll(height, 1, axis=0))
    inv = 1.0 / np.sqrt(dhx * dhx + dhy * dhy + 1.0)
    t[:, :, 4] = -dhx * inv
    t[:, :, 5] = -dhy * inv
    t[:, :, 6] = 0.5 + 0.5 * _fbm2d(size, rng)
    t[:, :, 7] = 0.5 + 0.5 * _fbm2d(size, rng, base_period=32.0)
    return t


def texture_set_u8(size: int = 4096, seed: int = 51) -> np.ndarray:
    """(size, size, 9) uint8 texture set: the eight channels of the neural
    target (albedo RGB, roughness, tangent normal x and y mapped from [-1, 1]
    to [0, 1], two fBm detail channels) plus a third fBm detail channel,
    quantised as round(255 v) after clamping to [0, 1]."""
    t = neural_target(size, seed)
    rng = np.random.default_rng(seed + 1)
    out = np.empty((size, size, 9), np.uint8)
    for c in range(8):
        v = t[:, :, c].astype(np.float64)
        if c in (4, 5):
            v = 0.5 * (v + 1.0)
        out[:, :, c] = np.round(np.clip(v, 0.0, 1.0) * 255.0).astype(np.uint8)
    extra = 0.5 + 0.5 * _fbm2d(size, rng, base_period=16.0)
    out[:, :, 8] = np.round(np.clip(extra, 0.0, 1.0) * 255.0).astype(np.uint8)
    return out


def neural_init(latent_size: int = 1024, seed: int = 42):
    """Initial latents (latent_size, latent_size, 8) ~ N(0, 0.1^2) and MLP
    parameters (5256,) with He-normal weights and zero biases, float32.
    Layout: W1[64][8], b1[64], W2[64][64], b2[64], W3[8][64], b3[8]."""
    rng = np.random.default_rng(seed)
    lat = rng.normal(0.0, 0.1, (latent_size, latent_size, 8)).astype(np.float32)
    w1 = rng.normal(0.0, np.sqrt(2.0 / 8), (64, 8))
    w2 = rng.normal(0.0, np.sqrt(2.0 / 64), (64, 64))
    w3 = rng.normal(0.0, np.sqrt(1.0 / 64), (8, 64))
    mlp = np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), w3.ravel(), np.zeros(8)])
    return lat, mlp.astype(np.float32)


def neural_queries(n: int = 1 << 24, seed: int = 43) -> np.ndarray:
    return uv_queries(n, seed)


# ----------------------------------------------------------------------------
# large sparse grid for the serving workload
# ----------------------------------------------------------------------------
def coarse_fbm_grid(dims=(2048, 2048, 2048), occupancy: float = 0.02, seed: int = 13,
                    base_period_leaves: float = 16.0) -> SparseGrid:
    """A sparse grid whose active leaves are chosen at leaf resolution: the
    fBm of _FbmOctaves evaluated at leaf centres (one value per 8^3 leaf) is
    thresholded at the quantile that keeps `occupancy` of the leaves; a voxel
    of an active leaf holds (leaf value - threshold) * (0.5 + xi), xi uniform
    in [0, 1) per voxel.  Cheap enough for a 2048^3 domain."""
    nb = tuple(d // 8 for d in dims)
    coarse = _FbmOctaves(nb, base_period_leaves, seed).slab(0, nb[2])    # (bz, by, bx)
    thr = np.quantile(coarse, 1.0 - occupancy)
    kz, ky, kx = np.nonzero(coarse > thr)
    origins = np.stack([kx * 8, ky * 8, kz * 8], axis=1).astype(np.int32)
    rng = np.random.default_rng(seed + 1)
    base = (coarse[kz, ky, kx] - thr).astype(np.float32)
    values = base[:, None, None, None] * (np.float32(0.5) + rng.random((kz.size, 8, 8, 8), dtype=np.float32))
    return SparseGrid(dims, origins, values)

"""Seeded synthetic stereo inputs.

The paper measures on Middlebury pairs and on pairs with exposure and
lighting changes (Section 4).  Those datasets are not used here; these
generators stand in for them with natural-image-like 8-bit RGB content of the
same kind: band-limited texture, fronto-parallel and slanted surfaces,
occlusions, sensor noise and a global radiometric change.

This module holds input generation only (no step of the matching method), and
it is the one module that both the GPU path's tests and the CPU oracle's
tests draw inputs from.  Everything is driven by numpy ``Generator(PCG64)``.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
from scipy.ndimage import gaussian_filter


@dataclass
class Scene:
    left: np.ndarray            # uint8 [H][W][3]
    right: np.ndarray           # uint8 [H][W][3]
    dmax: int
    gt: np.ndarray              # float32 [H][W] left-view disparity
    seed: int
    meta: dict = field(default_factory=dict)


def _unit_noise(rng, H, W, blur):
    z = rng.standard_normal((H, W))
    z = gaussian_filter(z, blur, mode="reflect")
    z -= z.mean()
    s = z.std()
    return z / s if s > 0 else z


def texture(rng, H, W, blur=1.2, amp=48.0):
    """Band-limited colour texture, float64 [H][W][3] around 128."""
    lum = _unit_noise(rng, H, W, blur)
    out = np.empty((H, W, 3))
    for c in range(3):
        out[..., c] = 128.0 + amp * (0.8 * lum + 0.45 * _unit_noise(rng, H, W, blur))
    return out


def to_u8(x):
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def add_noise(rng, img_f, sigma):
    if sigma <= 0:
        return img_f
    return img_f + rng.normal(0.0, sigma, img_f.shape)


def constant_shift_pair(seed, W, H, d0, blur=1.2):
    """Noise-free fronto-parallel textured plane at disparity d0.

    right(u) = left(u + d0): the left pixel (u, v) and the right pixel
    (u - d0, v) see the same surface point.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    canvas = to_u8(texture(rng, H, W + d0, blur))
    left = np.ascontiguousarray(canvas[:, :W])
    right = np.ascontiguousarray(canvas[:, d0:d0 + W])
    gt = np.full((H, W), float(d0), np.float32)
    return Scene(left, right, d0 + 1, gt, seed, {"kind": "constant", "d0": d0})


def rect_scene(seed=14022020, W=128, H=96, dmax=16, n_rects=4, bg_d=2,
               noise=2.0):
    """Background plane plus axis-aligned fronto-parallel rectangles.

    Each rectangle has its own texture and a distinct integer disparity in
    [3, dmax - 2]; the right view is rendered layer by layer with a z-test
    (larger disparity is nearer), so disoccluded pixels show the background.
    The right view gets additive Gaussian noise.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    Wc = W + dmax
    layers = [(0, 0, Wc, H, bg_d)]
    ds = rng.choice(np.arange(3, dmax - 1), size=n_rects, replace=False)
    for k in range(n_rects):
        rw = int(rng.integers(16, 49))
        rh = int(rng.integers(16, 49))
        x0 = int(rng.integers(0, max(1, W - rw)))
        y0 = int(rng.integers(0, max(1, H - rh)))
        layers.append((x0, y0, rw, rh, int(ds[k])))
    tex = [texture(rng, H, Wc) for _ in layers]

    left = np.zeros((H, W, 3))
    gt = np.zeros((H, W), np.float32)
    zl = np.full((H, W), -1.0)
    right = np.zeros((H, W, 3))
    zr = np.full((H, W), -1.0)
    for (x0, y0, rw, rh, d), t in zip(layers, tex):
        # left view: layer covers [x0, x0+rw) x [y0, y0+rh)
        ys = slice(y0, min(H, y0 + rh))
        u = np.arange(W)
        inside = (u >= x0) & (u < x0 + rw)
        for v in range(ys.start, ys.stop):
            sel = inside & (d > zl[v])
            left[v, sel] = t[v, u[sel]]
            gt[v, sel] = d
            zl[v, sel] = d
            # right view: right pixel ur sees left position ur + d
            ul = u + d
            selr = (ul >= x0) & (ul < x0 + rw) & (ul < Wc) & (d > zr[v])
            right[v, selr] = t[v, ul[selr]]
            zr[v, selr] = d
    right = add_noise(rng, right, noise)
    return Scene(to_u8(left), to_u8(right), dmax, gt, seed,
                 {"kind": "rects", "layers": layers})


def _bilinear(t, x, y):
    """Samples texture t [H][Wc][3] at float x (row y integer)."""
    Wc = t.shape[1]
    x = np.clip(x, 0, Wc - 1.000001)
    x0 = np.floor(x).astype(np.int64)
    fx = (x - x0)[:, None]
    return t[y, x0] * (1.0 - fx) + t[y, x0 + 1] * fx


def slanted_scene(seed=14022021, W=450, H=375, dmax=60, n_regions=7,
                  noise=3.0, max_grad=0.2, radiometric=False, tinted=False,
                  tex_amp=48.0, tex_blur=1.2):
    """Slanted-plane scene: a background plane and n_regions planar patches.

    Patch k covers a rectangle or an ellipse (10-40 % of W and H) in left
    coordinates with disparity d_k(u, v) = a_k (u - u_k) + b_k (v - v_k) + c_k,
    |a_k|, |b_k| <= max_grad, d in [1, dmax - 2].  Nearer surfaces (larger d)
    win in both views, which leaves occlusion bands at discontinuities.  Each
    surface has its own texture, sampled bilinearly.  Both views get Gaussian
    noise; optionally the right view gets a global gain, gamma and
    per-channel offset.  With tinted=True every surface's texture gets its
    own colour offset (objects of distinct colours, as in natural scenes);
    tex_amp and tex_blur set the texture's contrast and grain (weak, coarse
    texture leaves the surfaces' colour steps as the strongest structure in a
    window).  The defaults draw exactly the random numbers they always did.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    Wc = W + dmax + 2
    lo_d, hi_d = 1.0, float(dmax - 2)

    planes = []
    # background: gentle slant, far away
    for k in range(n_regions + 1):
        if k == 0:
            kind = "all"
            uc, vc, rw, rh = W / 2, H / 2, W, H
        else:
            kind = "rect" if rng.random() < 0.5 else "ellipse"
            rw = rng.uniform(0.10, 0.40) * W
            rh = rng.uniform(0.10, 0.40) * H
            uc = rng.uniform(rw / 2, W - rw / 2)
            vc = rng.uniform(rh / 2, H - rh / 2)
        a = rng.uniform(-max_grad, max_grad)
        b = rng.uniform(-max_grad, max_grad)
        # choose c so that d stays in [lo_d, hi_d] over the patch
        span = abs(a) * rw / 2 + abs(b) * rh / 2
        if k == 0:
            a *= 0.25
            b *= 0.25
            span = abs(a) * rw / 2 + abs(b) * rh / 2
            c = rng.uniform(lo_d + span, max(lo_d + span, 0.35 * hi_d))
        else:
            c = rng.uniform(min(lo_d + span, hi_d), max(hi_d - span, lo_d + span))
        planes.append(dict(kind=kind, uc=uc, vc=vc, rw=rw, rh=rh, a=a, b=b, c=c))
    tex = [texture(rng, H, Wc, tex_blur, tex_amp) for _ in planes]
    if tinted:
        tint_rng = np.random.Generator(np.random.PCG64(seed + 0x7E57))
        tex = [t + tint_rng.uniform(-60.0, 60.0, 3) for t in tex]

    def disp(p, u, v):
        d = p["a"] * (u - p["uc"]) + p["b"] * (v - p["vc"]) + p["c"]
        return np.clip(d, lo_d, hi_d)

    def covers(p, u, v):
        if p["kind"] == "all":
            return np.ones_like(u, dtype=bool)
        du = (u - p["uc"]) / (p["rw"] / 2)
        dv = (v - p["vc"]) / (p["rh"] / 2)
        if p["kind"] == "rect":
            return (np.abs(du) <= 1) & (np.abs(dv) <= 1)
        return du * du + dv * dv <= 1

    left = np.zeros((H, W, 3))
    right = np.zeros((H, W, 3))
    gt = np.zeros((H, W), np.float32)
    gt_right = np.full((H, W), -1.0, np.float32)  # right-view disparity, -1: no surface
    u = np.arange(W, dtype=np.float64)
    for v in range(H):
        zl = np.full(W, -1.0)
        zr = np.full(W, -1.0)
        for p, t in zip(planes, tex):
            d = disp(p, u, v)
            sel = covers(p, u, v) & (d > zl)
            if sel.any():
                left[v, sel] = _bilinear(t, u[sel], v)
                gt[v, sel] = d[sel]
                zl[sel] = d[sel]
            # right pixel ur sees left position ul with ul - d(ul) = ur;
            # d is affine in u, so ul = (ur + c - a uc + b (v - vc)) / (1 - a)
            ul = (u + p["c"] - p["a"] * p["uc"] + p["b"] * (v - p["vc"])) / (1.0 - p["a"])
            dl = ul - u
            selr = covers(p, ul, v) & (ul >= 0) & (ul <= Wc - 1) & (dl > zr) \
                & (dl >= lo_d - 1e-9) & (dl <= hi_d + 1e-9)
            if selr.any():
                right[v, selr] = _bilinear(t, ul[selr], v)
                zr[selr] = dl[selr]
        gt_right[v] = zr
        # right pixels no surface reaches (background clamping at edges)
        hole = zr < 0
        if hole.any():
            right[v, hole] = _bilinear(tex[0], u[hole] + planes[0]["c"], v)
    left = add_noise(rng, left, noise)
    right = add_noise(rng, right, noise)
    meta = {"kind": "slanted", "planes": planes, "gt_right": gt_right}
    if radiometric:
        g = rng.uniform(0.5, 2.0)
        gamma = rng.uniform(0.7, 1.4)
        off = rng.uniform(-20.0, 20.0, 3)
        x = np.clip(right, 0, 255)
        right = 255.0 * np.minimum(1.0, g * x / 255.0) ** gamma + off
        meta.update(gain=g, gamma=gamma, offset=off.tolist())
    return Scene(to_u8(left), to_u8(right), dmax, gt, seed, meta)


# --- the workloads -------------------------------------------------------

def radiometric(img: np.ndarray, gain=1.0, gamma=1.0, offset=(0.0, 0.0, 0.0)) -> np.ndarray:
    """A global radiometric change of an 8-bit RGB view (exposure gain, gamma
    and per-channel offset, clamped), the kind of change the paper's
    radiometric experiments apply to one view."""
    x = img.astype(np.float64)
    y = 255.0 * np.minimum(1.0, gain * x / 255.0) ** gamma + np.asarray(offset, np.float64)
    return to_u8(y)


def near_discontinuity(scene: Scene, band=5, jump=1.0) -> np.ndarray:
    """Left pixels within `band` columns or rows of a ground-truth depth jump
    larger than `jump` px (where fattening errors appear)."""
    from scipy.ndimage import binary_dilation
    gt = scene.gt
    edge = np.zeros(gt.shape, bool)
    edge[:, 1:] |= np.abs(np.diff(gt, axis=1)) > jump
    edge[1:, :] |= np.abs(np.diff(gt, axis=0)) > jump
    return binary_dilation(edge, iterations=band)


def non_occluded(scene: Scene, tol=1.0) -> np.ndarray:
    """Left pixels whose ground-truth partner in the right view shows the
    same surface (the right view's ground truth agrees within tol)."""
    gt, gtr = scene.gt, scene.meta["gt_right"]
    H, W = gt.shape
    ur = np.rint(np.arange(W)[None, :] - gt).astype(np.int64)
    inside = (ur >= 0) & (ur < W)
    partner = np.take_along_axis(gtr, np.clip(ur, 0, W - 1), axis=1)
    return inside & (partner >= 0) & (np.abs(partner - gt) <= tol)


def config_scene(cfg: int) -> Scene:
    """The single-pair workloads: 0 = 128x96 rectangles (dmax 16),
    1 = 450x375 slanted planes (dmax 60), 2 = 1400x1100 slanted planes with a
    radiometric change (dmax 256)."""
    if cfg == 0:
        return rect_scene(14022020, 128, 96, 16)
    if cfg == 1:
        return slanted_scene(14022021, 450, 375, 60)
    if cfg == 2:
        return slanted_scene(14022022, 1400, 1100, 256, radiometric=True)
    raise ValueError(cfg)


CONFIG_PARAMS = {
    # n bits, window S, sigma, dmax, volume wanted
    0: dict(n=256, S=15, sigma=4.0 * 15 / 26, dmax=16, want_cost=False),
    1: dict(n=1024, S=31, sigma=4.0 * 31 / 26, dmax=60, want_cost=True),
    2: dict(n=1024, S=31, sigma=4.0 * 31 / 26, dmax=256, want_cost=False),
}
PATTERN_SEED = 0x1402202000000001


@dataclass
class BatchSpec:
    W: int
    H: int
    dmax: int
    seed: int


def batch_specs(count=64, base_seed=14022020 + 100) -> List[BatchSpec]:
    """Uneven pairs: W ~ U{320..1920}, H ~ U{240..1080},
    dmax ~ U{32, 64, 128, 256}; pair j uses seed base_seed + j."""
    out = []
    for j in range(count):
        rng = np.random.Generator(np.random.PCG64(base_seed + j))
        W = int(rng.integers(320, 1921))
        H = int(rng.integers(240, 1081))
        dmax = int(rng.choice([32, 64, 128, 256]))
        out.append(BatchSpec(W, H, dmax, base_seed + j))
    return out


def batch_scene(spec: BatchSpec, scale: float = 1.0) -> Scene:
    """One pair of the uneven batch (optionally scaled down for tests)."""
    W = max(16, int(spec.W * scale))
    H = max(16, int(spec.H * scale))
    dmax = max(4, min(int(spec.dmax * scale) if scale < 1 else spec.dmax, W))
    return slanted_scene(spec.seed, W, H, dmax)


def poisson_arrivals(rate, duration, n_items, seed):
    """Arrival times (s) of a Poisson process and the item drawn for each
    arrival (uniform with replacement over n_items)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    times = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        times.append(t)
    items = rng.integers(0, n_items, len(times))
    return np.array(times), items


def random_image(seed, W, H, lo=0, hi=255):
    """Uniform random RGB image (for parity cases that need no structure)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, (H, W, 3), dtype=np.int64).astype(np.uint8)


def all_colours_image():
    """4096 x 4096 RGB image holding each of the 2^24 colours once."""
    c = np.arange(1 << 24, dtype=np.uint32)
    img = np.empty((1 << 24, 3), np.uint8)
    img[:, 0] = (c >> 16) & 255
    img[:, 1] = (c >> 8) & 255
    img[:, 2] = c & 255
    return img.reshape(4096, 4096, 3)


def grey_image(values: np.ndarray) -> np.ndarray:
    v = np.asarray(values, np.uint8)
    return np.repeat(v[..., None], 3, axis=-1)

"""Seeded synthetic inputs for the deconvolution sampler.

This module only *produces inputs*: point spread functions, ground-truth
objects, sCMOS calibration maps and simulated raw frames.  It holds none of
the sampler's arithmetic (no likelihood, no proposal, no moments) and is
shared by the tests, the benchmark and the CPU oracle's callers alike.

Physical model of the simulated frames follows the image-formation section of
the paper (Methods, "Image Formation Model", Eqs. 1-4): the expected photon
image is the pixel-integrated PSF convolved with the object, photon counts are
Poisson, and the camera reads ``G*phi + o`` plus Normal read noise of standard
deviation ``sigma`` (all in ADU).  The convolution here is scipy's library
routine with zero padding ("same" size), which matches the object-lattice =
pixel-lattice reading used by the sampler.

The paper's datasets (the TestImages.jl Siemens star and the HeLa
mitochondria frames) are not available; the generators below are procedural
stand-ins with the photon levels, PSFs and camera parameters the paper quotes
(Results; Fig. "siemens", Fig. "experimentaldata").
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy import signal, special


# ----------------------------------------------------------------------------
# Point spread functions
# ----------------------------------------------------------------------------

def gaussian_psf(sigma_px: float, size: int) -> np.ndarray:
    """Pixel-integrated isotropic Gaussian PSF on a ``size x size`` grid.

    Each pixel holds the integral of N(0, sigma^2) over its unit square
    (separable erf differences), the array is then renormalised to sum 1
    after truncation (Eq. 1 integrates the PSF over the pixel area).
    """
    if size % 2 != 1:
        raise ValueError("PSF side must be odd")
    r = size // 2
    edges = (np.arange(-r, r + 2, dtype=np.float64) - 0.5) / (sigma_px * math.sqrt(2.0))
    cdf = 0.5 * special.erf(edges)
    p1 = np.diff(cdf)
    psf = np.outer(p1, p1)
    return psf / psf.sum()


def airy_psf(na: float, wavelength_um: float, pixel_um: float, size: int,
             supersample: int = 16) -> np.ndarray:
    """Pixel-integrated Airy-disk PSF, ``(2 J1(v)/v)^2`` with v = 2 pi NA r / lambda.

    Each pixel is integrated by ``supersample x supersample`` midpoint
    sampling, then the truncated array is normalised to sum 1.
    """
    if size % 2 != 1:
        raise ValueError("PSF side must be odd")
    r = size // 2
    sub = (np.arange(supersample, dtype=np.float64) + 0.5) / supersample - 0.5
    coords = (np.arange(-r, r + 1, dtype=np.float64)[:, None] + sub[None, :]).ravel()
    yy, xx = np.meshgrid(coords, coords, indexing="ij")
    rr = np.hypot(yy, xx) * pixel_um
    v = 2.0 * math.pi * na * rr / wavelength_um
    with np.errstate(invalid="ignore", divide="ignore"):
        amp = np.where(v > 0, 2.0 * special.j1(v) / v, 1.0)
    inten = amp * amp
    psf = inten.reshape(size, supersample, size, supersample).mean(axis=(1, 3))
    return psf / psf.sum()


def airy_psf_matched(sigma_px: float, size: int, pixel_um: float = 0.065,
                     wavelength_um: float = 0.6) -> np.ndarray:
    """Airy PSF whose core matches a Gaussian of ``sigma_px`` (sigma ~ 0.21 lambda/NA)."""
    na = 0.21 * wavelength_um / (sigma_px * pixel_um)
    return airy_psf(na, wavelength_um, pixel_um, size)


# ----------------------------------------------------------------------------
# Objects (photons per object pixel per frame)
# ----------------------------------------------------------------------------

def _splat(img: np.ndarray, y: np.ndarray, x: np.ndarray, val: np.ndarray) -> None:
    """Bilinear splat of point masses into ``img`` (points outside are dropped)."""
    h, w = img.shape
    y0 = np.floor(y).astype(np.int64)
    x0 = np.floor(x).astype(np.int64)
    fy = y - y0
    fx = x - x0
    for dy, wy in ((0, 1.0 - fy), (1, fy)):
        for dx, wx in ((0, 1.0 - fx), (1, fx)):
            yy = y0 + dy
            xx = x0 + dx
            ok = (yy >= 0) & (yy < h) & (xx >= 0) & (xx < w)
            np.add.at(img, (yy[ok], xx[ok]), (val * wy * wx)[ok])


def add_beads(img: np.ndarray, rng: np.random.Generator, n: int,
              shape: float = 2.0, scale: float = 50.0) -> None:
    """Single-pixel beads with Gamma(shape, scale) photon intensities."""
    h, w = img.shape
    ys = rng.integers(0, h, n)
    xs = rng.integers(0, w, n)
    np.add.at(img, (ys, xs), rng.gamma(shape, scale, n))


def add_segments(img: np.ndarray, rng: np.random.Generator, n: int,
                 len_lo: float = 8.0, len_hi: float = 32.0,
                 shape: float = 2.0, scale: float = 50.0, step: float = 0.25) -> None:
    """Straight segments, splatted every ``step`` px, carrying I photons per px of length."""
    h, w = img.shape
    for _ in range(n):
        cy, cx = rng.uniform(0, h), rng.uniform(0, w)
        length = rng.uniform(len_lo, len_hi)
        ang = rng.uniform(0, math.pi)
        inten = rng.gamma(shape, scale)
        tt = np.arange(-length / 2, length / 2, step)
        _splat(img, cy + tt * math.sin(ang), cx + tt * math.cos(ang),
               np.full(tt.shape, inten * step))


def _catmull_rom(pts: np.ndarray, step: float) -> np.ndarray:
    """Dense points along a Catmull-Rom spline through ``pts`` (k x 2), ~``step`` px apart."""
    p = np.vstack([pts[0], pts, pts[-1]])
    out = []
    for i in range(1, len(p) - 2):
        p0, p1, p2, p3 = p[i - 1], p[i], p[i + 1], p[i + 2]
        seg_len = np.linalg.norm(p2 - p1)
        m = max(2, int(math.ceil(seg_len / step)))
        t = np.arange(m, dtype=np.float64)[:, None] / m
        t2, t3 = t * t, t * t * t
        out.append(0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t2
                          + (-p0 + 3 * p1 - 3 * p2 + p3) * t3))
    return np.vstack(out)


def add_filaments(img: np.ndarray, rng: np.random.Generator, n: int,
                  shape: float = 2.0, scale: float = 50.0, step: float = 0.25) -> None:
    """Catmull-Rom filaments: 4-6 control points, random-walk steps U(10, 60) px."""
    h, w = img.shape
    for _ in range(n):
        k = int(rng.integers(4, 7))
        pts = np.empty((k, 2))
        pts[0] = (rng.uniform(0, h), rng.uniform(0, w))
        ang = rng.uniform(0, 2 * math.pi)
        for j in range(1, k):
            ang += rng.normal(0.0, 0.6)
            d = rng.uniform(10, 60)
            pts[j] = pts[j - 1] + d * np.array([math.sin(ang), math.cos(ang)])
        dense = _catmull_rom(pts, step)
        seglen = np.linalg.norm(np.diff(dense, axis=0), axis=1)
        inten = rng.gamma(shape, scale)
        _splat(img, dense[:-1, 0], dense[:-1, 1], inten * seglen)


# ----------------------------------------------------------------------------
# Camera and frame simulation
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Camera:
    """sCMOS calibration: gain (ADU/e), offset (ADU), read-noise std (ADU).

    Each field is either a 0-d array (a global constant, the paper's fallback
    when no calibration maps exist) or an (H, W) map.
    """
    gain: np.ndarray
    offset: np.ndarray
    sigma: np.ndarray

    @property
    def per_pixel(self) -> bool:
        return np.ndim(self.gain) == 2

    def maps(self, h: int, w: int):
        f = lambda a: np.broadcast_to(np.asarray(a, np.float64), (h, w)).copy()
        return f(self.gain), f(self.offset), f(self.sigma)


def scalar_camera(gain: float = 2.0, offset: float = 100.0, sigma: float = 1.5) -> Camera:
    return Camera(np.asarray(gain, np.float64), np.asarray(offset, np.float64),
                  np.asarray(sigma, np.float64))


def scmos_maps(rng: np.random.Generator, h: int, w: int) -> Camera:
    """Per-pixel maps: G ~ N(2, 0.1), o ~ N(100, 3), sigma ~ LogNormal(0.4, 0.5) ADU."""
    gain = rng.normal(2.0, 0.1, (h, w))
    offset = rng.normal(100.0, 3.0, (h, w))
    sigma = np.exp(rng.normal(0.4, 0.5, (h, w)))
    return Camera(gain, offset, sigma)


def expected_image(obj: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """Noise-free photon image (library 2-D convolution, zero padding, same size)."""
    if obj.size * psf.size > 2e7:
        return signal.fftconvolve(obj, psf, mode="same")
    return signal.convolve2d(obj, psf, mode="same", boundary="fill", fillvalue=0.0)


def simulate_frame(obj: np.ndarray, psf: np.ndarray, cam: Camera,
                   rng: np.random.Generator) -> np.ndarray:
    """Raw frame in ADU: phi ~ Poisson(mu), w ~ Normal(G phi + o, sigma^2)."""
    h, w = obj.shape
    mu = np.clip(expected_image(obj, psf), 0.0, None)
    phi = rng.poisson(mu)
    g, o, s = cam.maps(h, w)
    return g * phi + o + s * rng.standard_normal((h, w))


def simulate_frame_emccd(obj: np.ndarray, psf: np.ndarray, cam: Camera,
                         rng: np.random.Generator) -> np.ndarray:
    """Raw EMCCD frame in ADU: phi ~ Poisson(mu); the multiplication register
    gives x ~ Gamma(phi, 1) photon units for phi >= 1 and x = 0 for phi = 0;
    w = o + G x, plus Normal(0, sigma^2) read noise on zero-photon readings."""
    h, w = obj.shape
    mu = np.clip(expected_image(obj, psf), 0.0, None)
    phi = rng.poisson(mu)
    x = np.where(phi > 0, rng.gamma(np.maximum(phi, 1), 1.0), 0.0)
    g, o, s = cam.maps(h, w)
    return o + g * x + np.where(phi == 0, s * rng.standard_normal((h, w)), 0.0)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Frame:
    """One deconvolution problem: raw frame, PSF, camera and the ground truth."""
    name: str
    image: np.ndarray            # (H, W) ADU, float64
    psf: np.ndarray              # (s, s), sums to 1
    camera: Camera
    truth: np.ndarray            # (H, W) photons per object pixel
    seed: int
    n_sweeps: int = 500
    n_chains: int = 1

    @property
    def shape(self):
        return self.image.shape


AIRY_NA, AIRY_LAMBDA_UM, AIRY_PIXEL_UM = 1.4, 0.6, 0.065


def frame_beads_segments(n: int = 64, seed: int = 0, n_prims: int = 20,
                         background: float = 2.0, psf: Optional[np.ndarray] = None,
                         camera: Optional[Camera] = None) -> Frame:
    """64x64-class frame: Gaussian sigma=1.5 px PSF (11x11), beads + segments on 2 ph/px."""
    rng = np.random.default_rng(seed)
    obj = np.full((n, n), background, np.float64)
    add_beads(obj, rng, n_prims // 2)
    add_segments(obj, rng, n_prims - n_prims // 2)
    psf = gaussian_psf(1.5, 11) if psf is None else psf
    cam = scalar_camera() if camera is None else camera
    img = simulate_frame(obj, psf, cam, rng)
    return Frame("beads_segments_%d" % n, img, psf, cam, obj, seed, 500, 1)


def frame_filaments(n: int = 512, seed: int = 1, n_filaments: int = 200,
                    background: float = 2.0, psf_size: int = 31) -> Frame:
    """512x512-class frame: Airy (NA 1.4, 0.6 um, 65 nm) 31x31, filaments, per-pixel sCMOS maps."""
    rng = np.random.default_rng(seed)
    obj = np.full((n, n), background, np.float64)
    add_filaments(obj, rng, n_filaments)
    psf = airy_psf(AIRY_NA, AIRY_LAMBDA_UM, AIRY_PIXEL_UM, psf_size)
    cam = scmos_maps(rng, n, n)
    img = simulate_frame(obj, psf, cam, rng)
    return Frame("filaments_%d" % n, img, psf, cam, obj, seed, 2000, 1)


def frame_dense(n: int = 2048, seed: int = 2, n_beads: int = 5000, n_filaments: int = 2000,
                bg_lo: float = 1.0, bg_hi: float = 10.0, n_chains: int = 4,
                psf_size: int = 31) -> Frame:
    """2048x2048-class frame: same Airy PSF, beads + filaments on a 1..10 ph/px x-gradient."""
    rng = np.random.default_rng(seed)
    grad = np.linspace(bg_lo, bg_hi, n, dtype=np.float64)
    obj = np.broadcast_to(grad[None, :], (n, n)).copy()
    add_beads(obj, rng, n_beads)
    add_filaments(obj, rng, n_filaments)
    psf = airy_psf(AIRY_NA, AIRY_LAMBDA_UM, AIRY_PIXEL_UM, psf_size)
    cam = scmos_maps(rng, n, n)
    img = simulate_frame(obj, psf, cam, rng)
    return Frame("dense_%d" % n, img, psf, cam, obj, seed, 1000, n_chains)


def tile_batch(n_tiles: int = 256, seed: int = 3, side_lo: int = 64, side_hi: int = 512,
               max_side: Optional[int] = None):
    """Heterogeneous tiles: sides U{side_lo..side_hi}, Gaussian or Airy PSF with sigma U[1, 3].

    Gaussian tiles use s = 2 ceil(4 sigma) + 1 (9..25), Airy tiles s = 2 ceil(5 sigma) + 1
    (11..31).  Peak photons per tile are log-uniform in [10, 1000]; camera maps as in the
    filament frame.
    """
    rng = np.random.default_rng(seed)
    tiles = []
    for i in range(n_tiles):
        side = int(rng.integers(side_lo, side_hi + 1))
        if max_side is not None:
            side = min(side, max_side)
        sig = float(rng.uniform(1.0, 3.0))
        if i % 2 == 0:
            s = 2 * int(math.ceil(4 * sig)) + 1
            psf = gaussian_psf(sig, s)
        else:
            s = 2 * int(math.ceil(5 * sig)) + 1
            psf = airy_psf_matched(sig, s)
        peak = float(math.exp(rng.uniform(math.log(10.0), math.log(1000.0))))
        obj = np.full((side, side), 0.02 * peak, np.float64)
        add_beads(obj, rng, max(1, side * side // 400), scale=peak / 2)
        add_filaments(obj, rng, max(1, side // 16), scale=peak / 2 / 4)
        cam = scmos_maps(rng, side, side)
        img = simulate_frame(obj, psf, cam, rng)
        tiles.append(Frame("tile_%d" % i, img, psf, cam, obj, seed * 100003 + i, 200, 1))
    return tiles


def frame_mixed(n: int, seed: int, psf: Optional[np.ndarray] = None, n_chains: int = 1) -> Frame:
    """n x n frame with the dense frame's statistics per unit area: beads at
    5000 / 2048^2 and filaments at 2000 / 2048^2 per pixel, on a linear background
    between two levels drawn from U[1, 10] photons/px along a random direction;
    Airy 31x31 unless a PSF is given; per-pixel sCMOS maps.  Training crops for
    the learned warm start and fresh frames for its evaluation."""
    rng = np.random.default_rng(seed)
    b0, b1 = rng.uniform(1.0, 10.0, 2)
    ang = rng.uniform(0.0, 2.0 * math.pi)
    yy, xx = np.mgrid[0:n, 0:n] / max(n - 1, 1)
    t = np.clip(0.5 + (xx - 0.5) * math.cos(ang) + (yy - 0.5) * math.sin(ang), 0.0, 1.0)
    obj = b0 + (b1 - b0) * t
    area = n * n / float(2048 * 2048)
    add_beads(obj, rng, max(1, int(round(5000 * area))))
    add_filaments(obj, rng, max(1, int(round(2000 * area))))
    if psf is None:
        psf = airy_psf(AIRY_NA, AIRY_LAMBDA_UM, AIRY_PIXEL_UM, 31)
    cam = scmos_maps(rng, n, n)
    img = simulate_frame(obj, psf, cam, rng)
    return Frame("mixed_%d" % n, img, psf, cam, obj, seed, 1000, n_chains)


def frame_spokes(n: int = 128, seed: int = 10, n_spokes: int = 36, peak: float = 150.0,
                 background: float = 2.0) -> Frame:
    """A procedurally generated spoke target (a star of n_spokes alternating
    bright and dark wedges, bright value `peak` photons, on `background`),
    blurred by a pixel-integrated Gaussian PSF of NA 1.3 at 510 nm with 65 nm
    pixels (sigma = 0.21 lambda / NA), Poisson shot noise and a near-ideal
    camera (G 1, o 0, read noise 0.25): the kind of simulated test object the
    paper deconvolves with RL and with the sampler (no item of any image set)."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:n, 0:n] + 0.5 - n / 2.0
    ang = np.arctan2(yy, xx)
    rad = np.hypot(yy, xx)
    wedge = (np.floor((ang + np.pi) / (2 * np.pi) * n_spokes) % 2 == 0)
    obj = np.where(wedge & (rad < 0.45 * n), peak, background).astype(np.float64)
    sig = 0.21 * 0.510 / 1.3 / 0.065
    psf = gaussian_psf(sig, 2 * int(math.ceil(4 * sig)) + 1)
    cam = scalar_camera(1.0, 0.0, 0.25)
    img = simulate_frame(obj, psf, cam, rng)
    return Frame("spokes_%d" % n, img, psf, cam, obj, seed, 1000, 4)


def crop(fr: Frame, y0: int, x0: int, n: int) -> Frame:
    """The n x n window at (y0, x0) of a frame: raw image, camera maps and truth
    cut out, PSF unchanged.  The window is a problem of its own (the object
    outside it is not modelled), with the statistics of the frame it comes from."""
    sl = (slice(y0, y0 + n), slice(x0, x0 + n))
    cam = fr.camera
    if cam.per_pixel:
        cam = Camera(cam.gain[sl].copy(), cam.offset[sl].copy(), cam.sigma[sl].copy())
    return Frame("%s_crop%d_%d_%d" % (fr.name, n, y0, x0), fr.image[sl].copy(), fr.psf, cam, fr.truth[sl].copy(),
                 fr.seed, fr.n_sweeps, fr.n_chains)


def frame_by_name(name: str) -> Frame:
    """Named workloads used by the benchmark and the tests."""
    table = {
        "beads_segments_64": lambda: frame_beads_segments(64, 0),
        "filaments_512": lambda: frame_filaments(512, 1),
        "dense_2048": lambda: frame_dense(2048, 2),
    }
    return table[name]()

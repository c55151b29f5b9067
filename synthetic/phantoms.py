"""Seeded phantoms: projected-thickness maps of ellipsoids, a soft-tissue body with bone-like
inclusions, a bundle of parallel fibres, global scaling to stated limits, and Poisson counting noise.

All maps are float64 arrays indexed [y][x] (x is the fast axis), thickness in metres.  The
"gradient" used for scaling is a plain forward difference per pixel: it only steers the phantom
into the intended shift regime and is not the derivative operator of the method.
"""

import numpy as np
from scipy.ndimage import gaussian_filter


def _grid(ny, nx):
    """Broadcastable coordinate vectors: y is (ny, 1), x is (1, nx)."""
    return (np.arange(ny, dtype=np.float64)[:, None], np.arange(nx, dtype=np.float64)[None, :])


def _box(ny, nx, cy, cx, r):
    """Index window [y0, y1) x [x0, x1) covering a disc of radius r (clipped to the grid)."""
    y0 = max(int(np.floor(cy - r)) - 1, 0)
    y1 = min(int(np.ceil(cy + r)) + 2, ny)
    x0 = max(int(np.floor(cx - r)) - 1, 0)
    x1 = min(int(np.ceil(cx + r)) + 2, nx)
    return y0, y1, x0, x1


def _ellipse_rho2(y, x, cy, cx, ay, ax, theta):
    """Squared normalised radius of a rotated ellipse (semi-axes ax along the rotated x)."""
    c, s = np.cos(theta), np.sin(theta)
    xr = (x - cx) * c + (y - cy) * s
    yr = -(x - cx) * s + (y - cy) * c
    return (xr / ax) ** 2 + (yr / ay) ** 2


def _ellipsoid_chord(rho2, half_depth):
    """Projected thickness 2c*sqrt(1 - rho^2) of an ellipsoid with beam semi-axis c."""
    return 2.0 * half_depth * np.sqrt(np.maximum(1.0 - rho2, 0.0))


def max_forward_difference(f):
    """Largest magnitude of the forward-difference gradient of f (units of f per pixel)."""
    gx = f[:-1, 1:] - f[:-1, :-1]
    gy = f[1:, :-1] - f[:-1, :-1]
    return float(np.sqrt(gx * gx + gy * gy).max())


def forward_difference_field(f):
    gx = f[:-1, 1:] - f[:-1, :-1]
    gy = f[1:, :-1] - f[:-1, :-1]
    return gx, gy


def ellipsoid_phantom(shape, rng, n=20, centre_range=(32.0, 224.0), axis_range_px=(8.0, 40.0),
                      depth_range_m=(0.05e-3, 1.0e-3), blur_px=2.0):
    """Sum of `n` random ellipsoids (projected thickness, metres), Gaussian-blurred.

    Draw order per ellipsoid: centre y, centre x, semi-axis y, semi-axis x, angle, beam semi-axis.
    """
    ny, nx = shape
    y, x = _grid(ny, nx)
    tau = np.zeros(shape)
    for _ in range(n):
        cy = rng.uniform(*centre_range)
        cx = rng.uniform(*centre_range)
        ay = rng.uniform(*axis_range_px)
        ax = rng.uniform(*axis_range_px)
        th = rng.uniform(0.0, np.pi)
        c = rng.uniform(*depth_range_m)
        y0, y1, x0, x1 = _box(ny, nx, cy, cx, max(ay, ax))
        tau[y0:y1, x0:x1] += _ellipsoid_chord(
            _ellipse_rho2(y[y0:y1], x[:, x0:x1], cy, cx, ay, ax, th), c)
    if blur_px > 0:
        tau = gaussian_filter(tau, blur_px, mode="constant")
    return tau


def fibre_phantom(shape, rng, n=14, margin_px=40.0, radius_px=(4.0, 12.0), wobble=0.15,
                  blur_px=1.5):
    """Bamboo-like bundle of `n` parallel fibres running along y (projected thickness, in pixel
    units, unscaled).  Each fibre is the chord 2 sqrt(r(y)^2 - (x - c)^2) of a cylinder whose
    radius varies periodically along y, r(y) = r (1 + wobble sin(2 pi (y / ny + phase))), so the
    map is periodic in y and flat within `margin_px` of the left and right edges.  The sum is
    Gaussian-blurred (wrapped along y).

    Draw order per fibre: radius, centre x, phase.
    """
    ny, nx = shape
    y, x = _grid(ny, nx)
    t = np.zeros(shape)
    reach = radius_px[1] * (1.0 + wobble)
    for _ in range(n):
        r = rng.uniform(*radius_px)
        c = rng.uniform(margin_px + reach, nx - margin_px - reach)
        ph = rng.uniform()
        ry = r * (1.0 + wobble * np.sin(2.0 * np.pi * (y / ny + ph)))
        t = t + 2.0 * np.sqrt(np.maximum(ry * ry - (x - c) ** 2, 0.0))
    return gaussian_filter(t, blur_px, mode=("wrap", "constant"))


def scale_thickness(tau, max_thickness=None, max_grad_per_px=None):
    """Scale `tau` by s = min(1, max_thickness / max(tau), max_grad_per_px / max|grad tau|).

    Returns (scaled map, s).
    """
    s = 1.0
    if max_thickness is not None:
        s = min(s, max_thickness / float(tau.max()))
    if max_grad_per_px is not None:
        s = min(s, max_grad_per_px / max_forward_difference(tau))
    return tau * s, s


def soft_bone_phantom(shape, rng, pixel_m, soft_depth_m=3.0e-3, soft_blur_px=4.0,
                      texture=0.05, texture_blur_px=8.0, n_bones=12, bone_axis_frac=(0.02, 0.08),
                      bone_blur_px=0.7, shift_per_grad_soft=None, shift_per_grad_bone=None,
                      target_max_shift_px=6.0, soft_max_shift_px=4.0):
    """Soft-tissue body with sharp bone-like inclusions.

    Returns (tau_soft, tau_bone, info): two thickness maps in metres.  The soft body is an
    ellipsoid with in-plane semi-axes (0.40 nx, 0.35 ny) and beam semi-axis `soft_depth_m`,
    blurred by `soft_blur_px`, with a multiplicative texture of relative size `texture`.  Bones
    are `n_bones` ellipsoids inside the body (half of them hollow shells), blurred by
    `bone_blur_px`.

    `shift_per_grad_*` convert a thickness gradient (metres per pixel) into a displacement in
    pixels for each material.  When given, the soft body is scaled so its own largest
    displacement is at most `soft_max_shift_px`, then the bone map is scaled so that the largest
    combined displacement equals `target_max_shift_px` (bisection on the bone scale).
    """
    ny, nx = shape
    y, x = _grid(ny, nx)
    n = min(ny, nx)
    cy = ny / 2 + rng.uniform(-0.02, 0.02) * n
    cx = nx / 2 + rng.uniform(-0.02, 0.02) * n
    rho2_body = _ellipse_rho2(y, x, cy, cx, 0.35 * ny, 0.40 * nx, 0.0)
    soft = _ellipsoid_chord(rho2_body, soft_depth_m)
    soft = gaussian_filter(soft, soft_blur_px, mode="constant")
    tex = gaussian_filter(rng.standard_normal(shape), texture_blur_px, mode="wrap")
    tex /= tex.std()
    soft = soft * (1.0 + texture * tex)
    soft = np.maximum(soft, 0.0)

    bone = np.zeros(shape)
    for i in range(n_bones):
        # centre inside the body (normalised radius <= 0.6)
        r = 0.6 * np.sqrt(rng.uniform())
        phi = rng.uniform(0.0, 2.0 * np.pi)
        by = cy + r * 0.35 * ny * np.sin(phi)
        bx = cx + r * 0.40 * nx * np.cos(phi)
        ay = rng.uniform(*bone_axis_frac) * n
        ax = rng.uniform(*bone_axis_frac) * n
        th = rng.uniform(0.0, np.pi)
        depth = 0.5 * (ay + ax) * pixel_m
        y0, y1, x0, x1 = _box(ny, nx, by, bx, max(ay, ax))
        rho2 = _ellipse_rho2(y[y0:y1], x[:, x0:x1], by, bx, ay, ax, th)
        chord = _ellipsoid_chord(rho2, depth)
        if i % 2 == 1:  # hollow shell: remove a concentric ellipsoid of 0.7 the size
            chord = chord - _ellipsoid_chord(rho2 / 0.49, 0.7 * depth)
        bone[y0:y1, x0:x1] += chord
    bone = gaussian_filter(bone, bone_blur_px, mode="constant")

    info = {"soft_scale": 1.0, "bone_scale": 1.0}
    if shift_per_grad_soft is not None and shift_per_grad_bone is not None:
        sgx, sgy = forward_difference_field(soft)
        soft_max = shift_per_grad_soft * float(np.sqrt(sgx * sgx + sgy * sgy).max())
        if soft_max > soft_max_shift_px:
            f = soft_max_shift_px / soft_max
            soft *= f
            sgx *= f
            sgy *= f
            info["soft_scale"] = f
        bgx, bgy = forward_difference_field(bone)
        ux_s, uy_s = shift_per_grad_soft * sgx, shift_per_grad_soft * sgy
        ux_b, uy_b = shift_per_grad_bone * bgx, shift_per_grad_bone * bgy
        mag_s = np.sqrt(ux_s ** 2 + uy_s ** 2)
        mag_b = np.sqrt(ux_b ** 2 + uy_b ** 2)

        def max_shift(b):
            return float(np.sqrt((ux_s + b * ux_b) ** 2 + (uy_s + b * uy_b) ** 2).max())

        lo, hi = 0.0, 1.0
        while max_shift(hi) < target_max_shift_px:
            hi *= 2.0
        # only pixels whose triangle-inequality bound reaches the target at b <= hi can decide
        # the comparison with the target; bisect on those
        cand = (mag_s + hi * mag_b) >= target_max_shift_px
        ux_s, uy_s, ux_b, uy_b = ux_s[cand], uy_s[cand], ux_b[cand], uy_b[cand]
        for _ in range(50):
            mid = 0.5 * (lo + hi)
            if max_shift(mid) < target_max_shift_px:
                lo = mid
            else:
                hi = mid
        b = 0.5 * (lo + hi)
        bone *= b
        info["bone_scale"] = b
        info["max_shift_px"] = max_shift(b)
        info["soft_max_shift_px"] = float(mag_s.max())
    return soft, bone, info


def poisson_counts(intensity, photons_per_px, rng):
    """Counting noise: Poisson(photons * I) / photons (float64)."""
    lam = np.maximum(np.asarray(intensity, dtype=np.float64), 0.0) * photons_per_px
    return rng.poisson(lam).astype(np.float64) / photons_per_px

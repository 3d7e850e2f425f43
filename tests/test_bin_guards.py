"""Bins of the observables (section 2: each observable sums the weighted kernel of
the particles in one bin of a binning) and the guard bands of the FP32 decisions.

The oracle's bins are pinned to closed forms: pixel centres and shell midpoints
land in the pixel or shell they are the centre of, and points beyond a binning
land nowhere.

The fused kernel decides each bin in FP32 and re-decides in FP64 when the FP32
coordinate lies within a guard band of an edge.  The guard is twice a bound on
|f32 - f64| built from the FP32 unit roundoff u = 2^-24:
  grid x:  2 (u sx |x0| + 3u |fx|)                       (rounded origin; three roundings)
  grid y:  the same plus 2 sy (3u (|y cos i| + |z sin i|)) (rounded projection)
  radius:  12u r, plus 6u (|y cos i| + |z sin i|) for the projected radius
(plus a floor of 1e-6 bins).  These tests restate that FP32 arithmetic with numpy
float32 (IEEE round-to-nearest, like the GPU's add, multiply and fused
multiply-add; the hardware square root as the rounded root moved by up to two
ulp), with and without contraction of the projection into an FMA, on
particles packed within a few 1e-5 bins of the edges, and check against the
oracle's FP64 bins of the same FP32 particles that no decision the guard calls
sure is wrong -- and that a guard ten times narrower would be wrong somewhere
(the sample reaches the region the bound is about).
"""
import numpy as np

import oracle
from synth import configs

F32 = np.float32
U = 2.0 ** -24
FLOOR = 1e-6


# ------------------------------------------------------------------ oracle pins
def test_pixel_centres_and_outside():
    lay = configs.layout_cfg2()
    inc = lay["incl"]
    rng = np.random.default_rng(3)
    for b, d in enumerate(lay["binnings"]):
        nx, ny = d["nx"], d["ny"]
        ix, iy = rng.integers(0, nx, 500), rng.integers(0, ny, 500)
        X = d["x0"] + (ix + 0.5) * (d["x1"] - d["x0"]) / nx
        Ys = d["y0"] + (iy + 0.5) * (d["y1"] - d["y0"]) / ny
        # any (y, z) with y cos i - z sin i = Ys projects there
        z = rng.uniform(-3, 3, 500)
        y = (Ys + z * np.sin(inc)) / np.cos(inc)
        got = oracle.bins(lay, np.array([X, y, z]))[b]
        np.testing.assert_array_equal(got, iy * nx + ix)
        # beyond the grid on either axis
        Xo = np.where(rng.random(500) < 0.5, d["x0"] - 0.01, d["x1"] + 0.01)
        got = oracle.bins(lay, np.array([Xo, y, z]))[b]
        assert np.all(got == -1)


def test_shell_and_annulus_midpoints():
    lay = configs.layout_cfg1()
    rng = np.random.default_rng(4)
    for b, d in enumerate(lay["binnings"]):
        e = np.asarray(d["edges"])
        k = rng.integers(0, e.size - 1, 400)
        r = 0.5 * (e[k] + e[k + 1])
        u = rng.normal(size=(3, 400))
        u /= np.linalg.norm(u, axis=0)
        if d["kind"] == "annulus":   # line of sight along z: R = sqrt(x^2 + y^2)
            u[2] = rng.uniform(-5, 5, 400)
            n = np.hypot(u[0], u[1])
            pos = np.array([u[0] / n * r, u[1] / n * r, u[2]])
        else:
            pos = u * r
        np.testing.assert_array_equal(oracle.bins(lay, pos)[b], k)
        out = np.array([[0.0, 0.0], [0.0, 0.0], [0.0, 0.0]])
        out[0] = [0.5 * e[0], 2.0 * e[-1]]
        assert np.all(oracle.bins(lay, out)[b] == -1)


# ----------------------------------------------------------- FP32 guard bands
def _near(f, n, g):
    inside = (f > -g) & (f < F32(n) + g)
    fr = f - np.floor(f)
    return inside & ((fr < g) | (fr > F32(1.0) - g))


def _projection(incl, y, z, fused):
    cf, sf = F32(np.cos(incl)), F32(np.sin(incl))
    yc = (y * cf).astype(F32)
    zs = (z * sf).astype(F32)
    if fused:   # fma(y, cos i, -z sin i): one rounding after the exact product
        Ys = (y.astype(np.float64) * np.float64(cf) - zs.astype(np.float64)).astype(F32)
    else:
        Ys = (yc - zs).astype(F32)
    return Ys, (np.abs(yc) + np.abs(zs)).astype(F32)


def grid_fp32(d, incl, x, y, z, fused, scale=1.0):
    """The kernel's FP32 pixel and guard decision: (bin or -1, sure)."""
    x0, y0 = F32(d["x0"]), F32(d["y0"])
    sx64, sy64 = d["nx"] / (d["x1"] - d["x0"]), d["ny"] / (d["y1"] - d["y0"])
    sx, sy = F32(sx64), F32(sy64)
    Ys, aYs = _projection(incl, y, z, fused)
    fx = ((x - x0).astype(F32) * sx).astype(F32)
    fy = ((Ys - y0).astype(F32) * sy).astype(F32)
    gx = F32(scale) * (F32(2 * U * sx64 * abs(d["x0"])) + F32(6 * U) * np.abs(fx) + F32(FLOOR))
    gy = F32(scale) * (F32(2 * U * sy64 * abs(d["y0"])) + F32(6 * U * sy64) * aYs + F32(6 * U) * np.abs(fy)
                       + F32(FLOOR))
    sure = ~_near(fx, d["nx"], gx) & ~_near(fy, d["ny"], gy)
    inside = (fx >= 0) & (fx < d["nx"]) & (fy >= 0) & (fy < d["ny"])
    k = np.where(inside, np.floor(fy).astype(np.int64) * d["nx"] + np.floor(fx).astype(np.int64), -1)
    grid_fp32.guards = (gx, gy)
    return k, sure


_WIG = np.random.default_rng(11)


def _hw_sqrt(s):
    """The hardware square root: the correctly rounded root moved at random by up
    to two ulp (its measured bound on gfx950 is 1.6u relative)."""
    r = np.sqrt(s.astype(np.float64)).astype(F32)
    k = _WIG.integers(-2, 3, r.shape)
    for step in (1, 2):
        r = np.where(k >= step, np.nextafter(r, F32(np.inf)), r)
        r = np.where(k <= -step, np.nextafter(r, F32(-np.inf)), r)
    return r.astype(F32)


def radial_fp32(d, incl, x, y, z, fused, scale=1.0):
    e = np.asarray(d["edges"]).astype(F32)
    if d["kind"] == "shell":
        a, b, c = x, y, z
        extra = F32(0.0)
    else:
        Ys, aYs = _projection(incl, y, z, fused)
        a, b, c = x, Ys, np.zeros_like(x)
        extra = F32(6 * U) * aYs
    if fused:   # fma(c, c, fma(b, b, a * a))
        s = (a.astype(np.float64) * a).astype(F32)
        s = (b.astype(np.float64) * b + s).astype(F32)
        s = (c.astype(np.float64) * c + s).astype(F32)
    else:
        s = ((a * a).astype(F32) + (b * b).astype(F32)).astype(F32)
        s = (s + (c * c).astype(F32)).astype(F32)
    rad = _hw_sqrt(s)
    g = F32(scale) * (F32(12 * U) * rad + extra)
    k = np.searchsorted(e, rad, side="right") - 1
    inside = (rad >= e[0]) & (rad < e[-1])
    k = np.where(inside, k, -1)
    kk = np.clip(k, 0, e.size - 2)
    sure_in = ~((rad - e[kk]).astype(F32) < g) & ~((e[kk + 1] - rad).astype(F32) < g)
    sure_out = ~(np.abs((rad - e[0]).astype(F32)) < g) & ~(np.abs((rad - e[-1]).astype(F32)) < g)
    return k, np.where(inside, sure_in, sure_out)


def _grid_sample(d, incl, n, spread, rng):
    """Particles whose sky coordinates lie within `spread` bins of a pixel edge,
    off the sky plane by up to 10 (large |y|, |z| for the projection term)."""
    ex = rng.integers(0, d["nx"] + 1, n) + rng.uniform(-spread, spread, n)
    ey = rng.integers(0, d["ny"] + 1, n) + rng.uniform(-spread, spread, n)
    # half the sample near an x edge, half near a y edge, the other axis anywhere
    half = rng.random(n) < 0.5
    ex = np.where(half, ex, rng.uniform(0, d["nx"], n))
    ey = np.where(half, rng.uniform(0, d["ny"], n), ey)
    X = d["x0"] + ex * (d["x1"] - d["x0"]) / d["nx"]
    Ys = d["y0"] + ey * (d["y1"] - d["y0"]) / d["ny"]
    z = rng.uniform(-10, 10, n)
    y = (Ys + z * np.sin(incl)) / np.cos(incl)
    return X.astype(F32), y.astype(F32), z.astype(F32)


def _check(wrong_sure, wrong_narrow, name):
    assert wrong_sure == 0, "%s: %d sure FP32 decisions differ from FP64" % (name, wrong_sure)
    assert wrong_narrow > 0, "%s: a ten times narrower guard is never wrong: the sample misses the edges" % name


def test_grid_guards_are_sound():
    lay = configs.layout_cfg2()
    inc = lay["incl"]
    rng = np.random.default_rng(5)
    for b, d in enumerate(lay["binnings"]):
        x, y, z = _grid_sample(d, inc, 400_000, 4e-5, rng)
        ref = oracle.bins(lay, np.array([x, y, z]).astype(np.float64))[b]
        for fused in (False, True):
            k, sure = grid_fp32(d, inc, x, y, z, fused)
            kn, suren = grid_fp32(d, inc, x, y, z, fused, scale=0.1)
            _check(int(np.sum(sure & (k != ref))), int(np.sum(suren & (kn != ref))), "grid %d fused %s" % (b, fused))
        # the guards stay below the flat 1e-4 bins they replace (y: off-plane sample)
        grid_fp32(d, inc, x, y, z, True)
        gx, gy = grid_fp32.guards
        assert np.max(gx) < 3e-5 and np.mean(gy) < 5e-5, (np.max(gx), np.mean(gy))


def test_radial_guards_are_sound():
    rng = np.random.default_rng(6)
    lay = {"incl": 1.0, "binnings": [
        {"kind": "shell", "edges": np.geomspace(0.05, 10.0, 51), "moments": (0,)},
        {"kind": "annulus", "edges": np.geomspace(0.1, 10.0, 21), "moments": (0,)},
    ]}
    n = 400_000
    for b, d in enumerate(lay["binnings"]):
        e = np.asarray(d["edges"])
        r = e[rng.integers(0, e.size, n)] * (1 + rng.uniform(-3e-6, 3e-6, n))
        u = rng.normal(size=(3, n))
        u /= np.linalg.norm(u, axis=0)
        if d["kind"] == "shell":
            pos = u * r
        else:
            # projected radius r on the sky plane (X, Ys), depth along the line of sight
            th = rng.uniform(0, 2 * np.pi, n)
            X, Ys, los = r * np.cos(th), r * np.sin(th), rng.uniform(-10, 10, n)
            c, s = np.cos(lay["incl"]), np.sin(lay["incl"])
            pos = np.array([X, Ys * c + los * s, -Ys * s + los * c])
        x, y, z = pos.astype(F32)
        ref = oracle.bins(lay, np.array([x, y, z]).astype(np.float64))[b]
        for fused in (False, True):
            k, sure = radial_fp32(d, lay["incl"], x, y, z, fused)
            kn, suren = radial_fp32(d, lay["incl"], x, y, z, fused, scale=0.1)
            _check(int(np.sum(sure & (k != ref))), int(np.sum(suren & (kn != ref))), "%s fused %s" % (d["kind"], fused))

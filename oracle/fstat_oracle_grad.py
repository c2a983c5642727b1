"""FP64 gradient oracle of the resampling F-statistic.  TEST INFRASTRUCTURE ONLY.

Only the test suite and the benchmark's baseline leg may import this module.

The resampled 2F of one template (Sec. 3, steps (iii)-(vii), with the same
readings as ``fstat_oracle``) written again with PyTorch CPU float64 tensor
operations, so that reverse-mode automatic differentiation gives
d(sum_m g_m 2F_m)/d(theta) for theta = (df, f1dot, alpha, delta, asini, porb,
tp).  The fixed-point solves are iterated to convergence inside the graph, so
their derivative is that of the converged map; the floor of the fractional
sample index carries no derivative (the interpolation kernel is continuous
with a continuous derivative across integer offsets, so the result does not
depend on which side is taken).

Pinned in tests against the numpy oracle's 2F (same value) and against central
finite differences of the numpy oracle (same slope).
"""
from __future__ import annotations

import math

import numpy as np
import torch

TWO_PI = 2.0 * math.pi
PARAMS = ("df", "f1dot", "alpha", "delta", "asini", "porb", "tp")


def _t(x):
    return torch.as_tensor(x, dtype=torch.float64)


def detector_position(model, det, t):
    """Detector position (light-s), analytic ephemeris (as the numpy oracle)."""
    th = model["orbit_phase0_rad"] + TWO_PI * t / model["period_orbit_s"]
    eps = model["obliquity_rad"]
    phi = det.lon + model["sidereal_angle0_rad"] + model["sidereal_rate_rad_s"] * t
    r_o, r_e = model["r_orbit_s"], model["r_earth_s"]
    x = r_o * torch.cos(th) + r_e * math.cos(det.lat) * torch.cos(phi)
    y = r_o * torch.sin(th) * math.cos(eps) + r_e * math.cos(det.lat) * torch.sin(phi)
    z = r_o * torch.sin(th) * math.sin(eps) + r_e * math.sin(det.lat) + 0.0 * t
    return x, y, z


def roemer(model, det, nhat, t):
    x, y, z = detector_position(model, det, t)
    return nhat[0] * x + nhat[1] * y + nhat[2] * z


def binary_delay(p, t_src):
    """R(t'): circular, or Keplerian with p["ecc"], p["argp"] (held fixed;
    E from Newton's iteration on Kepler's equation run to convergence inside
    the graph, so its derivative is the converged map's)."""
    M = TWO_PI * (t_src - p["tp"]) / p["porb"]
    ecc, argp = float(p.get("ecc", 0.0)), float(p.get("argp", 0.0))
    if ecc == 0.0 and argp == 0.0:
        return p["asini"] * torch.sin(M)
    E = M + ecc * torch.sin(M)
    for _ in range(40):
        E = E - (E - ecc * torch.sin(E) - M) / (1.0 - ecc * torch.cos(E))
    return p["asini"] * (math.sin(argp) * (torch.cos(E) - ecc) +
                         math.cos(argp) * math.sqrt(1.0 - ecc * ecc) * torch.sin(E))


def emission_delay(p, t_b, iters=60):
    """R(t_src) with t_src + R(t_src) = t_b, fixed point."""
    r = torch.zeros_like(t_b)
    for _ in range(iters):
        r = binary_delay(p, t_b - r)
    return r


def detector_delay(model, det, nhat, p, tau, iters=12):
    """T - tau where T + roemer(T) = tau + R(tau), fixed point."""
    rb = binary_delay(p, tau)
    t_b = tau + rb
    dr = roemer(model, det, nhat, t_b)
    for _ in range(iters):
        dr = roemer(model, det, nhat, t_b - dr)
    return rb - dr


def sinc_kernel(s, D):
    h = torch.sinc(s) * 0.5 * (1.0 + torch.cos(math.pi * s / D))
    return torch.where(torch.abs(s) < D, h, torch.zeros_like(s))


def interpolate(z, u, D):
    j0 = torch.floor(u.detach()).to(torch.int64)
    n = z.shape[0]
    out = torch.zeros(u.shape, dtype=torch.complex128)
    for i in range(2 * D):
        j = j0 - D + 1 + i
        ok = (j >= 0) & (j < n)
        w = sinc_kernel(u - j.to(torch.float64), D)
        zj = z[torch.clamp(j, 0, n - 1)]
        out = out + torch.where(ok, w.to(torch.complex128) * zj, torch.zeros_like(zj))
    return out


def antenna_ab(model, det, alpha, delta, t):
    """JKS a(t), b(t) (as the numpy oracle)."""
    lam = det.lat
    gam = 0.5 * (det.az_x + det.az_y)
    x = alpha - (det.lon + model["sidereal_angle0_rad"] + model["sidereal_rate_rad_s"] * t)
    s2g, c2g = math.sin(2 * gam), math.cos(2 * gam)
    sl, cl = math.sin(lam), math.cos(lam)
    s2l, c2l = math.sin(2 * lam), math.cos(2 * lam)
    sd, cd = torch.sin(delta), torch.cos(delta)
    s2d, c2d = torch.sin(2 * delta), torch.cos(2 * delta)
    a = (s2g * (3 - c2l) * (3 - c2d) * torch.cos(2 * x) / 16.0
         - c2g * sl * (3 - c2d) * torch.sin(2 * x) / 4.0
         + s2g * s2l * s2d * torch.cos(x) / 4.0
         - c2g * cl * s2d * torch.sin(x) / 2.0
         + 0.75 * s2g * cl * cl * cd * cd)
    b = (c2g * sl * sd * torch.cos(2 * x)
         + s2g * (3 - c2l) * sd * torch.sin(2 * x) / 4.0
         + c2g * cl * cd * torch.cos(x)
         + s2g * s2l * cd * torch.sin(x) / 2.0)
    return a, b


def twoF_torch(ds, p):
    """2F over the output band for parameters p (dict of 0-d float64 tensors,
    keys as PARAMS plus f2dot)."""
    model = ds.ephem_model
    nhat = torch.stack([torch.cos(p["delta"]) * torch.cos(p["alpha"]),
                        torch.cos(p["delta"]) * torch.sin(p["alpha"]),
                        torch.sin(p["delta"])])
    k = torch.arange(ds.n_fft, dtype=torch.float64)
    tau = ds.tau0 + ds.dt * k
    ya = torch.zeros(ds.n_fft, dtype=torch.complex128)
    yb = torch.zeros(ds.n_fft, dtype=torch.complex128)
    A = B = C = 0.0
    for det, x, v in zip(ds.detectors, ds.x, ds.valid):
        t = det.t0 + ds.dt * torch.arange(det.n, dtype=torch.float64)
        xv = torch.as_tensor(np.asarray(x, dtype=np.complex128))
        # (iii) correction at the input samples
        roem = roemer(model, det, nhat, t)
        rbin = emission_delay(p, t + roem)
        cyc = ds.f_het * (roem - rbin)
        z = xv * torch.exp(-1j * TWO_PI * (cyc - torch.round(cyc.detach())))
        # (iv) detector epochs of the grid, (v) interpolation
        delay = detector_delay(model, det, nhat, p, tau)
        u = k + (ds.tau0 - det.t0) / ds.dt + delay / ds.dt
        zh = interpolate(z, u, ds.sinc_halfwidth)
        a, b = antenna_ab(model, det, p["alpha"], p["delta"], tau + delay)
        w = 1.0 / det.noise_var
        ya = ya + w * a * zh
        yb = yb + w * b * zh
        # A, B, C over the valid detector samples
        aa, bb = antenna_ab(model, det, p["alpha"], p["delta"], t)
        m = torch.as_tensor(np.asarray(v, dtype=np.float64))
        A = A + w * torch.sum(m * aa * aa)
        B = B + w * torch.sum(m * bb * bb)
        C = C + w * torch.sum(m * aa * bb)
    dtr = tau - ds.t_ref
    cyc = p["f1dot"] * dtr ** 2 / 2.0 + p["f2dot"] * dtr ** 3 / 6.0 + p["df"] * (tau - ds.tau0)
    rot = torch.exp(-1j * TWO_PI * (cyc - torch.round(cyc.detach())))
    Fa = torch.fft.fftshift(torch.fft.fft(ya * rot))[ds.bin_lo:ds.bin_lo + ds.n_bins]
    Fb = torch.fft.fftshift(torch.fft.fft(yb * rot))[ds.bin_lo:ds.bin_lo + ds.n_bins]
    D = A * B - C * C
    return 2.0 * (B * torch.abs(Fa) ** 2 + A * torch.abs(Fb) ** 2
                  - 2.0 * C * torch.real(Fa * torch.conj(Fb))) / D


def template_params(row):
    names = ("alpha", "delta", "df", "f1dot", "f2dot", "asini", "porb", "tp")
    p = {n: _t(float(v)) for n, v in zip(names, row)}
    if len(row) >= 10:
        p["ecc"], p["argp"] = float(row[8]), float(row[9])
    return p


def oracle_grad(ds, row, weights):
    """(2F, d(sum_m weights_m 2F_m)/d theta) for one template row, theta in
    PARAMS order.  For an isolated source (asini = 0) the orbit is not a
    parameter of the template: its three derivatives are reported as zero."""
    p = template_params(row)
    for n in PARAMS:
        p[n].requires_grad_(True)
    tf = twoF_torch(ds, p)
    loss = torch.sum(_t(np.asarray(weights, dtype=np.float64)) * tf)
    grads = torch.autograd.grad(loss, [p[n] for n in PARAMS], allow_unused=True)
    g = np.array([0.0 if gr is None else float(gr) for gr in grads])
    if float(row[5]) == 0.0:
        g[4:7] = 0.0
    return tf.detach().numpy(), g

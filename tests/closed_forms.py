"""Closed-form and quadrature references that pin the oracle (fp64, numpy/scipy).

Each function states the textbook result it evaluates.  None of them calls the
oracle or the GPU library.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special

LN10 = math.log(10.0)


# ---------------------------------------------------------------- spectra
def grid_lambda(n_bins, lo=300.0, hi=800.0):
    return lo + (hi - lo) / (n_bins - 1) * np.arange(n_bins)


def gauss_mix(lam, terms):
    lam = np.asarray(lam, float)
    return sum(w * np.exp(-0.5 * ((lam - mu) / sd) ** 2) for mu, sd, w in terms)


def emission_pmf(n_bins, terms):
    e = gauss_mix(grid_lambda(n_bins), terms)
    return e / e.sum()


def dye_sigma_a(lam, terms, epsilon, conc_uM, n_bins, decadic=True):
    """Dye absorption coefficient in 1/mm: (ln10) * eps[1/(M cm)] * c[uM] * 1e-7 * a_hat."""
    grid = grid_lambda(n_bins)
    peak = gauss_mix(grid, terms).max()
    base = LN10 if decadic else 1.0
    return base * epsilon * conc_uM * 1e-7 * gauss_mix(lam, terms) / peak


# ---------------------------------------------------------------- slab optics
def half_e2(tau):
    """Escape probability of an isotropic emitter at optical depth tau below a
    free surface, uncollided: (1/2) E_2(tau)."""
    return 0.5 * special.expn(2, tau)


def dye_slab_fluorescent_film(d, sig_t_x, sig_a_dye_x, qy, pmf, sig_t_em):
    """Non-scattering dye slab [0, d], collimated beam at excitation wavelength.

    First collisions at depth z have density sig_t_x * exp(-sig_t_x z); the dye
    takes a fraction sig_a_dye_x / sig_t_x; emission with probability qy at
    bin k with probability pmf[k], isotropic; the fluorescent photon escapes
    uncollided with probability E_2/2 of its optical distance to each face.
    Returns (R[k], T[k]) as fractions of source photons."""
    R = np.zeros(len(pmf))
    T = np.zeros(len(pmf))
    for k in range(len(pmf)):
        if pmf[k] < 1e-300:
            continue
        st = sig_t_em[k]
        fr = lambda z: math.exp(-sig_t_x * z) * half_e2(st * z)  # noqa: E731
        ft = lambda z: math.exp(-sig_t_x * z) * half_e2(st * (d - z))  # noqa: E731
        R[k] = qy * pmf[k] * sig_a_dye_x * integrate.quad(fr, 0.0, d, limit=200)[0]
        T[k] = qy * pmf[k] * sig_a_dye_x * integrate.quad(ft, 0.0, d, limit=200)[0]
    return R, T


def single_scatter_slab(tau, albedo=1.0):
    """Slab of optical thickness tau, normal collimated beam, isotropic phase.
    Probability that a photon scatters exactly once and leaves through the
    lit face (R1) or the far face (T1) without further collision."""
    r1 = integrate.quad(lambda mu: mu / (1 + mu) * (1 - math.exp(-tau * (1 + 1 / mu))),
                        0.0, 1.0, limit=200)[0]

    def t_int(mu):
        # int_0^tau exp(-t) exp(-(tau-t)/mu) dt
        if abs(mu - 1.0) < 1e-12:
            return tau * math.exp(-tau)
        a = 1.0 - 1.0 / mu
        return math.exp(-tau / mu) * (1 - math.exp(-a * tau)) / a

    t1 = integrate.quad(t_int, 0.0, 1.0, limit=200)[0]
    return 0.5 * albedo * r1, 0.5 * albedo * t1


def chandrasekhar_h(omega, mu, n=200, iters=20000, tol=1e-14):
    """H-function for isotropic scattering with single-scattering albedo omega,
    from the alternative form of its integral equation:
        1/H(mu) = sqrt(1-omega) + (omega/2) int_0^1 mu' H(mu') / (mu + mu') dmu'.
    Solved by damped fixed-point iteration on a Gauss-Legendre grid (fp64)."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    s = math.sqrt(max(0.0, 1.0 - omega))
    H = np.ones(n)
    K = (omega / 2.0) * (w * x)[None, :] / (x[:, None] + x[None, :])
    for _ in range(iters):
        # damped: the undamped map oscillates with period two near omega = 1
        Hn = 0.5 * (H + 1.0 / (s + K @ H))
        if np.max(np.abs(Hn - H)) < tol:
            H = Hn
            break
        H = Hn
    mu = np.atleast_1d(np.asarray(mu, float))
    Km = (omega / 2.0) * (w * x)[None, :] / (mu[:, None] + x[None, :])
    out = 1.0 / (s + Km @ H)
    return out, (x, w, H)


def halfspace_albedo(omega):
    """Total reflectance of a semi-infinite isotropically scattering medium under
    a normal collimated beam: 1 - H(1) sqrt(1 - omega) (Chandrasekhar)."""
    h1, _ = chandrasekhar_h(omega, [1.0])
    return 1.0 - h1[0] * math.sqrt(1.0 - omega)


# ---------------------------------------------------------------- camera
class Pinhole:
    def __init__(self, eye, look, up, fov_y_deg, width, height):
        self.eye = np.asarray(eye, float)
        f = np.asarray(look, float) - self.eye
        self.f = f / np.linalg.norm(f)
        r = np.cross(self.f, np.asarray(up, float))
        self.r = r / np.linalg.norm(r)
        self.u = np.cross(self.r, self.f)
        self.tany = math.tan(math.radians(fov_y_deg) / 2)
        self.tanx = self.tany * width / height
        self.W, self.H = width, height

    def ray(self, px, py):
        """Unit direction through image position (px, py) in pixel units."""
        xi = 2.0 * px / self.W - 1.0
        yi = 1.0 - 2.0 * py / self.H
        d = self.f + xi * self.tanx * self.r + yi * self.tany * self.u
        return d / np.linalg.norm(d)


def ray_box_exit(o, d, lo, hi):
    t = np.inf
    for a in range(3):
        if d[a] > 0:
            t = min(t, (hi[a] - o[a]) / d[a])
        elif d[a] < 0:
            t = min(t, (lo[a] - o[a]) / d[a])
    return t


def ray_plane_rect(o, d, corner, u, v):
    """Distance along ray to the parallelogram corner + a u + b v, or inf."""
    n = np.cross(u, v)
    dn = n @ d
    if dn == 0:
        return np.inf
    t = n @ (corner - o) / dn
    if t <= 0:
        return np.inf
    q = o + t * d - corner
    a = q @ u / (u @ u)
    b = q @ v / (v @ v)
    return t if (0 <= a <= 1 and 0 <= b <= 1) else np.inf


def ray_sphere(o, d, c, r):
    oc = o - c
    b = oc @ d
    cc = oc @ oc - r * r
    disc = b * b - cc
    if disc <= 0:
        return np.inf, np.inf
    s = math.sqrt(disc)
    return -b - s, -b + s


def quad_irradiance(x, normal, corner, u, v, radiance, n=48, medium=None):
    """Irradiance at x (surface normal `normal`, or None for the
    direction-independent integral int L cos_l T / r^2 dA seen by an isotropic
    scatterer) from a Lambertian parallelogram of radiance L, by Gauss-Legendre
    quadrature.  `medium` = (center, radius, sigma_t): attenuate the light
    through that sphere (Beer-Lambert along the chord)."""
    x = np.asarray(x, float)
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1)
    w = 0.5 * w
    nl = np.cross(u, v)
    area = np.linalg.norm(nl)
    nl = nl / area
    A, B = np.meshgrid(g, g, indexing="ij")
    W = np.outer(w, w)
    y = corner[None, None, :] + A[..., None] * u + B[..., None] * v
    dv = y - x
    r2 = (dv * dv).sum(-1)
    r = np.sqrt(r2)
    dirn = dv / r[..., None]
    cl = -(dirn @ nl)
    cx = np.ones_like(cl) if normal is None else dirn @ np.asarray(normal, float)
    ok = (cl > 0) & (cx > 0)
    tr = np.ones_like(cl)
    if medium is not None:
        c, rad, st = medium
        oc = x - np.asarray(c, float)
        b = dirn @ oc
        cc = oc @ oc - rad * rad
        disc = b * b - cc
        sq = np.sqrt(np.maximum(disc, 0.0))
        lo = np.maximum(-b - sq, 0.0)
        hi = np.minimum(-b + sq, r)
        ln = np.where((disc > 0) & (hi > lo), hi - lo, 0.0)
        tr = np.exp(-st * ln)
    val = np.where(ok, W * radiance * cl * cx * tr / r2, 0.0)
    return float(val.sum() * area)


def single_scatter_radiance(eye, d, c, rad, sig_s, sig_t, corner, u, v, radiance,
                            n_line=24, n_quad=32):
    """Radiance along the camera ray (eye, d) from photons scattered exactly once
    inside a sphere lit by a Lambertian quad (isotropic phase 1/4pi):
      L = int_{ray in sphere} T(eye, x) sigma_s/(4 pi) int_quad L_e T(x, y) cos_l / r^2 dA dt."""
    t0, t1 = ray_sphere(eye, d, np.asarray(c, float), rad)
    if not np.isfinite(t0):
        return 0.0
    g, w = np.polynomial.legendre.leggauss(n_line)
    ts = t0 + (t1 - t0) * 0.5 * (g + 1)
    ws = (t1 - t0) * 0.5 * w
    tot = 0.0
    for t, wt in zip(ts, ws):
        x = eye + t * d
        q = quad_irradiance(x, None, corner, u, v, radiance, n=n_quad, medium=(c, rad, sig_t))
        tot += wt * math.exp(-sig_t * (t - t0)) * q
    return sig_s / (4 * math.pi) * tot


# ---------------------------------------------------------------- dielectric boundaries
def fresnel_unpolarised(ci, n1, n2):
    """Reflectance of a smooth dielectric interface for unpolarised light going
    from index n1 into n2 at incidence cosine ci: the mean of the s and p
    intensities in their angle form (Born & Wolf 1.5.2)
        R_s = sin^2(ti - tt) / sin^2(ti + tt),  R_p = tan^2(ti - tt) / tan^2(ti + tt),
    with sin tt = (n1/n2) sin ti; 1 beyond the critical angle and
    ((n1 - n2)/(n1 + n2))^2 at normal incidence (the limit of both)."""
    ci = min(max(float(ci), 0.0), 1.0)
    ti = math.acos(ci)
    st = n1 / n2 * math.sin(ti)
    if st >= 1.0:
        return 1.0
    if ti < 1e-9:
        return ((n1 - n2) / (n1 + n2)) ** 2
    tt = math.asin(st)
    rs = math.sin(ti - tt) ** 2 / math.sin(ti + tt) ** 2
    rp = math.tan(ti - tt) ** 2 / math.tan(ti + tt) ** 2
    return 0.5 * (rs + rp)


def dielectric_slab_beam(n, ci, sigma, d):
    """(R, T) of a beam entering a non-scattering, absorbing slab (index n,
    thickness d, vacuum outside) at incidence cosine ci: incoherent multiple
    reflections between the faces, reflectance r at every encounter (the same
    inside, by reciprocity) and attenuation q = exp(-sigma d / ct) per crossing:
        R = r + (1-r)^2 r q^2 / (1 - r^2 q^2),   T = (1-r)^2 q / (1 - r^2 q^2)."""
    r = fresnel_unpolarised(ci, 1.0, n)
    ct = math.sqrt(1.0 - (1.0 - ci * ci) / (n * n))
    q = math.exp(-sigma * d / ct)
    den = 1.0 - r * r * q * q
    return r + (1 - r) ** 2 * r * q * q / den, (1 - r) ** 2 * q / den


def dielectric_slab_point(n, sigma, d, zs):
    """(bottom, top) escape fractions of an isotropic point source at height zs
    in a non-scattering absorbing slab [0, d] of index n: a ray of direction
    cosine mu keeps |mu| at every face, reflects with r(|mu|) (1 under total
    internal reflection) and is attenuated by exp(-sigma L); summing the
    bounces, a ray heading for the top first escapes there with
    (1-r) q_a / (1 - r^2 q_d^2) and at the bottom with (1-r) r q_a q_d / (1 - r^2 q_d^2),
    q_a = exp(-sigma (d - zs)/mu), q_d = exp(-sigma d/mu); averaged over mu
    uniform in (0, 1] for each hemisphere (weight 1/2)."""
    def parts(mu, first):
        r = fresnel_unpolarised(mu, n, 1.0)
        qa = math.exp(-sigma * first / mu)
        qd = math.exp(-sigma * d / mu)
        den = 1.0 - r * r * qd * qd
        return (1 - r) * qa / den, (1 - r) * r * qa * qd / den
    mc = math.sqrt(max(0.0, 1.0 - 1.0 / (n * n)))  # critical direction cosine
    def integ(f):
        lo = integrate.quad(f, 1e-12, mc, limit=200)[0] if mc > 0 else 0.0
        return lo + integrate.quad(f, mc, 1.0, limit=200)[0]
    top = 0.5 * integ(lambda mu: parts(mu, d - zs)[0]) + 0.5 * integ(lambda mu: parts(mu, zs)[1])
    bot = 0.5 * integ(lambda mu: parts(mu, zs)[0]) + 0.5 * integ(lambda mu: parts(mu, d - zs)[1])
    return bot, top


def dielectric_sphere_point(n, sigma, a, s):
    """Escape fraction of an isotropic point source at distance s from the
    centre of a non-scattering absorbing sphere of radius a and index n: a
    chord's impact parameter b = s sin(psi) is kept at every specular bounce,
    so the incidence (sin = b/a) is too, and
        escape = (1 - r) exp(-sigma L1) / (1 - r exp(-sigma C)),
    L1 = -s mu + sqrt(a^2 - b^2) to the first hit, C = 2 sqrt(a^2 - b^2), r the
    reflectance at that incidence (1 beyond the critical angle); averaged over
    mu = cos(psi) uniform in [-1, 1]."""
    def f(mu):
        b2 = s * s * (1.0 - mu * mu)
        h = math.sqrt(a * a - b2)
        r = fresnel_unpolarised(h / a, n, 1.0)
        return 0.5 * (1 - r) * math.exp(-sigma * (h - s * mu)) / (1.0 - r * math.exp(-sigma * 2 * h))
    # the critical impact parameter a/n splits the integrand where r reaches 1
    pts = []
    if s > a / n:
        mc = math.sqrt(1.0 - (a / n / s) ** 2)
        pts = [-mc, mc]
    return integrate.quad(f, -1.0, 1.0, points=pts or None, limit=200)[0]


def phong_lobe(n, wi, wo, normal, about_normal=False):
    """Normalised modified-Phong lobe over rho: (n+2)/(2 pi) cos^n(alpha), alpha
    between the outgoing direction wo and the mirror direction of the incoming
    travel direction wi about the wall normal (arrays of directions on the
    last axis; 0 where wo leaves through the back of the wall)."""
    wi, wo, normal = (np.asarray(a, float) for a in (wi, wo, normal))
    r = normal if about_normal else wi - 2.0 * (wi @ normal)[..., None] * normal
    c = np.maximum((r * wo).sum(-1), 0.0)
    return np.where((wo @ normal) > 0, (n + 2.0) / (2.0 * math.pi) * c ** n, 0.0)


def hemisphere_integral(fn, normal, n_theta=256, n_phi=256):
    """int over the hemisphere about `normal` of fn(w) cos(theta) dw, by
    Gauss-Legendre in cos(theta) and the trapezoid rule in phi (fn takes an
    array of directions)."""
    normal = np.asarray(normal, float)
    t1 = np.cross(normal, [1.0, 0.0, 0.0] if abs(normal[0]) < 0.9 else [0.0, 1.0, 0.0])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(normal, t1)
    g, wg = np.polynomial.legendre.leggauss(n_theta)
    mu = 0.5 * (g + 1.0)
    wmu = 0.5 * wg
    ph = (np.arange(n_phi) + 0.5) * 2.0 * math.pi / n_phi
    MU, PH = np.meshgrid(mu, ph, indexing="ij")
    S = np.sqrt(1.0 - MU * MU)
    w = (S * np.cos(PH))[..., None] * t1 + (S * np.sin(PH))[..., None] * t2 + MU[..., None] * normal
    vals = fn(w) * MU
    return float((vals * wmu[:, None]).sum() * 2.0 * math.pi / n_phi)


def glossy_wall_radiance(x, normal, w_eye, corner, u, v, radiance, rho, n_exp, n=64,
                         about_normal=False):
    """Radiance leaving a glossy wall point x toward w_eye (unit, from x) when
    the wall is lit only by a Lambertian parallelogram of radiance L:
    int_quad rho lobe(wi, w_eye) L cos_x cos_l / r^2 dA, wi the direction from
    the light point to x, by Gauss-Legendre quadrature over the quad."""
    x = np.asarray(x, float)
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1)
    w = 0.5 * w
    nl = np.cross(u, v)
    area = np.linalg.norm(nl)
    nl = nl / area
    A, B = np.meshgrid(g, g, indexing="ij")
    W = np.outer(w, w)
    y = corner[None, None, :] + A[..., None] * u + B[..., None] * v
    dv = x - y
    r2 = (dv * dv).sum(-1)
    wi = dv / np.sqrt(r2)[..., None]
    cl = wi @ nl
    cx = -(wi @ np.asarray(normal, float))
    f = rho * phong_lobe(n_exp, wi, np.broadcast_to(w_eye, wi.shape), normal, about_normal)
    val = np.where((cl > 0) & (cx > 0), f * radiance * cl * cx / r2, 0.0)
    return float((val * W).sum() * area)

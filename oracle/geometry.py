"""Star-family surfaces (optionally stretched along the axes) and the
cancellation-free point difference (oracle).

Surface (Sec. 2, eq. (2.1)): the paper's parametrisation r(t, theta) with
t in [0, L] along a generating curve and theta the 2*pi-periodic azimuth.  The
family used here is the radial perturbation of the unit sphere

    r(t, theta) = R(t, theta) * (sin t cos theta, sin t sin theta, cos t),
    R(t, theta) = 1 + sum_{l=1..lmax} sum_{m=0..mmax} a[l-1, m] sin(l t) cos(m theta),

with L = pi.  An empty amplitude table gives the unit sphere.

``delta_r`` evaluates r(v) - r(u) through the line integral of Remark 4.2,
    r(v) - r(u) = - int_0^1 Dr(v + lam (u - v)) [u - v] d lam,
by Gauss-Legendre quadrature in lam, which avoids the cancellation of the
direct difference when the two points are close (the paper uses 16 nodes;
the oracle uses 32).  Test infrastructure only.
"""
import numpy as np

_LAM_CACHE = {}


def _gl01(n):
    """Gauss-Legendre nodes/weights on [0, 1] (numpy's Golub-Welsch rule)."""
    if n not in _LAM_CACHE:
        x, w = np.polynomial.legendre.leggauss(n)
        _LAM_CACHE[n] = (0.5 * (x + 1.0), 0.5 * w)
    return _LAM_CACHE[n]


class Scaled:
    """A star surface stretched along the coordinate axes (the ellipsoid of
    Sec. 5, Example 1, is the unit sphere with axes (1, 2, 3)):
        r(t, theta) = D R(t, theta) omega(t, theta),  D = diag(axes).
    Every function of this module takes either a plain amplitude table or a
    Scaled surface."""

    def __init__(self, amp, axes):
        self.amp = as_amp(amp)
        self.axes = np.asarray(axes, dtype=np.float64).reshape(3)
        if not np.all(self.axes > 0):
            raise ValueError("axes must be positive")


def axes_of(surface):
    """The stretch D of a surface (ones for a plain amplitude table)."""
    return surface.axes if isinstance(surface, Scaled) else np.ones(3)


def is_axisymmetric(surface):
    """Rotation-invariant about the z axis: no amplitudes and equal x, y axes."""
    a, d = as_amp(surface), axes_of(surface)
    return not np.any(a) and d[0] == d[1]


def as_amp(amp):
    """Amplitude table as a float64 array of shape (lmax, mmax+1)."""
    if isinstance(amp, Scaled):
        return amp.amp
    if amp is None:
        return np.zeros((0, 1))
    a = np.asarray(amp, dtype=np.float64)
    if a.ndim != 2:
        raise ValueError("amplitude table must be 2-D [lmax][mmax+1]")
    return a


def radius(amp, t, th, dt=0, dth=0):
    """Partial derivative d^dt/dt^dt d^dth/dth^dth of R(t, theta)."""
    a = as_amp(amp)
    t = np.asarray(t, dtype=np.float64)
    th = np.asarray(th, dtype=np.float64)
    out = np.full(np.broadcast(t, th).shape, 1.0 if (dt == 0 and dth == 0) else 0.0)
    lmax, mp1 = a.shape
    for l in range(1, lmax + 1):
        # d^j/dt^j sin(l t) = l^j sin(l t + j pi/2)
        st = l ** dt * np.sin(l * t + dt * np.pi / 2)
        for m in range(mp1):
            if a[l - 1, m] == 0.0:
                continue
            cm = m ** dth * np.cos(m * th + dth * np.pi / 2) if dth else np.cos(m * th)
            out = out + a[l - 1, m] * st * cm
    return out


def _omega(t, th, dt=0, dth=0):
    """Derivatives of the unit vector (sin t cos th, sin t sin th, cos t)."""
    st = np.sin(t + dt * np.pi / 2)
    ct = np.cos(t + dt * np.pi / 2)
    cth = np.cos(th + dth * np.pi / 2)
    sth = np.sin(th + dth * np.pi / 2)
    z = ct if dth == 0 else np.zeros_like(ct * cth)
    return np.stack(np.broadcast_arrays(st * cth, st * sth, z), axis=-1)


def point(amp, t, th):
    """r(t, theta), shape (..., 3)."""
    return axes_of(amp) * (radius(amp, t, th)[..., None] * _omega(t, th))


def derivs(amp, t, th):
    """(r_t, r_theta) at (t, theta), each shape (..., 3)."""
    D = axes_of(amp)
    R = radius(amp, t, th)[..., None]
    Rt = radius(amp, t, th, dt=1)[..., None]
    Rth = radius(amp, t, th, dth=1)[..., None]
    rt = Rt * _omega(t, th) + R * _omega(t, th, dt=1)
    rth = Rth * _omega(t, th) + R * _omega(t, th, dth=1)
    return D * rt, D * rth


def second_theta(amp, t, th):
    """r_{theta theta}(t, theta), shape (..., 3)."""
    R = radius(amp, t, th)[..., None]
    Rth = radius(amp, t, th, dth=1)[..., None]
    Rthth = radius(amp, t, th, dth=2)[..., None]
    return axes_of(amp) * (Rthth * _omega(t, th) + 2.0 * Rth * _omega(t, th, dth=1)
                           + R * _omega(t, th, dth=2))


def second_derivs(amp, t, th):
    """(r_tt, r_t theta, r_theta theta) at (t, theta), each shape (..., 3)."""
    R = radius(amp, t, th)[..., None]
    Rt = radius(amp, t, th, dt=1)[..., None]
    Rth = radius(amp, t, th, dth=1)[..., None]
    Rtt = radius(amp, t, th, dt=2)[..., None]
    Rtth = radius(amp, t, th, dt=1, dth=1)[..., None]
    Rthth = radius(amp, t, th, dth=2)[..., None]
    w, wt, wth = _omega(t, th), _omega(t, th, dt=1), _omega(t, th, dth=1)
    rtt = Rtt * w + 2.0 * Rt * wt + R * _omega(t, th, dt=2)
    rtth = Rtth * w + Rt * wth + Rth * wt + R * _omega(t, th, dt=1, dth=1)
    rthth = Rthth * w + 2.0 * Rth * wth + R * _omega(t, th, dth=2)
    D = axes_of(amp)
    return D * rtt, D * rtth, D * rthth


def jacobian(amp, t, th):
    """J = |r_t x r_theta| (assumption (iii) of Sec. 2)."""
    rt, rth = derivs(amp, t, th)
    return np.linalg.norm(np.cross(rt, rth), axis=-1)


def normal(amp, t, th):
    """Unit normal (r_t x r_theta)/J; outward for this family."""
    rt, rth = derivs(amp, t, th)
    n = np.cross(rt, rth)
    return n / np.linalg.norm(n, axis=-1, keepdims=True)


def wrap(x):
    """Reduce an angle difference to (-pi, pi].

    Values already in range are returned unchanged (shifting them by pi and
    back would round away a small difference).
    """
    x = np.asarray(x, dtype=np.float64)
    shifted = -((-x + np.pi) % (2.0 * np.pi) - np.pi)
    return np.where((x > -np.pi) & (x <= np.pi), x, shifted)


def delta_r(amp, t, th, ts, dth, n_lambda=32, switch=0.5):
    """r(ts, th + dth) - r(t, th) without cancellation (Remark 4.2).

    The source azimuth is given by its offset ``dth`` from the target azimuth,
    so that a small offset is never rounded against the size of ``th``.  For
    |ts - t| + |wrap(dth)| < ``switch`` the line integral over the straight
    segment in parameter space is used, otherwise the direct difference (which
    is then accurate).  Broadcasts over all arguments.
    """
    t, th, ts, dth = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64)
                                           for v in (t, th, ts, dth)))
    dt = t - ts
    w = wrap(dth)
    near = (np.abs(dt) + np.abs(w)) < switch
    out = point(amp, ts, th + dth) - point(amp, t, th)
    if np.any(near):
        lam, wl = _gl01(n_lambda)
        tn, thn, dtn, wn = t[near], th[near], dt[near], w[near]
        # u = (t, th), v = (ts, th + w), u - v = (dt, -w), gamma = v + lam (u - v)
        g_t = (tn - dtn)[:, None] + lam[None, :] * dtn[:, None]
        g_th = thn[:, None] + (wn[:, None] - lam[None, :] * wn[:, None])
        rt, rth = derivs(amp, g_t, g_th)
        integrand = rt * dtn[:, None, None] - rth * wn[:, None, None]
        out[near] = -np.einsum('k,nkc->nc', wl, integrand)
    return out


def rho2(amp, t, th, ts, dth, **kw):
    """Squared distance rho^2 of eq. (3.21) at source azimuth th + dth,
    evaluated without cancellation."""
    d = delta_r(amp, t, th, ts, dth, **kw)
    return np.einsum('...c,...c->...', d, d)


def rho2_theta_derivs(amp, t, th, ts, dth, **kw):
    """(rho^2, d rho^2/d theta_s, d^2 rho^2/d theta_s^2) at theta_s = th + dth."""
    d = delta_r(amp, t, th, ts, dth, **kw)
    ths = th + dth
    rs_th = derivs(amp, ts, ths)[1]
    rs_thth = second_theta(amp, ts, ths)
    r2 = np.einsum('...c,...c->...', d, d)
    d1 = 2.0 * np.einsum('...c,...c->...', d, rs_th)
    d2 = 2.0 * (np.einsum('...c,...c->...', rs_th, rs_th)
                + np.einsum('...c,...c->...', d, rs_thth))
    return r2, d1, d2

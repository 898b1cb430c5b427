"""FP64 NumPy oracle of the registration on SE(n) for any n (TEST
INFRASTRUCTURE ONLY; tiny inputs).

Points live in R^n; the group SE(n) acts by h.x = R x + T.  Written from the
paper's general-n section (Sec. IV): the objective of eq. scalar with the
squared-exponential kernel, the infinitesimal generator xi_M x = Omega x + v
(Sec. IV-A), and the gradient in the coordinates of eq. flow:

    w^{pq} = 1/(a^2 l^2) sum_ij c_ij k_ij (x_i^p z~_j^q - x_i^q z~_j^p),   p < q
    v^m    = 1/(b^2 l^2) sum_ij c_ij k_ij (z~_j^m - x_i^m)

with z~_j = h^-1 z_j.  Readings (the same as for n = 3):
  * v: the sign of the kernel's derivative (the printed x - z~ is opposite);
  * the metric: the paper states that its normalisation makes the
    generators J^{pq} = E_pq - E_qp orthonormal (a = 1), which is what the
    coefficients of eq. flow assume; the printed factor (n - 2)/2 of the
    trace form gives that only for n = 3 (for n = 2 it vanishes).  Here the
    rotational part of the metric is -(a^2 / 2) tr(Omega Omega'), i.e.
    <J^{pq}, J^{rs}> = a^2 delta, and the translational part b^2 <v, v'>;
  * the direction of steepest ascent in so(n) is Omega = sum_{p<q} w^{pq}
    (E_qp - E_pq): with Omega = sum theta^{pq} J^{pq} the differential is
    dF = (1/l^2) sum c k (z~ - x) . (Omega z~ + v), whose J^{pq} component is
    (1/l^2) sum c k (x^q z~^p - x^p z~^q) = -a^2 w^{pq}.  For n = 3 this is
    the hat map of omega = (w^{23}, -w^{13}, w^{12}) = (w^{23}, w^{31}, w^{12}).
The step is h <- h exp(tau xi), xi = (Omega, v) as the (n+1) x (n+1) twist,
exp by a scaled and squared Taylor series (Sec. VI-A: the group exponential
is the matrix exponential), tau = eta l^2 / F.
"""
from __future__ import annotations

import numpy as np

from .np_oracle import expm_series


def pairs(n):
    return [(p, q) for p in range(n) for q in range(p + 1, n)]


def twist(Omega, v):
    n = len(v)
    X = np.zeros((n + 1, n + 1))
    X[:n, :n] = Omega
    X[:n, n] = v
    return X


def inverse(h):
    n = h.shape[0] - 1
    out = np.eye(n + 1)
    R, T = h[:n, :n], h[:n, n]
    out[:n, :n] = R.T
    out[:n, n] = -R.T @ T
    return out


def _terms(x, lx, z, lz, h, sigma, feat_scale, ell, kappa):
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = x.shape[1]
    hi = inverse(np.asarray(h, dtype=np.float64))
    zt = z @ hi[:n, :n].T + hi[:n, n]
    d = zt[None, :, :] - x[:, None, :]
    r2 = (d * d).sum(axis=2)
    c = feat_scale * (np.asarray(lx, dtype=np.float64) @ np.asarray(lz, dtype=np.float64).T)
    k = sigma ** 2 * np.exp(-r2 / (2.0 * ell * ell))
    if kappa > 0:
        k = np.where(r2 <= (kappa * ell) ** 2, k, 0.0)
    return c * k, d, zt


def objective(x, lx, z, lz, h, *, sigma=0.1, feat_scale=0.2, ell=0.1, kappa=0.0):
    """F(h) = sum_ij c_ij k(x_i, h^-1 z_j) (eq. scalar) for h in SE(n)."""
    w, _, _ = _terms(x, lx, z, lz, h, sigma, feat_scale, ell, kappa)
    return w.sum()


def gradient(x, lx, z, lz, h, *, sigma=0.1, feat_scale=0.2, ell=0.1, kappa=0.0, a2=None, b2=1.0):
    """(F, w, v): w[p, q] = w^{pq} of eq. flow (antisymmetric matrix, p < q
    the coordinates) and v^m, at the paper's pose h."""
    x = np.asarray(x, dtype=np.float64)
    if a2 is None:
        a2 = float((x * x).sum(axis=1).mean())
    wgt, d, zt = _terms(x, lx, z, lz, h, sigma, feat_scale, ell, kappa)
    n = x.shape[1]
    W = np.zeros((n, n))
    for p, q in pairs(n):
        W[p, q] = (wgt * (x[:, None, p] * zt[None, :, q] - x[:, None, q] * zt[None, :, p])).sum() / (a2 * ell * ell)
        W[q, p] = -W[p, q]
    v = (wgt[:, :, None] * d).sum(axis=(0, 1)) / (b2 * ell * ell)
    return wgt.sum(), W, v


def ascent_twist(W, v):
    """The steepest-ascent element of se(n): Omega = sum_{p<q} w^{pq} (E_qp - E_pq)."""
    return twist(-np.asarray(W), np.asarray(v))


def metric(xi1, xi2, a2, b2):
    """-(a^2/2) tr(Omega1 Omega2) + b^2 <v1, v2> on twists (n+1 x n+1)."""
    n = xi1.shape[0] - 1
    return -0.5 * a2 * np.trace(xi1[:n, :n] @ xi2[:n, :n]) + b2 * xi1[:n, n] @ xi2[:n, n]


def register(x, lx, z, lz, *, sigma=0.1, feat_scale=0.2, ell=0.1, kappa=0.0, a2=None, b2=1.0, eta=1.0,
             max_iters=50, h0=None, mask=None):
    """Gradient flow on SE(n) (or on the subgroup of generators in mask: a
    boolean vector over [J^{pq} for p < q, then e^m]), fixed step
    tau = eta l^2 / F.  Returns (h, trace of (F, tau))."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[1]
    if a2 is None:
        a2 = float((x * x).sum(axis=1).mean())
    h = np.eye(n + 1) if h0 is None else np.asarray(h0, dtype=np.float64).copy()
    trace = []
    for _ in range(max_iters):
        F, W, v = gradient(x, lx, z, lz, h, sigma=sigma, feat_scale=feat_scale, ell=ell, kappa=kappa, a2=a2, b2=b2)
        if mask is not None:
            m = np.asarray(mask, dtype=bool)
            for k, (p, q) in enumerate(pairs(n)):
                if not m[k]:
                    W[p, q] = W[q, p] = 0.0
            v = np.where(m[len(pairs(n)):], v, 0.0)
        tau = eta * ell * ell / F
        h = h @ expm_series(tau * ascent_twist(W, v))
        trace.append((F, tau))
    return h, np.array(trace)

"""NumPy FP64 oracle for tiny inputs (TEST INFRASTRUCTURE ONLY).

A second, independent transcription of the paper's definitions, kept apart
from cvo_oracle.c so that the two can check each other:
  * the objective F(h) = sum_ij c_ij k(x_i, h^-1 z_j)  (eq. scalar, Sec. III);
  * the gradient in the general-n coordinates of eq. flow (Sec. IV-C),
    omega^{pq} = 1/(a^2 l^2) sum c k (x^p z~^q - x^q z~^p),
    v^m        = 1/(b^2 l^2) sum c k (z~^m - x^m)   (sign from the kernel's
    derivative; the printed x - z~ is the opposite sign),
    read back as the 3-vector omega = (w^{23}, w^{31}, w^{12}) with
    w^ = [[0, -w3, w2], [w3, 0, -w1], [-w2, w1, 0]];
  * the group exponential as the matrix exponential of the 4x4 twist
    (Sec. VI-A: exp is "merely the matrix exponential"), via a scaled and
    squared Taylor series rather than the closed form.
Everything is O(N M) dense NumPy: keep N*M below ~1e7.
"""
from __future__ import annotations

import numpy as np


def hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def twist_matrix(w, u):
    X = np.zeros((4, 4))
    X[:3, :3] = hat(w)
    X[:3, 3] = u
    return X


def expm_series(A, terms=30):
    """exp(A) by scaling and squaring of a truncated Taylor series (FP64)."""
    nrm = np.abs(A).sum(axis=1).max()
    s = 0
    while nrm > 0.5:
        nrm /= 2.0
        s += 1
    B = A / (2.0 ** s)
    E = np.eye(A.shape[0])
    term = np.eye(A.shape[0])
    for k in range(1, terms):
        term = term @ B / k
        E = E + term
    for _ in range(s):
        E = E @ E
    return E


def terms(x, lx, z, lz, T, *, sigma=0.1, feat_scale=0.2, ell=0.1, kappa=0.0, a2=None, b2=1.0,
          kernel_floor=0.0):
    """Per-pair weights w_ij = c_ij k_ij, displacement z~_j - x_i and z~.

    T acts on target points (T = h^-1).  kernel_floor > 0 sparsifies by value
    as in the TUM experiment (Sec. VII-B, Table 1): kernel values
    k_ij = sigma^2 exp(-r^2 / (2 ell^2)) below the floor are set to zero.
    """
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    lx = np.asarray(lx, dtype=np.float64)
    lz = np.asarray(lz, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    zt = z @ T[:3, :3].T + T[:3, 3]
    d = zt[None, :, :] - x[:, None, :]            # [N, M, 3]
    r2 = (d * d).sum(axis=2)
    c = feat_scale * (lx @ lz.T)
    k = sigma ** 2 * np.exp(-r2 / (2.0 * ell * ell))
    if kappa > 0:
        k = np.where(r2 <= (kappa * ell) ** 2, k, 0.0)
    if kernel_floor > 0:
        k = np.where(k >= kernel_floor, k, 0.0)
    return c * k, d, zt, r2


def evaluate(x, lx, z, lz, T, *, sigma=0.1, feat_scale=0.2, ell=0.1, kappa=0.0, a2=None, b2=1.0,
             kernel_floor=0.0):
    """Returns (F, omega[3], v[3])."""
    x = np.asarray(x, dtype=np.float64)
    if a2 is None:
        a2 = float((x * x).sum(axis=1).mean())
    w, d, zt, _ = terms(x, lx, z, lz, T, sigma=sigma, feat_scale=feat_scale, ell=ell,
                        kappa=kappa, kernel_floor=kernel_floor)
    F = w.sum()
    W = np.zeros((3, 3))
    for p in range(3):
        for q in range(3):
            W[p, q] = (w * (x[:, None, p] * zt[None, :, q] - x[:, None, q] * zt[None, :, p])).sum()
    W /= a2 * ell * ell
    omega = np.array([W[1, 2], W[2, 0], W[0, 1]])
    v = (w[:, :, None] * d).sum(axis=(0, 1)) / (b2 * ell * ell)
    return F, omega, v


def objective(x, lx, z, lz, T, **kw):
    w, _, _, _ = terms(x, lx, z, lz, T, **kw)
    return w.sum()


def quartic(x, lx, z, lz, T, w, u, *, sigma=0.1, feat_scale=0.2, ell=0.1, kappa=0.0):
    """Taylor coefficients [F, A1, A2, A3, A4] of G(t) = F(h exp(t xi)) at t = 0
    (Sec. VI-B, eq. fourth), xi = (w^, u), T = h^-1 acting on targets.

    Computed here without the paper's alpha..epsilon / g^k formulas, by power
    series: the moved target is z~(t) = exp(-t Xi) z~ = sum_k (-t Xi)^k z~ / k!
    (4x4 twist Xi, homogeneous coordinates), the exponent
    e(t) = -|x - z~(t)|^2 / (2 ell^2) is truncated to degree 4 by polynomial
    products, and exp(e(t)) follows from the series recurrence
    k f_k = sum_{j=1..k} j e_j f_{k-j}.  The pair set is the one inside the
    cutoff at t = 0.
    """
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    c = feat_scale * (np.asarray(lx, dtype=np.float64) @ np.asarray(lz, dtype=np.float64).T)
    T = np.asarray(T, dtype=np.float64)
    Xi = twist_matrix(np.asarray(w, dtype=np.float64), np.asarray(u, dtype=np.float64))
    zh = np.concatenate([z, np.ones((z.shape[0], 1))], axis=1) @ T.T      # z~ (homogeneous)
    # coefficient k of x - z~(t): delta_k0 x - (-Xi)^k z~ / k!
    P = []
    Mk = np.eye(4)
    fact = 1.0
    for k in range(5):
        if k > 0:
            Mk = Mk @ (-Xi)
            fact *= k
        zk = (zh @ Mk.T)[:, :3] / fact                                       # [M, 3]
        P.append((x[:, None, :] if k == 0 else 0.0) - zk[None, :, :])      # [N, M, 3]
    e = []
    for k in range(5):
        s = sum((P[i] * P[k - i]).sum(axis=2) for i in range(k + 1))
        e.append(-s / (2.0 * ell * ell))
    f = [np.ones_like(e[0])]
    for k in range(1, 5):
        f.append(sum(j * e[j] * f[k - j] for j in range(1, k + 1)) / k)
    wgt = c * sigma ** 2 * np.exp(e[0])
    if kappa > 0:
        wgt = np.where(-2.0 * ell * ell * e[0] <= (kappa * ell) ** 2, wgt, 0.0)
    return np.array([(wgt * f[k]).sum() for k in range(5)])


def quartic_step(A):
    """t > 0 maximising P(t) = A1 t + A2 t^2 + A3 t^3 + A4 t^4 among its local
    maxima (largest P), or None.  Roots of P' from the companion-matrix
    eigenvalues (numpy.roots), polished by Newton's method; a root is a local
    maximum where P'' < 0 (a simple root).  Leading coefficients below 1e-14
    of the largest are dropped, as in the C oracle."""
    c = np.array([A[1], 2.0 * A[2], 3.0 * A[3], 4.0 * A[4]], dtype=np.float64)  # P', ascending
    big = np.abs(c).max()
    if not big > 0:
        return None
    deg = 3
    while deg > 0 and abs(c[deg]) <= 1e-14 * big:
        deg -= 1
    if deg == 0:
        return None
    c = c[: deg + 1]
    dP = np.polynomial.polynomial.Polynomial(c)
    ddP = dP.deriv()
    best = None
    for z in np.roots(c[::-1]):
        if abs(z.imag) > 1e-9 * max(1.0, abs(z.real)):
            continue
        t = z.real
        for _ in range(50):
            f, fp = dP(t), ddP(t)
            if fp == 0:
                break
            tn = t - f / fp
            if tn == t:
                break
            t = tn
        if not t > 0 or not ddP(t) < 0:
            continue
        p = t * (A[1] + t * (A[2] + t * (A[3] + t * A[4])))
        if best is None or p > best[1]:
            best = (t, p)
    return None if best is None else float(best[0])


def quartic_printed(x, lx, z, lz, T, w, u, *, sigma=0.1, feat_scale=0.2, ell=0.1):
    """[F, A1..A4] from the coefficients exactly as printed with eq. fourth
    (comparison mode only): alpha = -|d|^2/(2 ell^2) (the printed alpha lacks
    the square), beta = -<u1, d>/ell^2, gamma = -(|u1|^2 + 2<u2, d>)/(2 ell^2),
    delta = (<-u1, u2> + <-u3, d>)/ell^2,
    eps = -(|u2|^2 + 2<u1, u3> + 2<u4, d>)/(2 ell^2), with d = x - z~,
    u1 = w^ z~ + u, u_{k+1} = w^ u_k (the printed "w^2 z + v" read as
    w^2 z + w^ v), and the paper's g^1..g^4.  These expand
    |d + t u1 + t^2 u2 + t^3 u3 + t^4 u4|^2, which agrees with G(t) to first
    order only."""
    x = np.asarray(x, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    zt = np.asarray(z, dtype=np.float64) @ T[:3, :3].T + T[:3, 3]
    W = hat(np.asarray(w, dtype=np.float64))
    u1 = zt @ W.T + np.asarray(u, dtype=np.float64)
    u2 = u1 @ W.T
    u3 = u2 @ W.T
    u4 = u3 @ W.T
    d = x[:, None, :] - zt[None, :, :]
    c = feat_scale * (np.asarray(lx, dtype=np.float64) @ np.asarray(lz, dtype=np.float64).T)
    il = 1.0 / ell ** 2
    dot = lambda a, b: (a * b).sum(-1)
    al = -0.5 * il * dot(d, d)
    be = -il * dot(u1[None], d)
    ga = -0.5 * il * (dot(u1, u1)[None] + 2 * dot(u2[None], d))
    de = il * (-dot(u1, u2)[None] - dot(u3[None], d))
    ep = -0.5 * il * (dot(u2, u2)[None] + 2 * dot(u1, u3)[None] + 2 * dot(u4[None], d))
    g = [be, ga + be ** 2 / 2, de + be * ga + be ** 3 / 6,
         ep + be * de + be ** 2 * ga / 2 + ga ** 2 / 2 + be ** 4 / 24]
    k = sigma ** 2 * c * np.exp(al)
    return np.array([k.sum()] + [(k * gk).sum() for gk in g])

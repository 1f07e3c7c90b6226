"""Best uniform exponential sums for 1/lambda on [1, M] (oracle).

Sec. 4.2, Proposition 1: there are alpha_j > 0, omega_j > 0 such that
s_R(lambda) = sum_j omega_j exp(-alpha_j lambda) satisfies
E_R(M) = sup_[1,M] |1/lambda - s_R(lambda)| <= 16 exp(-R pi^2 / log(8M)).
The paper takes the best (minimax) parameters from published tables, which
are not available here; they are recomputed with the Remez exchange
algorithm for the best uniform approximation, whose error equioscillates at
2R+1 points of [1, M] (Chebyshev alternation for the exponential family).

Procedure (all in the variables a_j = log alpha_j, b_j = log omega_j, so the
positivity of Proposition 1 holds by construction):
 1. R = 1: sinc-quadrature start of 1/x = int exp(t - x e^t) dt.
 2. R -> R+1: the R-term optimum is stretched to R+1 terms by interpolating
    (a_j, b_j) over a normalised index (fallbacks: extend at either end, or a
    few Lawson reweighted least-squares sweeps).
 3. Remez: Newton solve of 1/x_i - s(x_i) = (-1)^i E on the reference
    x_0 < .. < x_2R, then exchange the reference for the 2R+1 alternating
    extrema of the error; stop when max|error| = |E| to 1e-7 relative
    (de la Vallee Poussin: the optimum E_R lies between the two).
R_P = min{R : E_R(M_P) <= eps_prec / M_P}  (eq. estimate_prec_rel).
"""
from __future__ import annotations

import numpy as np

_GRID = 6000


def _terms(a, b, x):
    return np.exp(b[None, :] - np.exp(a)[None, :] * x[:, None])


def error(a, b, x):
    """e(x) = 1/x - sum_j omega_j exp(-alpha_j x)."""
    x = np.asarray(x, dtype=float)
    return 1.0 / x - _terms(a, b, x).sum(axis=1)


def _de_dt(a, b, x):
    """d e / d(log x) and its second derivative."""
    T = _terms(a, b, x)
    al = np.exp(a)[None, :]
    d1 = -1.0 / x + x * (T * al).sum(1)
    d2 = 1.0 / x + x * (T * al).sum(1) - x * x * (T * al * al).sum(1)
    return d1, d2


def _extrema(a, b, M):
    """Alternating extrema of e on [1, M]: split the log grid at sign
    changes, take the largest |e| of every sign run, refine interior ones by
    Newton on d e/d log x = 0."""
    t = np.linspace(0.0, np.log(M), _GRID)
    x = np.exp(t)
    e = error(a, b, x)
    sg = np.where(e >= 0, 1, -1)
    cuts = np.flatnonzero(sg[1:] != sg[:-1]) + 1
    starts = np.concatenate([[0], cuts])
    ends = np.concatenate([cuts, [_GRID]])
    pts = []
    for s0, s1 in zip(starts, ends):
        j = s0 + int(np.argmax(np.abs(e[s0:s1])))
        if j == 0 or j == _GRID - 1:
            pts.append(x[j])
            continue
        tt, lo, hi = t[j], t[j - 1], t[j + 1]
        for _ in range(30):
            d1, d2 = _de_dt(a, b, np.array([np.exp(tt)]))
            if d2[0] == 0:
                break
            step = d1[0] / d2[0]
            tn = min(max(tt - step, lo), hi)
            if abs(tn - tt) < 1e-14:
                tt = tn
                break
            tt = tn
        pts.append(np.exp(tt))
    return np.array(pts)


def _solve_reference(a, b, E, xr, iters=60):
    """Damped Newton for 1/x_i - s(x_i) - (-1)^i E = 0 (rows scaled by x_i)."""
    R = len(a)
    sg = (-1.0) ** np.arange(len(xr))
    z = np.concatenate([a, b, [E]])

    def F(z):
        return (1.0 / xr - _terms(z[:R], z[R:2 * R], xr).sum(1) - sg * z[-1]) * xr

    f = F(z)
    for _ in range(iters):
        T = _terms(z[:R], z[R:2 * R], xr)
        J = np.empty((len(xr), 2 * R + 1))
        J[:, :R] = T * np.exp(z[:R])[None, :] * xr[:, None]
        J[:, R:2 * R] = -T
        J[:, -1] = -sg
        J *= xr[:, None]
        try:
            dz = np.linalg.solve(J, -f)
        except np.linalg.LinAlgError:
            dz = np.linalg.lstsq(J, -f, rcond=None)[0]
        # keep the step bounded in the log variables
        scale = min(1.0, 2.0 / max(np.max(np.abs(dz[:2 * R])), 1e-300))
        lam = scale
        f0 = np.linalg.norm(f)
        while True:
            zn = z + lam * dz
            fn = F(zn)
            if np.all(np.isfinite(fn)) and np.linalg.norm(fn) < f0 * (1 - 1e-4 * lam):
                break
            lam *= 0.5
            if lam < 1e-6:
                return z[:R], z[R:2 * R], z[-1], bool(f0 < 1e-10)
        z, f = zn, fn
        if np.linalg.norm(lam * dz) < 1e-14 * (1 + np.linalg.norm(z)):
            break
    return z[:R], z[R:2 * R], z[-1], bool(np.linalg.norm(f) < 1e-10)


def _remez(a, b, M, xr=None, maxit=80):
    R = len(a)
    if xr is None:
        xr = _extrema(a, b, M)
    if len(xr) != 2 * R + 1:
        return None
    E = 0.0
    tt = np.exp(np.linspace(0.0, np.log(M), 4 * _GRID))
    for _ in range(maxit):
        a, b, E, ok = _solve_reference(a, b, E, xr)
        if not ok:
            return None
        xn = _extrema(a, b, M)
        if len(xn) != 2 * R + 1:
            return None
        emax = max(np.max(np.abs(error(a, b, tt))), np.max(np.abs(error(a, b, xn))))
        if emax - abs(E) <= 1e-7 * abs(E):
            return a, b, abs(E)
        xr = xn
    return None


def _lawson(a, b, M, sweeps=20, ng=3000):
    """Lawson's reweighted least squares toward the minimax fit (used only
    as a fallback to reach the right alternation count)."""
    from scipy.optimize import least_squares
    R = len(a)
    x = np.exp(np.linspace(0.0, np.log(M), ng))
    w = np.full(ng, 1.0 / ng)
    z = np.concatenate([a, b])
    for _ in range(sweeps):
        r = least_squares(lambda z: np.sqrt(w) * error(z[:R], z[R:], x), z,
                          method="lm", xtol=1e-14, ftol=1e-14, max_nfev=2000)
        z = r.x
        e = np.abs(error(z[:R], z[R:], x))
        w = np.maximum(w * e / np.sum(w * e), 1e-12 / ng)
    return z[:R], z[R:]


def _sinc_start(R, M):
    """Trapezoidal rule for 1/x = int exp(t - x e^t) dt with R nodes: pick
    the first node and the step on a small grid by the max absolute error."""
    xs = np.exp(np.linspace(0.0, np.log(M), 2000))
    best = None
    for t0 in np.linspace(-np.log(M) - 3.0, 2.0, 60):
        for h in np.linspace(0.3, 3.0, 28):
            t = t0 + h * np.arange(R)
            v = np.max(np.abs(error(t, np.log(h) + t, xs)))
            if best is None or v < best[0]:
                best = (v, t, np.log(h) + t)
    return best[1], best[2]


def _grow_candidates(a, b):
    o = np.argsort(a)
    a, b = a[o], b[o]
    R = len(a)
    if R >= 3:
        # the optimal nodes keep their spacing pattern from the slow end and
        # gain one node near the fast end (observed structure of the optimum)
        d = np.diff(a)
        c = b - a
        d_new = np.concatenate([d[:-1], [d[-2]], [d[-1]]])
        a_new = a[-1] + 0.04 - np.concatenate([np.cumsum(d_new[::-1])[::-1], [0.0]])
        c_new = np.concatenate([c[:-1], [2 * c[-2] - c[-3]], [c[-1]]])
        yield a_new, a_new + c_new
    if R >= 2:
        s_old = np.linspace(0.0, 1.0, R)
        s_new = np.linspace(0.0, 1.0, R + 1)
        yield np.interp(s_new, s_old, a), np.interp(s_new, s_old, b) + np.log(R / (R + 1.0))
        da, db = a[1] - a[0], b[1] - b[0]
        yield np.concatenate([[a[0] - da], a]), np.concatenate([[b[0] - db], b])
        da, db = a[-1] - a[-2], b[-1] - b[-2]
        yield np.concatenate([a, [a[-1] + da]]), np.concatenate([b, [b[-1] + db]])
    for d in (0.5, 1.0, 2.0):          # split the slowest term in two
        yield (np.concatenate([[a[0] - d, a[0] + d], a[1:]]),
               np.concatenate([[b[0] - d - np.log(2.0), b[0] + d - np.log(2.0)], b[1:]]))


def _fresh(R, M):
    a, b = _sinc_start(R, M)
    res = _remez(a, b, M)
    if res is None:
        a, b = _lawson(a, b, M)
        res = _remez(a, b, M)
    return res


def best_sequence(M: float, stop=None, Rmax: int = 40):
    """Best approximations for R = 1, 2, ... on [1, M]; yields (R, a, b, E).
    Stops after `stop(R, E)` returns True or at Rmax."""
    res = _fresh(1, M)
    if res is None:
        raise RuntimeError("Remez failed for R = 1")
    a, b, E = res
    yield 1, a, b, E
    if stop is not None and stop(1, E):
        return
    R = 1
    xr = _extrema(a, b, M)
    while R < Rmax:
        got = None
        t_old = np.log(xr)
        t_new = np.interp(np.linspace(0.0, 1.0, 2 * R + 3), np.linspace(0.0, 1.0, 2 * R + 1), t_old)
        for ga, gb in _grow_candidates(a, b):
            got = _remez(ga, gb, M, xr=np.exp(t_new))
            if got is not None:
                break
        if got is None:
            for ga, gb in _grow_candidates(a, b):
                got = _remez(ga, gb, M)
                if got is not None:
                    break
        if got is None:
            for ga, gb in _grow_candidates(a, b):
                la, lb = _lawson(ga, gb, M)
                got = _remez(la, lb, M)
                if got is not None:
                    break
        if got is None:
            got = _fresh(R + 1, M)
        if got is None:
            raise RuntimeError(f"Remez failed for R = {R + 1}, M = {M}")
        a, b, E = got
        R += 1
        xr = _extrema(a, b, M)
        yield R, a, b, E
        if stop is not None and stop(R, E):
            return


def exp_sum_for(M: float, eps_prec: float):
    """R_P = min{R : E_R(M) <= eps_prec/M} and its parameters
    (alpha ascending, omega, E_{R_P}(M), E_{R_P - 1}(M))."""
    prev = np.inf
    last = None
    for R, a, b, E in best_sequence(M, stop=lambda R, E: E <= eps_prec / M):
        if E <= eps_prec / M:
            o = np.argsort(a)
            return R, np.exp(a[o]), np.exp(b[o]), E, prev
        prev = E
        last = (R, E)
    raise RuntimeError(f"no R reached the tolerance (last {last})")


def bound_prop1(R: int, M: float) -> float:
    """The a-priori bound of Proposition 1."""
    return 16.0 * np.exp(-R * np.pi ** 2 / np.log(8.0 * M))

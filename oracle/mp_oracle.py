"""Arbitrary-precision brute force for tiny subsets (n <= 6).

TEST INFRASTRUCTURE ONLY.  Evaluates eq. (3) and eq. (4) of arXiv:1912.13132
(Sec. 2.1 / 2.2) at 50 significant digits with mpmath: the covariance of
Sec. 3 from mpmath.exp / mpmath.sqrt, the inverse of Sigma + lambda I by
mpmath's matrix inverse (no Cholesky), the prediction K^T M^{-1} y and the sum
of squared errors.  Used to pin the float64 oracle on inputs where rounding is
the only possible difference.

The kriging variance (mp_predict) is computed a different way from the
float64 oracle: as the conditional variance of a Gaussian vector, i.e. the
reciprocal of the last diagonal entry of the precision matrix of the joint
covariance of (y, Y(s_p)) under eq. (1), sigma^2 [[Sigma + lambda I, k],
[k^T, 1]] (latent value) or with 1 + lambda in the corner (a new noisy
observation).
"""
import mpmath

COV_EXP = 0
COV_MATERN32 = 1


def _c(kind, d, theta):
    t = d / theta
    if kind == COV_EXP:
        return mpmath.exp(-t)
    if kind == COV_MATERN32:
        return (1 + t) * mpmath.exp(-t)
    raise ValueError(kind)


def _dist(a, b):
    return mpmath.sqrt((a[0] - b[0]) ** 2 + (a[1] - b[1]) ** 2)


def mp_subset_cv(locs_T, y_T, locs_V, y_V, kind, theta, lam, dps=50):
    """Returns (sspe, [yhat]) as mpmath numbers, computed at `dps` digits."""
    with mpmath.workdps(dps):
        T = [(mpmath.mpf(float(p[0])), mpmath.mpf(float(p[1]))) for p in locs_T]
        V = [(mpmath.mpf(float(p[0])), mpmath.mpf(float(p[1]))) for p in locs_V]
        yT = [mpmath.mpf(float(v)) for v in y_T]
        yV = [mpmath.mpf(float(v)) for v in y_V]
        th = mpmath.mpf(float(theta))
        lm = mpmath.mpf(float(lam))
        n = len(T)
        if n == 0:
            yhat = [mpmath.mpf(0)] * len(V)
        else:
            M = mpmath.matrix(n, n)
            for a in range(n):
                for b in range(n):
                    M[a, b] = _c(kind, _dist(T[a], T[b]), th) + (lm if a == b else 0)
            Minv = M ** -1
            w = Minv * mpmath.matrix(yT)
            yhat = []
            for v in V:
                yhat.append(mpmath.fsum(_c(kind, _dist(T[a], v), th) * w[a] for a in range(n)))
        sspe = mpmath.fsum((yhat[j] - yV[j]) ** 2 for j in range(len(V)))
        return sspe, yhat


def mp_predict(locs_T, y_T, q, kind, theta, lam, sigma2, obs_noise=False, dps=50):
    """Kriging mean and variance at each query location, at `dps` digits,
    from the joint Gaussian law of eq. (1): with C the covariance matrix of
    (y_T, Y(q)) and P = C^{-1}, Var(Y(q) | y_T) = 1 / P[q, q] and
    E(Y(q) | y_T) = -sum_a P[q, a] y_a / P[q, q].  Returns two lists."""
    with mpmath.workdps(dps):
        T = [(mpmath.mpf(float(p[0])), mpmath.mpf(float(p[1]))) for p in locs_T]
        yT = [mpmath.mpf(float(v)) for v in y_T]
        th = mpmath.mpf(float(theta))
        lm = mpmath.mpf(float(lam))
        s2 = mpmath.mpf(float(sigma2))
        n = len(T)
        means, vars_ = [], []
        for p in q:
            s = (mpmath.mpf(float(p[0])), mpmath.mpf(float(p[1])))
            C = mpmath.matrix(n + 1, n + 1)
            for a in range(n):
                for b in range(n):
                    C[a, b] = s2 * (_c(kind, _dist(T[a], T[b]), th) + (lm if a == b else 0))
                C[a, n] = C[n, a] = s2 * _c(kind, _dist(T[a], s), th)
            C[n, n] = s2 * (1 + (lm if obs_noise else 0))
            Pm = C ** -1
            vars_.append(1 / Pm[n, n])
            means.append(-mpmath.fsum(Pm[n, a] * yT[a] for a in range(n)) / Pm[n, n])
        return means, vars_

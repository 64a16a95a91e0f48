"""Plain FP64 definition of the parallel-CV loss, kriging prediction and the
per-subset quantities that fall out of the same factorisation.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Source: Gerber & Nychka, arXiv:1912.13132.
  * model           -- Sec. 2.1, eq. (1): y ~ N(0, sigma^2 Sigma(theta) + tau I)
  * likelihood      -- Sec. 2.1, eq. (2)
  * kriging         -- Sec. 2.1, eq. (3), with lambda = tau / sigma^2
  * hold-out loss   -- Sec. 2.2, eq. (4) (sum of squared prediction errors)
  * parallel CV     -- Sec. 2.3, eq. (7) and Algorithm 1 (sum of subset losses)
  * covariance      -- Sec. 3: c(s1, s2, theta) = exp(-||s1 - s2|| / theta)
  * GLS mean        -- Sec. 5, eq. (8)

Readings where the paper is silent (each is listed in the design notes):
  * Matern nu = 3/2 is taken in the same parametrisation as the paper's
    exponential (its nu = 1/2 member): c(d) = (1 + d/theta) exp(-d/theta).
  * The nugget lambda is added on the diagonal by index, never by zero
    distance; cross-covariances carry no nugget (eq. (3): Sigma_p has none).
  * A subset without validation points contributes nothing and is not
    factored (Sec. 4.3.1 ignores such subsets); its loss and log-det are 0.
  * A subset with validation but no training points predicts the prior
    mean 0.
  * Sums use math.fsum (correctly rounded, order independent).

Nothing here is blocked, fused or reordered: each function is the definition
evaluated with dense float64 NumPy / LAPACK calls.
"""
import math

import numpy as np
import scipy.linalg as sla

COV_EXP = 0
COV_MATERN32 = 1


def pairwise_distance(a, b):
    """Euclidean distances ||a_i - b_j|| (Sec. 3), as sqrt(dx*dx + dy*dy) in
    float64.  a: (p, 2), b: (q, 2) -> (p, q)."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 2)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 2)
    dx = a[:, 0][:, None] - b[:, 0][None, :]
    dy = a[:, 1][:, None] - b[:, 1][None, :]
    return np.sqrt(dx * dx + dy * dy)


def covariance(kind, d, theta):
    """Correlation c(d; theta) of Sec. 3 (exponential) or its Matern-3/2
    sibling.  Unit marginal variance: sigma^2 factors out of eq. (3)."""
    t = np.asarray(d, dtype=np.float64) / float(theta)
    if kind == COV_EXP:
        return np.exp(-t)
    if kind == COV_MATERN32:
        return (1.0 + t) * np.exp(-t)
    raise ValueError(f"unknown covariance kind {kind}")


def _train_matrix(kind, locs_T, theta, lam):
    """M = Sigma(theta) + lambda I over the training locations (eq. (1)/(3))."""
    n = locs_T.shape[0]
    return covariance(kind, pairwise_distance(locs_T, locs_T), theta) + lam * np.eye(n)


def subset_cv(locs_T, y_T, locs_V, y_V, kind, theta, lam):
    """One subset's term CV(y~^i_T, y^i_V, zeta) of eq. (7).

    Kriging predictor eq. (3) at the validation locations from the training
    data, M = Sigma + lambda I factored by LAPACK dpotrf, then the SSPE of
    eq. (4).  Returns a dict with sspe, logdet (= log det M = 2 sum log L_aa),
    yhat (m,), alpha (n,) and n_val.
    """
    locs_T = np.asarray(locs_T, dtype=np.float64).reshape(-1, 2)
    locs_V = np.asarray(locs_V, dtype=np.float64).reshape(-1, 2)
    y_T = np.asarray(y_T, dtype=np.float64)
    y_V = np.asarray(y_V, dtype=np.float64)
    n, m = y_T.shape[0], y_V.shape[0]
    if m == 0:
        return dict(sspe=0.0, logdet=0.0, yhat=np.zeros(0), alpha=np.zeros(n), n_val=0)
    if n == 0:
        yhat = np.zeros(m)
        alpha = np.zeros(0)
        logdet = 0.0
    else:
        M = _train_matrix(kind, locs_T, theta, lam)
        L = sla.cholesky(M, lower=True)
        alpha = sla.cho_solve((L, True), y_T)
        K = covariance(kind, pairwise_distance(locs_T, locs_V), theta)  # n x m, no nugget
        yhat = K.T @ alpha
        logdet = 2.0 * math.fsum(np.log(np.diag(L)))
    sspe = math.fsum((yhat - y_V) ** 2)
    return dict(sspe=sspe, logdet=logdet, yhat=yhat, alpha=alpha, n_val=m)


def cv_loss(locs, y, train_ptr, train_idx, val_ptr, val_idx, kind, theta, lam,
            subsets=None):
    """Parallel CV loss of eq. (7) / Algorithm 1: z = sum_i z_i.

    locs (N, 2) float64, y (N,) float64; subset i trains on
    train_idx[train_ptr[i]:train_ptr[i+1]] and validates on
    val_idx[val_ptr[i]:val_ptr[i+1]] (CSR, 0-based).  `subsets` restricts the
    evaluation to the listed subset indices (used to sample large problems);
    the total then covers those subsets only.

    Returns dict(sspe, n_val, mse, per_subset_sspe, per_subset_logdet,
    per_subset_nval, subsets).
    """
    locs = np.asarray(locs, dtype=np.float64).reshape(-1, 2)
    y = np.asarray(y, dtype=np.float64)
    train_ptr = np.asarray(train_ptr, dtype=np.int64)
    val_ptr = np.asarray(val_ptr, dtype=np.int64)
    S = train_ptr.shape[0] - 1
    ids = range(S) if subsets is None else [int(i) for i in subsets]
    z, ld, nv = [], [], []
    for i in ids:
        T = np.asarray(train_idx[train_ptr[i]:train_ptr[i + 1]], dtype=np.int64)
        V = np.asarray(val_idx[val_ptr[i]:val_ptr[i + 1]], dtype=np.int64)
        r = subset_cv(locs[T], y[T], locs[V], y[V], kind, theta, lam)
        z.append(r["sspe"])
        ld.append(r["logdet"])
        nv.append(r["n_val"])
    total = math.fsum(z)
    n_val = int(sum(nv))
    return dict(sspe=total, n_val=n_val, mse=(total / n_val if n_val else 0.0),
                per_subset_sspe=np.array(z), per_subset_logdet=np.array(ld),
                per_subset_nval=np.array(nv, dtype=np.int64), subsets=list(ids))


def route_queries(q, core_rect):
    """Owning core of each query location.

    Cores are the disjoint rectangles D_i of Sec. 2.3 / 2.4, given as rows
    (xlo, ylo, xhi, yhi).  Reading of the boundary rule: each core is
    half-open [lo, hi) per axis except that an edge lying on the domain's
    maximum (the largest hi over all cores) is closed; a point inside several
    (only possible on shared edges) goes to the lowest index; a point inside
    none goes to the core rectangle at the smallest Euclidean distance
    (lowest index on ties).
    """
    q = np.asarray(q, dtype=np.float64).reshape(-1, 2)
    R = np.asarray(core_rect, dtype=np.float64).reshape(-1, 4)
    xmax, ymax = R[:, 2].max(), R[:, 3].max()
    out = np.empty(q.shape[0], dtype=np.int64)
    for j in range(q.shape[0]):
        x, yy = q[j]
        inx = (R[:, 0] <= x) & ((x < R[:, 2]) | ((x == R[:, 2]) & (R[:, 2] == xmax)))
        iny = (R[:, 1] <= yy) & ((yy < R[:, 3]) | ((yy == R[:, 3]) & (R[:, 3] == ymax)))
        hit = np.nonzero(inx & iny)[0]
        if hit.size:
            out[j] = hit[0]
            continue
        dx = np.maximum(np.maximum(R[:, 0] - x, 0.0), x - R[:, 2])
        dy = np.maximum(np.maximum(R[:, 1] - yy, 0.0), yy - R[:, 3])
        out[j] = int(np.argmin(dx * dx + dy * dy))
    return out


def predict(locs_T, y_T, q, kind, theta, lam, sigma2=1.0, obs_noise=False):
    """Simple-kriging mean (eq. (3)) and variance at query locations q from
    one subset's training data.

    Reading for the variance (the paper motivates but does not write it): the
    textbook simple-kriging variance of the latent Y(s_p),
    sigma^2 (1 - k^T (Sigma + lambda I)^{-1} k), plus sigma^2 * lambda (= tau)
    when obs_noise is set.  With no training points: mean 0, variance sigma^2
    (+ tau).
    """
    locs_T = np.asarray(locs_T, dtype=np.float64).reshape(-1, 2)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 2)
    y_T = np.asarray(y_T, dtype=np.float64)
    nq = q.shape[0]
    extra = sigma2 * lam if obs_noise else 0.0
    if locs_T.shape[0] == 0:
        return np.zeros(nq), np.full(nq, sigma2 + extra)
    M = _train_matrix(kind, locs_T, theta, lam)
    L = sla.cholesky(M, lower=True)
    alpha = sla.cho_solve((L, True), y_T)
    K = covariance(kind, pairwise_distance(locs_T, q), theta)  # n x q
    mean = K.T @ alpha
    W = sla.solve_triangular(L, K, lower=True)
    var = sigma2 * (1.0 - np.sum(W * W, axis=0)) + extra
    return mean, var


def predict_problem(locs, y, train_ptr, train_idx, core_rect, q, kind, theta, lam,
                    sigma2=1.0, obs_noise=False):
    """Prediction over a divided domain: route each query to its core
    (route_queries) and krige it from that core's training subset."""
    locs = np.asarray(locs, dtype=np.float64).reshape(-1, 2)
    y = np.asarray(y, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 2)
    owner = route_queries(q, core_rect)
    mean = np.zeros(q.shape[0])
    var = np.zeros(q.shape[0])
    for i in np.unique(owner):
        sel = np.nonzero(owner == i)[0]
        T = np.asarray(train_idx[train_ptr[i]:train_ptr[i + 1]], dtype=np.int64)
        mu, v = predict(locs[T], y[T], q[sel], kind, theta, lam, sigma2, obs_noise)
        mean[sel] = mu
        var[sel] = v
    return mean, var, owner


def neg2_loglik_subset(locs_T, y_T, kind, theta, lam, sigma2):
    """Two times the negative log-likelihood, eq. (2), of one subset's
    training data with tau = lambda * sigma^2:
    n log(2 pi) + log det(sigma^2 M) + y^T (sigma^2 M)^{-1} y, M = Sigma + lambda I."""
    locs_T = np.asarray(locs_T, dtype=np.float64).reshape(-1, 2)
    y_T = np.asarray(y_T, dtype=np.float64)
    n = y_T.shape[0]
    M = _train_matrix(kind, locs_T, theta, lam)
    L = sla.cholesky(M, lower=True)
    alpha = sla.cho_solve((L, True), y_T)
    logdet_M = 2.0 * math.fsum(np.log(np.diag(L)))
    return n * math.log(2.0 * math.pi) + n * math.log(sigma2) + logdet_M + float(y_T @ alpha) / sigma2


def gls_beta_subset(locs_T, y_T, X, kind, theta, lam):
    """GLS estimate of the mean coefficients, Sec. 5 eq. (8):
    beta = (X^T M^{-1} X)^{-1} X^T M^{-1} y with M = Sigma + lambda I."""
    locs_T = np.asarray(locs_T, dtype=np.float64).reshape(-1, 2)
    X = np.asarray(X, dtype=np.float64)
    M = _train_matrix(kind, locs_T, theta, lam)
    Minv_X = np.linalg.solve(M, X)
    Minv_y = np.linalg.solve(M, np.asarray(y_T, dtype=np.float64))
    return np.linalg.solve(X.T @ Minv_X, X.T @ Minv_y)

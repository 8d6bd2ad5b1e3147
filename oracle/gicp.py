"""CPU oracle of the pose refinement after the search.

TEST INFRASTRUCTURE ONLY (see `oracle/__init__.py`).

The paper accepts a BBS pose when it is close enough for local fine
registration with GICP to finish the job (Sec. IV, the success criterion, and
Sec. IV-B, where GICP also aligns the ground truth).  It gives no GICP
arithmetic; the readings below follow generalized ICP (Segal et al.) with
voxel statistics as its distributions: every scan point is paired with the
nearest voxel mean around it.

Readings:
- Distributions.  Points are grouped by voxel floor(p / voxel) (double).  A
  voxel with at least min_points points has mean mu = S1 / n and covariance
  S2 / n - mu mu^T (S1, S2 the sums of p and p p^T in double).  The covariance
  is regularized as in GICP's plane-to-plane form: with eigenvectors U of
  ascending eigenvalues, C = U diag(eps, 1, 1) U^T, eps = 1e-3.
- The scan's own voxels (same edge) give each scan point its covariance C_i;
  points of scan voxels below min_points take no part.
- Correspondence (GICP pairs a point with its nearest target point; here the
  target points are the voxel means): q_i = R p_i + t is paired with the
  distribution whose mean is nearest among the 27 voxels around floor(q_i /
  voxel) (offsets in lexicographic order, the first of equal distances), if
  that mean is closer than one voxel edge.
- Cost at pose (R, t): with r_i = mu_i - q_i and Omega_i = (C_i' + R C_i
  R^T)^-1 (C_i' the paired distribution's covariance), the sum of
  r_i^T Omega_i r_i over paired points.
- Gauss-Newton on the perturbation q' = Exp(w) q + tau (w the rotation
  vector): dr/d(w, tau) = [ [q]_x , -I ], H = sum J^T Omega J,
  g = sum J^T Omega r, (w, tau) = -H^-1 g, then R <- Exp(w) R,
  t <- Exp(w) t + tau.  Stop after max_iterations steps, or once |w| < eps_rot
  and |tau| < eps_trans (that step applied).
"""
from __future__ import annotations

import numpy as np

REG_EPS = 1e-3


def regularize(cov: np.ndarray) -> np.ndarray:
    """GICP plane-to-plane: eigenvalues replaced by (eps, 1, 1), ascending."""
    w, U = np.linalg.eigh(cov)
    return U @ np.diag([REG_EPS, 1.0, 1.0]) @ U.T


def voxel_distributions(points, voxel: float, min_points: int):
    """(keys (m, 3) int64 in lexicographic order, means (m, 3), regularized
    covariances (m, 3, 3)) of the voxels with at least min_points points."""
    p = np.asarray(points, np.float32).reshape(-1, 3).astype(np.float64)
    keys = np.floor(p / voxel).astype(np.int64)
    uk, inv, cnt = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    s1 = np.zeros((len(uk), 3))
    s2 = np.zeros((len(uk), 3, 3))
    np.add.at(s1, inv, p)
    np.add.at(s2, inv, p[:, :, None] * p[:, None, :])
    keep = cnt >= min_points
    n = cnt[keep].astype(np.float64)
    mu = s1[keep] / n[:, None]
    cov = s2[keep] / n[:, None, None] - mu[:, :, None] * mu[:, None, :]
    regs = np.array([regularize(c) for c in cov]).reshape(-1, 3, 3)
    return uk[keep], mu, regs


def scan_covariances(points, voxel: float, min_points: int):
    """(points used, their covariances) from the scan's own voxels."""
    p = np.asarray(points, np.float32).reshape(-1, 3).astype(np.float64)
    keys, _, covs = voxel_distributions(p, voxel, min_points)
    pk = np.floor(p / voxel).astype(np.int64)
    j = _lookup(keys, pk)
    use = j >= 0
    return p[use], covs[j[use]]


_OFFSETS = np.array([(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)], np.int64)


def _pack(k):
    k = np.asarray(k, np.int64) + (1 << 20)
    return (k[..., 0] << 42) | (k[..., 1] << 21) | k[..., 2]


def _lookup(keys, q):
    """Row of each key of q in the sorted key table, or -1."""
    table = _pack(keys)
    x = _pack(q)
    j = np.searchsorted(table, x)
    j = np.minimum(j, len(table) - 1)
    return np.where((len(table) > 0) & (table[j] == x), j, -1)


def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def so3_exp(w):
    th = float(np.linalg.norm(w))
    if th < 1e-12:
        return np.eye(3) + skew(w)
    k = w / th
    K = skew(k)
    return np.eye(3) + np.sin(th) * K + (1.0 - np.cos(th)) * (K @ K)


def correspond(target, q, voxel: float):
    """Index of the paired distribution of every transformed point (or -1)."""
    keys, mu, _ = target
    base = np.floor(q / voxel).astype(np.int64)
    best = np.full(len(q), -1, np.int64)
    best_d = np.full(len(q), voxel * voxel)
    for off in _OFFSETS:
        j = _lookup(keys, base + off)
        ok = j >= 0
        d = mu[np.maximum(j, 0)] - q
        d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        better = ok & (d2 < best_d)
        best = np.where(better, j, best)
        best_d = np.where(better, d2, best_d)
    return best


def linearize(target, pts, covs, R, t, voxel: float):
    """(H 6x6, g 6, cost, pairs) at pose (R, t)."""
    _, mu, tc = target
    q = pts @ R.T + t
    j = correspond(target, q, voxel)
    ok = j >= 0
    q, C, jj = q[ok], covs[ok], j[ok]
    r = mu[jj] - q
    Om = np.linalg.inv(tc[jj] + R @ C @ R.T)
    J = np.zeros((len(q), 3, 6))
    J[:, 0, 1], J[:, 0, 2] = -q[:, 2], q[:, 1]
    J[:, 1, 0], J[:, 1, 2] = q[:, 2], -q[:, 0]
    J[:, 2, 0], J[:, 2, 1] = -q[:, 1], q[:, 0]
    J[:, :, 3:] = -np.eye(3)
    JO = np.einsum("nki,nkl->nil", J, Om)
    H = np.einsum("nil,nlj->ij", JO, J)
    g = np.einsum("nil,nl->i", JO, r)
    cost = float(np.einsum("ni,nij,nj->", r, Om, r))
    return H, g, cost, int(len(q))


def refine(target_points, scan_points, R0, t0, voxel: float = 1.0, min_points: int = 5,
           max_iterations: int = 20, eps_rot: float = 1e-6, eps_trans: float = 1e-5):
    """Gauss-Newton GICP from (R0, t0).  Returns (R, t, info dict)."""
    target = voxel_distributions(target_points, voxel, min_points)
    pts, covs = scan_covariances(scan_points, voxel, min_points)
    R = np.asarray(R0, np.float64).copy()
    t = np.asarray(t0, np.float64).copy()
    it = 0
    converged = False
    while it < max_iterations:
        H, g, cost, n = linearize(target, pts, covs, R, t, voxel)
        if n < 6:
            break
        dx = -np.linalg.solve(H, g)
        E = so3_exp(dx[:3])
        R = E @ R
        t = E @ t + dx[3:]
        it += 1
        if np.linalg.norm(dx[:3]) < eps_rot and np.linalg.norm(dx[3:]) < eps_trans:
            converged = True
            break
    H, g, cost, n = linearize(target, pts, covs, R, t, voxel)
    return R, t, {"iterations": it, "converged": converged, "cost": cost, "pairs": n}

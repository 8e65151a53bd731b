"""Comparison metrics for singular triplets (test-side; no method arithmetic here)."""
import numpy as np


def rel_sigma_err(s_test, s_ref, rank):
    r = int(rank)
    if r == 0:
        return 0.0
    return float(np.max(np.abs(s_test[:r] - s_ref[:r]) / s_ref[:r]))


def relgaps(s_ref, rank):
    """relgap_i = min_{j != i} |lambda_i - lambda_j| / lambda_i over the retained lambdas = sigma^2."""
    lam = np.asarray(s_ref[:rank], dtype=np.float64) ** 2
    out = np.full(rank, np.inf)
    for i in range(rank):
        d = np.abs(lam - lam[i])
        d[i] = np.inf
        if rank > 1:
            out[i] = d.min() / lam[i]
    return out


def sin_angles(X, Y):
    """Per-column sin of the angle between x_i and y_i (sign-free), as ||y - (x.y) x|| on unit
    vectors (no cancellation near zero angle)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    Xn = X / np.maximum(np.linalg.norm(X, axis=0), 1e-300)
    Yn = Y / np.maximum(np.linalg.norm(Y, axis=0), 1e-300)
    c = np.sum(Xn * Yn, axis=0)
    return np.minimum(1.0, np.linalg.norm(Yn - Xn * c, axis=0))


def clusters(s_ref, rank, rel=1e-3):
    """Groups of consecutive retained sigmas whose lambdas are within rel of each other."""
    lam = np.asarray(s_ref[:rank], dtype=np.float64) ** 2
    groups, cur = [], [0] if rank else []
    for i in range(1, rank):
        if abs(lam[i - 1] - lam[i]) <= rel * lam[i - 1]:
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    if cur:
        groups.append(cur)
    return groups


def subspace_sin(X, Y):
    """Largest principal-angle sine between span(X) and span(Y) (orthonormal columns):
    the 2-norm of the part of Y outside span(X)."""
    R = Y - X @ (X.T @ Y)
    return float(min(1.0, np.linalg.norm(R, 2)))


def vector_errors(U_test, U_ref, s_ref, rank, rel=1e-3):
    """Max over clusters of the subspace sine, each cluster divided by its bar scale 1/relgap
    (relative gap to the nearest sigma^2 outside the cluster).  Returns (worst sine*relgap, worst sine)."""
    lam = np.asarray(s_ref[:rank], dtype=np.float64) ** 2
    worst_scaled, worst = 0.0, 0.0
    for g in clusters(s_ref, rank, rel):
        out = [j for j in range(rank) if j not in g]
        if out:
            gap = min(abs(lam[i] - lam[j]) for i in g for j in out) / max(lam[i] for i in g)
        else:
            gap = 1.0
        si = subspace_sin(U_ref[:, g] / np.linalg.norm(U_ref[:, g], axis=0),
                          U_test[:, g] / np.linalg.norm(U_test[:, g], axis=0))
        worst = max(worst, si)
        worst_scaled = max(worst_scaled, si * min(gap, 1.0))
    return worst_scaled, worst


def paper_e_sigma(s_test, s_ref, k):
    """e_sigma of Sec. IV: sum_i |sigma_hat_i - sigma_i| over the k returned values."""
    return float(np.sum(np.abs(np.asarray(s_test[:k]) - np.asarray(s_ref[:k]))))


def paper_e_u(U_test, U_ref, k):
    """e_u of Sec. IV read as sum_i sum_m |s_i u_hat_mi - u_mi| with s_i = sign<u_hat_i, u_i>."""
    tot = 0.0
    for i in range(k):
        s = 1.0 if float(np.dot(U_test[:, i], U_ref[:, i])) >= 0 else -1.0
        tot += float(np.sum(np.abs(s * U_test[:, i] - U_ref[:, i])))
    return tot


def canonical_sign_ok(U):
    """Every column's entry of largest magnitude is positive (lowest index on exact ties)."""
    for i in range(U.shape[1]):
        j = int(np.argmax(np.abs(U[:, i])))
        if U[j, i] < 0:
            return False
    return True

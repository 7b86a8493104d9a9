"""Rounding bounds that the parity tests use to tell near-ties from real
differences between the GPU's float32 scores and the float64 oracle.

Test arithmetic only: nothing here is a step of the method.

For unit signatures u (float32, from the GPU) and shat (float64, from the
oracle), with d = u - shat, the float32 chain score c = fl(sum_c u_ic u_jc)
(one rounding per fused multiply-add, k terms) satisfies

    |c - shat_i . shat_j| <= gamma_k * sum_c |u_ic| |u_jc|     (the chain's rounding)
                            + |d_i| |u_j| + |shat_i| |d_j|       (Cauchy-Schwarz on
                                                                  u_i.u_j - shat_i.shat_j)
                            + k * 2^-52                          (float64 evaluation)

where gamma_k = k u / (1 - k u), u = 2^-24 (the standard bound for a
recursive sum of k products; a fused multiply-add rounds once per step).
"""
import numpy as np

U32 = 2.0 ** -24


def gamma(k: int) -> float:
    return k * U32 / (1.0 - k * U32)


def pair_bound(u32, shat, i, j):
    """Bound for listed pairs (rows i and j of the same matrices)."""
    u = np.asarray(u32, np.float64)
    s = np.asarray(shat, np.float64)
    k = u.shape[1]
    i = np.asarray(i)
    j = np.asarray(j)
    d = np.linalg.norm(u - s, axis=1)
    nu = np.linalg.norm(u, axis=1)
    ns = np.linalg.norm(s, axis=1)
    au = np.abs(u)
    prod = np.einsum("pc,pc->p", au[i], au[j])
    return gamma(k) * prod + d[i] * nu[j] + ns[i] * d[j] + k * 2.0 ** -52


def matrix_bound(u32_a, shat_a, u32_b, shat_b):
    """Bound for every pair (row a of the first, row b of the second)."""
    ua = np.asarray(u32_a, np.float64)
    ub = np.asarray(u32_b, np.float64)
    sa = np.asarray(shat_a, np.float64)
    sb = np.asarray(shat_b, np.float64)
    k = ua.shape[1]
    da = np.linalg.norm(ua - sa, axis=1)
    db = np.linalg.norm(ub - sb, axis=1)
    nub = np.linalg.norm(ub, axis=1)
    nsa = np.linalg.norm(sa, axis=1)
    return (gamma(k) * (np.abs(ua) @ np.abs(ub).T) + da[:, None] * nub[None, :] + nsa[:, None] * db[None, :]
            + k * 2.0 ** -52)

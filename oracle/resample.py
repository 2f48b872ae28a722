"""Balance particles and the conservative mass/momentum split (Sections 4.1.2-4.1.3).

  parent p(r)   the interior particle closest to surface sample s_r (Section 4.1.2);
                ties go to the lowest particle index, and the squared distance is
                ((dx_0^2 + dx_1^2) + dx_2^2) in FP64 with no fused multiply-add, so that
                any implementation evaluating it the same way takes the same decision;
  b_r           = s_r + 2 (x_p(r) - s_r)                              (eq. pbal);
  Pi_p          = { r : p(r) = p };  m~_p = m_p / (2 |Pi_p| + 1)      (Section 4.1.3);
  each split member (x_p, s_r, b_r for r in Pi_p) carries m~_p, v_p and A_p.

Parity pins: group mass = m_p and group centre of mass = x_p (eq. cons_mom), brute-force
nearest search on small inputs, exact dyadic ties (tests/test_oracle_transfer.py).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def dist2(a, b):
    """Squared distance, summed axis by axis in order (numpy does not fuse)."""
    d = a - b
    acc = d[..., 0] * d[..., 0]
    for k in range(1, d.shape[-1]):
        acc = acc + d[..., k] * d[..., k]
    return acc


def parents_bruteforce(s, x):
    out = np.empty(len(s), np.int64)
    for r in range(len(s)):
        d2 = dist2(x, s[r][None, :])
        out[r] = int(np.argmin(d2))          # argmin returns the first (lowest) index of the minimum
    return out


def parents(s, x, k=16):
    """Nearest interior particle of every surface sample (ties -> lowest index).

    A k-d tree proposes k candidates; the exact squared distance above picks among them.
    When the k-th candidate is not strictly farther than the winner, the sample falls
    back to the brute-force search."""
    s = np.asarray(s, np.float64)
    x = np.asarray(x, np.float64)
    if len(s) == 0:
        return np.zeros(0, np.int64)
    k = min(k, len(x))
    _, cand = cKDTree(x).query(s, k=k)
    cand = cand.reshape(len(s), k)
    d2 = dist2(x[cand], s[:, None, :])
    best = np.min(d2, axis=1)
    is_best = d2 == best[:, None]
    big = np.iinfo(np.int64).max
    winner = np.min(np.where(is_best, cand, big), axis=1)
    unsafe = (np.max(d2, axis=1) <= best * (1 + 1e-12)) if k < len(x) else np.zeros(len(s), bool)
    if np.any(unsafe):
        idx = np.nonzero(unsafe)[0]
        winner[idx] = parents_bruteforce(s[idx], x)
    return winner


def split(P, surf):
    """Parents, group sizes |Pi_p|, split masses m~_p and balance points b_r."""
    x = P["x"]
    s = surf["s"]
    par = parents(s, x)
    cnt = np.bincount(par, minlength=len(x)).astype(np.int64)
    mt = P["m"] / (2.0 * cnt + 1.0)
    b = s + 2.0 * (x[par] - s)
    return dict(parent=par, count=cnt, mtilde=mt, b=b)

"""Scoccimarro bispectrum multipoles (eq. bi_sco) and the compressed TripoSH
estimator restricted to B_l0l (eq. new_bispec), by plain grid sums.

Shell fields (the real c2r kernels the Scoccimarro section describes):
    X_i^(l)(x) = sum_{q in shell i} F_l(q) exp(i q.x)        (even l: real)
    I_i(x)     = sum_{q in shell i} exp(i q.x)
    G_l(x)     = sum_{all q} F_l(q) exp(i q.x)                (Nyquist, q = 0 zeroed)
Closed-triangle counts and estimators:
    N_T(i,j,k) = sum_x I_i I_j I_k / N^3                       (integer)
    B_l^raw(i;j,k) = (2l+1)/I33 * sum_x X_i^(l) X_j^(0) X_k^(0) / (N^3 N_T)
    BB_l0l^raw(i,j) = (2l+1)/I33 * sum_x X_i^(0) X_j^(0) G_l / (N^3 N_i N_j)

The B_l0l form follows from eq. new_bispec with l1 = L = l, l2 = 0: the
coefficient H N (3j) equals (2l+1)(-1)^m, and the addition theorem collapses
sum_m y_l^m*(k3hat) dn_l^-m(k3) into the Yamamoto F_l(k3).

Readings: "all closed triangles" = the largest bin index is at most the sum of
the other two (closure of the sorted bin centres when kmin = 0).  B_0: i <= j <= k.
B_l, l > 0: the l-leg i is free, j <= k.  Configurations with N_T = 0 are dropped.
"""

from __future__ import annotations

import numpy as np

from .spectra import Bins


def shell_field(F: np.ndarray, shells: np.ndarray, b: int) -> np.ndarray:
    nmesh = F.shape[0]
    return np.fft.ifftn(np.where(shells == b, F, 0.0)).real * nmesh ** 3


def indicator_field(shells: np.ndarray, b: int) -> np.ndarray:
    nmesh = shells.shape[0]
    return np.fft.ifftn((shells == b).astype(np.complex128)).real * nmesh ** 3


def full_field(F: np.ndarray, nyq: np.ndarray) -> np.ndarray:
    nmesh = F.shape[0]
    G = np.where(nyq, 0.0, F).copy()
    G[0, 0, 0] = 0.0
    return np.fft.ifftn(G).real * nmesh ** 3


def closed(i: int, j: int, k: int) -> bool:
    a = sorted((i, j, k))
    return a[2] <= a[0] + a[1]


def scoccimarro_configs(nbins: int, ell: int):
    """Ordered list of (i, j, k); i carries the l-leg."""
    out = []
    if ell == 0:
        for i in range(nbins):
            for j in range(i, nbins):
                for k in range(j, nbins):
                    if closed(i, j, k):
                        out.append((i, j, k))
    else:
        for i in range(nbins):
            for j in range(nbins):
                for k in range(j, nbins):
                    if closed(i, j, k):
                        out.append((i, j, k))
    return out


def triposh_pairs(nbins: int):
    return [(i, j) for i in range(nbins) for j in range(i, nbins)]


def triple_sum(a: np.ndarray, b: np.ndarray, c: np.ndarray) -> float:
    """sum_x a b c (plain definition)."""
    return float(np.dot((a * b).ravel(), c.ravel()))


def triangle_counts(bins: Bins, configs) -> np.ndarray:
    """N_T per configuration from the indicator fields (FP64, rounded)."""
    shells = bins.shell_index()
    nb = bins.nbins
    need = sorted({x for c in configs for x in c})
    ind = {b: indicator_field(shells, b) for b in need}
    n3 = float(bins.nmesh ** 3)
    out = np.empty(len(configs))
    for t, (i, j, k) in enumerate(configs):
        out[t] = triple_sum(ind[i], ind[j], ind[k]) / n3
    rounded = np.rint(out)
    if np.max(np.abs(out - rounded), initial=0.0) > 1e-6 * max(1.0, np.max(np.abs(out), initial=0.0)):
        raise ArithmeticError("triangle counts are not integral")
    del nb
    return rounded.astype(np.int64)


def scoccimarro_raw(F0, Fl, ell, bins: Bins, I33, configs, ntri):
    """B_l^raw per configuration, eq. bi_sco without the shot-noise term."""
    shells = bins.shell_index()
    needl = sorted({c[0] for c in configs})
    need0 = sorted({x for c in configs for x in c[1:]} | (set(needl) if ell == 0 else set()))
    X0 = {b: shell_field(F0, shells, b) for b in need0}
    Xl = X0 if ell == 0 else {b: shell_field(Fl, shells, b) for b in needl}
    n3 = float(bins.nmesh ** 3)
    out = np.empty(len(configs))
    for t, (i, j, k) in enumerate(configs):
        out[t] = (2 * ell + 1) / I33 * triple_sum(Xl[i], X0[j], X0[k]) / (n3 * ntri[t])
    return out


def triposh_raw(F0, Fl, ell, bins: Bins, I33, pairs=None):
    """BB_l0l^raw(i, j), i <= j, from eq. new_bispec."""
    from .mesh import nyquist_mask
    shells = bins.shell_index()
    counts = bins.counts()
    pairs = triposh_pairs(bins.nbins) if pairs is None else pairs
    X0 = {b: shell_field(F0, shells, b) for b in sorted({x for p in pairs for x in p})}
    G = full_field(Fl, nyquist_mask(bins.nmesh))
    n3 = float(bins.nmesh ** 3)
    out = np.empty(len(pairs))
    for t, (i, j) in enumerate(pairs):
        out[t] = (2 * ell + 1) / I33 * triple_sum(X0[i], X0[j], G) / (n3 * counts[i] * counts[j])
    return out


def brute_force_triangles(F_a, F_b, F_c, bins: Bins, i, j, k):
    """sum over q1 in shell i, q2 in shell j with q3 = -q1-q2 in shell k of
    F_a(q1) F_b(q2) F_c(q3), and the number of such triangles (tiny grids only)."""
    nmesh = bins.nmesh
    shells = bins.shell_index()
    idx = np.argwhere(shells >= 0)
    s_i = idx[shells[tuple(idx.T)] == i]
    s_j = idx[shells[tuple(idx.T)] == j]
    total = 0.0 + 0.0j
    count = 0
    for q1 in s_i:
        for q2 in s_j:
            q3 = (-q1 - q2) % nmesh
            if shells[tuple(q3)] == k:
                total += F_a[tuple(q1)] * F_b[tuple(q2)] * F_c[tuple(q3)]
                count += 1
    return total, count

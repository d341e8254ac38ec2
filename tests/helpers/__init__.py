"""Test-only helpers: the exact ISSA used to check the oracle in law."""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def issa_lib():
    global _LIB
    if _LIB is None:
        so = os.path.join(_HERE, "libissa.so")
        src = os.path.join(_HERE, "issa.c")
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
            subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-o", so + ".tmp", src, "-lm"], check=True)
            os.replace(so + ".tmp", so)
        L = C.CDLL(so)
        P = C.POINTER
        L.issa_run.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_int32), P(C.c_double), P(C.c_int32),
                               P(C.c_int32), P(C.c_int32), P(C.c_int32), P(C.c_double), P(C.c_int32),
                               C.c_int, P(C.c_double), C.c_uint64, P(C.c_int32)]
        L.issa_tree_run.argtypes = L.issa_run.argtypes
        _LIB = L
    return _LIB


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def issa_run(geo, D, reactions, init, times, seed, tree=False):
    """Exact RDME run on the oracle-pinned geometry; returns [n_samples, S, T].
    tree=True uses the sum-tree organisation of the same direct method."""
    from workloads import reaction_arrays

    nbr = np.ascontiguousarray(geo["nbr"], np.int32)
    T = nbr.shape[0]
    S = len(D)
    g, w, nav = geo["g"], geo["w"], geo["nav"]
    drate = np.zeros((S, T, 4))
    for m in range(S):
        drate[m] = D[m] * g[:, None] * w
    drate = np.ascontiguousarray(drate)
    rn, rid, pn, pid, k = reaction_arrays(reactions)
    R = len(reactions)
    c = np.zeros((max(R, 1), T))
    for r in range(R):
        if rn[r] == 0:
            c[r] = k[r] * nav
        elif rn[r] == 1:
            c[r] = k[r]
        else:
            c[r] = k[r] / nav
    counts = np.ascontiguousarray(init, np.int32).copy()
    times = np.ascontiguousarray(times, np.float64)
    out = np.zeros((len(times), S, T), np.int32)
    fn = issa_lib().issa_tree_run if tree else issa_lib().issa_run
    fn(T, S, R, _p(nbr, C.c_int32), _p(drate, C.c_double), _p(rn, C.c_int32), _p(rid, C.c_int32),
       _p(pn, C.c_int32), _p(pid, C.c_int32), _p(c, C.c_double), _p(counts, C.c_int32), len(times),
       _p(times, C.c_double), int(seed), _p(out, C.c_int32))
    return out


def exact_mean_linear(geo, D, production, t):
    """Exact mean counts at time t of a linear network on the mesh: every
    molecule hops t -> u at rate D g_t w_tu, and production[t] molecules per
    second appear in tet t (0th-order reactions), starting empty.  The mean of
    the exact RDME (ISSA) obeys dM/dt = Q^T M + s for such networks."""
    from scipy import sparse
    from scipy.sparse.linalg import expm_multiply

    nbr, w, g = geo["nbr"], geo["w"], geo["g"]
    T = nbr.shape[0]
    rows, cols, vals = [], [], []
    for tt in range(T):
        rows.append(tt)
        cols.append(tt)
        vals.append(-D * g[tt])
        for f in range(4):
            u = nbr[tt, f]
            if u >= 0:
                rows.append(u)      # inflow into u from tt
                cols.append(tt)
                vals.append(D * g[tt] * w[tt, f])
    # augmented with a constant state carrying the source
    rows += list(range(T))
    cols += [T] * T
    vals += list(production)
    A = sparse.csr_matrix((vals, (rows, cols)), shape=(T + 1, T + 1))
    x0 = np.zeros(T + 1)
    x0[T] = 1.0
    return expm_multiply(A * t, x0)[:T]


def annihilation_pmf(a, n_max):
    """Stationary law of the well-mixed birth / pair-annihilation chain:
    births at rate lam, n -> n - 2 at rate mu n (n - 1), a = lam / mu.
    Its generating function solves (1 + s) G'' = a G, whose solution regular
    on [-1, 1] is G(s) ~ sqrt(1 + s) I_1(2 sqrt(a (1 + s))); expanding,
    P(n) ~ sum_{k >= n - 1} a^k C(k + 1, n) / (k! (k + 1)!).  Summed in logs."""
    import math

    K = int(max(n_max, 4 * a ** 0.5 + 50 * a ** 0.25 + 50))
    while K < n_max + 60 or a / ((K + 1) * (K + 2)) > 1e-3:  # the series tail is negligible
        K *= 2
    logt = np.array([k * math.log(a) - math.lgamma(k + 1) - math.lgamma(k + 2) for k in range(K + 1)])
    p = np.zeros(n_max + 1)
    for n in range(n_max + 1):
        ks = np.arange(max(n - 1, 0), K + 1)
        lc = np.array([math.lgamma(k + 2) - math.lgamma(n + 1) - math.lgamma(k + 2 - n) for k in ks])
        v = logt[ks] + lc
        m = v.max()
        p[n] = math.exp(m) * np.exp(v - m).sum()
    # normalisation over all n: G(1) ~ sum_k a^k 2^(k+1) / (k! (k+1)!)
    v = logt + np.arange(K + 1) * math.log(2.0) + math.log(2.0)
    m = v.max()
    return p / (math.exp(m) * np.exp(v - m).sum())

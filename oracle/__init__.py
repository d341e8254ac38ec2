"""ctypes wrapper of the C reference oracle (TEST INFRASTRUCTURE ONLY).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborc.so")
SOURCES = [os.path.join(_HERE, "oracle.c")]
CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared"]


def build() -> str:
    """Compile the oracle with gcc (plain C, no FMA contraction)."""
    cmd = ["gcc", *CFLAGS, "-o", LIB_PATH + ".tmp", *SOURCES, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        i32, i64, u32, u64, f64 = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [i32, P(f64), i32, P(i32), i32, P(f64), i32, P(i32), P(i32),
                                 P(i32), P(i32), P(f64), f64, u64, i32, C.c_char_p]
        L.orc_create_surface.restype = C.c_void_p
        L.orc_create_surface.argtypes = L.orc_create.argtypes
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_tau.restype = f64
        L.orc_tau.argtypes = [C.c_void_p]
        L.orc_set_first_order.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_split_threshold.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_tau_outliers.restype = f64
        L.orc_set_tau_outliers.argtypes = [C.c_void_p, i32]
        L.orc_set_reaction_region.argtypes = [C.c_void_p, i32, i32, P(i32)]
        L.orc_split_many_threshold.argtypes = [i64, P(f64), P(i32), u64, i32, i32, P(i64)]
        L.orc_split_scaled_many.argtypes = [i64, f64, P(f64), P(i32), u64, i32, i32, P(i64)]
        L.orc_set_transfer_form.argtypes = [C.c_void_p, C.c_int]
        L.orc_geometry.argtypes = [C.c_void_p, P(i32), P(f64), P(f64), P(f64), P(f64), P(f64)]
        L.orc_set_counts.argtypes = [C.c_void_p, i32, P(i32)]
        L.orc_get_counts.argtypes = [C.c_void_p, i32, P(i32)]
        L.orc_set_state.argtypes = [C.c_void_p, i64, f64]
        L.orc_get_time.argtypes = [C.c_void_p, P(f64), P(i64)]
        L.orc_step.argtypes = [C.c_void_p, f64, P(f64), P(i32)]
        L.orc_run_steps.argtypes = [C.c_void_p, i64]
        L.orc_run_until.argtypes = [C.c_void_p, f64]
        L.orc_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        L.orc_uniform.restype = f64
        L.orc_uniform.argtypes = [u64, i32, u32, u32, u32, u32]
        L.orc_ln.restype = f64
        L.orc_ln.argtypes = [f64]
        L.orc_binomial.restype = i64
        L.orc_binomial.argtypes = [i64, f64, u64, i32, u32, u32, u32, P(u32)]
        L.orc_split.restype = u32
        L.orc_split.argtypes = [i64, P(f64), P(i32), u64, i32, u32, u32, u32, u32, P(i64)]
        L.orc_binomial_many.argtypes = [i64, f64, u64, i32, P(i64)]
        L.orc_split_many.argtypes = [i64, P(f64), P(i32), u64, i32, P(i64)]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class OracleSim:
    """One realization of one model, stepped on the CPU.  `tets` with 4
    columns is a tetrahedral volume mesh; with 3 columns, a surface of
    triangles (surface diffusion)."""

    def __init__(self, xyz, tets, D, reactions, tau_scale=1.0, seed=1, realization=0):
        from workloads import reaction_arrays

        L = lib()
        self._xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self._tets = np.ascontiguousarray(tets, dtype=np.int32)
        self.T = int(self._tets.shape[0])
        self.S = len(D)
        D = np.ascontiguousarray(D, dtype=np.float64)
        rn, rid, pn, pid, k = reaction_arrays(reactions)
        err = C.create_string_buffer(256)
        if self._tets.ndim != 2 or self._tets.shape[1] not in (3, 4):
            raise ValueError("oracle: cells must have 3 (triangles) or 4 (tetrahedra) vertices")
        create = L.orc_create_surface if self._tets.shape[1] == 3 else L.orc_create
        h = create(int(self._xyz.shape[0]), _p(self._xyz, C.c_double), self.T,
                         _p(self._tets, C.c_int32), self.S, _p(D, C.c_double), len(reactions),
                         _p(rn, C.c_int32), _p(rid, C.c_int32), _p(pn, C.c_int32),
                         _p(pid, C.c_int32), _p(k, C.c_double), float(tau_scale), int(seed),
                         int(realization), err)
        if not h:
            raise ValueError("oracle: " + err.value.decode())
        self._h = C.c_void_p(h)

    @classmethod
    def from_model(cls, model, realization=0, seed=None):
        sim = cls(model.xyz, model.tets, model.D, model.reactions, model.tau_scale,
                  model.seed if seed is None else seed, realization)
        for r, tets in (getattr(model, "regions", None) or {}).items():
            sim.set_reaction_region(r, tets)
        init = model.init[min(realization, model.init.shape[0] - 1)]
        for s in range(sim.S):
            sim.set_counts(s, init[s])
        return sim

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    def set_first_order(self, on: bool):
        lib().orc_set_first_order(self._h, 1 if on else 0)

    def set_split_threshold(self, threshold: int):
        lib().orc_set_split_threshold(self._h, int(threshold))

    def set_transfer_form(self, form: int):
        lib().orc_set_transfer_form(self._h, int(form))

    def set_tau_outliers(self, k: int) -> float:
        return lib().orc_set_tau_outliers(self._h, int(k))

    def set_reaction_region(self, reaction: int, tets):
        t = np.ascontiguousarray(tets, dtype=np.int32)
        lib().orc_set_reaction_region(self._h, int(reaction), int(t.size), _p(t, C.c_int32))

    @property
    def tau(self) -> float:
        return lib().orc_tau(self._h)

    def geometry(self):
        T = self.T
        nbr = np.empty((T, 4), np.int32)
        w = np.empty((T, 4), np.float64)
        g = np.empty(T, np.float64)
        nav = np.empty(T, np.float64)
        vol = np.empty(T, np.float64)
        area = np.empty((T, 4), np.float64)
        lib().orc_geometry(self._h, _p(nbr, C.c_int32), _p(w, C.c_double), _p(g, C.c_double),
                           _p(nav, C.c_double), _p(vol, C.c_double), _p(area, C.c_double))
        return dict(nbr=nbr, w=w, g=g, nav=nav, vol=vol, area=area)

    def set_counts(self, species, counts):
        c = np.ascontiguousarray(counts, dtype=np.int32)
        assert c.shape == (self.T,)
        lib().orc_set_counts(self._h, int(species), _p(c, C.c_int32))

    def get_counts(self, species=None):
        if species is None:
            return np.stack([self.get_counts(s) for s in range(self.S)])
        out = np.empty(self.T, np.int32)
        lib().orc_get_counts(self._h, int(species), _p(out, C.c_int32))
        return out

    def set_state(self, step_index, t):
        lib().orc_set_state(self._h, int(step_index), float(t))

    def time(self):
        t = C.c_double()
        k = C.c_int64()
        lib().orc_get_time(self._h, C.byref(t), C.byref(k))
        return t.value, k.value

    def step(self, tau_k: Optional[float] = None, record: bool = False):
        tk = self.tau if tau_k is None else float(tau_k)
        if record:
            nbar = np.empty((self.S, self.T), np.float64)
            n = np.empty((self.S, self.T), np.int32)
            lib().orc_step(self._h, tk, _p(nbar, C.c_double), _p(n, C.c_int32))
            return nbar, n
        lib().orc_step(self._h, tk, None, None)
        return None

    def run_steps(self, n: int):
        lib().orc_run_steps(self._h, int(n))

    def run_until(self, t_end: float):
        lib().orc_run_until(self._h, float(t_end))


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def uniform(seed, realization, stream, tet, step, j) -> float:
    return lib().orc_uniform(seed, realization, stream, tet, step, j)


def ln(x: float) -> float:
    return lib().orc_ln(float(x))


def binomial_many(n: int, p: float, seed: int, count: int) -> np.ndarray:
    out = np.empty(count, np.int64)
    lib().orc_binomial_many(int(n), float(p), int(seed), int(count), _p(out, C.c_int64))
    return out


def split_many(n: int, w, nbr, seed: int, count: int, threshold: int = 10) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    out = np.empty((count, 4), np.int64)
    lib().orc_split_many_threshold(int(n), _p(w, C.c_double), _p(nbr, C.c_int32), int(seed), int(count),
                                   int(threshold), _p(out, C.c_int64))
    return out


def split_scaled_many(n: int, zeta: float, w, nbr, seed: int, count: int, threshold: int = 10) -> np.ndarray:
    """count samples of the one-multinomial transfer form: n molecules over
    the faces with weights zeta w_f, the rest staying; [count, 4]."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    out = np.empty((count, 4), np.int64)
    lib().orc_split_scaled_many(int(n), float(zeta), _p(w, C.c_double), _p(nbr, C.c_int32), int(seed), int(count),
                                int(threshold), _p(out, C.c_int64))
    return out

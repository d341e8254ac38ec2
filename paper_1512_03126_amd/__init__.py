"""Python binding of the rdos C ABI (include/rdos.h): argument marshalling only.

Every computation runs in the HIP library ``librdos.so`` built in this
directory; importing this package fails loudly when the library is missing.
Functions carry the names of the C entry points and raise :class:`RdosError`
on a non-zero status.  :class:`Simulation` and :class:`Engine` are thin
object wrappers over the same calls.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RDOS_LIBRARY may name another build of the same library (for comparing builds)
LIB_PATH = os.environ.get("RDOS_LIBRARY") or os.path.join(_HERE, "librdos.so")

STATUS = {0: "RDOS_OK", -1: "RDOS_EINVAL", -2: "RDOS_ENOMEM", -3: "RDOS_EDEVICE", -4: "RDOS_ESTATE",
          -5: "RDOS_EOVERFLOW", -6: "RDOS_EBUSY"}
MAX_SPECIES = 16
MAX_REACTIONS = 32


class RdosError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None

# (name, restype, argtypes)
_P = C.POINTER
_SIGS = [
    ("rdos_create", C.c_int, [_P(C.c_void_p), C.c_int, C.c_uint64, C.c_int32]),
    ("rdos_set_mesh", C.c_int, [C.c_void_p, C.c_int32, _P(C.c_double), C.c_int32, _P(C.c_int32)]),
    ("rdos_set_surface_mesh", C.c_int, [C.c_void_p, C.c_int32, _P(C.c_double), C.c_int32, _P(C.c_int32)]),
    ("rdos_add_species", C.c_int, [C.c_void_p, C.c_double, _P(C.c_int32)]),
    ("rdos_add_reaction", C.c_int, [C.c_void_p, C.c_int32, _P(C.c_int32), C.c_int32, _P(C.c_int32), C.c_double,
                                    _P(C.c_int32)]),
    ("rdos_set_method", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]),
    ("rdos_set_transfer_form", C.c_int, [C.c_void_p, C.c_int32]),
    ("rdos_set_reaction_region", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _P(C.c_int32)]),
    ("rdos_finalize", C.c_int, [C.c_void_p, C.c_double, _P(C.c_double)]),
    ("rdos_set_counts", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _P(C.c_int32)]),
    ("rdos_get_counts", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _P(C.c_int32)]),
    ("rdos_device_counts", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _P(C.c_void_p)]),
    ("rdos_set_state", C.c_int, [C.c_void_p, C.c_int64, C.c_double]),
    ("rdos_get_time", C.c_int, [C.c_void_p, _P(C.c_double), _P(C.c_int64)]),
    ("rdos_step", C.c_int, [C.c_void_p, C.c_int64]),
    ("rdos_step_static", C.c_int, [C.c_void_p, C.c_int64]),
    ("rdos_run_until", C.c_int, [C.c_void_p, C.c_double]),
    ("rdos_set_launch_mode", C.c_int, [C.c_void_p, C.c_int32]),
    ("rdos_synchronize", C.c_int, [C.c_void_p]),
    ("rdos_set_stream", C.c_int, [C.c_void_p, C.c_void_p]),
    ("rdos_get_geometry", C.c_int, [C.c_void_p, _P(C.c_int32), _P(C.c_double), _P(C.c_double), _P(C.c_double)]),
    ("rdos_get_info", C.c_int, [C.c_void_p, _P(C.c_int32), _P(C.c_int32), _P(C.c_int32), _P(C.c_int32),
                                _P(C.c_size_t)]),
    ("rdos_last_error", C.c_char_p, [C.c_void_p]),
    ("rdos_destroy", None, [C.c_void_p]),
    ("rdos_engine_create", C.c_int, [_P(C.c_void_p), C.c_int, C.c_size_t]),
    ("rdos_engine_submit", C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_double, _P(C.c_uint64)]),
    ("rdos_engine_poll", C.c_int, [C.c_void_p, C.c_uint64, _P(C.c_int), _P(C.c_double)]),
    ("rdos_engine_ticket_times", C.c_int, [C.c_void_p, C.c_uint64, _P(C.c_double), _P(C.c_double), _P(C.c_double),
                                           _P(C.c_double)]),
    ("rdos_engine_hold", C.c_int, [C.c_void_p, C.c_int32]),
    ("rdos_engine_drain", C.c_int, [C.c_void_p]),
    ("rdos_engine_release", C.c_int, [C.c_void_p, C.c_uint64, _P(C.c_void_p)]),
    ("rdos_engine_stats", C.c_int, [C.c_void_p, _P(C.c_int64), _P(C.c_double), _P(C.c_double)]),
    ("rdos_engine_launch_shape", C.c_int, [C.c_void_p, _P(C.c_int32), _P(C.c_int32), _P(C.c_int32),
                                           _P(C.c_int32), _P(C.c_int32)]),
    ("rdos_engine_tuner_scores", C.c_int, [C.c_void_p, C.c_int32, _P(C.c_int32), _P(C.c_int32), _P(C.c_double),
                                           _P(C.c_double)]),
    ("rdos_engine_set_shape", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    ("rdos_engine_set_profiling", C.c_int, [C.c_void_p, C.c_int]),
    ("rdos_engine_work_counts", C.c_int, [C.c_void_p, _P(C.c_int64), _P(C.c_int64), _P(C.c_int64)]),
    ("rdos_engine_kernel_times", C.c_int, [C.c_void_p, _P(C.c_double), _P(C.c_int64), _P(C.c_double),
                                           _P(C.c_int64)]),
    ("rdos_bandwidth_probe", C.c_int, [C.c_int, C.c_size_t, C.c_int, _P(C.c_double)]),
    ("rdos_atomic_probe", C.c_int, [C.c_int, C.c_size_t, C.c_int64, C.c_int, _P(C.c_double)]),
    ("rdos_tune_split_threshold", C.c_int, [C.c_int, C.c_int32, _P(C.c_int32), _P(C.c_double), _P(C.c_double)]),
    ("rdos_engine_last_error", C.c_char_p, [C.c_void_p]),
    ("rdos_engine_destroy", None, [C.c_void_p]),
]
EXPORTED = [name for name, _, _ in _SIGS]


def _share_torch_runtime():
    """PyTorch wheels bundle their own HIP runtime and look it up by the
    unversioned name; loading torch first makes this library bind to that
    same runtime (matching soname) instead of a second copy from /opt/rocm,
    so torch streams and memory can be handed to it.  RDOS_WITHOUT_TORCH=1
    skips this."""
    if os.environ.get("RDOS_WITHOUT_TORCH") == "1":
        return
    try:
        import torch  # noqa: F401
    except Exception:
        pass


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        _share_torch_runtime()
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1512_03126_amd/build.py "
                              "(or __graft_entry__.build()); there is no fallback")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _check(status: int, handle=None, engine=False):
    if status != 0:
        if handle is None:
            msg = ""
        elif engine:
            msg = (lib().rdos_engine_last_error(handle) or b"").decode()
        else:
            msg = (lib().rdos_last_error(handle) or b"").decode()
        raise RdosError(status, msg)


# ---------------------------------------------------------------------------
# C entry points, one Python function each
# ---------------------------------------------------------------------------
def rdos_create(device: int, seed: int, n_realizations: int = 1) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().rdos_create(C.byref(h), int(device), int(seed), int(n_realizations)))
    return h


def rdos_set_mesh(sim, xyz, tet_verts):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tv = np.ascontiguousarray(tet_verts, dtype=np.int32)
    _check(lib().rdos_set_mesh(sim, int(xyz.shape[0]), _ptr(xyz, C.c_double), int(tv.shape[0]),
                               _ptr(tv, C.c_int32)), sim)


def rdos_set_surface_mesh(sim, xyz, tri_verts):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tv = np.ascontiguousarray(tri_verts, dtype=np.int32)
    _check(lib().rdos_set_surface_mesh(sim, int(xyz.shape[0]), _ptr(xyz, C.c_double), int(tv.shape[0]),
                                       _ptr(tv, C.c_int32)), sim)


def rdos_add_species(sim, D: float) -> int:
    out = C.c_int32()
    _check(lib().rdos_add_species(sim, float(D), C.byref(out)), sim)
    return out.value


def rdos_add_reaction(sim, reactants: Sequence[int], products: Sequence[int], k: float) -> int:
    r = np.ascontiguousarray(list(reactants) or [0], dtype=np.int32)
    p = np.ascontiguousarray(list(products) or [0], dtype=np.int32)
    out = C.c_int32()
    _check(lib().rdos_add_reaction(sim, len(reactants), _ptr(r, C.c_int32), len(products), _ptr(p, C.c_int32),
                                   float(k), C.byref(out)), sim)
    return out.value


def rdos_set_method(sim, occupancy_correction: bool = True, split_threshold: int = 10, tau_outliers: int = 0):
    _check(lib().rdos_set_method(sim, 1 if occupancy_correction else 0, int(split_threshold), int(tau_outliers)),
           sim)


def rdos_set_transfer_form(sim, form: int):
    _check(lib().rdos_set_transfer_form(sim, int(form)), sim)


def rdos_set_reaction_region(sim, reaction: int, tets):
    t = np.ascontiguousarray(tets, dtype=np.int32)
    _check(lib().rdos_set_reaction_region(sim, int(reaction), int(t.size), _ptr(t, C.c_int32)), sim)


def rdos_finalize(sim, tau_scale: float = 1.0) -> float:
    tau = C.c_double()
    _check(lib().rdos_finalize(sim, float(tau_scale), C.byref(tau)), sim)
    return tau.value


def rdos_set_counts(sim, realization: int, species: int, counts):
    c = np.ascontiguousarray(counts, dtype=np.int32)
    _check(lib().rdos_set_counts(sim, int(realization), int(species), _ptr(c, C.c_int32)), sim)


def rdos_get_counts(sim, realization: int, species: int, n_tets: int) -> np.ndarray:
    out = np.empty(int(n_tets), np.int32)
    _check(lib().rdos_get_counts(sim, int(realization), int(species), _ptr(out, C.c_int32)), sim)
    return out


def rdos_device_counts(sim, realization: int, species: int) -> int:
    """Device address of counts[n_tets] (int32) at the current period boundary."""
    p = C.c_void_p()
    _check(lib().rdos_device_counts(sim, int(realization), int(species), C.byref(p)), sim)
    return int(p.value)


class _DeviceArray:
    """A borrowed int32 device array exposed through __cuda_array_interface__
    (torch.as_tensor turns it into a tensor without a copy)."""

    def __init__(self, ptr: int, shape, strides_bytes):
        self.__cuda_array_interface__ = {"shape": tuple(int(x) for x in shape), "typestr": "<i4",
                                         "data": (ptr, False), "strides": tuple(int(x) for x in strides_bytes),
                                         "version": 2}


def rdos_set_state(sim, step_index: int, t: float):
    _check(lib().rdos_set_state(sim, int(step_index), float(t)), sim)


def rdos_get_time(sim) -> Tuple[float, int]:
    t = C.c_double()
    k = C.c_int64()
    _check(lib().rdos_get_time(sim, C.byref(t), C.byref(k)), sim)
    return t.value, k.value


def rdos_step(sim, n_steps: int):
    _check(lib().rdos_step(sim, int(n_steps)), sim)


def rdos_step_static(sim, n_steps: int):
    """rdos_step with the step kernels' queue in the library's static device
    array: allocates nothing."""
    _check(lib().rdos_step_static(sim, int(n_steps)), sim)


def rdos_run_until(sim, t_end: float):
    _check(lib().rdos_run_until(sim, float(t_end)), sim)


def rdos_set_launch_mode(sim, mode: int):
    """0: one cooperative launch for small work lists (default), 1: two
    launches per period, 2: always one launch, 3: one fused launch per
    period (up to 8 species)."""
    _check(lib().rdos_set_launch_mode(sim, int(mode)), sim)


def rdos_synchronize(sim):
    _check(lib().rdos_synchronize(sim), sim)


def rdos_set_stream(sim, stream):
    """stream: a raw hipStream_t (int), a torch.cuda.Stream, or None."""
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    _check(lib().rdos_set_stream(sim, C.c_void_p(stream) if stream else None), sim)


def rdos_get_geometry(sim, n_tets: int):
    nbr = np.empty((n_tets, 4), np.int32)
    w = np.empty((n_tets, 4), np.float64)
    g = np.empty(n_tets, np.float64)
    nav = np.empty(n_tets, np.float64)
    _check(lib().rdos_get_geometry(sim, _ptr(nbr, C.c_int32), _ptr(w, C.c_double), _ptr(g, C.c_double),
                                   _ptr(nav, C.c_double)), sim)
    return dict(nbr=nbr, w=w, g=g, nav=nav)


def rdos_get_info(sim):
    T, S, R, Rz = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    b = C.c_size_t()
    _check(lib().rdos_get_info(sim, C.byref(T), C.byref(S), C.byref(R), C.byref(Rz), C.byref(b)), sim)
    return dict(n_tets=T.value, n_species=S.value, n_reactions=R.value, n_realizations=Rz.value,
                device_bytes=b.value)


def rdos_last_error(sim) -> str:
    return (lib().rdos_last_error(sim) or b"").decode()


def rdos_destroy(sim):
    lib().rdos_destroy(sim)


def rdos_engine_create(device: int = 0, hbm_budget_bytes: int = 0):
    h = C.c_void_p()
    _check(lib().rdos_engine_create(C.byref(h), int(device), int(hbm_budget_bytes)))
    return h


def rdos_engine_submit(engine, sim, n_steps: int, tau_scale: float = 1.0) -> int:
    t = C.c_uint64()
    _check(lib().rdos_engine_submit(engine, sim, int(n_steps), float(tau_scale), C.byref(t)), engine, True)
    return t.value


def rdos_engine_poll(engine, ticket: int):
    done = C.c_int()
    lat = C.c_double()
    _check(lib().rdos_engine_poll(engine, int(ticket), C.byref(done), C.byref(lat)), engine, True)
    return bool(done.value), lat.value


def rdos_engine_ticket_times(engine, ticket: int):
    """Latency breakdown of a completed ticket (seconds)."""
    w, su, j, r = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    _check(lib().rdos_engine_ticket_times(engine, int(ticket), C.byref(w), C.byref(su), C.byref(j), C.byref(r)),
           engine, True)
    return dict(wait_s=w.value, setup_s=su.value, join_s=j.value, run_s=r.value)


def rdos_engine_hold(engine, on: bool):
    """on: start no new chunk; off: admit every queued request that fits, then
    run them together."""
    _check(lib().rdos_engine_hold(engine, 1 if on else 0), engine, True)


def rdos_engine_drain(engine):
    _check(lib().rdos_engine_drain(engine), engine, True)


def rdos_engine_release(engine, ticket: int):
    h = C.c_void_p()
    _check(lib().rdos_engine_release(engine, int(ticket), C.byref(h)), engine, True)
    return h


def rdos_engine_stats(engine):
    n = C.c_int64()
    u = C.c_double()
    b = C.c_double()
    _check(lib().rdos_engine_stats(engine, C.byref(n), C.byref(u), C.byref(b)), engine, True)
    return dict(launches=n.value, updates=u.value, busy_s=b.value)


SHAPE_SOURCES = {0: "default", 1: "tuned", 2: "cached", 3: "fixed", 4: "small work"}


def rdos_engine_launch_shape(engine):
    a, b, c, d, src = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().rdos_engine_launch_shape(engine, C.byref(a), C.byref(b), C.byref(c), C.byref(d), C.byref(src)),
           engine, True)
    return dict(chunk=a.value, scan_grid=b.value, update_blocks_per_segment=c.value, chains=d.value,
                fused=c.value == 0, source=SHAPE_SOURCES.get(src.value, src.value))


def rdos_engine_tuner_scores(engine):
    """The tuner's measurements for the current size bucket: one dict per
    candidate shape, in the order tried, with the device ms per period of its
    scored chunk in each of the two passes (0.0 where not measured)."""
    n = C.c_int32()
    _check(lib().rdos_engine_tuner_scores(engine, 0, C.byref(n), None, None, None), engine, True)
    m = n.value
    shapes = (C.c_int32 * (4 * max(m, 1)))()
    first, second = (C.c_double * max(m, 1))(), (C.c_double * max(m, 1))()
    _check(lib().rdos_engine_tuner_scores(engine, m, C.byref(n), shapes, first, second), engine, True)
    return [dict(chunk=shapes[4 * c], scan_grid=shapes[4 * c + 1], update_blocks_per_segment=shapes[4 * c + 2],
                 chains=shapes[4 * c + 3], ms_first=first[c], ms_second=second[c]) for c in range(m)]


def rdos_engine_set_shape(engine, chunk: int, scan_grid: int = 0, update_bps: int = 0, chains: int = 0):
    """Fix the launch shape (no tuning); chunk 0 returns to the tuner;
    update_bps 0: one fused launch per period."""
    _check(lib().rdos_engine_set_shape(engine, int(chunk), int(scan_grid), int(update_bps), int(chains)), engine,
           True)


def rdos_engine_set_profiling(engine, on: bool, tally: bool = True):
    """on: time every launch with events (direct launches); tally: the update
    kernel also counts its work (slower by about 8%)."""
    _check(lib().rdos_engine_set_profiling(engine, (1 if tally else 2) if on else 0), engine, True)


def rdos_engine_kernel_times(engine):
    a, c = C.c_double(), C.c_double()
    b, d = C.c_int64(), C.c_int64()
    _check(lib().rdos_engine_kernel_times(engine, C.byref(a), C.byref(b), C.byref(c), C.byref(d)), engine, True)
    return dict(scan_ms=a.value, scan_launches=b.value, update_ms=c.value, update_launches=d.value)


def rdos_engine_work_counts(engine):
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().rdos_engine_work_counts(engine, C.byref(a), C.byref(b), C.byref(c)), engine, True)
    return dict(tets=a.value, additions=b.value, transfers=c.value)


def rdos_tune_split_threshold(device: int = 0, n_max: int = 48):
    """Measured switch point of the split (Sec. II.B) and the per-launch
    times of both methods for n = 1..n_max."""
    t = C.c_int32()
    one = np.zeros(int(n_max), np.float64)
    seq = np.zeros(int(n_max), np.float64)
    _check(lib().rdos_tune_split_threshold(int(device), int(n_max), C.byref(t), _ptr(one, C.c_double),
                                           _ptr(seq, C.c_double)))
    return dict(threshold=t.value, ms_one_by_one=one, ms_sequential=seq)


def rdos_bandwidth_probe(device: int = 0, nbytes: int = 1 << 30, reps: int = 20) -> float:
    g = C.c_double()
    _check(lib().rdos_bandwidth_probe(int(device), int(nbytes), int(reps), C.byref(g)))
    return g.value


def rdos_atomic_probe(device: int = 0, nbytes: int = 1 << 30, n_atomics: int = 1 << 22, reps: int = 10) -> float:
    """Random int32 atomic additions per second into a buffer of nbytes."""
    r = C.c_double()
    _check(lib().rdos_atomic_probe(int(device), int(nbytes), int(n_atomics), int(reps), C.byref(r)))
    return r.value


def rdos_engine_destroy(engine):
    lib().rdos_engine_destroy(engine)


# ---------------------------------------------------------------------------
# Object wrappers
# ---------------------------------------------------------------------------
class Simulation:
    """A simulation handle: mesh (tetrahedra, or a surface of triangles when
    the cells have 3 vertices), species, reactions, counts, stepping."""

    def __init__(self, xyz, tets, D: Iterable[float], reactions=(), seed: int = 1, n_realizations: int = 1,
                 device: int = 0, tau_scale: Optional[float] = 1.0, occupancy_correction: bool = True,
                 split_threshold: int = 10, tau_outliers: int = 0, regions=None, transfer_form: int = 0):
        self.h = rdos_create(device, seed, n_realizations)
        self.T = int(np.asarray(tets).shape[0])
        self.Rz = int(n_realizations)
        cells = np.asarray(tets)
        if cells.ndim != 2 or cells.shape[1] not in (3, 4):
            raise ValueError("cells must have 3 (surface triangles) or 4 (tetrahedra) vertices")
        if cells.shape[1] == 3:
            rdos_set_surface_mesh(self.h, xyz, cells)
        else:
            rdos_set_mesh(self.h, xyz, cells)
        self.S = 0
        for d in D:
            rdos_add_species(self.h, d)
            self.S += 1
        for re, pr, k in reactions:
            rdos_add_reaction(self.h, re, pr, k)
        if not occupancy_correction or split_threshold != 10 or tau_outliers:
            rdos_set_method(self.h, occupancy_correction, split_threshold, tau_outliers)
        if transfer_form:
            rdos_set_transfer_form(self.h, transfer_form)
        for r, tets_r in (regions or {}).items():
            rdos_set_reaction_region(self.h, r, tets_r)
        self.tau = None
        if tau_scale is not None:
            self.tau = rdos_finalize(self.h, tau_scale)

    @classmethod
    def from_model(cls, model, device: int = 0, n_realizations: Optional[int] = None, finalize: bool = True,
                   **method):
        """A handle for a workload model; `method` takes the keyword options
        of the constructor (occupancy_correction, split_threshold, tau_outliers,
        transfer_form)."""
        Rz = model.init.shape[0] if n_realizations is None else n_realizations
        sim = cls(model.xyz, model.tets, model.D, model.reactions, seed=model.seed, n_realizations=Rz,
                  device=device, tau_scale=model.tau_scale if finalize else None,
                  regions=getattr(model, "regions", None), **method)
        for r in range(Rz):
            init = model.init[min(r, model.init.shape[0] - 1)]
            for s in range(sim.S):
                sim.set_counts(s, init[s], realization=r)
        return sim

    def finalize(self, tau_scale: float = 1.0) -> float:
        self.tau = rdos_finalize(self.h, tau_scale)
        return self.tau

    def set_counts(self, species: int, counts, realization: int = 0):
        rdos_set_counts(self.h, realization, species, counts)

    def get_counts(self, species: Optional[int] = None, realization: int = 0) -> np.ndarray:
        if species is None:
            return np.stack([rdos_get_counts(self.h, realization, s, self.T) for s in range(self.S)])
        return rdos_get_counts(self.h, realization, species, self.T)

    def device_counts(self, species: int, realization: int = 0):
        """Zero-copy torch view of one species' counts on the device; valid
        until the next step (synchronise before reading)."""
        import torch

        ptr = rdos_device_counts(self.h, realization, species)
        return torch.as_tensor(_DeviceArray(ptr, (self.T,), (4,)), device="cuda")

    def step(self, n: int = 1):
        rdos_step(self.h, n)

    def run_until(self, t_end: float):
        rdos_run_until(self.h, t_end)

    def synchronize(self):
        rdos_synchronize(self.h)

    def set_state(self, step_index: int, t: float):
        rdos_set_state(self.h, step_index, t)

    def time(self):
        return rdos_get_time(self.h)

    def geometry(self):
        return rdos_get_geometry(self.h, self.T)

    def info(self):
        return rdos_get_info(self.h)

    def set_stream(self, stream):
        rdos_set_stream(self.h, stream)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            rdos_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

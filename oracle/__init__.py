"""CPU oracle of the Digital Brain per-timestep step.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no code
with the GPU library (``paper_2211_15963_amd``); both take their network from the
seeded generator in ``netgen``.

``Oracle`` wraps ``liboracle.so`` (plain C, FP32 or FP64; see ``oracle.c`` for the
equations and the readings of the paper). ``brute`` holds a dense numpy simulator
for networks of at most ~50 neurons, used to pin the oracle's sparse fan-in.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_uint8, c_uint32, c_uint64, c_void_p

import numpy as np

from netgen.desc import Desc, NetSpec

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "liboracle.so")
    if not os.path.exists(path):
        raise RuntimeError(f"oracle library missing: {path} (run oracle/build.py)")
    L = ctypes.CDLL(path)
    L.orc_create.argtypes = [POINTER(Desc), c_int, c_char_p, c_size_t]
    L.orc_create.restype = c_void_p
    L.orc_create_ex.argtypes = [POINTER(Desc), c_int, c_uint32, c_char_p, c_size_t]
    L.orc_create_ex.restype = c_void_p
    L.orc_point_arrivals.argtypes = [c_void_p, c_uint64, c_uint64, POINTER(c_uint64), POINTER(c_uint32), c_uint32,
                                     POINTER(c_uint32), POINTER(c_float), POINTER(c_uint64)]
    L.orc_point_arrivals.restype = c_int
    L.orc_point_step.argtypes = [c_void_p, c_uint32, c_uint64, POINTER(c_float), POINTER(c_float), POINTER(c_float),
                                 POINTER(c_int32), POINTER(c_int)]
    L.orc_point_step.restype = c_int
    L.orc_destroy.argtypes = [c_void_p]
    L.orc_step.argtypes = [c_void_p, c_uint64]
    L.orc_set_injection.argtypes = [c_void_p, POINTER(c_float), c_uint32, c_uint64]
    L.orc_set_ou.argtypes = [c_void_p, POINTER(c_float), POINTER(c_float), POINTER(c_float), c_uint32]
    L.orc_set_ou.restype = c_int
    L.orc_get_ou.argtypes = [c_void_p, POINTER(c_double)]
    L.orc_ou_normal.argtypes = [c_uint64, c_uint32, c_uint64, c_uint32]
    L.orc_ou_normal.restype = c_float
    L.orc_step.restype = c_int
    for nm, rt in [("orc_num_neurons", c_uint32), ("orc_num_receptors", c_uint32), ("orc_steps_per_bin", c_uint32),
                   ("orc_steps_done", c_uint64), ("orc_num_edges", c_uint64), ("orc_edge_events", c_uint64),
                   ("orc_num_spikes", c_uint64), ("orc_bins_recorded", c_uint64)]:
        f = getattr(L, nm)
        f.argtypes = [c_void_p]
        f.restype = rt
    L.orc_get_spikes.argtypes = [c_void_p, POINTER(c_uint64), POINTER(c_uint32)]
    L.orc_get_region_signal.argtypes = [c_void_p, POINTER(c_double), POINTER(c_uint32)]
    L.orc_get_state.argtypes = [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_int32)]
    L.orc_set_state.argtypes = [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_int32)]
    L.orc_receptor_currents.argtypes = [c_void_p, POINTER(c_double)]
    L.orc_receptor_currents.restype = None
    L.orc_set_state.restype = c_int
    L.orc_get_in_edges.argtypes = [c_void_p, POINTER(c_uint64), POINTER(c_uint32), POINTER(c_float), POINTER(c_float), POINTER(c_uint8)]
    L.orc_philox4x32_10.argtypes = [POINTER(c_uint32), POINTER(c_uint32), POINTER(c_uint32)]
    L.orc_bg_word.argtypes = [c_uint64, c_uint32, c_uint64, c_uint32]
    L.orc_bg_word.restype = c_uint32
    L.orc_poisson_table.argtypes = [c_double, POINTER(c_uint32), c_int]
    L.orc_poisson_table.restype = c_int
    L.orc_poisson_count.argtypes = [c_uint32, POINTER(c_uint32), c_int]
    L.orc_poisson_count.restype = c_uint32
    L.orc_quantize.argtypes = [c_float, c_uint32]
    L.orc_quantize.restype = c_int64
    L.orc_set_threads.argtypes = [c_void_p, c_uint32]
    L.orc_set_threads.restype = c_int
    L.orc_pop_constants.argtypes = [c_void_p, c_uint32, POINTER(c_float), POINTER(c_float), POINTER(c_int32),
                                    POINTER(c_int), POINTER(c_uint32), c_int]
    L.orc_pop_constants.restype = c_int
    L.orc_i64_to_f32.argtypes = [c_int64]
    L.orc_i64_to_f32.restype = c_float
    _LIB = L
    return L


def _p(a, ct):
    return a.ctypes.data_as(POINTER(ct))


class Oracle:
    """One oracle simulation of a ``NetSpec`` in FP32 (``precision=32``) or FP64."""

    def __init__(self, spec: NetSpec, precision: int = 32, params_only: bool = False):
        L = lib()
        self.spec = spec
        self._holder = spec.to_c()
        err = ctypes.create_string_buffer(512)
        h = L.orc_create_ex(self._holder.ptr, precision, 1 if params_only else 0, err, 512)
        if not h:
            raise ValueError(f"oracle rejected the description: {err.value.decode()}")
        self._h = h
        self.precision = precision
        self.N = int(L.orc_num_neurons(h))
        self.U = int(L.orc_num_receptors(h))
        self.S = int(L.orc_steps_per_bin(h))

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def set_threads(self, threads: int) -> None:
        """Host threads for step() (the neurons split into ranges; same results on any count)."""
        if lib().orc_set_threads(self._h, int(threads)) != 0:
            raise ValueError("threads must lie in 1..256")

    def step(self, n: int) -> None:
        if lib().orc_step(self._h, int(n)) != 0:
            raise MemoryError("oracle ran out of host memory")

    def set_injection(self, prob, until_bin: int) -> None:
        """Initial spike injection in bins below until_bin (absolute bin index), per-population
        probability per bin (a scalar applies to every population)."""
        n = len(self.spec.pops)
        pr = np.broadcast_to(np.asarray(prob, np.float32), (n,)).copy()
        if lib().orc_set_injection(self._h, pr.ctypes.data_as(POINTER(c_float)), n, int(until_bin)) != 0:
            raise ValueError("bad injection arguments")

    def set_ou(self, mu, sigma, tau_ms) -> None:
        """Ornstein-Uhlenbeck background current per population (eq. 1 / eq. 4): mean mu,
        stationary standard deviation sigma, time constant tau_ms (<= 0: off); scalars
        apply to every population. The current starts at mu."""
        n = len(self.spec.pops)
        a = [np.broadcast_to(np.asarray(x, np.float32), (n,)).copy() for x in (mu, sigma, tau_ms)]
        if lib().orc_set_ou(self._h, *[_p(x, c_float) for x in a], n) != 0:
            raise ValueError("bad OU arguments")

    def ou_current(self):
        """OU current per neuron (float64; exact for the FP32 variant)."""
        out = np.zeros(self.N, np.float64)
        lib().orc_get_ou(self._h, _p(out, c_double))
        return out

    @property
    def steps_done(self) -> int:
        return int(lib().orc_steps_done(self._h))

    @property
    def edge_events(self) -> int:
        return int(lib().orc_edge_events(self._h))

    @property
    def num_edges(self) -> int:
        return int(lib().orc_num_edges(self._h))

    def spikes(self):
        """(steps uint64, ids uint32) sorted by (step, id)."""
        n = int(lib().orc_num_spikes(self._h))
        st = np.zeros(max(n, 1), np.uint64)
        ids = np.zeros(max(n, 1), np.uint32)
        lib().orc_get_spikes(self._h, _p(st, c_uint64), _p(ids, c_uint32))
        return st[:n], ids[:n]

    def region_signal(self):
        """(sig float64 [bins, regions], counts uint32 [bins, regions])."""
        nb = int(lib().orc_bins_recorded(self._h))
        R = self.spec.n_regions
        sig = np.zeros(max(nb * R, 1), np.float64)
        cnt = np.zeros(max(nb * R, 1), np.uint32)
        lib().orc_get_region_signal(self._h, _p(sig, c_double), _p(cnt, c_uint32))
        return sig[: nb * R].reshape(nb, R), cnt[: nb * R].reshape(nb, R)

    def state(self):
        """(V [N], J [U, N], ref [N]) as float64/int32 (exact for the FP32 variant)."""
        V = np.zeros(self.N, np.float64)
        J = np.zeros(self.U * self.N, np.float64)
        ref = np.zeros(self.N, np.int32)
        lib().orc_get_state(self._h, _p(V, c_double), _p(J, c_double), _p(ref, c_int32))
        return V, J.reshape(self.U, self.N), ref

    def receptor_currents(self):
        """[n_pops, 4] mean current per receptor (AMPA, NMDA, GABA_A, GABA_B) of every
        population at the current state (Suppl. Algorithm 1's measurement)."""
        out = np.zeros(4 * len(self.spec.pops), np.float64)
        lib().orc_receptor_currents(self._h, _p(out, c_double))
        return out.reshape(len(self.spec.pops), 4)

    def set_state(self, V, J, ref=None) -> None:
        V = np.ascontiguousarray(V, np.float64)
        J = np.ascontiguousarray(J, np.float64).reshape(-1)
        ref = np.zeros(self.N, np.int32) if ref is None else np.ascontiguousarray(ref, np.int32)
        assert V.size == self.N and J.size == self.U * self.N and ref.size == self.N
        lib().orc_set_state(self._h, _p(V, c_double), _p(J, c_double), _p(ref, c_int32))

    def point_arrivals(self, bin_k: int, spk_steps, spk_ids, targets):
        """Arrivals A [len(targets), U] due at the start of bin_k, from the given spikes."""
        st = np.ascontiguousarray(spk_steps, np.uint64)
        ids = np.ascontiguousarray(spk_ids, np.uint32)
        tg = np.ascontiguousarray(targets, np.uint32)
        A = np.zeros(len(tg) * self.U, np.float32)
        ev = c_uint64(0)
        rc = lib().orc_point_arrivals(self._h, int(bin_k), len(st), _p(st, c_uint64), _p(ids, c_uint32), len(tg),
                                      _p(tg, c_uint32), _p(A, c_float), ctypes.byref(ev))
        if rc != 0:
            raise RuntimeError("point arrivals failed")
        return A.reshape(len(tg), self.U), int(ev.value)

    def point_step(self, i: int, n: int, A, V: float, J, ref: int):
        """One FP32 Euler step of neuron i at step n from the given state; returns (V, J, ref, spiked)."""
        a = np.ascontiguousarray(A, np.float32)
        v = np.array([V], np.float32)
        j = np.ascontiguousarray(J, np.float32).copy()
        r = np.array([ref], np.int32)
        sp = ctypes.c_int(0)
        if lib().orc_point_step(self._h, int(i), int(n), _p(a, c_float), _p(v, c_float), _p(j, c_float),
                                _p(r, c_int32), ctypes.byref(sp)) != 0:
            raise RuntimeError("point step failed")
        return float(v[0]), j, int(r[0]), bool(sp.value)

    def pop_constants(self, p: int) -> dict:
        """Derived constants of population p as the FP32 step uses them (float32 / int)."""
        k = c_float(0)
        dec = (c_float * 4)()
        r = c_int32(0)
        n = c_int(0)
        T = (c_uint32 * 256)()
        if lib().orc_pop_constants(self._h, int(p), ctypes.byref(k), dec, ctypes.byref(r), ctypes.byref(n), T, 256) != 0:
            raise ValueError("bad population index")
        return {"k": np.float32(k.value), "decay": np.array(dec[:self.U], np.float32), "ref_steps": int(r.value),
                "poisson_T": np.array(T[:n.value], np.uint32)}

    def in_edges(self):
        E = self.num_edges
        ptr = np.zeros(self.N + 1, np.uint64)
        src = np.zeros(max(E, 1), np.uint32)
        w0 = np.zeros(max(E, 1), np.float32)
        w1 = np.zeros(max(E, 1), np.float32)
        dl = np.zeros(max(E, 1), np.uint8)
        lib().orc_get_in_edges(self._h, _p(ptr, c_uint64), _p(src, c_uint32), _p(w0, c_float), _p(w1, c_float), _p(dl, c_uint8))
        return ptr.astype(np.int64), src[:E], w0[:E], w1[:E], dl[:E]


def philox(ctr, key):
    c = (c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def bg_word(seed: int, net_id: int, n: int, i: int) -> int:
    return int(lib().orc_bg_word(seed, net_id, n, i))


def ou_normal(seed: int, net_id: int, n: int, i: int) -> float:
    return float(lib().orc_ou_normal(seed, net_id, n, i))


def poisson_table(lam: float):
    T = (c_uint32 * 256)()
    c = lib().orc_poisson_table(float(lam), T, 256)
    if c < 0:
        raise ValueError("rate out of range")
    return np.array(T[:c], dtype=np.uint64)


def poisson_count(x: int, table) -> int:
    t = np.ascontiguousarray(table, np.uint32)
    return int(lib().orc_poisson_count(int(x), _p(t, c_uint32), len(t)))


def quantize(w: float, F: int) -> int:
    return int(lib().orc_quantize(float(w), int(F)))


def i64_to_f32(v: int) -> float:
    return float(lib().orc_i64_to_f32(int(v)))

"""ctypes mirror of ``include/dbnet.h`` plus a Python-side network specification.

``NetSpec`` is a plain dataclass description of a network (populations,
projections, regions, seed, time steps). ``NetSpec.to_c()`` returns a
``DescHolder`` whose ``.ptr`` is a ``POINTER(Desc)`` valid for as long as the
holder lives; both the GPU library binding and the oracle binding take it.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, c_float, c_int32, c_uint32, c_uint64, c_int64, c_uint8, c_void_p, c_char_p, c_size_t
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

ABI_VERSION = 1
RECEPTORS_2 = 0x5   # AMPA + GABA_A, one weight per edge
RECEPTORS_4 = 0xF   # AMPA, NMDA, GABA_A, GABA_B, two weights per edge
SRC_ALL, SRC_SAME_REGION, SRC_OTHER_REGIONS, SRC_POP = 0, 1, 2, 3
CLASS_ANY, CLASS_EXC, CLASS_INH = 0, 1, 2
W_UNIFORM, W_LOGNORMAL, W_CONST = 0, 1, 2
D_FIXED, D_UNIFORM, D_DISTANCE = 0, 1, 2


class Pop(ctypes.Structure):
    _fields_ = [("size", c_uint32), ("exc", c_uint32), ("region", c_uint32), ("reserved", c_uint32),
                ("C", c_float), ("g_L", c_float), ("V_L", c_float), ("V_th", c_float),
                ("V_reset", c_float), ("T_ref", c_float), ("I_ext", c_float),
                ("g", c_float * 4), ("V_rev", c_float * 4), ("tau", c_float * 4),
                ("bg_rate_hz", c_float), ("w_bg", c_float), ("v0_lo", c_float), ("v0_hi", c_float)]


class Proj(ctypes.Structure):
    _fields_ = [("dst_pop", c_int32), ("src_mode", c_uint32), ("src_class", c_uint32), ("src_pop", c_int32),
                ("indegree", c_uint32), ("w_dist", c_uint32), ("w_a", c_float), ("w_b", c_float),
                ("w_scale_exc", c_float), ("w_scale_inh", c_float), ("d_mode", c_uint32),
                ("d_min", c_uint32), ("d_max", c_uint32), ("reserved", c_uint32)]


class Desc(ctypes.Structure):
    _fields_ = [("abi_version", c_uint32), ("n_pops", c_uint32), ("n_projs", c_uint32), ("n_regions", c_uint32),
                ("seed", c_uint64), ("dt_ms", c_float), ("bin_ms", c_float), ("receptor_mask", c_uint32),
                ("frac_bits", c_uint32), ("velocity_mm_per_ms", c_float), ("net_id", c_uint32),
                ("pops", POINTER(Pop)), ("projs", POINTER(Proj)), ("region_xyz_mm", POINTER(c_float))]


# Default membrane/receptor constants (units mV, ms, nS, pF, pA). The paper
# prints none; these follow common LIF choices (tau_m = C/g_L = 20 ms).
DEFAULT_V_REV = (0.0, 0.0, -70.0, -90.0)
DEFAULT_TAU = (2.0, 100.0, 10.0, 150.0)


@dataclass
class PopSpec:
    size: int
    exc: bool
    region: int = 0
    C: float = 500.0
    g_L: float = 25.0
    V_L: float = -70.0
    V_th: float = -50.0
    V_reset: float = -55.0
    T_ref: float = 2.0
    I_ext: float = 0.0
    g: Sequence[float] = (0.0, 0.0, 0.0, 0.0)
    V_rev: Sequence[float] = DEFAULT_V_REV
    tau: Sequence[float] = DEFAULT_TAU
    bg_rate_hz: float = 0.0
    w_bg: float = 0.0
    v0_lo: float = -60.0
    v0_hi: float = -50.0


@dataclass
class ProjSpec:
    indegree: int
    dst_pop: int = -1
    src_mode: int = SRC_ALL
    src_class: int = CLASS_ANY
    src_pop: int = -1
    w_dist: int = W_UNIFORM
    w_a: float = 0.0
    w_b: float = 1.0
    w_scale_exc: float = 1.0
    w_scale_inh: float = 1.0
    d_mode: int = D_FIXED
    d_min: int = 1
    d_max: int = 1


@dataclass
class NetSpec:
    pops: List[PopSpec]
    projs: List[ProjSpec] = field(default_factory=list)
    n_regions: int = 1
    seed: int = 0
    dt_ms: float = 0.1
    bin_ms: float = 1.0
    receptor_mask: int = RECEPTORS_4
    frac_bits: int = 32
    velocity_mm_per_ms: float = 5.0
    net_id: int = 0
    region_xyz_mm: Optional[np.ndarray] = None
    name: str = "net"

    @property
    def num_neurons(self) -> int:
        return int(sum(p.size for p in self.pops))

    @property
    def steps_per_bin(self) -> int:
        return int(round(self.bin_ms / self.dt_ms))

    @property
    def weights_per_edge(self) -> int:
        return 1 if self.receptor_mask == RECEPTORS_2 else 2

    @property
    def receptors(self) -> int:
        return 2 * self.weights_per_edge

    @property
    def max_delay(self) -> int:
        return max([1] + [p.d_max for p in self.projs if p.indegree > 0])

    def pop_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([p.size for p in self.pops])]).astype(np.int64)

    def region_of_neuron(self) -> np.ndarray:
        return np.concatenate([np.full(p.size, p.region, dtype=np.int64) for p in self.pops])

    def is_exc_neuron(self) -> np.ndarray:
        return np.concatenate([np.full(p.size, bool(p.exc)) for p in self.pops])

    def num_edges(self) -> int:
        tot = 0
        for pi, p in enumerate(self.pops):
            k = sum(pr.indegree for pr in self.projs if pr.dst_pop in (-1, pi))
            tot += k * p.size
        return int(tot)

    def to_c(self) -> "DescHolder":
        return DescHolder(self)


class DescHolder:
    """Owns the ctypes arrays behind one ``Desc``; keep it alive while in use."""

    def __init__(self, spec: NetSpec):
        self.spec = spec
        n_p = len(spec.pops)
        self.pops = (Pop * max(1, n_p))()
        for i, p in enumerate(spec.pops):
            q = self.pops[i]
            q.size, q.exc, q.region = int(p.size), int(bool(p.exc)), int(p.region)
            for nm in ("C", "g_L", "V_L", "V_th", "V_reset", "T_ref", "I_ext", "bg_rate_hz", "w_bg", "v0_lo", "v0_hi"):
                setattr(q, nm, float(getattr(p, nm)))
            for u in range(4):
                q.g[u] = float(p.g[u])
                q.V_rev[u] = float(p.V_rev[u])
                q.tau[u] = float(p.tau[u])
        n_j = len(spec.projs)
        self.projs = (Proj * max(1, n_j))()
        for i, p in enumerate(spec.projs):
            q = self.projs[i]
            q.dst_pop, q.src_mode, q.src_class, q.src_pop = int(p.dst_pop), int(p.src_mode), int(p.src_class), int(p.src_pop)
            q.indegree, q.w_dist = int(p.indegree), int(p.w_dist)
            q.w_a, q.w_b, q.w_scale_exc, q.w_scale_inh = float(p.w_a), float(p.w_b), float(p.w_scale_exc), float(p.w_scale_inh)
            q.d_mode, q.d_min, q.d_max = int(p.d_mode), int(p.d_min), int(p.d_max)
        self.xyz = None
        if spec.region_xyz_mm is not None:
            arr = np.ascontiguousarray(np.asarray(spec.region_xyz_mm, dtype=np.float32).reshape(-1))
            self.xyz = (c_float * len(arr))(*arr.tolist())
        d = Desc()
        d.abi_version = ABI_VERSION
        d.n_pops, d.n_projs, d.n_regions = n_p, n_j, int(spec.n_regions)
        d.seed = int(spec.seed) & 0xFFFFFFFFFFFFFFFF
        d.dt_ms, d.bin_ms = float(spec.dt_ms), float(spec.bin_ms)
        d.receptor_mask, d.frac_bits = int(spec.receptor_mask), int(spec.frac_bits)
        d.velocity_mm_per_ms, d.net_id = float(spec.velocity_mm_per_ms), int(spec.net_id)
        d.pops = ctypes.cast(self.pops, POINTER(Pop))
        d.projs = ctypes.cast(self.projs, POINTER(Proj))
        d.region_xyz_mm = ctypes.cast(self.xyz, POINTER(c_float)) if self.xyz is not None else POINTER(c_float)()
        self.desc = d
        self.ptr = ctypes.pointer(self.desc)


_GEN = None


def load_generator():
    """Loads ``netgen/libdbnet.so`` (built by ``netgen/build.py``)."""
    global _GEN
    if _GEN is not None:
        return _GEN
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdbnet.so")
    if not os.path.exists(path):
        raise RuntimeError(f"network generator library missing: {path} (run netgen/build.py)")
    lib = ctypes.CDLL(path)
    P = POINTER(Desc)
    lib.dbnet_validate.argtypes = [P, c_char_p, c_size_t]
    lib.dbnet_validate.restype = ctypes.c_int
    lib.dbnet_num_neurons.argtypes = [P]
    lib.dbnet_num_neurons.restype = c_uint64
    lib.dbnet_indegree.argtypes = [P, c_uint32]
    lib.dbnet_indegree.restype = c_uint32
    lib.dbnet_scratch_bytes.argtypes = [P]
    lib.dbnet_scratch_bytes.restype = c_size_t
    lib.dbnet_in_edges.argtypes = [P, c_uint32, POINTER(c_uint32), POINTER(c_float), POINTER(c_float),
                                   POINTER(c_uint8), c_void_p]
    lib.dbnet_in_edges.restype = c_int64
    lib.dbnet_v0.argtypes = [P, c_uint32]
    lib.dbnet_v0.restype = c_float
    lib.dbnet_max_delay.argtypes = [P]
    lib.dbnet_max_delay.restype = c_uint32
    _GEN = lib
    return lib


def validate(spec: NetSpec) -> Optional[str]:
    """Returns None if the generator accepts the description, else its message."""
    lib = load_generator()
    h = spec.to_c()
    buf = ctypes.create_string_buffer(512)
    rc = lib.dbnet_validate(h.ptr, buf, 512)
    return None if rc == 0 else buf.value.decode()


def generate(spec: NetSpec):
    """Generates the whole network in Python-visible arrays (small networks only).

    Returns dict with ``ptr`` (N+1 int64), ``src`` (uint32), ``w0``/``w1`` (float32),
    ``delay`` (uint8) grouped by target, and ``v0`` (float32).
    """
    lib = load_generator()
    h = spec.to_c()
    err = validate(spec)
    if err:
        raise ValueError(err)
    N = spec.num_neurons
    deg = np.array([lib.dbnet_indegree(h.ptr, i) for i in range(N)], dtype=np.int64)
    ptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    E = int(ptr[-1])
    src = np.zeros(max(E, 1), np.uint32)
    w0 = np.zeros(max(E, 1), np.float32)
    w1 = np.zeros(max(E, 1), np.float32)
    dl = np.zeros(max(E, 1), np.uint8)
    scratch = ctypes.create_string_buffer(int(lib.dbnet_scratch_bytes(h.ptr)))
    for i in range(N):
        a = int(ptr[i])
        k = lib.dbnet_in_edges(h.ptr, i, src[a:].ctypes.data_as(POINTER(c_uint32)),
                               w0[a:].ctypes.data_as(POINTER(c_float)), w1[a:].ctypes.data_as(POINTER(c_float)),
                               dl[a:].ctypes.data_as(POINTER(c_uint8)), scratch)
        if k != deg[i]:
            raise RuntimeError(f"generator returned {k} edges for target {i}, expected {deg[i]}")
    v0 = np.array([lib.dbnet_v0(h.ptr, i) for i in range(N)], dtype=np.float32)
    return {"ptr": ptr, "src": src[:E], "w0": w0[:E], "w1": w1[:E], "delay": dl[:E], "v0": v0}

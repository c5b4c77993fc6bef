"""ctypes binding of libdbsim.so (include/dbsim.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels. PyTorch is used
only as the source of device memory (its caching allocator, through the
library's allocator callbacks) and of the HIP stream the work is queued on.
If the library is missing, importing the binding fails loudly: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (CFUNCTYPE, POINTER, Structure, byref, c_char_p, c_double, c_float, c_int, c_int32, c_size_t,
                    c_uint8, c_uint32, c_uint64, c_void_p)
from typing import Optional

import numpy as np

from netgen.desc import Desc, NetSpec

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdbsim.so")

ABI_VERSION = 3
REC_REGIONS = 1
F_NO_GRAPH = 1
F_SINGLE_PASS = 2
F_HOST_BUILD = 8
F_NO_HOST_RECORD = 4
STATIC_BYTES = 64 << 20  # DBSIM_STATIC_BYTES: the static region of dbsim_create_static

OK, EINVAL, ENOMEM, EHBM, EDEVICE, ETRUNC, EOVERFLOW, ESTATE, ERANGE = 0, -1, -2, -3, -4, -5, -6, -7, -8
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHBM: "EHBM", EDEVICE: "EDEVICE", ETRUNC: "ETRUNC",
          EOVERFLOW: "EOVERFLOW", ESTATE: "ESTATE", ERANGE: "ERANGE"}

ALLOC_FN = CFUNCTYPE(c_void_p, c_void_p, c_size_t)
FREE_FN = CFUNCTYPE(None, c_void_p, c_void_p, c_size_t)


class SimDesc(Structure):
    _fields_ = [("abi_version", c_uint32), ("record_flags", c_uint32), ("net", Desc),
                ("spike_record_capacity", c_uint64), ("record_bins", c_uint32), ("device", c_int32),
                ("hip_stream", c_void_p), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_ctx", c_void_p),
                ("host_threads", c_uint32), ("flags", c_uint32), ("host_spike_capacity", c_uint64),
                ("stream_permille", c_uint32), ("arena_permille", c_uint32)]


class SimStats(Structure):
    _fields_ = [("steps", c_uint64), ("bins", c_uint64), ("spikes", c_uint64), ("edge_events", c_uint64),
                ("num_neurons", c_uint64), ("num_edges", c_uint64), ("hbm_bytes", c_uint64),
                ("timed_bins", c_uint64), ("ms_scatter", c_double), ("ms_gather", c_double),
                ("ms_neuron", c_double), ("ms_readout", c_double), ("build_seconds", c_double),
                ("spilled_events", c_uint64), ("overflow_events", c_uint64)]


class SimInfo(Structure):
    _fields_ = [("num_neurons", c_uint64), ("num_edges", c_uint64), ("receptors", c_uint32),
                ("weights_per_edge", c_uint32), ("steps_per_bin", c_uint32), ("max_delay", c_uint32),
                ("n_regions", c_uint32), ("tile_neurons", c_uint32), ("n_tiles", c_uint32), ("frac_bits", c_uint32),
                ("n_members", c_uint32), ("fanin_passes", c_uint32), ("device_built", c_uint32),
                ("stream_record_bytes", c_uint32), ("reserved", c_uint32), ("stream_records", c_uint64),
                ("arena_records", c_uint64)]


class SimMember(Structure):
    _fields_ = [("first_neuron", c_uint64), ("num_neurons", c_uint64), ("first_region", c_uint32),
                ("num_regions", c_uint32)]


class SimTuning(Structure):
    _fields_ = [("scatter_wgs_per_cu", c_uint32), ("round_events", c_uint32), ("chunks_per_wg", c_uint32),
                ("ahead_passes", c_uint32)]


MAX_POISSON = 64


class PopConstants(Structure):
    _fields_ = [("first_neuron", c_uint32), ("end_neuron", c_uint32), ("member", c_uint32), ("region", c_uint32),
                ("k", c_float), ("g_L", c_float), ("V_L", c_float), ("V_th", c_float), ("V_reset", c_float),
                ("I_ext", c_float), ("w_bg", c_float), ("g", c_float * 4), ("V_rev", c_float * 4),
                ("decay", c_float * 4), ("ref_steps", c_int32), ("poisson_len", c_uint32),
                ("poisson_T", c_uint32 * MAX_POISSON)]

    def as_dict(self, U: int) -> dict:
        f32 = np.float32
        return {"first_neuron": int(self.first_neuron), "end_neuron": int(self.end_neuron), "member": int(self.member),
                "region": int(self.region), "k": f32(self.k), "g_L": f32(self.g_L), "V_L": f32(self.V_L),
                "V_th": f32(self.V_th), "V_reset": f32(self.V_reset), "I_ext": f32(self.I_ext), "w_bg": f32(self.w_bg),
                "g": np.array(self.g[:U], f32), "V_rev": np.array(self.V_rev[:U], f32),
                "decay": np.array(self.decay[:U], f32), "ref_steps": int(self.ref_steps),
                "poisson_T": np.array(self.poisson_T[:self.poisson_len], np.uint32)}


class NetworkView(Structure):
    _fields_ = [("row_ptr", POINTER(c_uint64)), ("seg", POINTER(c_uint32)), ("tgt", POINTER(c_uint32)),
                ("w0", POINTER(c_float)), ("w1", POINTER(c_float)), ("V0", POINTER(c_float)),
                ("pops", POINTER(PopConstants)), ("pops_cap", c_uint32), ("n_pops", c_uint32)]


class BoldParams(Structure):
    _fields_ = [("kappa", c_double), ("gamma", c_double), ("tau", c_double), ("alpha", c_double),
                ("rho", c_double), ("V0", c_double), ("k1", c_double), ("k2", c_double), ("k3", c_double),
                ("activity_scale", c_double), ("tr_bins", c_uint32), ("reserved", c_uint32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


def bold_defaults(**overrides) -> BoldParams:
    p = BoldParams()
    lib().dbsim_bold_defaults(byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


class DbsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


_LIB = None

EXPORTED = ["dbsim_abi_version", "dbsim_last_error", "dbsim_create", "dbsim_footprint", "dbsim_get_info",
            "dbsim_create_ensemble", "dbsim_footprint_ensemble", "dbsim_member_info", "dbsim_get_tuning",
            "dbsim_set_tuning",
            "dbsim_step", "dbsim_sync", "dbsim_read_spikes", "dbsim_read_region_signal", "dbsim_read_state",
            "dbsim_write_state", "dbsim_export_csr", "dbsim_set_timing", "dbsim_get_stats", "dbsim_destroy",
            "dbsim_derive_constants", "dbsim_export_network", "dbsim_create_static", "dbsim_receptor_currents",
            "dbsim_build", "dbsim_create_built", "dbsim_built_free", "dbsim_checkpoint_size",
            "dbsim_checkpoint_save", "dbsim_checkpoint_restore", "dbsim_check_device_generator"]


def lib():
    """Loads libdbsim.so; raises if it has not been built (no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library missing: {LIB_PATH}; build it with paper_2211_15963_amd/build.py")
    try:
        # torch ships its own HIP runtime; loading it first makes libdbsim bind to that same
        # runtime (one HIP runtime per process), so torch's memory and streams are valid here
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    H = c_void_p
    L.dbsim_abi_version.restype = c_uint32
    L.dbsim_last_error.restype = c_char_p
    L.dbsim_create.argtypes = [POINTER(SimDesc), POINTER(c_void_p)]
    L.dbsim_create_static.argtypes = [POINTER(SimDesc), POINTER(c_void_p)]
    L.dbsim_build.argtypes = [POINTER(SimDesc), POINTER(c_void_p)]
    L.dbsim_create_built.argtypes = [c_void_p, POINTER(SimDesc), POINTER(c_void_p)]
    L.dbsim_built_free.argtypes = [c_void_p]
    L.dbsim_footprint.argtypes = [POINTER(SimDesc), POINTER(c_uint64)]
    L.dbsim_get_info.argtypes = [H, POINTER(SimInfo)]
    L.dbsim_create_ensemble.argtypes = [POINTER(SimDesc), POINTER(Desc), c_uint32, POINTER(c_void_p)]
    L.dbsim_footprint_ensemble.argtypes = [POINTER(SimDesc), POINTER(Desc), c_uint32, POINTER(c_uint64)]
    L.dbsim_member_info.argtypes = [H, c_uint32, POINTER(SimMember)]
    L.dbsim_get_tuning.argtypes = [H, POINTER(SimTuning)]
    L.dbsim_set_tuning.argtypes = [H, POINTER(SimTuning)]
    L.dbsim_step.argtypes = [H, c_uint64]
    L.dbsim_sync.argtypes = [H]
    L.dbsim_read_spikes.argtypes = [H, c_uint64, c_uint64, POINTER(c_uint64), POINTER(c_uint32), c_uint64,
                                    POINTER(c_uint64)]
    L.dbsim_read_region_signal.argtypes = [H, c_uint64, c_uint64, POINTER(c_double), POINTER(c_uint32), c_uint64,
                                           POINTER(c_uint64)]
    L.dbsim_read_state.argtypes = [H, POINTER(c_float), POINTER(c_float), POINTER(c_int32)]
    L.dbsim_write_state.argtypes = [H, POINTER(c_float), POINTER(c_float), POINTER(c_int32)]
    L.dbsim_check_device_generator.argtypes = [POINTER(Desc), c_uint32, c_uint64, POINTER(c_uint32), POINTER(c_float),
                                               POINTER(c_float), POINTER(c_uint8), POINTER(c_uint32), c_uint64,
                                               POINTER(c_uint64)]
    L.dbsim_checkpoint_size.argtypes = [H, POINTER(c_uint64)]
    L.dbsim_checkpoint_save.argtypes = [H, c_void_p, c_uint64, POINTER(c_uint64)]
    L.dbsim_checkpoint_restore.argtypes = [H, c_void_p, c_uint64]
    L.dbsim_export_csr.argtypes = [H, POINTER(c_uint64), POINTER(c_uint32), POINTER(c_uint32), POINTER(c_float),
                                   POINTER(c_float)]
    L.dbsim_derive_constants.argtypes = [POINTER(SimDesc), POINTER(Desc), c_uint32, POINTER(PopConstants), c_uint32,
                                         POINTER(c_uint32)]
    L.dbsim_export_network.argtypes = [H, POINTER(NetworkView)]
    L.dbsim_set_timing.argtypes = [H, c_int]
    L.dbsim_receptor_currents.argtypes = [H, POINTER(c_double), c_uint32]
    L.dbsim_get_stats.argtypes = [H, POINTER(SimStats)]
    L.dbsim_destroy.argtypes = [H]
    L.dbsim_bold_defaults.argtypes = [POINTER(BoldParams)]
    L.dbsim_bold_defaults.restype = None
    L.dbsim_set_bold.argtypes = [H, POINTER(BoldParams)]
    L.dbsim_read_bold.argtypes = [H, c_uint64, c_uint64, POINTER(c_double), c_uint64, POINTER(c_uint64)]
    L.dbsim_read_bold_state.argtypes = [H, POINTER(c_double), POINTER(c_uint64)]
    L.dbsim_set_spike_injection.argtypes = [H, POINTER(c_float), c_uint32, c_uint64]
    L.dbsim_set_ou_background.argtypes = [H, POINTER(c_float), POINTER(c_float), POINTER(c_float), c_uint32]
    for nm in EXPORTED:
        if nm not in ("dbsim_abi_version", "dbsim_last_error", "dbsim_built_free"):
            getattr(L, nm).restype = c_int
    L.dbsim_built_free.restype = None
    if L.dbsim_abi_version() != ABI_VERSION:
        raise RuntimeError("libdbsim ABI version mismatch")
    _LIB = L
    return L


def _check(rc: int) -> None:
    if rc != OK:
        raise DbsimError(rc, lib().dbsim_last_error().decode())


def _p(a, ct):
    return a.ctypes.data_as(POINTER(ct))


class _TorchAllocator:
    """Device memory from torch's caching allocator, handed to the library as callbacks."""

    def __init__(self, device: int, stream_handle: int):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream_handle
        self.alloc = ALLOC_FN(self._alloc)
        self.free = FREE_FN(self._free)

    def _alloc(self, ctx, nbytes):
        try:
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream or None)
        except Exception:
            return None

    def _free(self, ctx, ptr, nbytes):
        try:
            self.torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass


def make_desc(spec: NetSpec, record_regions: bool = True, spike_record_capacity: int = 0, record_bins: int = 0,
              device: int = -1, stream_handle: Optional[int] = None, allocator: Optional[_TorchAllocator] = None,
              host_threads: int = 0, no_graph: bool = False, single_pass: bool = False, host_record: bool = True,
              host_spike_capacity: int = 0, host_build: bool = False, stream_permille: int = 0,
              arena_permille: int = 0):
    holder = spec.to_c()
    d = SimDesc()
    d.abi_version = ABI_VERSION
    d.record_flags = REC_REGIONS if record_regions else 0
    d.net = holder.desc
    d.spike_record_capacity = int(spike_record_capacity)
    d.record_bins = int(record_bins)
    d.device = int(device)
    d.hip_stream = c_void_p(stream_handle) if stream_handle else None
    if allocator is not None:
        d.dev_alloc = allocator.alloc
        d.dev_free = allocator.free
    d.host_threads = int(host_threads)
    d.flags = ((F_NO_GRAPH if no_graph else 0) | (F_SINGLE_PASS if single_pass else 0) |
               (0 if host_record else F_NO_HOST_RECORD) | (F_HOST_BUILD if host_build else 0))
    d.host_spike_capacity = int(host_spike_capacity)
    d.stream_permille = int(stream_permille)
    d.arena_permille = int(arena_permille)
    return d, holder


def _member_array(specs):
    holders = [sp.to_c() for sp in specs]
    arr = (Desc * len(holders))()
    for k, h in enumerate(holders):
        arr[k] = h.desc
    return arr, holders


def footprint(spec, record_regions: bool = True, **kw) -> int:
    """Device bytes for one network (NetSpec) or an ensemble (list of NetSpec)."""
    out = c_uint64(0)
    if isinstance(spec, (list, tuple)):
        d, holder = make_desc(spec[0], record_regions=record_regions, **kw)
        arr, holders = _member_array(spec)
        _check(lib().dbsim_footprint_ensemble(byref(d), arr, len(spec), byref(out)))
    else:
        d, holder = make_desc(spec, record_regions=record_regions, **kw)
        _check(lib().dbsim_footprint(byref(d), byref(out)))
    return int(out.value)


def device_generator_in_edges(spec, target: int):
    """In-edges of one target (global id) as the device construction draws them, evaluated
    on the host: (src global ids, w0, w1, delays, projection indices)."""
    specs = list(spec) if isinstance(spec, (list, tuple)) else [spec]
    arr, holders = _member_array(specs)
    n = c_uint64(0)
    rc = lib().dbsim_check_device_generator(arr, len(specs), int(target), None, None, None, None, None, 0, byref(n))
    if rc not in (OK, ETRUNC):
        _check(rc)
    k = int(n.value)
    src = np.zeros(max(k, 1), np.uint32)
    w0 = np.zeros(max(k, 1), np.float32)
    w1 = np.zeros(max(k, 1), np.float32)
    dl = np.zeros(max(k, 1), np.uint8)
    pj = np.zeros(max(k, 1), np.uint32)
    _check(lib().dbsim_check_device_generator(arr, len(specs), int(target), _p(src, c_uint32), _p(w0, c_float),
                                              _p(w1, c_float), _p(dl, c_uint8), _p(pj, c_uint32), k, byref(n)))
    return src[:k], w0[:k], w1[:k], dl[:k], pj[:k]


def derive_constants(spec, **kw) -> list:
    """Derived per-population constants (dicts, members one after another) of one network
    (NetSpec) or an ensemble (list of NetSpec), computed by the library on the host
    without a device."""
    specs = list(spec) if isinstance(spec, (list, tuple)) else [spec]
    d, holder = make_desc(specs[0], **kw)
    arr, holders = _member_array(specs)
    n = c_uint32(0)
    rc = lib().dbsim_derive_constants(byref(d), arr, len(specs), None, 0, byref(n))
    if rc not in (OK, ETRUNC):
        _check(rc)
    out = (PopConstants * max(1, n.value))()
    _check(lib().dbsim_derive_constants(byref(d), arr, len(specs), out, n.value, byref(n)))
    U = 2 * specs[0].weights_per_edge
    return [out[q].as_dict(U) for q in range(n.value)]


class Built:
    """A network built on the host (dbsim_build: validation, plan and every table; no HIP
    call, so worker threads may build while another thread drives the GPU). Simulator(...,
    built=b) deploys it (dbsim_create_built), which consumes it."""

    def __init__(self, spec: NetSpec, record_regions: bool = True, spike_record_capacity: int = 0,
                 record_bins: int = 0, host_threads: Optional[int] = None, no_graph: bool = False,
                 single_pass: bool = False, host_record: bool = True, host_spike_capacity: int = 0,
                 host_build: bool = False, stream_permille: int = 0, arena_permille: int = 0):
        if host_threads is None:
            host_threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
        self.spec = spec
        self._desc, self._holder = make_desc(spec, record_regions, spike_record_capacity, record_bins, -1, None, None,
                                             host_threads, no_graph, single_pass, host_record, host_spike_capacity,
                                             host_build, stream_permille, arena_permille)
        h = c_void_p()
        _check(lib().dbsim_build(byref(self._desc), byref(h)))
        self._b = h

    def take(self):
        b, self._b = self._b, None
        if not b:
            raise ValueError("this built network was already deployed or freed")
        return b

    def free(self) -> None:
        if getattr(self, "_b", None):
            lib().dbsim_built_free(self._b)
            self._b = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Simulator:
    """One network (a NetSpec) or an ensemble (a list of NetSpec) on one GPU, driven
    through the C ABI.

    use_torch: take device memory from torch's caching allocator and queue work on
    torch's current HIP stream (otherwise the library uses hipMalloc and its own stream).
    For an ensemble, reads return global neuron ids; member(m) gives each member's
    id range and member_spikes / member_state its own view.
    static_region: create with dbsim_create_static (no device allocation; the device's
    static region of STATIC_BYTES, one such handle per device at a time).
    host_record: record every bin's spikes into a pinned host ring of host_spike_capacity
    entries (0: the library default), from which spikes() reads; off, spikes() copies from
    the device ring.
    stream_permille: records each super-tile stream holds per partition pass, in thousandths
    of its in-edges (0: the library default; 1000: every edge). Events that find their
    stream full are placed in the tile arena directly (stats()["spilled_events"]).
    arena_permille: likewise for each tile's arena slice per bin; events that find it full
    are summed into a per-target accumulator (stats()["overflow_events"]).
    built: deploy a network built on the host (Built, made from this same spec); the build's
    recording and form options apply, this call's device, stream and allocator.
    """

    def __init__(self, spec: NetSpec, record_regions: bool = True, use_torch: bool = True, device: int = 0,
                 spike_record_capacity: int = 0, record_bins: int = 0, host_threads: Optional[int] = None,
                 no_graph: bool = False, stream=None, single_pass: bool = False, static_region: bool = False,
                 host_record: bool = True, host_spike_capacity: int = 0, built: Optional["Built"] = None,
                 host_build: bool = False, stream_permille: int = 0, arena_permille: int = 0):
        L = lib()
        if host_threads is None:
            # the process's CPU share (OMP_NUM_THREADS) rather than every core of the machine
            host_threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
        self.spec = spec
        self._alloc = None
        stream_handle = None
        if use_torch:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible to torch")
            torch.cuda.set_device(device)
            st = stream if stream is not None else torch.cuda.current_stream(device)
            stream_handle = int(st.cuda_stream) or None
            if not static_region:  # dbsim_create_static takes no allocator
                self._alloc = _TorchAllocator(device, int(st.cuda_stream))
        self.specs = list(spec) if isinstance(spec, (list, tuple)) else [spec]
        first = self.specs[0]
        self._desc, self._holder = make_desc(first, record_regions, spike_record_capacity, record_bins, device,
                                             stream_handle, self._alloc, host_threads, no_graph, single_pass,
                                             host_record, host_spike_capacity, host_build, stream_permille,
                                             arena_permille)
        h = c_void_p()
        if isinstance(spec, (list, tuple)):
            self._members, self._member_holders = _member_array(self.specs)
            _check(L.dbsim_create_ensemble(byref(self._desc), self._members, len(self.specs), byref(h)))
        elif built is not None:  # the device phase of a network built on the host
            if built.spec is not spec:
                raise ValueError("built was made from another description")
            _check(L.dbsim_create_built(built.take(), byref(self._desc), byref(h)))
        elif static_region:
            _check(L.dbsim_create_static(byref(self._desc), byref(h)))
        else:
            _check(L.dbsim_create(byref(self._desc), byref(h)))
        self._h = h
        info = SimInfo()
        _check(L.dbsim_get_info(h, byref(info)))
        self.info = info
        self.N = int(info.num_neurons)
        self.U = int(info.receptors)
        self.S = int(info.steps_per_bin)
        self.steps_done = 0

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().dbsim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n: int) -> None:
        _check(lib().dbsim_step(self._h, int(n)))
        self.steps_done += int(n)

    def sync(self) -> None:
        _check(lib().dbsim_sync(self._h))

    def set_timing(self, on: bool) -> None:
        _check(lib().dbsim_set_timing(self._h, 1 if on else 0))

    def tuning(self) -> dict:
        t = SimTuning()
        _check(lib().dbsim_get_tuning(self._h, byref(t)))
        return {"scatter_wgs_per_cu": t.scatter_wgs_per_cu, "round_events": t.round_events,
                "chunks_per_wg": t.chunks_per_wg, "ahead_passes": t.ahead_passes}

    def set_tuning(self, scatter_wgs_per_cu: int = 2, round_events: int = 0, chunks_per_wg: int = 4,
                   ahead_passes: int = 0) -> None:
        t = SimTuning(int(scatter_wgs_per_cu), int(round_events), int(chunks_per_wg), int(ahead_passes))
        _check(lib().dbsim_set_tuning(self._h, byref(t)))

    def spikes(self, step_lo: int = 0, step_hi: Optional[int] = None):
        """(steps uint64, ids uint32) of completed bins, sorted by (step, id)."""
        hi = (1 << 63) if step_hi is None else int(step_hi)
        n = c_uint64(0)
        rc = lib().dbsim_read_spikes(self._h, int(step_lo), hi, None, None, 0, byref(n))
        if rc not in (OK, ETRUNC):
            _check(rc)
        cap = int(n.value)
        st = np.zeros(max(cap, 1), np.uint64)
        ids = np.zeros(max(cap, 1), np.uint32)
        _check(lib().dbsim_read_spikes(self._h, int(step_lo), hi, _p(st, c_uint64), _p(ids, c_uint32), cap, byref(n)))
        return st[: n.value], ids[: n.value]

    def member(self, m: int):
        """(first global neuron id, neurons, first global region, regions) of member m."""
        mi = SimMember()
        _check(lib().dbsim_member_info(self._h, int(m), byref(mi)))
        return int(mi.first_neuron), int(mi.num_neurons), int(mi.first_region), int(mi.num_regions)

    def member_spikes(self, m: int, step_lo: int = 0, step_hi: Optional[int] = None):
        """Spikes of member m with member-local neuron ids."""
        a, n, _, _ = self.member(m)
        st, ids = self.spikes(step_lo, step_hi)
        sel = (ids >= a) & (ids < a + n)
        return st[sel], (ids[sel] - a).astype(np.uint32)

    def member_state(self, m: int):
        a, n, _, _ = self.member(m)
        V, J, ref = self.state()
        return V[a:a + n], J[:, a:a + n], ref[a:a + n]

    def set_bold(self, params: Optional[BoldParams] = None, **overrides) -> None:
        """Turns the region BOLD model on (defaults, optionally overridden) and resets it
        to rest; set_bold(False) turns it off."""
        if params is False:
            _check(lib().dbsim_set_bold(self._h, None))
            return
        p = params if params is not None else bold_defaults()
        for k, v in overrides.items():
            setattr(p, k, v)
        _check(lib().dbsim_set_bold(self._h, byref(p)))

    def set_spike_injection(self, prob, bins: int) -> None:
        """Initial spike injection for the next `bins` bins: per-population probability per
        bin (a scalar applies to every population); bins = 0 turns it off."""
        n = sum(len(sp.pops) for sp in self.specs)
        pr = np.broadcast_to(np.asarray(prob, np.float32), (n,)).copy()
        _check(lib().dbsim_set_spike_injection(self._h, _p(pr, c_float), n, int(bins)))

    def set_ou_background(self, mu, sigma, tau_ms) -> None:
        """OU background current per population (scalars apply to every population);
        tau_ms <= 0 turns it off for that population."""
        n = sum(len(sp.pops) for sp in self.specs)
        a = [np.broadcast_to(np.asarray(x, np.float32), (n,)).copy() for x in (mu, sigma, tau_ms)]
        _check(lib().dbsim_set_ou_background(self._h, _p(a[0], c_float), _p(a[1], c_float), _p(a[2], c_float), n))

    def bold(self, sample_lo: int = 0, sample_hi: Optional[int] = None) -> np.ndarray:
        """BOLD samples [samples][regions]."""
        R = int(self.info.n_regions)
        if sample_hi is None:
            sample_hi = self.bold_state()[1]
        nb = max(0, int(sample_hi) - int(sample_lo))
        y = np.zeros(max(nb * R, 1), np.float64)
        n = c_uint64(0)
        _check(lib().dbsim_read_bold(self._h, int(sample_lo), int(sample_hi), _p(y, c_double), nb * R, byref(n)))
        return y[: nb * R].reshape(nb, R)

    def bold_state(self):
        """(state [4][regions]: s, f, v, q; samples taken)."""
        R = int(self.info.n_regions)
        st = np.zeros(4 * R, np.float64)
        n = c_uint64(0)
        _check(lib().dbsim_read_bold_state(self._h, _p(st, c_double), byref(n)))
        return st.reshape(4, R), int(n.value)

    def region_signal(self, bin_lo: int = 0, bin_hi: Optional[int] = None):
        R = int(self.info.n_regions)
        hi = (self.steps_done // self.S) if bin_hi is None else int(bin_hi)
        nb = max(0, hi - int(bin_lo))
        sig = np.zeros(max(nb * R, 1), np.float64)
        cnt = np.zeros(max(nb * R, 1), np.uint32)
        n = c_uint64(0)
        _check(lib().dbsim_read_region_signal(self._h, int(bin_lo), hi, _p(sig, c_double), _p(cnt, c_uint32),
                                              nb * R, byref(n)))
        k = int(n.value) // R
        return sig[: k * R].reshape(k, R), cnt[: k * R].reshape(k, R)

    def state(self):
        V = np.zeros(self.N, np.float32)
        J = np.zeros(self.U * self.N, np.float32)
        ref = np.zeros(self.N, np.int32)
        _check(lib().dbsim_read_state(self._h, _p(V, c_float), _p(J, c_float), _p(ref, c_int32)))
        return V, J.reshape(self.U, self.N), ref

    def receptor_currents(self) -> np.ndarray:
        """[n_pops, 4] mean current per receptor (AMPA, NMDA, GABA_A, GABA_B) of every
        population at the current state, reduced on the device (Suppl. Algorithm 1)."""
        n = sum(len(sp.pops) for sp in self.specs)
        out = np.zeros(4 * n, np.float64)
        _check(lib().dbsim_receptor_currents(self._h, _p(out, c_double), n))
        return out.reshape(n, 4)

    def write_state(self, V, J, ref) -> None:
        V = np.ascontiguousarray(V, np.float32)
        J = np.ascontiguousarray(J, np.float32).reshape(-1)
        ref = np.ascontiguousarray(ref, np.int32)
        _check(lib().dbsim_write_state(self._h, _p(V, c_float), _p(J, c_float), _p(ref, c_int32)))

    def checkpoint(self) -> bytes:
        """Byte image of the run's state at the current bin boundary (dbsim_checkpoint_save)."""
        n = c_uint64(0)
        _check(lib().dbsim_checkpoint_size(self._h, byref(n)))
        buf = np.zeros(int(n.value), np.uint8)
        _check(lib().dbsim_checkpoint_save(self._h, buf.ctypes.data_as(c_void_p), buf.size, byref(n)))
        return buf[: int(n.value)].tobytes()

    def restore(self, image: bytes) -> None:
        """Loads a checkpoint into this not yet stepped handle (dbsim_checkpoint_restore)."""
        buf = np.frombuffer(image, np.uint8)
        _check(lib().dbsim_checkpoint_restore(self._h, buf.ctypes.data_as(c_void_p), buf.size))
        self.steps_done = int(self.stats()["steps"])

    def export_csr(self, edges: bool = True):
        """(row_ptr, seg [N, D+1], tgt, w0, w1); with edges=False only row_ptr and seg."""
        E = int(self.info.num_edges)
        D = int(self.info.max_delay)
        row_ptr = np.zeros(self.N + 1, np.uint64)
        seg = np.zeros(self.N * (D + 1), np.uint32)
        if not edges:
            _check(lib().dbsim_export_csr(self._h, _p(row_ptr, c_uint64), _p(seg, c_uint32), None, None, None))
            return row_ptr, seg.reshape(self.N, D + 1), None, None, None
        tgt = np.zeros(max(E, 1), np.uint32)
        w0 = np.zeros(max(E, 1), np.float32)
        w1 = np.zeros(max(E, 1), np.float32)
        _check(lib().dbsim_export_csr(self._h, _p(row_ptr, c_uint64), _p(seg, c_uint32), _p(tgt, c_uint32),
                                      _p(w0, c_float), _p(w1, c_float)))
        return row_ptr, seg.reshape(self.N, D + 1), tgt[:E], w0[:E], w1[:E]

    def export_network(self) -> dict:
        """The network the handle built: CSR (row_ptr, seg [N, D+1], tgt, w0, w1), the initial
        potentials V0 and the per-population constants read back from the device."""
        E = int(self.info.num_edges)
        D = int(self.info.max_delay)
        n_pops = sum(len(sp.pops) for sp in self.specs)
        row_ptr = np.zeros(self.N + 1, np.uint64)
        seg = np.zeros(self.N * (D + 1), np.uint32)
        tgt = np.zeros(max(E, 1), np.uint32)
        w0 = np.zeros(max(E, 1), np.float32)
        w1 = np.zeros(max(E, 1), np.float32)
        V0 = np.zeros(max(self.N, 1), np.float32)
        pops = (PopConstants * max(1, n_pops))()
        v = NetworkView(_p(row_ptr, c_uint64), _p(seg, c_uint32), _p(tgt, c_uint32), _p(w0, c_float), _p(w1, c_float),
                        _p(V0, c_float), pops, n_pops, 0)
        _check(lib().dbsim_export_network(self._h, byref(v)))
        return {"row_ptr": row_ptr, "seg": seg.reshape(self.N, D + 1), "tgt": tgt[:E], "w0": w0[:E], "w1": w1[:E],
                "V0": V0[:self.N], "pops": [pops[q].as_dict(self.U) for q in range(v.n_pops)]}

    def stats(self) -> dict:
        s = SimStats()
        _check(lib().dbsim_get_stats(self._h, byref(s)))
        return {f: getattr(s, f) for f, _ in SimStats._fields_}

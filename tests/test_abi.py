"""CPU checks of the C-ABI library: it loads, exports every declared symbol, its
structs match the ctypes mirrors, and description errors are reported before any
device work."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from netgen import configs
from netgen.desc import Desc, Pop, Proj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2211_15963_amd import dbsim as D
    if not os.path.exists(D.LIB_PATH):
        import paper_2211_15963_amd.build as b
        b.build()
    return D.lib()


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(dbsim_\w+|dbnet_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol(L):
    names = _declared("dbsim.h") + _declared("dbnet.h")
    assert "dbsim_create" in names and "dbnet_in_edges" in names
    for nm in names:
        assert hasattr(L, nm), f"libdbsim.so does not export {nm}"


def test_generator_library_exports(L):
    from netgen.desc import load_generator
    G = load_generator()
    for nm in _declared("dbnet.h"):
        assert hasattr(G, nm)


LAYOUT_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "dbsim.h"
#define P(T) printf(#T " %zu\n", sizeof(T))
#define O(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  P(dbnet_pop); P(dbnet_proj); P(dbnet_desc); P(dbsim_desc); P(dbsim_stats); P(dbsim_info);
  O(dbnet_desc, seed); O(dbnet_desc, pops); O(dbnet_desc, region_xyz_mm);
  O(dbsim_desc, net); O(dbsim_desc, spike_record_capacity); O(dbsim_desc, hip_stream); O(dbsim_desc, flags);
  O(dbsim_desc, host_spike_capacity); O(dbsim_desc, stream_permille); O(dbsim_desc, arena_permille);
  O(dbsim_stats, ms_scatter); O(dbsim_stats, build_seconds); O(dbsim_stats, spilled_events); O(dbsim_stats, overflow_events);
  O(dbsim_info, frac_bits); O(dbsim_info, n_members); O(dbsim_info, fanin_passes); O(dbsim_info, stream_records); O(dbsim_info, arena_records);
  P(dbsim_member); O(dbsim_member, first_region);
  P(dbsim_bold_params); O(dbsim_bold_params, activity_scale); O(dbsim_bold_params, tr_bins);
  return 0;
}
"""


def test_struct_layouts_match_ctypes(L):
    from paper_2211_15963_amd import dbsim as D
    d = tempfile.mkdtemp()
    src, exe = os.path.join(d, "p.c"), os.path.join(d, "p")
    open(src, "w").write(LAYOUT_PROBE)
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
    out = dict(line.split() for line in subprocess.run([exe], capture_output=True, text=True).stdout.splitlines())
    assert int(out["dbnet_pop"]) == ctypes.sizeof(Pop)
    assert int(out["dbnet_proj"]) == ctypes.sizeof(Proj)
    assert int(out["dbnet_desc"]) == ctypes.sizeof(Desc)
    assert int(out["dbsim_desc"]) == ctypes.sizeof(D.SimDesc)
    assert int(out["dbsim_stats"]) == ctypes.sizeof(D.SimStats)
    assert int(out["dbsim_info"]) == ctypes.sizeof(D.SimInfo)
    assert int(out["dbnet_desc.seed"]) == Desc.seed.offset
    assert int(out["dbnet_desc.pops"]) == Desc.pops.offset
    assert int(out["dbsim_desc.net"]) == D.SimDesc.net.offset
    assert int(out["dbsim_desc.hip_stream"]) == D.SimDesc.hip_stream.offset
    assert int(out["dbsim_desc.flags"]) == D.SimDesc.flags.offset
    assert int(out["dbsim_desc.host_spike_capacity"]) == D.SimDesc.host_spike_capacity.offset
    assert int(out["dbsim_desc.stream_permille"]) == D.SimDesc.stream_permille.offset
    assert int(out["dbsim_stats.ms_scatter"]) == D.SimStats.ms_scatter.offset
    assert int(out["dbsim_stats.spilled_events"]) == D.SimStats.spilled_events.offset
    assert int(out["dbsim_info.stream_records"]) == D.SimInfo.stream_records.offset
    assert int(out["dbsim_desc.arena_permille"]) == D.SimDesc.arena_permille.offset
    assert int(out["dbsim_stats.overflow_events"]) == D.SimStats.overflow_events.offset
    assert int(out["dbsim_info.arena_records"]) == D.SimInfo.arena_records.offset
    assert int(out["dbsim_info.frac_bits"]) == D.SimInfo.frac_bits.offset
    assert int(out["dbsim_info.n_members"]) == D.SimInfo.n_members.offset
    assert int(out["dbsim_info.fanin_passes"]) == D.SimInfo.fanin_passes.offset
    assert int(out["dbsim_member"]) == ctypes.sizeof(D.SimMember)
    assert int(out["dbsim_member.first_region"]) == D.SimMember.first_region.offset
    assert int(out["dbsim_bold_params"]) == ctypes.sizeof(D.BoldParams)
    assert int(out["dbsim_bold_params.activity_scale"]) == D.BoldParams.activity_scale.offset
    assert int(out["dbsim_bold_params.tr_bins"]) == D.BoldParams.tr_bins.offset


def _create(L, spec, **kw):
    from paper_2211_15963_amd import dbsim as D
    d, holder = D.make_desc(spec, **kw)
    h = ctypes.c_void_p()
    rc = L.dbsim_create(ctypes.byref(d), ctypes.byref(h))
    return rc, L.dbsim_last_error().decode(), h


def test_description_errors_before_device_work(L):
    from paper_2211_15963_amd import dbsim as D
    s = configs.tiny()
    s.pops[0].T_ref = 0.5   # shorter than a bin: two spikes per bin would be possible
    rc, msg, _ = _create(L, s)
    assert rc == D.EINVAL and "T_ref" in msg
    s = configs.tiny()
    s.receptor_mask = 0x3
    rc, msg, _ = _create(L, s)
    assert rc == D.EINVAL and "receptor_mask" in msg
    s = configs.tiny(bg_rate_hz=5e6)
    rc, msg, _ = _create(L, s)
    assert rc == D.EINVAL and "background" in msg
    s = configs.tiny()
    s.pops[0].T_ref = 30.0  # 300 steps > 255
    rc, msg, _ = _create(L, s)
    assert rc == D.EINVAL and "255" in msg


def test_null_arguments(L):
    from paper_2211_15963_amd import dbsim as D
    assert L.dbsim_create(None, None) == D.EINVAL
    assert L.dbsim_step(None, 10) == D.EINVAL
    assert L.dbsim_destroy(None) == D.OK
    assert L.dbsim_sync(None) == D.EINVAL


def _stream_records(n, k, permille=0, tile=4096, even=True):
    """Records of the super-tile streams of a one-population network of n neurons with
    in-degree k (at most 64 super-tiles, so one tile each up to 64 tiles): a share of each
    super-tile's in-edges, by default 1/8 and at least 2^20 records (or all of them)."""
    T = (n + tile - 1) // tile
    per = 1
    while (T + per - 1) // per > 64:
        per *= 2
    total = 0
    for x in range((T + per - 1) // per):
        lo, hi = x * per * tile, min(n, (x + 1) * per * tile)
        inn = k * (hi - lo)
        ln = -(-inn * (permille or 125) // 1000)
        if not permille:
            ln = max(ln, min(inn, 1 << 20))
        ln = max(ln, 2)
        total += ln + (ln & 1 if even else 0)
    return total


def _arena_records(n, k, permille=0, tile=4096):
    """Records of the tile arena of a one-population network: a share of each tile's
    in-edges, by default 1/8 and at least 2^16 records (or all of them)."""
    total = 0
    for lo in range(0, n, tile):
        inn = k * (min(n, lo + tile) - lo)
        ln = -(-inn * (permille or 125) // 1000)
        if not permille:
            ln = max(ln, min(inn, 1 << 16))
        total += max(ln, 1)
    return total


def test_footprint_matches_layout(L):
    from paper_2211_15963_amd import dbsim as D
    n, k = 100000, 556
    s = configs.share(n=n, indegree=k)
    E = s.num_edges()
    assert E == n * k
    # every edge in the intermediate buffers: 12 B edge records (target and two weights), 10 B
    # narrow super-tile stream records and 10 B tile arena records (2 B key beside the
    # weights) per edge, and the per-target overflow sums (4 receptors x 8 B)
    fpw = D.footprint(s, stream_permille=1000, arena_permille=1000)
    assert 32 * E + 32 * n < fpw < 32 * E + 32 * n + 60 * n + (64 << 20)
    # default: a share of each super-tile's and tile's in-edges; the arena's weight slot holds
    # the device construction's temporaries at least (E bytes of projections, 12 B of counts
    # and cursors per (neuron, delay), 16 B of row lengths and starts per neuron)
    fp = D.footprint(s)
    st, ta = _stream_records(n, k), _arena_records(n, k)
    assert st < E // 2 and ta < E // 2
    gen = E + 12 * n * 10 + 16 * n
    lo = 12 * E + 10 * st + 2 * ta + max(8 * ta, gen) + 32 * n
    assert lo < fp < lo + 60 * n + (64 << 20)
    # with the construction on the host the arena is its own size
    fph = D.footprint(s, host_build=True)
    lo = 12 * E + 10 * st + 10 * ta + 32 * n
    assert lo < fph < lo + 60 * n + (64 << 20)
    # 12 B stream records where a weight may be negative
    neg = configs.share(n=n, indegree=k)
    neg.projs[0].w_scale_inh = -4.0
    fpn = D.footprint(neg, stream_permille=250, arena_permille=1000, host_build=True)
    st = 12 * _stream_records(n, k, 250, even=False)
    assert 22 * E + st < fpn < 22 * E + st + 32 * n + 60 * n + (64 << 20)
    with pytest.raises(D.DbsimError, match="stream_permille"):
        D.footprint(s, stream_permille=1001)
    with pytest.raises(D.DbsimError, match="arena_permille"):
        D.footprint(s, arena_permille=1001)
    # single pass: the 12 B edge records and the event arena of 256-record blocks (2 B key +
    # 8 B weights + a 4 B count per block): every one of the 25 tiles of 4096 neurons gets its
    # in-degree in whole blocks plus two part-filled blocks per workgroup (at most 512) and bin
    def arena(n, k, T, K=256, G=512):
        tin = [k * (min(n, (t + 1) * 4096) - t * 4096) for t in range(T)]
        blocks = sum(x // K + 2 * G for x in tin)
        return blocks * K * 10 + blocks * 4
    fp1 = D.footprint(s, single_pass=True)
    lo = 12 * E + arena(100000, 556, 25)
    assert lo < fp1 < lo + 60 * 100000 + (64 << 20)
    # 1490 tiles still fit the carry buffers (8 records each)
    s = configs.share(n=6100000, indegree=20)
    fp1, E = D.footprint(s, single_pass=True), s.num_edges()
    lo = 12 * E + arena(6100000, 20, 1490)
    # per neuron: a 64 B row header, the state, and the spike-history ring of at least
    # (D + 1) N entries rounded up to a power of two
    assert lo < fp1 < lo + 220 * 6100000 + (64 << 20)
    fp2 = D.footprint(s, host_build=True)
    st, ta = 10 * _stream_records(6100000, 20), 10 * _arena_records(6100000, 20)
    lo = 12 * E + st + ta + 32 * 6100000
    assert lo < fp2 < lo + 220 * 6100000 + (64 << 20)


def test_ensemble_footprint_and_validation(L):
    from paper_2211_15963_amd import dbsim as D
    a = configs.share(n=20000, indegree=100, seed=1)
    b = configs.share(n=30000, indegree=200, seed=2)
    fa, fb, fab = D.footprint(a), D.footprint(b), D.footprint([a, b])
    assert fab > max(fa, fb)
    c = configs.tiny()   # two receptors: cannot share kernels with four-receptor members
    with pytest.raises(D.DbsimError, match="share dt_ms"):
        D.footprint([a, c])


def test_host_build_phase_runs_on_threads_without_a_device(L):
    """dbsim_build makes no HIP call: several networks build at once on worker threads (as the
    server does) on a machine without a GPU; deploying one here fails cleanly (no device) and
    consumes it; an unused build is freed."""
    import concurrent.futures as cf
    from paper_2211_15963_amd import dbsim as D
    specs = [configs.share(n=3000 + 500 * k, indegree=80, seed=40 + k) for k in range(4)] + [configs.tiny(seed=44)]
    with cf.ThreadPoolExecutor(max_workers=3) as ex:
        built = list(ex.map(lambda s: D.Built(s, host_threads=2), specs))
    assert all(b._b for b in built)
    b = built[0]
    h = ctypes.c_void_p()
    d, holder = D.make_desc(specs[0])
    rc = L.dbsim_create_built(b.take(), ctypes.byref(d), ctypes.byref(h))
    assert rc == D.EDEVICE and not h.value
    for b in built[1:]:
        b.free()
    bad = configs.tiny()
    bad.pops[0].T_ref = 0.5
    with pytest.raises(D.DbsimError) as e:
        D.Built(bad)
    assert e.value.code == D.EINVAL and "T_ref" in str(e.value)

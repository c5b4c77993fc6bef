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
  O(dbsim_stats, ms_scatter); O(dbsim_stats, build_seconds); O(dbsim_info, frac_bits); O(dbsim_info, n_members);
  O(dbsim_info, fanin_passes);
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
    assert int(out["dbsim_stats.ms_scatter"]) == D.SimStats.ms_scatter.offset
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


def test_footprint_matches_layout(L):
    from paper_2211_15963_amd import dbsim as D
    s = configs.share(n=100000, indegree=556)
    fp = D.footprint(s)
    E = s.num_edges()
    assert E == 100000 * 556
    # dominant terms: targets (4 B), two weights (8 B) and the tile arena record (12 B) per
    # edge; 25 tiles of 4096 neurons are written directly in 16-record chunks, with room
    # for one padded chunk per partition workgroup (at most 2048) and launch (two per bin)
    # in every tile slice
    pad = 25 * (15 + 2 * 16 * 2048) * 12
    assert 24 * E + pad < fp < 24 * E + pad + 60 * 100000 + (64 << 20)
    # 1490 tiles are too many for the write-combining buffers: two passes, with a 12 B
    # super-tile stream record per edge as well
    s = configs.share(n=6100000, indegree=20)
    fp, E = D.footprint(s), s.num_edges()
    # per neuron: a 64 B row header, the state, and the spike-history ring of at least
    # (D + 1) N entries rounded up to a power of two
    assert 36 * E < fp < 36 * E + 220 * 6100000 + (64 << 20)


def test_ensemble_footprint_and_validation(L):
    from paper_2211_15963_amd import dbsim as D
    a = configs.share(n=20000, indegree=100, seed=1)
    b = configs.share(n=30000, indegree=200, seed=2)
    fa, fb, fab = D.footprint(a), D.footprint(b), D.footprint([a, b])
    assert fab > max(fa, fb)
    c = configs.tiny()   # two receptors: cannot share kernels with four-receptor members
    with pytest.raises(D.DbsimError, match="share dt_ms"):
        D.footprint([a, c])

"""C-ABI checks that need no GPU: the library loads, exports every function
include/dm.h declares, sizes workspaces, and rejects bad input with the
documented status code before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1808_10375_amd import dm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dm.h")

pytestmark = pytest.mark.skipif(not os.path.exists(dm.LIB_PATH),
                                reason="libdm.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dm_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(dm.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(dm.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_struct_layouts():
    assert ctypes.sizeof(dm.dm_desc) == 36
    assert ctypes.sizeof(dm.dm_errors) == 80
    assert ctypes.sizeof(dm.dm_tuning) == 16


def desc(**kw):
    base = dict(n_frames=10, frame=32, n_modes=2, obj_h=100, obj_w=90, beta=0.8)
    base.update(kw)
    return dm.make_desc(**base)


def test_workspace_bytes_valid_and_invalid():
    n = dm.dm_workspace_bytes(desc())
    psi = 10 * 2 * 32 * 32 * 8
    assert n > psi
    assert dm.dm_workspace_bytes(desc(n_frames=20)) > n
    for bad in (dict(frame=48), dict(frame=8), dict(frame=512), dict(n_modes=0),
                dict(n_modes=17), dict(beta=1.5), dict(beta=-0.1), dict(obj_h=16),
                dict(n_frames=0), dict(precision=7), dict(flags=32), dict(flags=6)):
        assert dm.dm_workspace_bytes(desc(**bad)) == 0, bad
    # the paper's frame edges 188 and 200 run the three-kernel path: psi
    # and the spectrum buffer
    for f in (188, 200):
        assert dm.dm_workspace_bytes(desc(frame=f, obj_h=300, obj_w=300)) > \
            2 * 10 * 2 * f * f * 8, f
    for bad in (dict(frame=189), dict(frame=100), dict(frame=200, precision=dm.DM_BF16X3_DFT)):
        assert dm.dm_workspace_bytes(desc(obj_h=300, obj_w=300, **bad)) == 0, bad
    # F = 256 needs the multi-pass spectrum buffer as well
    d256 = desc(frame=256, obj_h=300, obj_w=300)
    assert dm.dm_workspace_bytes(d256) > 2 * 10 * 2 * 256 * 256 * 8
    # the BF16x3 form holds a full spectrum buffer plus its 128 KB split DFT
    # matrix; the FP32 path at F <= 128 holds spectra for at most 256 views
    # in flight (one slot per persistent workgroup of the streamed kernel)
    f32 = desc(frame=128, obj_h=200, obj_w=200)
    b16 = desc(frame=128, obj_h=200, obj_w=200, precision=dm.DM_BF16X3_DFT)
    ff = 128 * 128
    # BF16x3: spectrum buffer [N][M][F][F] + split DFT matrix; FP32: one slot
    # per view in flight (here all 10) of M spectra and a float scale
    expect = (10 * 2 * ff * 8 + 128 * 1024) - 10 * ff * (8 * 2 + 4)
    got = dm.dm_workspace_bytes(b16) - dm.dm_workspace_bytes(f32)
    assert abs(got - expect) <= 4096, (got, expect)
    many = dict(frame=128, obj_h=200, obj_w=200, n_frames=600)
    more = dict(many, n_frames=700)
    per_view = 2 * 128 * 128 * 8 + 128 * 128 * (8 + 4) + 2 * 4 + 4 + 4
    grown = dm.dm_workspace_bytes(desc(**more)) - dm.dm_workspace_bytes(desc(**many))
    assert 100 * per_view <= grown <= 100 * per_view + 64 * 1024


def test_workspace_bytes_object_modes():
    """L object modes: psi and the spectrum buffer hold L M frames per view,
    the object L planes, and the view numerators L per view; L > 1 takes the
    three-kernel path (spectrum buffer) at any power-of-two F."""
    one = desc(frame=64, obj_h=200, obj_w=200, flags=dm.DM_FLAG_MULTIPASS)
    two = desc(frame=64, obj_h=200, obj_w=200, n_obj_modes=2)
    ff = 64 * 64
    grown = dm.dm_workspace_bytes(two) - dm.dm_workspace_bytes(one)
    expect = 2 * 10 * 2 * ff * 8 + 10 * ff * 8 + 200 * 200 * 8
    assert expect <= grown <= expect + 128 * 1024, (grown, expect)
    assert dm.dm_workspace_bytes(desc(n_obj_modes=1)) == dm.dm_workspace_bytes(desc())
    for bad in (dict(n_obj_modes=-1), dict(n_obj_modes=5), dict(n_obj_modes=3, n_modes=11),
                dict(n_obj_modes=2, frame=188, obj_h=300, obj_w=300),
                dict(n_obj_modes=2, frame=128, obj_h=200, obj_w=200,
                     precision=dm.DM_BF16X3_DFT)):
        assert dm.dm_workspace_bytes(desc(**bad)) == 0, bad
    assert dm.dm_workspace_bytes(desc(n_obj_modes=4, n_modes=8)) > 0


def _init_status(d, pos, ws_bytes=None, ptrs=(256, 256, 256, 256)):
    L = dm.lib()
    ctx = ctypes.c_void_p()
    pos = np.ascontiguousarray(np.asarray(pos, dtype=np.int32))
    ws = dm.dm_workspace_bytes(d) if ws_bytes is None else ws_bytes
    st = L.dm_init(ctypes.byref(ctx), ctypes.byref(d), ptrs[0],
                   pos.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ptrs[1], ptrs[2],
                   ptrs[3], ws, None)
    assert not ctx.value
    return st, dm.dm_last_error(None)


def test_init_rejects_out_of_bounds_positions():
    d = desc()
    pos = np.zeros((10, 2), np.int32)
    pos[3] = (100 - 32 + 1, 0)
    st, msg = _init_status(d, pos)
    assert st == dm.DM_E_BOUNDS and "view 3" in msg
    pos[3] = (0, -1)
    assert _init_status(d, pos)[0] == dm.DM_E_BOUNDS


def test_init_rejects_small_workspace_and_bad_pointers():
    d = desc()
    pos = np.zeros((10, 2), np.int32)
    assert _init_status(d, pos, ws_bytes=dm.dm_workspace_bytes(d) - 1)[0] == dm.DM_E_WORKSPACE
    assert _init_status(d, pos, ptrs=(0, 256, 256, 256))[0] == dm.DM_E_ARG
    assert _init_status(d, pos, ptrs=(260, 256, 256, 256))[0] == dm.DM_E_ARG  # misaligned I
    assert _init_status(d, pos, ptrs=(256, 256, 256, 264))[0] == dm.DM_E_ARG  # workspace
    assert _init_status(desc(frame=24), pos)[0] == dm.DM_E_UNSUPPORTED
    assert _init_status(desc(beta=2.0), pos)[0] == dm.DM_E_ARG
    assert _init_status(desc(precision=dm.DM_BF16X3_DFT, frame=64), pos)[0] \
        == dm.DM_E_UNSUPPORTED
    big = desc(precision=dm.DM_BF16X3_DFT, frame=128, obj_h=200, obj_w=200, n_modes=9)
    assert _init_status(big, pos)[0] == dm.DM_E_UNSUPPORTED


def test_calls_on_null_context():
    L = dm.lib()
    assert L.dm_iterate(None, 1) == dm.DM_E_ARG
    assert L.dm_error(None, ctypes.byref(dm.dm_errors())) == dm.DM_E_ARG
    assert L.dm_iterations(None) == -1
    L.dm_free(None)
    for s in range(0, -8, -1):
        assert dm.dm_status_str(s).startswith("DM_")


def test_batch_workspace_and_validation():
    a = desc(n_frames=10)
    b = desc(n_frames=30, obj_h=120, obj_w=100, beta=0.5)
    one = dm.dm_batch_workspace_bytes([a])
    assert one == dm.dm_workspace_bytes(a)
    two = dm.dm_batch_workspace_bytes([a, b])
    assert two > one + dm.dm_workspace_bytes(b) // 2
    # mixed frame sizes or mode counts are rejected
    assert dm.dm_batch_workspace_bytes([a, desc(frame=64)]) == 0
    assert dm.dm_batch_workspace_bytes([a, desc(n_modes=3)]) == 0
    assert dm.dm_batch_workspace_bytes([a, desc(flags=1)]) == 0


def test_batch_init_bounds_reported_per_scan():
    import numpy as np
    a = desc(n_frames=4)
    b = desc(n_frames=3)
    L = dm.lib()
    arr = (dm.dm_desc * 2)(a, b)
    pa = np.zeros((4, 2), np.int32)
    pb = np.zeros((3, 2), np.int32)
    pb[2] = (0, 90)
    vp = ctypes.c_void_p
    ptrs = (vp * 2)(256, 256)
    pos_arr = (ctypes.POINTER(ctypes.c_int32) * 2)(
        pa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        pb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    ctx = ctypes.c_void_p()
    st = L.dm_batch_init(ctypes.byref(ctx), 2, arr, ptrs, pos_arr, ptrs, ptrs, 256,
                         dm.dm_batch_workspace_bytes([a, b]), None)
    assert st == dm.DM_E_BOUNDS and "scan 1: view 2" in dm.dm_last_error(None)
    # graph capture needs a stream
    g = desc(n_frames=4, flags=dm.DM_FLAG_GRAPH)
    arr1 = (dm.dm_desc * 1)(g)
    st = L.dm_batch_init(ctypes.byref(ctx), 1, arr1, ptrs, pos_arr, ptrs, ptrs, 256,
                         dm.dm_batch_workspace_bytes([g]), None)
    assert st == dm.DM_E_ARG and "stream" in dm.dm_last_error(None)


# ---- warm-start network (include/dmnet.h) --------------------------------
NET_HEADER = os.path.join(ROOT, "include", "dmnet.h")


def net_declared_functions():
    text = open(NET_HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmnet_[a-z_]+)\s*\(", text)))


def test_dmnet_header_binding_and_exports_agree():
    from paper_1808_10375_amd import dmnet
    assert net_declared_functions() == sorted(dmnet.EXPORTED)
    L = ctypes.CDLL(dm.LIB_PATH)
    for name in net_declared_functions():
        assert hasattr(L, name), name
    assert ctypes.sizeof(dmnet.dmnet_desc) == 40


def test_dmnet_parameter_count_matches_oracle_layout():
    from oracle import cnn_oracle
    from paper_1808_10375_amd import dmnet
    for c0, levels in ((32, 4), (4, 3), (2, 2), (3, 5)):
        d = dmnet.make_desc(2, size=32, base_ch=c0, levels=levels)
        assert dmnet.dmnet_n_params(d) == cnn_oracle.n_params(c0, levels)
    assert dmnet.dmnet_n_params(dmnet.make_desc(1)) == cnn_oracle.n_params(32, 4)


def test_dmnet_rejects_invalid_descriptions():
    from paper_1808_10375_amd import dmnet
    good = dmnet.make_desc(4, size=64)
    assert dmnet.dmnet_workspace_bytes(good) > 4 * 2 * 64 * 64 * 4
    for bad in (dict(batch=0), dict(size=36), dict(levels=1), dict(levels=7),
                dict(base_ch=0), dict(lr=0.0), dict(beta1=1.0), dict(flags=2)):
        kw = dict(batch=4, size=64)
        kw.update(bad)
        d = dmnet.make_desc(**kw)
        assert dmnet.dmnet_workspace_bytes(d) == 0, bad
        assert dmnet.dmnet_n_params(d) == 0, bad
    L = dmnet.lib()
    net = ctypes.c_void_p()
    need = dmnet.dmnet_workspace_bytes(good)
    assert L.dmnet_create(ctypes.byref(net), ctypes.byref(good), None, need, None) == dm.DM_E_ARG
    assert L.dmnet_create(ctypes.byref(net), ctypes.byref(good), 256, need - 1,
                          None) == dm.DM_E_WORKSPACE
    assert L.dmnet_create(ctypes.byref(net), ctypes.byref(good), 264, need,
                          None) == dm.DM_E_ARG  # misaligned workspace
    assert not net.value
    assert L.dmnet_forward(None, 256, 256, 1) == dm.DM_E_ARG
    L.dmnet_free(None)


def test_warm_start_on_null_context():
    L = dm.lib()
    assert L.dm_warm_start(None, 256) == dm.DM_E_ARG
    assert L.dm_scan_warm_start(None, 0, 256) == dm.DM_E_ARG

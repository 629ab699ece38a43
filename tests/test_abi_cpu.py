"""CPU checks of the C ABI: the library loads without a GPU and exports every function
include/fd3d.h declares; host-only calls validate their arguments."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?(?:int|void|char|size_t)\s*\*?\s*(fd3d_\w+)\s*\(", text, re.M))
    return names


def test_every_declared_symbol_is_exported():
    import ctypes

    from paper_2112_15071_amd import _abi

    names = declared()
    assert len(names) >= 9
    lib = ctypes.CDLL(_abi.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names <= set(_abi.exported_symbols()) | set(), names - set(_abi.exported_symbols())


def test_host_only_calls():
    from paper_2112_15071_amd import _abi

    assert _abi.fd3d_version().startswith("fd3d")
    o = _abi.fd3d_opts()
    o.dtype = _abi.FD3D_F32
    a = _abi.fd3d_workspace_bytes(64, 64, 64, o)
    o.dtype = _abi.FD3D_F64
    b = _abi.fd3d_workspace_bytes(64, 64, 64, o)
    assert a >= 9 * 64 ** 3 * 4 and b >= 9 * 64 ** 3 * 8
    for bad in [(3, 64, 64), (64, 0, 64)]:
        with pytest.raises(_abi.FD3DError) as e:
            _abi.fd3d_workspace_bytes(*bad, o)
        assert e.value.code == _abi.FD3D_EINVAL
    o.dtype = 7
    with pytest.raises(_abi.FD3DError):
        _abi.fd3d_workspace_bytes(64, 64, 64, o)
    o.dtype = 0
    o.sponge[2] = -1
    with pytest.raises(_abi.FD3DError):
        _abi.fd3d_workspace_bytes(64, 64, 64, o)
    assert "sponge" in _abi.fd3d_last_error()
    o.sponge[2] = 0
    o.dz = -1.0
    with pytest.raises(_abi.FD3DError):
        _abi.fd3d_workspace_bytes(64, 64, 64, o)
    assert "dz" in _abi.fd3d_last_error()
    o.dz = 0.0
    o.vacuum_top = -1
    with pytest.raises(_abi.FD3DError):
        _abi.fd3d_workspace_bytes(64, 64, 64, o)
    o.vacuum_top = 4
    o.free_surface = 1
    with pytest.raises(_abi.FD3DError):
        _abi.fd3d_workspace_bytes(64, 64, 64, o)
    assert "exclude" in _abi.fd3d_last_error()
    o.free_surface = 0
    assert _abi.fd3d_workspace_bytes(64, 64, 64, o) > 0
    # argument checks of the upsampler run before any device work
    with pytest.raises(_abi.FD3DError) as e:
        _abi.fd3d_upsample(None, (4, 4, 4), None, (8, 8, 8), _abi.FD3D_F32, None)
    assert e.value.code == _abi.FD3D_EINVAL
    with pytest.raises(_abi.FD3DError):
        _abi.fd3d_upsample(256, (0, 4, 4), 1 << 20, (8, 8, 8), _abi.FD3D_F32, None)
    with pytest.raises(_abi.FD3DError) as e:
        _abi.fd3d_upsample(4096, (4, 4, 4), 4096 + 128, (8, 8, 8), _abi.FD3D_F32, None)
    assert "overlap" in _abi.fd3d_last_error()


def test_layout_option():
    from paper_2112_15071_amd import _abi

    o = _abi.fd3d_opts()
    o.dtype = _abi.FD3D_F32
    size = {}
    for lay in (_abi.FD3D_LAYOUT_AUTO, _abi.FD3D_LAYOUT_SEPARATE, _abi.FD3D_LAYOUT_ROWS):
        o.layout = lay
        size[lay] = _abi.fd3d_workspace_bytes(64, 64, 64, o)
    # interleaved rows keep the model's copy beside the two state blocks
    assert size[_abi.FD3D_LAYOUT_ROWS] >= size[_abi.FD3D_LAYOUT_SEPARATE] + 8 * 64 ** 3 * 4
    # small planes: a whole-depth sweep fits one window, so automatic means rows
    assert size[_abi.FD3D_LAYOUT_AUTO] == size[_abi.FD3D_LAYOUT_ROWS]
    # 512 x 512 planes: 264 planes of 9 rows exceed 1 GiB, so automatic means separate arrays
    big = {}
    for lay in (_abi.FD3D_LAYOUT_AUTO, _abi.FD3D_LAYOUT_SEPARATE):
        o.layout = lay
        big[lay] = _abi.fd3d_workspace_bytes(512, 512, 256, o)
    assert big[_abi.FD3D_LAYOUT_AUTO] == big[_abi.FD3D_LAYOUT_SEPARATE]
    # forced rows need 12 planes of 9 nx ny samples within 1 GiB
    o.layout = _abi.FD3D_LAYOUT_ROWS
    assert _abi.fd3d_workspace_bytes(1024, 1024, 64, o) > 0
    with pytest.raises(_abi.FD3DError) as e:
        _abi.fd3d_workspace_bytes(4096, 4096, 16, o)
    assert e.value.code == _abi.FD3D_EINVAL and "rows" in _abi.fd3d_last_error()
    o.layout = 3
    with pytest.raises(_abi.FD3DError) as e:
        _abi.fd3d_workspace_bytes(64, 64, 64, o)
    assert "layout" in _abi.fd3d_last_error()

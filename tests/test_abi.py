"""The C-ABI library loads and exports every symbol its header declares;
host-only entry points validate their arguments (no GPU needed)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "resoct.h")
LIB = os.path.join(ROOT, "paper_2309_04393_amd", "_lib", "libresoct.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ro_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("library not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_host_entry_points_validate():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2309_04393_amd import resoct
    v = resoct.Volume((64, 64, 64), (1, 1, 1), 1, 1, 16, 3)
    assert v.brick_count() == 73
    d, f, nb = v.levels()
    assert nb.tolist() == [[4, 4, 4], [2, 2, 2], [1, 1, 1]]
    i = v.encode(0, 1, (1, 0, 1))
    assert i == (1 << 24) | (1 << 16) | 1
    assert v.decode(i) == (0, 1, (1, 0, 1))
    with pytest.raises(resoct.ResoctError):
        v.decode(0x00050000)  # bz = 5 does not exist
    with pytest.raises(resoct.ResoctError):
        resoct.Volume((64, 64, 64), (1, 1, 1), 1, 3, 16, 3)  # 3 bytes per voxel
    with pytest.raises(resoct.ResoctError) as e:
        resoct.Volume((8192 * 2, 64, 64), (1, 1, 1), 1, 2, 32, 3)  # 512 bricks on x
    assert e.value.code == -2
    with pytest.raises(resoct.ResoctError) as e:
        resoct.Volume((64, 64, 64), (1, 1, 1), 16, 2, 16, 17)
    # config sizes: 2 GiB cache of 32^3 u16 bricks with halo
    v2 = resoct.Volume((2048, 2048, 64), (1, 1, 4), 4, 2, 32, 7)
    assert v2.brick_count() == 4 * 10837
    d = resoct.CacheDesc(27318, 512)
    sz = resoct.CacheSizes()
    assert resoct._lib.ro_cache_query(v2.h, ctypes.byref(d), ctypes.byref(sz)) == 0
    assert sz.slot_stride == 78848 and sz.slots == 78848 * 27318
    od = resoct.OctreeDesc()
    od.leaf[:] = [16, 16, 4]
    od.depth, od.start_level = 7, 2
    osz = resoct.OctreeSizes()
    assert resoct._lib.ro_octree_query(v2.h, ctypes.byref(od), ctypes.byref(osz)) == 0
    assert osz.n_nodes == 299605 and osz.n_leaves == 262144
    od.leaf[:] = [16, 16, 3]  # not a power of two
    assert resoct._lib.ro_octree_query(v2.h, ctypes.byref(od), ctypes.byref(osz)) == -1
    assert "power of two" in resoct.last_error()

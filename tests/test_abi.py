"""The C-ABI library loads on the host and exports every function the header
declares; the host-only size query works without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "semfuse.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lf_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2111_11103_amd import build, semfuse
    if not os.path.exists(semfuse.LIB_PATH):
        build.build()
    return semfuse.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"lf_load_mesh", "lf_fuse_frames", "lf_render_labels"} <= set(names)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_size_query_on_host(lib):
    from paper_2111_11103_amd import semfuse as sf
    nx, ws = sf.mesh_sizes(1000, 2100, s=1, scheme=sf.SPLIT, n_classes=13)
    assert nx == 2100 and ws > 0
    nx, _ = sf.mesh_sizes(10, 501908, s=3, scheme=sf.SPLIT, n_classes=40)
    assert nx == 501908 * 9
    nx, _ = sf.mesh_sizes(10, 4, s=6, scheme=sf.SQUARE, n_classes=40)
    assert nx == 4 * 21
    nx, _ = sf.mesh_sizes(10, 3, s_face=[1, 3, 2], scheme=sf.SPLIT, n_classes=4)
    assert nx == 1 + 9 + 4
    with pytest.raises(sf.SemfuseError) as e:
        sf.mesh_sizes(10, 3, n_classes=0)
    assert e.value.status == sf.LF_EINVAL
    with pytest.raises(sf.SemfuseError):
        sf.mesh_sizes(10, 3, n_classes=300)
    with pytest.raises(sf.SemfuseError):
        sf.mesh_sizes(10, 3, s_face=[1, 0, 2], n_classes=4)
    with pytest.raises(sf.SemfuseError):
        sf.mesh_sizes(10, 2 ** 30, s=64, n_classes=4)    # more than 2^31 texels
    assert "gfx950" in sf.version()


def test_load_mesh_rejects_texel_counts_beyond_int32(lib):
    """Texel rows are int32 on the device: lf_load_mesh refuses a texel count
    of 2^31 or more (given, or implied by a uniform s) before it touches any
    buffer (the device pointers here are never dereferenced)."""
    from paper_2111_11103_amd import semfuse as sf
    fake = C.c_void_p(1 << 20)                   # 256-byte aligned, never used
    h = C.c_void_p()
    opts = sf._MeshOpts(sf.SPLIT, 64, 4, sf.AGG_SUM, sf.F32, 0.05)
    n_faces = 2 ** 20                            # 2^20 triangles x 64^2 texels = 2^32 rows
    st = lib.lf_load_mesh(C.byref(opts), fake, 3, fake, n_faces, None, fake, 1 << 40, fake, None,
                          n_faces * 64 * 64, None, C.byref(h))
    assert st == sf.LF_EINVAL and b"2^31" in lib.lf_last_error()
    opts = sf._MeshOpts(sf.SPLIT, 1, 4, sf.AGG_SUM, sf.F32, 0.05)
    st = lib.lf_load_mesh(C.byref(opts), fake, 3, fake, 2 ** 31 - 1, None, fake, 1 << 40, fake, None,
                          2 ** 31, None, C.byref(h))
    assert st == sf.LF_EINVAL and b"2^31" in lib.lf_last_error()
    assert not h.value

"""Graph files (graph_save / graph_load): a saved and reloaded graph equals the
built one bit for bit and the oracle's graph; damaged files are refused with
EIO, and files whose hash is right but whose content breaks the tree, the rows
or the depth recurrence (Sec. 2.1, 2.2) with EINVAL."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2606_11402_amd import Graph, VecchiaError, _lib

from test_graph_native import assert_same_graph

HEADER = 32


def fnv1a64(data):
    """64-bit FNV-1a (Fowler, Noll and Vo), written out byte by byte."""
    h = 0xcbf29ce484222325
    for c in data:
        h = ((h ^ c) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def same(a, b):
    assert (a.n, a.d, a.k, a.kp, a.n0, a.n_levels) == (b.n, b.d, b.k, b.kp, b.n0, b.n_levels)
    for name in ("order", "slot", "depth", "level_ptr"):
        assert (getattr(a, name) == getattr(b, name)).all(), name
    for layout in (0, 1):
        assert (a.nbr(layout) == b.nbr(layout)).all()
    assert (a.points().view(np.uint64) == b.points().view(np.uint64)).all()
    pa, ca = a.children()
    pb, cb = b.children()
    assert (pa == pb).all() and (ca == cb).all()


def _cases():
    rng = np.random.default_rng(11)
    ties = np.repeat(rng.random((40, 2)), 5, axis=0)          # every point five times
    signed = rng.standard_normal((300, 3))
    signed[::7, 1] = -0.0
    return [("uniform3d", rng.random((700, 3)), 8, 16),
            ("ties2d", ties, 5, 1),
            ("line1d", rng.random(257), 3, 4),
            ("signed_zero3d", signed, 12, 32),
            ("dense_only", rng.random((20, 3)), 4, 20),
            ("k_above_n", rng.random((9, 2)), 16, 2)]


@pytest.mark.parametrize("name,x,k,n0", _cases(), ids=[c[0] for c in _cases()])
def test_round_trip(tmp_path, name, x, k, n0):
    g = Graph(x, k, n0)
    path = tmp_path / (name + ".graph")
    g.save(path)
    h = Graph.load(path, n_threads=2)
    same(g, h)
    x2 = x[:, None] if x.ndim == 1 else x
    assert_same_graph(h, oracle.build_graph(x2, k, n0))
    size = HEADER + g.n * g.d * 8 + 4 * (3 * g.n + (g.n - g.n0) * g.k) + 8
    assert path.stat().st_size == size
    data = path.read_bytes()
    assert data[:8] == b"VCGRAPH1"
    assert int.from_bytes(data[-8:], "little") == fnv1a64(data[:-8])


def _parts(path):
    data = bytearray(path.read_bytes())
    n = int.from_bytes(data[8:16], "little")
    d, k, n0 = (int.from_bytes(data[16 + 4 * i:20 + 4 * i], "little") for i in range(3))
    o = HEADER
    offs = {}
    for name, size in (("x", n * d * 8), ("perm", 4 * n), ("sdim", 4 * n), ("rows", 4 * (n - n0) * k),
                       ("depth", 4 * n)):
        offs[name] = (o, size)
        o += size
    return data, (n, d, k, n0), offs


def _rehash(data):
    data[-8:] = fnv1a64(bytes(data[:-8])).to_bytes(8, "little")
    return data


@pytest.fixture(scope="module")
def saved(tmp_path_factory):
    x = np.random.default_rng(3).random((400, 3))
    g = Graph(x, 8, 16)
    path = tmp_path_factory.mktemp("g") / "g.graph"
    g.save(path)
    return g, path


def _expect(path, code):
    with pytest.raises(VecchiaError) as e:
        Graph.load(path)
    assert e.value.code == code, str(e.value)


def test_damaged_files_refused(saved, tmp_path):
    g, path = saved
    data = path.read_bytes()
    bad = tmp_path / "bad.graph"
    flipped = bytearray(data)
    flipped[HEADER + 1000] ^= 0x10                            # a coordinate bit: hash mismatch
    bad.write_bytes(bytes(flipped))
    _expect(bad, _lib.EIO)
    bad.write_bytes(data[:-9])                                # truncated
    _expect(bad, _lib.EIO)
    bad.write_bytes(data + b"\0")                             # trailing byte
    _expect(bad, _lib.EIO)
    bad.write_bytes(b"XCGRAPH1" + data[8:])                   # wrong magic
    _expect(bad, _lib.EIO)
    hdr = bytearray(data)
    hdr[16:20] = (4).to_bytes(4, "little")                    # d = 4
    bad.write_bytes(bytes(_rehash(hdr)))
    _expect(bad, _lib.EIO)
    _expect(tmp_path / "missing.graph", _lib.EIO)
    huge = bytearray(data[:HEADER])
    huge[8:16] = ((1 << 31) - 1).to_bytes(8, "little")        # a header claiming 2^31 - 1 points
    bad.write_bytes(bytes(huge))
    with pytest.raises(VecchiaError) as e:                    # refused by its length, before any allocation
        Graph.load(bad)
    assert e.value.code == _lib.EIO and "header implies" in str(e.value)


def test_wrong_content_refused(saved, tmp_path):
    """A file with a correct hash still has to describe a valid graph."""
    g, path = saved
    data, (n, d, k, n0), offs = _parts(path)
    bad = tmp_path / "content.graph"

    def rewrite(part, index, fn, itemsize=4, dtype=np.int32):
        buf = bytearray(data)
        o, size = offs[part]
        arr = np.frombuffer(bytes(buf[o:o + size]), dtype=dtype).copy()
        fn(arr, index)
        buf[o:o + size] = arr.tobytes()
        bad.write_bytes(bytes(_rehash(buf)))

    def swap(a, i):
        a[[i, i + 1]] = a[[i + 1, i]]

    rewrite("rows", 200 * k, swap)                            # a row out of (distance, slot) order
    _expect(bad, _lib.EINVAL)

    def later(a, i):
        a[i] = n0 + 150                                       # the row's own slot: not a predecessor
    rewrite("rows", 150 * k, later)
    _expect(bad, _lib.EINVAL)

    def deeper(a, i):
        a[i] += 1
    rewrite("depth", 300, deeper)                             # breaks the depth recurrence
    _expect(bad, _lib.EINVAL)
    rewrite("perm", 5, swap)                                  # not the tree of these points
    _expect(bad, _lib.EINVAL)

    def moved(a, i):
        a[i] += 0.5                                           # a point moved: its slot breaks the tree
    rewrite("x", 3 * 17, moved, dtype=np.float64)
    _expect(bad, _lib.EINVAL)


def test_pending_graph_not_saved(tmp_path):
    lib = _lib.load()
    x = np.random.default_rng(1).random((100, 3))
    h = ctypes.c_void_p()
    _lib.check(lib.graph_build_begin(x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 100, 3, 4, 8, 1,
                                     ctypes.byref(h)), "graph_build_begin")
    assert lib.graph_save(h, str(tmp_path / "p.graph").encode()) == _lib.EINVAL
    out = np.empty((100, 3))
    assert lib.graph_export_points(h, _lib.FP64, ctypes.c_void_p(out.ctypes.data)) == _lib.EINVAL
    lib.graph_free(h)

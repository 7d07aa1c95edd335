"""gs_export / gs_import file format, checked on the host (no GPU).

A host-only context (device -1) holds an explicitly installed setup -- the
CPU oracle's (Alg. 1) -- and writes it with gs_export.  A plain reader below,
written from the layout documented in include/gemslr.h, parses the file and
every array must equal the oracle's bit for bit and what gs_get_level /
gs_get_perm report; gs_import of the file into a second host-only context
reproduces the same arrays.  Malformed files are rejected with GS_EINVAL.
"""
import os
import struct

import numpy as np
import pytest

from paper_2205_03224_amd import gemslr, workloads as wl
from oracle import gemslr as og, partition as opart


def _oracle_levels(st):
    levels = []
    for lv in st.levels:
        d = {"d": lv.d, "block_ptr": lv.blocks,
             "L": (lv.Lf.indptr, lv.Lf.indices, lv.Lf.data),
             "U": (lv.Uf.indptr, lv.Uf.indices, lv.Uf.data)}
        if lv.s > 0:
            d.update(E=(lv.E.indptr, lv.E.indices, lv.E.data),
                     F=(lv.F.indptr, lv.F.indices, lv.F.data), W=lv.W, H=lv.H)
        levels.append(d)
    return levels


class _Reader:
    def __init__(self, raw, vt):
        self.raw, self.o, self.vt = raw, 0, np.dtype(vt)

    def take(self, dtype, count):
        dt = np.dtype(dtype)
        a = np.frombuffer(self.raw, dtype=dt, count=count, offset=self.o)
        self.o += dt.itemsize * count
        return a

    def one(self, dtype):
        return int(self.take(dtype, 1)[0])

    def csr(self, rows):
        nnz = self.one("<i8")
        return self.take("<i8", rows + 1), self.take("<i4", nnz), self.take(self.vt, nnz)


def read_export(path):
    """Plain reader of the gs_export layout."""
    raw = open(path, "rb").read()
    assert raw[:8] == b"GEMSLR01" and raw[-8:] == b"GEMSLREN"
    dtype, L, n = struct.unpack_from("<iiq", raw, 8)
    r = _Reader(raw, "<c16" if dtype == gemslr.GS_C128 else "<f8")
    r.o = 24
    out = {"dtype": dtype, "L": L, "n": n, "A": r.csr(n), "perm": r.take("<i8", n), "levels": []}
    start = 0
    for l in range(L + 1):
        d = r.one("<i8")
        nb = r.one("<i8")
        lv = {"d": d, "block_ptr": r.take("<i8", nb + 1), "L": r.csr(d), "U": r.csr(d)}
        if l < L:
            s = n - start - d
            lv["E"], lv["F"] = r.csr(s), r.csr(d)
            k = r.one("<i4")
            assert r.one("<i4") == 0
            lv["W"] = r.take(r.vt, s * k).reshape((s, k), order="F")
            lv["H"] = r.take(r.vt, k * k).reshape((k, k), order="F")
        out["levels"].append(lv)
        start += d
    assert r.o == len(raw) - 8, "trailing bytes"
    return out


def _same_csr(got, ref):
    rp, ci, v = got
    assert np.array_equal(rp, ref.indptr) and np.array_equal(ci, ref.indices)
    assert np.array_equal(v, ref.data)


@pytest.mark.parametrize("case", ["convdiff8", "helmholtz8"])
def test_export_matches_oracle_setup(case, tmp_path):
    if case == "convdiff8":
        w = wl.convdiff3d_64(N=8, nparts=8)
    else:
        w = wl.helmholtz3d_128(N=8, nparts=8)
    part = opart.wirebasket(w.dims, w.nparts, w.levels, w.rowptr, w.col)
    st = og.setup(w.rowptr, w.col, w.val, part, ilu="ilut", drop_tol=w.drop_tol, lfil=10, rank=4)
    ctx = gemslr.Context(-1)
    ctx.setup_explicit(w.rowptr, w.col, w.val, st.perm, _oracle_levels(st))
    path = str(tmp_path / "pre.gslr")
    ctx.export(path)
    f = read_export(path)
    assert f["n"] == w.n and f["L"] == len(st.levels) - 1
    assert f["dtype"] == (gemslr.GS_C128 if np.iscomplexobj(w.val) else gemslr.GS_F64)
    assert np.array_equal(f["perm"], st.perm) and np.array_equal(f["perm"], ctx.perm())
    assert np.array_equal(f["A"][0], w.rowptr) and np.array_equal(f["A"][1], w.col)
    assert np.array_equal(f["A"][2], w.val)
    for l, (lv, ref) in enumerate(zip(f["levels"], st.levels)):
        assert lv["d"] == ref.d
        assert np.array_equal(lv["block_ptr"], ref.blocks)
        _same_csr(lv["L"], ref.Lf)
        _same_csr(lv["U"], ref.Uf)
        got = ctx.level(l)
        assert np.array_equal(got["L"][2], lv["L"][2]) and np.array_equal(got["U"][1], lv["U"][1])
        if ref.s > 0:
            _same_csr(lv["E"], ref.E)
            _same_csr(lv["F"], ref.F)
            assert np.array_equal(lv["W"], ref.W) and np.array_equal(lv["H"], ref.H)
            assert np.array_equal(got["W"], lv["W"]) and np.array_equal(got["H"], lv["H"])
    # import into a second host-only context: the same arrays come back
    ctx2 = gemslr.Context(-1).import_setup(path)
    assert np.array_equal(ctx2.perm(), st.perm)
    for l in range(len(st.levels)):
        a, b = ctx.level(l), ctx2.level(l)
        for key in ("L", "U", "E", "F"):
            if key in a and a[key] is not None:
                for x, y in zip(a[key], b[key]):
                    assert np.array_equal(x, y)
        if st.levels[l].s > 0:
            assert np.array_equal(a["W"], b["W"]) and np.array_equal(a["H"], b["H"])
    # an export of the import is the same file
    path2 = str(tmp_path / "pre2.gslr")
    ctx2.export(path2)
    assert open(path, "rb").read() == open(path2, "rb").read()
    ctx.close()
    ctx2.close()


def test_export_import_errors(tmp_path):
    ctx = gemslr.Context(-1)
    with pytest.raises(gemslr.GemslrError) as e:
        ctx.export(str(tmp_path / "x.gslr"))
    assert e.value.code == gemslr.GS_ESTATE
    w = wl.laplace2d_32(N=8)
    part = opart.wirebasket(w.dims, 4, 2, w.rowptr, w.col)
    st = og.setup(w.rowptr, w.col, w.val, part, ilu="ilu0", rank=2)
    ctx.setup_explicit(w.rowptr, w.col, w.val, st.perm, _oracle_levels(st))
    good = str(tmp_path / "good.gslr")
    ctx.export(good)
    raw = open(good, "rb").read()
    bad = str(tmp_path / "bad.gslr")
    for blob in (raw[:-20], b"NOTGSLR1" + raw[8:], raw[:-8] + b"XXXXXXXX", raw[:30]):
        open(bad, "wb").write(blob)
        with pytest.raises(gemslr.GemslrError) as e:
            gemslr.Context(-1).import_setup(bad)
        assert e.value.code == gemslr.GS_EINVAL
    with pytest.raises(gemslr.GemslrError) as e:
        gemslr.Context(-1).import_setup(str(tmp_path / "missing.gslr"))
    assert e.value.code == gemslr.GS_EINVAL
    # a corrupted column index is caught by the setup's validation
    f = read_export(good)
    off = 24 + 8 + 8 * (f["n"] + 1)  # first int32 column of A
    corrupt = bytearray(raw)
    corrupt[off:off + 4] = struct.pack("<i", 10 ** 6)
    open(bad, "wb").write(bytes(corrupt))
    with pytest.raises(gemslr.GemslrError) as e:
        gemslr.Context(-1).import_setup(bad)
    assert e.value.code == gemslr.GS_EINVAL
    with pytest.raises(gemslr.GemslrError):
        ctx.export(str(tmp_path / "no_such_dir" / "x.gslr"))
    ctx.close()
